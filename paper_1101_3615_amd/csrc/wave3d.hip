// 3D time-step kernels of the Born / reverse-time sweeps (gfx950).
//
// A workgroup (256 threads, 4 wavefronts) owns a 64 x 16 tile of the xy plane
// and marches down a chunk of z planes.  Each 16-lane row of a wavefront holds
// 64 consecutive x cells (4 per lane, 16-byte loads), so one wavefront covers
// 4 y rows and the workgroup 16.  Per plane:
//   z-neighbours: a 9-plane register queue of the lane's own cells;
//   x-neighbours: DPP row shifts inside each 16-lane row, plus a 4-cell halo
//                 loaded by the first and last lane of the row;
//   y-neighbours: the tile's centre plane plus 4 halo rows above and below,
//                 staged in LDS (double buffered: one barrier per plane).
// Every input of a plane (queue row, halos, kappa, previous level, g, image) is
// loaded through buffer resources one plane ahead (FP32 sweeps), so its latency
// overlaps the work on the plane before; lanes and planes outside the grid read
// zero from the hardware range check instead of branching.
// Workgroups are persistent and walk their XCD's items tiles fastest, so the
// workgroups of a round hold a block of neighbouring tiles of one pair of shots and
// each tile's halo rows come from that XCD's L2.
// The arithmetic per cell is that of the 2D kernel with the y axis added,
// including its two forms of the imaging condition (g^{k-1} nu^k, or u^k times
// c^2 (L nu^{k+1} + R^T d) when the slots hold background levels).
#include <algorithm>

#include "common.h"
#include "wave.h"

namespace mp {

// Buffer-resource access (raw buffers, hardware range check on the per-lane
// offset: an inactive lane's offset lies past any resource, so its reads return
// zero and its writes are dropped).  Word 3: gfx9-family raw-buffer configuration.
using Rsrc3 = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x4_3 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_3 __attribute__((ext_vector_type(2)));
constexpr unsigned OFF_NONE3 = 0x80000000u;
// cache policy of the data that no other workgroup rereads soon (outputs, the
// cell's own previous level, g, image): non-temporal, so that L2 keeps the field
// rows that neighbouring tiles read as halos and the kappa and perturbation rows
// that the other pairs of shots on the tile read
constexpr int NT3 = 2;
__device__ __forceinline__ Rsrc3 rsrc3(const void* base, long long bytes) {
  const int n = bytes >= 0xffffffffLL ? -1 : (int)(unsigned)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}
template <int CP = 0>
__device__ __forceinline__ V4<float> bld4(Rsrc3 r, unsigned vo, unsigned so, float) {
  const u32x4_3 v = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, CP);
  V4<float> o;
  o.v[0] = __uint_as_float(v.x);
  o.v[1] = __uint_as_float(v.y);
  o.v[2] = __uint_as_float(v.z);
  o.v[3] = __uint_as_float(v.w);
  return o;
}
template <int CP = 0>
__device__ __forceinline__ V4<double> bld4(Rsrc3 r, unsigned vo, unsigned so, double) {
  const u32x4_3 a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, CP);
  const u32x4_3 b = __builtin_amdgcn_raw_buffer_load_b128(r, vo + 16, so, CP);
  V4<double> o;
  o.v[0] = __longlong_as_double(((long long)a.y << 32) | a.x);
  o.v[1] = __longlong_as_double(((long long)a.w << 32) | a.z);
  o.v[2] = __longlong_as_double(((long long)b.y << 32) | b.x);
  o.v[3] = __longlong_as_double(((long long)b.w << 32) | b.z);
  return o;
}
// 16-byte stores take the uniform offset in the per-lane offset and a constant
// zero SOFFSET: a VALU write to the data registers of a store wider than 8 bytes
// right after it issues can change the data stored, and the compiler inserts the
// wait states that prevent this only for stores with a constant SOFFSET.  (With
// the plane offset in an SGPR SOFFSET, the field stores were seen to take such
// later values.)  An inactive lane's OFF_NONE3 plus the plane offset stays past
// the resource: a field slice is kept below 1 GiB when the context is created.
template <int CP = 0>
__device__ __forceinline__ void bst4(const V4<float>& a, Rsrc3 r, unsigned vo, unsigned so) {
  u32x4_3 v;
  v.x = __float_as_uint(a.v[0]);
  v.y = __float_as_uint(a.v[1]);
  v.z = __float_as_uint(a.v[2]);
  v.w = __float_as_uint(a.v[3]);
  __builtin_amdgcn_raw_buffer_store_b128(v, r, vo + so, 0, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bst4(const V4<double>& a, Rsrc3 r, unsigned vo, unsigned so) {
  u32x4_3 v0, v1;
  const long long b0 = __double_as_longlong(a.v[0]), b1 = __double_as_longlong(a.v[1]);
  const long long b2 = __double_as_longlong(a.v[2]), b3 = __double_as_longlong(a.v[3]);
  v0.x = (unsigned)b0;
  v0.y = (unsigned)(b0 >> 32);
  v0.z = (unsigned)b1;
  v0.w = (unsigned)(b1 >> 32);
  v1.x = (unsigned)b2;
  v1.y = (unsigned)(b2 >> 32);
  v1.z = (unsigned)b3;
  v1.w = (unsigned)(b3 >> 32);
  __builtin_amdgcn_raw_buffer_store_b128(v0, r, vo + so, 0, CP);
  __builtin_amdgcn_raw_buffer_store_b128(v1, r, vo + so + 16, 0, CP);
}
__device__ __forceinline__ int depth3(int i, int n, int nb) { return max(max(nb - i, i - (n + nb - 1)), 0); }
// a = 1 / (1 + e), b = (1 - e) a with e = ec * dd (dd: sum of squared layer depths)
__device__ __forceinline__ void damp3(float ec, int dd, float& a, float& b) {
  const float e = ec * (float)dd;
  a = dd > 0 ? __builtin_amdgcn_rcpf(1.0f + e) : 1.0f;
  b = (1.0f - e) * a;
}
__device__ __forceinline__ void damp3(double ec, int dd, double& a, double& b) {
  const double e = ec * (double)dd;
  a = dd > 0 ? 1.0 / (1.0 + e) : 1.0;
  b = (1.0 - e) * a;
}

constexpr int TX = 64;   // x cells per tile
constexpr int TY = 16;   // y rows per tile

// Laplacian of the lane's four cells.  x: DPP row shifts, the first and last lane
// of a 16-lane row taking the halo xh; y: the LDS plane P (tile rows plus four
// halo rows above and below); z: the register queue.
template <typename T>
__device__ __forceinline__ void lap_row(const V4<T>* qa, int r, const V4<T>& xh, const T (*P)[TX], int yl,
                                        int c4, const Step<T>& p, T out[4]) {
  const V4<T>& C = qa[(r + 4) % 9];
  T w[12];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    w[i] = rshr1(C.v[i], xh.v[i]);
    w[4 + i] = C.v[i];
    w[8 + i] = rshl1(C.v[i], xh.v[i]);
  }
  V4<T> ym[4], yp[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ym[j] = *reinterpret_cast<const V4<T>*>(&P[yl + 4 - (j + 1)][c4]);
    yp[j] = *reinterpret_cast<const V4<T>*>(&P[yl + 4 + (j + 1)][c4]);
  }
  // difference form, smallest weights first (see the 2D kernel)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T c = w[4 + i];
    T s = p.c4 * (((w[0 + i] - c) + (w[8 + i] - c)) + ((ym[3].v[i] - c) + (yp[3].v[i] - c)) +
                  ((qa[(r + 0) % 9].v[i] - c) + (qa[(r + 8) % 9].v[i] - c)));
    s += p.c3 * (((w[1 + i] - c) + (w[7 + i] - c)) + ((ym[2].v[i] - c) + (yp[2].v[i] - c)) +
                 ((qa[(r + 1) % 9].v[i] - c) + (qa[(r + 7) % 9].v[i] - c)));
    s += p.c2 * (((w[2 + i] - c) + (w[6 + i] - c)) + ((ym[1].v[i] - c) + (yp[1].v[i] - c)) +
                 ((qa[(r + 2) % 9].v[i] - c) + (qa[(r + 6) % 9].v[i] - c)));
    s += p.c1 * (((w[3 + i] - c) + (w[5 + i] - c)) + ((ym[0].v[i] - c) + (yp[0].v[i] - c)) +
                 ((qa[(r + 3) % 9].v[i] - c) + (qa[(r + 5) % 9].v[i] - c)));
    out[i] = s;
  }
}

// A workgroup (512 threads) carries one tile for a pair of consecutive job shots:
// threads 0..255 the even shot, 256..511 the odd one.  The two halves march in
// step (one barrier per plane serves both), so the second read of kappa and the
// perturbation hits in cache, and the adjoint images the pair into one FP64 image
// (the pair's contributions summed in shot order in LDS, one read-modify-write).
// The background sweeps that store no checkpoint (the recomputation) are held to
// four waves per SIMD (128 VGPRs), so that two workgroups share a CU; the others
// would spill at that bound.
template <typename T, int MODE, int CK>
__global__ __launch_bounds__(512, (MODE == M_BG && CK != CK_F32 && CK != CK_BF16) ? 4 : 1) void k_step3d(
    Step<T> p, int n, int hslot, int ck_store, int ck_max) {
  constexpr bool TWO = (MODE == M_FUSED);
  // LDS plane per half and field: the tile's rows plus four halo rows above and
  // below (double buffered: one barrier per plane)
  constexpr int NB = TWO ? 2 : 1;
  __shared__ __align__(32) T PL[2][NB][2][TY + 8][TX];
  // adjoint: each half's image contribution to a plane, read one plane later
  __shared__ __align__(32) V4<double> RED[(MODE == M_ADJ) ? 2 : 1][2][(MODE == M_ADJ) ? 256 : 1];

  const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 8);
  const int tid = threadIdx.x & 255;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int c = lane & 15;
  const int yl = wv * 4 + (lane >> 4);     // 0..15 within the tile
  // Persistent workgroups: the grid holds as many workgroups as the device keeps
  // resident (a multiple of 8), workgroup b runs on XCD b % 8 and walks that XCD's
  // contiguous range of items with the stride of the XCD's workgroups, so the
  // workgroups that run together start their items together and march in step.
  const int per = (p.nwg + 7) >> 3;
  const int xcd = (int)(blockIdx.x & 7u);
  const int spx = (int)(gridDim.x >> 3);
  int buf = 0;   // LDS buffer parity, continued across items
  for (int k = (int)(blockIdx.x >> 3); k < per; k += spx) {
  const int item = xcd * per + k;
  if (item >= p.nwg) break;
  // x tiles fastest, then y tiles, pairs of shots and z chunks: the workgroups that
  // run together on one XCD carry one pair over a block of neighbouring tiles, so the
  // x and y halo rows a tile reads are the rows its neighbours are loading at the
  // same plane, from that XCD's L2 (marching in step).  (Pairs fastest, which
  // shares kappa and the perturbation of a tile between the pairs instead, moved
  // more bytes: halo rows are a third of the reads.)
  const int npair = p.nsh >> 1;
  const int ntile = p.L.nstrips * p.L.nytiles;
  const int tile = item % ntile;
  int rest = item / ntile;
  const int tx = tile % p.L.nstrips;
  const int ty = tile / p.L.nstrips;
  const int ls = (rest % npair) * 2 + half;
  const int chunk = rest / npair;
  const int z0 = chunk * p.zc;
  const int z1 = min(z0 + p.zc, p.L.nzp);
  // odd chunks march with z decreasing (z1 - 1 .. z0), even chunks with z increasing, so that two neighbouring
  // chunks reach the planes around their shared boundary together (both at the end
  // or both at the start of their march) and the second read of those planes finds
  // them in the last-level cache; the Laplacian sums each symmetric pair of planes
  // commutatively, so the direction changes no result bit
  const int dz3 = (chunk & 1) ? -1 : 1;
  const int zs = dz3 > 0 ? z0 : z1 - 1;
  const int nit = z1 - z0;

  const int pitch = p.L.pitch;
  const long long plane = p.L.plane;
  const int nxp = p.L.nxp, nyp = p.L.nyp;
  const int x = tx * TX + c * 4 - XL;          // propagation x of the lane's first cell
  const int y = ty * TY + yl;
  const bool yin = y < nyp;
  const bool xin = (x >= 0) && (x < nxp);
  const bool act = xin && yin;
  const bool hl_in = (c == 0) && (x - 4 >= 0) && (x - 4 < nxp) && yin;
  const bool hr_in = (c == 15) && (x + 4 < nxp) && yin;
  const int shot = p.shot0 + ls;
  const bool live = p.srcx[shot] >= 0;   // a null shot (group padding) has no source and no data

  bool xvalid[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) xvalid[i] = (x + i >= 0) && (x + i < nxp);
  const int xm = x - p.L.nb, ym = y - p.L.nb;
  bool xmod[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) xmod[i] = (xm + i >= 0) && (xm + i < p.L.nx);
  const bool xmodany = xmod[0] || xmod[1] || xmod[2] || xmod[3];
  const bool ymod = (ym >= 0) && (ym < p.L.ny);

  // squared layer depths along x and y of the lane's cells (damping from the
  // layer's closed form: e = eta_c (dx^2 + dy^2 + dz^2))
  int dxy2[4];
  const int dy = depth3(y, p.L.ny, p.L.nb);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int dx = depth3(x + i, p.L.nx, p.L.nb);
    dxy2[i] = dx * dx + dy * dy;
  }
  // tile interior: every cell of the 64 x 16 tile outside the layer in x and y
  const int tx0 = tx * TX - XL, ty0 = ty * TY;
  const bool tile_free = tx0 >= p.L.nb && tx0 + TX <= nxp - p.L.nb && ty0 >= p.L.nb && ty0 + TY <= nyp - p.L.nb;

  int sx = -1, sy = -1, sz = -1;
  if (MODE == M_FUSED || MODE == M_BG) {
    sx = p.srcx[shot];
    sy = p.srcy[shot];
    sz = p.srcz[shot];
  }
  const T wsrc = (MODE == M_FUSED || MODE == M_BG) ? p.wav[n] : T(0);

  // background in increment form (see the 2D kernel)
  constexpr bool BGM = (MODE == M_FUSED || MODE == M_BG);

  // Buffer resources on the shot's field slices: a lane adds its offset within a
  // z plane (OFF_NONE3 outside the grid: reads zero, writes dropped), a plane the
  // uniform offset soff(z).  Field A is the background (u, D) or the single wave
  // field of the Born / adjoint sweeps, B the Born field of the fused sweep.
  const long long sb = (long long)ls * p.L.fstride;
  const long long fbytes3 = p.L.fstride * (long long)sizeof(T);
  const Rsrc3 rAc = rsrc3((BGM ? p.u_cur : p.du_cur) + sb, fbytes3);
  const Rsrc3 rAn = rsrc3((BGM ? p.u_next : p.du_prev) + sb, fbytes3);   // level n+1 (in place over n-1)
  const Rsrc3 rAp = rsrc3((BGM ? p.u_inc : p.du_prev) + sb, fbytes3);   // increment / level n-1
  const Rsrc3 rBc = rsrc3(TWO ? p.du_cur + sb : p.u_cur, TWO ? fbytes3 : 0);
  const Rsrc3 rBp = rsrc3(TWO ? p.du_prev + sb : p.u_cur, TWO ? fbytes3 : 0);
  const Rsrc3 rK = rsrc3(p.kappa, fbytes3);
  const Rsrc3 rM = rsrc3(p.dmbar + (long long)p.dm_slot[shot] * p.L.fstride, fbytes3);
  const unsigned esz = (unsigned)sizeof(T);
  const unsigned lvo = act ? (unsigned)((long long)(y + GY) * pitch + XL + x) * esz : OFF_NONE3;
  // x halo: the first lane of a 16-lane row loads the 4 cells left of the row,
  // the last lane the 4 cells right of it
  const unsigned xvo = hl_in   ? (unsigned)((long long)(y + GY) * pitch + XL + x - 4) * esz
                       : hr_in ? (unsigned)((long long)(y + GY) * pitch + XL + x + 4) * esz
                               : OFF_NONE3;
  auto soff = [&](int zz) -> unsigned { return (unsigned)((long long)SLACK + (long long)(zz + GZ) * plane) * esz; };
  // model-grid resources (g slot of the shot, FP64 image of the shot): the plane
  // offset is added to the lane offset as an unsigned value, so planes above or
  // below the model wrap past the end of the resource and read zero
  const long long hoff = (long long)(p.hmod > 0 ? ls % p.hmod : ls) * p.hstride + (long long)hslot * p.L.mstride;
  const long long mbytes3 = p.L.mstride * (long long)sizeof(T);
  const Rsrc3 rG = rsrc3(hslot >= 0 ? p.hist + hoff : p.hist, hslot >= 0 ? mbytes3 : 0);
  const Rsrc3 rI = rsrc3(MODE == M_ADJ ? p.img + (long long)(shot >> 1) * p.L.mstride : p.img,
                         MODE == M_ADJ ? p.L.mstride * 8LL : 0);
  const bool mlane = act && ymod && xmodany;
  const unsigned gvo = mlane ? (unsigned)((long long)ym * p.L.mpitch + xm) * esz : OFF_NONE3;
  const unsigned ivo = (mlane && half == 0) ? (unsigned)((long long)ym * p.L.mpitch + xm) * 8u : OFF_NONE3;
  const unsigned gplane = (unsigned)(p.L.mplane * (long long)esz);
  const unsigned iplane = (unsigned)(p.L.mplane * 8LL);
  const int nb = p.L.nb;

  // halo rows of the LDS plane: waves 0-1 load field A, waves 2-3 field B
  const int wvu = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool hfieldB = wvu >= 2;
  const int ht = tid & 127;
  const int hrow = ht >> 4;                 // 0..3: rows -4..-1, 4..7: rows TY..TY+3
  const int hcol = (ht & 15) * 4;
  const int hy = (hrow < 4) ? ty * TY - 4 + hrow : ty * TY + TY + (hrow - 4);
  const int hlds = (hrow < 4) ? hrow : TY + hrow;   // row of the LDS plane
  const int hx = tx * TX + hcol - XL;
  const bool hload = (hx >= 0) && (hx < nxp) && (hy >= 0) && (hy < nyp) && (TWO || !hfieldB);
  const unsigned hvo = hload ? (unsigned)((long long)(hy + GY) * pitch + XL + hx) * esz : OFF_NONE3;
  const Rsrc3 rHv = hfieldB ? rBc : rAc;

  // CK_LF32 / CK_LBF16 (background recomputation, first step of a segment): the
  // input level u^n and increment D^n come from checkpoint ck_store in its compact
  // layout [z][y][cpitch], converted as the expansion pass would (same bits), in
  // place of the field slices; the same lane masks apply, and planes outside
  // [0, nzp) wrap past the resource.
  constexpr bool LDCK = (CK == CK_LF32 || CK == CK_LBF16);
  constexpr unsigned cesz = (CK == CK_LBF16) ? 2u : (unsigned)sizeof(T);
  const long long clv = ((long long)ls * p.nck + max(ck_store, 0)) * 2;
  const Rsrc3 rC0 = rsrc3(LDCK ? static_cast<char*>(p.ck) + clv * p.cstride * cesz : static_cast<char*>(p.ck),
                          LDCK ? p.cstride * (long long)cesz : 0);
  const Rsrc3 rC1 = rsrc3(LDCK ? static_cast<char*>(p.ck) + (clv + 1) * p.cstride * cesz : static_cast<char*>(p.ck),
                          LDCK ? p.cstride * (long long)cesz : 0);
  const unsigned clvo = act ? (unsigned)((long long)y * p.cpitch + x) * cesz : OFF_NONE3;
  const unsigned cxvo = hl_in   ? (unsigned)((long long)y * p.cpitch + x - 4) * cesz
                        : hr_in ? (unsigned)((long long)y * p.cpitch + x + 4) * cesz
                                : OFF_NONE3;
  const unsigned chvo = hload ? (unsigned)((long long)hy * p.cpitch + hx) * cesz : OFF_NONE3;
  const unsigned cplane = (unsigned)((long long)nyp * p.cpitch * cesz);
  float cs0 = 1.0f, cs1 = 1.0f;
  if (CK == CK_LBF16) {
    cs0 = p.ck_scale[clv];
    cs1 = p.ck_scale[clv + 1];
  }
  auto ldck = [&](int lev, unsigned lo, int zz) -> V4<T> {
    const unsigned off = lo + (unsigned)zz * cplane;
    if (CK == CK_LF32) return bld4(lev ? rC1 : rC0, off, 0u, T(0));
    const u32x2_3 w = __builtin_amdgcn_raw_buffer_load_b64(lev ? rC1 : rC0, off, 0u, 0);
    const float sc = lev ? cs1 : cs0;
    V4<T> r;
    r.v[0] = (T)bf16_scaled((unsigned short)(w.x & 0xffffu), sc);
    r.v[1] = (T)bf16_scaled((unsigned short)(w.x >> 16), sc);
    r.v[2] = (T)bf16_scaled((unsigned short)(w.y & 0xffffu), sc);
    r.v[3] = (T)bf16_scaled((unsigned short)(w.y >> 16), sc);
    return r;
  };

  // Inputs of one z plane.  FP32 sweeps load them one plane ahead (a second set of
  // registers); FP64 sweeps (small test grids, twice the registers) at the start
  // of the plane.
  struct In3 {
    V4<T> qa, qb;          // plane z + 4d of fields A, B (enters the queue; d = march direction)
    V4<T> hv;              // y-halo row of plane z (field A or B)
    V4<T> xa, xb;          // x halos of plane z
    V4<T> kap, ap, bp, dm; // kappa, A increment / level n-1, B level n-1, perturbation
    V4<T> g;               // Born / adjoint: g of plane z
    V4<double> im;         // adjoint: the pair's image on the previous plane z - d (even half)
  };
  auto fetch = [&](int z, In3& f) {
    const unsigned s = soff(z);
    if (LDCK) {
      f.qa = ldck(0, clvo, z + 4 * dz3);
      f.hv = ldck(0, chvo, z);
      f.xa = ldck(0, cxvo, z);
      f.ap = ldck(1, clvo, z);
    } else {
      f.qa = bld4(rAc, lvo, soff(z + 4 * dz3), T(0));
      f.hv = bld4(rHv, hvo, s, T(0));
      f.xa = bld4(rAc, xvo, s, T(0));
      f.ap = bld4<NT3>(rAp, lvo, s, T(0));
    }
    if (TWO) f.qb = bld4(rBc, lvo, soff(z + 4 * dz3), T(0));
    if (TWO) f.xb = bld4(rBc, xvo, s, T(0));
    f.kap = bld4(rK, lvo, s, T(0));
    if (TWO) f.bp = bld4<NT3>(rBp, lvo, s, T(0));
    if (TWO || MODE == M_BORN) f.dm = bld4(rM, lvo, s, T(0));
    const unsigned zm = (unsigned)(z - nb);
    if (MODE == M_BORN || MODE == M_ADJ) f.g = bld4<NT3>(rG, gvo + zm * gplane, 0u, T(0));
    if (MODE == M_ADJ) f.im = bld4<NT3>(rI, ivo + (zm - (unsigned)dz3) * iplane, 0u, double(0));
  };
  constexpr bool PF3 = sizeof(T) == 4;

  // Image of plane zz for the pair: old + (even half's + odd half's contribution),
  // written by the even half (the contributions were put in LDS before a barrier)
  auto pair_image = [&](int zz, const V4<double>& old) {
    const int zmm = zz - nb;
    if (half == 0 && zmm >= 0 && zmm < p.L.nz) {   // uniform
      V4<double> acc = old;
      const V4<double>& a0 = RED[0][zz & 1][tid];
      const V4<double>& a1 = RED[MODE == M_ADJ ? 1 : 0][zz & 1][tid];
  #pragma unroll
      for (int i = 0; i < 4; ++i) acc.v[i] += a0.v[i] + a1.v[i];
      bst4<NT3>(acc, rI, ivo + (unsigned)zmm * iplane, 0u);
    }
  };
  float mx0 = 0.0f, mx1 = 0.0f;
  V4<T> qa[9], qb[9];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    qa[s] = LDCK ? ldck(0, clvo, zs + (s - 4) * dz3) : bld4(rAc, lvo, soff(zs + (s - 4) * dz3), T(0));
    if (TWO) qb[s] = bld4(rBc, lvo, soff(zs + (s - 4) * dz3), T(0));
  }
  In3 cur, nxt;
  if (PF3) fetch(zs, cur);

  for (int tb = 0; tb < nit; tb += 9) {
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int t = tb + r;
      const int z = zs + t * dz3;
      if (t < nit) {   // uniform; a constant trip count keeps the loop fully unrolled
        if (PF3) fetch(t + 1 < nit ? z + dz3 : z, nxt);   // the last plane reloads itself
        else fetch(z, cur);
        qa[(r + 8) % 9] = cur.qa;
        if (TWO) qb[(r + 8) % 9] = cur.qb;
        // centre rows and y halo into LDS
        *reinterpret_cast<V4<T>*>(&PL[half][0][buf][yl + 4][c * 4]) = qa[(r + 4) % 9];
        if (TWO) *reinterpret_cast<V4<T>*>(&PL[half][NB - 1][buf][yl + 4][c * 4]) = qb[(r + 4) % 9];
        if (!hfieldB) *reinterpret_cast<V4<T>*>(&PL[half][0][buf][hlds][hcol]) = cur.hv;
        else if (TWO) *reinterpret_cast<V4<T>*>(&PL[half][NB - 1][buf][hlds][hcol]) = cur.hv;
        lds_barrier();
        T lapA[4], lapB[4];
        lap_row(qa, r, cur.xa, PL[half][0][buf], yl, c * 4, p, lapA);
        if (TWO) lap_row(qb, r, cur.xb, PL[half][NB - 1][buf], yl, c * 4, p, lapB);
        buf ^= 1;
        if (MODE == M_ADJ && t > 0) pair_image(z - dz3, cur.im);
        const unsigned sz_ = soff(z);

        if ((MODE == M_FUSED || MODE == M_BG) && z == sz && y == sy) {
  #pragma unroll
          for (int i = 0; i < 4; ++i)
            if (x + i == sx) lapA[i] += wsrc;
        }
        const int rp = (z < p.rec_lo || z > p.rec_hi) ? -1 : p.recplane[z];
        const bool recrow = rp >= 0;   // uniform
        int rm[4] = {-1, -1, -1, -1};
        if (recrow && act && live) {
          const int4 m4 = *reinterpret_cast<const int4*>(p.recmap + ((long long)rp * nyp + y) * p.cpitch + x);
          rm[0] = m4.x;
          rm[1] = m4.y;
          rm[2] = m4.z;
          rm[3] = m4.w;
          if (MODE == M_ADJ) {
            const T* drow = p.data + ((long long)shot * p.nt + (n - 1)) * p.nr;
  #pragma unroll
            for (int i = 0; i < 4; ++i)
              if (rm[i] >= 0) lapA[i] += drow[rm[i]];
          }
        }

        const V4<T>& kap4 = cur.kap;
        const int dz = depth3(z, p.L.nz, nb);
        T a[4], b[4];
        if (tile_free && dz == 0) {
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            a[i] = T(1);
            b[i] = T(1);
          }
        } else {
  #pragma unroll
          for (int i = 0; i < 4; ++i) damp3(p.eta_c, dxy2[i] + dz * dz, a[i], b[i]);
        }

        const int zm = z - nb;
        const bool zmod = (zm >= 0) && (zm < p.L.nz);   // uniform

        T g[4];
        if (BGM) {
  #pragma unroll
          for (int i = 0; i < 4; ++i) g[i] = kap4.v[i] * lapA[i] * p.inv_dt2;
        } else {
  #pragma unroll
          for (int i = 0; i < 4; ++i) g[i] = cur.g.v[i];
        }

        // cells past the grid's x extent (the last tile column) keep zero
        const V4<T>& aprev = cur.ap;
        V4<T> anew, ainc;
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const T cc = qa[(r + 4) % 9].v[i];
          if (BGM) {
            ainc.v[i] = b[i] * aprev.v[i] + a[i] * (kap4.v[i] * lapA[i]);
            anew.v[i] = cc + ainc.v[i];
          } else {
            const T src = (MODE == M_BORN) ? kap4.v[i] * (lapA[i] - cur.dm.v[i] * g[i]) : kap4.v[i] * lapA[i];
            anew.v[i] = a[i] * (T(2) * cc + src) - b[i] * aprev.v[i];
          }
          if (!xvalid[i]) {
            anew.v[i] = T(0);
            ainc.v[i] = T(0);
          }
        }
        bst4<NT3>(anew, rAn, lvo, sz_);
        if (BGM) bst4<NT3>(ainc, rAp, lvo, sz_);

        V4<T> bnew;
        if (TWO) {
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const T cc = qb[(r + 4) % 9].v[i];
            bnew.v[i] = a[i] * (T(2) * cc + kap4.v[i] * (lapB[i] - cur.dm.v[i] * g[i])) - b[i] * cur.bp.v[i];
            if (!xvalid[i]) bnew.v[i] = T(0);
          }
          bst4<NT3>(bnew, rBp, lvo, sz_);
        }

        if ((CK == CK_F32 || CK == CK_BF16) && BGM && ck_store >= 0 && act) {
          const long long co = ((long long)z * nyp + y) * p.cpitch + x;
          const long long lv = ((long long)ls * p.nck + ck_store) * 2;
          if (CK == CK_F32) {
            // one 16-byte store per level; the lane's cells past nxp land in the
            // checkpoint row's padding (cpitch is a multiple of 4), holding zero
            const Rsrc3 rc = rsrc3(static_cast<T*>(p.ck) + lv * p.cstride, 2 * p.cstride * (long long)sizeof(T));
            const unsigned cvo = (unsigned)co * esz;
            bst4(qa[(r + 4) % 9], rc, cvo, 0u);
            bst4(aprev, rc, cvo + (unsigned)(p.cstride * (long long)sizeof(T)), 0u);
          } else {
            const float* sc = p.ck_scale + lv;
            const float s0 = sc[0], s1 = sc[1];
            const float i0 = s0 > 0.0f ? 1.0f / s0 : 1.0f, i1 = s1 > 0.0f ? 1.0f / s1 : 1.0f;
            unsigned short h0[4], h1[4];
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float uc = (float)qa[(r + 4) % 9].v[i];
              h0[i] = bf16_rne(uc * i0);
              h1[i] = bf16_rne((float)aprev.v[i] * i1);
            }
            // one 8-byte store per level (cells past nxp: zero, into the row's padding)
            const Rsrc3 rc = rsrc3(static_cast<unsigned short*>(p.ck) + lv * p.cstride, 2 * p.cstride * 2LL);
            const unsigned cvo = (unsigned)co * 2u;
            u32x2_3 w0, w1;
            w0.x = h0[0] | ((unsigned)h0[1] << 16);
            w0.y = h0[2] | ((unsigned)h0[3] << 16);
            w1.x = h1[0] | ((unsigned)h1[1] << 16);
            w1.y = h1[2] | ((unsigned)h1[3] << 16);
            __builtin_amdgcn_raw_buffer_store_b64(w0, rc, cvo, 0u, 0);
            __builtin_amdgcn_raw_buffer_store_b64(w1, rc, cvo + (unsigned)(p.cstride * 2LL), 0u, 0);
          }
        }
        if (CK == CK_BF16 && BGM && ck_max >= 0 && act) {
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            mx0 = fmaxf(mx0, fabsf((float)anew.v[i]));   // zero past the grid
            mx1 = fmaxf(mx1, fabsf((float)ainc.v[i]));
          }
        }

        if (hslot >= 0 && BGM && zmod) {   // g^n, or u^{n+1} for the summed-by-parts imaging
          V4<T> gg;
  #pragma unroll
          for (int i = 0; i < 4; ++i) gg.v[i] = xmod[i] ? (p.hist_u ? anew.v[i] : g[i]) : T(0);   // model pad columns keep zero
          bst4<NT3>(gg, rG, gvo + (unsigned)zm * gplane, 0u);
        }

        if ((MODE == M_FUSED || MODE == M_BORN) && recrow && act && live) {
          T* drow = p.data + ((long long)shot * p.nt + n) * p.nr;
  #pragma unroll
          for (int i = 0; i < 4; ++i)
            if (rm[i] >= 0) drow[rm[i]] = TWO ? bnew.v[i] : anew.v[i];
        }
        if (MODE == M_BG && p.rec_bg != nullptr && recrow && act && live) {   // nonlinear modelling
          T* drow = p.rec_bg + ((long long)shot * p.nt + n) * p.nr;
  #pragma unroll
          for (int i = 0; i < 4; ++i)
            if (rm[i] >= 0) drow[rm[i]] = anew.v[i];
        }

        if (MODE == M_ADJ) {   // this half's contribution, added to the image one plane later
          V4<double> cw;
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double img = p.hist_u ? (double)(kap4.v[i] * lapA[i] * p.inv_dt2) : (double)anew.v[i];
            cw.v[i] = xmod[i] ? -((double)g[i] * img) : 0.0;
          }
          RED[half][z & 1][tid] = cw;
        }
        if (PF3) cur = nxt;
      }
    }
  }
  if (MODE == M_ADJ) {   // the item's last plane
    lds_barrier();
    const int zl = zs + (nit - 1) * dz3;
    pair_image(zl, bld4<NT3>(rI, ivo + (unsigned)(zl - nb) * iplane, 0u, double(0)));
  }
  if (CK == CK_BF16 && (MODE == M_FUSED || MODE == M_BG) && ck_max >= 0) {
    for (int o = 32; o > 0; o >>= 1) {
      mx0 = fmaxf(mx0, __shfl_xor(mx0, o));
      mx1 = fmaxf(mx1, __shfl_xor(mx1, o));
    }
    if (lane == 0) {
      unsigned int* sc = reinterpret_cast<unsigned int*>(p.ck_scale + ((long long)ls * p.nck + ck_max) * 2);
      atomicMax(sc, __float_as_uint(mx0));
      atomicMax(sc + 1, __float_as_uint(mx1));
    }
  }
  }   // items
}

static int device_cus3() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      ncu = v;
    else
      ncu = 256;
  }
  return ncu;
}

template <typename T, int MODE, int CK>
static void go3(const Step<T>& p, int n, int hslot, int cs, int cm, hipStream_t st) {
  static int occ = 0;   // resident workgroups per CU
  if (occ == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_step3d<T, MODE, CK>, 512, 0) != hipSuccess || b < 1) b = 1;
    occ = b;
  }
  const long long resident = std::max(8LL, (long long)device_cus3() * occ / 8 * 8);
  const long long grid = std::min<long long>(xcd_grid(p.nwg), resident);
  hipLaunchKernelGGL((k_step3d<T, MODE, CK>), dim3((unsigned)grid), dim3(512), 0, st, p, n, hslot, cs, cm);
}

template <typename T>
static void launch3(int mode, const Step<T>& p, int n, int hs, int ck, int cs, int cm, hipStream_t st) {
  switch (mode) {
    case M_FUSED:
      if (ck == CK_F32) go3<T, M_FUSED, CK_F32>(p, n, hs, cs, cm, st);
      else if (ck == CK_BF16) go3<T, M_FUSED, CK_BF16>(p, n, hs, cs, cm, st);
      else go3<T, M_FUSED, CK_NONE>(p, n, hs, -1, -1, st);
      break;
    case M_BG:
      if (ck == CK_F32) go3<T, M_BG, CK_F32>(p, n, hs, cs, cm, st);
      else if (ck == CK_BF16) go3<T, M_BG, CK_BF16>(p, n, hs, cs, cm, st);
      else if (ck == CK_LF32) go3<T, M_BG, CK_LF32>(p, n, hs, cs, -1, st);
      else if (ck == CK_LBF16) go3<T, M_BG, CK_LBF16>(p, n, hs, cs, -1, st);
      else go3<T, M_BG, CK_NONE>(p, n, hs, -1, -1, st);
      break;
    case M_BORN: go3<T, M_BORN, CK_NONE>(p, n, hs, -1, -1, st); break;
    default: go3<T, M_ADJ, CK_NONE>(p, n, hs, -1, -1, st); break;
  }
}

void step3d(int mode, const Step<float>& p, int n, int hs, int ck, int cs, int cm, hipStream_t s) {
  launch3(mode, p, n, hs, ck, cs, cm, s);
}
void step3d(int mode, const Step<double>& p, int n, int hs, int ck, int cs, int cm, hipStream_t s) {
  launch3(mode, p, n, hs, ck, cs, cm, s);
}

}  // namespace mp
