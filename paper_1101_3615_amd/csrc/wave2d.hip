// 2D sweep kernels of the Born / reverse-time sweeps (gfx950): one or two time
// steps per launch.
//
// Decomposition.  A wavefront owns an x strip of 64 lanes x 2 cells and a chunk
// of rows [z0, z1) in z.  Lanes 4..59 (SW2 = 112 cells) are the strip's output;
// lanes 0-3 and 60-63 are an 8-cell x halo, enough for two steps of the
// radius-4 stencil without loading any halo separately.  With two steps per
// launch the wave computes the intermediate level on its chunk widened by 4 rows
// above and below (from level-0 rows [z0-8, z1+8)), and level 2 on [z0, z1), so
// it needs nothing that another wave computes; neighbouring chunks march in
// opposite directions so that they read their shared rows at the same time.
// Recomputed halo values come from the same inputs through the same roundings as
// in the wave that owns the cell, and outputs go to other buffers than the
// inputs, which neighbouring waves are still reading.
//
// Rows march in z through 9-row register queues (level 0 and level 1); x
// neighbours come from adjacent lanes through DPP wavefront shifts.  The GW2 waves
// of a workgroup take GW2 shots on one strip and chunk, so the rows of the arrays
// all shots share hit in L1/L2 (LDS only for the background's level-1 increment and
// the adjoint's group image).  Row indices are uniform across
// the wavefront.  Rows outside [0, nzp) are zero and never read; cells outside
// [0, nxp) read as zero from the ghost columns and are never written.
//
// Scheme (damped leapfrog, 8th-order Laplacian, fields zero outside the grid):
//   background  Lam = L u + f,  g = c^2 Lam,  D+ = b D + a kappa Lam,  u+ = u + D+
//               (u+ = a (2u + kappa Lam) - b u- written with the increment D = u - u-)
//   Born        du+ = a (2 du + kappa (L du - dm g)) - b du-          (Sec. 2)
//   adjoint     nu  = a (2 nu' + kappa (L nu' + R^T d)) - b nu''      (exact transpose)
//   imaging     I  -= g^{k-1} nu^k                                    (FP64, per group of 4 shots)
//               or, with the background levels u^k in the slots (checkpoint recomputation),
//               I  -= u^k c^2 (L nu^{k+1} + R^T d^{k-1}): the same sum over k taken by parts
//               in time (u^0 = u^{-1} = 0 = nu^{nt+1} = nu^{nt+2}), in which the rounding
//               of a stored level is not amplified by the Laplacian
#include <algorithm>
#include <cmath>

#include "common.h"
#include "wave.h"

namespace mp {

template <typename T>
struct alignas(2 * sizeof(T)) V2 {
  T v[2];
};
template <typename T>
__device__ __forceinline__ V2<T> ld2(const T* p) {
  return *reinterpret_cast<const V2<T>*>(p);
}
template <typename T>
__device__ __forceinline__ void st2(T* p, const V2<T>& v) {
  *reinterpret_cast<V2<T>*>(p) = v;
}
template <typename T>
__device__ __forceinline__ V2<T> zero2() {
  V2<T> r;
  r.v[0] = T(0);
  r.v[1] = T(0);
  return r;
}

// Buffer-resource access (raw buffers: byte offsets, a per-lane offset plus a
// wave-uniform one, hardware range check against the resource's size; reads
// past it return zero, writes past it are dropped).  Word 3 of the resource is
// the gfx9-family raw-buffer configuration (32-bit data format).
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ Rsrc rsrc(const void* base, long long bytes) {
  const int n = bytes >= 0xffffffffLL ? -1 : (int)(unsigned)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}
template <int CP = 0>
__device__ __forceinline__ V2<float> bld2(Rsrc r, unsigned vo, unsigned so, float) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, CP);
  V2<float> o;
  o.v[0] = __uint_as_float(v.x);
  o.v[1] = __uint_as_float(v.y);
  return o;
}
template <int CP = 0>
__device__ __forceinline__ V2<double> bld2(Rsrc r, unsigned vo, unsigned so, double) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, CP);
  V2<double> o;
  o.v[0] = __longlong_as_double(((long long)v.y << 32) | v.x);
  o.v[1] = __longlong_as_double(((long long)v.w << 32) | v.z);
  return o;
}
template <int CP = 0>
__device__ __forceinline__ void bst2(const V2<float>& a, Rsrc r, unsigned vo, unsigned so) {
  u32x2 v;
  v.x = __float_as_uint(a.v[0]);
  v.y = __float_as_uint(a.v[1]);
  __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bst2(const V2<double>& a, Rsrc r, unsigned vo, unsigned so) {
  const long long b0 = __double_as_longlong(a.v[0]), b1 = __double_as_longlong(a.v[1]);
  u32x4 v;
  v.x = (unsigned)b0;
  v.y = (unsigned)(b0 >> 32);
  v.z = (unsigned)b1;
  v.w = (unsigned)(b1 >> 32);
  __builtin_amdgcn_raw_buffer_store_b128(v, r, vo, so, CP);
}
// Cells x-4 .. x+5 around the lane's pair (x, x+1): the pairs of lanes l-2, l-1,
// l, l+1, l+2 (lanes past either end of the wavefront read zero; their results
// are not used).
template <typename T>
__device__ __forceinline__ T mov_shr1(T v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
template <typename T>
__device__ __forceinline__ T mov_shl1(T v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}
template <>
__device__ __forceinline__ double mov_shr1<double>(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <>
__device__ __forceinline__ double mov_shl1<double>(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Products and fused multiply-adds with the rounding spelled out, so that the
// damped and undamped forms of the update below give the same bits where a = b = 1.
// A product is rounded on its own: the pragma keeps the compiler from fusing it
// into a later add (which it may do with a plain product, at some unrolled copies
// of the march body and not at others).
__device__ __forceinline__ float rmul(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ double rmul(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ float rfma(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double rfma(double a, double b, double c) { return __fma_rn(a, b, c); }

// First differences along x around the lane's two cells (2L, 2L+1):
// X[j] = u_{2L-3+j} - u_{2L-4+j}, j = 0..8 (lanes L-2 .. L+2 via DPP shifts).
template <typename T>
__device__ __forceinline__ void xdiff(const V2<T>& C, T X[9]) {
  const T e0 = C.v[1] - C.v[0];
  const T e1 = mov_shl1(C.v[0]) - C.v[1];
  X[4] = e0;
  X[5] = e1;
  X[2] = mov_shr1(e0);
  X[3] = mov_shr1(e1);
  X[0] = mov_shr1(X[2]);
  X[1] = mov_shr1(X[3]);
  X[6] = mov_shl1(e0);
  X[7] = mov_shl1(e1);
  X[8] = mov_shl1(X[6]);
}

// 8th-order Laplacian of the lane's two cells from first differences.  With
// e_m = u_{m+1} - u_m, the pair term (u_{x+j} - u_x) + (u_{x-j} - u_x) equals
// sum_{k<j} (e_{x+k} - e_{x-1-k}), so
//   sum_j c_j [pairs along x and z] = sum_k t_k [(e_{x+k} - e_{x-1-k}) + (same along z)]
// with the tail sums t_k = c_{k+1} + ... + c_4 (the smallest first).  In FP32 it
// rounds relative to the differences, not to u, which keeps smooth, well-resolved
// fields accurate over thousands of steps, and each difference is formed once per
// cell instead of once per weight.  E[(rb + m) % 9] holds row(m + 1) - row(m) of
// the queue (rows in march order, the centre is row 4); a march in the other
// direction negates every difference, which leaves each result bit unchanged.
template <typename T>
__device__ __forceinline__ void lapE(const T (&X)[9], const V2<T>* E, int rb, const Step<T>& p, T out[2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    T s = p.t3 * ((X[7 + i] - X[0 + i]) + (E[(rb + 7) % 9].v[i] - E[(rb + 0) % 9].v[i]));
    s = rfma(p.t2, (X[6 + i] - X[1 + i]) + (E[(rb + 6) % 9].v[i] - E[(rb + 1) % 9].v[i]), s);
    s = rfma(p.t1, (X[5 + i] - X[2 + i]) + (E[(rb + 5) % 9].v[i] - E[(rb + 2) % 9].v[i]), s);
    s = rfma(p.t0, (X[4 + i] - X[3 + i]) + (E[(rb + 4) % 9].v[i] - E[(rb + 3) % 9].v[i]), s);
    out[i] = s;
  }
}

// Leapfrog update of one pair with damping (a, b).
//   background: t = kappa Lam, nd = b D + a t, nv = u + nd
//   Born:       nv = a (2c + kappa (L - dm g)) - b prev
//   adjoint:    nv = a (2c + kappa L) - b prev
// Outside the layer (a = b = 1) the multiplications by one are dropped; every
// other operation is rounded as in the damped form.
template <typename T, int MODE, bool DAMP>
__device__ __forceinline__ void update(const T lap[2], const V2<T>& c, const V2<T>& prev, const V2<T>& kap,
                                       const T* a, const T* b, const T g[2], const V2<T>& dm, V2<T>& nv,
                                       V2<T>& nd) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (MODE == M_BG) {
      const T t = rmul(kap.v[i], lap[i]);
      nd.v[i] = DAMP ? rfma(b[i], prev.v[i], rmul(a[i], t)) : prev.v[i] + t;
      nv.v[i] = c.v[i] + nd.v[i];
    } else {
      const T src = (MODE == M_BORN) ? rmul(kap.v[i], rfma(-dm.v[i], g[i], lap[i])) : rmul(kap.v[i], lap[i]);
      const T X = rfma(T(2), c.v[i], src);
      nv.v[i] = DAMP ? rfma(a[i], X, -rmul(b[i], prev.v[i])) : X - prev.v[i];
    }
  }
}

// Inputs of one loop iteration (level 1 on row z, level 2 on row z - 4d for the
// march direction d = +-1), loaded one or two iterations ahead so that their
// latency overlaps the work of the rows before.
// Every load is unconditional: rows outside the grid and lanes outside the
// model fall outside their buffer resource and read zero.
template <typename T>
struct RowIn {
  V2<T> q;          // level-0 row z + 4d (enters the queue)
  V2<T> pv;         // row z: level -1 (Born, adjoint) or background increment D^n
  V2<T> k1;         // kappa on row z (row z - 4d of level 2: kept from four rows back)
  V2<T> m1;         // Born: extended perturbation on row z (likewise)
  V2<T> g1, g2;     // Born: g^n (row z), g^{n+1} (row z - 4d); adjoint: g^{k-1}, g^{k-2} (imaging row)
  V2<double> im;    // adjoint: image pair on the imaging row
};

// Per-lane byte offset that every buffer access of an inactive lane uses: past
// the end of any resource, so reads return zero and writes are dropped.
// cache policy of g and the image (read or written once per launch, never reused
// from L2 or the last-level cache): non-temporal
constexpr int NT2 = 2;
constexpr unsigned OFF_NONE = 0x80000000u;

// Damping of the 2D sweeps: e = (eta_x + eta_z) dt / 2 = ec (dx^2 + dz^2) with dx, dz
// the cell's distances into the layer and ec = eta_max dt / (2 nb^2); a = 1 / (1 + e),
// b = (1 - e) a.  a = b = 1 exactly where e = 0.
__device__ __forceinline__ void damp_ab(float ec, int dd, float& a, float& b) {
  const float e = ec * (float)dd;
  a = dd > 0 ? __builtin_amdgcn_rcpf(1.0f + e) : 1.0f;
  b = (1.0f - e) * a;
}
__device__ __forceinline__ void damp_ab(double ec, int dd, double& a, double& b) {
  const double e = ec * (double)dd;
  a = dd > 0 ? 1.0 / (1.0 + e) : 1.0;
  b = (1.0 - e) * a;
}
__device__ __forceinline__ int layer_depth(int i, int n, int nb) { return max(max(nb - i, i - (n + nb - 1)), 0); }

// One launch of NS (1 or 2) time steps of every shot of a wave.
//   M_BG:   in0 = u^n, in1 = D^n            -> out0 = u^{n+NS}, out1 = D^{n+NS};
//           g^n -> slot hs1, g^{n+1} -> slot hs2 (a negative slot is not written);
//           checkpoint ck_store <- (u^n, D^n); BF16 maxima of the last level -> ck_max;
//           with rec_bg set, records u^{n+1}(x_r), u^{n+2}(x_r) (nonlinear modelling).
//   M_BORN: in0 = du^n, in1 = du^{n-1}      -> out0 = du^{n+1}, out1 = du^{n+2};
//           reads g^n (hs1), g^{n+1} (hs2); records d[n], d[n+1].
//   M_ADJ:  in0 = nu^{k+1}, in1 = nu^{k+2}  -> out0 = nu^k, out1 = nu^{k-1}  (n = k);
//           injects d[k-1], d[k-2]; images with g^{k-1} (hs1), g^{k-2} (hs2).
//
// Lane l holds cells x = strip * SW2 - 2 HL2 + 2 l and x + 1.  Field rows are
// read through buffer resources that cover exactly rows [0, nzp) of the strip:
// the row pitch covers every lane of every strip and cells outside the grid are
// zero ghost cells, rows outside the grid fall outside the resource.  Every
// value computed for a cell outside the grid is replaced by zero.  Row indices
// are wave-uniform.
template <typename T, int MODE, int NS, int CK>
__global__ __launch_bounds__(64 * GW2) void k_sweep2d(Step<T> p, int n, int hs1, int hs2, int ck_store, int ck_max) {
  constexpr bool BG = (MODE == M_BG);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = xcd_item(p.nwg);
  if (item >= p.nwg) return;
  // workgroup = GW2 shots on one (strip, chunk): the rows of the arrays they
  // share (kappa, perturbation) are read by its waves together
  const int chunk = item % p.nchunks;
  const int rest = item / p.nchunks;
  const int strip = rest % p.L.nstrips;
  const int ls = (rest / p.L.nstrips) * GW2 + wv;   // the launch holds whole groups of GW2 shots
  const int nzp = p.L.nzp;
  const int nxp = p.L.nxp;
  const int nb = p.L.nb;
  const int nz = p.L.nz;
  const int z0 = chunk * p.zc;
  const int z1 = min(z0 + p.zc, nzp);
  const long long pitch = p.L.pitch;
  const int shot = p.shot0 + ls;

  const int sx0 = strip * SW2 - 2 * HL2;                 // first cell of lane 0 (uniform)
  const int x = sx0 + 2 * lane;                          // first cell of the lane's pair
  const bool xin = (x >= 0) && (x < nxp);
  const bool outl = xin && (lane >= HL2) && (lane < LANES - HL2);
  const bool xv1 = x + 1 < nxp;
  const bool all_in = (sx0 >= 0) && (sx0 + 2 * LANES <= nxp);               // every cell of the strip is in the grid
  const bool x_free = (sx0 >= nb) && (sx0 + 2 * LANES <= nxp - nb);          // no damping along x in the strip
  int dx2[2];                                                                // squared layer distance along x
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int dxi = layer_depth(x + i, p.L.nx, nb);
    dx2[i] = dxi * dxi;
  }
  const int xm = x - nb;                                                     // model column of the pair
  const bool xmod = (xm >= 0) && (xm < p.L.nx);
  const bool xmod1 = xm + 1 < p.L.nx;
  int sx = -1, sz = -1;
  if (BG) {
    sx = p.srcx[shot];
    sz = p.srcz[shot];
  }
  // a null shot (no source: padding of a group) records and injects no data
  const bool live = p.srcx[shot] >= 0;
  T* const recbg = BG ? p.rec_bg : nullptr;   // background traces (modelling), uniform
  const bool rec = !BG || recbg != nullptr;    // whether receiver rows are looked up

  // field resources based at the strip's cell (sx0, 0), nzp rows long
  const long long kofs = (long long)SLACK + (long long)GZ * pitch + XL + sx0;
  const long long fo = (long long)ls * p.L.fstride + kofs;
  const unsigned rowb = (unsigned)(pitch * (long long)sizeof(T));
  const long long fbytes = (long long)nzp * rowb;
  const Rsrc rI0 = rsrc(p.in0 + fo, fbytes);
  const Rsrc rI1 = rsrc(p.in1 + fo, fbytes);
  const Rsrc rO0 = rsrc(p.out0 + fo, fbytes);
  const Rsrc rO1 = rsrc(p.out1 + fo, fbytes);
  const Rsrc rK = rsrc(p.kappa + kofs, fbytes);
  const Rsrc rM = rsrc(p.dmbar + (long long)p.dm_slot[shot] * p.L.fstride + kofs, fbytes);
  const unsigned vo = (unsigned)(2 * lane) * (unsigned)sizeof(T);          // lane offset in a field row
  const unsigned vs = outl ? vo : OFF_NONE;                                  // ... for stores
  // model resources (g slots, image): nz rows of mpitch from model column 0
  const long long hbase = (long long)(p.hmod > 0 ? ls % p.hmod : ls) * p.hstride;
  const long long mbytes = (long long)nz * p.L.mpitch * (long long)sizeof(T);
  const int mxl = p.L.mxl;
  const Rsrc rH1 = rsrc(hs1 >= 0 ? p.hist + hbase + (long long)hs1 * p.L.mstride + mxl : p.hist, hs1 >= 0 ? mbytes : 0);
  const Rsrc rH2 = rsrc(hs2 >= 0 ? p.hist + hbase + (long long)hs2 * p.L.mstride + mxl : p.hist, hs2 >= 0 ? mbytes : 0);
  // adjoint: one FP64 image per group of GW2 consecutive shots (the workgroup)
  const Rsrc rIm = rsrc(MODE == M_ADJ ? p.img + (long long)((unsigned)shot / GW2) * p.L.mstride + mxl : p.img,
                        MODE == M_ADJ ? (long long)nz * p.L.mpitch * 8 : 0);
  const unsigned mrowb = (unsigned)p.L.mpitch * (unsigned)sizeof(T);
  const unsigned gvo = xmod ? (unsigned)xm * (unsigned)sizeof(T) : OFF_NONE;             // g on every lane
  const unsigned gvs = (xmod && outl) ? (unsigned)xm * (unsigned)sizeof(T) : OFF_NONE;   // g on output lanes
  const unsigned irowb = (unsigned)p.L.mpitch * 8u;
  // Imaging of the group: the GW2 waves' contributions to a row are summed in LDS
  // in shot order, then wave w updates the image of lane pairs PPW*w .. PPW*w + PPW-1
  // (lanes 0..PPW-1 of the wave).  gj: the pair this lane updates.
  constexpr int PPW = LANES / GW2;
  __shared__ V2<double> red[(MODE == M_ADJ) ? 2 : 1][GW2][(MODE == M_ADJ) ? LANES : 1];
  const int gj = wv * PPW + (lane & (PPW - 1));
  const int gx = sx0 + 2 * gj;
  const bool gout = (lane < PPW) && (gj >= HL2) && (gj < LANES - HL2) && (gx < nxp) && (gx - nb >= 0) &&
                    (gx - nb < p.L.nx);
  const unsigned ivo = gout ? (unsigned)(gx - nb) * 8u : OFF_NONE;
  int rbuf = 0;
  auto image = [&](int zm, const V2<double>& cw, const V2<double>& old) {
    red[rbuf][wv][lane] = cw;
    lds_barrier();
    if (lane < PPW) {
      V2<double> acc = old;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        double sum = red[rbuf][0][gj].v[i];
#pragma unroll
        for (int w = 1; w < GW2; ++w) sum += red[rbuf][w][gj].v[i];
        acc.v[i] += sum;
      }
      bst2<NT2>(acc, rIm, ivo + (unsigned)zm * irowb, 0u);
    }
    rbuf ^= 1;
  };
  float mx0 = 0.0f, mx1 = 0.0f;   // BF16 checkpoints: running max |u|, |D| of the last level

  // row offsets wrap to past the end of the resource for rows above the grid
  auto frow = [&](int z) -> unsigned { return vo + (unsigned)z * rowb; };
  // Input levels (u^n, D^n): the field slices, or (CK_LF32 / CK_LBF16) checkpoint
  // ck_store in its compact layout [z][cpitch], converted as the expansion pass
  // would (same bits).  A lane outside [0, nxp) and rows outside [0, nzp) read zero
  // through the range check; a pair never reaches past a compact row (x is even,
  // and cpitch > nxp when nxp is odd).
  constexpr bool LDCK = (CK == CK_LF32 || CK == CK_LBF16);
  constexpr unsigned cesz = (CK == CK_LBF16) ? 2u : (unsigned)sizeof(T);
  const long long lvl = ((long long)ls * p.nck + max(ck_store, 0)) * 2;
  const Rsrc rC0 = rsrc(LDCK ? static_cast<char*>(p.ck) + lvl * p.cstride * cesz : static_cast<char*>(p.ck),
                        LDCK ? p.cstride * (long long)cesz : 0);
  const Rsrc rC1 = rsrc(LDCK ? static_cast<char*>(p.ck) + (lvl + 1) * p.cstride * cesz : static_cast<char*>(p.ck),
                        LDCK ? p.cstride * (long long)cesz : 0);
  const unsigned cvo = xin ? (unsigned)x * cesz : OFF_NONE;
  const unsigned crow = (unsigned)p.cpitch * cesz;
  float cs0 = 1.0f, cs1 = 1.0f;
  if (CK == CK_LBF16) {
    cs0 = p.ck_scale[lvl];
    cs1 = p.ck_scale[lvl + 1];
  }
  auto in_row = [&](int lev, int z) -> V2<T> {
    if (!LDCK) return bld2(lev ? rI1 : rI0, frow(z), 0u, T(0));
    if (CK == CK_LF32) return bld2(lev ? rC1 : rC0, cvo + (unsigned)z * crow, 0u, T(0));
    const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(lev ? rC1 : rC0, cvo + (unsigned)z * crow, 0u, 0);
    const float sc = lev ? cs1 : cs0;
    V2<T> r;
    r.v[0] = (T)bf16_scaled((unsigned short)(w & 0xffffu), sc);
    r.v[1] = (T)bf16_scaled((unsigned short)(w >> 16), sc);
    return r;
  };
  // g rows: a pair that ends past nx stores zero into the model row's pad column,
  // so loads of such a pair need no mask
  auto gld = [&](const Rsrc& r, unsigned vo_lane, int zm) -> V2<T> {
    return bld2<NT2>(r, vo_lane + (unsigned)zm * mrowb, 0u, T(0));
  };
  auto gst = [&](const Rsrc& r, int zm, const T g[2]) {
    V2<T> gg;
    gg.v[0] = g[0];
    gg.v[1] = xmod1 ? g[1] : T(0);
    bst2<NT2>(gg, r, gvs + (unsigned)zm * mrowb, 0u);
  };
  // receiver indices of the pair on row z (-1: none); false if the row has none
  auto recs = [&](int z, int rm[2]) -> bool {
    rm[0] = rm[1] = -1;
    if (z < p.rec_lo || z > p.rec_hi) return false;   // no lookup outside the receiver rows
    const int rp = p.recplane[z];
    if (rp < 0) return false;
    if (xin) {
      const int2 m2 = *reinterpret_cast<const int2*>(p.recmap + (long long)rp * p.cpitch + x);
      rm[0] = m2.x;
      rm[1] = xv1 ? m2.y : -1;
    }
    return true;
  };
  // FP32 / BF16 checkpoint of (u^n, D^n) on an output row (the pad column of the
  // compact rows absorbs a zero past nxp)
  const long long lv = ((long long)ls * p.nck + max(ck_store, 0)) * 2;   // checkpoint level pair
  float i0 = 1.0f, i1 = 1.0f;   // BF16: reciprocal scales of the stored levels
  if (CK == CK_BF16 && ck_store >= 0) {
    const float s0 = p.ck_scale[lv], s1 = p.ck_scale[lv + 1];
    if (s0 > 0.0f) i0 = 1.0f / s0;
    if (s1 > 0.0f) i1 = 1.0f / s1;
  }
  auto ckstore = [&](int z, const V2<T>& u, const V2<T>& d) {
    if (!outl) return;
    const long long co = (long long)z * p.cpitch + x;
    if (CK == CK_F32) {
      T* c0 = static_cast<T*>(p.ck) + lv * p.cstride + co;
      st2(c0, u);
      st2(c0 + p.cstride, d);
    } else if (CK == CK_BF16) {
      unsigned short* c0 = static_cast<unsigned short*>(p.ck) + lv * p.cstride + co;
      const unsigned short a0 = bf16_rne((float)u.v[0] * i0), a1 = bf16_rne((float)u.v[1] * i0);
      const unsigned short b0 = bf16_rne((float)d.v[0] * i1), b1 = bf16_rne((float)d.v[1] * i1);
      *reinterpret_cast<unsigned int*>(c0) = a0 | ((unsigned)a1 << 16);
      *reinterpret_cast<unsigned int*>(c0 + p.cstride) = b0 | ((unsigned)b1 << 16);
    }
  };
  auto track = [&](const V2<T>& u, const V2<T>& d) {
    if (outl) {
      mx0 = fmaxf(mx0, fmaxf(fabsf((float)u.v[0]), fabsf((float)u.v[1])));
      mx1 = fmaxf(mx1, fmaxf(fabsf((float)d.v[0]), fabsf((float)d.v[1])));
    }
  };
  // one level on row z from the centre pair c, its Laplacian, kappa, dm and the previous level
  auto level = [&](int z, const V2<T>& c, T lap[2], const V2<T>& kp, const V2<T>& dm, const V2<T>& pv,
                   const T g[2], V2<T>& nv, V2<T>& nd) {
    const int dz = layer_depth(z, nz, nb);
    if (x_free && dz == 0) {
      update<T, MODE, false>(lap, c, pv, kp, nullptr, nullptr, g, dm, nv, nd);
    } else {
      T a[2], b[2];
      damp_ab(p.eta_c, dx2[0] + dz * dz, a[0], b[0]);
      damp_ab(p.eta_c, dx2[1] + dz * dz, a[1], b[1]);
      update<T, MODE, true>(lap, c, pv, kp, a, b, g, dm, nv, nd);
    }
    if (!all_in) {
      if (!xin) {
        nv = zero2<T>();
        nd = zero2<T>();
      } else if (!xv1) {
        nv.v[1] = T(0);
        nd.v[1] = T(0);
      }
    }
  };
  // March direction: even chunks with z increasing, odd chunks with z decreasing, so that
  // two neighbouring chunks reach the rows around their shared boundary at the
  // same time and the second reads of those rows hit in L2.  The queue holds rows
  // in march order; the Laplacian sums each symmetric pair commutatively, so the
  // direction does not change any result bit.
  const int d = (chunk & 1) ? -1 : 1;
  const int nit = (z1 - z0) + ((NS == 2) ? 8 : 0);          // level-1 rows of the march
  const int zs = (d > 0) ? ((NS == 2) ? z0 - 4 : z0) : ((NS == 2) ? z1 + 3 : z1 - 1);
  auto fetch = [&](int z, RowIn<T>& f) {
    f.q = in_row(0, z + 4 * d);
    f.pv = in_row(1, z);
    f.k1 = bld2(rK, frow(z), 0u, T(0));
    if (MODE == M_BORN) {
      f.m1 = bld2(rM, frow(z), 0u, T(0));
      f.g1 = gld(rH1, gvo, z - nb);   // level 1 runs on the halo lanes too
    }
    if (NS == 2 && MODE == M_BORN) f.g2 = gld(rH2, gvs, z - 4 * d - nb);
    if (MODE == M_ADJ) {
      const int zm = (NS == 2 ? z - 4 * d : z) - nb;   // imaging row
      f.g1 = gld(rH1, gvs, zm);
      if (NS == 2) f.g2 = gld(rH2, gvs, zm);
      f.im = bld2<NT2>(rIm, ivo + (unsigned)zm * irowb, 0u, 0.0);
    }
  };

  V2<T> q0[9], q1[9];   // level-0 rows, level-1 rows
  V2<T> e0[9], e1[9];   // their first differences along the march
  V2<T> kq[9], mq[9];   // kappa and (Born) perturbation / (adjoint) c^2 Lam of the level-1 rows, for level 2
  auto diff = [](const V2<T>& a, const V2<T>& b) {
    V2<T> r;
    r.v[0] = a.v[0] - b.v[0];
    r.v[1] = a.v[1] - b.v[1];
    return r;
  };
  // background: the increment D^{n+1} of level-1 rows, read back four rows later
  // at the centre of level 2 (kept in LDS: each wave reads only its own entries)
  __shared__ V2<T> dq[(BG && NS == 2) ? GW2 : 1][9][(BG && NS == 2) ? LANES : 1];
#pragma unroll
  for (int s = 0; s < 8; ++s) q0[s] = in_row(0, zs + (s - 4) * d);
#pragma unroll
  for (int s = 0; s < 7; ++s) e0[s] = diff(q0[s + 1], q0[s]);
  if (NS == 2) q1[8] = zero2<T>();
  // prefetch depth: two rows for the background kernel (fewer loads per row, more
  // latency to cover), one row for the Born and adjoint kernels
  constexpr int PF = BG ? 2 : 1;
  RowIn<T> cur, nx1, nx2;   // inputs of this iteration and of the next PF
  fetch(zs, cur);
  if (PF == 2) fetch(zs + d, nx1);

  for (int tb = 0; tb < nit; tb += 9) {
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int t = tb + r;   // iteration: level 1 on row z, level 2 on row z - 4d
      if (t >= nit) break;
      const int z = zs + t * d;
      if (PF == 2) fetch(z + 2 * d, nx2);
      else fetch(z + d, nx1);
      q0[(r + 8) % 9] = cur.q;
      if (NS == 2) {   // level 2 reaches row z four iterations from now
        kq[r] = cur.k1;
        if (MODE == M_BORN) mq[r] = cur.m1;
      }
      e0[(r + 7) % 9] = diff(q0[(r + 8) % 9], q0[(r + 7) % 9]);
      const bool out_row = (z >= z0) && (z < z1);

      // ---- level 1 on row z ----
      if (z >= 0 && z < nzp) {
        const unsigned so = (unsigned)z * rowb;
        const V2<T>& c0 = q0[(r + 4) % 9];
        T X[9];
        xdiff(c0, X);
        T lap[2];
        lapE(X, e0, r, p, lap);
        if (BG && z == sz) {
          const T ws = p.wav[n];
          if (x == sx) lap[0] += ws;
          if (x + 1 == sx) lap[1] += ws;
        }
        int rm[2] = {-1, -1};
        const bool recrow = rec && recs(z, rm);
        if (MODE == M_ADJ && recrow && live) {
          const T* drow = p.data + ((long long)shot * p.nt + (n - 1)) * p.nr;
          if (rm[0] >= 0) lap[0] += drow[rm[0]];
          if (rm[1] >= 0) lap[1] += drow[rm[1]];
        }
        T g[2];
        if (BG) {
          g[0] = rmul(rmul(cur.k1.v[0], lap[0]), p.inv_dt2);
          g[1] = rmul(rmul(cur.k1.v[1], lap[1]), p.inv_dt2);
        } else {
          g[0] = cur.g1.v[0];   // Born: g^n (unused by the adjoint update)
          g[1] = cur.g1.v[1];
        }
        V2<T> nv, nd;
        level(z, c0, lap, cur.k1, cur.m1, cur.pv, g, nv, nd);
        if (NS == 2) {
          q1[r] = nv;
          if (BG) dq[wv][r][lane] = nd;
          if (MODE == M_ADJ) {   // c^2 (L nu^{k+1} + R^T d) of the row, imaged at level 2
            mq[r].v[0] = rmul(rmul(cur.k1.v[0], lap[0]), p.inv_dt2);
            mq[r].v[1] = rmul(rmul(cur.k1.v[1], lap[1]), p.inv_dt2);
          }
        }
        if (out_row) {
          if (BG) {
            if ((CK == CK_F32 || CK == CK_BF16) && ck_store >= 0) ckstore(z, c0, cur.pv);
            gst(rH1, z - nb, p.hist_u ? nv.v : g);
            if (NS == 1) {
              bst2(nv, rO0, vs + so, 0u);
              bst2(nd, rO1, vs + so, 0u);
              if (CK == CK_BF16 && ck_max >= 0) track(nv, nd);
            }
            if (recrow && outl && live) {
              T* drow = recbg + ((long long)shot * p.nt + n) * p.nr;
              if (rm[0] >= 0) drow[rm[0]] = nv.v[0];
              if (rm[1] >= 0) drow[rm[1]] = nv.v[1];
            }
          } else {
            bst2(nv, rO0, vs + so, 0u);
            if (MODE == M_BORN && recrow && outl && live) {
              T* drow = p.data + ((long long)shot * p.nt + n) * p.nr;
              if (rm[0] >= 0) drow[rm[0]] = nv.v[0];
              if (rm[1] >= 0) drow[rm[1]] = nv.v[1];
            }
            if (MODE == M_ADJ && NS == 1) {
              const int zm = z - nb;
              if (zm >= 0 && zm < nz) {   // uniform over the workgroup
                V2<double> cw;
#pragma unroll
                for (int i = 0; i < 2; ++i)
                  cw.v[i] = p.hist_u ? -((double)cur.g1.v[i] * (double)rmul(rmul(cur.k1.v[i], lap[i]), p.inv_dt2))
                                     : -((double)cur.g1.v[i] * (double)nv.v[i]);
                image(zm, cw, cur.im);
              }
            }
          }
        }
      } else if (NS == 2) {
        q1[r] = zero2<T>();
        if (BG) dq[wv][r][lane] = zero2<T>();
        if (MODE == M_ADJ) mq[r] = zero2<T>();
      }
      if (NS == 2) e1[(r + 8) % 9] = diff(q1[r], q1[(r + 8) % 9]);

      // ---- level 2 on row z - 4d ----
      if (NS == 2 && t >= 8) {
        const int y = z - 4 * d;
        const unsigned so = (unsigned)y * rowb;
        const V2<T>& c1 = q1[(r + 5) % 9];
        T X[9];
        xdiff(c1, X);
        T lap[2];
        lapE(X, e1, r + 1, p, lap);
        if (BG && y == sz) {
          const T ws = p.wav[n + 1];
          if (x == sx) lap[0] += ws;
          if (x + 1 == sx) lap[1] += ws;
        }
        int rm[2] = {-1, -1};
        const bool recrow = rec && recs(y, rm);
        if (MODE == M_ADJ && recrow && live) {
          const T* drow = p.data + ((long long)shot * p.nt + (n - 2)) * p.nr;
          if (rm[0] >= 0) lap[0] += drow[rm[0]];
          if (rm[1] >= 0) lap[1] += drow[rm[1]];
        }
        const V2<T> pv = BG ? dq[wv][(r + 5) % 9][lane] : q0[r % 9];
        T g[2];
        if (BG) {
          g[0] = rmul(rmul(kq[(r + 5) % 9].v[0], lap[0]), p.inv_dt2);
          g[1] = rmul(rmul(kq[(r + 5) % 9].v[1], lap[1]), p.inv_dt2);
        } else {
          g[0] = cur.g2.v[0];
          g[1] = cur.g2.v[1];
        }
        V2<T> nv, nd;
        level(y, c1, lap, kq[(r + 5) % 9], mq[(r + 5) % 9], pv, g, nv, nd);
        if (BG) {
          bst2(nv, rO0, vs + so, 0u);
          bst2(nd, rO1, vs + so, 0u);
          gst(rH2, y - nb, p.hist_u ? nv.v : g);
          if (CK == CK_BF16 && ck_max >= 0) track(nv, nd);
          if (recrow && outl && live) {
            T* drow = recbg + ((long long)shot * p.nt + n + 1) * p.nr;
            if (rm[0] >= 0) drow[rm[0]] = nv.v[0];
            if (rm[1] >= 0) drow[rm[1]] = nv.v[1];
          }
        } else {
          bst2(nv, rO1, vs + so, 0u);
          if (MODE == M_BORN && recrow && outl && live) {
            T* drow = p.data + ((long long)shot * p.nt + n + 1) * p.nr;
            if (rm[0] >= 0) drow[rm[0]] = nv.v[0];
            if (rm[1] >= 0) drow[rm[1]] = nv.v[1];
          }
          if (MODE == M_ADJ) {
            const int zm = y - nb;
            if (zm >= 0 && zm < nz) {   // uniform over the workgroup
              V2<double> cw;
#pragma unroll
              for (int i = 0; i < 2; ++i) {
                if (p.hist_u) {   // u^k with level 1's c^2 Lam, u^{k-1} with level 2's
                  cw.v[i] = -((double)cur.g1.v[i] * (double)mq[(r + 5) % 9].v[i]);
                  cw.v[i] -= (double)cur.g2.v[i] * (double)rmul(rmul(kq[(r + 5) % 9].v[i], lap[i]), p.inv_dt2);
                } else {
                  cw.v[i] = -((double)cur.g1.v[i] * (double)c1.v[i]);
                  cw.v[i] -= (double)cur.g2.v[i] * (double)nv.v[i];
                }
              }
              image(zm, cw, cur.im);
            }
          }
        }
      }
      cur = nx1;
      if (PF == 2) nx1 = nx2;
    }
  }
  if (CK == CK_BF16 && BG && ck_max >= 0) {
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
}

// ---- host side ----

static int device_cus() {
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

// z chunking: one wave per (shot, strip, chunk), GW2 shots per workgroup.
// Cost of a launch with nch chunks (calibrated on MI355X with four-wave
// workgroups): rounds x m^e x (zc + H), with m the four-wave units on the busiest
// CU in a round, zc the chunk
// height and H = 30 rows of halo traffic per two-step chunk (12 for one step).
// e = 0.7 for the Born and adjoint kernels, 0.38 for the background kernel,
// which gains more from a fuller CU.  One workgroup per CU (four waves) hides too
// little latency, so m counts as at least 2.  zc_fixed > 0 forces the chunk height.
template <typename T>
static void chunking(Step<T>& p, int mode, int nsh, int nsteps, int wg_per_cu, int zc_fixed) {
  const int nzp = p.L.nzp;
  const long long ncu = device_cus();
  const long long cap = ncu * std::max(1, wg_per_cu);
  const long long cols = (long long)((nsh + GW2 - 1) / GW2) * p.L.nstrips;
  const double ex = (mode == M_BG) ? 0.38 : 0.7;
  const double halo = (nsteps == 2) ? 30.0 : 12.0;
  int best_zc = nzp;
  double best = 1e300;
  for (int nch = 1; nch <= std::max(1, nzp / 4); ++nch) {
    const int zc = (nzp + nch - 1) / nch;
    if ((nzp + zc - 1) / zc != nch) continue;
    const long long wgs = cols * nch;
    const long long rounds = (wgs + cap - 1) / cap;
    const long long m = (wgs + rounds * ncu - 1) / (rounds * ncu);
    const long long m4 = m * GW2 / 4;   // in workgroups of four waves, the unit the model was fitted in
    const double cost = (double)rounds * std::pow((double)std::max<long long>(m4, 2), ex) * (zc + halo);
    if (cost < best) {
      best = cost;
      best_zc = zc;
    }
  }
  if (zc_fixed > 0) best_zc = std::min(zc_fixed, nzp);
  p.zc = best_zc;
  p.nchunks = (nzp + best_zc - 1) / best_zc;
  p.ngroups = 1;
  p.nsh = nsh;
  p.nwg = (int)(cols * p.nchunks);
}

template <typename T, int MODE, int NS, int CK>
static void go(Step<T> p, int nsh, int n, int hs1, int hs2, int cs, int cm, int zc_fixed, hipStream_t st) {
  static int occ = 0;   // resident workgroups per CU for this kernel
  if (occ == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_sweep2d<T, MODE, NS, CK>, 64 * GW2, 0) != hipSuccess || b < 1)
      b = 1;
    occ = b;
  }
  chunking(p, MODE, nsh, NS, occ, zc_fixed);
  hipLaunchKernelGGL((k_sweep2d<T, MODE, NS, CK>), dim3(xcd_grid(p.nwg)), dim3(64 * GW2), 0, st, p, n, hs1, hs2, cs, cm);
}

template <typename T, int MODE, int NS>
static void go_ck(int ck, const Step<T>& p, int nsh, int n, int hs1, int hs2, int cs, int cm, int zc, hipStream_t st) {
  if (MODE == M_BG && ck == CK_F32) go<T, MODE, NS, CK_F32>(p, nsh, n, hs1, hs2, cs, cm, zc, st);
  else if (MODE == M_BG && ck == CK_BF16) go<T, MODE, NS, CK_BF16>(p, nsh, n, hs1, hs2, cs, cm, zc, st);
  else if (MODE == M_BG && ck == CK_LF32) go<T, MODE, NS, CK_LF32>(p, nsh, n, hs1, hs2, cs, -1, zc, st);
  else if (MODE == M_BG && ck == CK_LBF16) go<T, MODE, NS, CK_LBF16>(p, nsh, n, hs1, hs2, cs, -1, zc, st);
  else go<T, MODE, NS, CK_NONE>(p, nsh, n, hs1, hs2, -1, -1, zc, st);
}

template <typename T>
static void sweep_t(int mode, int nsteps, int ck, const Step<T>& p, int nsh, int n, int hs1, int hs2, int cs,
                    int cm, int zc, hipStream_t st) {
  if (mode == M_BG) {
    if (nsteps == 2) go_ck<T, M_BG, 2>(ck, p, nsh, n, hs1, hs2, cs, cm, zc, st);
    else go_ck<T, M_BG, 1>(ck, p, nsh, n, hs1, hs2, cs, cm, zc, st);
  } else if (mode == M_BORN) {
    if (nsteps == 2) go<T, M_BORN, 2, CK_NONE>(p, nsh, n, hs1, hs2, -1, -1, zc, st);
    else go<T, M_BORN, 1, CK_NONE>(p, nsh, n, hs1, hs2, -1, -1, zc, st);
  } else {
    if (nsteps == 2) go<T, M_ADJ, 2, CK_NONE>(p, nsh, n, hs1, hs2, -1, -1, zc, st);
    else go<T, M_ADJ, 1, CK_NONE>(p, nsh, n, hs1, hs2, -1, -1, zc, st);
  }
}

void sweep2d(int mode, int nsteps, int ck, const Step<float>& p, int nsh, int n, int hs1, int hs2, int cs, int cm,
             int zc, hipStream_t s) {
  sweep_t(mode, nsteps, ck, p, nsh, n, hs1, hs2, cs, cm, zc, s);
}
void sweep2d(int mode, int nsteps, int ck, const Step<double>& p, int nsh, int n, int hs1, int hs2, int cs, int cm,
             int zc, hipStream_t s) {
  sweep_t(mode, nsteps, ck, p, nsh, n, hs1, hs2, cs, cm, zc, s);
}

}  // namespace mp
