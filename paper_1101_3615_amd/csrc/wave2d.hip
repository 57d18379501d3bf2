// 2D time-step kernels of the Born / reverse-time sweeps (gfx950).
//
// One wavefront owns a strip of 256 cells along x (4 per lane, 16-byte loads)
// and marches down a chunk of rows in z.  The 9 rows of the z-stencil sit in a
// register queue, the x-neighbours come from the adjacent lanes through DPP
// wavefront shifts, and the two lanes at the strip ends load the 4-cell halo.
// No LDS and no barriers: the four waves of a workgroup are independent and
// take consecutive z-chunks of the same strip, so their halo rows hit in L1/L2.
//
// Scheme (damped leapfrog, 8th-order Laplacian, fields zero outside the grid):
//   background  Lam = L u + f,  g = c^2 Lam,  u+ = a (2u + kappa Lam) - b u-
//   Born        du+ = a (2 du + kappa (L du - dm g)) - b du-        (Sec. 2)
//   adjoint     nu  = a (2 nu' + kappa (L nu' + R^T d)) - b nu''    (exact transpose)
//   imaging     I  -= g^{k-1} nu^k                                   (FP64)
#include "common.h"
#include "wave.h"

namespace mp {

// 8th-order Laplacian of the 4 cells of a lane in difference form:
// sum_j c_j [(u_{x-j} - u) + (u_{x+j} - u) + (u_{z-j} - u) + (u_{z+j} - u)], the
// smallest weights first.  Algebraically equal to c0 u + sum_j c_j (pairs);
// in FP32 it rounds relative to the differences instead of to u, which keeps
// smooth, well-resolved fields accurate over thousands of steps.
template <typename T>
__device__ __forceinline__ void lap_diff(const T (&w)[12], const V4<T>* q, int r, const Step<T>& p, T out[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T c = w[4 + i];
    T s = p.c4 * (((w[0 + i] - c) + (w[8 + i] - c)) + ((q[(r + 0) % 9].v[i] - c) + (q[(r + 8) % 9].v[i] - c)));
    s += p.c3 * (((w[1 + i] - c) + (w[7 + i] - c)) + ((q[(r + 1) % 9].v[i] - c) + (q[(r + 7) % 9].v[i] - c)));
    s += p.c2 * (((w[2 + i] - c) + (w[6 + i] - c)) + ((q[(r + 2) % 9].v[i] - c) + (q[(r + 6) % 9].v[i] - c)));
    s += p.c1 * (((w[3 + i] - c) + (w[5 + i] - c)) + ((q[(r + 3) % 9].v[i] - c) + (q[(r + 5) % 9].v[i] - c)));
    out[i] = s;
  }
}

template <typename T, int MODE, int CK>
__global__ __launch_bounds__(256) void k_step2d(Step<T> p, int n, int hslot, int ck_store, int ck_max) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int item = xcd_item(p.nwg);
  if (item >= p.nwg) return;
  const int group = item % p.ngroups;
  const int rest = item / p.ngroups;
  const int strip = rest % p.L.nstrips;
  const int ls = rest / p.L.nstrips;
  const int chunk = group * 4 + wv;
  if (chunk >= p.nchunks) return;
  const int z0 = chunk * p.zc;
  const int z1 = min(z0 + p.zc, p.L.nzp);

  const int pitch = p.L.pitch;
  const int nxp = p.L.nxp;
  const int x = strip * STRIP + lane * CPL - XL;   // prop x of this lane's first cell
  const bool xin = (x >= 0) && (x < nxp);          // lane holds propagation cells
  const bool hl_in = (lane == 0) && (x - 4 >= 0) && (x - 4 < nxp);
  const bool hr_in = (lane == 63) && (x + 4 < nxp);
  const long long fo = (long long)ls * p.L.fstride + SLACK + (long long)GZ * pitch + XL;
  const long long col = x;
  const int shot = p.shot0 + ls;

  // model-grid column of this lane
  const int xm = x - p.L.nb;
  bool xmod[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) xmod[i] = (xm + i >= 0) && (xm + i < p.L.nx);
  const bool xmodall = xmod[0] && xmod[1] && xmod[2] && xmod[3];
  const bool xmodany = xmod[0] || xmod[1] || xmod[2] || xmod[3];

  T ex[4];
  bool xsponge = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int xi = x + i;
    ex[i] = (xi >= 0 && xi < nxp) ? p.etax[xi] : T(0);
    xsponge = xsponge || (ex[i] != T(0));
  }
  bool xvalid[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) xvalid[i] = (x + i >= 0) && (x + i < nxp);
  const bool xvalall = xvalid[0] && xvalid[1] && xvalid[2] && xvalid[3];

  // source cell of this shot (background modes)
  int sx = -1, sz = -1;
  if (MODE == M_FUSED || MODE == M_BG) {
    sx = p.srcx[shot];
    sz = p.srcz[shot];
  }
  const T wsrc = (MODE == M_FUSED || MODE == M_BG) ? p.wav[n] : T(0);

  // field pointers: queue field A (u0 / du / nu), optional B (du in fused mode)
  // A: the queued field (background u in FUSED/BG, Born or adjoint field otherwise).
  // The background is stepped in increment form: Ainc holds u^n - u^{n-1} (updated
  // in place), u^{n+1} goes to Anext; the other fields keep two levels (Anext
  // holds level n-1 and receives level n+1).
  constexpr bool BGM = (MODE == M_FUSED || MODE == M_BG);
  const T* Acur;
  T* Anext;
  T* Ainc = nullptr;
  const T* Bcur = nullptr;
  T* Bnext = nullptr;
  if (BGM) {
    Acur = p.u_cur + fo;
    Anext = p.u_next + fo;
    Ainc = p.u_inc + fo;
    if (MODE == M_FUSED) {
      Bcur = p.du_cur + fo;
      Bnext = p.du_prev + fo;
    }
  } else {
    Acur = p.du_cur + fo;
    Anext = p.du_prev + fo;
  }
  constexpr bool TWO = (MODE == M_FUSED);

  V4<T> qa[9], qb[9];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const long long o = (long long)(z0 - 4 + s) * pitch + col;
    qa[s] = xin ? ld4(Acur + o) : zero4<T>();
    if (TWO) qb[s] = xin ? ld4(Bcur + o) : zero4<T>();
  }

  const long long kofs = (long long)SLACK + (long long)GZ * pitch + XL;
  const T* kap = p.kappa + kofs;
  const T* dmb = p.dmbar + (long long)p.dm_slot[shot] * p.L.fstride + kofs;
  const T* hist_n = p.hist + (long long)ls * p.hstride + (long long)hslot * p.L.mstride;
  double* img = (MODE == M_ADJ) ? p.img + (long long)shot * p.L.mstride : nullptr;
  T* hist_w = (MODE == M_FUSED || MODE == M_BG) ? const_cast<T*>(hist_n) : nullptr;
  const T* dat = p.data;
  float mx0 = 0.0f, mx1 = 0.0f;   // running max |u^{n+1}|, |u^{n+1} - u^n| (BF16 checkpoints)

  for (int zb = z0; zb < z1; zb += 9) {
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int z = zb + r;
      if (z >= z1) break;
      // bring in row z+4
      {
        const long long o = (long long)(z + 4) * pitch + col;
        qa[(r + 8) % 9] = xin ? ld4(Acur + o) : zero4<T>();
        if (TWO) qb[(r + 8) % 9] = xin ? ld4(Bcur + o) : zero4<T>();
      }
      const long long orow = (long long)z * pitch + col;
      // x halo of the centre row
      V4<T> ahl = zero4<T>(), ahr = zero4<T>(), bhl = zero4<T>(), bhr = zero4<T>();
      if (hl_in) {
        ahl = ld4(Acur + orow - 4);
        if (TWO) bhl = ld4(Bcur + orow - 4);
      }
      if (hr_in) {
        ahr = ld4(Acur + orow + 4);
        if (TWO) bhr = ld4(Bcur + orow + 4);
      }
      // Laplacian of A (and B)
      T lapA[4], lapB[4];
      {
        const V4<T>& C = qa[(r + 4) % 9];
        T w[12];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          w[i] = shr1(C.v[i], ahl.v[i]);
          w[4 + i] = C.v[i];
          w[8 + i] = shl1(C.v[i], ahr.v[i]);
        }
        lap_diff(w, qa, r, p, lapA);
      }
      if (TWO) {
        const V4<T>& C = qb[(r + 4) % 9];
        T w[12];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          w[i] = shr1(C.v[i], bhl.v[i]);
          w[4 + i] = C.v[i];
          w[8 + i] = shl1(C.v[i], bhr.v[i]);
        }
        lap_diff(w, qb, r, p, lapB);
      }
      if (!xin) continue;   // nothing to write for padding lanes (after all DPP use)

      // point source (background) / receiver injection (adjoint)
      if ((MODE == M_FUSED || MODE == M_BG) && z == sz) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (x + i == sx) lapA[i] += wsrc;
      }
      const int rp = p.recplane[z];
      const bool recrow = rp >= 0;
      int rm[4] = {-1, -1, -1, -1};
      if (recrow) {
        const int4 m4 = *reinterpret_cast<const int4*>(p.recmap + (long long)rp * p.cpitch + x);
        rm[0] = m4.x;
        rm[1] = m4.y;
        rm[2] = m4.z;
        rm[3] = m4.w;
        if (MODE == M_ADJ) {
          const T* drow = dat + ((long long)shot * p.nt + (n - 1)) * p.nr;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (rm[i] >= 0) lapA[i] += drow[rm[i]];
        }
      }

      const V4<T> kap4 = ld4(kap + orow);
      const T ez = p.etaz[z];
      T a[4], b[4];
      if (ez == T(0) && !xsponge) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = T(1);
          b[i] = T(1);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) damping(ex[i] + ez, p.hdt, a[i], b[i]);
      }

      const int zm = z - p.L.nb;
      const bool zmod = (zm >= 0) && (zm < p.L.nz);
      const long long mo = (long long)zm * p.L.mpitch + xm;

      // g on this row: computed (background modes) or read (Born, adjoint)
      T g[4] = {T(0), T(0), T(0), T(0)};
      if (MODE == M_FUSED || MODE == M_BG) {
#pragma unroll
        for (int i = 0; i < 4; ++i) g[i] = kap4.v[i] * lapA[i] * p.inv_dt2;
      } else if (zmod && xmodany) {
        if (xmodall) {
          const V4<T> gg = ld4(hist_n + mo);
#pragma unroll
          for (int i = 0; i < 4; ++i) g[i] = gg.v[i];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (xmod[i]) g[i] = hist_n[mo + i];
        }
      }

      // aprev: level n-1 (two-level fields) or the increment u^n - u^{n-1} (background)
      const V4<T> aprev = ld4((BGM ? Ainc : Anext) + orow);
      V4<T> adm = zero4<T>();
      if (MODE == M_BORN) adm = ld4(dmb + orow);
      V4<T> anew, ainc;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T c = qa[(r + 4) % 9].v[i];
        if (BGM) {
          // u+ = a (2u + kappa Lam) - b u-  written as  d+ = b d + a kappa Lam,  u+ = u + d+
          ainc.v[i] = b[i] * aprev.v[i] + a[i] * (kap4.v[i] * lapA[i]);
          anew.v[i] = c + ainc.v[i];
        } else {
          const T src = (MODE == M_BORN) ? kap4.v[i] * (lapA[i] - adm.v[i] * g[i]) : kap4.v[i] * lapA[i];
          anew.v[i] = a[i] * (T(2) * c + src) - b[i] * aprev.v[i];
        }
      }
      if (xvalall) {
        st4(Anext + orow, anew);
        if (BGM) st4(Ainc + orow, ainc);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (xvalid[i]) {
            Anext[orow + i] = anew.v[i];
            if (BGM) Ainc[orow + i] = ainc.v[i];
          }
      }

      V4<T> bnew;
      if (TWO) {
        const V4<T> bprev = ld4(Bnext + orow);
        const V4<T> dm4 = ld4(dmb + orow);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const T c = qb[(r + 4) % 9].v[i];
          bnew.v[i] = a[i] * (T(2) * c + kap4.v[i] * (lapB[i] - dm4.v[i] * g[i])) - b[i] * bprev.v[i];
        }
        if (xvalall) {
          st4(Bnext + orow, bnew);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (xvalid[i]) Bnext[orow + i] = bnew.v[i];
        }
      }

      // background checkpoint (u^n, u^n - u^{n-1}) and running maxima for the next one
      if (CK != CK_NONE && (MODE == M_FUSED || MODE == M_BG)) {
        if (ck_store >= 0) {
          const long long co = (long long)z * p.cpitch + x;
          const long long lv = ((long long)ls * p.nck + ck_store) * 2;
          if (CK == CK_F32) {
            T* c0 = static_cast<T*>(p.ck) + lv * p.cstride + co;
            T* c1 = c0 + p.cstride;
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (xvalid[i]) {
                c0[i] = qa[(r + 4) % 9].v[i];
                c1[i] = aprev.v[i];
              }
          } else {
            const float* sc = p.ck_scale + lv;
            const float s0 = sc[0], s1 = sc[1];
            const float i0 = s0 > 0.0f ? 1.0f / s0 : 1.0f, i1 = s1 > 0.0f ? 1.0f / s1 : 1.0f;
            unsigned short* c0 = static_cast<unsigned short*>(p.ck) + lv * p.cstride + co;
            unsigned short* c1 = c0 + p.cstride;
            unsigned short h0[4], h1[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float uc = (float)qa[(r + 4) % 9].v[i];
              h0[i] = bf16_rne(uc * i0);
              h1[i] = bf16_rne((float)aprev.v[i] * i1);
            }
            if (xvalall) {
              *reinterpret_cast<uint2*>(c0) = make_uint2(h0[0] | ((unsigned)h0[1] << 16), h0[2] | ((unsigned)h0[3] << 16));
              *reinterpret_cast<uint2*>(c1) = make_uint2(h1[0] | ((unsigned)h1[1] << 16), h1[2] | ((unsigned)h1[3] << 16));
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (xvalid[i]) {
                  c0[i] = h0[i];
                  c1[i] = h1[i];
                }
            }
          }
        }
        if (CK == CK_BF16 && ck_max >= 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (xvalid[i]) {
              mx0 = fmaxf(mx0, fabsf((float)anew.v[i]));
              mx1 = fmaxf(mx1, fabsf((float)ainc.v[i]));
            }
        }
      }

      // history of g (background modes)
      if (CK == CK_NONE && (MODE == M_FUSED || MODE == M_BG) && zmod && xmodany) {
        V4<T> gg;
#pragma unroll
        for (int i = 0; i < 4; ++i) gg.v[i] = g[i];
        if (xmodall) {
          st4(hist_w + mo, gg);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (xmod[i]) hist_w[mo + i] = g[i];
        }
      }

      // receiver gather of du^{n+1} (Born modes)
      if ((MODE == M_FUSED || MODE == M_BORN) && recrow) {
        T* drow = p.data + ((long long)shot * p.nt + n) * p.nr;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rm[i] >= 0) drow[rm[i]] = TWO ? bnew.v[i] : anew.v[i];
      }

      // zero-lag imaging I -= g^{k-1} nu^k in FP64 (adjoint)
      if (MODE == M_ADJ && zmod && xmodany) {
        if (xmodall) {
          V4<double> acc = *reinterpret_cast<V4<double>*>(img + mo);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc.v[i] -= (double)g[i] * (double)anew.v[i];
          *reinterpret_cast<V4<double>*>(img + mo) = acc;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (xmod[i]) img[mo + i] -= (double)g[i] * (double)anew.v[i];
        }
      }
    }
    // rotate nothing: the queue is addressed modulo 9 and zb advances by 9
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
}

// u_cur <- u^{jk}, u_inc <- u^{jk} - u^{jk-1} on the propagation cells of every
// local shot (2D and 3D layouts).
template <typename T, int CK>
__global__ void k_expand(Step<T> p, int nshots, int j) {
  const long long cells = (long long)p.L.nzp * p.L.nyp * p.L.nxp;
  const long long total = cells * nshots;
  const int gy = (p.L.ndim == 3) ? GY : 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    const int ls = (int)(i / cells);
    const long long c = i % cells;
    const int x = (int)(c % p.L.nxp);
    const long long t = c / p.L.nxp;
    const int y = (int)(t % p.L.nyp);
    const int z = (int)(t / p.L.nyp);
    const long long fo = (long long)ls * p.L.fstride + SLACK + (long long)(z + GZ) * p.L.plane +
                         (long long)(y + gy) * p.L.pitch + XL + x;
    const long long lv = ((long long)ls * p.nck + j) * 2;
    const long long co = ((long long)z * p.L.nyp + y) * p.cpitch + x;
    T un, ui;
    if (CK == CK_F32) {
      const T* c0 = static_cast<const T*>(p.ck) + lv * p.cstride + co;
      un = c0[0];
      ui = c0[p.cstride];
    } else {
      const unsigned short* c0 = static_cast<const unsigned short*>(p.ck) + lv * p.cstride + co;
      const float s0 = p.ck_scale[lv], s1 = p.ck_scale[lv + 1];
      un = (T)(bf16_to_f(c0[0]) * s0);
      ui = (T)(bf16_to_f(c0[p.cstride]) * s1);
    }
    p.u_cur[fo] = un;
    p.u_inc[fo] = ui;
  }
}

template <typename T, int MODE, int CK>
static void go(const Step<T>& p, int n, int hslot, int cs, int cm, hipStream_t st) {
  hipLaunchKernelGGL((k_step2d<T, MODE, CK>), dim3(xcd_grid(p.nwg)), dim3(256), 0, st, p, n, hslot, cs, cm);
}

template <typename T>
static void launch(int mode, const Step<T>& p, int n, int hs, int ck, int cs, int cm, hipStream_t st) {
  switch (mode) {
    case M_FUSED:
      if (ck == CK_F32) go<T, M_FUSED, CK_F32>(p, n, hs, cs, cm, st);
      else if (ck == CK_BF16) go<T, M_FUSED, CK_BF16>(p, n, hs, cs, cm, st);
      else go<T, M_FUSED, CK_NONE>(p, n, hs, -1, -1, st);
      break;
    case M_BG:
      if (ck == CK_F32) go<T, M_BG, CK_F32>(p, n, hs, cs, cm, st);
      else if (ck == CK_BF16) go<T, M_BG, CK_BF16>(p, n, hs, cs, cm, st);
      else go<T, M_BG, CK_NONE>(p, n, hs, -1, -1, st);
      break;
    case M_BORN: go<T, M_BORN, CK_NONE>(p, n, hs, -1, -1, st); break;
    default: go<T, M_ADJ, CK_NONE>(p, n, hs, -1, -1, st); break;
  }
}

template <typename T>
static void expand_t(const Step<T>& p, int nshots, int ck, int j, hipStream_t st) {
  const long long total = (long long)p.L.nzp * p.L.nyp * p.L.nxp * nshots;
  long long b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (ck == CK_F32) hipLaunchKernelGGL((k_expand<T, CK_F32>), dim3((unsigned)b), dim3(256), 0, st, p, nshots, j);
  else hipLaunchKernelGGL((k_expand<T, CK_BF16>), dim3((unsigned)b), dim3(256), 0, st, p, nshots, j);
}

void step2d(int mode, const Step<float>& p, int n, int hs, int ck, int cs, int cm, hipStream_t s) {
  launch(mode, p, n, hs, ck, cs, cm, s);
}
void step2d(int mode, const Step<double>& p, int n, int hs, int ck, int cs, int cm, hipStream_t s) {
  launch(mode, p, n, hs, ck, cs, cm, s);
}
void expand(const Step<float>& p, int ns, int ck, int j, hipStream_t s) { expand_t(p, ns, ck, j, s); }
void expand(const Step<double>& p, int ns, int ck, int j, hipStream_t s) { expand_t(p, ns, ck, j, s); }

}  // namespace mp
