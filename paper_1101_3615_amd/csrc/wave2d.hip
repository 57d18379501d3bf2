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

template <typename T>
__device__ __forceinline__ V4<T> ld4(const T* p) {
  return *reinterpret_cast<const V4<T>*>(p);
}
template <typename T>
__device__ __forceinline__ void st4(T* p, const V4<T>& v) {
  *reinterpret_cast<V4<T>*>(p) = v;
}
template <typename T>
__device__ __forceinline__ V4<T> zero4() {
  V4<T> r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.v[i] = T(0);
  return r;
}

enum { M_FUSED = 0, M_BORN = 1, M_BG = 2, M_ADJ = 3 };

// Background step size at cell: a and b of the damped leapfrog.
template <typename T>
__device__ __forceinline__ void damping(T eta, T hdt, T& a, T& b) {
  if (eta == T(0)) {
    a = T(1);
    b = T(1);
  } else {
    const T e = eta * hdt;
    a = T(1) / (T(1) + e);
    b = (T(1) - e) * a;
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_step2d(Step2D<T> p, int n, int hslot) {
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
  const T* Acur;
  T* Anext;
  const T* Bcur = nullptr;
  T* Bnext = nullptr;
  if (MODE == M_FUSED) {
    Acur = p.u_cur + fo;
    Anext = p.u_prev + fo;
    Bcur = p.du_cur + fo;
    Bnext = p.du_prev + fo;
  } else if (MODE == M_BG) {
    Acur = p.u_cur + fo;
    Anext = p.u_prev + fo;
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
  const T* dmb = p.dmbar + kofs;
  const int* rmap = p.recmap + kofs;
  const T* hist_n = p.hist + (long long)ls * p.hstride + (long long)hslot * p.L.mstride;
  double* img = (MODE == M_ADJ) ? p.img + (long long)shot * p.L.mstride : nullptr;
  T* hist_w = (MODE == M_FUSED || MODE == M_BG) ? const_cast<T*>(hist_n) : nullptr;
  const T* dat = p.data;

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
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          T s = p.c0x2 * w[4 + i];
          s += p.c1 * ((w[3 + i] + w[5 + i]) + (qa[(r + 3) % 9].v[i] + qa[(r + 5) % 9].v[i]));
          s += p.c2 * ((w[2 + i] + w[6 + i]) + (qa[(r + 2) % 9].v[i] + qa[(r + 6) % 9].v[i]));
          s += p.c3 * ((w[1 + i] + w[7 + i]) + (qa[(r + 1) % 9].v[i] + qa[(r + 7) % 9].v[i]));
          s += p.c4 * ((w[0 + i] + w[8 + i]) + (qa[(r + 0) % 9].v[i] + qa[(r + 8) % 9].v[i]));
          lapA[i] = s;
        }
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
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          T s = p.c0x2 * w[4 + i];
          s += p.c1 * ((w[3 + i] + w[5 + i]) + (qb[(r + 3) % 9].v[i] + qb[(r + 5) % 9].v[i]));
          s += p.c2 * ((w[2 + i] + w[6 + i]) + (qb[(r + 2) % 9].v[i] + qb[(r + 6) % 9].v[i]));
          s += p.c3 * ((w[1 + i] + w[7 + i]) + (qb[(r + 1) % 9].v[i] + qb[(r + 7) % 9].v[i]));
          s += p.c4 * ((w[0 + i] + w[8 + i]) + (qb[(r + 0) % 9].v[i] + qb[(r + 8) % 9].v[i]));
          lapB[i] = s;
        }
      }
      if (!xin) continue;   // nothing to write for padding lanes (after all DPP use)

      // point source (background) / receiver injection (adjoint)
      if ((MODE == M_FUSED || MODE == M_BG) && z == sz) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (x + i == sx) lapA[i] += wsrc;
      }
      const bool recrow = p.recrow[z] != 0;
      int rm[4] = {-1, -1, -1, -1};
      if (recrow) {
        const int4 m4 = *reinterpret_cast<const int4*>(rmap + orow);
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

      const V4<T> aprev = ld4(Anext + orow);
      V4<T> adm = zero4<T>();
      if (MODE == M_BORN) adm = ld4(dmb + orow);
      V4<T> anew;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T c = qa[(r + 4) % 9].v[i];
        const T src = (MODE == M_BORN) ? kap4.v[i] * (lapA[i] - adm.v[i] * g[i])
                                       : kap4.v[i] * lapA[i];
        anew.v[i] = a[i] * (T(2) * c + src) - b[i] * aprev.v[i];
      }
      if (xvalall) {
        st4(Anext + orow, anew);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (xvalid[i]) Anext[orow + i] = anew.v[i];
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

      // history of g (background modes)
      if ((MODE == M_FUSED || MODE == M_BG) && zmod && xmodany) {
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
}

template <typename T>
static void launch(int mode, const Step2D<T>& p, int n, int hslot, hipStream_t st) {
  const dim3 grid(xcd_grid(p.nwg)), block(256);
  switch (mode) {
    case M_FUSED: hipLaunchKernelGGL((k_step2d<T, M_FUSED>), grid, block, 0, st, p, n, hslot); break;
    case M_BORN: hipLaunchKernelGGL((k_step2d<T, M_BORN>), grid, block, 0, st, p, n, hslot); break;
    case M_BG: hipLaunchKernelGGL((k_step2d<T, M_BG>), grid, block, 0, st, p, n, hslot); break;
    default: hipLaunchKernelGGL((k_step2d<T, M_ADJ>), grid, block, 0, st, p, n, hslot); break;
  }
}

void step2d_fused(const Step2D<float>& p, int n, int hs, hipStream_t s) { launch(M_FUSED, p, n, hs, s); }
void step2d_fused(const Step2D<double>& p, int n, int hs, hipStream_t s) { launch(M_FUSED, p, n, hs, s); }
void step2d_born(const Step2D<float>& p, int n, int hs, hipStream_t s) { launch(M_BORN, p, n, hs, s); }
void step2d_born(const Step2D<double>& p, int n, int hs, hipStream_t s) { launch(M_BORN, p, n, hs, s); }
void step2d_bg(const Step2D<float>& p, int n, int hs, hipStream_t s) { launch(M_BG, p, n, hs, s); }
void step2d_bg(const Step2D<double>& p, int n, int hs, hipStream_t s) { launch(M_BG, p, n, hs, s); }
void step2d_adj(const Step2D<float>& p, int k, int hs, hipStream_t s) { launch(M_ADJ, p, k, hs, s); }
void step2d_adj(const Step2D<double>& p, int k, int hs, hipStream_t s) { launch(M_ADJ, p, k, hs, s); }

}  // namespace mp
