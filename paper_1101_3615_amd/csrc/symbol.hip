// Probing basis on the model grid: FFT multipliers, the FP64 least-squares
// fit (paper Sec. 1.4) and the fast application of the fitted series.
//
//   B_(a,q) v = P_a(x~) * Re IFFT( rho^q FFT v ),   rho = |k| h / pi
//
// FFT: radix-2 Stockham passes in LDS over lines of one axis (power-of-two
// lengths up to 1024); several lines per workgroup so that strided axes load
// contiguous runs.  Twiddles and Legendre factors are host FP64 tables.
//
// Fit: the stacked columns A = [B_i x_t] and b = [y_t] are materialised in FP64
// (column-major), and the least-squares problem is solved by shifted
// Cholesky-QR in three passes (Fukaya, Kannan, Nakatsukasa, Zhang, Yamamoto,
// SIAM J. Sci. Comput. 42 (2020)): each pass forms the Gram matrix of the
// current columns on the FP64 matrix cores (v_mfma_f64_16x16x4f64), factors it
// in one workgroup and right-multiplies the columns by the inverse factor.
// The first pass equilibrates the columns and adds the shift
// 11 (m p + p (p + 1)) u ||A||_F^2 to the diagonal.  The residual norm is
// formed explicitly from the final orthonormal columns.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "runtime.h"
#include "symbol.h"

namespace mp {

#define SY_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call);   \
      return MP_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)
#define SY_LAUNCH()                                                                   \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_));       \
      return MP_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)

template <typename R>
struct Cx {
  R x, y;
};

constexpr int MAXP = 64;          // basis terms
constexpr int GT = 16;            // MFMA tile
constexpr int GCOL = MAXP + GT;   // padded column count of [A b]
constexpr int GRB = 64;           // rows per LDS stage of the Gram kernel
constexpr int GWGMAX = 2048;      // Gram workgroups at most (each takes every nwg-th block, at least 8 blocks)

// ---------------------------------------------------------------- FFT --

struct LineMap {
  int n;           // line length (power of two)
  int logn;
  int nlines;
  int lpb;         // lines per workgroup
  long long es;    // element stride
  int B;           // lines -> offset: (l / B) * S1 + (l % B) * S0
  long long S0, S1;
};

template <typename R>
__global__ __launch_bounds__(256) void k_fft(Cx<R>* data, LineMap m, const Cx<R>* tw, int inverse) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* buf0 = reinterpret_cast<Cx<R>*>(smem_raw);
  Cx<R>* buf1 = buf0 + (size_t)m.lpb * m.n;
  const int l0 = blockIdx.x * m.lpb;
  const int tot = m.lpb * m.n;
  const bool unit = (m.es == 1);
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    int j, e;
    if (unit) { j = t / m.n; e = t % m.n; }
    else { j = t % m.lpb; e = t / m.lpb; }
    const int l = l0 + j;
    Cx<R> v = {R(0), R(0)};
    if (l < m.nlines) v = data[(long long)(l / m.B) * m.S1 + (long long)(l % m.B) * m.S0 + (long long)e * m.es];
    buf0[j * m.n + e] = v;
  }
  Cx<R>* src = buf0;
  Cx<R>* dst = buf1;
  const int half = m.n >> 1;
  for (int p = 0; p < m.logn; ++p) {
    __syncthreads();
    const int ns = 1 << p;
    const int twstep = m.n / (2 * ns);
    for (int t = threadIdx.x; t < m.lpb * half; t += blockDim.x) {
      const int j = t / half, b = t % half;
      const Cx<R> a0 = src[j * m.n + b];
      const Cx<R> a1 = src[j * m.n + b + half];
      const int k = b & (ns - 1);
      Cx<R> w = tw[k * twstep];
      if (inverse) w.y = -w.y;
      const Cx<R> v = {a1.x * w.x - a1.y * w.y, a1.x * w.y + a1.y * w.x};
      const int o = (b - k) * 2 + k;
      dst[j * m.n + o] = {a0.x + v.x, a0.y + v.y};
      dst[j * m.n + o + ns] = {a0.x - v.x, a0.y - v.y};
    }
    Cx<R>* t = src;
    src = dst;
    dst = t;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    int j, e;
    if (unit) { j = t / m.n; e = t % m.n; }
    else { j = t % m.lpb; e = t / m.lpb; }
    const int l = l0 + j;
    if (l < m.nlines) data[(long long)(l / m.B) * m.S1 + (long long)(l % m.B) * m.S0 + (long long)e * m.es] = src[j * m.n + e];
  }
}

// real field (any precision) -> complex
template <typename R, typename T>
__global__ void k_to_complex(Cx<R>* out, const T* in, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = {(R)in[i], R(0)};
}

struct Grid3 {
  int n[3];        // nx, ny, nz (ny = 1 in 2D)
  long long cells;
};

template <typename R>
__device__ __forceinline__ R rho_at(long long i, const Grid3& g) {
  const int x = (int)(i % g.n[0]);
  const long long t = i / g.n[0];
  const int y = (int)(t % g.n[1]);
  const int z = (int)(t / g.n[1]);
  const int jx = (x <= g.n[0] / 2 - (g.n[0] % 2 == 0 ? 1 : 0)) ? x : x - g.n[0];
  const int jy = (y <= g.n[1] / 2 - (g.n[1] % 2 == 0 ? 1 : 0)) ? y : y - g.n[1];
  const int jz = (z <= g.n[2] / 2 - (g.n[2] % 2 == 0 ? 1 : 0)) ? z : z - g.n[2];
  const R fx = (R)jx / (R)g.n[0], fy = (R)jy / (R)g.n[1], fz = (R)jz / (R)g.n[2];
  return R(2) * sqrt(fx * fx + fy * fy + fz * fz);
}

// signed frequencies j/N of FFT cell i per axis (x, y, z)
template <typename R>
__device__ __forceinline__ void freq_at(long long i, const Grid3& g, R f[3]) {
  const int c[3] = {(int)(i % g.n[0]), (int)((i / g.n[0]) % g.n[1]), (int)(i / ((long long)g.n[0] * g.n[1]))};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int j = (c[a] <= g.n[a] / 2 - (g.n[a] % 2 == 0 ? 1 : 0)) ? c[a] : c[a] - g.n[a];
    f[a] = (R)j / (R)g.n[a];
  }
}

// Angular harmonic `a` of the direction of k (f: frequencies per axis, fn = |f| > 0):
// 2D (x, z): 1, cos(j theta), sin(j theta) for a = 0, 2j-1, 2j, theta = atan2(f_z, f_x);
// 3D: the real spherical harmonics of degree <= 2 as polynomials of n = f / |f|.
template <typename R>
__device__ __forceinline__ R angular(int a, const R f[3], R fn, int ndim) {
  if (ndim == 2) {
    const R th = atan2(f[2], f[0]);
    const R j = (R)((a + 1) / 2);
    return (a & 1) ? cos(j * th) : sin(j * th);
  }
  const R nx = f[0] / fn, ny = f[1] / fn, nz = f[2] / fn;
  switch (a) {
    case 1: return nx;
    case 2: return ny;
    case 3: return nz;
    case 4: return nx * ny;
    case 5: return ny * nz;
    case 6: return R(3) * nz * nz - R(1);
    case 7: return nx * nz;
    default: return nx * nx - ny * ny;
  }
}

// rational Chebyshev TL_n(r) = T_n((r - L)/(r + L)) by the three-term recurrence
template <typename R>
__device__ __forceinline__ R rational_chebyshev(int n, R r, R L) {
  const R t = (r - L) / (r + L);
  R t0 = R(1), t1 = t;
  if (n == 0) return t0;
  for (int k = 1; k < n; ++k) {
    const R t2 = R(2) * t * t1 - t0;
    t0 = t1;
    t1 = t2;
  }
  return t1;
}

// Multiplier of basis family `family` (see mp_basis_desc) times X:
// out = X * sum_k coef[k] m_k.  Family 0: m_k = rho^qs[k]; family 1:
// m_k = A_{qs[2k]}(k/|k|) TL_{qs[2k+1]}(rho) rho^order.
template <typename R>
__global__ void k_multiplier(Cx<R>* out, const Cx<R>* X, Grid3 g, int nq, const int* qs, const double* coef,
                             int family, int ndim, int order, double tl_scale) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.cells; i += (long long)gridDim.x * blockDim.x) {
    const R r = rho_at<R>(i, g);
    R m = R(0);
    if (family == 0) {
      for (int k = 0; k < nq; ++k) {
        R pw = R(1);
        for (int e = 0; e < qs[k]; ++e) pw *= r;
        m += (R)coef[k] * pw;
      }
    } else {
      R f[3];
      freq_at<R>(i, g, f);
      const R fn = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      R rp = R(1);   // rho^order, 0 at k = 0 unless order = 0
      if (order != 0 && r == R(0)) rp = R(0);
      else
        for (int e = 0; e < abs(order); ++e) rp *= (order > 0) ? r : R(1) / r;
      for (int k = 0; k < nq; ++k) {
        const int a = qs[2 * k];
        const R ang = (a == 0) ? R(1) : (fn == R(0) ? R(0) : angular<R>(a, f, fn, ndim));
        m += (R)coef[k] * ang * rational_chebyshev<R>(qs[2 * k + 1], r, (R)tl_scale) * rp;
      }
    }
    const Cx<R> v = X[i];
    out[i] = {v.x * m, v.y * m};
  }
}

// Position factor at cell i of the term spec sp = (kind, n_x, n_y, n_z, phase):
// kind 0: product of Legendre polynomials of degrees n (per-axis tables
// leg[axis][deg][N_axis]); kind 1: cos (phase 0) or sin (phase 1) of
// pi (n_x x~ + n_y y~ + n_z z~) at the cell centres x~ = -1 + (2i+1)/N.
__device__ __forceinline__ double pfac(long long i, const Grid3& g, const double* leg, int maxdeg, const int* sp) {
  const int x = (int)(i % g.n[0]);
  const long long t = i / g.n[0];
  const int y = (int)(t % g.n[1]);
  const int z = (int)(t / g.n[1]);
  if (sp[0] == 1) {
    const double pi = 3.14159265358979323846;
    const double arg = pi * (sp[1] * (-1.0 + (2.0 * x + 1.0) / g.n[0]) + sp[2] * (-1.0 + (2.0 * y + 1.0) / g.n[1]) +
                             sp[3] * (-1.0 + (2.0 * z + 1.0) / g.n[2]));
    return sp[4] ? sin(arg) : cos(arg);
  }
  const int* deg = sp + 1;
  const int nmax = max(g.n[0], max(g.n[1], g.n[2]));
  const long long as = (long long)(maxdeg + 1) * nmax;
  return leg[0 * as + (long long)deg[0] * nmax + x] * leg[1 * as + (long long)deg[1] * nmax + y] *
         leg[2 * as + (long long)deg[2] * nmax + z];
}

// out (+)= P_a * Re(V) / N, sp: the term's position-factor spec
template <typename R, typename T>
__global__ void k_accum_out(T* out, const Cx<R>* V, Grid3 g, const double* leg, int maxdeg, const int* sp,
                            double scale, int first) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.cells; i += (long long)gridDim.x * blockDim.x) {
    const R v = (R)(pfac(i, g, leg, maxdeg, sp) * scale) * V[i].x;
    out[i] = first ? (T)v : (T)(out[i] + (T)v);
  }
}

// A[col(a, q)][row0 + i] = P_a(i) * Re(V[i]) / N for every a (one q)
__global__ void k_columns(double* A, long long lda, long long row0, const Cx<double>* V, Grid3 g, const double* leg,
                          int maxdeg, int na, int nq, int q, const int* specs, double scale) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.cells; i += (long long)gridDim.x * blockDim.x) {
    const double v = V[i].x * scale;
    for (int a = 0; a < na; ++a) {
      A[(long long)(a * nq + q) * lda + row0 + i] = pfac(i, g, leg, maxdeg, specs + 5 * a) * v;
    }
  }
}

template <typename T>
__global__ void k_column_copy(double* A, long long lda, int col, long long row0, const T* y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    A[(long long)col * lda + row0 + i] = (double)y[i];
}

// ------------------------------------------------------- Gram on MFMA --

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Partial Gram of the columns [0, ncol) of A (NT 16-column tiles) over the GRB-row
// blocks wg, wg + nwg, wg + 2 nwg, ... (nwg workgroups): part[wg][i][j] for the
// 16x16 tiles with tj >= ti.  One MFMA consumes a 16x4 block of rows of column
// tile ti and of column tile tj.  Each wave takes a quarter of the rows of every
// block for all NT (NT + 1) / 2 tile pairs (accumulators indexed by constants,
// NP independent MFMA chains per wave, the same work on every SIMD); the four
// waves' sums are added in a fixed order at the end.  The workgroups of a launch
// sweep the rows together, so the rows in use at any time lie in one narrow band
// of each column (few pages, long contiguous runs), not in nwg bands far apart.
template <int NT>
__global__ __launch_bounds__(256) void k_gram(const double* A, long long lda, long long nrows, int ncol, double* part) {
  constexpr int NP = NT * (NT + 1) / 2;
  constexpr int NCP = NT * GT;                 // padded column count
  constexpr int TILE = NCP * (GRB + 1);        // LDS stage [NCP][GRB + 1]
  constexpr int RED = 2 * NP * 256;            // two waves' accumulators
  __shared__ double lds[TILE > RED ? TILE : RED];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  dbl4 acc[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = (dbl4){0.0, 0.0, 0.0, 0.0};
  const long long step = (long long)gridDim.x * GRB;   // rows between this workgroup's blocks
  const long long r0 = (long long)blockIdx.x * GRB;
  // the next block's rows are loaded into registers while the MFMAs consume the
  // current one: thread t loads rows t % GRB of columns t / GRB + 4 q
  constexpr int LPT = NCP * GRB / 256;
  double nx[LPT];
  auto load = [&](long long rb) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int t = (int)threadIdx.x + q * 256;
      const int c = t / GRB, r = t % GRB;
      const long long row = rb + r;
      nx[q] = (c < ncol && row < nrows) ? A[(long long)c * lda + row] : 0.0;
    }
  };
  load(r0);
  constexpr int KW = GRB / 4;   // rows of a block per wave
  for (long long rb = r0; rb < nrows; rb += step) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int t = (int)threadIdx.x + q * 256;
      lds[(t / GRB) * (GRB + 1) + t % GRB] = nx[q];
    }
    __syncthreads();
    if (rb + step < nrows) load(rb + step);
#pragma unroll
    for (int kk = wv * KW; kk < (wv + 1) * KW; kk += 4) {
      double av[NT];
#pragma unroll
      for (int ti = 0; ti < NT; ++ti) av[ti] = lds[(ti * GT + (lane & 15)) * (GRB + 1) + kk + (lane >> 4)];
      int k = 0;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj, ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], av[tj], acc[k], 0, 0, 0);
    }
  }
  // waves 2, 3 hand their sums to waves 0, 1 (w0 + w2, w1 + w3), then wave 1 to
  // wave 0: G_part = (w0 + w2) + (w1 + w3)
  __syncthreads();
  auto put = [&](int slot) {
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) lds[((slot * NP + k) * 4 + v) * 64 + lane] = acc[k][v];
  };
  auto add = [&](int slot) {
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[k][v] += lds[((slot * NP + k) * 4 + v) * 64 + lane];
  };
  if (wv >= 2) put(wv - 2);
  __syncthreads();
  if (wv < 2) add(wv);
  __syncthreads();
  if (wv == 1) put(0);
  __syncthreads();
  if (wv == 0) {
    add(0);
    // f64 16x16x4 accumulator layout (checked on gfx950): element v of lane l holds
    // D[row = l/16 + 4 v][col = l % 16] of tile (ti, tj) = sum_r A[ti*16+row][r] A[tj*16+col][r]
    double* out = part + (long long)blockIdx.x * GCOL * GCOL;
    int k = 0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int tj = ti; tj < NT; ++tj, ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = ti * GT + (lane >> 4) + 4 * v;
          const int j = tj * GT + (lane & 15);
          out[i * GCOL + j] = acc[k][v];
        }
  }
}

static void gram_partials(dim3 grid, hipStream_t s, const double* A, long long lda, long long nrows, int ncol,
                          double* part) {
  switch ((ncol + GT - 1) / GT) {
    case 1: hipLaunchKernelGGL(k_gram<1>, grid, dim3(256), 0, s, A, lda, nrows, ncol, part); break;
    case 2: hipLaunchKernelGGL(k_gram<2>, grid, dim3(256), 0, s, A, lda, nrows, ncol, part); break;
    case 3: hipLaunchKernelGGL(k_gram<3>, grid, dim3(256), 0, s, A, lda, nrows, ncol, part); break;
    case 4: hipLaunchKernelGGL(k_gram<4>, grid, dim3(256), 0, s, A, lda, nrows, ncol, part); break;
    default: hipLaunchKernelGGL(k_gram<5>, grid, dim3(256), 0, s, A, lda, nrows, ncol, part); break;
  }
}

// G = sum over workgroups of the partial Grams, symmetrised.  A block of RDW
// waves takes 64 consecutive entries of G (lane = entry, so every load of a
// wave reads consecutive partial entries); wave k sums the k-th of RDW equal
// ranges of workgroups in order, and the RDW range sums are added in order
// (a fixed order: the result does not depend on timing).
constexpr int RDW = 16;
__global__ __launch_bounds__(64 * RDW) void k_gram_reduce(const double* part, int nwg, int ncol, double* G) {
  __shared__ double q[RDW][64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const int nn = ncol * ncol;
  double s = 0.0;
  if (t < nn) {
    int i = t / ncol, j = t % ncol;
    if (i / GT > j / GT) {   // only tiles with tj >= ti were accumulated
      const int x = i;
      i = j;
      j = x;
    }
    const double* src = part + i * GCOL + j;
    const int per = (nwg + RDW - 1) / RDW;
    const int w0 = wv * per, w1 = min(nwg, w0 + per);
#pragma unroll 8
    for (int w = w0; w < w1; ++w) s += src[(long long)w * GCOL * GCOL];
  }
  q[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && t < nn) {
    double g = q[0][lane];
#pragma unroll
    for (int k = 1; k < RDW; ++k) g += q[k][lane];
    G[t] = g;
  }
}

// ------------------------------------------------- small dense algebra --

// Work area of the solve kernels (device, FP64).
struct Small {
  double G[GCOL * GCOL];      // current Gram of [Q b] (p + 1 columns)
  double M[MAXP * MAXP];      // transform applied to the columns this pass
  double Racc[MAXP * MAXP];   // accumulated R (upper): R = R3 R2 R1 D^-1
  double d[MAXP];             // column scaling of pass 1
  double bb;                  // ||b||^2
  double w[MAXP];             // combination of the current columns giving A c
  double c[MAXP];             // solution
  double sig[MAXP];           // singular values of R (equilibrated problem)
  int status;                 // 0 ok, 1 Cholesky failure (rank deficient)
};

// Cholesky of the leading p x p block of S (row-major, ld) in place: upper R with
// R^T R = S.  Executed by one workgroup; returns false on a non-positive pivot.
__device__ bool chol_upper(double* S, int ld, int p) {
  __shared__ int ok;
  if (threadIdx.x == 0) ok = 1;
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    __syncthreads();
    const double piv = S[k * ld + k];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) ok = 0;
      __syncthreads();
      return false;
    }
    const double r = sqrt(piv);
    __syncthreads();
    for (int j = k + threadIdx.x; j < p; j += blockDim.x) S[k * ld + j] = (j == k) ? r : S[k * ld + j] / r;
    __syncthreads();
    for (int t = threadIdx.x; t < (p - k - 1) * (p - k - 1); t += blockDim.x) {
      const int i = k + 1 + t / (p - k - 1), j = k + 1 + t % (p - k - 1);
      if (j >= i) S[i * ld + j] -= S[k * ld + i] * S[k * ld + j];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    const int i = t / p, j = t % p;
    if (j < i) S[i * ld + j] = 0.0;
  }
  __syncthreads();
  return ok != 0;
}

// Inverse of an upper-triangular p x p matrix U (row-major, ld) into V (ld).
__device__ void inv_upper(const double* U, int ldu, double* V, int ldv, int p) {
  // column j of V solves U v = e_j; one thread per column
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    for (int i = p - 1; i >= 0; --i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) s -= U[i * ldu + k] * V[k * ldv + j];
      V[i * ldv + j] = (i <= j) ? s / U[i * ldu + i] : 0.0;
    }
  }
  __syncthreads();
}

// One Cholesky-QR pass on the Gram S of [Q b] (p + 1 columns).
// pass 0: equilibrate with d = diag(S)^-1/2, add the shift, factor, M = D R^-1.
// pass k: factor, M = R^-1.  Racc <- R Racc.  M left in W->M.
__global__ __launch_bounds__(256) void k_cqr_pass(Small* W, int p, long long m, int pass) {
  __shared__ double S[MAXP * MAXP];
  __shared__ double R[MAXP * MAXP];
  const int ldg = p + 1;
  if (pass == 0) {
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
      const double g = W->G[i * ldg + i];
      W->d[i] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
    }
    if (threadIdx.x == 0) {
      W->bb = W->G[p * ldg + p];
      W->status = 0;
    }
    __syncthreads();
  }
  if (W->status) return;
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    const int i = t / p, j = t % p;
    double v = W->G[i * ldg + j];
    if (pass == 0) v *= W->d[i] * W->d[j];
    S[i * MAXP + j] = v;
  }
  __syncthreads();
  if (pass == 0) {
    // ||A D||_F^2 = p after equilibration; u = 2^-53
    const double shift = 11.0 * ((double)m * p + (double)p * (p + 1)) * 1.1102230246251565e-16 * (double)p;
    for (int i = threadIdx.x; i < p; i += blockDim.x) S[i * MAXP + i] += shift;
    __syncthreads();
  }
  if (!chol_upper(S, MAXP, p)) {
    if (threadIdx.x == 0) W->status = 1;
    return;
  }
  inv_upper(S, MAXP, R, MAXP, p);   // R <- S^-1 (S now holds the factor)
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    const int i = t / p, j = t % p;
    W->M[i * MAXP + j] = (pass == 0) ? W->d[i] * R[i * MAXP + j] : R[i * MAXP + j];
  }
  __syncthreads();
  // Racc <- S * Racc (pass 0: Racc = S D^-1)
  if (pass == 0) {
    for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
      const int i = t / p, j = t % p;
      W->Racc[i * MAXP + j] = (j >= i) ? S[i * MAXP + j] / W->d[j] : 0.0;
    }
  } else {
    for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
      const int i = t / p, j = t % p;
      double s = 0.0;
      for (int k = i; k <= j; ++k) s += S[i * MAXP + k] * W->Racc[k * MAXP + j];
      R[i * MAXP + j] = (j >= i) ? s : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < p * p; t += blockDim.x) W->Racc[t / p * MAXP + t % p] = R[t / p * MAXP + t % p];
  }
}

// Columns 0..p-1 of A <- A M (M upper triangular, from the pass kernel).  One row
// per thread, its p values in registers: the column count is a template bound PB
// (p rounded up to a multiple of 8) and the sum over the row runs over all PB
// entries, so that every index into the row is a compile-time constant (a
// runtime-indexed array would live in scratch memory).  M is held with zeros below
// the diagonal and past p, and row entries past p read as zero: each output is the
// sum over i <= j in increasing i followed by exact zeros, the same bits.
template <int PB>
__global__ __launch_bounds__(256) void k_qupdate(double* A, long long lda, long long nrows, int p, const Small* W) {
  __shared__ double M[PB * PB];
  for (int t = threadIdx.x; t < PB * PB; t += blockDim.x) {
    const int i = t / PB, j = t % PB;
    M[t] = (i <= j && j < p) ? W->M[i * MAXP + j] : 0.0;
  }
  __syncthreads();
  if (W->status) return;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (long long)gridDim.x * blockDim.x) {
    double a[PB];
#pragma unroll
    for (int i = 0; i < PB; ++i) a[i] = i < p ? A[(long long)i * lda + r] : 0.0;
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < PB; ++i) s += a[i] * M[i * PB + j];
      A[(long long)j * lda + r] = s;
    }
  }
}

static void qupdate(dim3 grid, hipStream_t s, double* A, long long lda, long long nrows, int p, const Small* W) {
  const int pb = (p + 7) / 8 * 8;
  switch (pb) {
    case 8: hipLaunchKernelGGL(k_qupdate<8>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
    case 16: hipLaunchKernelGGL(k_qupdate<16>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
    case 24: hipLaunchKernelGGL(k_qupdate<24>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
    case 32: hipLaunchKernelGGL(k_qupdate<32>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
    case 40: hipLaunchKernelGGL(k_qupdate<40>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
    case 48: hipLaunchKernelGGL(k_qupdate<48>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
    case 56: hipLaunchKernelGGL(k_qupdate<56>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
    default: hipLaunchKernelGGL(k_qupdate<64>, grid, dim3(256), 0, s, A, lda, nrows, p, W); break;
  }
}

// One-sided Jacobi SVD of the p x p matrix in X (row-major, ld MAXP): on exit
// the columns of X are U Sigma, V (ld MAXP) the right singular vectors.  Parallel
// (round-robin) ordering: each sweep is P - 1 rounds (P = p rounded up to even) of
// P/2 disjoint column pairs, one group of 8 threads per pair; a pair with the padding
// index p (odd p) is skipped.  One barrier per round.
__device__ void jacobi_svd(double* X, double* V, int p) {
  __shared__ int rot;
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) V[t / p * MAXP + t % p] = (t / p == t % p) ? 1.0 : 0.0;
  __syncthreads();
  const int P = (p + 1) & ~1;
  const int grp = threadIdx.x >> 3, gl = threadIdx.x & 7;   // 32 groups of 8 (blockDim 256)
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) rot = 0;
    __syncthreads();
    for (int r = 0; r < P - 1; ++r) {
      for (int k = grp; k < P / 2; k += (int)(blockDim.x >> 3)) {
        // circle method: element 0 fixed, 1 .. P-1 rotate by r
        const int ka = k, kb = P - 1 - k;
        const int ea = (ka == 0) ? 0 : 1 + (ka - 1 + r) % (P - 1);
        const int eb = (kb == 0) ? 0 : 1 + (kb - 1 + r) % (P - 1);
        const int i = min(ea, eb), j = max(ea, eb);
        if (j >= p) continue;                                  // the padding column (group-uniform)
        double a = 0.0, b = 0.0, g = 0.0;
        for (int q = gl; q < p; q += 8) {
          const double xi = X[q * MAXP + i], xj = X[q * MAXP + j];
          a += xi * xi;
          b += xj * xj;
          g += xi * xj;
        }
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
          a += __shfl_xor(a, o);
          b += __shfl_xor(b, o);
          g += __shfl_xor(g, o);
        }
        if (fabs(g) > 1e-15 * sqrt(a * b) && g != 0.0) {
          const double zeta = (b - a) / (2.0 * g);
          const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
          for (int q = gl; q < p; q += 8) {
            const double xi = X[q * MAXP + i], xj = X[q * MAXP + j];
            X[q * MAXP + i] = cs * xi - sn * xj;
            X[q * MAXP + j] = sn * xi + cs * xj;
            const double vi = V[q * MAXP + i], vj = V[q * MAXP + j];
            V[q * MAXP + i] = cs * vi - sn * vj;
            V[q * MAXP + j] = sn * vi + cs * vj;
          }
          if (gl == 0) rot = 1;
        }
      }
      __syncthreads();
    }
    if (!rot) break;
    __syncthreads();
  }
}

// Final solve.  G holds the Gram of [Q b] after the last pass (Q^T Q ~ I,
// z = Q^T b in its last column).  c_eq = Racc^-1 (G_QQ^-1 z) ... with the
// last pass folded in: w = combination of the current columns, c = D-scaled.
// Also the singular values of Racc (of the equilibrated A) for the rank test.
__global__ __launch_bounds__(256) void k_cqr_solve(Small* W, int p) {
  __shared__ double S[MAXP * MAXP];
  __shared__ double V[MAXP * MAXP];
  __shared__ double z[MAXP], y[MAXP];
  const int ldg = p + 1;
  if (W->status) return;
  // S = Gram of the current columns, factor it (third pass, R3)
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) S[t / p * MAXP + t % p] = W->G[(t / p) * ldg + t % p];
  for (int i = threadIdx.x; i < p; i += blockDim.x) z[i] = W->G[i * ldg + p];
  __syncthreads();
  if (!chol_upper(S, MAXP, p)) {
    if (threadIdx.x == 0) W->status = 1;
    return;
  }
  // w = S^-1 S^-T z  (the least-squares combination of the current columns)
  if (threadIdx.x == 0) {
    for (int i = 0; i < p; ++i) {           // S^T y = z
      double s = z[i];
      for (int k = 0; k < i; ++k) s -= S[k * MAXP + i] * y[k];
      y[i] = s / S[i * MAXP + i];
    }
    for (int i = p - 1; i >= 0; --i) {      // S w = y
      double s = y[i];
      for (int k = i + 1; k < p; ++k) s -= S[i * MAXP + k] * W->w[k];
      W->w[i] = s / S[i * MAXP + i];
    }
  }
  __syncthreads();
  // Racc <- S Racc (full R of the equilibrated-then-unscaled problem)
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    const int i = t / p, j = t % p;
    double s = 0.0;
    for (int k = i; k <= j; ++k) s += S[i * MAXP + k] * W->Racc[k * MAXP + j];
    V[i * MAXP + j] = (j >= i) ? s : 0.0;
  }
  __syncthreads();
  // c = Rprev^-1 w where Rprev = Racc before this product (columns = A Rprev^-1);
  // solve with the stored Racc (upper): Racc c = w
  if (threadIdx.x == 0) {
    for (int i = p - 1; i >= 0; --i) {
      double s = W->w[i];
      for (int k = i + 1; k < p; ++k) s -= W->Racc[i * MAXP + k] * W->c[k];
      W->c[i] = s / W->Racc[i * MAXP + i];
    }
  }
  __syncthreads();
  // singular values of the full R scaled back to the equilibrated columns: R D
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    const int i = t / p, j = t % p;
    S[i * MAXP + j] = V[i * MAXP + j] * W->d[j];
  }
  __syncthreads();
  jacobi_svd(S, V, p);
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < p; ++k) s += S[k * MAXP + j] * S[k * MAXP + j];
    W->sig[j] = sqrt(s);
  }
}

// Minimum-norm solution from the equilibrated normal equations (used when a
// Cholesky pass fails): c = D sum_{lambda_i > tol lambda_max} v_i v_i^T r / lambda_i.
__global__ __launch_bounds__(256) void k_minnorm(Small* W, const double* G0, int p, double tol) {
  __shared__ double S[MAXP * MAXP];
  __shared__ double V[MAXP * MAXP];
  __shared__ double lam[MAXP], r[MAXP];
  const int ldg = p + 1;
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    const double g = G0[i * ldg + i];
    W->d[i] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    const int i = t / p, j = t % p;
    S[i * MAXP + j] = G0[i * ldg + j] * W->d[i] * W->d[j];
  }
  for (int i = threadIdx.x; i < p; i += blockDim.x) r[i] = G0[i * ldg + p] * W->d[i];
  __syncthreads();
  jacobi_svd(S, V, p);
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < p; ++k) s += S[k * MAXP + j] * S[k * MAXP + j];
    lam[j] = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double lmax = 0.0;
    for (int j = 0; j < p; ++j) lmax = fmax(lmax, lam[j]);
    for (int i = 0; i < p; ++i) W->c[i] = 0.0;
    for (int j = 0; j < p; ++j) {
      if (!(lam[j] > tol * lmax)) continue;
      double vr = 0.0;
      for (int k = 0; k < p; ++k) vr += V[k * MAXP + j] * r[k];
      for (int i = 0; i < p; ++i) W->c[i] += V[i * MAXP + j] * vr / lam[j];
    }
    for (int i = 0; i < p; ++i) {
      W->c[i] *= W->d[i];
      W->sig[i] = sqrt(fmax(lam[i], 0.0));
    }
    W->bb = G0[p * ldg + p];
  }
}

// sum over rows of (b - Q w)^2 per workgroup (fixed order), Q = columns 0..p-1.
__global__ __launch_bounds__(256) void k_resid(const double* A, long long lda, long long nrows, int p,
                                                const Small* W, double* part) {
  __shared__ double red[256];
  __shared__ double w[MAXP];
  for (int i = threadIdx.x; i < p; i += blockDim.x) w[i] = W->w[i];
  __syncthreads();
  double acc = 0.0;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (long long)gridDim.x * blockDim.x) {
    double s = A[(long long)p * lda + r];
    for (int i = 0; i < p; ++i) s -= A[(long long)i * lda + r] * w[i];
    acc += s * s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------- host side --

struct SymbolWS {
  DevBuf cx0, cx1;          // complex work fields
  DevBuf A;                 // [p+1][nrows] FP64
  DevBuf part;              // partial Grams / residual partials
  DevBuf G0;                // first Gram (kept for the fallback)
  DevBuf small;             // Small
  DevBuf twd[3], twf[3];    // twiddles per axis, FP64 and FP32
  DevBuf leg;               // Legendre tables [3][maxdeg+1][nmax]
  DevBuf qs, coef, degs;
  int maxdeg = -1;
};

static long long cells_of(const Config& c) { return (long long)c.nx * c.ny * c.nz; }

static bool pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

static dim3 egrid(long long n) {
  long long b = (n + 255) / 256;
  return dim3((unsigned)std::max<long long>(1, std::min<long long>(b, 16384)));
}

static int ensure_tables(mp_ctx* ctx, SymbolWS* ws, int maxdeg, hipStream_t s) {
  const Config& c = ctx->cfg;
  const int n3[3] = {c.nx, c.ny, c.nz};
  int rc;
  for (int a = 0; a < 3; ++a) {
    const int n = n3[a];
    if (ws->twd[a].get()) continue;
    const int half = std::max(1, n / 2);
    std::vector<double> td(2 * half);
    std::vector<float> tf(2 * half);
    const double pi = 3.14159265358979323846;
    for (int m = 0; m < half; ++m) {
      td[2 * m] = std::cos(2.0 * pi * m / n);
      td[2 * m + 1] = -std::sin(2.0 * pi * m / n);
      tf[2 * m] = (float)td[2 * m];
      tf[2 * m + 1] = (float)td[2 * m + 1];
    }
    if ((rc = ws->twd[a].ensure(td.size() * 8, &ctx->budget, "twiddles"))) return rc;
    if ((rc = ws->twf[a].ensure(tf.size() * 4, &ctx->budget, "twiddles"))) return rc;
    SY_HIP(hipMemcpyAsync(ws->twd[a].get(), td.data(), td.size() * 8, hipMemcpyHostToDevice, s));
    SY_HIP(hipMemcpyAsync(ws->twf[a].get(), tf.data(), tf.size() * 4, hipMemcpyHostToDevice, s));
  }
  if (maxdeg > ws->maxdeg) {
    const int nmax = std::max(c.nx, std::max(c.ny, c.nz));
    std::vector<double> leg((size_t)3 * (maxdeg + 1) * nmax, 0.0);
    for (int a = 0; a < 3; ++a) {
      const int n = n3[a];
      for (int i = 0; i < n; ++i) {
        const double t = -1.0 + (2.0 * i + 1.0) / n;
        double p0 = 1.0, p1 = t;
        for (int d = 0; d <= maxdeg; ++d) {
          double v;
          if (d == 0) v = 1.0;
          else if (d == 1) v = t;
          else {
            const double p2 = ((2.0 * (d - 1) + 1.0) * t * p1 - (d - 1) * p0) / d;
            p0 = p1;
            p1 = p2;
            v = p2;
          }
          leg[((size_t)a * (maxdeg + 1) + d) * nmax + i] = (n == 1 && d > 0) ? (d == 0 ? 1.0 : 0.0) : v;
        }
      }
    }
    if ((rc = ws->leg.ensure(leg.size() * 8, &ctx->budget, "legendre"))) return rc;
    SY_HIP(hipMemcpyAsync(ws->leg.get(), leg.data(), leg.size() * 8, hipMemcpyHostToDevice, s));
    SY_HIP(hipStreamSynchronize(s));
    ws->maxdeg = maxdeg;
  }
  return MP_OK;
}

template <typename R>
static int fft_nd(mp_ctx* ctx, SymbolWS* ws, Cx<R>* data, int inverse, hipStream_t s) {
  const Config& c = ctx->cfg;
  const int n3[3] = {c.nx, c.ny, c.nz};
  const long long stride3[3] = {1, (long long)c.nx, (long long)c.nx * c.ny};
  const long long total = cells_of(c);
  for (int a = 0; a < 3; ++a) {
    const int n = n3[a];
    if (n == 1) continue;
    LineMap m;
    m.n = n;
    m.logn = 0;
    while ((1 << m.logn) < n) ++m.logn;
    m.nlines = (int)(total / n);
    m.lpb = std::max(1, 2048 / n);
    m.es = stride3[a];
    if (a == 0) {
      m.B = 1; m.S0 = 0; m.S1 = n;
    } else {
      m.B = (int)stride3[a];
      m.S0 = 1;
      m.S1 = stride3[a] * n;
    }
    const Cx<R>* tw = (sizeof(R) == 8) ? ws->twd[a].as<Cx<R>>() : ws->twf[a].as<Cx<R>>();
    const size_t shm = 2 * (size_t)m.lpb * n * sizeof(Cx<R>);
    const int blocks = (m.nlines + m.lpb - 1) / m.lpb;
    hipLaunchKernelGGL(k_fft<R>, dim3(blocks), dim3(256), shm, s, data, m, tw, inverse);
    SY_LAUNCH();
  }
  return MP_OK;
}

static int check_grid(const Config& c) {
  if (!pow2(c.nx) || !pow2(c.ny) || !pow2(c.nz) || c.nx > 1024 || c.ny > 1024 || c.nz > 1024) {
    set_error("the probing basis needs power-of-two model sizes up to 1024 per axis");
    return MP_EUNSUPPORTED;
  }
  return MP_OK;
}

static SymbolWS* ws_of(mp_ctx* ctx) {
  if (!ctx->symbol_ws) ctx->symbol_ws = new SymbolWS();
  return static_cast<SymbolWS*>(ctx->symbol_ws);
}

static Grid3 grid3(const Config& c) {
  Grid3 g;
  g.n[0] = c.nx;
  g.n[1] = c.ny;
  g.n[2] = c.nz;
  g.cells = cells_of(c);
  return g;
}

// position-factor specs (kind, n_x, n_y, n_z, phase) of the basis terms: Legendre
// degrees (family 0, y = 0 in 2D) or Fourier mode numbers and phase (family 1)
static std::vector<int> specs5(const Basis& b) {
  std::vector<int> d((size_t)b.na() * 5, 0);
  for (int a = 0; a < b.na(); ++a) {
    int* o = &d[5 * (size_t)a];
    if (b.family == 0) {
      o[1] = b.degs[(size_t)a * b.ndim + 0];
      if (b.ndim == 3) o[2] = b.degs[(size_t)a * b.ndim + 1];
      o[3] = b.degs[(size_t)a * b.ndim + (b.ndim - 1)];
    } else {
      o[0] = 1;
      for (int k = 0; k < 4; ++k) o[1 + k] = b.modes[4 * (size_t)a + k];
    }
  }
  return d;
}
static int max_degree(const Basis& b) {
  int m = 0;
  if (b.family == 0)
    for (int v : b.degs) m = std::max(m, v);
  return m;
}
// multiplier parameters as the kernel reads them: powers of rho (family 0) or
// (angular index, rational Chebyshev degree) pairs (family 1)
static const std::vector<int>& mult_table(const Basis& b) { return b.family == 0 ? b.qs : b.mults; }

template <typename T, typename R>
static int apply_t(mp_ctx* ctx, const Basis& b, const double* c, const void* img, void* out, hipStream_t s) {
  SymbolWS* ws = ws_of(ctx);
  const Config& cf = ctx->cfg;
  const long long n = cells_of(cf);
  const std::vector<int> sp = specs5(b);
  const std::vector<int>& mt = mult_table(b);
  int rc;
  if ((rc = ensure_tables(ctx, ws, max_degree(b), s))) return rc;
  if ((rc = ws->cx0.ensure(sizeof(Cx<R>) * n, &ctx->budget, "fft work"))) return rc;
  if ((rc = ws->cx1.ensure(sizeof(Cx<R>) * n, &ctx->budget, "fft work"))) return rc;
  if ((rc = ws->qs.ensure(sizeof(int) * 2 * MAXP, &ctx->budget, "basis"))) return rc;
  if ((rc = ws->coef.ensure(sizeof(double) * MAXP, &ctx->budget, "basis"))) return rc;
  if ((rc = ws->degs.ensure(sizeof(int) * 5 * MAXP, &ctx->budget, "basis"))) return rc;
  SY_HIP(hipMemcpyAsync(ws->degs.get(), sp.data(), sizeof(int) * sp.size(), hipMemcpyHostToDevice, s));
  Cx<R>* X = ws->cx0.as<Cx<R>>();
  Cx<R>* Y = ws->cx1.as<Cx<R>>();
  hipLaunchKernelGGL((k_to_complex<R, T>), egrid(n), dim3(256), 0, s, X, static_cast<const T*>(img), n);
  SY_LAUNCH();
  if ((rc = fft_nd<R>(ctx, ws, X, 0, s))) return rc;
  const Grid3 g = grid3(cf);
  const int nq = b.nq();
  SY_HIP(hipMemcpyAsync(ws->qs.get(), mt.data(), sizeof(int) * mt.size(), hipMemcpyHostToDevice, s));
  // p <= MAXP coefficients into the workspace's table (stream-ordered after earlier users)
  SY_HIP(hipMemcpyAsync(ws->coef.get(), c, sizeof(double) * (size_t)b.na() * nq, hipMemcpyHostToDevice, s));
  for (int a = 0; a < b.na(); ++a) {
    hipLaunchKernelGGL(k_multiplier<R>, egrid(n), dim3(256), 0, s, Y, X, g, nq, ws->qs.as<int>(),
                       ws->coef.as<double>() + (size_t)a * nq, b.family, b.ndim, b.order, b.tl_scale);
    SY_LAUNCH();
    if ((rc = fft_nd<R>(ctx, ws, Y, 1, s))) return rc;
    hipLaunchKernelGGL((k_accum_out<R, T>), egrid(n), dim3(256), 0, s, static_cast<T*>(out), Y, g,
                       ws->leg.as<double>(), ws->maxdeg, ws->degs.as<int>() + 5 * a, 1.0 / (double)n, a == 0 ? 1 : 0);
    SY_LAUNCH();
  }
  SY_HIP(hipStreamSynchronize(s));   // the host tables copied above outlive the copies
  return MP_OK;
}

int model_fft(mp_ctx* ctx, void* data, bool f64, int inverse, hipStream_t s) {
  int rc = check_grid(ctx->cfg);
  if (rc) return rc;
  SymbolWS* ws = ws_of(ctx);
  if ((rc = ensure_tables(ctx, ws, 0, s))) return rc;
  if (f64) return fft_nd<double>(ctx, ws, static_cast<Cx<double>*>(data), inverse, s);
  return fft_nd<float>(ctx, ws, static_cast<Cx<float>*>(data), inverse, s);
}

int symbol_apply(mp_ctx* ctx, const Basis& b, const double* c, const void* img, void* out, hipStream_t s) {
  int rc = check_grid(ctx->cfg);
  if (rc) return rc;
  if (ctx->cfg.dtype == MP_F32) return apply_t<float, float>(ctx, b, c, img, out, s);
  return apply_t<double, double>(ctx, b, c, img, out, s);
}

template <typename T>
static int fit_t(mp_ctx* ctx, const Basis& b, int T_, const void* const* y, const void* const* x, double* c,
                 double* relres, hipStream_t s) {
  SymbolWS* ws = ws_of(ctx);
  const Config& cf = ctx->cfg;
  const long long n = cells_of(cf);
  const int p = b.na() * b.nq();
  const long long nrows = n * T_;
  const long long lda = (nrows + 63) / 64 * 64;
  const std::vector<int> sp = specs5(b);
  const std::vector<int>& mt = mult_table(b);
  int rc;
  if ((rc = ensure_tables(ctx, ws, max_degree(b), s))) return rc;
  if ((rc = ws->cx0.ensure(sizeof(Cx<double>) * n, &ctx->budget, "fft work"))) return rc;
  if ((rc = ws->cx1.ensure(sizeof(Cx<double>) * n, &ctx->budget, "fft work"))) return rc;
  if ((rc = ws->A.ensure(sizeof(double) * (size_t)(p + 1) * lda, &ctx->budget, "fit columns"))) return rc;
  const int nwg = (int)std::min<long long>(GWGMAX, std::max<long long>(1, (nrows + 8 * GRB - 1) / (8 * GRB)));
  if ((rc = ws->part.ensure(sizeof(double) * (size_t)std::max(nwg * GCOL * GCOL, 4096), &ctx->budget, "partials")))
    return rc;
  if ((rc = ws->G0.ensure(sizeof(double) * GCOL * GCOL, &ctx->budget, "gram"))) return rc;
  if ((rc = ws->small.ensure(sizeof(Small), &ctx->budget, "solve"))) return rc;
  if ((rc = ws->qs.ensure(sizeof(int) * 2 * MAXP, &ctx->budget, "basis"))) return rc;
  if ((rc = ws->coef.ensure(sizeof(double) * MAXP, &ctx->budget, "basis"))) return rc;
  if ((rc = ws->degs.ensure(sizeof(int) * 5 * MAXP, &ctx->budget, "basis"))) return rc;
  SY_HIP(hipMemcpyAsync(ws->degs.get(), sp.data(), sizeof(int) * sp.size(), hipMemcpyHostToDevice, s));
  double* A = ws->A.as<double>();
  Cx<double>* X = ws->cx0.as<Cx<double>>();
  Cx<double>* Y = ws->cx1.as<Cx<double>>();
  const Grid3 g = grid3(cf);
  const int nq = b.nq();
  SY_HIP(hipMemcpyAsync(ws->qs.get(), mt.data(), sizeof(int) * mt.size(), hipMemcpyHostToDevice, s));
  const double one = 1.0;
  SY_HIP(hipMemcpyAsync(ws->coef.get(), &one, sizeof(double), hipMemcpyHostToDevice, s));
  SY_HIP(hipStreamSynchronize(s));
  // columns: A[(a, q)][t*n + i] = P_a(i) Re IFFT(m_q FFT x_t)(i); A[p][t*n + i] = y_t(i)
  for (int t = 0; t < T_; ++t) {
    hipLaunchKernelGGL((k_to_complex<double, T>), egrid(n), dim3(256), 0, s, X, static_cast<const T*>(x[t]), n);
    SY_LAUNCH();
    if ((rc = fft_nd<double>(ctx, ws, X, 0, s))) return rc;
    for (int q = 0; q < nq; ++q) {
      hipLaunchKernelGGL(k_multiplier<double>, egrid(n), dim3(256), 0, s, Y, X, g, 1,
                         ws->qs.as<int>() + (b.family == 0 ? q : 2 * q), ws->coef.as<double>(), b.family, b.ndim,
                         b.order, b.tl_scale);
      SY_LAUNCH();
      if ((rc = fft_nd<double>(ctx, ws, Y, 1, s))) return rc;
      hipLaunchKernelGGL(k_columns, egrid(n), dim3(256), 0, s, A, lda, (long long)t * n, Y, g, ws->leg.as<double>(),
                         ws->maxdeg, b.na(), nq, q, ws->degs.as<int>(), 1.0 / (double)n);
      SY_LAUNCH();
    }
    hipLaunchKernelGGL((k_column_copy<T>), egrid(n), dim3(256), 0, s, A, lda, p, (long long)t * n,
                       static_cast<const T*>(y[t]), n);
    SY_LAUNCH();
  }
  Small* W = ws->small.as<Small>();
  auto gram = [&](double* Gdst) -> int {
    gram_partials(dim3(nwg), s, A, lda, nrows, p + 1, ws->part.as<double>());
    SY_LAUNCH();
    hipLaunchKernelGGL(k_gram_reduce, dim3(((p + 1) * (p + 1) + 63) / 64), dim3(64 * RDW), 0, s, ws->part.as<double>(), nwg,
                       p + 1, Gdst);
    SY_LAUNCH();
    return MP_OK;
  };
  const dim3 qgrid = egrid(nrows);
  // pass 1 (equilibrated, shifted), pass 2, then the final solve on the third Gram
  if ((rc = gram(ws->G0.as<double>()))) return rc;
  SY_HIP(hipMemcpyAsync(W->G, ws->G0.get(), sizeof(double) * (p + 1) * (p + 1), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_cqr_pass, dim3(1), dim3(256), 0, s, W, p, nrows, 0);
  SY_LAUNCH();
  qupdate(qgrid, s, A, lda, nrows, p, W);
  SY_LAUNCH();
  if ((rc = gram(W->G))) return rc;
  hipLaunchKernelGGL(k_cqr_pass, dim3(1), dim3(256), 0, s, W, p, nrows, 1);
  SY_LAUNCH();
  qupdate(qgrid, s, A, lda, nrows, p, W);
  SY_LAUNCH();
  if ((rc = gram(W->G))) return rc;
  hipLaunchKernelGGL(k_cqr_solve, dim3(1), dim3(256), 0, s, W, p);
  SY_LAUNCH();
  hipLaunchKernelGGL(k_resid, dim3(256), dim3(256), 0, s, A, lda, nrows, p, W, ws->part.as<double>());
  SY_LAUNCH();
  Small h;
  SY_HIP(hipMemcpyAsync(&h, W, sizeof(Small), hipMemcpyDeviceToHost, s));
  std::vector<double> rp(256);
  SY_HIP(hipMemcpyAsync(rp.data(), ws->part.get(), sizeof(double) * 256, hipMemcpyDeviceToHost, s));
  SY_HIP(hipStreamSynchronize(s));
  bool deficient = false;
  if (!h.status) {
    double smax = 0.0, smin = 1e300;
    for (int i = 0; i < p; ++i) {
      smax = std::max(smax, h.sig[i]);
      smin = std::min(smin, h.sig[i]);
    }
    deficient = !(smin > 1e-12 * smax);
    double rr = 0.0;
    for (int i = 0; i < 256; ++i) rr += rp[i];
    if (relres) *relres = (h.bb > 0.0) ? std::sqrt(rr / h.bb) : 0.0;
  }
  if (h.status || deficient) {
    // rank deficient (a Cholesky pivot failed, or the singular-value test): the
    // minimum-norm solution of the column-equilibrated normal equations, from the
    // first Gram matrix; the residual from the same Gram, ||b||^2 - 2 c.r + c.G c
    hipLaunchKernelGGL(k_minnorm, dim3(1), dim3(256), 0, s, W, ws->G0.as<double>(), p, 1e-13);
    SY_LAUNCH();
    std::vector<double> G((size_t)(p + 1) * (p + 1));
    SY_HIP(hipMemcpyAsync(&h, W, sizeof(Small), hipMemcpyDeviceToHost, s));
    SY_HIP(hipMemcpyAsync(G.data(), ws->G0.get(), sizeof(double) * G.size(), hipMemcpyDeviceToHost, s));
    SY_HIP(hipStreamSynchronize(s));
    deficient = true;
    if (relres) {
      const int ld = p + 1;
      double rr = G[(size_t)p * ld + p];
      for (int i = 0; i < p; ++i) {
        rr -= 2.0 * h.c[i] * G[(size_t)i * ld + p];
        for (int j = 0; j < p; ++j) rr += h.c[i] * G[(size_t)i * ld + j] * h.c[j];
      }
      const double bb = G[(size_t)p * ld + p];
      *relres = (bb > 0.0) ? std::sqrt(std::max(rr, 0.0) / bb) : 0.0;
    }
  }
  for (int i = 0; i < p; ++i) c[i] = h.c[i];
  if (deficient) {
    set_error("probing system is numerically rank deficient; minimum-norm coefficients returned");
    return MP_ENUMERIC;
  }
  return MP_OK;
}

int symbol_fit(mp_ctx* ctx, const Basis& b, int T, const void* const* y, const void* const* x, double* c,
               double* relres, hipStream_t s) {
  int rc = check_grid(ctx->cfg);
  if (rc) return rc;
  if (b.na() * b.nq() > MAXP) {
    set_error("at most 64 basis terms");
    return MP_EUNSUPPORTED;
  }
  if (ctx->cfg.dtype == MP_F32) return fit_t<float>(ctx, b, T, y, x, c, relres, s);
  return fit_t<double>(ctx, b, T, y, x, c, relres, s);
}

void symbol_release(mp_ctx* ctx) {
  delete static_cast<SymbolWS*>(ctx->symbol_ws);
  ctx->symbol_ws = nullptr;
}

}  // namespace mp
