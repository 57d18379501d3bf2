// Curvelet-space trial functions and the illumination mask (paper Sec. 1.5, Sec. 2) on
// the 2D model grid.
//
// Frame: undecimated curvelets built in the frequency domain.  With the normalised
// frequency u = (f_x / (nx/2), f_z / (nz/2)), r = |u|, theta = atan2(u_z, u_x) mod pi,
// the smooth step nu(t) = t^4 (35 - 84 t + 70 t^2 - 20 t^3) and the octave lowpass
// Phi(s) (1 up to s = 1, cos(pi/2 nu(s - 1)) to 0 at s = 2): L_j(r) = Phi(r / 2^(j-J+1))
// for j < J-1, L_(J-1) = 1; W_0 = L_0 and W_j = sqrt(L_j^2 - L_(j-1)^2); band j >= 1 has
// A_j = A_1 2^floor((j-1)/2) directions over a half turn with windows V_(j,l) (rising
// sin(pi/2 nu(s)), falling cos(pi/2 nu(s - 1)), s = theta A_j / pi - l + 1/2 mod A_j).
// Wedge windows U = W_j V_(j,l) (U_0 = W_0) are replaced by the root mean square of
// their values at xi and -xi (the Nyquist row and column alias +f and -f), so each is
// even and sum_w U_w^2 = 1: the atoms IFFT(U_w)(x - x_k), one per grid point, are a
// tight frame.  Synthesis sum_w IFFT(U_w FFT(weight_w mask_w C_w)); analysis
// C_w = IFFT(U_w FFT f).  The windows are tabulated on the host in FP64.
//
// Visibility: from each coarse node (every `stride` cells) and each wedge direction,
// a fan of ray pairs leaves along the upward normal turned by +alpha and -alpha; the
// curvelet centre is visible if, for some alpha, one ray reaches the source row inside
// the sources' span and the other the receiver row inside the receivers' span (spans
// widened by half a cell).  Rays solve dx/dt = c^2 p, dp/dt = -grad(c)/c (traveltime
// parameter) with Dormand-Prince 5(4) steps in FP64: a step is accepted when the
// position difference of the two orders is at most rtol h (else dt halves) and dt
// doubles after a step whose difference is below rtol h / 32; the step length is capped
// at 8 h.  c and its centred-difference gradient (one-sided at the edges) are
// interpolated bilinearly between the model nodes.  A ray that leaves the model's box
// before crossing the row, or runs out of steps, misses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "curvelet.h"
#include "symbol.h"

namespace mp {

#define CV_HIP(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_));                  \
      return MP_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)
#define CV_LAUNCH()                                                                   \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_));       \
      return MP_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)

template <typename R>
struct Cx2 {
  R x, y;
};

// ----------------------------------------------------------- host tables --

static double smooth_step(double t) {
  t = std::min(1.0, std::max(0.0, t));
  return t * t * t * t * (35.0 - 84.0 * t + 70.0 * t * t - 20.0 * t * t * t);
}
static double lowpass(double s) {
  if (s <= 1.0) return 1.0;
  if (s >= 2.0) return 0.0;
  return std::cos(0.5 * M_PI * smooth_step(s - 1.0));
}
static double angular(double theta, int l, int A) {
  double s = std::fmod(theta * A / M_PI - l + 0.5, (double)A);
  if (s < 0.0) s += A;
  if (s < 1.0) return std::sin(0.5 * M_PI * smooth_step(s));
  if (s < 2.0) return std::cos(0.5 * M_PI * smooth_step(s - 1.0));
  return 0.0;
}

int cv_directions(int j, int A1) { return A1 << ((j - 1) / 2); }

std::vector<int> cv_wedges(int J, int A1) {
  std::vector<int> w = {0, 0, 0};
  for (int j = 1; j < J; ++j) {
    const int A = cv_directions(j, A1);
    for (int l = 0; l < A; ++l) {
      w.push_back(j);
      w.push_back(l);
      w.push_back(A);
    }
  }
  return w;
}

// distinct directions (A, l), A increasing
static std::vector<int> direction_set(int J, int A1) {
  std::vector<int> As;
  for (int j = 1; j < J; ++j) {
    const int A = cv_directions(j, A1);
    if (std::find(As.begin(), As.end(), A) == As.end()) As.push_back(A);
  }
  std::sort(As.begin(), As.end());
  std::vector<int> d;
  for (int A : As)
    for (int l = 0; l < A; ++l) {
      d.push_back(A);
      d.push_back(l);
    }
  return d;
}

// U[w][z][x] before symmetrisation
static void raw_windows(int nz, int nx, int J, int A1, std::vector<double>& U) {
  const std::vector<int> wl = cv_wedges(J, A1);
  const int nw = (int)wl.size() / 3;
  const long long n = (long long)nz * nx;
  U.assign((size_t)nw * n, 0.0);
  for (int iz = 0; iz < nz; ++iz) {
    const int fz = iz < nz / 2 ? iz : iz - nz;
    const double uz = fz / (nz / 2.0);
    for (int ix = 0; ix < nx; ++ix) {
      const int fx = ix < nx / 2 ? ix : ix - nx;
      const double ux = fx / (nx / 2.0);
      const double r = std::hypot(ux, uz);
      double th = std::fmod(std::atan2(uz, ux), M_PI);
      if (th < 0.0) th += M_PI;
      double L[32];
      for (int j = 0; j < J - 1; ++j) L[j] = lowpass(r / std::ldexp(1.0, j - J + 1));
      L[J - 1] = 1.0;
      double W[32];
      W[0] = L[0];
      for (int j = 1; j < J; ++j) W[j] = std::sqrt(std::max(L[j] * L[j] - L[j - 1] * L[j - 1], 0.0));
      const long long i = (long long)iz * nx + ix;
      for (int w = 0; w < nw; ++w) {
        const int j = wl[3 * w], l = wl[3 * w + 1], A = wl[3 * w + 2];
        U[(size_t)w * n + i] = (j == 0) ? W[0] : W[j] * angular(th, l, A);
      }
    }
  }
}

static void windows(int nz, int nx, int J, int A1, std::vector<double>& U) {
  std::vector<double> raw;
  raw_windows(nz, nx, J, A1, raw);
  const long long n = (long long)nz * nx;
  const int nw = (int)(raw.size() / n);
  U.resize(raw.size());
  for (int w = 0; w < nw; ++w)
    for (int iz = 0; iz < nz; ++iz)
      for (int ix = 0; ix < nx; ++ix) {
        const double a = raw[(size_t)w * n + (long long)iz * nx + ix];
        const double b = raw[(size_t)w * n + (long long)((nz - iz) % nz) * nx + (nx - ix) % nx];
        U[(size_t)w * n + (long long)iz * nx + ix] = std::sqrt(0.5 * (a * a + b * b));
      }
}

// ---------------------------------------------------------------- kernels --

static dim3 cgrid(long long n) {
  long long b = (n + 255) / 256;
  return dim3((unsigned)std::max<long long>(1, std::min<long long>(b, 16384)));
}

// out = weight * mask * coef as complex
template <typename T, typename R>
__global__ void k_cv_prep(Cx2<R>* out, const T* coef, const unsigned char* mask, double weight, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R v = (mask == nullptr || mask[i]) ? (R)(weight * (double)coef[i]) : R(0);
    out[i] = {v, R(0)};
  }
}

// acc (+)= U * X
template <typename R>
__global__ void k_cv_accum(Cx2<R>* acc, const Cx2<R>* X, const R* U, long long n, int first) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R u = U[i];
    const Cx2<R> x = X[i];
    if (first) acc[i] = {u * x.x, u * x.y};
    else acc[i] = {acc[i].x + u * x.x, acc[i].y + u * x.y};
  }
}

// Y = U * F
template <typename R>
__global__ void k_cv_mul(Cx2<R>* Y, const Cx2<R>* F, const R* U, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R u = U[i];
    Y[i] = {u * F[i].x, u * F[i].y};
  }
}

template <typename T, typename R>
__global__ void k_cv_real(T* out, const Cx2<R>* X, double scale, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = (T)((double)X[i].x * scale);
}

template <typename T>
__global__ void k_cv_to_complex(Cx2<T>* out, const T* in, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = {in[i], T(0)};
}

// coef <- sign(coef) where |coef| >= t, 0 elsewhere (magnitudes to one, signs kept)
template <typename T>
__global__ void k_cv_sign(T* coef, long long n, double t) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = (double)coef[i];
    coef[i] = (T)(fabs(v) >= t ? (v > 0.0 ? 1.0 : -1.0) : 0.0);
  }
}

// medium tables: c (FP64) and its centred-difference gradient, one-sided at the edges
template <typename T>
__global__ void k_cv_medium(double* c, double* gx, double* gz, const T* cin, int nx, int nz, double h) {
  const long long n = (long long)nx * nz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % nx), iz = (int)(i / nx);
    auto at = [&](int x, int z) { return (double)cin[(long long)z * nx + x]; };
    c[i] = at(ix, iz);
    double ddx = 0.0, ddz = 0.0;
    if (nx > 1) {
      if (ix == 0) ddx = (at(1, iz) - at(0, iz)) / h;
      else if (ix == nx - 1) ddx = (at(nx - 1, iz) - at(nx - 2, iz)) / h;
      else ddx = (at(ix + 1, iz) - at(ix - 1, iz)) / (2.0 * h);
    }
    if (nz > 1) {
      if (iz == 0) ddz = (at(ix, 1) - at(ix, 0)) / h;
      else if (iz == nz - 1) ddz = (at(ix, nz - 1) - at(ix, nz - 2)) / h;
      else ddz = (at(ix, iz + 1) - at(ix, iz - 1)) / (2.0 * h);
    }
    gx[i] = ddx;
    gz[i] = ddz;
  }
}

struct RayJob {
  const double* c;
  const double* gx;
  const double* gz;
  int nx, nz;
  double h;
  int nnx, nnz, stride;     // coarse nodes per axis, node spacing
  const double* dirs;       // [ndir][nfan][4]: (dx+, dz+, dx-, dz-)
  int ndir, nfan;
  double zS, sl, sh, zR, rl, rh;
  double tol2;              // (rtol h)^2
  int max_steps;
  unsigned char* hits;      // [ndir][nnz][nnx][nfan]
};

struct Med3 {
  double c, cx, cz;
};

__device__ __forceinline__ double bil(const double* a, int nx, long long i00, int dx1, int dz1, double tx, double tz) {
  const double top = a[i00] * (1.0 - tx) + a[i00 + dx1] * tx;
  const double bot = a[i00 + dz1] * (1.0 - tx) + a[i00 + dz1 + dx1] * tx;
  return top * (1.0 - tz) + bot * tz;
}

__device__ __forceinline__ Med3 medium_at(const RayJob& J, double x, double z) {
  const double fx = fmin(fmax(x / J.h, 0.0), (double)(J.nx - 1));
  const double fz = fmin(fmax(z / J.h, 0.0), (double)(J.nz - 1));
  const int ix = J.nx > 1 ? min((int)floor(fx), J.nx - 2) : 0;
  const int iz = J.nz > 1 ? min((int)floor(fz), J.nz - 2) : 0;
  const double tx = fx - ix, tz = fz - iz;
  const int dx1 = J.nx > 1 ? 1 : 0;
  const int dz1 = J.nz > 1 ? J.nx : 0;
  const long long i00 = (long long)iz * J.nx + ix;
  Med3 m;
  m.c = bil(J.c, J.nx, i00, dx1, dz1, tx, tz);
  m.cx = bil(J.gx, J.nx, i00, dx1, dz1, tx, tz);
  m.cz = bil(J.gz, J.nx, i00, dx1, dz1, tx, tz);
  return m;
}

__device__ __forceinline__ void ray_rhs(const RayJob& J, const double y[4], double k[4]) {
  const Med3 m = medium_at(J, y[0], y[1]);
  k[0] = m.c * m.c * y[2];
  k[1] = m.c * m.c * y[3];
  k[2] = -m.cx / m.c;
  k[3] = -m.cz / m.c;
}

// Dormand-Prince 5(4) tableau (Dormand and Prince, 1980)
__constant__ double DPA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
__constant__ double DPB5[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
__constant__ double DPB4[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100,
                               1.0 / 40};

// true if the ray from (x0, z0) along (dx, dz) crosses depth zs upwards inside the box;
// xc: the crossing abscissa
__device__ bool trace(const RayJob& J, double x0, double z0, double dx, double dz, double zs, double& xc) {
  if (z0 <= zs) {
    xc = x0;
    return z0 == zs;
  }
  const double h = J.h;
  const double xmax = (J.nx - 1) * h, zmax = (J.nz - 1) * h;
  const double c0 = medium_at(J, x0, z0).c;
  double y[4] = {x0, z0, dx / c0, dz / c0};
  double dt = 0.5 * h / c0;
  for (int step = 0; step < J.max_steps; ++step) {
    double k[7][4];
    for (int s = 0; s < 7; ++s) {
      double ys[4] = {y[0], y[1], y[2], y[3]};
      for (int m = 0; m < s; ++m) {
        const double a = DPA[s][m];
        if (a != 0.0)
          for (int q = 0; q < 4; ++q) ys[q] = ys[q] + dt * a * k[m][q];
      }
      ray_rhs(J, ys, k[s]);
    }
    double y5[4] = {y[0], y[1], y[2], y[3]}, y4[4] = {y[0], y[1], y[2], y[3]};
    for (int m = 0; m < 7; ++m) {
      for (int q = 0; q < 4; ++q) {
        if (DPB5[m] != 0.0) y5[q] = y5[q] + dt * DPB5[m] * k[m][q];
        if (DPB4[m] != 0.0) y4[q] = y4[q] + dt * DPB4[m] * k[m][q];
      }
    }
    const double ex = y5[0] - y4[0], ez = y5[1] - y4[1];
    const double e2 = ex * ex + ez * ez;
    if (!(e2 <= J.tol2)) {
      dt = dt * 0.5;
      continue;
    }
    if (y5[1] <= zs) {
      const double f = (y[1] - zs) / (y[1] - y5[1]);
      xc = y[0] + (y5[0] - y[0]) * f;
      return xc >= 0.0 && xc <= xmax;
    }
    if (y5[0] < 0.0 || y5[0] > xmax || y5[1] > zmax) return false;
    for (int q = 0; q < 4; ++q) y[q] = y5[q];
    const double nd = (e2 < J.tol2 / 1024.0) ? dt * 2.0 : dt;
    dt = fmin(nd, 8.0 * h / medium_at(J, y[0], y[1]).c);
  }
  return false;
}

// one thread per (direction, node, fan angle): 1 if the pair links the two manifolds
__global__ __launch_bounds__(256) void k_cv_rays(RayJob J) {
  const long long total = (long long)J.ndir * J.nnz * J.nnx * J.nfan;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % J.nfan);
    long long r = t / J.nfan;
    const int b = (int)(r % J.nnx);
    r /= J.nnx;
    const int a = (int)(r % J.nnz);
    const int d = (int)(r / J.nnz);
    const int zi = min(a * J.stride + (J.stride - 1) / 2, J.nz - 1);
    const int xi = min(b * J.stride + (J.stride - 1) / 2, J.nx - 1);
    const double x0 = xi * J.h, z0 = zi * J.h;
    const double* dv = J.dirs + ((long long)d * J.nfan + i) * 4;
    bool sp, rp, sm, rm;
    double xc;
    {
      const bool okS = trace(J, x0, z0, dv[0], dv[1], J.zS, xc);
      sp = okS && xc >= J.sl && xc <= J.sh;
      if (J.zR == J.zS) rp = okS && xc >= J.rl && xc <= J.rh;
      else {
        const bool okR = trace(J, x0, z0, dv[0], dv[1], J.zR, xc);
        rp = okR && xc >= J.rl && xc <= J.rh;
      }
    }
    {
      const bool okS = trace(J, x0, z0, dv[2], dv[3], J.zS, xc);
      sm = okS && xc >= J.sl && xc <= J.sh;
      if (J.zR == J.zS) rm = okS && xc >= J.rl && xc <= J.rh;
      else {
        const bool okR = trace(J, x0, z0, dv[2], dv[3], J.zR, xc);
        rm = okR && xc >= J.rl && xc <= J.rh;
      }
    }
    J.hits[t] = ((sp && rm) || (rp && sm)) ? 1 : 0;
  }
}

// mask[w][iz][ix] from the fan hits: wedge (j, l) its direction's value at its node,
// the lowpass any direction of band 1
__global__ void k_cv_mask(unsigned char* mask, const unsigned char* hits, const int* wdir, int nw, int nx, int nz,
                          int stride, int nnx, int nnz, int nfan, int lp_first, int lp_count) {
  const long long n = (long long)nw * nz * nx;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(t % nx);
    const long long r = t / nx;
    const int iz = (int)(r % nz);
    const int w = (int)(r / nz);
    const int a = iz / stride, b = ix / stride;
    const int d0 = (w == 0) ? lp_first : wdir[w];
    const int d1 = (w == 0) ? lp_first + lp_count : wdir[w] + 1;
    unsigned char v = 0;
    for (int d = d0; d < d1 && !v; ++d) {
      const unsigned char* hp = hits + (((long long)d * nnz + a) * nnx + b) * nfan;
      for (int i = 0; i < nfan; ++i) v |= hp[i];
    }
    mask[t] = v;
  }
}

// ---------------------------------------------------------------- host --

struct CurveletWS {
  int J = -1, A1 = -1, dtype = -1;
  int nw = 0;
  DevBuf U;            // [nw][n] R
  DevBuf F, X, acc;    // complex work
  DevBuf med;          // c, gx, gz (FP64)
  DevBuf dirs, hits, wdir;
  std::vector<double> norms;
};

static CurveletWS* cws(mp_ctx* ctx) {
  if (!ctx->curvelet_ws) ctx->curvelet_ws = new CurveletWS();
  return static_cast<CurveletWS*>(ctx->curvelet_ws);
}

static int check_cv(const mp_ctx* ctx, const Curvelets& cv) {
  const Config& c = ctx->cfg;
  if (c.ndim != 2) {
    set_error("curvelets are built for 2D grids");
    return MP_EUNSUPPORTED;
  }
  auto pow2 = [](int n) { return n >= 2 && (n & (n - 1)) == 0; };
  if (!pow2(c.nx) || !pow2(c.nz) || c.nx > 1024 || c.nz > 1024) {
    set_error("curvelets need power-of-two model sizes up to 1024 per axis");
    return MP_EUNSUPPORTED;
  }
  (void)cv;
  return MP_OK;
}

template <typename R>
static int ensure_windows(mp_ctx* ctx, CurveletWS* ws, const Curvelets& cv, hipStream_t s) {
  const Config& c = ctx->cfg;
  const long long n = (long long)c.nx * c.nz;
  int rc;
  if (ws->J == cv.nscales && ws->A1 == cv.nangles && ws->dtype == c.dtype) return MP_OK;
  std::vector<double> U;
  windows(c.nz, c.nx, cv.nscales, cv.nangles, U);
  const int nw = (int)(U.size() / n);
  std::vector<R> Ur(U.begin(), U.end());
  if ((rc = ws->U.ensure(sizeof(R) * Ur.size(), &ctx->budget, "curvelet windows"))) return rc;
  CV_HIP(hipMemcpyAsync(ws->U.get(), Ur.data(), sizeof(R) * Ur.size(), hipMemcpyHostToDevice, s));
  ws->norms.assign(nw, 0.0);
  for (int w = 0; w < nw; ++w) {
    double acc = 0.0;
    for (long long i = 0; i < n; ++i) acc += U[(size_t)w * n + i] * U[(size_t)w * n + i];
    ws->norms[w] = std::sqrt(acc / (double)n);
  }
  CV_HIP(hipStreamSynchronize(s));   // host table outlives the copy
  ws->J = cv.nscales;
  ws->A1 = cv.nangles;
  ws->dtype = c.dtype;
  ws->nw = nw;
  return MP_OK;
}

template <typename T>
static int synth_t(mp_ctx* ctx, const Curvelets& cv, const void* coef, const unsigned char* mask,
                   const double* weights, void* out, hipStream_t s) {
  using R = T;
  CurveletWS* ws = cws(ctx);
  const Config& c = ctx->cfg;
  const long long n = (long long)c.nx * c.nz;
  int rc;
  if ((rc = ensure_windows<R>(ctx, ws, cv, s))) return rc;
  if ((rc = ws->X.ensure(sizeof(Cx2<R>) * n, &ctx->budget, "curvelet work"))) return rc;
  if ((rc = ws->acc.ensure(sizeof(Cx2<R>) * n, &ctx->budget, "curvelet work"))) return rc;
  Cx2<R>* X = ws->X.as<Cx2<R>>();
  Cx2<R>* A = ws->acc.as<Cx2<R>>();
  for (int w = 0; w < ws->nw; ++w) {
    const double wt = weights ? weights[w] : 1.0;
    hipLaunchKernelGGL((k_cv_prep<T, R>), cgrid(n), dim3(256), 0, s, X, static_cast<const T*>(coef) + (long long)w * n,
                       mask ? mask + (long long)w * n : nullptr, wt, n);
    CV_LAUNCH();
    if ((rc = model_fft(ctx, X, sizeof(R) == 8, 0, s))) return rc;
    hipLaunchKernelGGL(k_cv_accum<R>, cgrid(n), dim3(256), 0, s, A, X, ws->U.as<R>() + (long long)w * n, n,
                       w == 0 ? 1 : 0);
    CV_LAUNCH();
  }
  if ((rc = model_fft(ctx, A, sizeof(R) == 8, 1, s))) return rc;
  hipLaunchKernelGGL((k_cv_real<T, R>), cgrid(n), dim3(256), 0, s, static_cast<T*>(out), A, 1.0 / (double)n, n);
  CV_LAUNCH();
  return MP_OK;
}

template <typename T>
static int analysis_t(mp_ctx* ctx, const Curvelets& cv, const void* img, void* coef, hipStream_t s) {
  using R = T;
  CurveletWS* ws = cws(ctx);
  const Config& c = ctx->cfg;
  const long long n = (long long)c.nx * c.nz;
  int rc;
  if ((rc = ensure_windows<R>(ctx, ws, cv, s))) return rc;
  if ((rc = ws->F.ensure(sizeof(Cx2<R>) * n, &ctx->budget, "curvelet work"))) return rc;
  if ((rc = ws->X.ensure(sizeof(Cx2<R>) * n, &ctx->budget, "curvelet work"))) return rc;
  Cx2<R>* F = ws->F.as<Cx2<R>>();
  Cx2<R>* X = ws->X.as<Cx2<R>>();
  hipLaunchKernelGGL(k_cv_to_complex<T>, cgrid(n), dim3(256), 0, s, F, static_cast<const T*>(img), n);
  CV_LAUNCH();
  if ((rc = model_fft(ctx, F, sizeof(R) == 8, 0, s))) return rc;
  for (int w = 0; w < ws->nw; ++w) {
    hipLaunchKernelGGL(k_cv_mul<R>, cgrid(n), dim3(256), 0, s, X, F, ws->U.as<R>() + (long long)w * n, n);
    CV_LAUNCH();
    if ((rc = model_fft(ctx, X, sizeof(R) == 8, 1, s))) return rc;
    hipLaunchKernelGGL((k_cv_real<T, R>), cgrid(n), dim3(256), 0, s, static_cast<T*>(coef) + (long long)w * n, X,
                       1.0 / (double)n, n);
    CV_LAUNCH();
  }
  return MP_OK;
}

// sources or receivers as (row depth, x_lo, x_hi) in metres; false if not on one row
static bool manifold(const std::vector<int>& pts, int count, double h, double& z, double& lo, double& hi) {
  int zr = pts[1], xmin = pts[0], xmax = pts[0];
  for (int i = 0; i < count; ++i) {
    if (pts[2 * i + 1] != zr) return false;
    xmin = std::min(xmin, pts[2 * i]);
    xmax = std::max(xmax, pts[2 * i]);
  }
  z = zr * h;
  lo = (xmin - 0.5) * h;
  hi = (xmax + 0.5) * h;
  return true;
}

template <typename T>
static int illum_t(mp_ctx* ctx, const Curvelets& cv, const void* cdev, unsigned char* mask, hipStream_t s) {
  CurveletWS* ws = cws(ctx);
  const Config& c = ctx->cfg;
  const long long n = (long long)c.nx * c.nz;
  int rc;
  if ((rc = ensure_windows<T>(ctx, ws, cv, s))) return rc;
  RayJob J;
  J.nx = c.nx;
  J.nz = c.nz;
  J.h = c.h;
  J.stride = cv.mask_stride;
  J.nnx = (c.nx + cv.mask_stride - 1) / cv.mask_stride;
  J.nnz = (c.nz + cv.mask_stride - 1) / cv.mask_stride;
  J.nfan = cv.nfan;
  J.tol2 = (cv.ray_rtol * c.h) * (cv.ray_rtol * c.h);
  J.max_steps = cv.max_steps;
  if (!manifold(c.src, c.ns, c.h, J.zS, J.sl, J.sh) || !manifold(c.rec, c.nr, c.h, J.zR, J.rl, J.rh)) {
    set_error("the illumination mask needs the sources on one row and the receivers on one row");
    return MP_EUNSUPPORTED;
  }
  // ray-pair directions of every (A, l) and fan angle, FP64 on the host
  const std::vector<int> ds = direction_set(cv.nscales, cv.nangles);
  J.ndir = (int)ds.size() / 2;
  std::vector<double> dv((size_t)J.ndir * cv.nfan * 4);
  for (int d = 0; d < J.ndir; ++d) {
    const int A = ds[2 * d], l = ds[2 * d + 1];
    const double th = (l + 0.5) * M_PI / A;
    const double ux = -std::cos(th), uz = -std::sin(th);   // the normal, pointing up
    for (int i = 0; i < cv.nfan; ++i) {
      const double al = (i + 0.5) * 0.5 * M_PI / cv.nfan;
      const double ca = std::cos(al), sa = std::sin(al);
      double* o = &dv[((size_t)d * cv.nfan + i) * 4];
      o[0] = ux * ca - uz * sa;
      o[1] = ux * sa + uz * ca;
      o[2] = ux * ca + uz * sa;
      o[3] = -ux * sa + uz * ca;
    }
  }
  // wedge -> direction index
  const std::vector<int> wl = cv_wedges(cv.nscales, cv.nangles);
  const int nw = (int)wl.size() / 3;
  std::vector<int> wdir(nw, 0);
  int lp_first = -1;
  const int A_1 = cv_directions(1, cv.nangles);
  for (int d = 0; d < J.ndir; ++d)
    if (ds[2 * d] == A_1 && ds[2 * d + 1] == 0) lp_first = d;
  for (int w = 1; w < nw; ++w)
    for (int d = 0; d < J.ndir; ++d)
      if (ds[2 * d] == wl[3 * w + 2] && ds[2 * d + 1] == wl[3 * w + 1]) wdir[w] = d;
  const long long nhits = (long long)J.ndir * J.nnz * J.nnx * cv.nfan;
  if ((rc = ws->med.ensure(sizeof(double) * 3 * n, &ctx->budget, "ray medium"))) return rc;
  if ((rc = ws->dirs.ensure(sizeof(double) * dv.size(), &ctx->budget, "ray directions"))) return rc;
  if ((rc = ws->hits.ensure((size_t)nhits, &ctx->budget, "ray hits"))) return rc;
  if ((rc = ws->wdir.ensure(sizeof(int) * nw, &ctx->budget, "ray hits"))) return rc;
  double* med = ws->med.as<double>();
  CV_HIP(hipMemcpyAsync(ws->dirs.get(), dv.data(), sizeof(double) * dv.size(), hipMemcpyHostToDevice, s));
  CV_HIP(hipMemcpyAsync(ws->wdir.get(), wdir.data(), sizeof(int) * nw, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_cv_medium<T>, cgrid(n), dim3(256), 0, s, med, med + n, med + 2 * n, static_cast<const T*>(cdev),
                     c.nx, c.nz, c.h);
  CV_LAUNCH();
  J.c = med;
  J.gx = med + n;
  J.gz = med + 2 * n;
  J.dirs = ws->dirs.as<double>();
  J.hits = ws->hits.as<unsigned char>();
  hipLaunchKernelGGL(k_cv_rays, cgrid(nhits), dim3(256), 0, s, J);
  CV_LAUNCH();
  hipLaunchKernelGGL(k_cv_mask, cgrid((long long)nw * n), dim3(256), 0, s, mask, ws->hits.as<unsigned char>(),
                     ws->wdir.as<int>(), nw, c.nx, c.nz, cv.mask_stride, J.nnx, J.nnz, cv.nfan, lp_first, A_1);
  CV_LAUNCH();
  CV_HIP(hipStreamSynchronize(s));   // host tables outlive the copies
  return MP_OK;
}

int curvelet_wedges(const Curvelets& cv, std::vector<int>& list) {
  list = cv_wedges(cv.nscales, cv.nangles);
  return MP_OK;
}

int curvelet_norms(mp_ctx* ctx, const Curvelets& cv, std::vector<double>& norms, hipStream_t s) {
  int rc = check_cv(ctx, cv);
  if (rc) return rc;
  CurveletWS* ws = cws(ctx);
  rc = ctx->cfg.dtype == MP_F32 ? ensure_windows<float>(ctx, ws, cv, s) : ensure_windows<double>(ctx, ws, cv, s);
  if (rc) return rc;
  norms = ws->norms;
  return MP_OK;
}

int curvelet_synthesis(mp_ctx* ctx, const Curvelets& cv, const void* coef, const unsigned char* mask,
                       const double* weights, void* out, hipStream_t s) {
  int rc = check_cv(ctx, cv);
  if (rc) return rc;
  if (ctx->cfg.dtype == MP_F32) return synth_t<float>(ctx, cv, coef, mask, weights, out, s);
  return synth_t<double>(ctx, cv, coef, mask, weights, out, s);
}

int curvelet_analysis(mp_ctx* ctx, const Curvelets& cv, const void* img, void* coef, hipStream_t s) {
  int rc = check_cv(ctx, cv);
  if (rc) return rc;
  if (ctx->cfg.dtype == MP_F32) return analysis_t<float>(ctx, cv, img, coef, s);
  return analysis_t<double>(ctx, cv, img, coef, s);
}

int curvelet_illumination(mp_ctx* ctx, const Curvelets& cv, const void* c, unsigned char* mask, hipStream_t s) {
  int rc = check_cv(ctx, cv);
  if (rc) return rc;
  if (ctx->cfg.dtype == MP_F32) return illum_t<float>(ctx, cv, c, mask, s);
  return illum_t<double>(ctx, cv, c, mask, s);
}

int curvelet_sign_threshold(mp_ctx* ctx, const Curvelets& cv, void* coef, double t, hipStream_t s) {
  int rc = check_cv(ctx, cv);
  if (rc) return rc;
  const long long n = (long long)cv_wedges(cv.nscales, cv.nangles).size() / 3 * ctx->cfg.nx * ctx->cfg.nz;
  if (ctx->cfg.dtype == MP_F32)
    hipLaunchKernelGGL(k_cv_sign<float>, cgrid(n), dim3(256), 0, s, static_cast<float*>(coef), n, t);
  else
    hipLaunchKernelGGL(k_cv_sign<double>, cgrid(n), dim3(256), 0, s, static_cast<double*>(coef), n, t);
  CV_LAUNCH();
  return MP_OK;
}

void curvelet_release(mp_ctx* ctx) {
  delete static_cast<CurveletWS*>(ctx->curvelet_ws);
  ctx->curvelet_ws = nullptr;
}

}  // namespace mp
