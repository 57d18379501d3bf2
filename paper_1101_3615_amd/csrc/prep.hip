// Element-wise preparation kernels: fills, model <-> propagation-grid
// transfers, the background's kappa, reductions of the per-shot images.
#include "common.h"
#include "prep.h"

namespace mp {

// Fill with 16-byte stores: the body runs from the first 16-byte aligned element;
// the head before it and the tail after it (under 16 bytes each) are stored
// element by element.  p is aligned to sizeof(T).
template <typename T>
__global__ void k_fill(T* p, long long n, T v) {
  constexpr int V = 16 / (int)sizeof(T);
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long step = (long long)gridDim.x * blockDim.x;
  long long head = (long long)((16u - ((unsigned)(unsigned long long)p & 15u)) & 15u) / (long long)sizeof(T);
  if (head > n) head = n;
  const long long nv = (n - head) / V;
  union {
    T e[V];
    uint4 u;
  } pat;
#pragma unroll
  for (int k = 0; k < V; ++k) pat.e[k] = v;
  uint4* q = reinterpret_cast<uint4*>(p + head);
  for (long long i = tid; i < nv; i += step) q[i] = pat.u;
  const long long t0 = head + nv * V;
  if (tid < head) p[tid] = v;
  if (tid < n - t0) p[t0 + tid] = v;
}

template <typename T>
static void fill_t(T* p, long long n, T v, hipStream_t s) {
  if (n <= 0) return;
  constexpr long long V = 16 / (long long)sizeof(T);
  long long blocks = (n / V + 255) / 256 + 1;   // covers the head and tail lanes too
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}
void fill(float* p, long long n, float v, hipStream_t s) { fill_t(p, n, v, s); }
void fill(double* p, long long n, double v, hipStream_t s) { fill_t(p, n, v, s); }
void fill(int* p, long long n, int v, hipStream_t s) { fill_t(p, n, v, s); }
void fill(unsigned short* p, long long n, unsigned short v, hipStream_t s) { fill_t(p, n, v, s); }

// Generic index map between a dense model array [nz][ny][nx] and a padded
// propagation-grid field (2D: y dimension absent).
struct PadMap {
  int nx, ny, nz, nb;
  int nxp, nyp, nzp;
  long long row;     // elements between consecutive propagation rows (x lines)
  long long plane;   // elements between consecutive z planes (3D) or rows (2D)
  long long origin;  // offset of propagation cell (0,0,0)
};

// dst(prop) = model value for model cells, 0 in the layer (zero extension E).
template <typename T>
__global__ void k_extend(T* dst, const T* src, PadMap m) {
  const long long n = (long long)m.nxp * m.nyp * m.nzp;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long step = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    const int x = (int)(i % m.nxp);
    const long long t = i / m.nxp;
    const int y = (int)(t % m.nyp);
    const int z = (int)(t / m.nyp);
    const int xm = x - m.nb, ym = (m.nyp == 1) ? 0 : y - m.nb, zm = z - m.nb;
    T v = T(0);
    if (xm >= 0 && xm < m.nx && ym >= 0 && ym < m.ny && zm >= 0 && zm < m.nz)
      v = src[((long long)zm * m.ny + ym) * m.nx + xm];
    dst[m.origin + (long long)z * m.plane + (long long)y * m.row + x] = v;
  }
}

// kappa(prop) = c^2 dt^2 with c extended by edge replication.
template <typename T>
__global__ void k_kappa(T* dst, const T* c, PadMap m, T dt2) {
  const long long n = (long long)m.nxp * m.nyp * m.nzp;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long step = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    const int x = (int)(i % m.nxp);
    const long long t = i / m.nxp;
    const int y = (int)(t % m.nyp);
    const int z = (int)(t / m.nyp);
    const int xm = min(max(x - m.nb, 0), m.nx - 1);
    const int ym = (m.nyp == 1) ? 0 : min(max(y - m.nb, 0), m.ny - 1);
    const int zm = min(max(z - m.nb, 0), m.nz - 1);
    const T cv = c[((long long)zm * m.ny + ym) * m.nx + xm];
    dst[m.origin + (long long)z * m.plane + (long long)y * m.row + x] = cv * cv * dt2;
  }
}

// max |c| and the count of non-finite or non-positive entries.
template <typename T>
__global__ void k_cstats(const T* c, long long n, unsigned long long* maxbits, unsigned int* bad) {
  // maximum in the field precision, exact: positive doubles order as their bit patterns
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long step = (long long)gridDim.x * blockDim.x;
  double m = 0.0;
  unsigned int nb = 0;
  for (; i < n; i += step) {
    const T v = c[i];
    if (!(v > T(0)) || !(v < T(1e30))) ++nb;
    else m = fmax(m, (double)v);
  }
  for (int o = 32; o > 0; o >>= 1) {
    m = fmax(m, __shfl_xor(m, o));
    nb += __shfl_xor(nb, o);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
    if (nb) atomicAdd(bad, nb);
  }
}

// out[model] = sum over shots (in increasing order) of img[s][model], rounded to T.
template <typename T>
__global__ void k_stack(T* out, const double* img, int nshots, long long mstride, int nx, int ny,
                        int nz, int mpitch, int myp) {
  const long long n = (long long)nx * ny * nz;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long step = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    const int x = (int)(i % nx);
    const long long t = i / nx;
    const int y = (int)(t % ny);
    const int z = (int)(t / ny);
    const long long o = ((long long)z * myp + y) * mpitch + x;
    double s = 0.0;
    for (int k = 0; k < nshots; ++k) s += img[(long long)k * mstride + o];
    out[i] = (T)s;
  }
}

static dim3 grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 32768) b = 32768;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

static PadMap padmap(const Pad& p) {
  PadMap m;
  m.nx = p.nx; m.ny = p.ny; m.nz = p.nz; m.nb = p.nb;
  m.nxp = p.nx + 2 * p.nb;
  m.nyp = (p.ny == 1 && p.ndim == 2) ? 1 : p.ny + 2 * p.nb;
  m.nzp = p.nz + 2 * p.nb;
  m.row = p.row; m.plane = p.plane; m.origin = p.origin;
  return m;
}

template <typename T>
static void extend_t(T* dst, const T* src, const Pad& p, hipStream_t s) {
  const PadMap m = padmap(p);
  hipLaunchKernelGGL(k_extend<T>, grid_for((long long)m.nxp * m.nyp * m.nzp), dim3(256), 0, s, dst, src, m);
}
void extend(float* d, const float* m, const Pad& p, hipStream_t s) { extend_t(d, m, p, s); }
void extend(double* d, const double* m, const Pad& p, hipStream_t s) { extend_t(d, m, p, s); }

template <typename T>
static void kappa_t(T* dst, const T* c, const Pad& p, double dt, hipStream_t s) {
  const PadMap m = padmap(p);
  hipLaunchKernelGGL(k_kappa<T>, grid_for((long long)m.nxp * m.nyp * m.nzp), dim3(256), 0, s, dst, c, m,
                     (T)(dt * dt));
}
void kappa(float* d, const float* c, const Pad& p, double dt, hipStream_t s) { kappa_t(d, c, p, dt, s); }
void kappa(double* d, const double* c, const Pad& p, double dt, hipStream_t s) { kappa_t(d, c, p, dt, s); }

template <typename T>
static void cstats_t(const T* c, long long n, unsigned int* out2, hipStream_t s) {
  fill((int*)out2, 3, 0, s);
  hipLaunchKernelGGL(k_cstats<T>, grid_for(n), dim3(256), 0, s, c, n, reinterpret_cast<unsigned long long*>(out2),
                     out2 + 2);
}
void cstats(const float* c, long long n, unsigned int* o, hipStream_t s) { cstats_t(c, n, o, s); }
void cstats(const double* c, long long n, unsigned int* o, hipStream_t s) { cstats_t(c, n, o, s); }

template <typename T>
static void stack_t(T* out, const double* img, int nshots, long long mstride, int nx, int ny, int nz,
                    int mpitch, int myp, hipStream_t s) {
  hipLaunchKernelGGL(k_stack<T>, grid_for((long long)nx * ny * nz), dim3(256), 0, s, out, img, nshots,
                     mstride, nx, ny, nz, mpitch, myp);
}
void stack(float* o, const double* i, int ns, long long ms, int nx, int ny, int nz, int mp, int myp,
           hipStream_t s) {
  stack_t(o, i, ns, ms, nx, ny, nz, mp, myp, s);
}
void stack(double* o, const double* i, int ns, long long ms, int nx, int ny, int nz, int mp, int myp,
           hipStream_t s) {
  stack_t(o, i, ns, ms, nx, ny, nz, mp, myp, s);
}

}  // namespace mp
