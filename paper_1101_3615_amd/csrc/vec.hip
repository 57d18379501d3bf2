// Vector kernels of the solvers built on the operators (steepest descent, conjugate
// gradients, Gauss-Newton): dot products with FP64 accumulation in a fixed order,
// y = alpha x + beta y, and the update of the velocity from a step in m = 1/c^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "prep.h"
#include "vec.h"

namespace mp {

#define VC_HIP(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_));                  \
      return MP_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)
#define VC_LAUNCH() VC_HIP(hipGetLastError())

constexpr int VB = 256;      // threads per block
constexpr int VBLOCKS = 1024;  // blocks of the partial sums (fixed: the summation order is too)

// partial[b] = sum over the elements b, b + VBLOCKS*VB, ... of this block's threads, in a
// fixed tree order
template <typename T>
__global__ __launch_bounds__(VB) void k_dot_part(const T* a, const T* b, long long n, double* partial) {
  __shared__ double s[VB];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * VB + threadIdx.x; i < n; i += (long long)VBLOCKS * VB)
    acc += (double)a[i] * (double)b[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = VB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(VB) void k_dot_final(const double* partial, double* out) {
  __shared__ double s[VB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < VBLOCKS; i += VB) acc += partial[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = VB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// beta == 0 overwrites y without reading it (what y held, NaN included, does not matter)
template <typename T>
__global__ void k_axpby(long long n, double alpha, const T* x, double beta, T* y) {
  const bool read_y = beta != 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = (T)(read_y ? alpha * (double)x[i] + beta * (double)y[i] : alpha * (double)x[i]);
}

// count of cells where c^-2 + dm <= 0 or is not finite
template <typename T>
__global__ void k_vel_check(const T* c, const T* dm, long long n, unsigned int* bad) {
  unsigned int nb = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double cc = (double)c[i];
    const double m = 1.0 / (cc * cc) + (double)dm[i];
    if (!(m > 0.0) || !(m < 1e300)) ++nb;
  }
  if (nb) atomicAdd(bad, nb);
}

template <typename T>
__global__ void k_vel_update(T* c, const T* dm, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double cc = (double)c[i];
    const double m = 1.0 / (cc * cc) + (double)dm[i];
    c[i] = (T)(1.0 / sqrt(m));
  }
}

struct VecWS {
  DevBuf part;   // [VBLOCKS + 1] doubles: partial sums and the result
  DevBuf flag;
};

static VecWS* vws(mp_ctx* ctx) {
  if (!ctx->vec_ws) ctx->vec_ws = new VecWS();
  return static_cast<VecWS*>(ctx->vec_ws);
}

static dim3 vgrid(long long n) {
  long long b = (n + VB - 1) / VB;
  return dim3((unsigned)std::max<long long>(1, std::min<long long>(b, 16384)));
}

template <typename T>
static int dot_t(mp_ctx* ctx, long long n, const void* a, const void* b, double* out, hipStream_t s) {
  VecWS* ws = vws(ctx);
  int rc;
  if ((rc = ws->part.ensure(sizeof(double) * (VBLOCKS + 1), &ctx->budget, "dot partials"))) return rc;
  double* part = ws->part.as<double>();
  hipLaunchKernelGGL(k_dot_part<T>, dim3(VBLOCKS), dim3(VB), 0, s, static_cast<const T*>(a), static_cast<const T*>(b),
                     n, part);
  VC_LAUNCH();
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(VB), 0, s, part, part + VBLOCKS);
  VC_LAUNCH();
  VC_HIP(hipMemcpyAsync(out, part + VBLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
  VC_HIP(hipStreamSynchronize(s));
  return MP_OK;
}

int vec_dot(mp_ctx* ctx, long long n, const void* a, const void* b, double* out, hipStream_t s) {
  return ctx->cfg.dtype == MP_F32 ? dot_t<float>(ctx, n, a, b, out, s) : dot_t<double>(ctx, n, a, b, out, s);
}

int vec_axpby(mp_ctx* ctx, long long n, double alpha, const void* x, double beta, void* y, hipStream_t s) {
  if (ctx->cfg.dtype == MP_F32)
    hipLaunchKernelGGL(k_axpby<float>, vgrid(n), dim3(VB), 0, s, n, alpha, static_cast<const float*>(x), beta,
                       static_cast<float*>(y));
  else
    hipLaunchKernelGGL(k_axpby<double>, vgrid(n), dim3(VB), 0, s, n, alpha, static_cast<const double*>(x), beta,
                       static_cast<double*>(y));
  VC_LAUNCH();
  return MP_OK;
}

template <typename T>
static int vel_t(mp_ctx* ctx, void* c, const void* dm, hipStream_t s) {
  VecWS* ws = vws(ctx);
  const long long n = ctx->cfg.model_cells();
  int rc;
  if ((rc = ws->flag.ensure(sizeof(unsigned int), &ctx->budget, "velocity check"))) return rc;
  unsigned int* bad = ws->flag.as<unsigned int>();
  fill(reinterpret_cast<int*>(bad), 1, 0, s);
  hipLaunchKernelGGL(k_vel_check<T>, vgrid(n), dim3(VB), 0, s, static_cast<const T*>(c), static_cast<const T*>(dm), n,
                     bad);
  VC_LAUNCH();
  unsigned int h = 0;
  VC_HIP(hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s));
  VC_HIP(hipStreamSynchronize(s));
  if (h) {
    set_error("the step leaves c^-2 + dm non-positive or non-finite at " + std::to_string(h) + " cells");
    return MP_ENUMERIC;
  }
  hipLaunchKernelGGL(k_vel_update<T>, vgrid(n), dim3(VB), 0, s, static_cast<T*>(c), static_cast<const T*>(dm), n);
  VC_LAUNCH();
  return MP_OK;
}

int velocity_update(mp_ctx* ctx, void* c, const void* dm, hipStream_t s) {
  return ctx->cfg.dtype == MP_F32 ? vel_t<float>(ctx, c, dm, s) : vel_t<double>(ctx, c, dm, s);
}

// ---- the allocation-free dot product ----
// Its only device memory beyond the caller's buffers is the VBLOCKS partial sums, held
// in this file-scope array: one copy per GPU, kept until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in, not a device
// address): the address is resolved once per device with hipGetSymbolAddress, with that
// device current, and the kernels take the resolved pointer.
constexpr int SCRATCH_DOUBLES = VBLOCKS;   // 8 KiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[MAX_DEVICES] = {};

int vec_scratch_init() {
  int dev = 0;
  VC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("device index beyond the scratch table");
    return MP_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return MP_EDEVICE;
    }
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return MP_OK;
}

int vec_dot_noalloc(mp_ctx* ctx, long long n, const void* a, const void* b, double* out_dev, hipStream_t s) {
  static_assert(VBLOCKS <= SCRATCH_DOUBLES, "the partial sums of one call must fit the scratch");
  int dev = 0;
  VC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("device index beyond the scratch table");
    return MP_EUNSUPPORTED;
  }
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    part = g_scratch_ptr[dev];
  }
  if (!part) {   // a context created on another device: resolve this device's copy now
    int rc = vec_scratch_init();
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    part = g_scratch_ptr[dev];
  }
  // the same two kernels, grid and summation order as vec_dot: equal results, bit for bit
  if (ctx->cfg.dtype == MP_F32)
    hipLaunchKernelGGL(k_dot_part<float>, dim3(VBLOCKS), dim3(VB), 0, s, static_cast<const float*>(a),
                       static_cast<const float*>(b), n, part);
  else
    hipLaunchKernelGGL(k_dot_part<double>, dim3(VBLOCKS), dim3(VB), 0, s, static_cast<const double*>(a),
                       static_cast<const double*>(b), n, part);
  VC_LAUNCH();
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(VB), 0, s, part, out_dev);
  VC_LAUNCH();
  return MP_OK;
}

void vec_release(mp_ctx* ctx) {
  delete static_cast<VecWS*>(ctx->vec_ws);
  ctx->vec_ws = nullptr;
}

}  // namespace mp
