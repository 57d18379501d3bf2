// Shared device-side definitions: field layout and lane-shuffle helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mp {

// Field layout on the propagation grid (2D slice per shot, 3D volume per shot):
//   element (x, z) of a 2D field lives at  base + SLACK + (z + GZ) * pitch + (x + XL)
// The GZ ghost rows above and below, the XL left columns and the columns past
// nxp are never written and stay zero, so a stencil may read a radius of 4
// cells around every propagation cell; the SLACK elements in front of and
// behind every slice cover the 4-column halo read of the first and last ghost
// rows.  (The 3D sweeps rely on this; the 2D sweeps skip reads outside the grid.)
constexpr int XL = 8;
constexpr int GZ = 4;
constexpr int GY = 4;            // ghost rows in y (3D)
constexpr int SLACK = 64;
constexpr int LANES = 64;        // wavefront size on gfx950
constexpr int HL2 = 4;           // 2D sweeps: halo lanes at each end of a strip
constexpr int SW2 = 2 * (LANES - 2 * HL2);   // 2D sweeps: output cells per strip (2 per lane)
constexpr int GW2 = 4;           // 2D sweeps: shots (wavefronts) per workgroup and per FP64 image

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T v[4];
};

// Lane shifts across the whole 64-lane wavefront (DPP wave_shr:1 / wave_shl:1).
// shr1: lane l receives lane l-1, lane 0 keeps `old`.
// shl1: lane l receives lane l+1, lane 63 keeps `old`.
// Both must be executed by all 64 lanes (uniform control flow).
__device__ __forceinline__ int dpp_shr1_i(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_shl1_i(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float shr1(float v, float old) {
  return __int_as_float(dpp_shr1_i(__float_as_int(v), __float_as_int(old)));
}
__device__ __forceinline__ float shl1(float v, float old) {
  return __int_as_float(dpp_shl1_i(__float_as_int(v), __float_as_int(old)));
}
__device__ __forceinline__ double shr1(double v, double old) {
  long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  int lo = dpp_shr1_i((int)(b & 0xffffffffll), (int)(o & 0xffffffffll));
  int hi = dpp_shr1_i((int)(b >> 32), (int)(o >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double shl1(double v, double old) {
  long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  int lo = dpp_shl1_i((int)(b & 0xffffffffll), (int)(o & 0xffffffffll));
  int hi = dpp_shl1_i((int)(b >> 32), (int)(o >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP shifts inside each 16-lane row: row_shr:1 / row_shl:1 (lane 0 / 15 of the
// row keeps `old`).
__device__ __forceinline__ float rshr1(float v, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x111, 0xF, 0xF, false));
}
__device__ __forceinline__ float rshl1(float v, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x101, 0xF, 0xF, false));
}
__device__ __forceinline__ double rshr1(double v, double old) {
  long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), 0x111, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), 0x111, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double rshl1(double v, double old) {
  long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), 0x101, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), 0x101, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// FP32 -> BF16 with round-to-nearest-even on the bit pattern (finite inputs).
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  const unsigned int b = __float_as_uint(f);
  return (unsigned short)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
// A BF16 code times its level's scale, rounded on its own: the pragma keeps the
// compiler from fusing the product into a later add (which it may do at some
// unrolled copies of a march body and not at others), so a decoded value does not
// depend on where it is decoded.
__device__ __forceinline__ float bf16_scaled(unsigned short h, float s) {
#pragma clang fp contract(off)
  return bf16_to_f(h) * s;
}

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

// Workgroup barrier for an LDS exchange: orders this wave's LDS accesses around
// the barrier without waiting for its global memory operations (a full
// __syncthreads would also drain the loads in flight).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Damping coefficients of the leapfrog at a cell: a = 1/(1 + eta dt/2), b = (1 - eta dt/2) a.
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

// Map a workgroup index to a work item so that each of the 8 XCDs (which
// receive workgroups round-robin) processes one contiguous range of the work
// list; neighbouring items then share that XCD's L2.
__device__ __forceinline__ int xcd_item(int nitems) {
  const int per = (nitems + 7) >> 3;
  return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}
inline int xcd_grid(int nitems) { return ((nitems + 7) / 8) * 8; }

// Compute units of the current device (256 on MI355X if the query fails).
inline int device_cu_count() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    return v;
  return 256;
}

}  // namespace mp
