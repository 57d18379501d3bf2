// Shared device-side definitions: field layout and lane-shuffle helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mp {

// Field layout on the propagation grid (2D slice per shot, 3D volume per shot):
//   element (x, z) of a 2D field lives at  base + SLACK + (z + GZ) * pitch + (x + XL)
// The GZ ghost rows above and below, the XL left columns and the columns past
// nxp are never written and stay zero, so the 8th-order stencil can read a
// radius of 4 cells around every propagation cell without bounds checks; the
// SLACK elements in front of and behind every slice cover the 4-column halo
// read of the first and last ghost rows.
constexpr int XL = 4;
constexpr int GZ = 4;
constexpr int SLACK = 64;
constexpr int LANES = 64;        // wavefront size on gfx950
constexpr int CPL = 4;           // cells per lane along x
constexpr int STRIP = LANES * CPL;

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

// Map a workgroup index to a work item so that each of the 8 XCDs (which
// receive workgroups round-robin) processes one contiguous range of the work
// list; neighbouring items then share that XCD's L2.
__device__ __forceinline__ int xcd_item(int nitems) {
  const int per = (nitems + 7) >> 3;
  return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}
inline int xcd_grid(int nitems) { return ((nitems + 7) / 8) * 8; }

}  // namespace mp
