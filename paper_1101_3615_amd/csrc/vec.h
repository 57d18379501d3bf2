// Vector kernels of the solvers built on the operators.
#pragma once
#include <hip/hip_runtime.h>

#include "prep.h"
#include "runtime.h"

namespace mp {

// out (host) = sum_i a_i b_i, FP64 accumulation in a fixed order; synchronises the stream
int vec_dot(mp_ctx* ctx, long long n, const void* a, const void* b, double* out, hipStream_t s);
// y = alpha x + beta y, in FP64 rounded to the field precision
int vec_axpby(mp_ctx* ctx, long long n, double alpha, const void* x, double beta, void* y, hipStream_t s);
// c <- (c^-2 + dm)^(-1/2) on the model grid; MP_ENUMERIC (c untouched) if some c^-2 + dm <= 0
int velocity_update(mp_ctx* ctx, void* c, const void* dm, hipStream_t s);
// Resolve this device's copy of the allocation-free dot product's scratch (current device).
int vec_scratch_init();
// *out_dev (device) = sum_i a_i b_i as vec_dot, with the partial sums in the static
// scratch: no allocation, no synchronisation
int vec_dot_noalloc(mp_ctx* ctx, long long n, const void* a, const void* b, double* out_dev, hipStream_t s);
void vec_release(mp_ctx* ctx);

}  // namespace mp
