// Probing fit and fitted-inverse application (FFT multipliers, FP64 Gram,
// Cholesky-QR) on the model grid.
#pragma once
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace mp {

int symbol_fit(mp_ctx* ctx, const Basis& b, int T, const void* const* y, const void* const* x, double* c,
               double* relres, hipStream_t s);
int symbol_apply(mp_ctx* ctx, const Basis& b, const double* c, const void* img, void* out, hipStream_t s);
void symbol_release(mp_ctx* ctx);
// In-place unnormalised FFT (inverse: conjugate twiddles) of one complex model-grid
// field, FP64 (f64) or FP32 interleaved pairs; power-of-two sizes.
int model_fft(mp_ctx* ctx, void* data, bool f64, int inverse, hipStream_t s);

}  // namespace mp
