// Launchers of the element-wise preparation kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mp {

// Geometry of a padded propagation-grid field: propagation cell (x, y, z) is at
// origin + z * plane + y * row + x.
struct Pad {
  int ndim;
  int nx, ny, nz, nb;   // model grid and layer width
  long long row;
  long long plane;
  long long origin;
};

void fill(float* p, long long n, float v, hipStream_t s);
void fill(double* p, long long n, double v, hipStream_t s);
void fill(int* p, long long n, int v, hipStream_t s);
void fill(unsigned short* p, long long n, unsigned short v, hipStream_t s);

void extend(float* dst, const float* model, const Pad& p, hipStream_t s);
void extend(double* dst, const double* model, const Pad& p, hipStream_t s);
void kappa(float* dst, const float* c, const Pad& p, double dt, hipStream_t s);
void kappa(double* dst, const double* c, const Pad& p, double dt, hipStream_t s);
// out[0..1] = bits of max c as a double (8-byte aligned), out[2] = count of non-finite /
// non-positive entries
void cstats(const float* c, long long n, unsigned int* out, hipStream_t s);
void cstats(const double* c, long long n, unsigned int* out, hipStream_t s);
// dense model out = sum over shots of FP64 images (model layout with pitch mpitch, myp y-rows)
void stack(float* out, const double* img, int nshots, long long mstride, int nx, int ny, int nz,
           int mpitch, int myp, hipStream_t s);
void stack(double* out, const double* img, int nshots, long long mstride, int nx, int ny, int nz,
           int mpitch, int myp, hipStream_t s);

}  // namespace mp
