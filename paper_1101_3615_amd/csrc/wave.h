// Host/device parameter blocks and launchers of the wave-sweep kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mp {

struct Layout2D {
  int nxp, nzp;        // propagation grid
  int pitch;           // field row pitch in elements (nstrips * 256)
  long long fstride;   // elements per field slice of one shot
  int nx, nz, nb;      // model grid and layer width
  int mpitch;          // model-grid row pitch (multiple of 4)
  long long mstride;   // model-grid elements per slice (mpitch * nz)
  int nstrips;         // 256-cell strips per row
};

template <typename T>
struct Step2D {
  Layout2D L;
  T c0x2, c1, c2, c3, c4;   // 8th-order weights / h^2 (centre weight doubled for 2 axes)
  T hdt;                     // dt / 2
  T inv_dt2;                 // 1 / dt^2
  const T* kappa;            // field layout, shared by all shots
  const T* etax;             // [nxp]
  const T* etaz;             // [nzp]
  const T* dmbar;            // field layout: zero-extended model perturbation
  const int* srcx;           // [ns] propagation-grid source cell
  const int* srcz;
  const T* wav;              // [nt] wavelet / h^2
  const int* recrow;         // [nzp] 1 if the row holds a receiver
  const int* recmap;         // field layout, receiver index or -1
  int nr, nt;
  int shot0;                 // global index of local shot 0 of this wave
  int zc, nchunks, ngroups, nwg;
  T* u_cur;                  // background levels n and n-1 (n-1 overwritten by n+1)
  T* u_prev;
  T* du_cur;                 // Born / adjoint levels
  T* du_prev;
  T* hist;                   // g store: [local shot][slot][model]
  long long hstride;         // elements per local shot in hist
  T* data;                   // [ns][nt][nr] (global shot index)
  double* img;               // [ns][model] FP64 per-shot images
};

void step2d_fused(const Step2D<float>& p, int n, int hslot, hipStream_t s);
void step2d_fused(const Step2D<double>& p, int n, int hslot, hipStream_t s);
void step2d_born(const Step2D<float>& p, int n, int hslot, hipStream_t s);
void step2d_born(const Step2D<double>& p, int n, int hslot, hipStream_t s);
void step2d_bg(const Step2D<float>& p, int n, int hslot, hipStream_t s);
void step2d_bg(const Step2D<double>& p, int n, int hslot, hipStream_t s);
void step2d_adj(const Step2D<float>& p, int k, int hslot, hipStream_t s);
void step2d_adj(const Step2D<double>& p, int k, int hslot, hipStream_t s);

}  // namespace mp
