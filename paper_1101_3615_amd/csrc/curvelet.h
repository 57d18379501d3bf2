// Curvelet frame, masked synthesis and the ray-traced illumination mask (2D model grid).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "runtime.h"

namespace mp {

struct Curvelets {
  int nscales;      // J >= 2
  int nangles;      // A_1: directions of band 1 over a half turn
  int mask_stride;  // mask nodes every stride cells
  int nfan;         // half-opening angles of the ray pairs
  int max_steps;    // Runge-Kutta steps (accepted or rejected) per ray
  double ray_rtol;  // position tolerance per step, in cells
};

int cv_directions(int j, int A1);
std::vector<int> cv_wedges(int J, int A1);   // [nw][3]: (j, l, A_j)
int curvelet_wedges(const Curvelets& cv, std::vector<int>& list);
int curvelet_norms(mp_ctx* ctx, const Curvelets& cv, std::vector<double>& norms, hipStream_t s);
int curvelet_synthesis(mp_ctx* ctx, const Curvelets& cv, const void* coef, const unsigned char* mask,
                       const double* weights, void* out, hipStream_t s);
int curvelet_analysis(mp_ctx* ctx, const Curvelets& cv, const void* img, void* coef, hipStream_t s);
int curvelet_illumination(mp_ctx* ctx, const Curvelets& cv, const void* c, unsigned char* mask, hipStream_t s);
int curvelet_sign_threshold(mp_ctx* ctx, const Curvelets& cv, void* coef, double t, hipStream_t s);
void curvelet_release(mp_ctx* ctx);

}  // namespace mp

struct mp_curvelets {
  mp::Curvelets cv;
};
