// Host/device parameter blocks and launchers of the wave-sweep kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mp {

// Propagation-grid field layout (one slice per shot):
//   cell (x, y, z) at  SLACK + (z + GZ) * plane + (y + gy) * pitch + (x + XL)
// with gy = GY in 3D and 0 in 2D (nyp = 1, ypitch = 1, plane = pitch).
struct Layout {
  int ndim;
  int nxp, nyp, nzp;   // propagation grid
  int pitch;           // x-row pitch in elements
  int ypitch;          // x rows per z plane, ghost rows included
  long long plane;     // elements per z plane (ypitch * pitch)
  long long fstride;   // elements per field slice of one shot
  int nx, ny, nz, nb;  // model grid and layer width
  int mpitch;          // model-grid x pitch (2D: multiple of 32; 3D: of 4)
  int mxl;             // 2D: lead elements before model column 0 of every model row (row alignment)
  long long mplane;    // model elements per z plane (mpitch * ny)
  long long mstride;   // model elements per slice (mplane * nz)
  int nstrips;         // 2D: 120-cell output strips per row; 3D: 64-cell x tiles
  int nytiles;         // 3D: 16-row y tiles (1 in 2D)
};

template <typename T>
struct Step {
  Layout L;
  T c0x, c1, c2, c3, c4;     // 8th-order weights / h^2; c0x = ndim * w0 / h^2
  T t0, t1, t2, t3;          // tail sums t_k = (c_{k+1} + ... + c_4) / h^2 (2D first-difference form)
  T hdt;                     // dt / 2
  T inv_dt2;                 // 1 / dt^2
  const T* kappa;            // field layout, shared by all shots
  const T* etax;             // [nxp]
  const T* etay;             // [nyp]
  const T* etaz;             // [nzp]
  T eta_c;                   // 2D: eta_max dt / (2 nb^2): damping e = eta_c (dx^2 + dz^2)
  const T* dmbar;            // [slot][field layout]: zero-extended model perturbations
  const int* dm_slot;        // [shots of the job] perturbation slot of each shot
  const int* srcx;           // [shots of the job] propagation-grid source cell
  const int* srcy;
  const int* srcz;
  const T* wav;              // [nt] wavelet / h^ndim
  const int* recplane;       // [nzp] receiver map of the plane, or -1
  const int* recmap;         // [maps][nyp][cpitch]: receiver index or -1
  int rec_lo, rec_hi;        // first and last z plane holding receivers (rec_lo > rec_hi: none)
  int nr, nt;
  int shot0;                 // job index of local shot 0 of this wave
  int zc, nchunks, ngroups, nwg;
  int nsh;                   // shots of the launch (3D: a multiple of 2)
  // 2D sweeps (one or two steps per launch): inputs and outputs of the launch
  T* in0;                    // background u^n / field level 0
  T* in1;                    // background increment D^n / field level -1
  T* out0;                   // background u^{n+NS} / field level 1
  T* out1;                   // background D^{n+NS} / field level 2
  // 3D sweeps (one step per launch)
  T* u_cur;                  // background level n (read)
  T* u_next;                 // background level n+1 (written)
  T* u_inc;                  // background increment u^n - u^{n-1}, updated in place
  T* du_cur;                 // Born / adjoint levels
  T* du_prev;
  T* hist;                   // g store: [local shot][slot][model]
  long long hstride;         // elements per local shot in hist
  int hmod;                  // > 0: local shot ls takes the slots of background entry ls % hmod
                             // (requests sharing one background sweep); 0: its own
  int hist_u;                // 1: slot n - n0 holds the background level u^{n+1} instead of g^n,
                             // and the adjoint images in the summed-by-parts form
                             // I -= u^k c^2 (L nu^{k+1} + R^T d^{k-1}) (checkpoint recomputation)
  T* data;                   // [shots of the job][nt][nr]
  T* rec_bg;                 // M_BG records u^{n+1}(x_r) into [shots of the job][nt][nr] when non-null
  double* img;               // [shots of the job][model] FP64 per-shot images
  // background checkpoints (checkpoint snapshot modes); compact layout
  // [z][y][cpitch] per level
  void* ck;                  // [local shot][nck][2][cstride]: (u^n, u^n - u^{n-1}) in FP32 or BF16
  float* ck_scale;           // [local shot][nck][2] max-abs scale of each BF16 level
  long long cstride;         // elements per checkpoint level (nzp * nyp * cpitch)
  int cpitch;                // compact row pitch (multiple of 4)
  int nck;                   // checkpoints per shot
};

// Checkpoint encodings of the background sweep: written by the launch (CK_F32,
// CK_BF16), or read as the launch's input levels (CK_LF32, CK_LBF16: the first
// recomputed launch of a segment, in place of a separate expansion pass).
enum { CK_NONE = 0, CK_F32 = 1, CK_BF16 = 2, CK_LF32 = 3, CK_LBF16 = 4 };
// Sweep kernels.
enum { M_FUSED = 0, M_BORN = 1, M_BG = 2, M_ADJ = 3 };

// 2D: nsteps (1 or 2) time steps of every shot of a wave in one launch.
// mode: M_BG, M_BORN or M_ADJ; n: first step (adjoint: k, the first level
// computed is nu^k); hs1, hs2: g slots of the two steps (written by M_BG, -1 for
// none; read by M_BORN and M_ADJ; u^{n+1} instead of g^n when p.hist_u); ck:
// CK_* encoding of M_BG; ck_store: the checkpoint written from the launch's input
// level (u^n, D^n) (CK_F32, CK_BF16) or read as that level (CK_LF32, CK_LBF16),
// or -1; ck_max: checkpoint whose BF16 scales take the maxima of the launch's
// last level or -1; zc > 0 forces the z-chunk height.  nsh: shots in the wave.
void sweep2d(int mode, int nsteps, int ck, const Step<float>& p, int nsh, int n, int hs1, int hs2, int ck_store,
             int ck_max, int zc, hipStream_t s);
void sweep2d(int mode, int nsteps, int ck, const Step<double>& p, int nsh, int n, int hs1, int hs2, int ck_store,
             int ck_max, int zc, hipStream_t s);
// 3D: one time step of every shot of a wave.  mode: M_*; n: step (adjoint: k);
// hslot: g slot written (background modes; -1: none) or read (Born, adjoint;
// u^{n+1} instead of g^n when p.hist_u); ck: CK_* encoding; ck_store: the
// checkpoint written from (u^n, u^{n-1}) at this step (CK_F32, CK_BF16) or read
// as that level (CK_LF32, CK_LBF16), or -1; ck_max: checkpoint whose BF16 scales
// accumulate max |u^{n+1}| and max |u^{n+1} - u^n| at this step or -1.
void step3d(int mode, const Step<float>& p, int n, int hslot, int ck, int ck_store, int ck_max, hipStream_t s);
void step3d(int mode, const Step<double>& p, int n, int hslot, int ck, int ck_store, int ck_max, hipStream_t s);

}  // namespace mp
