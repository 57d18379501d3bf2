/*
 * matprobe: the normal operator of the acoustic wave equation and its probed
 * inverse, on one MI355X (gfx950).
 *
 * The operators follow the problem statement of Demanet et al., "Matrix
 * probing: a randomized preconditioner for the wave-equation Hessian":
 *   F      demigration, the Frechet derivative of the modelling map at the
 *          background m0 = 1/c^2 (Sec. 1.1; the linearised wave equation of
 *          Sec. 2);
 *   F*     migration, its adjoint, computed by reverse-time propagation
 *          (Sec. 1.1);
 *   H      the normal operator F*F (Sec. 1.1), stacked over shots (Sec. 2);
 *   fit    least-squares coefficients of H^-1 ~ sum_i c_i B_i from x_t = H y_t
 *          (Sec. 1.4, expansion H^-1 = sum c_i B_i of Sec. 1.2);
 *   Hinv   the fast application of the fitted series (end of Sec. 1.5).
 *
 * Discretisation (fixed by this library, identical in its CPU reference):
 *   - model grid nx x nz (x ny in 3D), spacing h; an absorbing layer of nb
 *     cells on every side gives the propagation grid;
 *   - 8th-order central Laplacian, zero outside the propagation grid;
 *   - damped leapfrog u+ = a (2u + kappa (L u + f)) - b u-, kappa = c^2 dt^2,
 *     a = 1/(1 + eta dt/2), b = (1 - eta dt/2) a, eta quadratic in the layer
 *     with eta_max = 3 c_max ln(1/R) / (2 nb h), zero in the model region;
 *   - point source w(t_n) / h^ndim at one cell, w a Ricker wavelet of peak
 *     frequency f_peak delayed by t0 (Sec. 2);
 *   - F is the exact derivative of this scheme with respect to m, F* its exact
 *     transpose; inner products are plain sums (Sec. 1.1).
 *
 * Layouts (all caller buffers are dense, C order, in the context's field
 * precision unless stated otherwise):
 *   model vector   [nz][ny][nx]   (ny = 1 in 2D), row iz = 0 is the surface
 *   data           [ns][nt][nr],  d[s][n][r] = du^{n+1}(receiver r)
 *   positions      int32 [count][ndim] model-grid indices (ix, [iy,] iz)
 *
 * Ownership: the caller owns every buffer passed in; pointers named *_dev
 * are device pointers, everything else is host memory.  The library owns the
 * context's internal device memory (wavefields, snapshot stores, images,
 * workspaces, the cached background), allocates it lazily within the budget
 * and frees it in mp_destroy.
 *
 * Ordering: calls are enqueued on the given HIP stream (a hipStream_t; NULL is
 * the default stream) and return before the device finishes, except
 * mp_set_background and mp_probe_fit, which synchronise that stream.  One
 * context must not be used from two host threads at once.
 *
 * Errors: every call returns MP_OK or a negative code; mp_last_error() gives a
 * message for the calling thread.  After MP_EDEVICE the context is poisoned and
 * every later call on it returns MP_EDEVICE.
 */
#ifndef MATPROBE_H
#define MATPROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MP_OK 0
#define MP_EINVAL (-1)       /* bad shape, index, pointer, option, or CFL violated */
#define MP_ENOMEM (-2)       /* budget or device memory exhausted; nothing launched */
#define MP_EDEVICE (-3)      /* HIP error; the context is poisoned */
#define MP_ESTATE (-4)       /* no background set */
#define MP_ENUMERIC (-5)     /* non-finite input/output or rank-deficient fit */
#define MP_EUNSUPPORTED (-6) /* valid request outside what the library implements */

#define MP_F32 1
#define MP_F64 2

#define MP_SNAP_FULL 0      /* keep every background time level */
#define MP_SNAP_CKPT_F32 1  /* two-level checkpoints in the field precision every k steps, recompute */
#define MP_SNAP_CKPT_BF16 2 /* BF16 checkpoints (level and increment) with FP32 scales */
/* In the checkpoint modes F* (and the adjoint half of H) images with the recomputed
 * background levels in the summed-by-parts form -sum_k u^k c^2 (L nu^{k+1} + R^T d^{k-1}),
 * equal in exact arithmetic to -sum_k g^{k-1} nu^k (Sec. 1.1, F* as the transpose of F),
 * so the checkpoint's rounding reaches the image without the Laplacian's amplification. */

#define MP_OP_F 1
#define MP_OP_FADJ 2
#define MP_OP_H 3
#define MP_OP_FIT 4
#define MP_OP_HINV 5

typedef struct mp_ctx mp_ctx;
typedef struct mp_basis mp_basis;

typedef struct mp_grid {
  int ndim;   /* 2 or 3 */
  int n[3];   /* model cells nx, ny, nz (ny = 1 in 2D) */
  double h;   /* grid spacing [m] */
  int nb;     /* absorbing cells on each side; a multiple of 4 */
} mp_grid;

typedef struct mp_acq {
  int ns;          /* shots */
  const int* src;  /* host int32 [ns][ndim]: source cell of each shot */
  int nr;          /* receivers, shared by every shot */
  const int* rec;  /* host int32 [nr][ndim]: receiver cells, pairwise distinct */
  double f_peak;   /* Ricker peak frequency [Hz] */
  double t0;       /* wavelet delay [s] */
  double dt;       /* time step [s] */
  int nt;          /* time steps */
} mp_acq;

typedef struct mp_opts {
  int dtype;           /* MP_F32 or MP_F64: field, data and model precision */
  int snap;            /* MP_SNAP_* */
  int ckpt_every;      /* k for the checkpoint modes (>= 1) */
  size_t budget_bytes; /* device-memory budget of the context; 0 = 90% of free memory */
  double sponge_R;     /* nominal reflection coefficient of the layer (0 < R < 1) */
  int timing;          /* 1: record HIP events around every sweep (read by mp_last_stats) */
} mp_opts;

#define MP_SWEEP_FUSED 0       /* forward: background and Born fields together (3D) */
#define MP_SWEEP_BORN 1        /* forward: Born field from the resident background */
#define MP_SWEEP_BACKGROUND 2  /* forward: background field only (store or recompute) */
#define MP_SWEEP_ADJOINT 3     /* reverse: adjoint field and imaging */

typedef struct mp_stats {
  double cell_steps;      /* propagation-grid cell-steps of the last operator call */
  int waves;              /* shot waves the last call was split into */
  int background_cached;  /* 1 if the last call reused the resident background */
  size_t bytes_reserved;  /* device memory the context holds */
  /* with mp_opts.timing: device time of the sweeps enqueued since the previous
   * mp_last_stats call, per sweep kind MP_SWEEP_*, from HIP events recorded on
   * the calls' streams around each sweep; kernel launches and time steps they
   * covered (2D sweeps take two steps per launch, 3D sweeps one) */
  double ms_sweep[4];
  long long launches_sweep[4];
  long long steps_sweep[4];
} mp_stats;

/* Create a context for one grid and acquisition.  Validates every index and
 * option; allocates only small tables.  *out receives the context.
 * MP_EINVAL also for grids whose padded wavefield slice or FP64 model-grid image
 * reaches 1 GiB (the sweeps address them with 32-bit buffer offsets). */
int mp_create(const mp_grid* g, const mp_acq* a, const mp_opts* o, mp_ctx** out);
void mp_destroy(mp_ctx* ctx);

/* Set the background velocity c [m/s] (device, model layout, field precision;
 * m0 = 1/c^2).  Checks the CFL bound c_max dt / h <= 2 / sqrt(ndim 2048/315)
 * (MP_EINVAL) and finiteness (MP_ENUMERIC), builds the damping profile and
 * drops any cached background wavefield.  Synchronises the stream. */
int mp_set_background(mp_ctx* ctx, const void* c_dev, void* stream);

/* Device bytes an operator needs with the current settings (MP_OP_*) for a
 * job of nshots shots (nshots <= 0: every acquisition shot), counting the
 * context's resident state; used for admission control.  Jobs are laid out in
 * image groups per request (four shots in 2D, two in 3D; padded), so for a batch
 * pass the sum of the requests' shot counts each rounded up to the group size. */
int mp_footprint(const mp_ctx* ctx, int op, int nshots, size_t* bytes);

/* F: model perturbation dm_dev -> data d_dev (overwritten), Sec. 1.1 / Sec. 2. */
int mp_apply_F(mp_ctx* ctx, const void* dm_dev, void* d_dev, void* stream);

/* Nonlinear modelling (Sec. 1.1, the map from m = 1/c^2 to data): d_dev
 * (overwritten; layout and precision of mp_apply_F's data, [ns][nt][nr]) gets
 * the background wavefield of every shot at the receivers, d[s][n][r] =
 * u_s^{n+1}(x_r), for the velocity given to mp_set_background (same scheme,
 * source, sponge and time axis as the background of F, whose Born field is the
 * derivative of this map with respect to m on the model grid, damping held
 * fixed).  Stores no background history, so a cached one stays valid.
 * MP_ESTATE without a background; MP_EINVAL for a null buffer. */
int mp_model(mp_ctx* ctx, void* d_dev, void* stream);

/* F*: data d_dev -> image img_dev (overwritten); the exact transpose of F. */
int mp_apply_Fadj(mp_ctx* ctx, const void* d_dev, void* img_dev, void* stream);

/* H = F*F: out_dev = F*(F dm_dev), fused (the data stay internal).  The
 * image is accumulated in FP64 and rounded once to the field precision. */
int mp_apply_H(mp_ctx* ctx, const void* dm_dev, void* out_dev, void* stream);

/* Batched normal operator for serving: request r applies
 * sum over s in its shot list of F_s* F_s to dm_dev[r] and writes out_dev[r].
 * counts: host int32 [nreq] shots per request; shots: host int32, the shot
 * lists of all requests concatenated (indices into the acquisition, repeats
 * allowed).  All shots of all requests are propagated together, one kernel
 * launch per time step; each result is bit-identical to the same request
 * submitted alone (per-shot work is independent and images are stacked per
 * request in the order given).  Overwrites the resident background store. */
int mp_apply_H_batch(mp_ctx* ctx, int nreq, const int* counts, const int* shots, const void* const* dm_dev,
                     void* const* out_dev, void* stream);

/* Batched F, F* or H for serving, for requests that share one shot list (the
 * operators of Sec. 1.1 restricted to those shots, Sec. 2): request r applies
 * op to in_dev[r] and writes out_dev[r].
 *   op MP_OP_F:    in = model perturbation (model layout), out = data
 *                  [nshots][nt][nr] in the order of shots;
 *   op MP_OP_FADJ: in = data [nshots][nt][nr], out = image (model layout);
 *   op MP_OP_H:    in = model perturbation, out = sum over the shots of F_s* F_s in.
 * shots: host int32 [nshots], acquisition indices (repeats allowed).  The
 * background of each shot is propagated, and recomputed from its checkpoints,
 * once for all nreq requests; their Born and adjoint fields run in the same
 * launches.  Each result is bit-identical to the same request submitted alone
 * (nreq = 1).  Device buffers are the caller's and must stay valid until the
 * stream reaches the call's end.  All requests run in one wave: MP_ENOMEM (with
 * the bytes needed in mp_last_error) if mp_footprint_batch exceeds the budget;
 * MP_EINVAL for a bad op, count, shot index or null buffer; MP_ESTATE without a
 * background.  Overwrites the resident background store. */
int mp_apply_batch(mp_ctx* ctx, int op, int nreq, int nshots, const int* shots, const void* const* in_dev,
                   void* const* out_dev, void* stream);

/* Device bytes of mp_apply_batch for nreq requests over nshots shots, counting
 * the context's resident state (admission control of a serving loop). */
int mp_footprint_batch(const mp_ctx* ctx, int op, int nshots, int nreq, size_t* bytes);

/* Drop the cached background wavefield and free the memory it holds. */
int mp_release_cache(mp_ctx* ctx);

/* Probing basis (Sec. 1.2, eq. (1); Sec. 1.4): element i = a * nq + q is
 * B_i v = P_a(x~) * Re IFFT(m_q(k) FFT v), a position factor P_a of the cell
 * centres x~ = -1 + (2i+1)/N times a Fourier multiplier m_q, periodic FFT on the
 * model grid, rho = |k| h / pi.  Two families:
 *  MP_BASIS_LEGENDRE_RHO (0): P_a = prod over axes of Legendre polynomials of
 *    degree degs[a][axis]; m_q = rho^qs[q].
 *    degs: host int32 [na][ndim] in axis order (x, [y,] z); qs: host int32 [nq].
 *  MP_BASIS_FOURIER_ANGULAR (1), the expansion of Sec. 1.2 (Fourier modes in x,
 *    angular harmonics of k, rational Chebyshev functions of |k|, times |k|^e):
 *    P_a = cos (phase 0) or sin (phase 1) of pi (m_x x~ + m_y y~ + m_z z~) with
 *    modes[a] = (m_x, m_y, m_z, phase) (m_y = 0 in 2D);
 *    m_q = A_{mults[q][0]}(k/|k|) * TL_{mults[q][1]}(rho) * rho^order with
 *    TL_n(r) = T_n((r - L)/(r + L)), L = tl_scale > 0; A_0 = 1 and, in 2D,
 *    A_{2j-1} = cos(j theta), A_{2j} = sin(j theta) (theta the angle of k from the
 *    x axis toward z, j <= 8), in 3D the real spherical harmonics of degree <= 2
 *    of n = k/|k| (1, n_x, n_y, n_z, n_x n_y, n_y n_z, 3 n_z^2 - 1, n_x n_z,
 *    n_x^2 - n_y^2); at k = 0, A_0 = 1, every other A and rho^order (order != 0)
 *    are 0.  modes: host int32 [na][4]; mults: host int32 [nq][2];
 *    |m| <= 64, TL degree <= 16, -2 <= order <= 2.
 * The descriptor is copied; the arrays may be freed after mp_basis_create. */
#define MP_BASIS_LEGENDRE_RHO 0
#define MP_BASIS_FOURIER_ANGULAR 1
typedef struct mp_basis_desc {
  int ndim;
  int na;
  const int* degs;    /* family 0 */
  int nq;
  const int* qs;      /* family 0 */
  int family;         /* MP_BASIS_* */
  const int* modes;   /* family 1 */
  const int* mults;   /* family 1 */
  int order;          /* family 1 */
  double tl_scale;    /* family 1 */
} mp_basis_desc;

int mp_basis_create(const mp_basis_desc* desc, mp_basis** out);
void mp_basis_destroy(mp_basis* b);

/* Least-squares fit of c (host, FP64, p = na * nq entries) minimising
 * sum_t || sum_i c_i B_i x_t - y_t ||^2 over T trials (Sec. 1.4).
 * y_dev[t], x_dev[t]: device model vectors in the field precision (x_t = H y_t).
 * The stacked system is solved on the device in FP64 by shifted
 * Cholesky-QR (three passes), its Gram products on the FP64 matrix cores.
 * *relres = ||A c - b|| / ||b||.  Model sizes must be powers of two
 * (MP_EUNSUPPORTED otherwise).  Returns MP_ENUMERIC when the system is
 * numerically rank deficient.  Synchronises the stream. */
int mp_probe_fit(mp_ctx* ctx, const mp_basis* basis, int T, const void* const* y_dev,
                 const void* const* x_dev, double* c, double* relres, void* stream);

/* out_dev = sum_i c_i B_i img_dev (c: host FP64 [p]); end of Sec. 1.5. */
int mp_apply_Hinv(mp_ctx* ctx, const mp_basis* basis, const double* c, const void* img_dev,
                  void* out_dev, void* stream);

/* ---- Vector kernels of the solvers built on the operators (steepest descent and
 * conjugate gradients on the normal equations, Sec. 1.1 and Sec. 2; Gauss-Newton,
 * Sec. 1.1).  Vectors are n contiguous elements in the context's precision (device);
 * n may be a model-grid or a data-space size; with n = 0 the pointers are not used. */

/* *out (host) = sum_i a_i b_i with FP64 products and accumulation in a fixed order
 * (results repeat bit for bit).  Synchronises the stream. */
int mp_vec_dot(mp_ctx* ctx, long long n, const void* a_dev, const void* b_dev, double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving or solver loops, harnesses that forbid hipMalloc): mp_vec_dot with the result
 * left on the device and nothing allocated.  *out_dev (device, one double) = sum_i a_i b_i,
 * computed by the same kernels in the same order as mp_vec_dot (equal bits).  The partial
 * sums live in a static 8 KiB device array, one per GPU, resolved at mp_create (or at the
 * first call on another device) and held until the process ends; the call allocates
 * nothing, does not synchronise and is stream-ordered.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (other streams, other threads) race: order
 * them on one stream.  n = 0 writes 0.  MP_EINVAL for n < 0, n > MP_NOALLOC_MAX_N or a null
 * pointer. */
#define MP_NOALLOC_MAX_N (1LL << 40)
int mp_vec_dot_noalloc(mp_ctx* ctx, long long n, const void* a_dev, const void* b_dev, double* out_dev,
                       void* stream);

/* y = alpha x + beta y, computed in FP64 and rounded to the field precision (x and y may
 * be the same buffer).  With beta = 0, y is overwritten and not read, so it may hold
 * anything (NaN included).  MP_ENUMERIC for a non-finite alpha or beta. */
int mp_vec_axpby(mp_ctx* ctx, long long n, double alpha, const void* x_dev, double beta, void* y_dev, void* stream);

/* The Gauss-Newton model update on the model grid: m = c^-2 + dm, c <- m^(-1/2) (c_dev
 * in place, dm_dev a step in m = 1/c^2).  MP_ENUMERIC, with c untouched, if m is not
 * positive and finite everywhere.  Synchronises the stream. */
int mp_velocity_update(mp_ctx* ctx, void* c_dev, const void* dm_dev, void* stream);

/* ---- Curvelet-space trial functions (Sec. 1.5; the mask's construction, Sec. 2) ----
 * 2D contexts with power-of-two model sizes up to 1024 per axis (MP_EUNSUPPORTED
 * otherwise).  The frame is undecimated and built in the frequency domain of the
 * periodic model grid: a lowpass wedge and nscales-1 directional bands; band j >= 1
 * has A_j = nangles * 2^floor((j-1)/2) directions over a half turn, centred at
 * theta = (l + 1/2) pi / A_j (the angle of the wavevector, x to z, z down).  The
 * wedge windows are smooth, even and square-sum to one, so analysis followed by
 * synthesis is the identity.  Coefficient arrays are [nwedges][nz][nx] in the
 * context's precision (device); masks [nwedges][nz][nx] bytes (device, 0 or 1). */
typedef struct mp_curvelet_desc {
  int nscales;      /* J in [2, 8]: the lowpass and J-1 directional bands */
  int nangles;      /* directions of band 1 over a half turn: even, in [4, 64] */
  int mask_stride;  /* the mask is evaluated at nodes every mask_stride cells, [1, 64] */
  int nfan;         /* half-opening angles alpha_i = (i + 1/2) pi / (2 nfan) of the ray pairs */
  int max_steps;    /* Runge-Kutta steps (accepted or rejected) per ray before it counts as a miss */
  double ray_rtol;  /* position error allowed per step, in cells, (0, 1] */
} mp_curvelet_desc;
typedef struct mp_curvelets mp_curvelets;

/* Validate a descriptor (MP_EINVAL) and create a host-side handle. */
int mp_curvelet_create(const mp_curvelet_desc* desc, mp_curvelets** out);
void mp_curvelet_destroy(mp_curvelets* cv);

/* Number of wedges; list (host, nullable) receives [nwedges][3] = (j, l, A_j),
 * the lowpass first as (0, 0, 0), then band by band. */
int mp_curvelet_wedges(const mp_curvelets* cv, int* nwedges, int* list);

/* ||phi_w||_2 of every wedge's atom (host FP64 [nwedges]). */
int mp_curvelet_norms(mp_ctx* ctx, const mp_curvelets* cv, double* norms, void* stream);

/* Illumination mask (Sec. 1.5: the set S of visible curvelet centres; Sec. 2: ray
 * tracing in smooth media).  c_dev: the velocity the rays see (model layout, field
 * precision).  At nodes every mask_stride cells and for each wedge direction, a fan of
 * ray pairs leaves along the upward normal turned by +alpha_i and -alpha_i; the centre
 * is visible if for some alpha_i one ray reaches the sources' row inside their span and
 * the other the receivers' row inside theirs (spans widened by half a cell).  Rays
 * solve the kinematic ray equations with Dormand-Prince 5(4) steps in FP64 through a
 * bilinear c and its centred-difference gradient; a ray that leaves the model's box
 * first, or exhausts max_steps, misses.  mask_dev (written) takes, for each cell, the
 * value of its node; the lowpass wedge is visible where a band-1 direction is.  Needs
 * the sources on one row and the receivers on one row (MP_EUNSUPPORTED otherwise).
 * Synchronises the stream. */
int mp_illumination(mp_ctx* ctx, const mp_curvelets* cv, const void* c_dev, unsigned char* mask_dev,
                    void* stream);

/* out_dev = sum_w IFFT(U_w FFT(weights[w] mask_w coef_w)): the curvelet synthesis of
 * the coefficients on the mask (mask_dev null: all ones; weights host FP64 [nwedges],
 * null: all ones).  A randomized trial function of Sec. 1.5 is coef ~ N(0, 1) i.i.d.
 * with weights sigma ||phi_w|| on the illumination mask. */
int mp_curvelet_synthesis(mp_ctx* ctx, const mp_curvelets* cv, const void* coef_dev, const unsigned char* mask_dev,
                          const double* weights, void* out_dev, void* stream);

/* In place on a coefficient array: c <- sign(c) where |c| >= threshold, 0 elsewhere (the
 * magnitudes set to one or to zero, the signs kept: the thresholded trial functions of
 * Sec. 2.4).  MP_EINVAL for a negative or non-finite threshold. */
int mp_curvelet_sign_threshold(mp_ctx* ctx, const mp_curvelets* cv, void* coef_dev, double threshold, void* stream);

/* coef_dev[w] = IFFT(U_w FFT img_dev): the curvelet coefficients of an image at every
 * grid position (the adjoint of the synthesis, and its inverse on the frame's range). */
int mp_curvelet_analysis(mp_ctx* ctx, const mp_curvelets* cv, const void* img_dev, void* coef_dev, void* stream);

/* Statistics of the last operator call; with timing enabled, waits for the
 * recorded events and restarts the timing accumulation. */
int mp_last_stats(const mp_ctx* ctx, mp_stats* out);
const char* mp_strerror(int code);
const char* mp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MATPROBE_H */
