// Operator engine (2D and 3D): memory plan, shot waves, forward / reverse sweeps.
//
// Per shot the sweeps keep the field slices of the background u and of the
// Born / adjoint field (2D: input and output levels of launches that take two
// time steps; 3D: two levels stepped in place), the g = c^2 (L u + f) store on
// the model grid, and an FP64 image.  Shots that
// do not fit the budget together are processed in waves; images of every shot
// are kept and stacked in shot order at the end, so the result does not depend
// on how shots were grouped.  When all shots fit, the g store of the last
// background sweep is kept as the resident background and reused until the
// background changes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "prep.h"
#include "runtime.h"
#include "tables.h"
#include "wave.h"

namespace mp {

#define MP_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call); \
      return MP_EDEVICE;                                                    \
    }                                                                       \
  } while (0)

#define MP_CHECK_LAUNCH()                                                   \
  do {                                                                      \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess) {                                                 \
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_)); \
      return MP_EDEVICE;                                                    \
    }                                                                       \
  } while (0)

static long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

template <typename T>
class EngineT final : public Engine {
 public:
  EngineT(const Config& c, Budget* b) : cfg_(c), budget_(b) {
    L_.ndim = c.ndim;
    L_.nx = c.nx;
    L_.ny = c.ny;
    L_.nz = c.nz;
    L_.nb = c.nb;
    L_.nxp = c.nx + 2 * c.nb;
    L_.nyp = (c.ndim == 3) ? c.ny + 2 * c.nb : 1;
    L_.nzp = c.nz + 2 * c.nb;
    if (c.ndim == 2) {
      // strips of SW2 output cells; the row pitch covers every lane of every
      // strip (8 halo cells on either side), so the sweeps load rows unmasked
      L_.nstrips = (L_.nxp + SW2 - 1) / SW2;
      L_.pitch = (int)round_up(XL + (long long)L_.nstrips * SW2 + 8, 32);
      L_.nytiles = 1;
      L_.ypitch = 1;
    } else {
      L_.nstrips = (int)((L_.nxp + XL + 63) / 64);
      L_.pitch = L_.nstrips * 64;
      L_.nytiles = (L_.nyp + 15) / 16;
      L_.ypitch = L_.nytiles * 16 + 2 * GY;
    }
    L_.plane = (long long)L_.ypitch * L_.pitch;
    L_.fstride = round_up(2LL * SLACK + (long long)(L_.nzp + 2 * GZ) * L_.plane, 64);
    if (c.ndim == 2) {
      // model rows start so that every strip's first output cell lands on a
      // 64-byte boundary (128 bytes for even strips)
      L_.mxl = c.nb % 32;
      L_.mpitch = (int)round_up(L_.mxl + c.nx + 1, 32);
    } else {
      L_.mxl = 0;
      L_.mpitch = (int)round_up(c.nx, 4);
    }
    L_.mplane = (long long)L_.mpitch * c.ny;
    L_.mstride = L_.mplane * c.nz;
    cpitch_ = (int)round_up(L_.nxp, 4);
    cstride_ = (long long)cpitch_ * L_.nyp * L_.nzp;
    cu_count_ = device_cu_count();
    const char* zc = getenv("MP_ZC");
    zc_target_ = zc ? std::max(4, atoi(zc)) : 0;
  }

  int init() {
    const Config& c = cfg_;
    const int nd = c.ndim;
    // host tables
    std::vector<double> w = ricker(c.f_peak, c.t0, c.dt, c.nt);
    std::vector<T> wt(c.nt);
    const double hd = std::pow(c.h, nd);
    for (int n = 0; n < c.nt; ++n) wt[n] = (T)(w[n] / hd);
    std::vector<int> sx(c.ns), sy(c.ns, 0), sz(c.ns);
    for (int s = 0; s < c.ns; ++s) {
      sx[s] = c.src[(size_t)nd * s] + c.nb;
      if (nd == 3) sy[s] = c.src[(size_t)nd * s + 1] + c.nb;
      sz[s] = c.src[(size_t)nd * s + nd - 1] + c.nb;
    }
    // receiver maps: one [nyp][cpitch] map per z plane holding receivers
    std::vector<int> recplane(L_.nzp, -1);
    int nmaps = 0;
    for (int r = 0; r < c.nr; ++r) {
      const int z = c.rec[(size_t)nd * r + nd - 1] + c.nb;
      if (recplane[z] < 0) recplane[z] = nmaps++;
    }
    const long long msz = (long long)L_.nyp * cpitch_;
    std::vector<int> recmap((size_t)std::max(1, nmaps) * msz, -1);
    for (int r = 0; r < c.nr; ++r) {
      const int x = c.rec[(size_t)nd * r] + c.nb;
      const int y = (nd == 3) ? c.rec[(size_t)nd * r + 1] + c.nb : 0;
      const int z = c.rec[(size_t)nd * r + nd - 1] + c.nb;
      recmap[(size_t)recplane[z] * msz + (size_t)y * cpitch_ + x] = r;
    }
    hsx_ = sx;
    hsy_ = sy;
    hsz_ = sz;
    rec_lo_ = L_.nzp;
    rec_hi_ = -1;
    for (int z = 0; z < L_.nzp; ++z)
      if (recplane[z] >= 0) {
        rec_lo_ = std::min(rec_lo_, z);
        rec_hi_ = std::max(rec_hi_, z);
      }
    int rc;
    if ((rc = wav_.ensure(sizeof(T) * c.nt, budget_, "wavelet"))) return rc;
    if ((rc = recplane_.ensure(sizeof(int) * L_.nzp, budget_, "receivers"))) return rc;
    if ((rc = recmap_.ensure(sizeof(int) * recmap.size(), budget_, "receivers"))) return rc;
    if ((rc = kappa_.ensure(sizeof(T) * L_.fstride, budget_, "kappa"))) return rc;
    if ((rc = etax_.ensure(sizeof(T) * L_.nxp, budget_, "sponge"))) return rc;
    if ((rc = etay_.ensure(sizeof(T) * L_.nyp, budget_, "sponge"))) return rc;
    if ((rc = etaz_.ensure(sizeof(T) * L_.nzp, budget_, "sponge"))) return rc;
    if ((rc = small_.ensure(64, budget_, "scratch"))) return rc;
    MP_HIP(hipMemcpy(wav_.get(), wt.data(), sizeof(T) * c.nt, hipMemcpyHostToDevice));
    MP_HIP(hipMemcpy(recplane_.get(), recplane.data(), sizeof(int) * L_.nzp, hipMemcpyHostToDevice));
    MP_HIP(hipMemcpy(recmap_.get(), recmap.data(), sizeof(int) * recmap.size(), hipMemcpyHostToDevice));
    MP_HIP(hipMemset(kappa_.get(), 0, sizeof(T) * L_.fstride));
    MP_HIP(hipMemset(etay_.get(), 0, sizeof(T) * L_.nyp));
    MP_HIP(hipDeviceSynchronize());
    return MP_OK;
  }

  // ---- memory plan ----
  bool ckpt_mode() const { return cfg_.snap != MP_SNAP_FULL; }
  int ck_kind() const {
    return cfg_.snap == MP_SNAP_CKPT_BF16 ? CK_BF16 : cfg_.snap == MP_SNAP_CKPT_F32 ? CK_F32 : CK_NONE;
  }
  int nck() const { return ckpt_mode() ? (cfg_.nt + cfg_.ckpt_every - 1) / cfg_.ckpt_every : 0; }
  size_t ck_elem() const { return cfg_.snap == MP_SNAP_CKPT_BF16 ? 2 : sizeof(T); }
  // g slots per shot: every step (full history) or one checkpoint segment
  long long g_slots() const { return ckpt_mode() ? std::min(cfg_.ckpt_every, cfg_.nt) : cfg_.nt; }
  // field slices per shot: 2D keeps input and output levels of the background and
  // of the Born / adjoint field (4 + 4); 3D steps them in place (5)
  int nslices() const { return cfg_.ndim == 2 ? 8 : 5; }
  size_t per_shot_bytes() const {
    size_t b = sizeof(T) * (size_t)(nslices() * L_.fstride + g_slots() * L_.mstride);
    if (ckpt_mode()) b += (size_t)nck() * 2 * (ck_elem() * (size_t)cstride_ + sizeof(float));
    return b;
  }
  // Shots per image: the adjoint images the shots of a workgroup (four in 2D, a
  // pair in 3D) into one FP64 image, so jobs are laid out in such groups (each
  // request padded with null shots).
  int gsz() const { return cfg_.ndim == 2 ? GW2 : 2; }
  int pad_group(int n) const { return (n + gsz() - 1) / gsz() * gsz(); }
  // bytes that scale with the job (data, images, perturbation slots)
  size_t job_bytes(int nb, int nslots) const {
    return sizeof(T) * (size_t)nb * cfg_.nt * cfg_.nr + sizeof(double) * (size_t)(nb / gsz()) * L_.mstride +
           sizeof(T) * (size_t)nslots * L_.fstride + 4 * sizeof(int) * (size_t)nb;
  }
  int footprint(int op, int nshots, size_t* bytes) const override {
    (void)op;
    const int nb = pad_group(nshots > 0 ? nshots : cfg_.ns);
    const int w = std::max(1, std::min(nb, max_wave(SIZE_MAX, nb, 1)));
    *bytes = budget_->used - reserved_sweep() + job_bytes(nb, 1) + per_shot_bytes() * (size_t)w;
    return MP_OK;
  }
  size_t reserved_sweep() const {
    return fields_.bytes() + hist_.bytes() + data_.bytes() + img_.bytes() + ck_.bytes() + cks_.bytes() +
           dmbar_.bytes() + jtab_.bytes();
  }
  size_t reserved() const override { return budget_->used; }

  int max_wave(size_t limit, int nb, int nslots) const {
    const size_t base = budget_->used - reserved_sweep() + job_bytes(nb, nslots);
    if (limit <= base) return 0;
    const size_t w = (limit - base) / per_shot_bytes();
    return (int)std::min<size_t>(w, (size_t)nb);
  }

  // Buffers for a job of nb shots (a multiple of the group size) and nslots
  // perturbations.  Wave size: the fewest waves that fit, shots split evenly
  // between them in whole groups.
  int plan(int nb, int nslots, int* W) {
    const int g = gsz();
    const int wmax = max_wave(budget_->limit, nb, nslots) / g * g;
    if (wmax < g) {
      set_error("budget too small for one group of shots of the sweep");
      return MP_ENOMEM;
    }
    // MP_MAX_WAVE caps the shots per wave (a tuning knob)
    int cap = wmax;
    if (const char* mw = getenv("MP_MAX_WAVE")) cap = std::max(g, std::min(cap, atoi(mw) / g * g));
    const int ngr = nb / g, cgr = cap / g;
    const int nw = (ngr + cgr - 1) / cgr;
    const int w = (ngr + nw - 1) / nw * g;
    int rc;
    if ((rc = data_.ensure(sizeof(T) * (size_t)nb * cfg_.nt * cfg_.nr, budget_, "data"))) return rc;
    if ((rc = img_.ensure(sizeof(double) * (size_t)(nb / g) * L_.mstride, budget_, "images"))) return rc;
    if ((rc = dmbar_.ensure(sizeof(T) * (size_t)nslots * L_.fstride, budget_, "dm"))) return rc;
    if ((rc = jtab_.ensure(4 * sizeof(int) * (size_t)nb, budget_, "job tables"))) return rc;
    if ((rc = fields_.ensure(sizeof(T) * nslices() * (size_t)w * L_.fstride, budget_, "fields"))) return rc;
    if ((rc = hist_.ensure(sizeof(T) * (size_t)w * g_slots() * L_.mstride, budget_, "g store"))) return rc;
    if (ckpt_mode()) {
      if ((rc = ck_.ensure(ck_elem() * (size_t)w * nck() * 2 * cstride_, budget_, "checkpoints"))) return rc;
      if ((rc = cks_.ensure(sizeof(float) * (size_t)w * nck() * 2, budget_, "checkpoint scales"))) return rc;
    }
    *W = w;
    whole_ = (w >= nb);
    bgW_ = fW_ = w;
    hmod_ = 0;
    return MP_OK;
  }

  // Buffers of a shared-background batch: nbg background entries (one per shot
  // of the common shot list, padded to whole groups) and nj = nreq * nbg
  // wavefield entries, all in one wave.  Byte count only when dry.
  size_t shared_bytes(int nbg, int nj, int nslots) const {
    const size_t fslices = cfg_.ndim == 2 ? 4 * (size_t)nbg + 4 * (size_t)nj : 3 * (size_t)nbg + 2 * (size_t)nj;
    size_t b = sizeof(T) * (size_t)nj * cfg_.nt * cfg_.nr + sizeof(double) * (size_t)(nj / gsz()) * L_.mstride +
               sizeof(T) * (size_t)std::max(nslots, 1) * L_.fstride + 4 * sizeof(int) * (size_t)nj +
               sizeof(T) * fslices * L_.fstride + sizeof(T) * (size_t)nbg * g_slots() * L_.mstride;
    if (ckpt_mode()) b += (size_t)nbg * nck() * 2 * (ck_elem() * (size_t)cstride_ + sizeof(float));
    return b;
  }
  int plan_shared(int nbg, int nj, int nslots) {
    const size_t need = budget_->used - reserved_sweep() + shared_bytes(nbg, nj, nslots);
    if (need > budget_->limit) {
      set_error("shared-background batch needs " + std::to_string(need) + " bytes, budget " +
                std::to_string(budget_->limit) + ": submit fewer requests at once");
      return MP_ENOMEM;
    }
    const size_t fslices = cfg_.ndim == 2 ? 4 * (size_t)nbg + 4 * (size_t)nj : 3 * (size_t)nbg + 2 * (size_t)nj;
    int rc;
    if ((rc = data_.ensure(sizeof(T) * (size_t)nj * cfg_.nt * cfg_.nr, budget_, "data"))) return rc;
    if ((rc = img_.ensure(sizeof(double) * (size_t)(nj / gsz()) * L_.mstride, budget_, "images"))) return rc;
    if ((rc = dmbar_.ensure(sizeof(T) * (size_t)std::max(nslots, 1) * L_.fstride, budget_, "dm"))) return rc;
    if ((rc = jtab_.ensure(4 * sizeof(int) * (size_t)nj, budget_, "job tables"))) return rc;
    if ((rc = fields_.ensure(sizeof(T) * fslices * L_.fstride, budget_, "fields"))) return rc;
    if ((rc = hist_.ensure(sizeof(T) * (size_t)nbg * g_slots() * L_.mstride, budget_, "g store"))) return rc;
    if (ckpt_mode()) {
      if ((rc = ck_.ensure(ck_elem() * (size_t)nbg * nck() * 2 * cstride_, budget_, "checkpoints"))) return rc;
      if ((rc = cks_.ensure(sizeof(float) * (size_t)nbg * nck() * 2, budget_, "checkpoint scales"))) return rc;
    }
    bgW_ = nbg;
    fW_ = nj;
    hmod_ = nbg;
    whole_ = false;
    return MP_OK;
  }

  // Job tables: per job shot, the source cell (x, y, z) and the perturbation slot
  // (shot -1: a null shot that pads a group).
  // Staged through pinned host memory; the previous upload must have landed
  // before the staging buffer is rewritten.
  int upload_job(const std::vector<int>& shots, const std::vector<int>& slots) {
    const size_t nb = shots.size();
    if (jev_) MP_HIP(hipEventSynchronize(jev_));
    else MP_HIP(hipEventCreateWithFlags(&jev_, hipEventDisableTiming));
    if (jcap_ < 4 * nb) {
      if (jhost_) MP_HIP(hipHostFree(jhost_));
      jhost_ = nullptr;
      MP_HIP(hipHostMalloc((void**)&jhost_, sizeof(int) * 4 * nb, hipHostMallocDefault));
      jcap_ = 4 * nb;
    }
    for (size_t b = 0; b < nb; ++b) {
      const bool null = shots[b] < 0;   // padding of a group: no source, no data
      jhost_[b] = null ? -1 : hsx_[shots[b]];
      jhost_[nb + b] = null ? -1 : hsy_[shots[b]];
      jhost_[2 * nb + b] = null ? -1 : hsz_[shots[b]];
      jhost_[3 * nb + b] = slots[b];
    }
    MP_HIP(hipMemcpyAsync(jtab_.get(), jhost_, sizeof(int) * 4 * nb, hipMemcpyHostToDevice, stream_));
    MP_HIP(hipEventRecord(jev_, stream_));
    jn_ = (int)nb;
    return MP_OK;
  }

  Step<T> params(int s0, int nsh, int W) {
    Step<T> p;
    p.L = L_;
    p.rec_bg = nullptr;
    const double ih2 = 1.0 / (cfg_.h * cfg_.h);
    p.c0x = (T)(cfg_.ndim * FD8[0] * ih2);
    p.c1 = (T)(FD8[1] * ih2);
    p.c2 = (T)(FD8[2] * ih2);
    p.c3 = (T)(FD8[3] * ih2);
    p.c4 = (T)(FD8[4] * ih2);
    p.t3 = (T)(FD8[4] * ih2);
    p.t2 = (T)((FD8[3] + FD8[4]) * ih2);
    p.t1 = (T)((FD8[2] + FD8[3] + FD8[4]) * ih2);
    p.t0 = (T)((FD8[1] + FD8[2] + FD8[3] + FD8[4]) * ih2);
    p.hdt = (T)(0.5 * cfg_.dt);
    p.inv_dt2 = (T)(1.0 / (cfg_.dt * cfg_.dt));
    p.kappa = kappa_.as<T>();
    p.etax = etax_.as<T>();
    p.etay = etay_.as<T>();
    p.etaz = etaz_.as<T>();
    p.eta_c = (T)eta_c_;
    p.dmbar = dmbar_.as<T>();
    const int* jt = jtab_.as<int>();
    p.srcx = jt;
    p.srcy = jt + jn_;
    p.srcz = jt + 2 * jn_;
    p.dm_slot = jt + 3 * jn_;
    p.wav = wav_.as<T>();
    p.recplane = recplane_.as<int>();
    p.recmap = recmap_.as<int>();
    p.rec_lo = rec_lo_;
    p.rec_hi = rec_hi_;
    p.nr = cfg_.nr;
    p.nt = cfg_.nt;
    p.shot0 = s0;
    if (cfg_.ndim == 3) {
      // one item per 64 x 16 tile of a pair of shots and z chunk.  Workgroups are
      // resident one per CU and split over the 8 XCDs, each XCD walking its item
      // range in rounds of its CU count; the chunk count minimises rounds x (chunk
      // height + the 8 planes each chunk rereads), so a launch of few shots still
      // fills the last round without cutting z into many short chunks.
      int zc = zc_target_;
      const long long tiles = (long long)(nsh / 2) * L_.nstrips * L_.nytiles;
      if (zc <= 0) {
        const long long per_xcd = std::max(1LL, (long long)cu_count_ / 8);
        long long best = -1;
        for (int nch = 1; nch <= std::max(1, L_.nzp / 16); ++nch) {
          const long long h = (L_.nzp + nch - 1) / nch;
          const long long items = tiles * nch;
          const long long rounds = ((items + 7) / 8 + per_xcd - 1) / per_xcd;
          const long long cost = rounds * (h + 8);
          if (best < 0 || cost < best) {
            best = cost;
            zc = (int)h;
          }
        }
      }
      p.nchunks = (L_.nzp + zc - 1) / zc;
      p.zc = (L_.nzp + p.nchunks - 1) / p.nchunks;
      p.ngroups = 1;
      p.nwg = (int)(tiles * p.nchunks);
      p.nsh = nsh;
    }   // 2D: the launcher picks the z chunking per kernel
    (void)W;
    T* f = fields_.as<T>();
    const long long bs = (long long)bgW_ * L_.fstride, fs = (long long)fW_ * L_.fstride;
    p.u_cur = f;
    p.u_next = f + bs;
    p.u_inc = f + 2 * bs;
    p.du_cur = f + 3 * bs;
    p.du_prev = f + 3 * bs + fs;
    p.in0 = p.in1 = p.out0 = p.out1 = nullptr;
    p.hist = hist_.as<T>();
    p.data = data_.as<T>();
    p.img = img_.as<double>();
    p.hstride = g_slots() * L_.mstride;
    p.hist_u = 0;
    p.hmod = hmod_;
    p.ck = ck_.get();
    p.ck_scale = cks_.as<float>();
    p.cstride = cstride_;
    p.cpitch = cpitch_;
    p.nck = nck();
    return p;
  }

  void step(int mode, const Step<T>& p, int n, int hslot, int ck, int cs, int cm) {
    step3d(mode, p, n, hslot, ck, cs, cm, stream_);
  }

  // ---- background ----
  int set_background(const void* cdev, hipStream_t s) override {
    const T* c = static_cast<const T*>(cdev);
    unsigned int* st = small_.as<unsigned int>();
    cstats(c, cfg_.model_cells(), st, s);
    MP_CHECK_LAUNCH();
    unsigned int h[3];
    MP_HIP(hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    if (h[2] != 0) {
      set_error("background velocity has non-finite or non-positive entries");
      return MP_ENUMERIC;
    }
    double cmax;
    std::memcpy(&cmax, &h[0], 8);
    const double courant = cmax * cfg_.dt / cfg_.h;
    if (courant > cfl_limit(cfg_.ndim)) {
      set_error("CFL violated: c_max dt / h = " + std::to_string(courant) + " > " +
                std::to_string(cfl_limit(cfg_.ndim)));
      return MP_EINVAL;
    }
    std::vector<double> ex = sponge_profile(cfg_.nx, cfg_.nb, cmax, cfg_.h, cfg_.sponge_R);
    eta_c_ = cfg_.nb > 0 ? sponge_max(cfg_.nb, cmax, cfg_.h, cfg_.sponge_R) * 0.5 * cfg_.dt / ((double)cfg_.nb * cfg_.nb)
                         : 0.0;
    std::vector<double> ez = sponge_profile(cfg_.nz, cfg_.nb, cmax, cfg_.h, cfg_.sponge_R);
    std::vector<T> ext(ex.begin(), ex.end()), ezt(ez.begin(), ez.end());
    MP_HIP(hipMemcpyAsync(etax_.get(), ext.data(), sizeof(T) * ext.size(), hipMemcpyHostToDevice, s));
    MP_HIP(hipMemcpyAsync(etaz_.get(), ezt.data(), sizeof(T) * ezt.size(), hipMemcpyHostToDevice, s));
    std::vector<T> eyt(L_.nyp, T(0));
    if (cfg_.ndim == 3) {
      std::vector<double> ey = sponge_profile(cfg_.ny, cfg_.nb, cmax, cfg_.h, cfg_.sponge_R);
      for (int i = 0; i < L_.nyp; ++i) eyt[i] = (T)ey[i];
    }
    MP_HIP(hipMemcpyAsync(etay_.get(), eyt.data(), sizeof(T) * eyt.size(), hipMemcpyHostToDevice, s));
    Pad pd = pad();
    kappa(kappa_.as<T>(), c, pd, cfg_.dt, s);
    MP_CHECK_LAUNCH();
    MP_HIP(hipStreamSynchronize(s));   // host tables above must outlive the copies
    cached_ = false;
    return MP_OK;
  }

  // perturbation slot k <- E dm, ghost cells zero
  void put_dm(int k, const void* dm, hipStream_t s) {
    T* dst = dmbar_.as<T>() + (long long)k * L_.fstride;
    fill(dst, L_.fstride, T(0), s);
    extend(dst, static_cast<const T*>(dm), pad(), s);
  }

  Pad pad() const {
    Pad pd;
    pd.ndim = cfg_.ndim;
    pd.nx = cfg_.nx;
    pd.ny = cfg_.ny;
    pd.nz = cfg_.nz;
    pd.nb = cfg_.nb;
    pd.row = (cfg_.ndim == 3) ? L_.pitch : 0;
    pd.plane = L_.plane;
    pd.origin = SLACK + (long long)GZ * L_.plane + (cfg_.ndim == 3 ? (long long)GY * L_.pitch : 0) + XL;
    return pd;
  }

  // ---- sweeps ----
  int zero_fields(int W, bool both) {
    (void)both;
    (void)W;
    const long long slices = cfg_.ndim == 2 ? 4LL * bgW_ + 4LL * fW_ : 3LL * bgW_ + 2LL * fW_;
    fill(fields_.as<T>(), slices * L_.fstride, T(0), stream_);
    MP_CHECK_LAUNCH();
    return MP_OK;
  }

  // HIP events around sweeps (timing option): pairs recorded on the call's stream
  struct Span {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
    long long launches = 0;
    long long steps = 0;
  };
  std::vector<Span> spans_;
  size_t nspans_ = 0;

  int span_begin(int kind, long long launches, Span** out, long long steps = -1) {
    *out = nullptr;
    if (!cfg_.timing || nspans_ >= 16384) return MP_OK;   // bounded until the next collection
    if (nspans_ == spans_.size()) {
      Span sp;
      MP_HIP(hipEventCreate(&sp.a));
      MP_HIP(hipEventCreate(&sp.b));
      spans_.push_back(sp);
    }
    Span* sp = &spans_[nspans_++];
    sp->kind = kind;
    sp->launches = launches;
    sp->steps = steps < 0 ? launches : steps;
    MP_HIP(hipEventRecord(sp->a, stream_));
    *out = sp;
    return MP_OK;
  }
  int span_end(Span* sp) {
    if (sp) MP_HIP(hipEventRecord(sp->b, stream_));
    return MP_OK;
  }

  int collect_timing() override {
    for (int k = 0; k < 4; ++k) {
      stats.ms_sweep[k] = 0.0;
      stats.launches_sweep[k] = 0;
      stats.steps_sweep[k] = 0;
    }
    for (size_t i = 0; i < nspans_; ++i) {
      MP_HIP(hipEventSynchronize(spans_[i].b));
      float ms = 0.0f;
      MP_HIP(hipEventElapsedTime(&ms, spans_[i].a, spans_[i].b));
      stats.ms_sweep[spans_[i].kind] += ms;
      stats.launches_sweep[spans_[i].kind] += spans_[i].launches;
      stats.steps_sweep[spans_[i].kind] += spans_[i].steps;
    }
    nspans_ = 0;
    return MP_OK;
  }

  ~EngineT() override {
    for (auto& sp : spans_) {
      (void)hipEventDestroy(sp.a);
      (void)hipEventDestroy(sp.b);
    }
    if (jev_) {
      (void)hipEventSynchronize(jev_);
      (void)hipEventDestroy(jev_);
    }
    if (jhost_) (void)hipHostFree(jhost_);
  }

  // ---- 2D sweeps: up to two time steps per launch ----
  // Buffer roles rotate between launches: the background keeps (u, D) in and
  // out; the Born / adjoint field keeps (level 0, level -1) in and two output
  // levels.
  struct Rot2 {
    T* bg[4];   // u in, D in, u out, D out
    T* wf[4];   // level 0, level -1, level 1 out, level 2 out
  };
  Rot2 rot2(int W) {
    (void)W;
    T* f = fields_.as<T>();
    const long long bs = (long long)bgW_ * L_.fstride, fs = (long long)fW_ * L_.fstride;
    Rot2 r;
    for (int i = 0; i < 4; ++i) {
      r.bg[i] = f + i * bs;
      r.wf[i] = f + 4 * bs + i * fs;
    }
    return r;
  }
  void launch_bg(Step<T>& p, Rot2& r, int nsh, int ns, int ck, int n, int hs1, int hs2, int cs, int cm) {
    p.in0 = r.bg[0];
    p.in1 = r.bg[1];
    p.out0 = r.bg[2];
    p.out1 = r.bg[3];
    sweep2d(M_BG, ns, ck, p, nsh, n, hs1, hs2, cs, cm, zc_target_, stream_);
    std::swap(r.bg[0], r.bg[2]);
    std::swap(r.bg[1], r.bg[3]);
  }
  void launch_wf(int mode, Step<T>& p, Rot2& r, int nsh, int ns, int n, int hs1, int hs2) {
    p.in0 = r.wf[0];
    p.in1 = r.wf[1];
    p.out0 = r.wf[2];
    p.out1 = r.wf[3];
    sweep2d(mode, ns, CK_NONE, p, nsh, n, hs1, hs2, -1, -1, zc_target_, stream_);
    T* w[4] = {r.wf[0], r.wf[1], r.wf[2], r.wf[3]};
    if (ns == 2) {   // next: level 0 <- level 2, level -1 <- level 1
      r.wf[0] = w[3]; r.wf[1] = w[2]; r.wf[2] = w[0]; r.wf[3] = w[1];
    } else {         // next: level 0 <- level 1, level -1 <- level 0
      r.wf[0] = w[2]; r.wf[1] = w[0]; r.wf[2] = w[1]; r.wf[3] = w[3];
    }
  }

  // Forward sweep of shots [s0, s0+nsh) in segments (the checkpoint interval, or
  // all nt steps): the background over the segment (g into the segment's slots,
  // checkpoint of the segment's first level), then the Born field over it.
  // mode 0: background + Born, 1: Born from the stored g, 2: background only,
  // 3: background only with its receiver traces into data (no g, no checkpoints).
  int forward2d(int mode, int s0, int nsh, int W, T* data) {
    int rc;
    if (nsh % gsz() || s0 % gsz()) {
      set_error("internal: a 2D sweep takes whole groups of shots");
      return MP_EINVAL;
    }
    if ((rc = zero_fields(W, true))) return rc;
    const bool model = (mode == 3);
    Step<T> p = params(s0, nsh, W);
    p.data = model ? nullptr : data;
    p.rec_bg = model ? data : nullptr;
    Rot2 r = rot2(W);
    const int ck = model ? CK_NONE : ck_kind();
    const int nbg = hmod_ > 0 ? hmod_ : nsh;   // background entries of the sweep
    if (ck == CK_BF16 && mode != 1) {
      fill(cks_.as<float>(), (long long)nbg * nck() * 2, 0.0f, stream_);
      MP_CHECK_LAUNCH();
    }
    const int kk = (ckpt_mode() && !model) ? cfg_.ckpt_every : cfg_.nt;
    // g is only needed by a Born sweep or the cache
    const bool keep_g = !model && !(mode == 2 && ckpt_mode());
    for (int n0 = 0; n0 < cfg_.nt; n0 += kk) {
      const int len = std::min(kk, cfg_.nt - n0);
      const int j = n0 / kk;
      const int base = ckpt_mode() ? n0 : 0;   // g slot of step n is n - base
      Span* sp;
      if (mode != 1) {
        if ((rc = span_begin(MP_SWEEP_BACKGROUND, (len + 1) / 2, &sp, len))) return rc;
        for (int n = n0; n < n0 + len;) {
          const int ns = std::min(2, n0 + len - n);
          const int cs = (ck != CK_NONE && n == n0) ? j : -1;
          const int cm = (ck == CK_BF16 && n + ns == n0 + len && j + 1 < nck()) ? j + 1 : -1;
          const int hs1 = keep_g ? n - base : -1;
          const int hs2 = (keep_g && ns == 2) ? n + 1 - base : -1;
          launch_bg(p, r, nbg, ns, ck, n, hs1, hs2, cs, cm);
          n += ns;
        }
        if ((rc = span_end(sp))) return rc;
      }
      if (mode < 2) {
        if ((rc = span_begin(MP_SWEEP_BORN, (len + 1) / 2, &sp, len))) return rc;
        for (int n = n0; n < n0 + len;) {
          const int ns = std::min(2, n0 + len - n);
          launch_wf(M_BORN, p, r, nsh, ns, n, n - base, ns == 2 ? n + 1 - base : -1);
          n += ns;
        }
        if ((rc = span_end(sp))) return rc;
      }
    }
    MP_CHECK_LAUNCH();
    return MP_OK;
  }

  int adjoint2d(int s0, int nsh, int W, const T* data) {
    int rc;
    if (nsh % gsz() || s0 % gsz()) {
      set_error("internal: a 2D sweep takes whole groups of shots");
      return MP_EINVAL;
    }
    if ((rc = zero_fields(W, false))) return rc;
    fill(img_.as<double>() + (long long)(s0 / gsz()) * L_.mstride, (long long)(nsh / gsz()) * L_.mstride, 0.0,
         stream_);
    Step<T> p = params(s0, nsh, W);
    p.data = const_cast<T*>(data);
    Rot2 r = rot2(W);
    Span* sp;
    if (!ckpt_mode()) {
      if ((rc = span_begin(MP_SWEEP_ADJOINT, (cfg_.nt + 1) / 2, &sp, cfg_.nt))) return rc;
      for (int k = cfg_.nt; k >= 1;) {
        const int ns = k >= 2 ? 2 : 1;
        launch_wf(M_ADJ, p, r, nsh, ns, k, k - 1, ns == 2 ? k - 2 : -1);
        k -= ns;
      }
      MP_CHECK_LAUNCH();
      return span_end(sp);
    }
    // checkpoint modes: per segment (last first) recompute the background levels
    // u^{n0+1} .. u^{n0+len} from the checkpoint into the segment's slots, then run
    // the adjoint down through the segment, imaging in the summed-by-parts form
    // (the checkpoint's rounding then enters the image without the Laplacian)
    const int kk = cfg_.ckpt_every;
    const int ck = ck_kind();
    const int nbg = hmod_ > 0 ? hmod_ : nsh;
    p.hist_u = 1;
    for (int j = nck() - 1; j >= 0; --j) {
      const int n0 = j * kk;
      const int len = std::min(kk, cfg_.nt - n0);
      if ((rc = span_begin(MP_SWEEP_BACKGROUND, (len + 1) / 2, &sp, len))) return rc;
      // the segment's first launch reads (u^{n0}, D^{n0}) from checkpoint j itself
      const int ckl = ck == CK_BF16 ? CK_LBF16 : CK_LF32;
      for (int n = n0; n < n0 + len;) {
        const int ns = std::min(2, n0 + len - n);
        launch_bg(p, r, nbg, ns, n == n0 ? ckl : CK_NONE, n, n - n0, ns == 2 ? n + 1 - n0 : -1,
                  n == n0 ? j : -1, -1);
        n += ns;
      }
      if ((rc = span_end(sp))) return rc;
      if ((rc = span_begin(MP_SWEEP_ADJOINT, (len + 1) / 2, &sp, len))) return rc;
      for (int k = n0 + len; k >= n0 + 1;) {
        const int ns = (k - n0 >= 2) ? 2 : 1;
        launch_wf(M_ADJ, p, r, nsh, ns, k, k - 1 - n0, ns == 2 ? k - 2 - n0 : -1);
        k -= ns;
      }
      if ((rc = span_end(sp))) return rc;
    }
    MP_CHECK_LAUNCH();
    return MP_OK;
  }

  // forward sweep of shots [s0, s0+nsh): mode 0 fused, 1 Born from stored g, 2 background only,
  // 3 background only with its receiver traces into data (no g, no checkpoints).
  // In the checkpoint modes the background levels are stored every ckpt_every steps
  // instead of g.
  int forward(int mode, int s0, int nsh, int W, T* data) {
    if (cfg_.ndim == 2) return forward2d(mode, s0, nsh, W, data);
    int rc;
    if (nsh % gsz() || s0 % gsz()) {
      set_error("internal: a 3D sweep takes whole pairs of shots");
      return MP_EINVAL;
    }
    if ((rc = zero_fields(W, true))) return rc;
    const bool model = (mode == 3);
    Step<T> p = params(s0, nsh, W);
    p.data = model ? nullptr : data;
    p.rec_bg = model ? data : nullptr;
    const int ck = model ? CK_NONE : ck_kind();
    const bool shared = hmod_ > 0;
    const int nbg = shared ? hmod_ : nsh;
    if (ck == CK_BF16 && mode != 1) {
      fill(cks_.as<float>(), (long long)nbg * nck() * 2, 0.0f, stream_);
      MP_CHECK_LAUNCH();
    }
    Span* sp;
    if ((rc = span_begin(mode == 0 ? MP_SWEEP_FUSED : mode == 1 ? MP_SWEEP_BORN : MP_SWEEP_BACKGROUND,
                         cfg_.nt, &sp)))
      return rc;
    const int k = std::max(1, cfg_.ckpt_every);
    // shared background: its own launch over the background entries (g of the
    // step into a slot), then the Born field of every job entry from that slot
    Step<T> pb = shared ? params(s0, nbg, W) : p;
    for (int n = 0; n < cfg_.nt; ++n) {
      const int cs = (ck != CK_NONE && n % k == 0) ? n / k : -1;
      const int cm = (ck == CK_BF16 && (n + 1) % k == 0 && (n + 1) / k < nck()) ? (n + 1) / k : -1;
      if (shared) {
        // g^n: slot n with a full history; while checkpointing only a Born sweep reads it
        const int hs = (ck == CK_NONE) ? n : (mode == 0 ? n % k : -1);
        step(M_BG, pb, n, hs, ck, cs, cm);
        if (mode == 0) step(M_BORN, p, n, hs, CK_NONE, -1, -1);
        std::swap(pb.u_cur, pb.u_next);
        std::swap(p.du_cur, p.du_prev);
        continue;
      }
      // g is not stored while checkpointing, nor by modelling
      const int hs = model ? -1 : (ck == CK_NONE) ? n : -1;
      if (mode == 0) step(M_FUSED, p, n, hs, ck, cs, cm);
      else if (mode == 1) step(M_BORN, p, n, n, CK_NONE, -1, -1);
      else step(M_BG, p, n, hs, ck, cs, cm);
      std::swap(p.u_cur, p.u_next);
      std::swap(p.du_cur, p.du_prev);
    }
    MP_CHECK_LAUNCH();
    return span_end(sp);
  }

  // 3D reverse sweeps (background recomputation, adjoint): twice the forward z-chunk
  // count, unless a height is forced.  Shorter items keep the workgroups of a round
  // in step through the planes, so more of their halo rows meet in L2; the fused
  // forward sweep, with the most bytes per plane, loses more to the extra chunk
  // boundaries than it gains.
  void rechunk_reverse3d(Step<T>& p) const {
    if (zc_target_ > 0) return;
    const int nch = p.nchunks * 2;
    const int zc = (L_.nzp + nch - 1) / nch;
    if (zc < 32) return;
    p.nchunks = (L_.nzp + zc - 1) / zc;
    p.zc = (L_.nzp + p.nchunks - 1) / p.nchunks;
    p.nwg = (int)((long long)(p.nsh / 2) * L_.nstrips * L_.nytiles * p.nchunks);
  }

  int adjoint(int s0, int nsh, int W, const T* data) {
    if (cfg_.ndim == 2) return adjoint2d(s0, nsh, W, data);
    int rc;
    if (nsh % gsz() || s0 % gsz()) {
      set_error("internal: a 3D sweep takes whole pairs of shots");
      return MP_EINVAL;
    }
    if ((rc = zero_fields(W, false))) return rc;
    fill(img_.as<double>() + (long long)(s0 / gsz()) * L_.mstride, (long long)(nsh / gsz()) * L_.mstride, 0.0,
         stream_);
    Step<T> p = params(s0, nsh, W);
    rechunk_reverse3d(p);
    p.data = const_cast<T*>(data);
    Span* sp;
    if (!ckpt_mode()) {
      if ((rc = span_begin(MP_SWEEP_ADJOINT, cfg_.nt, &sp))) return rc;
      for (int k = cfg_.nt; k >= 1; --k) {
        step(M_ADJ, p, k, k - 1, CK_NONE, -1, -1);
        std::swap(p.du_cur, p.du_prev);
      }
      MP_CHECK_LAUNCH();
      return span_end(sp);
    }
    // checkpoint modes: per segment (last first) recompute the background levels
    // u^{n0+1} .. u^{n0+len} from the checkpoint into the segment's slots, then run
    // the adjoint down through the segment, imaging in the summed-by-parts form
    // (the checkpoint's rounding then enters the image without the Laplacian)
    const int kk = cfg_.ckpt_every;
    const int ck = ck_kind();
    const int nbg = hmod_ > 0 ? hmod_ : nsh;
    p.hist_u = 1;
    Step<T> pb = p;   // the background entries' launches
    if (hmod_ > 0) {
      pb = params(s0, nbg, W);
      rechunk_reverse3d(pb);
    }
    pb.hist_u = 1;
    for (int j = nck() - 1; j >= 0; --j) {
      const int n0 = j * kk;
      const int len = std::min(kk, cfg_.nt - n0);
      if ((rc = span_begin(MP_SWEEP_BACKGROUND, len, &sp))) return rc;
      // the segment's first step reads (u^{n0}, D^{n0}) from checkpoint j itself
      const int ckl = ck == CK_BF16 ? CK_LBF16 : CK_LF32;
      for (int n = n0; n < n0 + len; ++n) {
        step(M_BG, pb, n, n - n0, n == n0 ? ckl : CK_NONE, n == n0 ? j : -1, -1);
        std::swap(pb.u_cur, pb.u_next);
      }
      if ((rc = span_end(sp))) return rc;
      if ((rc = span_begin(MP_SWEEP_ADJOINT, len, &sp))) return rc;
      for (int k = n0 + len; k >= n0 + 1; --k) {
        step(M_ADJ, p, k, k - 1 - n0, CK_NONE, -1, -1);
        std::swap(p.du_cur, p.du_prev);
      }
      if ((rc = span_end(sp))) return rc;
    }
    MP_CHECK_LAUNCH();
    return MP_OK;
  }

  void finish_stats(int waves, bool used_cache, long long shots) {
    stats.cell_steps = (double)cfg_.prop_cells() * cfg_.nt * (double)shots;
    stats.waves = waves;
    stats.background_cached = used_cache ? 1 : 0;
    stats.bytes_reserved = budget_->used;
  }

  // the job of a plain call: every acquisition shot once, perturbation slot 0
  int plain_job(int* W) {
    int rc;
    const int nb = pad_group(cfg_.ns);
    if ((rc = plan(nb, 1, W))) return rc;
    std::vector<int> shots(nb, -1), slots(nb, 0);
    for (int i = 0; i < cfg_.ns; ++i) shots[i] = i;
    return upload_job(shots, slots);
  }

  int apply_F(const void* dm, void* d, hipStream_t s) override {
    stream_ = s;
    int W, rc;
    if ((rc = plain_job(&W))) return rc;
    put_dm(0, dm, s);
    MP_CHECK_LAUNCH();
    // with checkpoints the Born field still needs g at every step
    const bool use_cache = cached_ && whole_ && !ckpt_mode();
    const int nb = pad_group(cfg_.ns);
    int waves = 0;
    for (int s0 = 0; s0 < nb; s0 += W, ++waves) {
      const int nsh = std::min(W, nb - s0);
      if ((rc = forward(use_cache ? 1 : 0, s0, nsh, W, static_cast<T*>(d)))) return rc;
    }
    cached_ = whole_;
    finish_stats(waves, use_cache, cfg_.ns);
    return MP_OK;
  }

  // Nonlinear modelling: the background field of every acquisition shot at the
  // receivers, d[s][n][r] = u^{n+1}(x_r).  Writes no g and no checkpoints, so a
  // cached background history stays valid.
  int model(void* d, hipStream_t s) override {
    stream_ = s;
    int W, rc;
    if ((rc = plain_job(&W))) return rc;
    const int nb = pad_group(cfg_.ns);
    int waves = 0;
    for (int s0 = 0; s0 < nb; s0 += W, ++waves) {
      const int nsh = std::min(W, nb - s0);
      if ((rc = forward(3, s0, nsh, W, static_cast<T*>(d)))) return rc;
    }
    finish_stats(waves, false, cfg_.ns);
    return MP_OK;
  }

  int apply_Fadj(const void* d, void* img, hipStream_t s) override {
    stream_ = s;
    int W, rc;
    if ((rc = plain_job(&W))) return rc;
    const bool use_cache = cached_ && whole_;
    const int nb = pad_group(cfg_.ns);
    int waves = 0;
    for (int s0 = 0; s0 < nb; s0 += W, ++waves) {
      const int nsh = std::min(W, nb - s0);
      if (!use_cache)
        if ((rc = forward(2, s0, nsh, W, nullptr))) return rc;
      if ((rc = adjoint(s0, nsh, W, static_cast<const T*>(d)))) return rc;
    }
    cached_ = whole_;
    stack(static_cast<T*>(img), img_.as<double>() + L_.mxl, nb / gsz(), L_.mstride, cfg_.nx, cfg_.ny, cfg_.nz,
          L_.mpitch, cfg_.ny, s);
    MP_CHECK_LAUNCH();
    finish_stats(waves, use_cache, cfg_.ns);
    return MP_OK;
  }

  int apply_H(const void* dm, void* out, hipStream_t s) override {
    stream_ = s;
    int W, rc;
    if ((rc = plain_job(&W))) return rc;
    put_dm(0, dm, s);
    MP_CHECK_LAUNCH();
    const bool use_cache = cached_ && whole_ && !ckpt_mode();
    const int nb = pad_group(cfg_.ns);
    int waves = 0;
    T* data = data_.as<T>();
    for (int s0 = 0; s0 < nb; s0 += W, ++waves) {
      const int nsh = std::min(W, nb - s0);
      if ((rc = forward(use_cache ? 1 : 0, s0, nsh, W, data))) return rc;
      if ((rc = adjoint(s0, nsh, W, data))) return rc;
    }
    cached_ = whole_;
    stack(static_cast<T*>(out), img_.as<double>() + L_.mxl, nb / gsz(), L_.mstride, cfg_.nx, cfg_.ny, cfg_.nz,
          L_.mpitch, cfg_.ny, s);
    MP_CHECK_LAUNCH();
    finish_stats(waves, use_cache, cfg_.ns);
    return MP_OK;
  }

  // Several normal-operator applications in one sweep: request r applies
  // sum over its shots of F_s* F_s to dm[r].  The shots of all requests are
  // propagated together (one launch per time step); each request occupies
  // whole image groups (padded with null shots), and its image is stacked from
  // its own groups in order, so a request gives the same bits alone or in a mix.
  int apply_H_batch(int nreq, const int* counts, const int* shots, const void* const* dm, void* const* out,
                    hipStream_t s) override {
    stream_ = s;
    std::vector<int> js, jslot, first(nreq);
    int real = 0;
    for (int r = 0, k = 0; r < nreq; ++r) {
      first[r] = (int)js.size();
      for (int i = 0; i < counts[r]; ++i, ++k) {
        js.push_back(shots[k]);
        jslot.push_back(r);
      }
      while ((int)js.size() % gsz()) {
        js.push_back(-1);
        jslot.push_back(r);
      }
      real += counts[r];
    }
    const int nb = (int)js.size();
    int W, rc;
    if ((rc = plan(nb, nreq, &W))) return rc;
    if ((rc = upload_job(js, jslot))) return rc;
    for (int r = 0; r < nreq; ++r) {
      put_dm(r, dm[r], s);
      MP_CHECK_LAUNCH();
    }
    cached_ = false;     // the stores now hold this job's shots
    int waves = 0;
    T* data = data_.as<T>();
    for (int s0 = 0; s0 < nb; s0 += W, ++waves) {
      const int nsh = std::min(W, nb - s0);
      if ((rc = forward(0, s0, nsh, W, data))) return rc;
      if ((rc = adjoint(s0, nsh, W, data))) return rc;
    }
    for (int r = 0; r < nreq; ++r) {
      const int g0 = first[r] / gsz(), ng = pad_group(counts[r]) / gsz();
      stack(static_cast<T*>(out[r]), img_.as<double>() + L_.mxl + (long long)g0 * L_.mstride, ng, L_.mstride,
            cfg_.nx, cfg_.ny, cfg_.nz, L_.mpitch, cfg_.ny, s);
      MP_CHECK_LAUNCH();
    }
    finish_stats(waves, false, real);
    return MP_OK;
  }

  // Requests that share one shot list and one background: request r applies op
  // (F, F* or H) over those shots to in[r].  The background of each shot is
  // propagated (and recomputed from its checkpoints) once for all requests; the
  // Born and adjoint fields run per (request, shot) from the shared g / level
  // slots.  Every result is bit-identical to the same request submitted alone:
  // the background launches do not depend on the number of requests, the other
  // per-shot work is independent of it, and each request's image is stacked
  // from its own groups.
  int footprint_batch(int op, int nshots, int nreq, size_t* bytes) const override {
    const int nbg = pad_group(nshots);
    *bytes = budget_->used - reserved_sweep() + shared_bytes(nbg, nreq * nbg, op == MP_OP_FADJ ? 0 : nreq);
    return MP_OK;
  }

  int apply_batch(int op, int nreq, int nshots, const int* shots, const void* const* in, void* const* out,
                  hipStream_t s) override {
    stream_ = s;
    const int nbg = pad_group(nshots), nj = nreq * nbg;
    int rc;
    if ((rc = plan_shared(nbg, nj, op == MP_OP_FADJ ? 0 : nreq))) return rc;
    std::vector<int> js(nj), jslot(nj);
    for (int r = 0; r < nreq; ++r)
      for (int i = 0; i < nbg; ++i) {
        js[r * nbg + i] = i < nshots ? shots[i] : -1;
        jslot[r * nbg + i] = op == MP_OP_FADJ ? 0 : r;
      }
    if ((rc = upload_job(js, jslot))) return rc;
    cached_ = false;   // the stores now hold this job's shots
    T* data = data_.as<T>();
    const long long rec = (long long)cfg_.nt * cfg_.nr;   // samples per shot
    if (op == MP_OP_FADJ) {
      for (int r = 0; r < nreq; ++r)
        MP_HIP(hipMemcpyAsync(data + (long long)r * nbg * rec, in[r], sizeof(T) * (size_t)nshots * rec,
                              hipMemcpyDeviceToDevice, s));
    } else {
      for (int r = 0; r < nreq; ++r) {
        put_dm(r, in[r], s);
        MP_CHECK_LAUNCH();
      }
    }
    const int mode = op == MP_OP_FADJ ? 2 : 0;
    if ((rc = forward(mode, 0, nj, nj, data))) { hmod_ = 0; return rc; }
    if (op != MP_OP_F && (rc = adjoint(0, nj, nj, data))) { hmod_ = 0; return rc; }
    for (int r = 0; r < nreq; ++r) {
      if (op == MP_OP_F) {
        MP_HIP(hipMemcpyAsync(out[r], data + (long long)r * nbg * rec, sizeof(T) * (size_t)nshots * rec,
                              hipMemcpyDeviceToDevice, s));
      } else {
        const int g0 = r * nbg / gsz(), ng = nbg / gsz();
        stack(static_cast<T*>(out[r]), img_.as<double>() + L_.mxl + (long long)g0 * L_.mstride, ng, L_.mstride,
              cfg_.nx, cfg_.ny, cfg_.nz, L_.mpitch, cfg_.ny, s);
        MP_CHECK_LAUNCH();
      }
    }
    hmod_ = 0;
    bgW_ = fW_ = 0;
    finish_stats(1, false, (long long)nreq * nshots);
    return MP_OK;
  }

  int release_cache() override {
    cached_ = false;
    hist_.release();
    fields_.release();
    data_.release();
    img_.release();
    ck_.release();
    cks_.release();
    dmbar_.release();
    jtab_.release();
    return MP_OK;
  }

 private:
  Config cfg_;
  Budget* budget_;
  Layout L_;
  int zc_target_ = 0;
  // Field slices hold bgW_ background entries and fW_ wavefield entries; with
  // hmod_ > 0 (a shared-background batch) job entry j takes the background, the
  // g / level slots and the checkpoints of entry j % hmod_.
  int bgW_ = 0, fW_ = 0, hmod_ = 0;
  int cu_count_ = 256;
  int cpitch_ = 0;
  long long cstride_ = 0;
  bool cached_ = false;
  bool whole_ = false;
  hipStream_t stream_ = nullptr;
  DevBuf wav_, recplane_, recmap_, kappa_, dmbar_, jtab_, etax_, etay_, etaz_, small_;
  double eta_c_ = 0.0;   // 2D damping: eta_max dt / (2 nb^2)
  std::vector<int> hsx_, hsy_, hsz_;
  int rec_lo_ = 0, rec_hi_ = -1;
  int* jhost_ = nullptr;
  size_t jcap_ = 0;
  hipEvent_t jev_ = nullptr;
  int jn_ = 0;
  DevBuf fields_, hist_, data_, img_, ck_, cks_;
};

Engine* make_engine(const Config& c, Budget* b) {
  if (c.dtype == MP_F32) {
    auto* e = new EngineT<float>(c, b);
    if (e->init() != MP_OK) { delete e; return nullptr; }
    return e;
  }
  auto* e = new EngineT<double>(c, b);
  if (e->init() != MP_OK) { delete e; return nullptr; }
  return e;
}

}  // namespace mp
