// 2D operator engine: memory plan, shot waves, forward / reverse sweeps.
//
// Per shot the sweeps keep four field slices (background u and Born / adjoint
// field, two time levels each; the leapfrog writes level n+1 over level n-1),
// the g = c^2 (L u + f) store on the model grid, and an FP64 image.  Shots that
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
class Engine2D final : public Engine {
 public:
  Engine2D(const Config& c, Budget* b) : cfg_(c), budget_(b) {
    L_.nx = c.nx;
    L_.nz = c.nz;
    L_.nb = c.nb;
    L_.nxp = c.nx + 2 * c.nb;
    L_.nzp = c.nz + 2 * c.nb;
    L_.nstrips = (int)((L_.nxp + XL + STRIP - 1) / STRIP);
    L_.pitch = L_.nstrips * STRIP;
    L_.fstride = round_up(2LL * SLACK + (long long)(L_.nzp + 2 * GZ) * L_.pitch, 64);
    L_.mpitch = (int)round_up(c.nx, 4);
    L_.mstride = (long long)L_.mpitch * c.nz;
    const char* zc = getenv("MP_ZC");
    zc_target_ = zc ? std::max(4, atoi(zc)) : 0;
  }

  int init() {
    const Config& c = cfg_;
    // host tables
    std::vector<double> w = ricker(c.f_peak, c.t0, c.dt, c.nt);
    std::vector<T> wt(c.nt);
    for (int n = 0; n < c.nt; ++n) wt[n] = (T)(w[n] / (c.h * c.h));
    std::vector<int> sx(c.ns), sz(c.ns);
    for (int s = 0; s < c.ns; ++s) {
      sx[s] = c.src[2 * s] + c.nb;
      sz[s] = c.src[2 * s + 1] + c.nb;
    }
    std::vector<int> recrow(L_.nzp, 0);
    std::vector<int> recmap((size_t)L_.fstride, -1);
    const long long o0 = SLACK + (long long)GZ * L_.pitch + XL;
    for (int r = 0; r < c.nr; ++r) {
      const int x = c.rec[2 * r] + c.nb, z = c.rec[2 * r + 1] + c.nb;
      recrow[z] = 1;
      recmap[o0 + (long long)z * L_.pitch + x] = r;
    }
    int rc;
    if ((rc = wav_.ensure(sizeof(T) * c.nt, budget_, "wavelet"))) return rc;
    if ((rc = srcx_.ensure(sizeof(int) * c.ns, budget_, "sources"))) return rc;
    if ((rc = srcz_.ensure(sizeof(int) * c.ns, budget_, "sources"))) return rc;
    if ((rc = recrow_.ensure(sizeof(int) * L_.nzp, budget_, "receivers"))) return rc;
    if ((rc = recmap_.ensure(sizeof(int) * L_.fstride, budget_, "receivers"))) return rc;
    if ((rc = kappa_.ensure(sizeof(T) * L_.fstride, budget_, "kappa"))) return rc;
    if ((rc = dmbar_.ensure(sizeof(T) * L_.fstride, budget_, "dm"))) return rc;
    if ((rc = etax_.ensure(sizeof(T) * L_.nxp, budget_, "sponge"))) return rc;
    if ((rc = etaz_.ensure(sizeof(T) * L_.nzp, budget_, "sponge"))) return rc;
    if ((rc = small_.ensure(64, budget_, "scratch"))) return rc;
    MP_HIP(hipMemcpy(wav_.get(), wt.data(), sizeof(T) * c.nt, hipMemcpyHostToDevice));
    MP_HIP(hipMemcpy(srcx_.get(), sx.data(), sizeof(int) * c.ns, hipMemcpyHostToDevice));
    MP_HIP(hipMemcpy(srcz_.get(), sz.data(), sizeof(int) * c.ns, hipMemcpyHostToDevice));
    MP_HIP(hipMemcpy(recrow_.get(), recrow.data(), sizeof(int) * L_.nzp, hipMemcpyHostToDevice));
    MP_HIP(hipMemcpy(recmap_.get(), recmap.data(), sizeof(int) * L_.fstride, hipMemcpyHostToDevice));
    MP_HIP(hipMemset(kappa_.get(), 0, sizeof(T) * L_.fstride));
    MP_HIP(hipMemset(dmbar_.get(), 0, sizeof(T) * L_.fstride));
    MP_HIP(hipDeviceSynchronize());
    return MP_OK;
  }

  // ---- memory plan ----
  size_t per_shot_bytes() const {
    return sizeof(T) * (size_t)(4 * L_.fstride + (long long)cfg_.nt * L_.mstride);
  }
  size_t fixed_bytes() const {
    return sizeof(T) * (size_t)cfg_.ns * cfg_.nt * cfg_.nr      // data (apply_H)
           + sizeof(double) * (size_t)cfg_.ns * L_.mstride;    // per-shot images
  }
  int footprint(int op, size_t* bytes) const override {
    (void)op;
    *bytes = budget_->used - reserved_sweep() + fixed_bytes() + per_shot_bytes() * (size_t)wave_size_for(budget_->limit);
    return MP_OK;
  }
  size_t reserved_sweep() const {
    return fields_.bytes() + hist_.bytes() + data_.bytes() + img_.bytes();
  }
  size_t reserved() const override { return budget_->used; }

  int wave_size_for(size_t limit) const {
    const size_t base = budget_->used - reserved_sweep() + fixed_bytes();
    if (limit <= base) return 0;
    const size_t w = (limit - base) / per_shot_bytes();
    return (int)std::min<size_t>(w, (size_t)cfg_.ns);
  }

  int plan(int* W) {
    const int w = wave_size_for(budget_->limit);
    if (w < 1) {
      set_error("budget too small for one shot of the sweep");
      return MP_ENOMEM;
    }
    int rc;
    if ((rc = data_.ensure(sizeof(T) * (size_t)cfg_.ns * cfg_.nt * cfg_.nr, budget_, "data"))) return rc;
    if ((rc = img_.ensure(sizeof(double) * (size_t)cfg_.ns * L_.mstride, budget_, "images"))) return rc;
    if ((rc = fields_.ensure(sizeof(T) * 4 * (size_t)w * L_.fstride, budget_, "fields"))) return rc;
    if ((rc = hist_.ensure(sizeof(T) * (size_t)w * cfg_.nt * L_.mstride, budget_, "history"))) return rc;
    *W = w;
    whole_ = (w >= cfg_.ns);
    return MP_OK;
  }

  Step2D<T> params(int s0, int nsh, int W) {
    Step2D<T> p;
    p.L = L_;
    const double ih2 = 1.0 / (cfg_.h * cfg_.h);
    p.c0x2 = (T)(2.0 * FD8[0] * ih2);
    p.c1 = (T)(FD8[1] * ih2);
    p.c2 = (T)(FD8[2] * ih2);
    p.c3 = (T)(FD8[3] * ih2);
    p.c4 = (T)(FD8[4] * ih2);
    p.hdt = (T)(0.5 * cfg_.dt);
    p.inv_dt2 = (T)(1.0 / (cfg_.dt * cfg_.dt));
    p.kappa = kappa_.as<T>();
    p.etax = etax_.as<T>();
    p.etaz = etaz_.as<T>();
    p.dmbar = dmbar_.as<T>();
    p.srcx = srcx_.as<int>();
    p.srcz = srcz_.as<int>();
    p.wav = wav_.as<T>();
    p.recrow = recrow_.as<int>();
    p.recmap = recmap_.as<int>();
    p.nr = cfg_.nr;
    p.nt = cfg_.nt;
    p.shot0 = s0;
    // z chunking: enough waves to fill the chip
    int zc = zc_target_;
    if (zc <= 0) {
      const long long waves_per_chunkrow = (long long)nsh * L_.nstrips;
      zc = (int)std::max<long long>(8, std::min<long long>(64, (long long)L_.nzp * waves_per_chunkrow / 4096));
    }
    const int ngroups = std::max(1, (int)((L_.nzp + 4LL * zc - 1) / (4LL * zc)));
    p.ngroups = ngroups;
    p.zc = (L_.nzp + 4 * ngroups - 1) / (4 * ngroups);
    p.nchunks = (L_.nzp + p.zc - 1) / p.zc;
    p.nwg = nsh * L_.nstrips * ngroups;
    T* f = fields_.as<T>();
    const long long fs = (long long)W * L_.fstride;
    p.u_cur = f;
    p.u_prev = f + fs;
    p.du_cur = f + 2 * fs;
    p.du_prev = f + 3 * fs;
    p.hist = hist_.as<T>();
    p.hstride = (long long)cfg_.nt * L_.mstride;
    p.data = data_.as<T>();
    p.img = img_.as<double>();
    return p;
  }

  // ---- background ----
  int set_background(const void* cdev, hipStream_t s) override {
    const T* c = static_cast<const T*>(cdev);
    unsigned int* st = small_.as<unsigned int>();
    cstats(c, cfg_.model_cells(), st, s);
    MP_CHECK_LAUNCH();
    unsigned int h[2];
    MP_HIP(hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    if (h[1] != 0) {
      set_error("background velocity has non-finite or non-positive entries");
      return MP_ENUMERIC;
    }
    float cmaxf;
    std::memcpy(&cmaxf, &h[0], 4);
    const double cmax = cmaxf;
    const double courant = cmax * cfg_.dt / cfg_.h;
    if (courant > cfl_limit(2)) {
      set_error("CFL violated: c_max dt / h = " + std::to_string(courant) + " > " +
                std::to_string(cfl_limit(2)));
      return MP_EINVAL;
    }
    std::vector<double> ex = sponge_profile(cfg_.nx, cfg_.nb, cmax, cfg_.h, cfg_.sponge_R);
    std::vector<double> ez = sponge_profile(cfg_.nz, cfg_.nb, cmax, cfg_.h, cfg_.sponge_R);
    std::vector<T> ext(ex.begin(), ex.end()), ezt(ez.begin(), ez.end());
    MP_HIP(hipMemcpyAsync(etax_.get(), ext.data(), sizeof(T) * ext.size(), hipMemcpyHostToDevice, s));
    MP_HIP(hipMemcpyAsync(etaz_.get(), ezt.data(), sizeof(T) * ezt.size(), hipMemcpyHostToDevice, s));
    Pad pd = pad();
    kappa(kappa_.as<T>(), c, pd, cfg_.dt, s);
    MP_CHECK_LAUNCH();
    MP_HIP(hipStreamSynchronize(s));
    cached_ = false;
    return MP_OK;
  }

  Pad pad() const {
    Pad pd;
    pd.ndim = 2;
    pd.nx = cfg_.nx;
    pd.ny = 1;
    pd.nz = cfg_.nz;
    pd.nb = cfg_.nb;
    pd.row = 0;
    pd.plane = L_.pitch;
    pd.origin = SLACK + (long long)GZ * L_.pitch + XL;
    return pd;
  }

  // ---- sweeps ----
  int zero_fields(int W, bool both) {
    (void)both;
    fill(fields_.as<T>(), 4LL * W * L_.fstride, T(0), stream_);
    MP_CHECK_LAUNCH();
    return MP_OK;
  }

  // HIP events around sweeps (timing option): pairs recorded on the call's stream
  struct Span {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
    long long launches = 0;
  };
  std::vector<Span> spans_;
  size_t nspans_ = 0;

  int span_begin(int kind, long long launches, Span** out) {
    *out = nullptr;
    if (!cfg_.timing || nspans_ >= 4096) return MP_OK;   // bounded until the next collection
    if (nspans_ == spans_.size()) {
      Span sp;
      MP_HIP(hipEventCreate(&sp.a));
      MP_HIP(hipEventCreate(&sp.b));
      spans_.push_back(sp);
    }
    Span* sp = &spans_[nspans_++];
    sp->kind = kind;
    sp->launches = launches;
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
    }
    for (size_t i = 0; i < nspans_; ++i) {
      MP_HIP(hipEventSynchronize(spans_[i].b));
      float ms = 0.0f;
      MP_HIP(hipEventElapsedTime(&ms, spans_[i].a, spans_[i].b));
      stats.ms_sweep[spans_[i].kind] += ms;
      stats.launches_sweep[spans_[i].kind] += spans_[i].launches;
    }
    nspans_ = 0;
    return MP_OK;
  }

  ~Engine2D() override {
    for (auto& sp : spans_) {
      (void)hipEventDestroy(sp.a);
      (void)hipEventDestroy(sp.b);
    }
  }

  // forward sweep of shots [s0, s0+nsh): mode 0 fused, 1 Born from stored g, 2 background only
  int forward(int mode, int s0, int nsh, int W, T* data) {
    int rc;
    if ((rc = zero_fields(W, true))) return rc;
    Step2D<T> p = params(s0, nsh, W);
    p.data = data;
    Span* sp;
    if ((rc = span_begin(mode == 0 ? MP_SWEEP_FUSED : mode == 1 ? MP_SWEEP_BORN : MP_SWEEP_BACKGROUND,
                         cfg_.nt, &sp)))
      return rc;
    for (int n = 0; n < cfg_.nt; ++n) {
      if (mode == 0) step2d_fused(p, n, n, stream_);
      else if (mode == 1) step2d_born(p, n, n, stream_);
      else step2d_bg(p, n, n, stream_);
      std::swap(p.u_cur, p.u_prev);
      std::swap(p.du_cur, p.du_prev);
    }
    MP_CHECK_LAUNCH();
    return span_end(sp);
  }

  int adjoint(int s0, int nsh, int W, const T* data) {
    int rc;
    if ((rc = zero_fields(W, false))) return rc;
    fill(img_.as<double>() + (long long)s0 * L_.mstride, (long long)nsh * L_.mstride, 0.0, stream_);
    Step2D<T> p = params(s0, nsh, W);
    p.data = const_cast<T*>(data);
    Span* sp;
    if ((rc = span_begin(MP_SWEEP_ADJOINT, cfg_.nt, &sp))) return rc;
    for (int k = cfg_.nt; k >= 1; --k) {
      step2d_adj(p, k, k - 1, stream_);
      std::swap(p.du_cur, p.du_prev);
    }
    MP_CHECK_LAUNCH();
    return span_end(sp);
  }

  void finish_stats(int waves, bool used_cache) {
    stats.cell_steps = (double)cfg_.prop_cells() * cfg_.nt * cfg_.ns;
    stats.waves = waves;
    stats.background_cached = used_cache ? 1 : 0;
    stats.bytes_reserved = budget_->used;
  }

  int apply_F(const void* dm, void* d, hipStream_t s) override {
    stream_ = s;
    int W, rc;
    if ((rc = plan(&W))) return rc;
    extend(dmbar_.as<T>(), static_cast<const T*>(dm), pad(), s);
    MP_CHECK_LAUNCH();
    const bool use_cache = cached_ && whole_;
    int waves = 0;
    for (int s0 = 0; s0 < cfg_.ns; s0 += W, ++waves) {
      const int nsh = std::min(W, cfg_.ns - s0);
      if ((rc = forward(use_cache ? 1 : 0, s0, nsh, W, static_cast<T*>(d)))) return rc;
    }
    cached_ = whole_;
    finish_stats(waves, use_cache);
    return MP_OK;
  }

  int apply_Fadj(const void* d, void* img, hipStream_t s) override {
    stream_ = s;
    int W, rc;
    if ((rc = plan(&W))) return rc;
    const bool use_cache = cached_ && whole_;
    int waves = 0;
    for (int s0 = 0; s0 < cfg_.ns; s0 += W, ++waves) {
      const int nsh = std::min(W, cfg_.ns - s0);
      if (!use_cache)
        if ((rc = forward(2, s0, nsh, W, nullptr))) return rc;
      if ((rc = adjoint(s0, nsh, W, static_cast<const T*>(d)))) return rc;
    }
    cached_ = whole_;
    stack(static_cast<T*>(img), img_.as<double>(), cfg_.ns, L_.mstride, cfg_.nx, 1, cfg_.nz, L_.mpitch, 1, s);
    MP_CHECK_LAUNCH();
    finish_stats(waves, use_cache);
    return MP_OK;
  }

  int apply_H(const void* dm, void* out, hipStream_t s) override {
    stream_ = s;
    int W, rc;
    if ((rc = plan(&W))) return rc;
    extend(dmbar_.as<T>(), static_cast<const T*>(dm), pad(), s);
    MP_CHECK_LAUNCH();
    const bool use_cache = cached_ && whole_;
    int waves = 0;
    T* data = data_.as<T>();
    for (int s0 = 0; s0 < cfg_.ns; s0 += W, ++waves) {
      const int nsh = std::min(W, cfg_.ns - s0);
      if ((rc = forward(use_cache ? 1 : 0, s0, nsh, W, data))) return rc;
      if ((rc = adjoint(s0, nsh, W, data))) return rc;
    }
    cached_ = whole_;
    stack(static_cast<T*>(out), img_.as<double>(), cfg_.ns, L_.mstride, cfg_.nx, 1, cfg_.nz, L_.mpitch, 1, s);
    MP_CHECK_LAUNCH();
    finish_stats(waves, use_cache);
    return MP_OK;
  }

  int release_cache() override {
    cached_ = false;
    hist_.release();
    fields_.release();
    data_.release();
    img_.release();
    return MP_OK;
  }

 private:
  Config cfg_;
  Budget* budget_;
  Layout2D L_;
  int zc_target_ = 0;
  bool cached_ = false;
  bool whole_ = false;
  hipStream_t stream_ = nullptr;
  DevBuf wav_, srcx_, srcz_, recrow_, recmap_, kappa_, dmbar_, etax_, etaz_, small_;
  DevBuf fields_, hist_, data_, img_;
};

Engine* make_engine_2d(const Config& c, Budget* b) {
  if (c.dtype == MP_F32) {
    auto* e = new Engine2D<float>(c, b);
    if (e->init() != MP_OK) { delete e; return nullptr; }
    return e;
  }
  auto* e = new Engine2D<double>(c, b);
  if (e->init() != MP_OK) { delete e; return nullptr; }
  return e;
}

}  // namespace mp
