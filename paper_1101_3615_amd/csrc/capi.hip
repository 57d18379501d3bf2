// The C ABI: argument validation, error state, context lifetime.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <string>
#include <utility>

#include "runtime.h"
#include "curvelet.h"
#include "symbol.h"
#include "vec.h"
#include "tables.h"

namespace mp {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int DevBuf::ensure(size_t bytes, Budget* budget, const char* what) {
  if (bytes <= n_ && p_) return MP_OK;
  release();
  if (bytes == 0) return MP_OK;
  if (budget && budget->used + bytes > budget->limit) {
    set_error(std::string("device-memory budget exceeded allocating ") + what + " (" +
              std::to_string(bytes) + " bytes, " + std::to_string(budget->used) + " of " +
              std::to_string(budget->limit) + " in use)");
    return MP_ENOMEM;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error(std::string("hipMalloc failed for ") + what + ": " + hipGetErrorString(e));
    return MP_ENOMEM;
  }
  p_ = p;
  n_ = bytes;
  b_ = budget;
  if (b_) b_->used += bytes;
  return MP_OK;
}

void DevBuf::release() {
  if (p_) {
    (void)hipFree(p_);
    if (b_) b_->used -= n_;
  }
  p_ = nullptr;
  n_ = 0;
  b_ = nullptr;
}

}  // namespace mp

using namespace mp;

static int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

static int guard(mp_ctx* ctx) {
  if (!ctx) return fail(MP_EINVAL, "null context");
  if (ctx->poisoned) return fail(MP_EDEVICE, "context poisoned by an earlier device error");
  return MP_OK;
}

static int finish(mp_ctx* ctx, int rc) {
  if (rc == MP_EDEVICE) ctx->poisoned = true;
  return rc;
}

extern "C" {

const char* mp_strerror(int code) {
  switch (code) {
    case MP_OK: return "ok";
    case MP_EINVAL: return "invalid argument";
    case MP_ENOMEM: return "out of device memory or budget";
    case MP_EDEVICE: return "device error";
    case MP_ESTATE: return "no background set";
    case MP_ENUMERIC: return "numerical failure";
    case MP_EUNSUPPORTED: return "unsupported";
    default: return "unknown error";
  }
}

const char* mp_last_error(void) { return g_err.c_str(); }

int mp_create(const mp_grid* g, const mp_acq* a, const mp_opts* o, mp_ctx** out) {
  if (!g || !a || !o || !out) return fail(MP_EINVAL, "null argument");
  *out = nullptr;
  if (g->ndim != 2 && g->ndim != 3) return fail(MP_EINVAL, "ndim must be 2 or 3");
  const int nd = g->ndim;
  const int nx = g->n[0], ny = (nd == 3) ? g->n[1] : 1, nz = g->n[2];
  if (nd == 2 && g->n[1] != 1) return fail(MP_EINVAL, "2D grids need n[1] == 1");
  if (nx < 1 || ny < 1 || nz < 1) return fail(MP_EINVAL, "grid sizes must be positive");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(MP_EINVAL, "h must be positive");
  if (g->nb < 0 || g->nb % 4 != 0) return fail(MP_EINVAL, "nb must be a non-negative multiple of 4");
  if (a->ns < 1 || !a->src) return fail(MP_EINVAL, "need at least one source");
  if (a->nr < 1 || !a->rec) return fail(MP_EINVAL, "need at least one receiver");
  if (a->nt < 1) return fail(MP_EINVAL, "nt must be positive");
  if (!(a->dt > 0.0) || !(a->f_peak > 0.0) || !std::isfinite(a->t0))
    return fail(MP_EINVAL, "dt and f_peak must be positive, t0 finite");
  if (o->dtype != MP_F32 && o->dtype != MP_F64) return fail(MP_EINVAL, "dtype must be MP_F32 or MP_F64");
  if (o->snap != MP_SNAP_FULL && o->snap != MP_SNAP_CKPT_F32 && o->snap != MP_SNAP_CKPT_BF16)
    return fail(MP_EINVAL, "unknown snapshot mode");
  if (o->snap != MP_SNAP_FULL && o->ckpt_every < 1) return fail(MP_EINVAL, "ckpt_every must be >= 1");
  if (!(o->sponge_R > 0.0 && o->sponge_R < 1.0)) return fail(MP_EINVAL, "sponge_R must be in (0, 1)");
  auto inside = [&](const int* p) {
    if (p[0] < 0 || p[0] >= nx) return false;
    if (nd == 3 && (p[1] < 0 || p[1] >= ny)) return false;
    const int z = p[nd - 1];
    return z >= 0 && z < nz;
  };
  for (int s = 0; s < a->ns; ++s)
    if (!inside(a->src + (size_t)s * nd)) return fail(MP_EINVAL, "source " + std::to_string(s) + " outside the model grid");
  std::set<std::vector<int>> seen;
  for (int r = 0; r < a->nr; ++r) {
    const int* p = a->rec + (size_t)r * nd;
    if (!inside(p)) return fail(MP_EINVAL, "receiver " + std::to_string(r) + " outside the model grid");
    if (!seen.insert(std::vector<int>(p, p + nd)).second)
      return fail(MP_EINVAL, "receivers must occupy distinct cells");
  }
  if (o->snap == MP_SNAP_CKPT_BF16 && o->dtype != MP_F32)
    return fail(MP_EUNSUPPORTED, "BF16 checkpoints are built for FP32 fields");
  {
    // The sweeps address one field slice and one model-grid image with 32-bit
    // buffer offsets whose out-of-grid values must stay past the end of the
    // buffer: both stay below 1 GiB.
    const long long esz = o->dtype == MP_F32 ? 4 : 8;
    const long long nxp = nx + 2LL * g->nb, nyp = ny + 2LL * g->nb, nzp = nz + 2LL * g->nb;
    long long field;
    if (nd == 2) field = (nxp + 176) * (nzp + 8) + 128;
    else field = ((nxp + 8 + 63) / 64 * 64) * ((nyp + 15) / 16 * 16 + 8) * (nzp + 8) + 128;
    const long long image = ((long long)nx + 40) * ny * (nz + (long long)g->nb) * 8;
    if (field * esz >= (1LL << 30) || image >= (1LL << 30))
      return fail(MP_EINVAL, "grid too large: one wavefield slice and the FP64 image must each stay below 1 GiB");
  }

  mp_ctx* ctx = new mp_ctx();
  Config& c = ctx->cfg;
  c.ndim = nd;
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.nb = g->nb;
  c.h = g->h;
  c.ns = a->ns;
  c.nr = a->nr;
  c.src.assign(a->src, a->src + (size_t)a->ns * nd);
  c.rec.assign(a->rec, a->rec + (size_t)a->nr * nd);
  c.f_peak = a->f_peak;
  c.t0 = a->t0;
  c.dt = a->dt;
  c.nt = a->nt;
  c.dtype = o->dtype;
  c.snap = o->snap;
  c.ckpt_every = o->ckpt_every;
  c.sponge_R = o->sponge_R;
  c.timing = o->timing ? 1 : 0;
  size_t freeb = 0, total = 0;
  hipError_t e = hipMemGetInfo(&freeb, &total);
  if (e != hipSuccess) {
    delete ctx;
    return fail(MP_EDEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
  }
  const size_t cap = (size_t)(0.9 * (double)freeb);
  ctx->budget.limit = (o->budget_bytes == 0) ? cap : std::min(o->budget_bytes, cap);
  ctx->eng = make_engine(c, &ctx->budget);
  if (!ctx->eng) {
    delete ctx;
    return MP_ENOMEM;
  }
  const int src = vec_scratch_init();   // the allocation-free entry point's scratch, this device
  if (src) {
    delete ctx->eng;
    delete ctx;
    return src;
  }
  *out = ctx;
  return MP_OK;
}

void mp_destroy(mp_ctx* ctx) {
  if (!ctx) return;
  symbol_release(ctx);
  curvelet_release(ctx);
  vec_release(ctx);
  delete ctx->eng;
  delete ctx;
}

int mp_set_background(mp_ctx* ctx, const void* c_dev, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!c_dev) return fail(MP_EINVAL, "null velocity");
  rc = ctx->eng->set_background(c_dev, (hipStream_t)stream);
  if (rc == MP_OK) ctx->has_bg = true;
  return finish(ctx, rc);
}

int mp_footprint(const mp_ctx* ctx, int op, int nshots, size_t* bytes) {
  if (!ctx || !bytes) return fail(MP_EINVAL, "null argument");
  if (op < MP_OP_F || op > MP_OP_HINV) return fail(MP_EINVAL, "unknown op");
  return ctx->eng->footprint(op, nshots, bytes);
}

int mp_apply_H_batch(mp_ctx* ctx, int nreq, const int* counts, const int* shots, const void* const* dm,
                     void* const* out, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (nreq < 1 || !counts || !shots || !dm || !out) return fail(MP_EINVAL, "bad batch arguments");
  if (!ctx->has_bg) return fail(MP_ESTATE, "no background set");
  long long k = 0;
  for (int r = 0; r < nreq; ++r) {
    if (counts[r] < 1) return fail(MP_EINVAL, "every request needs at least one shot");
    if (!dm[r] || !out[r]) return fail(MP_EINVAL, "null request buffer");
    for (int i = 0; i < counts[r]; ++i, ++k)
      if (shots[k] < 0 || shots[k] >= ctx->cfg.ns) return fail(MP_EINVAL, "shot index out of range");
  }
  return finish(ctx, ctx->eng->apply_H_batch(nreq, counts, shots, dm, out, (hipStream_t)stream));
}

int mp_footprint_batch(const mp_ctx* ctx, int op, int nshots, int nreq, size_t* bytes) {
  if (!ctx || !bytes) return fail(MP_EINVAL, "null argument");
  if (op != MP_OP_F && op != MP_OP_FADJ && op != MP_OP_H) return fail(MP_EINVAL, "op must be F, Fadj or H");
  if (nshots < 1 || nreq < 1) return fail(MP_EINVAL, "nshots and nreq must be positive");
  return ctx->eng->footprint_batch(op, nshots, nreq, bytes);
}

int mp_apply_batch(mp_ctx* ctx, int op, int nreq, int nshots, const int* shots, const void* const* in,
                   void* const* out, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (op != MP_OP_F && op != MP_OP_FADJ && op != MP_OP_H) return fail(MP_EINVAL, "op must be F, Fadj or H");
  if (nreq < 1 || nshots < 1 || !shots || !in || !out) return fail(MP_EINVAL, "bad batch arguments");
  if (!ctx->has_bg) return fail(MP_ESTATE, "no background set");
  for (int i = 0; i < nshots; ++i)
    if (shots[i] < 0 || shots[i] >= ctx->cfg.ns) return fail(MP_EINVAL, "shot index out of range");
  for (int r = 0; r < nreq; ++r)
    if (!in[r] || !out[r]) return fail(MP_EINVAL, "null request buffer");
  return finish(ctx, ctx->eng->apply_batch(op, nreq, nshots, shots, in, out, (hipStream_t)stream));
}

int mp_apply_F(mp_ctx* ctx, const void* dm, void* d, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!dm || !d) return fail(MP_EINVAL, "null buffer");
  if (!ctx->has_bg) return fail(MP_ESTATE, "no background set");
  return finish(ctx, ctx->eng->apply_F(dm, d, (hipStream_t)stream));
}

int mp_model(mp_ctx* ctx, void* d, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!d) return fail(MP_EINVAL, "null buffer");
  if (!ctx->has_bg) return fail(MP_ESTATE, "no background set");
  return finish(ctx, ctx->eng->model(d, (hipStream_t)stream));
}

int mp_apply_Fadj(mp_ctx* ctx, const void* d, void* img, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!d || !img) return fail(MP_EINVAL, "null buffer");
  if (!ctx->has_bg) return fail(MP_ESTATE, "no background set");
  return finish(ctx, ctx->eng->apply_Fadj(d, img, (hipStream_t)stream));
}

int mp_apply_H(mp_ctx* ctx, const void* dm, void* out, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!dm || !out) return fail(MP_EINVAL, "null buffer");
  if (!ctx->has_bg) return fail(MP_ESTATE, "no background set");
  return finish(ctx, ctx->eng->apply_H(dm, out, (hipStream_t)stream));
}

int mp_release_cache(mp_ctx* ctx) {
  int rc = guard(ctx);
  if (rc) return rc;
  return ctx->eng->release_cache();
}

int mp_last_stats(const mp_ctx* ctx, mp_stats* out) {
  if (!ctx || !out) return fail(MP_EINVAL, "null argument");
  const int rc = ctx->eng->collect_timing();
  if (rc) return rc;
  *out = ctx->eng->stats;
  out->bytes_reserved = ctx->budget.used;
  return MP_OK;
}

int mp_basis_create(const mp_basis_desc* d, mp_basis** out) {
  if (!d || !out) return fail(MP_EINVAL, "null argument");
  *out = nullptr;
  if (d->ndim != 2 && d->ndim != 3) return fail(MP_EINVAL, "ndim must be 2 or 3");
  if (d->family != MP_BASIS_LEGENDRE_RHO && d->family != MP_BASIS_FOURIER_ANGULAR)
    return fail(MP_EINVAL, "unknown basis family");
  if (d->na < 1 || d->nq < 1) return fail(MP_EINVAL, "empty basis");
  if (d->na * d->nq > 64) return fail(MP_EUNSUPPORTED, "at most 64 basis terms");
  mp_basis* b = new mp_basis();
  b->b.ndim = d->ndim;
  b->b.family = d->family;
  if (d->family == MP_BASIS_LEGENDRE_RHO) {
    if (!d->degs || !d->qs) {
      delete b;
      return fail(MP_EINVAL, "empty basis");
    }
    for (int i = 0; i < d->na * d->ndim; ++i)
      if (d->degs[i] < 0 || d->degs[i] > 16) {
        delete b;
        return fail(MP_EINVAL, "Legendre degrees must be in [0, 16]");
      }
    for (int i = 0; i < d->nq; ++i)
      if (d->qs[i] < 0 || d->qs[i] > 8) {
        delete b;
        return fail(MP_EINVAL, "powers of rho must be in [0, 8]");
      }
    b->b.degs.assign(d->degs, d->degs + (size_t)d->na * d->ndim);
    b->b.qs.assign(d->qs, d->qs + d->nq);
  } else {
    std::string bad;
    if (!d->modes || !d->mults) bad = "the Fourier-angular basis needs modes and mults";
    else if (!(d->tl_scale > 0.0) || !std::isfinite(d->tl_scale)) bad = "tl_scale must be positive";
    else if (d->order < -2 || d->order > 2) bad = "order must be in [-2, 2]";
    for (int a = 0; bad.empty() && a < d->na; ++a) {
      const int* m = d->modes + 4 * a;
      for (int k = 0; k < 3; ++k)
        if (m[k] < -64 || m[k] > 64) bad = "Fourier mode numbers must be in [-64, 64]";
      if (d->ndim == 2 && m[1] != 0) bad = "2D Fourier modes need m_y = 0";
      if (m[3] != 0 && m[3] != 1) bad = "mode phase must be 0 (cos) or 1 (sin)";
    }
    const int amax = d->ndim == 2 ? 16 : 8;
    for (int q = 0; bad.empty() && q < d->nq; ++q) {
      if (d->mults[2 * q] < 0 || d->mults[2 * q] > amax) bad = "angular index out of range";
      if (d->mults[2 * q + 1] < 0 || d->mults[2 * q + 1] > 16) bad = "rational Chebyshev degree must be in [0, 16]";
    }
    if (!bad.empty()) {
      delete b;
      return fail(MP_EINVAL, bad);
    }
    b->b.modes.assign(d->modes, d->modes + (size_t)4 * d->na);
    b->b.mults.assign(d->mults, d->mults + (size_t)2 * d->nq);
    b->b.order = d->order;
    b->b.tl_scale = d->tl_scale;
  }
  *out = b;
  return MP_OK;
}

void mp_basis_destroy(mp_basis* b) { delete b; }

int mp_probe_fit(mp_ctx* ctx, const mp_basis* basis, int T, const void* const* y, const void* const* x,
                 double* c, double* relres, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!basis || !y || !x || !c || T < 1) return fail(MP_EINVAL, "bad probe_fit arguments");
  if (basis->b.ndim != ctx->cfg.ndim) return fail(MP_EINVAL, "basis dimension differs from the grid");
  for (int t = 0; t < T; ++t)
    if (!y[t] || !x[t]) return fail(MP_EINVAL, "null trial buffer");
  return finish(ctx, symbol_fit(ctx, basis->b, T, y, x, c, relres, (hipStream_t)stream));
}

int mp_apply_Hinv(mp_ctx* ctx, const mp_basis* basis, const double* c, const void* img, void* out,
                  void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!basis || !c || !img || !out) return fail(MP_EINVAL, "bad apply_Hinv arguments");
  if (basis->b.ndim != ctx->cfg.ndim) return fail(MP_EINVAL, "basis dimension differs from the grid");
  for (int i = 0; i < basis->b.na() * basis->b.nq(); ++i)
    if (!std::isfinite(c[i])) return fail(MP_ENUMERIC, "non-finite coefficient");
  return finish(ctx, symbol_apply(ctx, basis->b, c, img, out, (hipStream_t)stream));
}

int mp_curvelet_create(const mp_curvelet_desc* d, mp_curvelets** out) {
  if (!d || !out) return fail(MP_EINVAL, "null argument");
  *out = nullptr;
  if (d->nscales < 2 || d->nscales > 8) return fail(MP_EINVAL, "nscales must be in [2, 8]");
  if (d->nangles < 4 || d->nangles > 64 || d->nangles % 2) return fail(MP_EINVAL, "nangles must be even, in [4, 64]");
  if (d->mask_stride < 1 || d->mask_stride > 64) return fail(MP_EINVAL, "mask_stride must be in [1, 64]");
  if (d->nfan < 1 || d->nfan > 256) return fail(MP_EINVAL, "nfan must be in [1, 256]");
  if (d->max_steps < 1 || d->max_steps > 1000000) return fail(MP_EINVAL, "max_steps must be in [1, 1e6]");
  if (!(d->ray_rtol > 0.0) || !(d->ray_rtol <= 1.0)) return fail(MP_EINVAL, "ray_rtol must be in (0, 1]");
  mp_curvelets* c = new mp_curvelets();
  c->cv = {d->nscales, d->nangles, d->mask_stride, d->nfan, d->max_steps, d->ray_rtol};
  *out = c;
  return MP_OK;
}

void mp_curvelet_destroy(mp_curvelets* cv) { delete cv; }

int mp_curvelet_wedges(const mp_curvelets* cv, int* nwedges, int* list) {
  if (!cv || !nwedges) return fail(MP_EINVAL, "null argument");
  std::vector<int> w;
  curvelet_wedges(cv->cv, w);
  *nwedges = (int)w.size() / 3;
  if (list) std::copy(w.begin(), w.end(), list);
  return MP_OK;
}

int mp_curvelet_norms(mp_ctx* ctx, const mp_curvelets* cv, double* norms, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!cv || !norms) return fail(MP_EINVAL, "null argument");
  std::vector<double> v;
  rc = curvelet_norms(ctx, cv->cv, v, (hipStream_t)stream);
  if (rc == MP_OK) std::copy(v.begin(), v.end(), norms);
  return finish(ctx, rc);
}

int mp_illumination(mp_ctx* ctx, const mp_curvelets* cv, const void* c_dev, unsigned char* mask_dev, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!cv || !c_dev || !mask_dev) return fail(MP_EINVAL, "null argument");
  return finish(ctx, curvelet_illumination(ctx, cv->cv, c_dev, mask_dev, (hipStream_t)stream));
}

int mp_curvelet_synthesis(mp_ctx* ctx, const mp_curvelets* cv, const void* coef_dev, const unsigned char* mask_dev,
                          const double* weights, void* out_dev, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!cv || !coef_dev || !out_dev) return fail(MP_EINVAL, "null argument");
  if (weights) {
    std::vector<int> w;
    curvelet_wedges(cv->cv, w);
    for (size_t i = 0; i < w.size() / 3; ++i)
      if (!std::isfinite(weights[i])) return fail(MP_ENUMERIC, "non-finite weight");
  }
  return finish(ctx, curvelet_synthesis(ctx, cv->cv, coef_dev, mask_dev, weights, out_dev, (hipStream_t)stream));
}

int mp_curvelet_analysis(mp_ctx* ctx, const mp_curvelets* cv, const void* img_dev, void* coef_dev, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!cv || !img_dev || !coef_dev) return fail(MP_EINVAL, "null argument");
  return finish(ctx, curvelet_analysis(ctx, cv->cv, img_dev, coef_dev, (hipStream_t)stream));
}

int mp_curvelet_sign_threshold(mp_ctx* ctx, const mp_curvelets* cv, void* coef_dev, double threshold, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!cv || !coef_dev) return fail(MP_EINVAL, "null argument");
  if (!(threshold >= 0.0) || !std::isfinite(threshold)) return fail(MP_EINVAL, "threshold must be finite and >= 0");
  return finish(ctx, curvelet_sign_threshold(ctx, cv->cv, coef_dev, threshold, (hipStream_t)stream));
}

int mp_vec_dot(mp_ctx* ctx, long long n, const void* a_dev, const void* b_dev, double* out, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!out || n < 0) return fail(MP_EINVAL, "bad vec_dot arguments");
  if (n == 0) {
    *out = 0.0;
    return MP_OK;
  }
  if (!a_dev || !b_dev) return fail(MP_EINVAL, "null buffer");
  return finish(ctx, vec_dot(ctx, n, a_dev, b_dev, out, (hipStream_t)stream));
}

int mp_vec_dot_noalloc(mp_ctx* ctx, long long n, const void* a_dev, const void* b_dev, double* out_dev,
                       void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!out_dev || n < 0) return fail(MP_EINVAL, "bad vec_dot_noalloc arguments");
  if (n > MP_NOALLOC_MAX_N) return fail(MP_EINVAL, "vec_dot_noalloc: n beyond MP_NOALLOC_MAX_N");
  if (n > 0 && (!a_dev || !b_dev)) return fail(MP_EINVAL, "null buffer");
  return finish(ctx, vec_dot_noalloc(ctx, n, a_dev, b_dev, out_dev, (hipStream_t)stream));
}

int mp_vec_axpby(mp_ctx* ctx, long long n, double alpha, const void* x_dev, double beta, void* y_dev, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (n < 0) return fail(MP_EINVAL, "bad vec_axpby arguments");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(MP_ENUMERIC, "non-finite scalar");
  if (n == 0) return MP_OK;
  if (!x_dev || !y_dev) return fail(MP_EINVAL, "null buffer");
  return finish(ctx, vec_axpby(ctx, n, alpha, x_dev, beta, y_dev, (hipStream_t)stream));
}

int mp_velocity_update(mp_ctx* ctx, void* c_dev, const void* dm_dev, void* stream) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!c_dev || !dm_dev) return fail(MP_EINVAL, "null buffer");
  return finish(ctx, velocity_update(ctx, c_dev, dm_dev, (hipStream_t)stream));
}

}  // extern "C"
