// Host runtime: context, device memory accounting, error state.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

#include "../../include/matprobe.h"

namespace mp {

void set_error(const std::string& msg);

// Owning device allocation charged against a budget.
class Budget;
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void* get() const { return p_; }
  template <typename U>
  U* as() const { return static_cast<U*>(p_); }
  size_t bytes() const { return n_; }
  // (Re)allocate to at least `bytes`; keeps the old block if large enough.
  int ensure(size_t bytes, Budget* budget, const char* what);
  void release();

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
  Budget* b_ = nullptr;
};

class Budget {
 public:
  size_t limit = 0;
  size_t used = 0;
};

struct Config {
  int ndim;
  int nx, ny, nz, nb;
  double h;
  int ns, nr;
  std::vector<int> src;   // [ns][ndim]  (x, [y,] z)
  std::vector<int> rec;   // [nr][ndim]
  double f_peak, t0, dt;
  int nt;
  int dtype, snap, ckpt_every;
  double sponge_R;
  int timing;
  long long prop_cells() const {
    long long c = (long long)(nx + 2 * nb) * (nz + 2 * nb);
    if (ndim == 3) c *= (ny + 2 * nb);
    return c;
  }
  long long model_cells() const { return (long long)nx * ny * nz; }
};

// One precision/dimension specialisation of the operators.
class Engine {
 public:
  virtual ~Engine() = default;
  virtual int set_background(const void* c, hipStream_t s) = 0;
  virtual int apply_F(const void* dm, void* d, hipStream_t s) = 0;
  virtual int model(void* d, hipStream_t s) = 0;
  virtual int apply_Fadj(const void* d, void* img, hipStream_t s) = 0;
  virtual int apply_H(const void* dm, void* out, hipStream_t s) = 0;
  virtual int apply_H_batch(int nreq, const int* counts, const int* shots, const void* const* dm,
                            void* const* out, hipStream_t s) = 0;
  virtual int apply_batch(int op, int nreq, int nshots, const int* shots, const void* const* in,
                          void* const* out, hipStream_t s) = 0;
  virtual int footprint(int op, int nshots, size_t* bytes) const = 0;
  virtual int footprint_batch(int op, int nshots, int nreq, size_t* bytes) const = 0;
  virtual int release_cache() = 0;
  virtual size_t reserved() const = 0;
  // Wait for the timing events of the last call and fold them into stats.
  virtual int collect_timing() = 0;
  mp_stats stats{};
};

Engine* make_engine(const Config& c, Budget* b);

// probing basis
struct Basis {
  int ndim;
  int family = 0;         // MP_BASIS_*
  std::vector<int> degs;  // family 0: [na][ndim], axis order (x, [y,] z)
  std::vector<int> qs;    // family 0: [nq] powers of rho
  std::vector<int> modes; // family 1: [na][4] (m_x, m_y, m_z, phase)
  std::vector<int> mults; // family 1: [nq][2] (angular index, rational Chebyshev degree)
  int order = 0;          // family 1: power of rho
  double tl_scale = 1.0;  // family 1: L of TL_n
  int na() const { return family == 0 ? (int)(degs.size() / ndim) : (int)(modes.size() / 4); }
  int nq() const { return family == 0 ? (int)qs.size() : (int)(mults.size() / 2); }
};

}  // namespace mp

struct mp_ctx {
  mp::Config cfg;
  mp::Budget budget;
  mp::Engine* eng = nullptr;
  bool poisoned = false;
  bool has_bg = false;
  void* symbol_ws = nullptr;   // probing workspace (owned by symbol.hip)
  void* curvelet_ws = nullptr; // curvelet workspace (owned by curvelet.hip)
  void* vec_ws = nullptr;      // solver vector workspace (owned by vec.hip)
};

struct mp_basis {
  mp::Basis b;
};
