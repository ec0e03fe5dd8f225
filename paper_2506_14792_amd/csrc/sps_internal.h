// Host-side internals shared by the C ABI and the problem implementations.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sps.h"

namespace sps {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SPS_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::sps::Error(SPS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define SPS_CHECK_LAUNCH() SPS_HIP(hipGetLastError())

#define SPS_REQUIRE(cond, msg)                                  \
  do {                                                          \
    if (!(cond)) throw ::sps::Error(SPS_E_ARG, (msg));          \
  } while (0)

// The caller's device allocator (sps_set_allocator), process-wide; null functions: hipMalloc.
struct AllocHooks {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
AllocHooks& alloc_hooks();

// Device allocation owned by a problem; freed in the destructor (through the allocator that
// made each block).
class DevArena {
 public:
  ~DevArena() {
    // hipFree waits for the device; a caller's free may not, so the work that used its blocks
    // is finished first
    bool hooked = false;
    for (const Block& b : blocks_) hooked = hooked || b.free != nullptr;
    if (hooked) (void)hipDeviceSynchronize();
    for (const Block& b : blocks_) {
      if (b.free) b.free(b.p, b.ctx);
      else (void)hipFree(b.p);
    }
  }
  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    const AllocHooks h = alloc_hooks();
    if (h.alloc) {
      p = h.alloc(bytes, h.ctx);
      if (!p) throw Error(SPS_E_NOMEM, "the caller's allocator returned no block of " + std::to_string(bytes) + " bytes");
      blocks_.push_back({p, h.free, h.ctx});
    } else {
      if (hipMalloc(&p, bytes) != hipSuccess)
        throw Error(SPS_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
      blocks_.push_back({p, nullptr, nullptr});
    }
    return static_cast<T*>(p);
  }
  template <typename T>
  T* upload(const std::vector<T>& h, hipStream_t s) {
    T* d = alloc<T>(h.size());
    SPS_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    SPS_HIP(hipStreamSynchronize(s));
    return d;
  }

 private:
  struct Block {
    void* p;
    void (*free)(void*, void*);
    void* ctx;
  };
  std::vector<Block> blocks_;
};

// HIP-event timing of one kernel class: launches are bracketed by events from a pool
// created when timing is enabled, so recording never synchronizes the stream.  Once the
// pool is used up further launches are not timed (the first `capacity` are a sample).
class KernelTimer {
 public:
  static constexpr int kCapacity = 8192;
  ~KernelTimer() { release(); }
  void enable(bool on) {
    release();
    on_ = on;
    if (!on) return;
    pool_.resize(2 * kCapacity);
    for (auto& e : pool_)
      if (hipEventCreate(&e) != hipSuccess) { e = nullptr; on_ = false; }
    used_ = 0;
  }
  // Event pair for the next timed launch (handed to hipExtLaunchKernelGGL, which stamps the
  // dispatch itself), or false when timing is off or the pool is used up.
  bool take(hipEvent_t* start, hipEvent_t* stop) {
    if (!on_ || used_ >= kCapacity) return false;
    *start = pool_[2 * used_];
    *stop = pool_[2 * used_ + 1];
    ++used_;
    return true;
  }
  void read(long long* launches, double* total_ms) {
    double tot = 0.0;
    long long n = 0;
    for (int i = 0; i < used_; ++i) {
      float ms = 0.f;
      if (hipEventSynchronize(pool_[2 * i + 1]) == hipSuccess &&
          hipEventElapsedTime(&ms, pool_[2 * i], pool_[2 * i + 1]) == hipSuccess) {
        tot += ms;
        ++n;
      }
    }
    used_ = 0;
    *launches = n;
    *total_ms = tot;
  }

 private:
  void release() {
    for (auto e : pool_)
      if (e) (void)hipEventDestroy(e);
    pool_.clear();
    used_ = 0;
    on_ = false;
  }
  bool on_ = false;
  int used_ = 0;
  std::vector<hipEvent_t> pool_;
};

class ProblemImpl {
 public:
  virtual ~ProblemImpl() = default;
  virtual long long state_size() const = 0;
  virtual void factor() = 0;
  virtual void step(double* X, int nsteps) = 0;
  virtual void adjoint_step(double* Xbar, int nsteps) = 0;
  virtual void cost(const double* X, double* J, double* dJdX) = 0;
  // dJdXN (nullable): the cotangent of the final state from the caller (the reverse sweep starts
  // there; J must then be null); null: the built-in cost J and its gradient.  dJdtheta (nullable):
  // the gradient with respect to the problem's parameters, where the problem has them.
  virtual void gradient(const double* X0, int nsteps, const double* dJdXN, double* XN, double* dJdX0,
                        double* dJdtheta, double* J) = 0;
  virtual void initial_state(const double* grid, double* X) = 0;
  virtual void initial_state_adjoint(const double* Xbar, double* grid) = 0;
  virtual void eval_F(const double* X, double* F) = 0;
  virtual void eval_F_vjp(const double* X, const double* Fbar, double* Xbar) = 0;
  virtual void couette_frame(const double*, double*, int, int) {
    throw Error(SPS_E_UNSUPPORTED, "the frame conversion is for plane Couette states");
  }
  virtual void eval_F_noalloc(const double*, double*) {
    throw Error(SPS_E_UNSUPPORTED, "the allocation-free evaluation is built for the 2D problem");
  }
  virtual void solve(const double* R, double* X, int adjoint) = 0;
  virtual void stability(double, int, double*, double*, double*, double*) {
    throw Error(SPS_E_UNSUPPORTED, "the eigenvalue problem is built for the 2D problem");
  }
  virtual void stability_vector_sens(double, int, const double*, const double*, const double*, const double*,
                                     double*) {
    throw Error(SPS_E_UNSUPPORTED, "the eigenvalue problem is built for the 2D problem");
  }
  virtual void stability_arnoldi(double, int, int, const double*, double*, double*, double*, double*) {
    throw Error(SPS_E_UNSUPPORTED, "the eigenvalue problem is built for the 2D problem");
  }
  virtual void set_dt(double) { throw Error(SPS_E_UNSUPPORTED, "the step is fixed for this problem"); }
  virtual void set_timesteps(const double*, int) {
    throw Error(SPS_E_UNSUPPORTED, "variable steps are built for the KS problem");
  }
  virtual void set_checkpointing(int, int) {
    throw Error(SPS_E_UNSUPPORTED, "checkpoint schedules are built for the RK222 problems");
  }
  virtual void set_outer_slots(int) {
    throw Error(SPS_E_UNSUPPORTED, "checkpoint schedules are built for the RK222 problems");
  }
  virtual void set_outer_costs(double, double) {
    throw Error(SPS_E_UNSUPPORTED, "checkpoint schedules are built for the RK222 problems");
  }
  virtual void set_checkpoint_file(const char*) {
    throw Error(SPS_E_UNSUPPORTED, "checkpoint schedules are built for the RK222 problems");
  }
  virtual void lbvp_solve(const double*, double*) {
    throw Error(SPS_E_UNSUPPORTED, "no boundary value problem for this equation");
  }
  virtual void lbvp_adjoint(const double*, double*) {
    throw Error(SPS_E_UNSUPPORTED, "no boundary value problem for this equation");
  }
  virtual void timer_enable(int kind, bool on) = 0;
  virtual void timer_read(long long* launches, double* ms) = 0;
  virtual int device_error() = 0;  // reads and clears the sticky device flag
  virtual void set_graph(bool on) {
    if (on) throw Error(SPS_E_UNSUPPORTED, "graph mode is not available for this problem");
  }
  hipStream_t stream = nullptr;
};

ProblemImpl* make_rbc(const sps_desc& d, hipStream_t s);
ProblemImpl* make_rbc_batch(const sps_desc& d, int batch, const double* ra, hipStream_t s);
ProblemImpl* make_ks(const sps_desc& d, hipStream_t s);
ProblemImpl* make_sh_batch(int batch, const int* n, const double* r, double lx, double dt, int max_steps,
                           hipStream_t s);
void sh_tuning(ProblemImpl* p, int* col_tile, int* row_tile, int* blocks, int* threads, double* tuned_ms);
struct CouetteSpec {
  int nx, ny, nz;
  double lx, lz, re, dt;
  int checkpoint_every, max_steps;
};
ProblemImpl* make_couette(const CouetteSpec& c, hipStream_t s);
ProblemImpl* make_kolmo(int batch, int N, double Re, double drag, double dt, int max_steps, int closure,
                        int keep_history, hipStream_t s);
void kolmo_set_params(ProblemImpl* p, const double* theta);
void kolmo_forward(ProblemImpl* p, const double* X0, int nsteps, double* XN, double* snap, int every, int Nc);
void kolmo_rollout(ProblemImpl* p, const double* X0, const double* targets, int nsteps, double* XN, double* J,
                   double* dJdX0, double* dJdtheta);
void kolmo_param_vjp(ProblemImpl* p, const double* X, const double* Fbar, double* th_bar);
void kolmo_adam(ProblemImpl* p, double* theta, const double* grad, double* m1, double* m2, double lr, int t);

ProblemImpl* make_poiseuille(int nz, int max_systems, hipStream_t s);
void poiseuille_run(ProblemImpl* p, int nsys, const double* params, int iters, int mode, double tol, int maxit,
                    double* lam, double* dlam, double* info, double* X, double* Y);
void poiseuille_host_band(int nz, double alpha, double re, double sig_re, double sig_im, int* S, int* kl, int* ku,
                          double* band, int* rowmap, int* colmap, double* rho);

// Host helpers shared by problem builders.
std::vector<double2> twiddles(int n);            // exp(-2 pi i t / n), t < n

}  // namespace sps
