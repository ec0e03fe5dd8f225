// C ABI entry points: argument checks, exception-to-status translation, error strings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ckpt.h"
#include "cnn.h"
#include "fft_plan.h"
#include "sps_internal.h"
#include "../../include/sps_host.h"

struct sps_problem {
  sps::ProblemImpl* impl;
};
struct sps_cnn {
  sps::Cnn* net;
  hipStream_t s;
};

namespace {
thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <typename F>
int guard(sps_problem* P, F&& f) {
  if (!P || !P->impl) return fail(SPS_E_ARG, "null problem handle");
  try {
    f(*P->impl);
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}
template <typename F>
int cnn_guard(sps_cnn* C, F&& f) {
  if (!C || !C->net) return fail(SPS_E_ARG, "null network handle");
  try {
    f(*C->net);
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

}  // namespace

namespace sps {

AllocHooks& alloc_hooks() {
  static AllocHooks h;
  return h;
}

std::vector<double2> twiddles(int n) {
  std::vector<double2> t(n);
  const long double tau = 6.28318530717958647692528676655900577L;
  for (int i = 0; i < n; ++i) {
    const long double a = tau * (long double)i / (long double)n;
    t[i] = make_double2((double)cosl(a), (double)-sinl(a));
  }
  return t;
}

// Radices for length n = 2^a 3^b: 8s first, then 4 or 2 (a 2 joined with a 3 as a 6), then 3s.
bool fft_plan(int n, FftPlan* p) {
  if (n < 2 || n > 16384) return false;
  int m = n, a = 0, b = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  if (m != 1) return false;
  int r[32], s = 0;
  for (; a >= 3; a -= 3) r[s++] = 8;
  if (a == 2) r[s++] = 4;
  if (a == 1) {
    if (b > 0) { r[s++] = 6; --b; }
    else r[s++] = 2;
  }
  for (; b > 0; --b) r[s++] = 3;
  if (s > 12) return false;
  auto mag = [](int d) -> unsigned {
    return d == 1 ? 0u : (unsigned)(((1ull << 32) + (unsigned long long)d - 1) / (unsigned long long)d);
  };
  p->n = n;
  p->nst = s;
  int Ns = 1;
  for (int i = 0; i < s; ++i) {
    p->radix[i] = r[i];
    p->ns[i] = Ns;
    p->tst[i] = n / (Ns * r[i]);
    p->mag_nr[i] = mag(n / r[i]);
    p->mag_ns[i] = mag(Ns);
    Ns *= r[i];
  }
  return true;
}

}  // namespace sps

extern "C" {

int sps_set_allocator(void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(SPS_E_ARG, "sps_set_allocator: give both functions or neither");
  sps::AllocHooks& h = sps::alloc_hooks();
  h.alloc = alloc_fn;
  h.free = free_fn;
  h.ctx = alloc_fn ? ctx : nullptr;
  return SPS_OK;
}

int sps_build_problem(const sps_desc* desc, void* hip_stream, sps_problem** out) {
  if (!desc || !out) return fail(SPS_E_ARG, "null argument");
  *out = nullptr;
  try {
    sps::ProblemImpl* impl = nullptr;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    switch (desc->equation) {
      case SPS_RBC2D: impl = sps::make_rbc(*desc, s); break;
      case SPS_KS1D: impl = sps::make_ks(*desc, s); break;
      default: return fail(SPS_E_ARG, "unknown equation");
    }
    *out = new sps_problem{impl};
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

int sps_build_rbc_batch(const sps_desc* desc, int batch, const double* ra, void* hip_stream, sps_problem** out) {
  if (!desc || !out) return fail(SPS_E_ARG, "null argument");
  *out = nullptr;
  if (desc->equation != SPS_RBC2D) return fail(SPS_E_ARG, "batches are built for the 2D problem");
  if (batch < 1) return fail(SPS_E_ARG, "batch must be positive");
  try {
    sps::ProblemImpl* impl = sps::make_rbc_batch(*desc, batch, ra, reinterpret_cast<hipStream_t>(hip_stream));
    *out = new sps_problem{impl};
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

long long sps_state_size(const sps_problem* P) { return (P && P->impl) ? P->impl->state_size() : -1; }

int sps_factor(sps_problem* P) {
  return guard(P, [](sps::ProblemImpl& p) { p.factor(); });
}

int sps_step(sps_problem* P, double* X, int nsteps) {
  return guard(P, [&](sps::ProblemImpl& p) { p.step(X, nsteps); });
}

int sps_adjoint_step(sps_problem* P, double* Xbar, int nsteps) {
  return guard(P, [&](sps::ProblemImpl& p) { p.adjoint_step(Xbar, nsteps); });
}

int sps_cost(sps_problem* P, const double* X, double* J_out, double* dJdX) {
  return guard(P, [&](sps::ProblemImpl& p) { p.cost(X, J_out, dJdX); });
}

int sps_gradient(sps_problem* P, const double* X0, int nsteps, const double* dJdXN, double* XN, double* dJdX0,
                 double* dJdtheta, double* J_out) {
  return guard(P, [&](sps::ProblemImpl& p) {
    SPS_REQUIRE(!(dJdXN && J_out), "J_out is the built-in cost: pass NULL with an upstream cotangent dJdXN");
    p.gradient(X0, nsteps, dJdXN, XN, dJdX0, dJdtheta, J_out);
  });
}

int sps_initial_state(sps_problem* P, const double* grid, double* X) {
  return guard(P, [&](sps::ProblemImpl& p) { p.initial_state(grid, X); });
}

int sps_initial_state_adjoint(sps_problem* P, const double* Xbar, double* grid_bar) {
  return guard(P, [&](sps::ProblemImpl& p) { p.initial_state_adjoint(Xbar, grid_bar); });
}

int sps_eval_F(sps_problem* P, const double* X, double* F) {
  return guard(P, [&](sps::ProblemImpl& p) { p.eval_F(X, F); });
}

int sps_couette_frame(sps_problem* P, const double* in, double* out, int to_library, int cotangent) {
  return guard(P, [&](sps::ProblemImpl& p) { p.couette_frame(in, out, to_library, cotangent); });
}

int sps_eval_F_noalloc(sps_problem* P, const double* X, double* F) {
  return guard(P, [&](sps::ProblemImpl& p) { p.eval_F_noalloc(X, F); });
}

int sps_eval_F_vjp(sps_problem* P, const double* X, const double* Fbar, double* Xbar) {
  return guard(P, [&](sps::ProblemImpl& p) { p.eval_F_vjp(X, Fbar, Xbar); });
}

int sps_solve(sps_problem* P, const double* R, double* X, int adjoint) {
  return guard(P, [&](sps::ProblemImpl& p) { p.solve(R, X, adjoint); });
}

int sps_stability(sps_problem* P, double sigma, int iters, double* lam, double* X, double* Y, double* dlam) {
  return guard(P, [&](sps::ProblemImpl& p) { p.stability(sigma, iters, lam, X, Y, dlam); });
}

int sps_stability_vector_sens(sps_problem* P, double sigma, int iters, const double* lam, const double* X,
                              const double* Y, const double* dlam, double* dX) {
  return guard(P, [&](sps::ProblemImpl& p) { p.stability_vector_sens(sigma, iters, lam, X, Y, dlam, dX); });
}

int sps_stability_arnoldi(sps_problem* P, double sigma, int m, int nev, const double* v0, double* lam, double* X,
                          double* res, double* H) {
  return guard(P, [&](sps::ProblemImpl& p) { p.stability_arnoldi(sigma, m, nev, v0, lam, X, res, H); });
}

int sps_set_dt(sps_problem* P, double dt) {
  return guard(P, [&](sps::ProblemImpl& p) { p.set_dt(dt); });
}

int sps_set_timesteps(sps_problem* P, const double* dts, int n) {
  return guard(P, [&](sps::ProblemImpl& p) { p.set_timesteps(dts, n); });
}

int sps_set_checkpointing(sps_problem* P, int scheme, int slots) {
  return guard(P, [&](sps::ProblemImpl& p) { p.set_checkpointing(scheme, slots); });
}

int sps_set_outer_slots(sps_problem* P, int slots) {
  return guard(P, [&](sps::ProblemImpl& p) { p.set_outer_slots(slots); });
}

int sps_set_outer_costs(sps_problem* P, double write_cost, double read_cost) {
  return guard(P, [&](sps::ProblemImpl& p) { p.set_outer_costs(write_cost, read_cost); });
}

int sps_set_checkpoint_file(sps_problem* P, const char* path) {
  return guard(P, [&](sps::ProblemImpl& p) { p.set_checkpoint_file(path); });
}

int sps_checkpoint_schedule(int nsteps, int slots, int phase, int* actions, int capacity, int* count) {
  if (!count) return fail(SPS_E_ARG, "null count");
  *count = 0;
  if (nsteps < 1 || slots < 1 || (phase != 0 && phase != 1)) return fail(SPS_E_ARG, "nsteps, slots >= 1 and phase 0 or 1");
  try {
    std::vector<sps::CkptAction> fwd, rev;
    sps::binomial_schedule(nsteps, slots, fwd, rev);
    const std::vector<sps::CkptAction>& v = phase == 0 ? fwd : rev;
    *count = (int)v.size();
    if (!actions || capacity < *count) return fail(SPS_E_ARG, "actions array too small");
    for (size_t i = 0; i < v.size(); ++i) {
      actions[3 * i] = v[i].op;
      actions[3 * i + 1] = v[i].a;
      actions[3 * i + 2] = v[i].b;
    }
  } catch (const std::exception& e) {
    return fail(SPS_E_NOMEM, e.what());
  }
  return SPS_OK;
}

int sps_checkpoint_schedule_costs(int nsteps, int slots, double adv, double wr, double rd, int phase, int* actions,
                                  int capacity, int* count, double* cost) {
  if (!count) return fail(SPS_E_ARG, "null count");
  *count = 0;
  if (nsteps < 1 || slots < 1 || (phase != 0 && phase != 1)) return fail(SPS_E_ARG, "nsteps, slots >= 1 and phase 0 or 1");
  if (!(adv >= 0.0 && wr >= 0.0 && rd >= 0.0) || !std::isfinite(adv + wr + rd))
    return fail(SPS_E_ARG, "costs must be finite and >= 0");
  // (the search takes nsteps^2 min(slots, nsteps) steps)
  if ((double)nsteps * nsteps * std::min(slots, nsteps) > 2e10) return fail(SPS_E_ARG, "too many steps for the cost search");
  try {
    std::vector<sps::CkptAction> fwd, rev;
    const double c = sps::cost_schedule(nsteps, slots, adv, wr, rd, fwd, rev);
    if (cost) *cost = c;
    const std::vector<sps::CkptAction>& v = phase == 0 ? fwd : rev;
    *count = (int)v.size();
    if (!actions || capacity < *count) return fail(SPS_E_ARG, "actions array too small");
    for (size_t i = 0; i < v.size(); ++i) {
      actions[3 * i] = v[i].op;
      actions[3 * i + 1] = v[i].a;
      actions[3 * i + 2] = v[i].b;
    }
  } catch (const std::exception& e) {
    return fail(SPS_E_NOMEM, e.what());
  }
  return SPS_OK;
}

int sps_lbvp_solve(sps_problem* P, const double* f, double* X) {
  return guard(P, [&](sps::ProblemImpl& p) { p.lbvp_solve(f, X); });
}

int sps_lbvp_adjoint(sps_problem* P, const double* Xbar, double* fbar) {
  return guard(P, [&](sps::ProblemImpl& p) { p.lbvp_adjoint(Xbar, fbar); });
}

int sps_timer_enable(sps_problem* P, int kind, int on) {
  return guard(P, [&](sps::ProblemImpl& p) { p.timer_enable(kind, on != 0); });
}

int sps_timer_read(sps_problem* P, long long* launches, double* total_ms) {
  if (!launches || !total_ms) return fail(SPS_E_ARG, "null argument");
  return guard(P, [&](sps::ProblemImpl& p) { p.timer_read(launches, total_ms); });
}

int sps_build_sh_batch(int batch, const int* n, const double* r, double lx, double dt, int max_steps,
                       void* hip_stream, sps_problem** out) {
  if (!out || !n || !r) return fail(SPS_E_ARG, "null argument");
  *out = nullptr;
  try {
    sps::ProblemImpl* impl =
        sps::make_sh_batch(batch, n, r, lx, dt, max_steps, reinterpret_cast<hipStream_t>(hip_stream));
    *out = new sps_problem{impl};
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

int sps_sh_tuning(const sps_problem* P, int* col_tile, int* row_tile, int* blocks, int* threads, double* step_ms) {
  if (!col_tile || !row_tile || !blocks || !threads || !step_ms) return fail(SPS_E_ARG, "null argument");
  return guard(const_cast<sps_problem*>(P),
               [&](sps::ProblemImpl& p) { sps::sh_tuning(&p, col_tile, row_tile, blocks, threads, step_ms); });
}

int sps_build_couette(int nx, int ny, int nz, double lx, double lz, double re, double dt, int checkpoint_every,
                      int max_steps, void* hip_stream, sps_problem** out) {
  if (!out) return fail(SPS_E_ARG, "null argument");
  *out = nullptr;
  try {
    const sps::CouetteSpec c{nx, ny, nz, lx, lz, re, dt, checkpoint_every, max_steps};
    sps::ProblemImpl* impl = sps::make_couette(c, reinterpret_cast<hipStream_t>(hip_stream));
    *out = new sps_problem{impl};
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

int sps_build_poiseuille(int nz, int max_systems, void* hip_stream, sps_problem** out) {
  if (!out) return fail(SPS_E_ARG, "null argument");
  *out = nullptr;
  try {
    sps::ProblemImpl* impl = sps::make_poiseuille(nz, max_systems, reinterpret_cast<hipStream_t>(hip_stream));
    *out = new sps_problem{impl};
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

int sps_poiseuille_solve(sps_problem* P, int nsys, const double* params, int iters, int mode, double tol, int maxit,
                         double* lam, double* dlam, double* info, double* X, double* Y) {
  return guard(P, [&](sps::ProblemImpl& p) {
    sps::poiseuille_run(&p, nsys, params, iters, mode, tol, maxit, lam, dlam, info, X, Y);
  });
}

int sps_poiseuille_host_band(int nz, double alpha, double re, double sig_re, double sig_im, int* S, int* kl, int* ku,
                             double* band, int* rowmap, int* colmap, double* rho) {
  if (!S || !kl || !ku) return fail(SPS_E_ARG, "null argument");
  try {
    sps::poiseuille_host_band(nz, alpha, re, sig_re, sig_im, S, kl, ku, band, rowmap, colmap, rho);
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  }
}

int sps_build_kolmo(int batch, int n, double re, double drag, double dt, int max_steps, int closure,
                    int keep_history, void* hip_stream, sps_problem** out) {
  if (!out) return fail(SPS_E_ARG, "null argument");
  *out = nullptr;
  try {
    sps::ProblemImpl* impl = sps::make_kolmo(batch, n, re, drag, dt, max_steps, closure, keep_history,
                                             reinterpret_cast<hipStream_t>(hip_stream));
    *out = new sps_problem{impl};
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

int sps_kolmo_set_params(sps_problem* P, const double* theta) {
  if (!theta) return fail(SPS_E_ARG, "null argument");
  return guard(P, [&](sps::ProblemImpl& p) { sps::kolmo_set_params(&p, theta); });
}

int sps_kolmo_forward(sps_problem* P, const double* X0, int nsteps, double* XN, double* snap, int every, int nc) {
  return guard(P, [&](sps::ProblemImpl& p) { sps::kolmo_forward(&p, X0, nsteps, XN, snap, every, nc); });
}

int sps_kolmo_rollout(sps_problem* P, const double* X0, const double* targets, int nsteps, double* XN, double* J,
                      double* dJdX0, double* dJdtheta) {
  if (!X0 || !targets) return fail(SPS_E_ARG, "null argument");
  return guard(P, [&](sps::ProblemImpl& p) { sps::kolmo_rollout(&p, X0, targets, nsteps, XN, J, dJdX0, dJdtheta); });
}

int sps_kolmo_param_vjp(sps_problem* P, const double* X, const double* Fbar, double* theta_bar) {
  if (!X || !Fbar || !theta_bar) return fail(SPS_E_ARG, "null argument");
  return guard(P, [&](sps::ProblemImpl& p) { sps::kolmo_param_vjp(&p, X, Fbar, theta_bar); });
}

int sps_kolmo_adam(sps_problem* P, double* theta, const double* grad, double* m1, double* m2, double lr, int t) {
  if (!theta || !grad || !m1 || !m2 || t < 1) return fail(SPS_E_ARG, "bad argument");
  return guard(P, [&](sps::ProblemImpl& p) { sps::kolmo_adam(&p, theta, grad, m1, m2, lr, t); });
}


int sps_cnn_build(int batch, int H, int W, void* hip_stream, sps_cnn** out) {
  if (!out) return fail(SPS_E_ARG, "null argument");
  *out = nullptr;
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    *out = new sps_cnn{new sps::Cnn(batch, H, W, s), s};
    return SPS_OK;
  } catch (const sps::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SPS_E_HIP, e.what());
  }
}

int sps_cnn_nparam(void) { return sps::Cnn::nparam(); }

int sps_cnn_set_params(sps_cnn* C, const double* theta) {
  if (!theta) return fail(SPS_E_ARG, "null argument");
  return cnn_guard(C, [&](sps::Cnn& n) { n.set_params(theta); });
}

int sps_cnn_forward(sps_cnn* C, const double* x, double* y) {
  if (!x || !y) return fail(SPS_E_ARG, "null argument");
  return cnn_guard(C, [&](sps::Cnn& n) { n.forward(x, y, 1.0, false); });
}

int sps_cnn_vjp(sps_cnn* C, const double* x, const double* ybar, double* xbar, double* theta_bar) {
  if (!x || !ybar || !xbar) return fail(SPS_E_ARG, "null argument");
  return cnn_guard(C, [&](sps::Cnn& n) { n.vjp(x, ybar, xbar, 1.0, false, theta_bar); });
}

void sps_cnn_destroy(sps_cnn* C) {
  if (!C) return;
  (void)hipStreamSynchronize(C->s);
  delete C->net;
  delete C;
}

int sps_set_graph(sps_problem* P, int on) {
  return guard(P, [&](sps::ProblemImpl& p) { p.set_graph(on != 0); });
}

int sps_sync(sps_problem* P) {
  int flag = 0;
  int rc = guard(P, [&](sps::ProblemImpl& p) {
    SPS_HIP(hipStreamSynchronize(p.stream));
    flag = p.device_error();
  });
  if (rc != SPS_OK) return rc;
  if (flag & 1) return fail(SPS_E_SINGULAR, "zero pivot in the LU factorization");
  if (flag & 2) return fail(SPS_E_NONFINITE, "state became non-finite");
  if (flag & 4) return fail(SPS_E_NOCONV, "an eigenvalue iteration did not converge");
  return SPS_OK;
}

const char* sps_last_error(void) { return g_last_error.c_str(); }

void sps_destroy(sps_problem* P) {
  if (!P) return;
  if (P->impl) {
    (void)hipStreamSynchronize(P->impl->stream);
    delete P->impl;
  }
  delete P;
}

}  // extern "C"
