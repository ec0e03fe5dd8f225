// Binomial checkpointing schedules for the reverse sweep (host code).
//
// The adjoint of an N-step run visits the steps in reverse and needs each step's stage data,
// recomputed from stored states.  With `slots` stored states the fewest forward steps follow
// from the binomial partition of the run: an interval of n steps whose first state is stored,
// with s further free slots, is reversible in t forward passes iff n <= C(s + 1 + t, s + 1);
// its optimal first snapshot splits it into a right part reversible with s slots and a left
// part reversible with s + 1 slots in one pass less.  Each part is then reversed recursively,
// right first; the slots of the right part are free again for the left part.
#include "ckpt.h"

#include <algorithm>

namespace sps {
namespace {

// C(n, k), saturating far above any step count
long long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  k = std::min(k, n - k);
  long long r = 1;
  for (int i = 1; i <= k; ++i) {
    r = r * (n - k + i) / i;
    if (r > (1LL << 40)) return 1LL << 40;
  }
  return r;
}

// Offset of the first snapshot in an interval of n > 1 steps with s >= 1 free slots besides the
// one holding its first state.  t is the smallest pass count with C(s + 1 + t, s + 1) >= n; the
// split keeps the right part within C(s + t - 1, s) steps and the left part within
// C(s + t, s + 1), which attains the minimal total of forward steps.
int split(int n, int s) {
  int t = 0;
  while (binom(s + 1 + t, s + 1) < n) ++t;
  const long long m = std::min<long long>(n - binom(s + t - 1, s), binom(s + t, s + 1));
  return (int)std::max<long long>(1, std::min<long long>(n - 1, m));
}

// Split choices of the cost model: D(n, s) reverses n steps whose first state is stored and in
// hand, with s more free slots; C(n, s) = rd + D(n, s) has to load that state first; F(n, s)
// reverses the steps that the forward sweep ran through, which takes the snapshots of the first
// descent without extra forward steps (and ends with X_n in hand, so its last part loads first).
//   D(1, s) = 0,  D(n, 0) = adv (n - 1) + (n - 1) rd + adv (n - 1)(n - 2) / 2,
//   D(n, s) = min(D(n, 0), min_j adv j + wr + D(n - j, s - 1) + C(j, s)),
//   F(1, s) = rd,  F(n, 0) = C(n, 0),  F(n, s) = min(C(n, 0), min_j wr + F(n - j, s - 1) + C(j, s)),
// j the length of the left part (the snapshot's offset), the right part reversed first; split 0
// stands for the first option (no further snapshot: every step recomputed from the interval's
// first state), which can win when a snapshot costs more than the steps it saves.
class CostSplits {
 public:
  // (more than n slots never help an interval of at most n steps: the table stops at n)
  CostSplits(int n, int slots, double adv, double wr, double rd)
      : n_(n), s_(std::min(slots, n)), adv_(adv), wr_(wr), rd_(rd),
        D_((size_t)(n + 1) * s_, 0.0), F_((size_t)(n + 1) * s_, 0.0),
        jd_((size_t)(n + 1) * s_, 1), jf_((size_t)(n + 1) * s_, 1) {
    for (int s = 0; s < s_; ++s)
      for (int n1 = 1; n1 <= n_; ++n1) {
        double& d = at(D_, n1, s);
        double& f = at(F_, n1, s);
        if (n1 == 1) {
          d = 0.0;
          f = rd_;
        } else if (s == 0) {
          d = adv_ * (n1 - 1) + (n1 - 1) * rd_ + adv_ * 0.5 * (double)(n1 - 1) * (n1 - 2);
          f = rd_ + d;
        } else {
          double bd = at(D_, n1, 0), bf = at(F_, n1, 0);
          int id = 0, jf = 0;
          for (int j = 1; j < n1; ++j) {
            const double left = rd_ + at(D_, j, s);
            const double vd = adv_ * j + wr_ + at(D_, n1 - j, s - 1) + left;
            const double vf = wr_ + at(F_, n1 - j, s - 1) + left;
            if (vd < bd) {
              bd = vd;
              id = j;
            }
            if (vf < bf) {
              bf = vf;
              jf = j;
            }
          }
          d = bd;
          f = bf;
          at(jd_, n1, s) = id;
          at(jf_, n1, s) = jf;
        }
      }
  }
  int split(int n, int s, bool descent) const { return at(descent ? jf_ : jd_, n, std::min(s, s_ - 1)); }
  double total() const { return wr_ + at(F_, n_, s_ - 1); }   // (X_0's snapshot included)

 private:
  template <typename T>
  T& at(std::vector<T>& v, int n, int s) { return v[(size_t)n * s_ + s]; }
  template <typename T>
  const T& at(const std::vector<T>& v, int n, int s) const { return v[(size_t)n * s_ + s]; }
  int n_, s_;
  double adv_, wr_, rd_;
  std::vector<double> D_, F_;
  std::vector<int> jd_, jf_;
};

class Generator {
 public:
  Generator(int n, int slots, std::vector<CkptAction>& fwd, std::vector<CkptAction>& rev,
            const CostSplits* cs = nullptr)
      : n_(n), slots_(slots), fwd_(fwd), rev_(rev), cs_(cs) {}

  void run() {
    fwd_.clear();
    rev_.clear();
    // forward sweep: X_0 stored, then the snapshots of the first (rightmost) descent of the
    // recursion, then on to X_N
    fwd_.push_back({CK_TAKESHOT, 0, 0});
    int l = 0, s = slots_ - 1, next = 1;
    while (n_ - l > 1 && s > 0 && pick(n_ - l, s, true) > 0) {
      const int m = l + pick(n_ - l, s, true);
      fwd_.push_back({CK_ADVANCE, l, m});
      fwd_.push_back({CK_TAKESHOT, next, m});
      l = m;
      ++next;
      --s;
    }
    if (l < n_) fwd_.push_back({CK_ADVANCE, l, n_});
    cur_ = n_;
    reverse(0, n_, 0, slots_ - 1, 1, true);
  }

 private:
  // reverse steps l .. r-1; X_l is in slot sl; s free slots from index `next`; `taken`: the
  // snapshots of this descent were stored by the forward sweep
  void reverse(int l, int r, int sl, int s, int next, bool taken) {
    const int n = r - l;
    if (n == 1) {
      reach(l, l, sl);
      youturn(l);
      return;
    }
    if (s == 0 || pick(n, s, taken) == 0) {
      for (int i = r - 1; i >= l; --i) {
        reach(i, l, sl);
        youturn(i);
      }
      return;
    }
    const int m = l + pick(n, s, taken);
    if (!taken) {
      reach(m, l, sl);
      rev_.push_back({CK_TAKESHOT, next, m});
    }
    reverse(m, r, next, s - 1, next + 1, taken);
    reverse(l, m, sl, s, next, false);
  }
  // bring the working state to step `target` of the interval that starts at l (X_l in sl)
  void reach(int target, int l, int sl) {
    if (cur_ < l || cur_ > target) {
      rev_.push_back({CK_RESTORE, sl, l});
      cur_ = l;
    }
    if (cur_ < target) {
      rev_.push_back({CK_ADVANCE, cur_, target});
      cur_ = target;
    }
  }
  void youturn(int i) {
    rev_.push_back({CK_YOUTURN, i, 0});
    cur_ = i + 1;
  }
  // the snapshot offset of an interval of n steps with s free slots (descent: one of the
  // intervals whose snapshots the forward sweep takes)
  int pick(int n, int s, bool descent) const { return cs_ ? cs_->split(n, s, descent) : split(n, s); }

  int n_, slots_, cur_ = 0;
  std::vector<CkptAction>& fwd_;
  std::vector<CkptAction>& rev_;
  const CostSplits* cs_;
};

}  // namespace

void binomial_schedule(int nsteps, int slots, std::vector<CkptAction>& fwd, std::vector<CkptAction>& rev) {
  Generator(nsteps, slots, fwd, rev).run();
}

double cost_schedule(int nsteps, int slots, double adv, double wr, double rd, std::vector<CkptAction>& fwd,
                     std::vector<CkptAction>& rev) {
  const CostSplits cs(nsteps, slots, adv, wr, rd);
  Generator(nsteps, slots, fwd, rev, &cs).run();
  return cs.total();
}

}  // namespace sps
