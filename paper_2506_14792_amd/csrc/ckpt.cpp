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

class Generator {
 public:
  Generator(int n, int slots, std::vector<CkptAction>& fwd, std::vector<CkptAction>& rev)
      : n_(n), slots_(slots), fwd_(fwd), rev_(rev) {}

  void run() {
    fwd_.clear();
    rev_.clear();
    // forward sweep: X_0 stored, then the snapshots of the first (rightmost) descent of the
    // recursion, then on to X_N
    fwd_.push_back({CK_TAKESHOT, 0, 0});
    int l = 0, s = slots_ - 1, next = 1;
    while (n_ - l > 1 && s > 0) {
      const int m = l + split(n_ - l, s);
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
    if (s == 0) {
      for (int i = r - 1; i >= l; --i) {
        reach(i, l, sl);
        youturn(i);
      }
      return;
    }
    const int m = l + split(n, s);
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

  int n_, slots_, cur_ = 0;
  std::vector<CkptAction>& fwd_;
  std::vector<CkptAction>& rev_;
};

}  // namespace

void binomial_schedule(int nsteps, int slots, std::vector<CkptAction>& fwd, std::vector<CkptAction>& rev) {
  Generator(nsteps, slots, fwd, rev).run();
}

}  // namespace sps
