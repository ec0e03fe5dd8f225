// Binomial checkpointing schedules for the reverse sweep (host code).
#pragma once
#include <vector>

namespace sps {

// One action of a schedule on a working state and `slots` snapshot states (slot 0 holds X_0):
//   {CK_ADVANCE, a, b}       run steps a .. b-1 forward on the working state (not recorded)
//   {CK_TAKESHOT, slot, n}   copy the working state (the state of step n) into the slot
//   {CK_RESTORE, slot, n}    copy the slot (the state of step n) into the working state
//   {CK_YOUTURN, a, 0}       run step a forward recording its stage data, then its adjoint;
//                            the working state holds X_a before and X_{a+1} after
enum CkptOp { CK_ADVANCE = 1, CK_TAKESHOT = 2, CK_RESTORE = 3, CK_YOUTURN = 4 };
struct CkptAction {
  int op, a, b;
};

// Schedule that reverses nsteps steps with `slots` >= 1 snapshot states and the fewest forward
// steps (binomial checkpointing).  fwd: the forward sweep from X_0 to X_N, which takes the
// snapshots of the schedule's first descent; rev: the reverse sweep, whose CK_YOUTURN actions
// visit the steps N-1 .. 0 in order.
void binomial_schedule(int nsteps, int slots, std::vector<CkptAction>& fwd, std::vector<CkptAction>& rev);

// The same kind of schedule with the snapshot positions chosen for the least total cost when
// storing and loading a state cost something (a slower level of storage: host memory, disk):
// adv per forward step of the reverse sweep, wr per snapshot taken (those of the forward sweep
// included), rd per snapshot loaded.  Every split of the recursion above is searched by dynamic
// programming; with wr = rd = 0 the forward steps are the fewest, as with binomial_schedule.
// Returns the schedule's cost.  O(nsteps^2 slots) time.
double cost_schedule(int nsteps, int slots, double adv, double wr, double rd, std::vector<CkptAction>& fwd,
                     std::vector<CkptAction>& rev);

}  // namespace sps
