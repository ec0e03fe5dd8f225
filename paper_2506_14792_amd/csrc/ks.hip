// 1D Kuramoto-Sivashinsky (Fourier, SBDF2) — placeholder until its kernels land.
#include "sps_internal.h"

namespace sps {
ProblemImpl* make_ks(const sps_desc&, hipStream_t) {
  throw Error(SPS_E_UNSUPPORTED, "KS problem not built yet");
}
}  // namespace sps
