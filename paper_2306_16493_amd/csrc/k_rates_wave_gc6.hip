// Wave-autonomous rate kernel instances: FP64, 6 phonon modes, per-state counts of the transition rates
// (iterative BTE).
#include "rates_wave.h"

namespace eph {
namespace wave {
template hipError_t dispatch_nm<double, 6, kCount>(const RatesArgs &, hipStream_t);
}  // namespace wave
}  // namespace eph
