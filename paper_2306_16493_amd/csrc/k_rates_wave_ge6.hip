// Wave-autonomous rate kernel instances: FP64, 6 phonon modes, rates and transition rates written out
// (iterative BTE).
#include "rates_wave.h"

namespace eph {
namespace wave {
template hipError_t dispatch_nm<double, 6, kEmit>(const RatesArgs &, hipStream_t);
}  // namespace wave
}  // namespace eph
