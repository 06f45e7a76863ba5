// Wave-autonomous rate kernel instances: FP64, 3 phonon modes, rates and transition rates written out
// (iterative BTE).
#include "rates_wave.h"

namespace eph {
namespace wave {
template hipError_t dispatch_nm<double, 3, kEmit>(const RatesArgs &, hipStream_t);
}  // namespace wave
}  // namespace eph
