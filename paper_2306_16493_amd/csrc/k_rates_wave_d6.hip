// Wave-autonomous rate kernel instances: FP64 transforms, 6 phonon modes.
#include "rates_wave.h"

namespace eph {
namespace wave {
template hipError_t dispatch_nm<double, 6, kRates>(const RatesArgs &, hipStream_t);
}  // namespace wave
}  // namespace eph
