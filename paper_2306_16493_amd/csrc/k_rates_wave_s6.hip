// Wave-autonomous rate kernel instances: FP32 transforms, 6 phonon modes.
#include "rates_wave.h"

namespace eph {
namespace wave {
template hipError_t dispatch_nm<float, 6, kRates>(const RatesArgs &, hipStream_t);
}  // namespace wave
}  // namespace eph
