// SERTA scattering rates, wave-autonomous form: shape selection and dispatch
// to the per-(precision, modes) instances of the kernel in rates_wave.h.
#include "internal.h"

namespace eph {
namespace wave {
template <class T, int NM, int MODE>
hipError_t dispatch_nm(const RatesArgs &a, hipStream_t st);
extern template hipError_t dispatch_nm<double, 3, kRates>(const RatesArgs &, hipStream_t);
extern template hipError_t dispatch_nm<double, 6, kRates>(const RatesArgs &, hipStream_t);
extern template hipError_t dispatch_nm<float, 3, kRates>(const RatesArgs &, hipStream_t);
extern template hipError_t dispatch_nm<float, 6, kRates>(const RatesArgs &, hipStream_t);
extern template hipError_t dispatch_nm<double, 3, kCount>(const RatesArgs &, hipStream_t);
extern template hipError_t dispatch_nm<double, 6, kCount>(const RatesArgs &, hipStream_t);
extern template hipError_t dispatch_nm<double, 3, kEmit>(const RatesArgs &, hipStream_t);
extern template hipError_t dispatch_nm<double, 6, kEmit>(const RatesArgs &, hipStream_t);
}  // namespace wave

// Shapes served by the wave-autonomous kernel: a cubic Rp box of edge 4 or
// 6 and final-state lines of at most 2048 energies (N * n_wann).  Returns
// the states per group, 0 when the shape is not served.
int rates_wave_group(int nw, int nm, RpBox box, int N, int precision) {
  const bool cube = box.n[0] == box.n[1] && box.n[1] == box.n[2] && (box.n[0] == 4 || box.n[0] == 6);
  if (!cube || N * nw > kMaxLine) return 0;
  (void)precision;
  if (nm == 3 && (nw == 1 || nw == 2 || nw == 4)) return 2;
  if (nm == 3 && nw == 8) return 1;
  if (nm == 6 && (nw == 1 || nw == 2)) return 2;
  if (nm == 6 && (nw == 4 || nw == 8)) return 1;
  return 0;
}

// mode kCount / kEmit (transition rates) are FP64 only.
hipError_t launch_rates_wave(int precision, const RatesArgs &a, hipStream_t st, int mode) {
  if (a.ng <= 0) return hipSuccess;
  const bool m3 = a.nm == 3;
  if (mode == kCount) {
    if (precision != EPH_FP64) return hipErrorNotSupported;
    return m3 ? wave::dispatch_nm<double, 3, kCount>(a, st) : wave::dispatch_nm<double, 6, kCount>(a, st);
  }
  if (mode == kEmit) {
    if (precision != EPH_FP64) return hipErrorNotSupported;
    return m3 ? wave::dispatch_nm<double, 3, kEmit>(a, st) : wave::dispatch_nm<double, 6, kEmit>(a, st);
  }
  if (precision == EPH_FP64) return m3 ? wave::dispatch_nm<double, 3, kRates>(a, st) : wave::dispatch_nm<double, 6, kRates>(a, st);
  return m3 ? wave::dispatch_nm<float, 3, kRates>(a, st) : wave::dispatch_nm<float, 6, kRates>(a, st);
}

}  // namespace eph
