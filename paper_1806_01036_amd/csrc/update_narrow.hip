// Narrow basis update sweep without a fused Gram (kernel in
// update_narrow.hpp): host dispatch on k, the Y width class and the Y layout.
#include "update_narrow.hpp"

namespace borth {

namespace {

template <int KN>
hipError_t launch_k(const UpdDev& d, int kp, hipStream_t st) {
  const GramLayout none{};
  const int64_t any = INT64_MAX;
  int grid = 0;
  const bool fast = nrw::fast_y(d);
  if (d.ky == 0) return nrw::launch_t<KN, 0, false, 0>(d, kp, none, any, &grid, st);
  if (d.ky <= 16)
    return fast ? nrw::launch_t<KN, 16, true, 0>(d, kp, none, any, &grid, st)
                : nrw::launch_t<KN, 16, false, 0>(d, kp, none, any, &grid, st);
  if (d.ky <= 32)
    return fast ? nrw::launch_t<KN, 32, true, 0>(d, kp, none, any, &grid, st)
                : nrw::launch_t<KN, 32, false, 0>(d, kp, none, any, &grid, st);
  return fast ? nrw::launch_t<KN, 64, true, 0>(d, kp, none, any, &grid, st)
              : nrw::launch_t<KN, 64, false, 0>(d, kp, none, any, &grid, st);
}

}  // namespace

bool update_narrow_ok(int k, int ky, int kp) {
  return k >= 1 && k <= 8 && ky >= 0 && ky <= 64 && kp >= nrw::kn_of(k);
}

hipError_t launch_update_narrow(const UpdDev& d, int kp, hipStream_t st) {
  if (!update_narrow_ok(d.k, d.ky, kp) || d.m < 1 || !d.Q) return hipErrorInvalidValue;
  switch (nrw::kn_of(d.k)) {
    case 1: return launch_k<1>(d, kp, st);
    case 2: return launch_k<2>(d, kp, st);
    case 4: return launch_k<4>(d, kp, st);
    default: return launch_k<8>(d, kp, st);
  }
}

}  // namespace borth
