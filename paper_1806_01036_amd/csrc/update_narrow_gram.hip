// Narrow basis update sweep with the next pass's Gram columns fused in
// (kernel in update_narrow.hpp): host dispatch.  Y must be stored densely
// with an even number of columns (or be absent), and ky + k <= 64.  With
// d.bw the Gram columns are B-weighted (B = diag(d.bw)).
#include "update_narrow.hpp"

namespace borth {

namespace {

template <int KN, int GR>
hipError_t launch_kg(const UpdDev& d, int kp, const GramLayout& G, int64_t max_wg, int* grid,
                     hipStream_t st) {
  if (d.ky == 0) return nrw::launch_t<KN, 0, false, GR>(d, kp, G, max_wg, grid, st);
  if (d.ky <= 16) return nrw::launch_t<KN, 16, true, GR>(d, kp, G, max_wg, grid, st);
  if (d.ky <= 32) return nrw::launch_t<KN, 32, true, GR>(d, kp, G, max_wg, grid, st);
  return nrw::launch_t<KN, 64, true, GR>(d, kp, G, max_wg, grid, st);
}

template <int GR>
hipError_t launch_g(const UpdDev& d, int kp, const GramLayout& G, int64_t max_wg, int* grid,
                    hipStream_t st) {
  switch (nrw::kn_of(d.k)) {
    case 1: return launch_kg<1, GR>(d, kp, G, max_wg, grid, st);
    case 2: return launch_kg<2, GR>(d, kp, G, max_wg, grid, st);
    case 4: return launch_kg<4, GR>(d, kp, G, max_wg, grid, st);
    default: return launch_kg<8, GR>(d, kp, G, max_wg, grid, st);
  }
}

}  // namespace

bool update_narrow_gram_ok(const UpdDev& d, int kp) {
  return update_narrow_ok(d.k, d.ky, kp) && d.ky + d.k <= 64 && (d.ky == 0 || nrw::fast_y(d));
}

hipError_t launch_update_narrow_gram(const UpdDev& d, int kp, int mode, const GramLayout& G,
                                     int64_t max_wg, int* nwg, hipStream_t st) {
  if (!update_narrow_gram_ok(d, kp) || d.m < 1 || !d.Q || !d.part || G.ky != d.ky || G.k != d.k)
    return hipErrorInvalidValue;
  if (d.bw) return mode ? launch_g<4>(d, kp, G, max_wg, nwg, st) : launch_g<3>(d, kp, G, max_wg, nwg, st);
  return mode ? launch_g<2>(d, kp, G, max_wg, nwg, st) : launch_g<1>(d, kp, G, max_wg, nwg, st);
}

}  // namespace borth
