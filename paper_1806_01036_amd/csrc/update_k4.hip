// Update-sweep kernels for padded width K = 4 (see update_impl.hpp).
#include "update_impl.hpp"

namespace borth {
hipError_t launch_update_k4(const UpdDev& d, const UpdateArgs& a, int nwg, hipStream_t st) {
  return upd::launch_upd_k<4>(d, a, nwg, st);
}
}  // namespace borth
