// Update-sweep kernels for padded width K = 4 (see update_impl.hpp).
#include "update_impl.hpp"

namespace borth {
hipError_t launch_update_k4(const UpdClass& c, int grid, const UpdDev& one, const UpdDev* tab,
                              const int* map, hipStream_t st) {
  return upd::launch_upd_k<4>(c, grid, one, tab, map, st);
}
}  // namespace borth
