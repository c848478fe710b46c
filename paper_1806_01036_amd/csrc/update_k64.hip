// Update-sweep kernels for padded width K = 64 (see update_impl.hpp).
#include "update_impl.hpp"

namespace borth {
hipError_t launch_update_k64(const UpdClass& c, int grid, const UpdDev& one, const UpdDev* tab,
                              const int* map, hipStream_t st) {
  return upd::launch_upd_k<64>(c, grid, one, tab, map, st);
}
}  // namespace borth
