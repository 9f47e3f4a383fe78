// The persistent COCG kernels with the nonlocal projector term, compiled
// apart from the projector-free ones (kernels in cocg_impl.h).
#include "cocg_impl.h"

namespace rpa {

hipError_t launch_cocg_nl(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                          hipStream_t s) {
  return launch_cocg_t<true>(a, fp32_refine, grid, block, shmem, s);
}

const void* cocg_nl_fn(bool fp32_refine, int m, int pitch) {
  return cocg_fn_t<true>(fp32_refine, m, pitch);
}

}  // namespace rpa
