// The persistent COCG kernels with preconditioned solves and no nonlocal
// term, compiled apart from the plain ones (kernels in cocg_impl.h).
#include "cocg_impl.h"

namespace rpa {

hipError_t launch_cocg_pc(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                          hipStream_t s) {
  return launch_cocg_t<2>(a, fp32_refine, grid, block, shmem, s);
}

const void* cocg_pc_fn(bool fp32_refine, int m, int pitch) {
  return cocg_fn_t<2>(fp32_refine, m, pitch);
}

}  // namespace rpa
