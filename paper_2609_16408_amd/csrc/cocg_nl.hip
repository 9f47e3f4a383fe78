// The persistent COCG kernels with the nonlocal projector term, compiled
// apart from the projector-free ones (kernels in cocg_impl.h).
#include "cocg_impl.h"

namespace rpa {

hipError_t launch_cocg_nl(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                          hipStream_t s) {
  if (a.prec) return launch_cocg_t<3>(a, fp32_refine, grid, block, shmem, s);
  return launch_cocg_t<1>(a, fp32_refine, grid, block, shmem, s);
}

const void* cocg_nl_fn(bool fp32_refine, int m, int pitch, bool prec) {
  return prec ? cocg_fn_t<3>(fp32_refine, m, pitch) : cocg_fn_t<1>(fp32_refine, m, pitch);
}

}  // namespace rpa
