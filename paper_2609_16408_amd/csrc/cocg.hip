// Batched Sternheimer COCG launches (kernels in cocg_impl.h), the plain
// operator application and the nonlocal term of the latter.
#include "cocg_impl.h"

namespace rpa {

namespace {

template <typename T, int M, int PITCH>
__global__ void __launch_bounds__(kMaxBlock) k_happly(Geom g, StencilCoef<T> cf, const T* v,
                                                       const double* sr, const double* si,
                                                       const void* x, void* y) {
  extern __shared__ double smem_d[];
  typedef typename V2<T>::t T2;
  constexpr bool FULL = M == 0;
  constexpr int HS = M == 2 ? 2 : 1;
  const int vec = blockIdx.y;
  const size_t base = (size_t)vec * g.N;
  HPol<T> p;
  p.x = reinterpret_cast<const T2*>(x) + base;
  p.y = reinterpret_cast<T2*>(y) + base;
  p.v = v; p.c0 = cf.c0;
  p.sr = (T)sr[vec]; p.si = (T)si[vec];
  march<T, FULL, HS, PITCH>(g, cf, p, reinterpret_cast<T2*>(smem_d), blockIdx.x, blockIdx.x + 1);
}

// Nonlocal term of the plain operator application: per vector, the
// projections (one workgroup each, coefficients through LDS to coef), then
// y += V_nl x point by point.
template <typename T>
__global__ void __launch_bounds__(256) k_nl_coef(NlArgs nl, const void* x, long long N,
                                                  void* coef) {
  typedef typename V2<T>::t T2;
  extern __shared__ double smem_d[];
  T2* c = reinterpret_cast<T2*>(smem_d);
  const T2* xv = reinterpret_cast<const T2*>(x) + (size_t)blockIdx.x * N;
  double d0 = 0.0, d1 = 0.0;
  nl_project<T, T>(nl, xv, c, d0, d1);
  __syncthreads();
  T2* out = reinterpret_cast<T2*>(coef) + (size_t)blockIdx.x * nl.n_proj;
  for (int p = threadIdx.x; p < nl.n_proj; p += blockDim.x) out[p] = c[p];
}

template <typename T>
__global__ void __launch_bounds__(256) k_nl_add(NlArgs nl, long long N, const void* coef,
                                                 void* y) {
  typedef typename V2<T>::t T2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const T2* c = reinterpret_cast<const T2*>(coef) + (size_t)blockIdx.y * nl.n_proj;
  T2* yv = reinterpret_cast<T2*>(y) + (size_t)blockIdx.y * N;
  T2 o = yv[i];
  nl_point<T>(nl.pm_ptr, nl.pm_proj, nl_pick<T>(nl.pm_v32, nl.pm_v64), c, i, o.x, o.y);
  yv[i] = o;
}

}  // namespace

bool geom_supported(const Geom& g) { return g.nz + 2 * R <= 128; }

size_t cocg_shmem_bytes(const Geom& g, int block, bool fp32_refine, int n_proj) {
  return lds_plane_bytes(g, pitch_for(g), fp32_refine) + red_bytes(block) +
         (size_t)n_proj * sizeof(double2);
}

int cocg_blocks_per_cu(const Geom& g, int block, bool fp32_refine, int n_proj) {
  const size_t shmem = cocg_shmem_bytes(g, block, fp32_refine, n_proj);
  const int m = tile_mode(g, block);
  int nb = 0;
  const void* fn = n_proj > 0 ? cocg_nl_fn(fp32_refine, m, pitch_for(g), g.prec != 0)
                   : g.prec   ? cocg_pc_fn(fp32_refine, m, pitch_for(g))
                              : cocg_fn_t<0>(fp32_refine, m, pitch_for(g));
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, shmem);
  if (e != hipSuccess || nb < 1) return 1;
  return nb;
}

int cocg_prec_regs(const Geom& g, int block) { return prec_regs(g, block); }
int cocg_prec_regs_max() { return kPrecRegs; }

long long cocg_slot_bytes(const Geom& g, bool fp32_refine) {
  // r, q, p_old, p_new (+ the FP32 correction d); preconditioned: + z and a transform buffer
  const long long extra = g.prec ? 2 : 0;
  return fp32_refine ? (5LL + extra) * g.N * (long long)sizeof(float2)
                     : (4LL + extra) * g.N * (long long)sizeof(double2);
}

namespace {
template <typename T, int M, int P>
hipError_t launch_h(const Geom& g, const StencilCoef<T>& cf, const T* v, const double* sr,
                    const double* si, const void* x, void* y, dim3 grid, int block, size_t shmem,
                    hipStream_t s) {
  hipLaunchKernelGGL((k_happly<T, M, P>), grid, dim3(block), shmem, s, g, cf, v, sr, si, x, y);
  return hipGetLastError();
}
template <typename T, int M>
hipError_t launch_hm(const Geom& g, const StencilCoef<T>& cf, const T* v, const double* sr,
                     const double* si, const void* x, void* y, dim3 grid, int block,
                     size_t shmem, hipStream_t s) {
  return pitch_for(g) == 64 ? launch_h<T, M, 64>(g, cf, v, sr, si, x, y, grid, block, shmem, s)
                            : launch_h<T, M, 128>(g, cf, v, sr, si, x, y, grid, block, shmem, s);
}
template <typename T>
hipError_t launch_ht(const Geom& g, const StencilCoef<T>& cf, const T* v, const double* sr,
                     const double* si, const void* x, void* y, dim3 grid, int block,
                     size_t shmem, hipStream_t s) {
  const int m = tile_mode(g, block);
  if (m == 0) return launch_hm<T, 0>(g, cf, v, sr, si, x, y, grid, block, shmem, s);
  if (m == 1) return launch_hm<T, 1>(g, cf, v, sr, si, x, y, grid, block, shmem, s);
  return launch_hm<T, 2>(g, cf, v, sr, si, x, y, grid, block, shmem, s);
}
}  // namespace

hipError_t launch_cocg(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                       hipStream_t s) {
  if (a.nl.n_proj > 0) return launch_cocg_nl(a, fp32_refine, grid, block, shmem, s);
  if (a.prec) return launch_cocg_pc(a, fp32_refine, grid, block, shmem, s);
  return launch_cocg_t<0>(a, fp32_refine, grid, block, shmem, s);
}

hipError_t launch_happly(const Geom& g, const StencilCoef<double>& c64, const StencilCoef<float>& c32,
                         const double* v64, const float* v32, int nvec, const double* shift_re,
                         const double* shift_im, const void* x, void* y, bool fp32,
                         int block, hipStream_t s) {
  const size_t shmem = cocg_shmem_bytes(g, block, fp32, 0);
  dim3 grid(g.ntiles, nvec);
  if (fp32) return launch_ht<float>(g, c32, v32, shift_re, shift_im, x, y, grid, block, shmem, s);
  return launch_ht<double>(g, c64, v64, shift_re, shift_im, x, y, grid, block, shmem, s);
}

hipError_t launch_nl_apply(const NlArgs& nl, long long N, int nvec, const void* x, void* y,
                           void* coef, bool fp32, hipStream_t s) {
  if (nl.n_proj == 0) return hipSuccess;
  const size_t shmem = (size_t)nl.n_proj * (fp32 ? sizeof(float2) : sizeof(double2));
  const dim3 ga((unsigned)((N + 255) / 256), (unsigned)nvec);
  if (fp32) {
    hipLaunchKernelGGL((k_nl_coef<float>), dim3(nvec), dim3(256), shmem, s, nl, x, N, coef);
    hipLaunchKernelGGL((k_nl_add<float>), ga, dim3(256), 0, s, nl, N, (const void*)coef, y);
  } else {
    hipLaunchKernelGGL((k_nl_coef<double>), dim3(nvec), dim3(256), shmem, s, nl, x, N, coef);
    hipLaunchKernelGGL((k_nl_add<double>), ga, dim3(256), 0, s, nl, N, (const void*)coef, y);
  }
  return hipGetLastError();
}

}  // namespace rpa
