// Internal declarations shared by the engine and the kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "rpa.h"

namespace rpa {

constexpr int kRadius = 6;               // 12th-order central differences
constexpr int kMaxLanczos = 64;          // largest supported n_lanczos
constexpr int kMaxLanczosPublic = kMaxLanczos;
constexpr int kMaxBlock = 768;           // largest stencil/COCG workgroup
constexpr int kMaxProj = 4096;           // projectors (their coefficients live in LDS)
constexpr int kMaxGroup = 4;             // projectors sharing one support per group

// (H - eps_n - i omega) p = (c0 + V - eps_n) p - i omega p
//                          + sum_d s_d sum_k w[k] (p_{+k e_d} + p_{-k e_d}),
// w[k] the unit-spacing FD weights, s_d = -1/(2 h_d^2), c0 = -1/2 w_0 sum_d 1/h_d^2.
template <typename T>
struct StencilCoef {
  T c0;
  T w[kRadius + 1];
  T sx, sy, sz;
};

struct Geom {
  int nx, ny, nz;
  int ty;          // rows per tile
  int ntiles;      // ny / ty
  long long N;     // nx*ny*nz
  int prec;        // 1: the COCG solves are preconditioned (workspaces and LDS grow)
};

constexpr int kMaxPrecDim = 64;          // largest grid dimension of the in-kernel preconditioner

// Shifted kinetic preconditioner M = -1/2 Lap_h + sigma_n, sigma_n =
// max(vbar - eps_n, floor) - i omega, applied exactly through the per-axis
// eigenbasis of the periodic FD second derivative.  Per axis d the basis
// is stored zero-padded to P_d = (n_d rounded up to 16): v[d][i*P_d + a] =
// mode a at grid point i, vt[d] its transpose, k[d][a] = -1/2 lambda_d(a)
// (0 beyond n_d); FP32 and FP64 copies.
struct PrecArgs {
  const float* v32[3];
  const float* vt32[3];
  const float* k32[3];
  const double* v64[3];
  const double* vt64[3];
  const double* k64[3];
  double vbar;             // mean local potential (Ha)
  double floor;            // lower bound of the real part of sigma (Ha)
};

// Separable nonlocal projectors V_nl = h^3 sum_p gamma_p chi_p chi_p^T
// (Background section) in two layouts: by support ("groups" of up to
// kMaxGroup consecutive projectors with identical support, e.g. the angular
// channels of one atom) for the projections c_p = chi_p^T x, and by grid
// point for the sums (V_nl x)_i = sum_p (gamma_p h^3 c_p) chi_p(i).
// n_proj == 0: no nonlocal term (all pointers null).
struct NlArgs {
  int n_proj;
  int n_groups;
  const int4* ginfo;       // [n_groups] {first support entry, end, first projector, count}
  const int* gvoff;        // [n_groups] offset of the group's values, stored [count][S]
  const int* bidx;         // support grid indices of all groups
  const float* bv32;       // group values
  const double* bv64;
  const double* gdv;       // [n_proj] gamma_p * h^3
  const int* pm_ptr;       // [N + 1] entries of point i: pm_ptr[i] .. pm_ptr[i+1]-1
  const int* pm_proj;      // projector of each entry
  const float* pm_v32;     // chi_p(i) of each entry
  const double* pm_v64;
};

// Arguments of the persistent COCG launch.
struct CocgArgs {
  Geom g;
  int n_items;                 // Sternheimer systems in this launch
  int n_occ;
  const int* order;            // [n_items] system ids, processing order
  const double* eps;           // [n_occ]
  const double* omega;         // [B] frequency of each start vector
  const int* active;           // [B] 1 = start vector still running (nullable)
  const double* psi64;         // [n_occ][N]
  const double* u64;           // [B][N]  (nu^1/2 q for each start vector)
  double2* x64;                // [B*n_occ][N] initial guess in, solution out
  const double* v64;
  const float* v32;
  StencilCoef<double> c64;
  StencilCoef<float> c32;
  char* slot_ws;               // per-workgroup workspaces
  long long slot_bytes;        // bytes per workspace
  int* counter;                // work counter, zero before launch
  const int* n_items_dev;      // non-null: the item count is read from here (fallback launch)
  int* fail_list;              // non-null (FP32 launch): systems handed to the FP64 launch
  int* fail_count;             // their number, zero before launch
  int* out_iters;              // [n_items] by system id
  int* out_cycles;
  int* out_status;             // 0 ok, 1 noconv, 2 breakdown
  unsigned long long* stats;   // [6]: iters total, iters max, cycles, noconv, breakdown, fallbacks
  double tol;
  int maxit;
  int maxit32;                 // FP32 iterations before a solve is handed to FP64
  double inner_tol;            // FP32 inner relative reduction
  int max_cycles;
  NlArgs nl;
  // per-frequency iteration statistics (nullable): bin of each start vector,
  // and six planes of n_bins counters: solves, sum, sum of squares, min, max,
  // reliable updates
  const int* obin;
  unsigned long long* ostats;
  int n_bins;
  const PrecArgs* prec;        // device copy of the preconditioner tables; null: plain COCG
  int is_followup;             // the FP64 launch that continues systems the FP32 one handed over
};

// Rows of the stencil tile: `requested` if nonzero, else the whole (y, z)
// plane when it fits one workgroup, else the tallest divisor of ny (>= 6)
// whose tile fits.  Returns 0 when no requested or automatic choice is valid.
int pick_tile_y(int ny, int nz, int requested);

// Device bytes lanczos_energy_density allocates for batches of B start
// vectors and n_lanczos steps on the problem `p` (the workspaces of the
// Lanczos basis, nu^1/2, the Galerkin guess, the persistent COCG slots and
// the bookkeeping), using the launch shape the handle would pick.  With
// query_occupancy the resident workgroups per CU come from the HIP occupancy
// calculator (needs a device), else two per CU are assumed.
uint64_t lanczos_workspace_bytes(const rpa_setup_params& p, int B, int n_lanczos, int num_cu,
                                 bool query_occupancy);

// Launchers (return hipError_t of the launch).
hipError_t launch_cocg(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                       hipStream_t s);
// the kernels with the nonlocal term (separate translation unit)
hipError_t launch_cocg_nl(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                          hipStream_t s);
const void* cocg_nl_fn(bool fp32_refine, int tile_mode, int pitch, bool prec);
// the preconditioned kernels without a nonlocal term (separate translation unit)
hipError_t launch_cocg_pc(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                          hipStream_t s);
const void* cocg_pc_fn(bool fp32_refine, int tile_mode, int pitch);
size_t cocg_shmem_bytes(const Geom& g, int block, bool fp32_refine, int n_proj);
int cocg_blocks_per_cu(const Geom& g, int block, bool fp32_refine, int n_proj);
bool geom_supported(const Geom& g);   // nz + 12 <= 128 (padded LDS rows)
long long cocg_slot_bytes(const Geom& g, bool fp32_refine);
// registers per thread the preconditioner's prefetched planes need, and the most it has
int cocg_prec_regs(const Geom& g, int block);
int cocg_prec_regs_max();

hipError_t launch_happly(const Geom& g, const StencilCoef<double>& c64, const StencilCoef<float>& c32,
                         const double* v64, const float* v32, int nvec, const double* shift_re,
                         const double* shift_im, const void* x, void* y, bool fp32,
                         int block, hipStream_t s);
// y[v] += V_nl x[v] for nvec vectors of N points (complex, FP32 or FP64);
// coef: workspace of nvec * n_proj complex values of that precision.
hipError_t launch_nl_apply(const NlArgs& nl, long long N, int nvec, const void* x, void* y,
                           void* coef, bool fp32, hipStream_t s);

hipError_t launch_fill_d(double* p, double v, long long n, hipStream_t s);
hipError_t launch_fill_i(int* p, int v, long long n, hipStream_t s);
hipError_t launch_d2f(const double* a, float* b, long long n, hipStream_t s);
hipError_t launch_set_onehot(double* q, long long stride, const long long* idx, int B, hipStream_t s);

// out = M applied along `axis` of a batch of 3D arrays.
// in dims (B, d0, d1, d2); M is (n_out x n_in) row-major, n_in = d[axis];
// out dims equal in dims with d[axis] replaced by n_out.  trans: use M^T
// (then M is (n_in x n_out)).  scale (nullable) multiplies the output
// elementwise (length = output 3D size, broadcast over the batch).
hipError_t launch_kin_scale(double* a, const double* kin, const double* sig_re,
                            const double* sig_im, int B, long long N, hipStream_t s);
hipError_t launch_axis(const double* in, double* out, int B, int d0, int d1, int d2, int axis,
                       int n_out, const double* M, bool trans, const double* scale, hipStream_t s);

hipError_t launch_gram(const double* psi, const double* u, int B, int n_occ, int ng, long long N,
                       int n_chunks, double* part, hipStream_t s);
hipError_t launch_gram_finish(const double* part, int B, int n_occ, int ng, int n_chunks, double dV,
                              const double* eps, const double* omega, double2* G, hipStream_t s);
hipError_t launch_expand(const double* psi, const double2* G, int B, int n_occ, int ng, long long N,
                         double2* x64, hipStream_t s);
hipError_t launch_accumulate(const double* psi, const double2* x64, int B, int n_occ, long long N,
                             const int* active, double* racc, hipStream_t s);

// Q layout [m_total][B][N]
// Block Lanczos over groups of batch columns (block_lanczos.hip).  A vector
// set of a group: blocks blk0 .. blk0 + n_blk - 1 of the basis at `base`
// (layout [block][batch column][N]), columns c0 .. c0 + ncol - 1 of the
// group (ncol <= 0: up to the group's size), clipped to the group's size.
constexpr int kMaxLzBlock = 8;           // largest block size
constexpr int kBgramChunk = 4096;        // grid rows per partial dot product
struct BVSet {
  double* base;
  int blk0, n_blk, c0, ncol;
};
int bgram_chunks(long long N);
hipError_t launch_bgram(const BVSet& X, const BVSet& Y, int max_x, int B, long long N, int G,
                        const int* gcol, const int* gsz, const int* gact, int pmax, double* part,
                        double* C, hipStream_t s);
hipError_t launch_bcombine(const BVSet& X, const BVSet& Y, int B, long long N, int G, const int* gcol,
                           const int* gsz, const int* gact, int pmax, const double* C, hipStream_t s);
hipError_t launch_bstep_diag(int G, int k, int m, const int* gsz, const int* gact, int pmax, double* C,
                             double* Ablk, const double* Bblk, double* amax, int* gm, hipStream_t s);
hipError_t launch_bqr_acc(int G, int k, int m, int j, const int* gsz, const int* gact, int pmax,
                          const double* C, double* Bblk, hipStream_t s);
hipError_t launch_bqr_norm(int G, int k, int m, int j, const int* gcol, const int* gsz, int* gact,
                           int pmax, const double* C, double* Bblk, const double* amax, double brk,
                           double* scale, int* active, hipStream_t s);
hipError_t launch_bqr_scale(double* Q, const double* W, int B, long long N, int G, int k, int j,
                            const int* gcol, const int* gsz, const int* gact, const double* scale,
                            hipStream_t s);
hipError_t launch_block_quad(int G, int m, const int* gcol, const int* gsz, const int* gm,
                             const double* Ablk, const double* Bblk, const long long* pos, double* dout,
                             int* fail, hipStream_t s);

hipError_t launch_lanczos_step(int k, int m_total, int B, long long N, double* Q, double* v,
                               double* alpha, double* beta, int* mlen, int* active, double brk,
                               hipStream_t s);
hipError_t launch_tridiag_quad(int B, int m_total, const double* alpha, const double* beta,
                               const int* mlen, const long long* out_pos, double* d, int* fail,
                               hipStream_t s);

hipError_t launch_scatter(const double* src, const long long* pos, int n, double* dst, hipStream_t s);
hipError_t launch_weighted_sum(const double* dhat, const double* w, int n_omega, long long N,
                               double scale_fine, double* e_fine, double* partials, int nblocks,
                               hipStream_t s);

}  // namespace rpa
