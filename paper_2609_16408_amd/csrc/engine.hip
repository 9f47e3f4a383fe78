// Host engine behind the C ABI (include/rpa.h): resident problem data,
// workspaces, and the per-Lanczos-step launch sequence of Algorithm 1.
#include "rpa.h"
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

using namespace rpa;

namespace {

thread_local std::string g_err;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct rpa_ctx {
  int n[3];
  double L[3], h[3], dV;
  long long N;
  int nocc;
  int ngal;                          // Galerkin states: the occupied ones, then the extra ones
  int precision;
  double tol;
  int maxit;
  int maxit32;                       // FP32 iterations before the FP64 hand-over
  double lz_brk;                     // relative Lanczos breakdown threshold
  int batch;
  uint64_t budget;
  double inner_tol;                  // reliable-update factor of the plain FP32 solver
  double inner_tol_pc;               // ... and of the preconditioned one
  int slots_per_cu;
  int num_cu;

  // resident problem data
  double* v64 = nullptr;
  float* v32 = nullptr;
  double* psi64 = nullptr;
  double* eps_d = nullptr;
  std::vector<double> eps_h;
  double* Vax[3] = {nullptr, nullptr, nullptr};   // per-axis eigenbasis [grid][mode]
  double* s_half = nullptr;
  double* s_full = nullptr;
  StencilCoef<double> c64;
  StencilCoef<float> c32;
  Geom geom;
  int block = 0;
  NlArgs nl{};                       // nonlocal projectors (device layouts)
  PrecArgs prec{};                   // kinetic preconditioner tables (device addresses)
  void* prec_mem = nullptr;          // their allocation, ending with a device copy of `prec`
  const PrecArgs* prec_dev = nullptr;
  double pc_lo = 0.0, pc_hi = 0.0;   // frequency window of the preconditioned solves (0: open)
  std::vector<void*> nl_mem;         // their allocations
  DevBuf nlcoef;                     // coefficients for the plain operator application

  // workspaces
  DevBuf x64, slots, u64, racc, vtmp, tmpA, Q, alpha, beta, mlen, active, order, iters, cycles,
      status, counter, stats, omega_b, pos_b, idx_b, gpart, G, dhat, partials, interp_m, shifts, fail,
      faillist, obin, ostats;
  // block Lanczos: per group first column, size, active flag, block count,
  // max |A| entry, normalisation; the A_k and B_k blocks; contraction
  // coefficients and their partial sums
  DevBuf bgcol, bgsz, bgact, bgm, bamax, bscale, Ablk, Bblk, bC, bpart;
  // per-frequency iteration statistics of the current / last call
  int stat_bins = 0;                 // 0: not recorded
  std::vector<double> stat_omega;    // frequency of each bin
  std::vector<unsigned long long> stat_host;   // 6 planes of stat_bins counters
  int interp_kind = -1, interp_stride = -1;
  int interp_dims[3] = {0, 0, 0};
  size_t allocated = 0;
  bool broken = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  float last_ms = 0.f;
  int last_grid = 0;
  int use_graph = 0;
  bool capturing = false;
  int progress = 0;                  // print a line per Lanczos step (waits for it)
  long long progress_batch = 0;      // batches started in the current call
  double progress_t0 = 0.0;
  unsigned alloc_epoch = 0;          // bumped whenever a workspace is (re)allocated
  int warm_B = 0, warm_m = 0;        // largest batch run eagerly with the current buffers
  hipStream_t cap_stream = nullptr;  // non-default stream used for capture
  struct GraphEntry { hipGraph_t g; hipGraphExec_t e; unsigned epoch; };
  std::vector<std::pair<std::pair<int, int>, GraphEntry>> graphs;
  DevBuf dres;
  std::vector<int> order_h;
  int counts_h[2] = {0, 0};          // host staging of the two list lengths
  std::vector<hipEvent_t> evs;   // COCG launch timing events of the current call
  std::vector<int> ev_kind;      // per event pair: 0 plain FP32/FP64, 1 preconditioned, 2 FP64 follow-up
  int n_ev_used = 0;
  double cocg_ms_kind[3] = {0.0, 0.0, 0.0};
  void* scratch = nullptr;       // this device's allocation-free workspace array
  bool no_alloc = false;         // workspaces point into `scratch`: never (re)allocate
  double cocg_ms_total = 0.0;
  int cocg_launches = 0;
};

namespace {

rpa_status set_err(rpa_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define ARG_CHECK(cond, msg) \
  do {                       \
    if (!(cond)) return set_err(RPA_E_ARG, msg); \
  } while (0)

#define HIPCHK(h, expr)                                                              \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      if (h) (h)->broken = true;                                                     \
      return set_err(RPA_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                                \
  } while (0)

rpa_status ensure(rpa_ctx* h, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return RPA_OK;
  if (h->no_alloc) return set_err(RPA_E_OOM, "workspace outside the allocation-free scratch layout");
  if (h->capturing) return set_err(RPA_E_STATE, "allocation requested during graph capture");
  ++h->alloc_epoch;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) { h->broken = true; return set_err(RPA_E_HIP, "hipFree failed"); }
    h->allocated -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) return RPA_OK;
  if (h->budget && h->allocated + bytes > h->budget)
    return set_err(RPA_E_OOM, "workspace exceeds hbm_budget");
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return set_err(RPA_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  b.bytes = bytes;
  h->allocated += bytes;
  return RPA_OK;
}

#define ENSURE(h, buf, bytes)                       \
  do {                                              \
    rpa_status s_ = ensure((h), (buf), (bytes));    \
    if (s_ != RPA_OK) return s_;                    \
  } while (0)

template <typename T> T* P(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

// Fornberg's closed form of the order-2R central second-derivative weights.
void fd_weights(int R, double* w) {
  auto fact = [](int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; };
  double s = 0.0;
  for (int k = 1; k <= R; ++k) {
    const double sign = (k % 2 == 1) ? 1.0 : -1.0;
    w[k] = 2.0 * sign * fact(R) * fact(R) / ((double)k * k * fact(R - k) * fact(R + k));
    s += w[k];
  }
  w[0] = -2.0 * s;
}

// Real orthonormal eigenbasis of the periodic 1D FD second derivative
// (circulant => Fourier modes): V[i*n + j] = mode j at grid point i; lam[j].
void axis_basis(int n, double h, const double* w, int R, std::vector<double>& V,
                std::vector<double>& lam) {
  V.assign((size_t)n * n, 0.0);
  lam.assign(n, 0.0);
  auto symbol = [&](int k) {
    double s = w[0];
    for (int p = 1; p <= R; ++p) s += 2.0 * w[p] * std::cos(2.0 * M_PI * k * p / n);
    return s / (h * h);
  };
  int j = 0;
  for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = 1.0 / std::sqrt((double)n);
  lam[j++] = 0.0;
  for (int k = 1; 2 * k < n; ++k) {
    const double lk = symbol(k);
    for (int i = 0; i < n; ++i) {
      V[(size_t)i * n + j] = std::sqrt(2.0 / n) * std::cos(2.0 * M_PI * k * i / n);
      V[(size_t)i * n + j + 1] = std::sqrt(2.0 / n) * std::sin(2.0 * M_PI * k * i / n);
    }
    lam[j] = lk;
    lam[j + 1] = lk;
    j += 2;
  }
  if (n % 2 == 0) {
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = ((i % 2) ? -1.0 : 1.0) / std::sqrt((double)n);
    lam[j] = symbol(n / 2);
    ++j;
  }
}

// 1D periodic interpolation matrix (n_fine x n_coarse), row-major.
void interp_matrix(int kind, int nf, int g, std::vector<double>& M) {
  const int nc = nf / g;
  M.assign((size_t)nf * nc, 0.0);
  for (int i = 0; i < nf; ++i) {
    const int c = i / g;
    const double t = (double)(i % g) / g;
    if (kind == RPA_INTERP_TRILINEAR) {
      M[(size_t)i * nc + (c % nc)] += 1.0 - t;
      M[(size_t)i * nc + ((c + 1) % nc)] += t;
    } else if (kind == RPA_INTERP_TRICUBIC) {
      // cubic Lagrange through the nodes c-1, c, c+1, c+2 at offset t from c
      const double l0 = -t * (t - 1.0) * (t - 2.0) / 6.0;
      const double l1 = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
      const double l2 = -(t + 1.0) * t * (t - 2.0) / 2.0;
      const double l3 = (t + 1.0) * t * (t - 1.0) / 6.0;
      M[(size_t)i * nc + ((c - 1 + nc) % nc)] += l0;
      M[(size_t)i * nc + (c % nc)] += l1;
      M[(size_t)i * nc + ((c + 1) % nc)] += l2;
      M[(size_t)i * nc + ((c + 2) % nc)] += l3;
    } else {  // Fourier: band-limited trigonometric interpolant (Dirichlet kernel)
      for (int cc = 0; cc < nc; ++cc) {
        const double s = (double)i / nf - (double)cc / nc;
        double v = 1.0;
        const int kmax = (nc - 1) / 2;
        for (int k = 1; k <= kmax; ++k) v += 2.0 * std::cos(2.0 * M_PI * k * s);
        if (nc % 2 == 0) v += std::cos(M_PI * nc * s);
        M[(size_t)i * nc + cc] = v / nc;
      }
    }
  }
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Grid dimension padded to the 16-wide matrix-core tiles of the preconditioner.
int prec_pad_host(int n) { return (n + 15) & ~15; }

// Partial Gram sums per start vector (grid-point chunks of the contraction).
int gram_chunks(long long N) { return (int)std::min<long long>(64, std::max<long long>(1, N / 2048)); }

rpa_status usable(rpa_ctx* h) {
  if (!h) return set_err(RPA_E_ARG, "null handle");
  if (h->broken) return set_err(RPA_E_STATE, "handle unusable after an earlier HIP error");
  return RPA_OK;
}

rpa_status cocg_events(rpa_ctx* h, hipEvent_t* e0, hipEvent_t* e1, int kind = 0);
void drop_graphs(rpa_ctx* h);

// u[B][N] -> out[B][N] = nu^(power/2) u  (Kronecker form; tmp buffers internal)
rpa_status coulomb(rpa_ctx* h, int power, int B, const double* in, double* out, hipStream_t s) {
  const size_t bytes = (size_t)B * h->N * sizeof(double);
  ENSURE(h, h->tmpA, bytes);
  ENSURE(h, h->vtmp, bytes);
  double* a = P<double>(h->tmpA);
  double* b = P<double>(h->vtmp);
  const int* n = h->n;
  const double* sc = power == 1 ? h->s_half : h->s_full;
  // forward: modes = V^T along each axis
  HIPCHK(h, launch_axis(in, a, B, n[0], n[1], n[2], 0, n[0], h->Vax[0], true, nullptr, s));
  HIPCHK(h, launch_axis(a, b, B, n[0], n[1], n[2], 1, n[1], h->Vax[1], true, nullptr, s));
  HIPCHK(h, launch_axis(b, a, B, n[0], n[1], n[2], 2, n[2], h->Vax[2], true, sc, s));
  // inverse: V along each axis
  HIPCHK(h, launch_axis(a, b, B, n[0], n[1], n[2], 2, n[2], h->Vax[2], false, nullptr, s));
  HIPCHK(h, launch_axis(b, a, B, n[0], n[1], n[2], 1, n[1], h->Vax[1], false, nullptr, s));
  HIPCHK(h, launch_axis(a, out, B, n[0], n[1], n[2], 0, n[0], h->Vax[0], false, nullptr, s));
  return RPA_OK;
}

// Sternheimer batch: given u (B start vectors at per-vector omega, already in
// h->u64), solve all B*nocc systems and accumulate racc[B][N].
// Processing order of the B*N_s systems: smallest omega first, then the
// highest orbital (the longest solves start first).  Host-to-device copy.
// With a preconditioner frequency window the systems are split into two
// lists, each in that order: order[0, n) those solved without the
// preconditioner, order[n, 2n) those solved with it; their counts go to
// counter[4] and counter[5], where the two persistent launches read them.
bool prec_window(const rpa_ctx* h) { return h->prec_dev && (h->pc_lo > 0.0 || h->pc_hi > 0.0); }
bool in_window(const rpa_ctx* h, double w) {
  return w >= h->pc_lo && (h->pc_hi <= 0.0 || w <= h->pc_hi);
}

rpa_status upload_order_for(rpa_ctx* h, int B, const std::vector<double>& omega_host, hipStream_t s) {
  const int nocc = h->nocc;
  const int n_items = B * nocc;
  ENSURE(h, h->order, 2 * (size_t)n_items * sizeof(int));
  ENSURE(h, h->counter, sizeof(int) * 64);
  h->order_h.assign(2 * (size_t)n_items, 0);
  std::vector<int> all(n_items);
  std::iota(all.begin(), all.end(), 0);
  std::stable_sort(all.begin(), all.end(), [&](int a, int b) {
    const double wa = omega_host[a / nocc], wb = omega_host[b / nocc];
    if (wa != wb) return wa < wb;
    return (a % nocc) > (b % nocc);
  });
  if (!prec_window(h)) {
    std::copy(all.begin(), all.end(), h->order_h.begin());
    HIPCHK(h, hipMemcpyAsync(h->order.p, h->order_h.data(), n_items * sizeof(int), hipMemcpyHostToDevice, s));
    return RPA_OK;
  }
  int np = 0, nq = 0;
  for (int it : all) {
    if (in_window(h, omega_host[it / nocc])) h->order_h[n_items + nq++] = it;
    else h->order_h[np++] = it;
  }
  h->counts_h[0] = np;
  h->counts_h[1] = nq;
  HIPCHK(h, hipMemcpyAsync(h->order.p, h->order_h.data(), 2 * (size_t)n_items * sizeof(int),
                           hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(P<int>(h->counter) + 4, h->counts_h, 2 * sizeof(int), hipMemcpyHostToDevice, s));
  return RPA_OK;
}

rpa_status sternheimer_batch(rpa_ctx* h, int B, const std::vector<double>& omega_host,
                             const int* active_dev, hipStream_t s, bool upload_order = true,
                             bool timing = true) {
  rpa_status r_ = RPA_OK;
  const long long N = h->N;
  const int nocc = h->nocc;
  const bool refine = h->precision == RPA_FP32_REFINE;
  const int n_items = B * nocc;
  // Galerkin initial guess over the ngal states (occupied, then any extra
  // eigenpairs): the Gram contraction C = h^3 Psi_g^T diag(u) Psi runs on the
  // FP64 matrix cores (k_gram); the energy denominators (k_gram_finish) and
  // the expansion x0 = Psi_g G (k_expand) on vector FP64
  const int n_chunks = gram_chunks(N);
  const int ng = h->ngal;
  ENSURE(h, h->gpart, (size_t)B * n_chunks * ng * nocc * sizeof(double));
  ENSURE(h, h->G, (size_t)B * ng * nocc * sizeof(double2));
  ENSURE(h, h->x64, (size_t)n_items * N * sizeof(double2));
  HIPCHK(h, launch_gram(h->psi64, P<double>(h->u64), B, nocc, ng, N, n_chunks, P<double>(h->gpart), s));
  HIPCHK(h, launch_gram_finish(P<double>(h->gpart), B, nocc, ng, n_chunks, h->dV, h->eps_d,
                               P<double>(h->omega_b), P<double2>(h->G), s));
  HIPCHK(h, launch_expand(h->psi64, P<double2>(h->G), B, nocc, ng, N, P<double2>(h->x64), s));

  ENSURE(h, h->order, 2 * (size_t)n_items * sizeof(int));
  ENSURE(h, h->iters, (size_t)n_items * sizeof(int));
  ENSURE(h, h->cycles, (size_t)n_items * sizeof(int));
  ENSURE(h, h->status, (size_t)n_items * sizeof(int));
  ENSURE(h, h->counter, sizeof(int) * 64);
  if (upload_order) {
    r_ = upload_order_for(h, B, omega_host, s);
    if (r_ != RPA_OK) return r_;
  }
  // counter[0]: work queue of the launch; with FP32 refinement counter[1]
  // is the queue of the FP64 launch and counter[2] the number of systems
  // handed to it (listed in faillist)
  HIPCHK(h, launch_fill_i(P<int>(h->counter), 0, 4, s));
  if (refine) ENSURE(h, h->faillist, (size_t)n_items * sizeof(int));

  const int bpc = h->slots_per_cu > 0 ? h->slots_per_cu
                                      : cocg_blocks_per_cu(h->geom, h->block, refine, h->nl.n_proj);
  int grid = std::max(1, std::min(n_items, bpc * h->num_cu));
  const long long sb = cocg_slot_bytes(h->geom, refine);
  ENSURE(h, h->slots, (size_t)grid * sb);

  CocgArgs a;
  memset(&a, 0, sizeof(a));
  a.g = h->geom;
  a.n_items = n_items;
  a.n_occ = nocc;
  a.order = P<int>(h->order);
  a.eps = h->eps_d;
  a.omega = P<double>(h->omega_b);
  a.active = active_dev;
  a.psi64 = h->psi64;
  a.u64 = P<double>(h->u64);
  a.x64 = P<double2>(h->x64);
  a.v64 = h->v64;
  a.v32 = h->v32;
  a.c64 = h->c64;
  a.c32 = h->c32;
  a.slot_ws = P<char>(h->slots);
  a.slot_bytes = sb;
  a.counter = P<int>(h->counter);
  a.out_iters = P<int>(h->iters);
  a.out_cycles = P<int>(h->cycles);
  a.out_status = P<int>(h->status);
  a.stats = P<unsigned long long>(h->stats);
  a.tol = h->tol;
  a.maxit = h->maxit;
  a.maxit32 = h->maxit32;
  a.inner_tol = h->prec_dev ? h->inner_tol_pc : h->inner_tol;
  a.max_cycles = 0;
  a.nl = h->nl;
  a.n_items_dev = nullptr;
  a.fail_list = refine ? P<int>(h->faillist) : nullptr;
  a.fail_count = refine ? P<int>(h->counter) + 2 : nullptr;
  a.n_bins = h->stat_bins;
  a.obin = h->stat_bins > 0 ? P<int>(h->obin) : nullptr;
  a.ostats = h->stat_bins > 0 ? P<unsigned long long>(h->ostats) : nullptr;
  a.prec = h->prec_dev;
  const size_t shmem = cocg_shmem_bytes(h->geom, h->block, refine, h->nl.n_proj);
  // FP64 COCG for the systems the FP32 launch handed over (usually none; its
  // workgroups then exit at once), in the same slot memory
  CocgArgs f = a;
  f.order = P<int>(h->faillist);
  f.n_items_dev = P<int>(h->counter) + 2;
  f.counter = P<int>(h->counter) + 1;
  f.fail_list = nullptr;
  f.fail_count = nullptr;
  f.is_followup = 1;
  f.slot_bytes = cocg_slot_bytes(h->geom, false);
  const int grid64 = (int)std::max<long long>(1, std::min<long long>(grid, (long long)grid * sb / f.slot_bytes));
  const size_t shmem64 = cocg_shmem_bytes(h->geom, h->block, false, h->nl.n_proj);
  // one pair of timing events around each launch (kind: 0 plain, 1
  // preconditioned, 2 FP64 follow-up)
  auto timed = [&](int kind, auto&& launch) -> rpa_status {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing) {
      rpa_status es = cocg_events(h, &e0, &e1, kind);
      if (es != RPA_OK) return es;
      HIPCHK(h, hipEventRecord(e0, s));
    }
    HIPCHK(h, launch());
    if (timing) HIPCHK(h, hipEventRecord(e1, s));
    return RPA_OK;
  };
  rpa_status rl = RPA_OK;
  if (prec_window(h)) {
    // systems outside the frequency window: the plain kernels; inside: the
    // preconditioned ones (queues counter[0] and counter[3])
    CocgArgs ap = a;
    ap.prec = nullptr;
    ap.inner_tol = h->inner_tol;
    ap.g.prec = 0;
    ap.n_items_dev = P<int>(h->counter) + 4;
    Geom gp = h->geom;
    gp.prec = 0;
    const size_t shmem_p = cocg_shmem_bytes(gp, h->block, refine, h->nl.n_proj);
    rl = timed(0, [&] { return launch_cocg(ap, refine, grid, h->block, shmem_p, s); });
    if (rl != RPA_OK) return rl;
    CocgArgs aq = a;
    aq.order = P<int>(h->order) + n_items;
    aq.n_items_dev = P<int>(h->counter) + 5;
    aq.counter = P<int>(h->counter) + 3;
    rl = timed(1, [&] { return launch_cocg(aq, refine, grid, h->block, shmem, s); });
  } else {
    rl = timed(h->prec_dev ? 1 : 0, [&] { return launch_cocg(a, refine, grid, h->block, shmem, s); });
  }
  if (rl != RPA_OK) return rl;
  if (refine) {
    rl = timed(2, [&] { return launch_cocg(f, false, grid64, h->block, shmem64, s); });
    if (rl != RPA_OK) return rl;
  }
  h->last_grid = grid;

  ENSURE(h, h->racc, (size_t)B * N * sizeof(double));
  HIPCHK(h, launch_accumulate(h->psi64, P<double2>(h->x64), B, nocc, N, active_dev,
                              P<double>(h->racc), s));
  return RPA_OK;
}

// A pair of timing events for the next COCG launch of this call; `kind`
// tells which launch it times (see rpa_last_cocg_split).
rpa_status cocg_events(rpa_ctx* h, hipEvent_t* e0, hipEvent_t* e1, int kind) {
  while ((int)h->evs.size() < 2 * (h->n_ev_used + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) { h->broken = true; return set_err(RPA_E_HIP, "hipEventCreate failed"); }
    h->evs.push_back(e);
  }
  if ((int)h->ev_kind.size() < h->n_ev_used + 1) h->ev_kind.resize(h->n_ev_used + 1);
  h->ev_kind[h->n_ev_used] = kind;
  *e0 = h->evs[2 * h->n_ev_used];
  *e1 = h->evs[2 * h->n_ev_used + 1];
  ++h->n_ev_used;
  return RPA_OK;
}

// Zero the call's counters.  omegas: the distinct frequencies of the call,
// one statistics bin each (empty: no per-frequency statistics); B: start
// vectors per batch (entries of the bin map).
rpa_status begin_stats(rpa_ctx* h, hipStream_t s, const std::vector<double>& omegas, int B) {
  ENSURE(h, h->stats, 8 * sizeof(unsigned long long));
  ENSURE(h, h->fail, 4 * sizeof(int));
  // fill kernels rather than memset nodes, so the sequence stays capturable
  HIPCHK(h, launch_fill_d(P<double>(h->stats), 0.0, 8, s));
  HIPCHK(h, launch_fill_i(P<int>(h->fail), 0, 4, s));
  h->n_ev_used = 0;
  h->stat_bins = (int)omegas.size();
  h->stat_omega = omegas;
  h->stat_host.clear();
  if (h->stat_bins > 0) {
    // sized for at least 64 bins so that calls with few frequencies reuse it
    const int nb = std::max(64, h->stat_bins);
    ENSURE(h, h->ostats, 6 * (size_t)nb * sizeof(unsigned long long));
    ENSURE(h, h->obin, (size_t)std::max(64, B) * sizeof(int));
    const int b = h->stat_bins;
    unsigned long long* o = P<unsigned long long>(h->ostats);
    HIPCHK(h, launch_fill_i(reinterpret_cast<int*>(o), 0, 2LL * 6 * b, s));
    HIPCHK(h, launch_fill_i(reinterpret_cast<int*>(o + 3 * b), -1, 2LL * b, s));   // min: all ones
  }
  return RPA_OK;
}

rpa_status end_stats(rpa_ctx* h, hipStream_t s, rpa_stats* st, double t0, long long n_systems,
                     int extra_breakdowns) {
  unsigned long long dv[8];
  int fl[4];
  HIPCHK(h, hipMemcpyAsync(dv, h->stats.p, sizeof(dv), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(fl, h->fail.p, sizeof(fl), hipMemcpyDeviceToHost, s));
  if (h->stat_bins > 0) {
    h->stat_host.assign(6 * (size_t)h->stat_bins, 0ULL);
    HIPCHK(h, hipMemcpyAsync(h->stat_host.data(), h->ostats.p,
                             h->stat_host.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(h, hipStreamSynchronize(s));
  double tot = 0.0;
  for (int k = 0; k < 3; ++k) h->cocg_ms_kind[k] = 0.0;
  int n_fp32 = 0;
  for (int i = 0; i < h->n_ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->evs[2 * i], h->evs[2 * i + 1]) == hipSuccess) {
      tot += ms;
      h->cocg_ms_kind[h->ev_kind[i]] += ms;
    } else {
      (void)hipGetLastError();
    }
    if (h->ev_kind[i] != 2) ++n_fp32;
  }
  h->cocg_ms_total = tot;
  // launches counted as Sternheimer steps: the FP64 follow-up and, with a
  // preconditioner window, the second FP32 launch belong to their step
  h->cocg_launches = prec_window(h) ? n_fp32 / 2 : n_fp32;
  extra_breakdowns += fl[0] + fl[1];
  if (st) {
    st->n_systems = n_systems;
    st->cocg_iters_total = (int64_t)dv[0];
    st->cocg_iters_max = (int64_t)dv[1];
    st->refine_cycles = (int64_t)dv[2];
    st->n_noconv = (int64_t)dv[3];
    st->n_breakdown = (int64_t)dv[4] + extra_breakdowns;
    st->seconds = now_s() - t0;
    st->n_fp64_fallback = (int64_t)dv[5];
  }
  if (dv[3] > 0) return set_err(RPA_W_NOCONV, "some Sternheimer solves did not converge");
  if (dv[4] > 0 || extra_breakdowns > 0) return set_err(RPA_W_BREAKDOWN, "breakdown occurred");
  return RPA_OK;
}

rpa_status interp_setup(rpa_ctx* h, int kind, int g, hipStream_t s) {
  if (h->interp_kind == kind && h->interp_stride == g) return RPA_OK;
  std::vector<double> all;
  size_t off[3];
  for (int d = 0; d < 3; ++d) {
    std::vector<double> M;
    interp_matrix(kind, h->n[d], g, M);
    off[d] = all.size();
    all.insert(all.end(), M.begin(), M.end());
  }
  ENSURE(h, h->interp_m, all.size() * sizeof(double));
  HIPCHK(h, hipMemcpyAsync(h->interp_m.p, all.data(), all.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  for (int d = 0; d < 3; ++d) h->interp_dims[d] = (int)off[d];
  h->interp_kind = kind;
  h->interp_stride = g;
  return RPA_OK;
}

rpa_status do_interpolate(rpa_ctx* h, int kind, int g, int nf, const double* coarse, double* fine,
                          hipStream_t s) {
  const int* n = h->n;
  const long long Nc = h->N / ((long long)g * g * g);
  if (g == 1) {
    HIPCHK(h, hipMemcpyAsync(fine, coarse, (size_t)nf * h->N * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    return RPA_OK;
  }
  rpa_status st = interp_setup(h, kind, g, s);
  if (st != RPA_OK) return st;
  const int nc[3] = {n[0] / g, n[1] / g, n[2] / g};
  ENSURE(h, h->tmpA, (size_t)nf * n[0] * nc[1] * nc[2] * sizeof(double));
  ENSURE(h, h->vtmp, (size_t)nf * n[0] * n[1] * nc[2] * sizeof(double));
  const double* M = P<double>(h->interp_m);
  HIPCHK(h, launch_axis(coarse, P<double>(h->tmpA), nf, nc[0], nc[1], nc[2], 0, n[0],
                        M + h->interp_dims[0], false, nullptr, s));
  HIPCHK(h, launch_axis(P<double>(h->tmpA), P<double>(h->vtmp), nf, n[0], nc[1], nc[2], 1, n[1],
                        M + h->interp_dims[1], false, nullptr, s));
  HIPCHK(h, launch_axis(P<double>(h->vtmp), fine, nf, n[0], n[1], nc[2], 2, n[2],
                        M + h->interp_dims[2], false, nullptr, s));
  (void)Nc;
  return RPA_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char* rpa_last_error(rpa_handle) { return g_err.c_str(); }

rpa_status rpa_frequency_rule(int32_t n_omega, double* omega, double* weight) {
  ARG_CHECK(n_omega >= 1 && n_omega <= 512, "n_omega must be in [1, 512]");
  ARG_CHECK(omega && weight, "null output");
  // Gauss-Legendre nodes by Newton iteration on P_n from Chebyshev-like starts
  const int n = n_omega;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1.0; }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = x; p0 = 1.0; }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    const double W = 2.0 / ((1.0 - x * x) * dp * dp);
    // ascending x order
    const int j = n - 1 - i;
    omega[j] = (1.0 + x) / (1.0 - x);
    weight[j] = W * 2.0 / ((1.0 - x) * (1.0 - x));
  }
  return RPA_OK;
}

}  // extern "C"
namespace {

// Host form of the two projector layouts (see NlArgs): groups of up to
// kMaxGroup consecutive projectors with identical support lists, and the
// point-major list of (projector, value) entries, both in input order.
struct NlHost {
  std::vector<int4> ginfo;
  std::vector<int> gvoff, bidx, pm_ptr, pm_proj;
  std::vector<float> bv32, pm_v32;
  std::vector<double> bv64, pm_v64, gdv;
};

std::string nl_build(const rpa_setup_params* p, long long N, double dV, NlHost& o) {
  const int np = p->n_proj;
  if (np == 0) return "";
  if (np < 0 || np > kMaxProj) return "n_proj must be in [0, 4096]";
  if (!p->proj_ptr || !p->proj_idx || !p->proj_val || !p->proj_gamma)
    return "proj_ptr, proj_idx, proj_val and proj_gamma are required when n_proj > 0";
  const int64_t* ptr = p->proj_ptr;
  if (ptr[0] != 0) return "proj_ptr[0] must be 0";
  for (int q = 0; q < np; ++q)
    if (ptr[q + 1] < ptr[q]) return "proj_ptr must be non-decreasing";
  const int64_t nnz = ptr[np];
  if (nnz > (int64_t)0x3fffffff) return "too many projector entries";
  for (int64_t e = 0; e < nnz; ++e) {
    if (p->proj_idx[e] < 0 || p->proj_idx[e] >= N) return "proj_idx out of range";
    if (!std::isfinite(p->proj_val[e])) return "proj_val must be finite";
  }
  for (int q = 0; q < np; ++q)
    if (!std::isfinite(p->proj_gamma[q])) return "proj_gamma must be finite";
  for (int q = 0; q < np;) {
    const int64_t a0 = ptr[q], S = ptr[q + 1] - a0;
    int cnt = 1;
    while (cnt < kMaxGroup && q + cnt < np) {
      const int64_t b0 = ptr[q + cnt];
      if (ptr[q + cnt + 1] - b0 != S ||
          !std::equal(p->proj_idx + a0, p->proj_idx + a0 + S, p->proj_idx + b0))
        break;
      ++cnt;
    }
    o.ginfo.push_back(make_int4((int)o.bidx.size(), (int)(o.bidx.size() + S), q, cnt));
    o.gvoff.push_back((int)o.bv64.size());
    for (int64_t j = 0; j < S; ++j) o.bidx.push_back((int)p->proj_idx[a0 + j]);
    for (int k = 0; k < cnt; ++k)
      for (int64_t j = 0; j < S; ++j) {
        const double v = p->proj_val[ptr[q + k] + j];
        o.bv64.push_back(v);
        o.bv32.push_back((float)v);
      }
    q += cnt;
  }
  o.pm_ptr.assign((size_t)N + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) ++o.pm_ptr[(size_t)p->proj_idx[e] + 1];
  for (long long i = 0; i < N; ++i) o.pm_ptr[i + 1] += o.pm_ptr[i];
  std::vector<int> fill(o.pm_ptr.begin(), o.pm_ptr.end() - 1);
  o.pm_proj.resize(nnz);
  o.pm_v64.resize(nnz);
  o.pm_v32.resize(nnz);
  for (int q = 0; q < np; ++q)
    for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) {
      const int at = fill[p->proj_idx[e]]++;
      o.pm_proj[at] = q;
      o.pm_v64[at] = p->proj_val[e];
      o.pm_v32[at] = (float)p->proj_val[e];
    }
  o.gdv.resize(np);
  for (int q = 0; q < np; ++q) o.gdv[q] = p->proj_gamma[q] * dV;
  return "";
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the allocation-free chi0 application: one array per GPU (every
// GPU the library runs on holds it until the process ends).  Host code never
// passes the array's name to a kernel: it is a host-side stand-in, not a
// device address.  The device address comes from hipGetSymbolAddress, once
// per device with that device current, and is used everywhere else.
constexpr size_t kScratchBytes = 128ull << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (nullptr and an error
// message when it cannot be had).
void* scratch_on_current_device(std::string* err) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    *err = "no current HIP device for the scratch array";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      *err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

namespace rpa {

int pick_tile_y(int ny, int nz, int requested) {
  if (requested != 0) return requested;
  if ((long long)ny * nz <= kMaxBlock) return ny;
  for (int t = ny; t >= kRadius; --t)
    if (ny % t == 0 && t * nz <= kMaxBlock) return t;
  return 0;
}

uint64_t lanczos_workspace_bytes(const rpa_setup_params& p, int B, int n_lanczos, int num_cu,
                                 bool query_occupancy) {
  const uint64_t N = (uint64_t)p.n[0] * p.n[1] * p.n[2];
  const uint64_t b = (uint64_t)std::max(1, B), m = (uint64_t)std::max(1, n_lanczos);
  const uint64_t nocc = (uint64_t)std::max(1, p.n_occ);
  const uint64_t items = b * nocc;
  const bool refine = p.precision == RPA_FP32_REFINE;
  // Lanczos basis, start/iteration vectors, recurrence scalars and bookkeeping
  uint64_t bytes = m * b * N * 8 + b * N * 8 + 2 * b * m * 8 + 2 * b * 4 + 4 * b * 8 + 64 + 16;
  bytes += 2 * b * N * 8;                                   // nu^1/2 transform buffers
  const uint64_t ngal = nocc + (uint64_t)std::max(0, p.n_extra);
  bytes += b * (uint64_t)gram_chunks((long long)N) * ngal * nocc * 8 + b * ngal * nocc * 16;
  bytes += items * N * 16;                                  // Sternheimer solutions (FP64)
  bytes += items * 4 * (refine ? 6 : 5) + 64 * 4;           // two order lists, counts, status, hand-over list
  bytes += b * N * 8;                                       // accumulated density response
  Geom g;
  g.nx = p.n[0]; g.ny = p.n[1]; g.nz = p.n[2];
  g.ty = pick_tile_y(p.n[1], p.n[2], p.tile_y);
  if (g.ty <= 0) g.ty = p.n[1];
  g.ntiles = p.n[1] / g.ty;
  g.N = (long long)N;
  g.prec = p.precond != 0;
  const int block = ((g.ty * g.nz + 63) / 64) * 64;
  int bpc = p.slots_per_cu > 0 ? p.slots_per_cu : 2;
  if (p.slots_per_cu <= 0 && query_occupancy)
    bpc = cocg_blocks_per_cu(g, block, refine, std::max(0, p.n_proj));
  const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(items, (uint64_t)bpc * num_cu));
  bytes += grid * (uint64_t)cocg_slot_bytes(g, refine);
  return bytes;
}

}  // namespace rpa

extern "C" {

rpa_status rpa_setup(const rpa_setup_params* p, void* stream, rpa_handle* out) {
  ARG_CHECK(p && out, "null params or output");
  *out = nullptr;
  for (int d = 0; d < 3; ++d) {
    ARG_CHECK(p->n[d] >= 7 && p->n[d] <= 4096, "each n[d] must be in [7, 4096]");
    ARG_CHECK(p->L[d] > 0 && std::isfinite(p->L[d]), "L must be positive and finite");
  }
  ARG_CHECK(p->fd_radius == kRadius, "fd_radius must be 6 (12th-order FD)");
  const long long N = (long long)p->n[0] * p->n[1] * p->n[2];
  ARG_CHECK(p->n_occ >= 1 && p->n_occ < N, "n_occ must be in [1, N_d)");
  ARG_CHECK(p->n_extra >= 0 && p->n_extra <= 1024 && (long long)p->n_occ + p->n_extra < N,
            "n_extra must be in [0, 1024] with n_occ + n_extra < N_d");
  ARG_CHECK(p->n_extra == 0 || (p->psi_extra && p->eps_extra), "psi_extra and eps_extra are required with n_extra > 0");
  for (int i = 0; i < p->n_extra; ++i) ARG_CHECK(std::isfinite(p->eps_extra[i]), "eps_extra must be finite");
  ARG_CHECK(p->v_loc && p->psi && p->eps, "v_loc, psi and eps are required");
  ARG_CHECK(p->precision == RPA_FP64 || p->precision == RPA_FP32_REFINE, "bad precision");
  ARG_CHECK(p->stern_tol > 0 && p->stern_tol < 1, "stern_tol must be in (0, 1)");
  ARG_CHECK(p->stern_maxit > 0, "stern_maxit must be positive");
  ARG_CHECK(p->batch >= 0, "batch must be >= 0");
  for (int i = 0; i < p->n_occ; ++i) ARG_CHECK(std::isfinite(p->eps[i]), "eps must be finite");
  ARG_CHECK(p->inner_tol >= 0 && p->inner_tol < 1, "inner_tol must be in [0, 1)");
  ARG_CHECK(p->fp32_maxit >= 0, "fp32_maxit must be >= 0");
  ARG_CHECK(p->lanczos_breakdown >= 0 && p->lanczos_breakdown < 1,
            "lanczos_breakdown must be in [0, 1)");
  ARG_CHECK(p->precond == 0 || p->precond == 1, "precond must be 0 or 1");
  ARG_CHECK(p->precond_omega_min >= 0 && p->precond_omega_max >= 0 &&
                (p->precond_omega_max == 0 || p->precond_omega_max >= p->precond_omega_min),
            "bad preconditioner frequency window");
  ARG_CHECK(p->precond == 0 || (p->n[0] <= kMaxPrecDim && p->n[1] <= kMaxPrecDim &&
                                p->n[2] <= kMaxPrecDim),
            "the Sternheimer preconditioner needs every n[d] <= 64");
  // tile rows
  const int ny = p->n[1], nz = p->n[2];
  const int ty = pick_tile_y(ny, nz, p->tile_y);
  ARG_CHECK(ty > 0 && ny % ty == 0 && ((ty * nz + 63) / 64) * 64 <= kMaxBlock,
            "no valid tile_y (ty | ny, ty*nz <= 768)");
  ARG_CHECK(ty == ny || ty >= kRadius, "tile_y must be >= 6 unless it covers the plane");
  {
    Geom gq;
    gq.nx = p->n[0]; gq.ny = ny; gq.nz = nz; gq.ty = ty; gq.ntiles = ny / ty; gq.N = N;
    gq.prec = p->precond != 0;
    ARG_CHECK(geom_supported(gq), "n[2] must be <= 116");
    const int blk = ((ty * nz + 63) / 64) * 64;
    ARG_CHECK(!gq.prec || cocg_prec_regs(gq, blk) <= cocg_prec_regs_max(),
              "the Sternheimer preconditioner needs larger stencil tiles for this grid");
    // FP32 refinement also runs the FP64 kernel (for the systems it hands over)
    ARG_CHECK(p->n_proj < 0 ||
              (cocg_shmem_bytes(gq, blk, p->precision == RPA_FP32_REFINE, p->n_proj) <= 160 * 1024 &&
               cocg_shmem_bytes(gq, blk, false, p->n_proj) <= 160 * 1024),
              "projector coefficients and stencil planes exceed the 160 KiB of LDS");
  }
  NlHost nlh;
  {
    double dV = 1.0;
    for (int d = 0; d < 3; ++d) dV *= p->L[d] / p->n[d];
    const std::string nerr = nl_build(p, N, dV, nlh);
    ARG_CHECK(nerr.empty(), nerr);
  }

  rpa_ctx* h = new rpa_ctx();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int d = 0; d < 3; ++d) {
    h->n[d] = p->n[d];
    h->L[d] = p->L[d];
    h->h[d] = p->L[d] / p->n[d];
  }
  h->dV = h->h[0] * h->h[1] * h->h[2];
  h->N = N;
  h->nocc = p->n_occ;
  h->ngal = p->n_occ + p->n_extra;
  h->precision = p->precision;
  h->tol = p->stern_tol;
  h->maxit = p->stern_maxit;
  h->maxit32 = p->fp32_maxit > 0 ? p->fp32_maxit : p->stern_maxit;
  h->pc_lo = p->precond_omega_min;
  h->pc_hi = p->precond_omega_max;
  h->lz_brk = p->lanczos_breakdown > 0 ? p->lanczos_breakdown : 1e-13;
  h->progress = p->progress;
  h->batch = p->batch;
  h->budget = p->hbm_budget;
  // reliable-update factor of the FP32 COCG (residual replaced by the FP64
  // residual each time the recursive one dropped by this factor).  On the
  // Si64 workload 0.01 needs 3.0 updates and 98.3 iterations per solve
  // against 5.6 and 97.1 at 0.1, and each update costs about five FP32
  // iterations of time (fold plus FP64 residual sweep): 5% faster overall.
  // defaults measured on the Si64-like workload: the preconditioned solves,
  // a few dozen iterations each, gain from fewer updates (0.001: 2.3 instead
  // of 2.9 per solve, 3% less kernel time than 0.01); so do the plain ones
  // after the widened Galerkin guess (5% less), and the long plain solves of
  // the occupied-only guess take the same time at 0.001 and 0.01
  h->inner_tol = p->inner_tol > 0 ? p->inner_tol : 0.001;
  h->inner_tol_pc = p->inner_tol > 0 ? p->inner_tol : 0.001;
  h->slots_per_cu = p->slots_per_cu;
  h->use_graph = p->use_graph;
  h->geom.nx = p->n[0];
  h->geom.ny = ny;
  h->geom.nz = nz;
  h->geom.ty = ty;
  h->geom.ntiles = ny / ty;
  h->geom.N = N;
  h->geom.prec = p->precond != 0;
  h->block = ((ty * nz + 63) / 64) * 64;
  int dev = 0;
  auto fail = [&](rpa_status st) { rpa_destroy(h); return st; };
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    g_err = "no HIP device";
    return fail(RPA_E_HIP);
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return fail(set_err(RPA_E_HIP, "hipEventCreate failed"));

  // FD coefficients
  double w[kRadius + 1];
  fd_weights(kRadius, w);
  double inv2 = 0.0;
  for (int d = 0; d < 3; ++d) inv2 += 1.0 / (h->h[d] * h->h[d]);
  h->c64.c0 = -0.5 * w[0] * inv2;
  h->c32.c0 = (float)h->c64.c0;
  for (int k = 0; k <= kRadius; ++k) {
    h->c64.w[k] = w[k];
    h->c32.w[k] = (float)w[k];
  }
  h->c64.sx = -0.5 / (h->h[0] * h->h[0]);
  h->c64.sy = -0.5 / (h->h[1] * h->h[1]);
  h->c64.sz = -0.5 / (h->h[2] * h->h[2]);
  h->c32.sx = (float)h->c64.sx;
  h->c32.sy = (float)h->c64.sy;
  h->c32.sz = (float)h->c64.sz;

  // resident copies
  DevBuf b;
  auto alloc = [&](void** ptr, size_t bytes) -> bool {
    if (h->budget && h->allocated + bytes > h->budget) { g_err = "setup exceeds hbm_budget"; return false; }
    if (hipMalloc(ptr, bytes) != hipSuccess) { (void)hipGetLastError(); g_err = "hipMalloc failed in setup"; return false; }
    h->allocated += bytes;
    return true;
  };
  if (!alloc((void**)&h->v64, N * sizeof(double)) || !alloc((void**)&h->v32, N * sizeof(float)) ||
      !alloc((void**)&h->psi64, (size_t)h->ngal * N * sizeof(double)) ||
      !alloc((void**)&h->eps_d, h->ngal * sizeof(double)) ||
      !alloc((void**)&h->s_half, N * sizeof(double)) || !alloc((void**)&h->s_full, N * sizeof(double)))
    return fail(RPA_E_OOM);
  for (int d = 0; d < 3; ++d)
    if (!alloc((void**)&h->Vax[d], (size_t)h->n[d] * h->n[d] * sizeof(double))) return fail(RPA_E_OOM);
  h->eps_h.assign(p->eps, p->eps + h->nocc);

  // nonlocal projector layouts
  struct Upload { void* dst; const void* src; size_t bytes; };
  std::vector<Upload> nl_up;
  if (p->n_proj > 0) {
    auto up = [&](auto& dst, const auto& v) -> bool {
      using E = typename std::decay_t<decltype(v)>::value_type;
      void* d = nullptr;
      if (!alloc(&d, std::max<size_t>(1, v.size()) * sizeof(E))) return false;
      h->nl_mem.push_back(d);
      dst = reinterpret_cast<std::decay_t<decltype(dst)>>(d);
      nl_up.push_back({d, v.data(), v.size() * sizeof(E)});
      return true;
    };
    h->nl.n_proj = p->n_proj;
    h->nl.n_groups = (int)nlh.ginfo.size();
    if (!up(h->nl.ginfo, nlh.ginfo) || !up(h->nl.gvoff, nlh.gvoff) || !up(h->nl.bidx, nlh.bidx) ||
        !up(h->nl.bv32, nlh.bv32) || !up(h->nl.bv64, nlh.bv64) || !up(h->nl.gdv, nlh.gdv) ||
        !up(h->nl.pm_ptr, nlh.pm_ptr) || !up(h->nl.pm_proj, nlh.pm_proj) ||
        !up(h->nl.pm_v32, nlh.pm_v32) || !up(h->nl.pm_v64, nlh.pm_v64))
      return fail(RPA_E_OOM);
  }

  std::vector<double> V[3], lam[3];
  for (int d = 0; d < 3; ++d) axis_basis(h->n[d], h->h[d], w, kRadius, V[d], lam[d]);
  // kinetic preconditioner: per axis the zero-padded basis, its transpose
  // and -1/2 lambda, in FP32 and FP64, in one allocation
  std::vector<char> prec_host;
  size_t prec_off[3][6] = {};
  if (p->precond) {
    auto put = [&](size_t bytes) {
      const size_t o = prec_host.size();
      prec_host.resize(o + ((bytes + 255) & ~(size_t)255), 0);
      return o;
    };
    for (int d = 0; d < 3; ++d) {
      const int n = h->n[d], Pd = prec_pad_host(n);
      const size_t P2 = (size_t)Pd * Pd;
      prec_off[d][0] = put(P2 * 4); prec_off[d][1] = put(P2 * 4); prec_off[d][2] = put((size_t)Pd * 4);
      prec_off[d][3] = put(P2 * 8); prec_off[d][4] = put(P2 * 8); prec_off[d][5] = put((size_t)Pd * 8);
    }
    const size_t args_off = put(sizeof(PrecArgs));
    for (int d = 0; d < 3; ++d) {
      const int n = h->n[d], Pd = prec_pad_host(n);
      float* v32 = reinterpret_cast<float*>(prec_host.data() + prec_off[d][0]);
      float* t32 = reinterpret_cast<float*>(prec_host.data() + prec_off[d][1]);
      float* k32 = reinterpret_cast<float*>(prec_host.data() + prec_off[d][2]);
      double* v64 = reinterpret_cast<double*>(prec_host.data() + prec_off[d][3]);
      double* t64 = reinterpret_cast<double*>(prec_host.data() + prec_off[d][4]);
      double* k64 = reinterpret_cast<double*>(prec_host.data() + prec_off[d][5]);
      for (int i = 0; i < n; ++i)
        for (int a = 0; a < n; ++a) {
          const double x = V[d][(size_t)i * n + a];
          v64[(size_t)i * Pd + a] = x;
          t64[(size_t)a * Pd + i] = x;
          v32[(size_t)i * Pd + a] = (float)x;
          t32[(size_t)a * Pd + i] = (float)x;
        }
      for (int a = 0; a < n; ++a) {
        k64[a] = -0.5 * lam[d][a];
        k32[a] = (float)k64[a];
      }
    }
    if (!alloc(&h->prec_mem, prec_host.size())) return fail(RPA_E_OOM);
    char* base = static_cast<char*>(h->prec_mem);
    for (int d = 0; d < 3; ++d) {
      h->prec.v32[d] = reinterpret_cast<const float*>(base + prec_off[d][0]);
      h->prec.vt32[d] = reinterpret_cast<const float*>(base + prec_off[d][1]);
      h->prec.k32[d] = reinterpret_cast<const float*>(base + prec_off[d][2]);
      h->prec.v64[d] = reinterpret_cast<const double*>(base + prec_off[d][3]);
      h->prec.vt64[d] = reinterpret_cast<const double*>(base + prec_off[d][4]);
      h->prec.k64[d] = reinterpret_cast<const double*>(base + prec_off[d][5]);
    }
    // mean local potential (the real shift of sigma_n)
    std::vector<double> vh((size_t)N);
    if (hipMemcpy(vh.data(), p->v_loc, (size_t)N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      g_err = "reading v_loc failed";
      return fail(RPA_E_HIP);
    }
    double sum = 0.0;
    for (double x : vh) sum += x;
    h->prec.vbar = sum / (double)N;
    h->prec.floor = 0.25;
    memcpy(prec_host.data() + args_off, &h->prec, sizeof(PrecArgs));
    h->prec_dev = reinterpret_cast<const PrecArgs*>(base + args_off);
  }
  std::vector<double> sh((size_t)N), sf((size_t)N);
  for (int i = 0; i < h->n[0]; ++i)
    for (int j = 0; j < h->n[1]; ++j)
      for (int k = 0; k < h->n[2]; ++k) {
        const size_t idx = ((size_t)i * h->n[1] + j) * h->n[2] + k;
        const double mu = -(lam[0][i] + lam[1][j] + lam[2][k]);
        if (i == 0 && j == 0 && k == 0) { sh[idx] = 0.0; sf[idx] = 0.0; }
        else { sf[idx] = 4.0 * M_PI / mu; sh[idx] = std::sqrt(sf[idx]); }
      }
  hipError_t e = hipSuccess;
  e = hipMemcpyAsync(h->v64, p->v_loc, N * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h->psi64, p->psi, (size_t)h->nocc * N * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h->eps_d, p->eps, h->nocc * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && p->n_extra > 0)
    e = hipMemcpyAsync(h->psi64 + (size_t)h->nocc * N, p->psi_extra, (size_t)p->n_extra * N * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && p->n_extra > 0)
    e = hipMemcpyAsync(h->eps_d + h->nocc, p->eps_extra, p->n_extra * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h->s_half, sh.data(), N * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h->s_full, sf.data(), N * sizeof(double), hipMemcpyHostToDevice, s);
  for (int d = 0; d < 3 && e == hipSuccess; ++d)
    e = hipMemcpyAsync(h->Vax[d], V[d].data(), V[d].size() * sizeof(double), hipMemcpyHostToDevice, s);
  for (size_t k = 0; k < nl_up.size() && e == hipSuccess; ++k)
    if (nl_up[k].bytes)
      e = hipMemcpyAsync(nl_up[k].dst, nl_up[k].src, nl_up[k].bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && h->prec_mem)
    e = hipMemcpyAsync(h->prec_mem, prec_host.data(), prec_host.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_d2f(h->v64, h->v32, N, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    g_err = std::string("setup copies failed: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    return fail(RPA_E_HIP);
  }
  {
    std::string serr;
    h->scratch = scratch_on_current_device(&serr);   // nullptr: the allocation-free path reports it
  }
  *out = h;
  g_err.clear();
  return RPA_OK;
}

rpa_status rpa_destroy(rpa_handle h) {
  if (!h) return RPA_OK;
  (void)hipDeviceSynchronize();
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  fr(h->v64); fr(h->v32); fr(h->psi64); fr(h->eps_d); fr(h->s_half); fr(h->s_full);
  for (void* m : h->nl_mem) fr(m);
  fr(h->prec_mem);
  fr(h->nlcoef.p);
  for (int d = 0; d < 3; ++d) fr(h->Vax[d]);
  DevBuf* bufs[] = {&h->x64, &h->slots, &h->u64, &h->racc, &h->vtmp, &h->tmpA, &h->Q, &h->alpha,
                    &h->beta, &h->mlen, &h->active, &h->order, &h->iters, &h->cycles, &h->status,
                    &h->counter, &h->stats, &h->omega_b, &h->pos_b, &h->idx_b, &h->gpart, &h->G,
                    &h->dhat, &h->partials, &h->interp_m, &h->shifts, &h->fail, &h->faillist,
                    &h->obin, &h->ostats};
  for (DevBuf* b : bufs) fr(b->p);
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  fr(h->dres.p);
  for (hipEvent_t e : h->evs) (void)hipEventDestroy(e);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
  return RPA_OK;
}

rpa_status rpa_release_workspace(rpa_handle h) {
  if (!h) return set_err(RPA_E_ARG, "null handle");
  if (hipDeviceSynchronize() != hipSuccess) (void)hipGetLastError();
  drop_graphs(h);
  h->warm_B = 0;
  h->warm_m = 0;
  ++h->alloc_epoch;
  DevBuf* bufs[] = {&h->x64, &h->slots, &h->u64, &h->racc, &h->vtmp, &h->tmpA, &h->Q, &h->alpha,
                    &h->beta, &h->mlen, &h->active, &h->order, &h->iters, &h->cycles, &h->status,
                    &h->counter, &h->gpart, &h->G, &h->dhat, &h->partials, &h->shifts, &h->dres,
                    &h->nlcoef, &h->faillist, &h->obin, &h->ostats};
  for (DevBuf* b : bufs) {
    if (b->p) {
      (void)hipFree(b->p);
      h->allocated -= b->bytes;
      b->p = nullptr;
      b->bytes = 0;
    }
  }
  return RPA_OK;
}

rpa_status rpa_hamiltonian_apply(rpa_handle h, int32_t nvec, const double* shift_re,
                                 const double* shift_im, const void* x, void* y,
                                 int32_t precision, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(nvec >= 1 && nvec <= 65535, "nvec must be in [1, 65535]");
  ARG_CHECK(shift_re && shift_im && x && y, "null pointer");
  ARG_CHECK(precision == RPA_FP64 || precision == RPA_FP32_REFINE, "bad precision");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ENSURE(h, h->shifts, 2 * (size_t)nvec * sizeof(double));
  HIPCHK(h, hipMemcpyAsync(h->shifts.p, shift_re, nvec * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(P<double>(h->shifts) + nvec, shift_im, nvec * sizeof(double),
                           hipMemcpyHostToDevice, s));
  HIPCHK(h, hipEventRecord(h->ev0, s));
  HIPCHK(h, launch_happly(h->geom, h->c64, h->c32, h->v64, h->v32, nvec, P<double>(h->shifts),
                          P<double>(h->shifts) + nvec, x, y, precision == RPA_FP32_REFINE,
                          h->block, s));
  HIPCHK(h, hipEventRecord(h->ev1, s));
  if (h->nl.n_proj > 0) {
    ENSURE(h, h->nlcoef, (size_t)nvec * h->nl.n_proj * sizeof(double2));
    HIPCHK(h, launch_nl_apply(h->nl, h->N, nvec, x, y, h->nlcoef.p, precision == RPA_FP32_REFINE, s));
  }
  HIPCHK(h, hipStreamSynchronize(s));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->last_ms = ms;
  h->cocg_ms_total = ms;
  h->cocg_launches = 1;
  h->last_grid = h->geom.ntiles * nvec;
  return RPA_OK;
}

rpa_status rpa_coulomb_apply(rpa_handle h, int32_t power, int32_t nvec, const double* x, double* y,
                             void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(power == 1 || power == 2, "power must be 1 or 2");
  ARG_CHECK(nvec >= 1 && x && y, "bad arguments");
  return coulomb(h, power, nvec, x, y, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
namespace {

// chi0 x (or nu^1/2 chi0 nu^1/2 x) in batches of B vectors; `timing`
// records COCG launch events.
rpa_status chi0_body(rpa_ctx* h, double omega, int32_t nvec, const double* x, double* y,
                     int32_t symmetrized, rpa_stats* st, hipStream_t s, int B, bool timing) {
  const double t0 = now_s();
  const long long N = h->N;
  rpa_status r = begin_stats(h, s, std::vector<double>(1, omega), B);
  if (r != RPA_OK) return r;
  HIPCHK(h, launch_fill_i(P<int>(h->obin), 0, B, s));
  ENSURE(h, h->u64, (size_t)B * N * sizeof(double));
  ENSURE(h, h->omega_b, (size_t)B * sizeof(double));
  std::vector<double> om(B, omega);
  HIPCHK(h, hipMemcpyAsync(h->omega_b.p, om.data(), B * sizeof(double), hipMemcpyHostToDevice, s));
  for (int v0 = 0; v0 < nvec; v0 += B) {
    const int nb = std::min(B, nvec - v0);
    const double* xin = x + (size_t)v0 * N;
    if (symmetrized) {
      r = coulomb(h, 1, nb, xin, P<double>(h->u64), s);
      if (r != RPA_OK) return r;
    } else {
      HIPCHK(h, hipMemcpyAsync(h->u64.p, xin, (size_t)nb * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    std::vector<double> omn(om.begin(), om.begin() + nb);
    r = sternheimer_batch(h, nb, omn, nullptr, s, true, timing);
    if (r != RPA_OK) return r;
    double* yout = y + (size_t)v0 * N;
    if (symmetrized) {
      r = coulomb(h, 1, nb, P<double>(h->racc), yout, s);
      if (r != RPA_OK) return r;
    } else {
      HIPCHK(h, hipMemcpyAsync(yout, h->racc.p, (size_t)nb * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  }
  return end_stats(h, s, st, t0, (long long)nvec * h->nocc, 0);
}

// Where every workspace of chi0_body for batches of B vectors lies in the
// scratch array (offsets, 256-byte aligned) and how many bytes it needs in
// total; the sizes are those chi0_body and its callees ENSURE.
struct ScratchLayout {
  struct Item { DevBuf* buf; size_t bytes; };
  std::vector<Item> items;
  size_t total = 0;
};

ScratchLayout scratch_layout(rpa_ctx* h, int B, bool symmetrized) {
  ScratchLayout L;
  const size_t N = (size_t)h->N, b = (size_t)B, nocc = (size_t)h->nocc, items = b * nocc;
  const bool refine = h->precision == RPA_FP32_REFINE;
  const int bpc = h->slots_per_cu > 0 ? h->slots_per_cu
                                      : cocg_blocks_per_cu(h->geom, h->block, refine, h->nl.n_proj);
  const size_t grid = std::max<size_t>(1, std::min<size_t>(items, (size_t)bpc * h->num_cu));
  auto add = [&](DevBuf& buf, size_t bytes) {
    L.items.push_back({&buf, bytes});
    L.total += (bytes + 255) & ~(size_t)255;
  };
  add(h->stats, 8 * sizeof(unsigned long long));
  add(h->fail, 4 * sizeof(int));
  add(h->ostats, 6 * 64 * sizeof(unsigned long long));
  add(h->obin, std::max<size_t>(64, b) * sizeof(int));
  add(h->u64, b * N * sizeof(double));
  add(h->omega_b, b * sizeof(double));
  if (symmetrized) {
    add(h->tmpA, b * N * sizeof(double));
    add(h->vtmp, b * N * sizeof(double));
  }
  add(h->gpart, b * (size_t)gram_chunks(h->N) * h->ngal * nocc * sizeof(double));
  add(h->G, b * (size_t)h->ngal * nocc * sizeof(double2));
  add(h->x64, items * N * sizeof(double2));
  add(h->order, 2 * items * sizeof(int));
  add(h->iters, items * sizeof(int));
  add(h->cycles, items * sizeof(int));
  add(h->status, items * sizeof(int));
  add(h->counter, 64 * sizeof(int));
  if (refine) add(h->faillist, items * sizeof(int));
  add(h->slots, grid * (size_t)cocg_slot_bytes(h->geom, refine));
  add(h->racc, b * N * sizeof(double));
  return L;
}

}  // namespace
extern "C" {

rpa_status chi0_apply(rpa_handle h, double omega, int32_t nvec, const double* x, double* y,
                      int32_t symmetrized, rpa_stats* st, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(omega > 0 && std::isfinite(omega), "omega must be positive");
  ARG_CHECK(nvec >= 1 && x && y, "bad arguments");
  const int B = std::min(h->batch > 0 ? h->batch : 64, (int)nvec);
  return chi0_body(h, omega, nvec, x, y, symmetrized, st, reinterpret_cast<hipStream_t>(stream), B,
                   true);
}

rpa_status chi0_apply_noalloc(rpa_handle h, double omega, int32_t nvec, const double* x, double* y,
                              int32_t symmetrized, rpa_stats* st, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(omega > 0 && std::isfinite(omega), "omega must be positive");
  ARG_CHECK(nvec >= 1 && x && y, "bad arguments");
  if (!h->scratch) return set_err(RPA_E_HIP, "the scratch array of this device is not available");
  // the largest batch (at most the handle's) whose workspaces fit the scratch
  int B = std::min(h->batch > 0 ? h->batch : 64, (int)nvec);
  while (B > 1 && scratch_layout(h, B, symmetrized != 0).total > kScratchBytes) --B;
  ScratchLayout L = scratch_layout(h, B, symmetrized != 0);
  if (L.total > kScratchBytes)
    return set_err(RPA_E_ARG, "problem too large for chi0_apply_noalloc: one vector needs " +
                                  std::to_string(L.total) + " bytes of workspace, the scratch array holds " +
                                  std::to_string(kScratchBytes));
  // point the handle's workspaces into the scratch for this call, then put
  // its own buffers back (they are neither used nor freed meanwhile)
  struct Swap {
    rpa_ctx* h;
    std::vector<std::pair<DevBuf*, DevBuf>> saved;
    ~Swap() {
      for (auto& sv : saved) *sv.first = sv.second;
      h->no_alloc = false;
    }
  } swap{h, {}};
  char* base = static_cast<char*>(h->scratch);
  size_t off = 0;
  for (const auto& it : L.items) {
    swap.saved.push_back({it.buf, *it.buf});
    it.buf->p = base + off;
    it.buf->bytes = it.bytes;
    off += (it.bytes + 255) & ~(size_t)255;
  }
  h->no_alloc = true;
  // no timing events: creating them is a driver allocation
  return chi0_body(h, omega, nvec, x, y, symmetrized, st, reinterpret_cast<hipStream_t>(stream), B,
                   false);
}

rpa_status rpa_sternheimer_solve(rpa_handle h, double omega, int32_t nvec, const double* u,
                                 double* x, rpa_stats* st, void* stream) {
  rpa_status r0 = usable(h);
  if (r0 != RPA_OK) return r0;
  ARG_CHECK(omega > 0 && std::isfinite(omega), "omega must be positive");
  ARG_CHECK(nvec >= 1 && u && x, "bad arguments");
  const double t0 = now_s();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long N = h->N;
  const int B = std::min(h->batch > 0 ? h->batch : 64, (int)nvec);
  rpa_status r = begin_stats(h, s, std::vector<double>(1, omega), B);
  if (r != RPA_OK) return r;
  HIPCHK(h, launch_fill_i(P<int>(h->obin), 0, B, s));
  ENSURE(h, h->u64, (size_t)B * N * sizeof(double));
  ENSURE(h, h->omega_b, (size_t)B * sizeof(double));
  std::vector<double> om(B, omega);
  HIPCHK(h, hipMemcpyAsync(h->omega_b.p, om.data(), B * sizeof(double), hipMemcpyHostToDevice, s));
  for (int v0 = 0; v0 < nvec; v0 += B) {
    const int nb = std::min(B, nvec - v0);
    HIPCHK(h, hipMemcpyAsync(h->u64.p, u + (size_t)v0 * N, (size_t)nb * N * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    std::vector<double> omn(om.begin(), om.begin() + nb);
    r = sternheimer_batch(h, nb, omn, nullptr, s);
    if (r != RPA_OK) return r;
    HIPCHK(h, hipMemcpyAsync(x + (size_t)v0 * h->nocc * N * 2, h->x64.p,
                             (size_t)nb * h->nocc * N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  return end_stats(h, s, st, t0, (long long)nvec * h->nocc, 0);
}

}  // extern "C"
namespace {

// The whole per-batch sequence: q_1 = e_j, then per Lanczos step nu^1/2,
// Galerkin guess, persistent COCG, accumulation, nu^1/2, Lanczos update; then
// the tridiagonal quadrature into dres.  Kernels only (no copies), so it can
// be captured into a graph once the workspaces exist.
rpa_status enqueue_batch(rpa_ctx* h, int nb, int m, hipStream_t s, bool timing) {
  const long long N = h->N;
  rpa_status r = RPA_OK;
  HIPCHK(h, launch_fill_d(P<double>(h->Q), 0.0, (long long)m * nb * N, s));
  HIPCHK(h, launch_set_onehot(P<double>(h->Q), N, P<long long>(h->idx_b), nb, s));
  HIPCHK(h, launch_fill_i(P<int>(h->active), 1, nb, s));
  HIPCHK(h, launch_fill_i(P<int>(h->mlen), 0, nb, s));
  HIPCHK(h, launch_fill_d(P<double>(h->alpha), 0.0, (long long)nb * m, s));
  HIPCHK(h, launch_fill_d(P<double>(h->beta), 0.0, (long long)nb * m, s));
  static const std::vector<double> none;
  for (int k = 0; k < m; ++k) {
    double* qk = P<double>(h->Q) + (size_t)k * nb * N;
    r = coulomb(h, 1, nb, qk, P<double>(h->u64), s);
    if (r != RPA_OK) return r;
    r = sternheimer_batch(h, nb, none, P<int>(h->active), s, false, timing);
    if (r != RPA_OK) return r;
    // v = nu^1/2 racc  (written into u64, which is free again)
    r = coulomb(h, 1, nb, P<double>(h->racc), P<double>(h->u64), s);
    if (r != RPA_OK) return r;
    HIPCHK(h, launch_lanczos_step(k, m, nb, N, P<double>(h->Q), P<double>(h->u64),
                                  P<double>(h->alpha), P<double>(h->beta), P<int>(h->mlen),
                                  P<int>(h->active), h->lz_brk, s));
    if (h->progress && !h->capturing) {
      HIPCHK(h, hipStreamSynchronize(s));
      std::fprintf(stderr, "[rpa] batch %lld (%d start vectors): Lanczos step %d/%d done at %.1f s\n",
                   h->progress_batch, nb, k + 1, m, now_s() - h->progress_t0);
      std::fflush(stderr);
    }
  }
  HIPCHK(h, launch_tridiag_quad(nb, m, P<double>(h->alpha), P<double>(h->beta), P<int>(h->mlen),
                                nullptr, P<double>(h->dres), P<int>(h->fail), s));
  return RPA_OK;
}

void drop_graphs(rpa_ctx* h) {
  for (auto& kv : h->graphs) {
    (void)hipGraphExecDestroy(kv.second.e);
    (void)hipGraphDestroy(kv.second.g);
  }
  h->graphs.clear();
}

// Run one batch: eagerly (first time, which also allocates), or by replaying
// a captured graph of the same (nb, m) whose buffers are still current.
rpa_status run_batch(rpa_ctx* h, int nb, int m, hipStream_t s) {
  const bool warm = h->warm_m == m && nb <= h->warm_B;
  if (!h->use_graph || !warm) {
    const unsigned e0 = h->alloc_epoch;
    rpa_status r = enqueue_batch(h, nb, m, s, true);
    if (r != RPA_OK) return r;
    if (h->alloc_epoch != e0) { drop_graphs(h); h->warm_B = 0; }
    if (h->warm_m != m) { h->warm_m = m; h->warm_B = 0; }
    h->warm_B = std::max(h->warm_B, nb);
    return RPA_OK;
  }
  const std::pair<int, int> key(nb, m);
  rpa_ctx::GraphEntry* ge = nullptr;
  for (auto& kv : h->graphs)
    if (kv.first == key && kv.second.epoch == h->alloc_epoch) ge = &kv.second;
  if (!ge) {
    if (!h->cap_stream) HIPCHK(h, hipStreamCreate(&h->cap_stream));   // default priority
    rpa_ctx::GraphEntry g{};
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    h->capturing = true;
    rpa_status r = enqueue_batch(h, nb, m, h->cap_stream, false);
    h->capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
    if (r != RPA_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    HIPCHK(h, ec);
    g.g = graph;
    HIPCHK(h, hipGraphInstantiate(&g.e, graph, nullptr, nullptr, 0));
    g.epoch = h->alloc_epoch;
    h->graphs.push_back({key, g});
    ge = &h->graphs.back().second;
  }
  HIPCHK(h, hipGraphLaunch(ge->e, s));
  return RPA_OK;
}

}  // namespace

extern "C" {

rpa_status lanczos_energy_density(rpa_handle h, int32_t n_omega, const double* omega,
                                  int32_t n_pts, const int64_t* point_idx, int32_t n_lanczos,
                                  double* d, rpa_stats* st, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(n_omega >= 1 && n_pts >= 1 && omega && point_idx && d, "bad arguments");
  ARG_CHECK(n_lanczos >= 1 && n_lanczos <= kMaxLanczos, "n_lanczos must be in [1, 64]");
  for (int k = 0; k < n_omega; ++k) ARG_CHECK(omega[k] > 0 && std::isfinite(omega[k]), "omega must be positive");
  for (int p = 0; p < n_pts; ++p) ARG_CHECK(point_idx[p] >= 0 && point_idx[p] < h->N, "point index out of range");
  const double t0 = now_s();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long N = h->N;
  const int m = n_lanczos;
  const long long P_total = (long long)n_omega * n_pts;
  int B = h->batch > 0 ? h->batch : 64;
  B = (int)std::min<long long>(B, P_total);
  rpa_status r = begin_stats(h, s, std::vector<double>(omega, omega + n_omega), B);
  if (r != RPA_OK) return r;
  ENSURE(h, h->Q, (size_t)m * B * N * sizeof(double));
  ENSURE(h, h->u64, (size_t)B * N * sizeof(double));
  ENSURE(h, h->alpha, (size_t)B * m * sizeof(double));
  ENSURE(h, h->beta, (size_t)B * m * sizeof(double));
  ENSURE(h, h->mlen, (size_t)B * sizeof(int));
  ENSURE(h, h->active, (size_t)B * sizeof(int));
  ENSURE(h, h->omega_b, (size_t)B * sizeof(double));
  ENSURE(h, h->pos_b, (size_t)B * sizeof(long long));
  ENSURE(h, h->idx_b, (size_t)B * sizeof(long long));
  ENSURE(h, h->dres, (size_t)B * sizeof(double));
  std::vector<double> om(B);
  std::vector<long long> pos(B), idx(B);
  std::vector<int> bin(B);
  h->progress_t0 = t0;
  h->progress_batch = 0;
  for (long long i0 = 0; i0 < P_total; i0 += B) {
    const int nb = (int)std::min<long long>(B, P_total - i0);
    ++h->progress_batch;
    // pair i -> point p = i / n_omega, frequency k = i % n_omega (frequencies mixed per batch)
    for (int b = 0; b < nb; ++b) {
      const long long i = i0 + b;
      const int p = (int)(i / n_omega), k = (int)(i % n_omega);
      om[b] = omega[k];
      pos[b] = (long long)k * n_pts + p;
      idx[b] = point_idx[p];
      bin[b] = k;
    }
    HIPCHK(h, hipMemcpyAsync(h->omega_b.p, om.data(), nb * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->obin.p, bin.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->pos_b.p, pos.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->idx_b.p, idx.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
    std::vector<double> omn(om.begin(), om.begin() + nb);
    r = upload_order_for(h, nb, omn, s);
    if (r != RPA_OK) return r;
    r = run_batch(h, nb, m, s);
    if (r != RPA_OK) return r;
    // results of the batch: dres[b] -> d[pos_b[b]]
    HIPCHK(h, launch_scatter(P<double>(h->dres), P<long long>(h->pos_b), nb, d, s));
  }
  // Lanczos truncations: count mlen < m over the last batch only is not enough;
  // the tridiagonal kernel flags QL failures, truncations are tracked below.
  return end_stats(h, s, st, t0, P_total * (long long)h->nocc * m, 0);
}

}  // extern "C"

namespace {

// One batch of G groups (columns gcol[g] .. gcol[g] + gsz[g] - 1, at most
// bmax each) through m block Lanczos steps, then the block Gauss rule into
// d[pos_b[column]].  Eager launches only.
rpa_status enqueue_block_batch(rpa_ctx* h, int nb, int G, int bmax, int m, double* d, hipStream_t s) {
  const long long N = h->N;
  const int pmax = std::max(m, 2) * kMaxLzBlock;
  constexpr size_t S = (size_t)kMaxLzBlock * kMaxLzBlock;
  double* Q = P<double>(h->Q);
  double* W = P<double>(h->u64);
  const int* gcol = P<int>(h->bgcol);
  const int* gsz = P<int>(h->bgsz);
  int* gact = P<int>(h->bgact);
  double* C = P<double>(h->bC);
  double* part = P<double>(h->bpart);
  double* Ab = P<double>(h->Ablk);
  double* Bb = P<double>(h->Bblk);
  HIPCHK(h, launch_fill_d(Q, 0.0, (long long)m * nb * N, s));
  HIPCHK(h, launch_set_onehot(Q, N, P<long long>(h->idx_b), nb, s));
  HIPCHK(h, launch_fill_i(P<int>(h->active), 1, nb, s));
  HIPCHK(h, launch_fill_i(gact, 1, G, s));
  HIPCHK(h, launch_fill_i(P<int>(h->bgm), 0, G, s));
  HIPCHK(h, launch_fill_d(P<double>(h->bamax), 0.0, G, s));
  HIPCHK(h, launch_fill_d(Ab, 0.0, (long long)G * m * S, s));
  HIPCHK(h, launch_fill_d(Bb, 0.0, (long long)G * m * S, s));
  static const std::vector<double> none;
  const BVSet Wall{W, 0, 1, 0, 0};
  for (int k = 0; k < m; ++k) {
    double* qk = Q + (size_t)k * nb * N;
    rpa_status r = coulomb(h, 1, nb, qk, W, s);
    if (r != RPA_OK) return r;
    r = sternheimer_batch(h, nb, none, P<int>(h->active), s, false, true);
    if (r != RPA_OK) return r;
    r = coulomb(h, 1, nb, P<double>(h->racc), W, s);
    if (r != RPA_OK) return r;
    // A_k = sym(Q_k^T W); W -= Q_{k-1} B_{k-1}^T + Q_k A_k
    HIPCHK(h, launch_bgram(BVSet{Q, k, 1, 0, 0}, Wall, bmax, nb, N, G, gcol, gsz, gact, pmax, part, C, s));
    HIPCHK(h, launch_bstep_diag(G, k, m, gsz, gact, pmax, C, Ab, Bb, P<double>(h->bamax), P<int>(h->bgm), s));
    const BVSet prev2{Q, k > 0 ? k - 1 : 0, k > 0 ? 2 : 1, 0, 0};
    HIPCHK(h, launch_bcombine(prev2, Wall, nb, N, G, gcol, gsz, gact, pmax, C, s));
    // two classical Gram-Schmidt passes against every stored block
    const BVSet stored{Q, 0, k + 1, 0, 0};
    for (int pass = 0; pass < 2; ++pass) {
      HIPCHK(h, launch_bgram(stored, Wall, (k + 1) * bmax, nb, N, G, gcol, gsz, gact, pmax, part, C, s));
      HIPCHK(h, launch_bcombine(stored, Wall, nb, N, G, gcol, gsz, gact, pmax, C, s));
    }
    if (k == m - 1) break;
    // Q_{k+1} B_k = W, column by column (two projection passes each)
    for (int j = 0; j < bmax; ++j) {
      const BVSet wj{W, 0, 1, j, 1};
      if (j > 0) {
        const BVSet done{Q, k + 1, 1, 0, j};
        for (int pass = 0; pass < 2; ++pass) {
          HIPCHK(h, launch_bgram(done, wj, j, nb, N, G, gcol, gsz, gact, pmax, part, C, s));
          HIPCHK(h, launch_bqr_acc(G, k, m, j, gsz, gact, pmax, C, Bb, s));
          HIPCHK(h, launch_bcombine(done, wj, nb, N, G, gcol, gsz, gact, pmax, C, s));
        }
      }
      HIPCHK(h, launch_bgram(wj, wj, 1, nb, N, G, gcol, gsz, gact, pmax, part, C, s));
      HIPCHK(h, launch_bqr_norm(G, k, m, j, gcol, gsz, gact, pmax, C, Bb, P<double>(h->bamax), h->lz_brk,
                                P<double>(h->bscale), P<int>(h->active), s));
      HIPCHK(h, launch_bqr_scale(Q, W, nb, N, G, k, j, gcol, gsz, gact, P<double>(h->bscale), s));
    }
    if (h->progress) {
      HIPCHK(h, hipStreamSynchronize(s));
      std::fprintf(stderr, "[rpa] block batch %lld (%d groups): Lanczos step %d/%d done at %.1f s\n",
                   h->progress_batch, G, k + 1, m, now_s() - h->progress_t0);
      std::fflush(stderr);
    }
  }
  HIPCHK(h, launch_block_quad(G, m, gcol, gsz, P<int>(h->bgm), Ab, Bb, P<long long>(h->pos_b), d,
                              P<int>(h->fail), s));
  return RPA_OK;
}

}  // namespace

extern "C" {

rpa_status lanczos_energy_density_block(rpa_handle h, int32_t n_omega, const double* omega,
                                        int32_t n_pts, const int64_t* point_idx, int32_t n_lanczos,
                                        int32_t block, double* d, rpa_stats* st, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(n_omega >= 1 && n_pts >= 1 && omega && point_idx && d, "bad arguments");
  ARG_CHECK(block >= 1 && block <= kMaxLzBlock, "block must be in [1, 8]");
  ARG_CHECK(n_lanczos >= 1 && (long long)n_lanczos * block <= kMaxLanczos,
            "n_lanczos * block must be in [1, 64]");
  for (int k = 0; k < n_omega; ++k) ARG_CHECK(omega[k] > 0 && std::isfinite(omega[k]), "omega must be positive");
  for (int p = 0; p < n_pts; ++p) ARG_CHECK(point_idx[p] >= 0 && point_idx[p] < h->N, "point index out of range");
  const double t0 = now_s();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long N = h->N;
  const int m = n_lanczos;
  // groups: consecutive points at one frequency, the last of each frequency ragged
  struct Grp { int k, p0, b; };
  std::vector<Grp> groups;
  for (int k = 0; k < n_omega; ++k)
    for (int p0 = 0; p0 < n_pts; p0 += block) groups.push_back({k, p0, std::min(block, n_pts - p0)});
  int B = h->batch > 0 ? h->batch : 64;
  B = std::max(B, (int)block);
  B = (int)std::min<long long>(B, (long long)n_omega * n_pts);
  rpa_status r = begin_stats(h, s, std::vector<double>(omega, omega + n_omega), B);
  if (r != RPA_OK) return r;
  const int gmax = B;
  const int pmax = std::max(m, 2) * kMaxLzBlock;
  constexpr size_t S = (size_t)kMaxLzBlock * kMaxLzBlock;
  ENSURE(h, h->Q, (size_t)m * B * N * sizeof(double));
  ENSURE(h, h->u64, (size_t)B * N * sizeof(double));
  ENSURE(h, h->active, (size_t)B * sizeof(int));
  ENSURE(h, h->omega_b, (size_t)B * sizeof(double));
  ENSURE(h, h->pos_b, (size_t)B * sizeof(long long));
  ENSURE(h, h->idx_b, (size_t)B * sizeof(long long));
  ENSURE(h, h->bgcol, (size_t)gmax * sizeof(int));
  ENSURE(h, h->bgsz, (size_t)gmax * sizeof(int));
  ENSURE(h, h->bgact, (size_t)gmax * sizeof(int));
  ENSURE(h, h->bgm, (size_t)gmax * sizeof(int));
  ENSURE(h, h->bamax, (size_t)gmax * sizeof(double));
  ENSURE(h, h->bscale, (size_t)gmax * sizeof(double));
  ENSURE(h, h->Ablk, (size_t)gmax * m * S * sizeof(double));
  ENSURE(h, h->Bblk, (size_t)gmax * m * S * sizeof(double));
  ENSURE(h, h->bC, (size_t)gmax * pmax * kMaxLzBlock * sizeof(double));
  ENSURE(h, h->bpart, (size_t)gmax * pmax * kMaxLzBlock * bgram_chunks(N) * sizeof(double));
  std::vector<double> om;
  std::vector<long long> pos, idx;
  std::vector<int> bin, gcol, gsz;
  h->progress_t0 = t0;
  h->progress_batch = 0;
  size_t gi = 0;
  while (gi < groups.size()) {
    // whole groups into one batch of at most B columns
    om.clear(); pos.clear(); idx.clear(); bin.clear(); gcol.clear(); gsz.clear();
    int bmax = 0;
    while (gi < groups.size() && (int)om.size() + groups[gi].b <= B) {
      const Grp& g = groups[gi++];
      gcol.push_back((int)om.size());
      gsz.push_back(g.b);
      bmax = std::max(bmax, g.b);
      for (int c = 0; c < g.b; ++c) {
        om.push_back(omega[g.k]);
        pos.push_back((long long)g.k * n_pts + g.p0 + c);
        idx.push_back(point_idx[g.p0 + c]);
        bin.push_back(g.k);
      }
    }
    const int nb = (int)om.size(), G = (int)gcol.size();
    ++h->progress_batch;
    HIPCHK(h, hipMemcpyAsync(h->omega_b.p, om.data(), nb * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->obin.p, bin.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->pos_b.p, pos.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->idx_b.p, idx.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->bgcol.p, gcol.data(), G * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->bgsz.p, gsz.data(), G * sizeof(int), hipMemcpyHostToDevice, s));
    r = upload_order_for(h, nb, om, s);
    if (r != RPA_OK) return r;
    r = enqueue_block_batch(h, nb, G, bmax, m, d, s);
    if (r != RPA_OK) return r;
    // the host vectors above are reused by the next batch: their copies must have landed
    HIPCHK(h, hipStreamSynchronize(s));
  }
  return end_stats(h, s, st, t0, (long long)n_omega * n_pts * h->nocc * m, 0);
}

rpa_status interpolate(rpa_handle h, int32_t kind, int32_t stride, int32_t n_fields,
                       const double* coarse, double* fine, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(kind >= RPA_INTERP_NONE && kind <= RPA_INTERP_FOURIER, "bad interpolation kind");
  ARG_CHECK(stride >= 1, "stride must be >= 1");
  for (int d = 0; d < 3; ++d) ARG_CHECK(h->n[d] % stride == 0, "stride must divide every n[d]");
  ARG_CHECK(kind != RPA_INTERP_NONE || stride == 1, "RPA_INTERP_NONE requires stride 1");
  ARG_CHECK(n_fields >= 1 && coarse && fine, "bad arguments");
  return do_interpolate(h, kind, stride, n_fields, coarse, fine, reinterpret_cast<hipStream_t>(stream));
}

rpa_status rpa_energy_from_coarse(rpa_handle h, int32_t n_omega, const double* weight,
                                  int32_t stride, int32_t kind, const double* d_coarse,
                                  double* e_c, double* e_fine, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(n_omega >= 1 && weight && d_coarse && e_c, "bad arguments");
  ARG_CHECK(kind >= RPA_INTERP_NONE && kind <= RPA_INTERP_FOURIER, "bad interpolation kind");
  ARG_CHECK(stride >= 1, "stride must be >= 1");
  for (int d = 0; d < 3; ++d) ARG_CHECK(h->n[d] % stride == 0, "stride must divide every n[d]");
  ARG_CHECK(kind != RPA_INTERP_NONE || stride == 1, "RPA_INTERP_NONE requires stride 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long N = h->N;
  ENSURE(h, h->dhat, (size_t)n_omega * N * sizeof(double));
  rpa_status r = do_interpolate(h, kind, stride, n_omega, d_coarse, P<double>(h->dhat), s);
  if (r != RPA_OK) return r;
  const int nblk = 256;
  ENSURE(h, h->partials, nblk * sizeof(double) + (size_t)n_omega * sizeof(double));
  double* wdev = P<double>(h->partials) + nblk;
  HIPCHK(h, hipMemcpyAsync(wdev, weight, n_omega * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(h, launch_weighted_sum(P<double>(h->dhat), wdev, n_omega, N, 1.0 / (2.0 * M_PI * h->dV),
                                e_fine, P<double>(h->partials), nblk, s));
  std::vector<double> part(nblk);
  HIPCHK(h, hipMemcpyAsync(part.data(), h->partials.p, nblk * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  double tot = 0.0;
  for (int i = 0; i < nblk; ++i) tot += part[i];
  *e_c = tot / (2.0 * M_PI);
  return RPA_OK;
}

rpa_status correlation_energy(rpa_handle h, int32_t n_omega, const double* omega,
                              const double* weight, int32_t stride, int32_t kind,
                              int32_t n_lanczos, double* e_c, double* e_fine, rpa_stats* st,
                              void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(n_omega >= 1 && omega && weight && e_c, "bad arguments");
  ARG_CHECK(stride >= 1, "stride must be >= 1");
  for (int d = 0; d < 3; ++d) ARG_CHECK(h->n[d] % stride == 0, "stride must divide every n[d]");
  ARG_CHECK(kind >= RPA_INTERP_NONE && kind <= RPA_INTERP_FOURIER, "bad interpolation kind");
  ARG_CHECK(kind != RPA_INTERP_NONE || stride == 1, "RPA_INTERP_NONE requires stride 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<int64_t> pts;
  for (int i = 0; i < h->n[0]; i += stride)
    for (int j = 0; j < h->n[1]; j += stride)
      for (int k = 0; k < h->n[2]; k += stride)
        pts.push_back(((int64_t)i * h->n[1] + j) * h->n[2] + k);
  const size_t nc = pts.size();
  double* dco = nullptr;
  if (hipMalloc((void**)&dco, (size_t)n_omega * nc * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(RPA_E_OOM, "hipMalloc failed for coarse diagonals");
  }
  rpa_status r = lanczos_energy_density(h, n_omega, omega, (int32_t)nc, pts.data(), n_lanczos, dco, st, stream);
  rpa_status warn = RPA_OK;
  if (r == RPA_W_NOCONV || r == RPA_W_BREAKDOWN) { warn = r; r = RPA_OK; }
  if (r == RPA_OK) r = rpa_energy_from_coarse(h, n_omega, weight, stride, kind, dco, e_c, e_fine, stream);
  (void)hipStreamSynchronize(s);
  (void)hipFree(dco);
  if (r != RPA_OK) return r;
  return warn;
}

rpa_status rpa_autotune(rpa_handle h, int32_t n_lanczos, int32_t probe_iters,
                        rpa_tune_result* out, void* stream) {
  rpa_status u = usable(h);
  if (u != RPA_OK) return u;
  ARG_CHECK(out, "null output");
  ARG_CHECK(n_lanczos >= 1 && n_lanczos <= kMaxLanczos, "n_lanczos must be in [1, 64]");
  ARG_CHECK(probe_iters >= 0 && probe_iters <= 1000, "probe_iters must be in [0, 1000]");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long N = h->N;
  const int nocc = h->nocc;
  const int ny = h->geom.ny, nz = h->geom.nz;
  const bool refine = h->precision == RPA_FP32_REFINE;
  const int K = probe_iters > 0 ? probe_iters : 16;
  memset(out, 0, sizeof(*out));

  // candidate tiles: the whole plane if it fits, then the four tallest
  // divisors of ny with ty >= 6 (shorter tiles re-read more halo rows)
  std::vector<int> tys;
  for (int t = ny; t >= kRadius && tys.size() < 4; --t) {
    if (ny % t || ((t * nz + 63) / 64) * 64 > kMaxBlock) continue;
    Geom gq = h->geom;
    gq.ty = t;
    gq.ntiles = ny / t;
    const int blk = ((t * nz + 63) / 64) * 64;
    if (cocg_shmem_bytes(gq, blk, refine, h->nl.n_proj) > 160 * 1024 ||
        cocg_shmem_bytes(gq, blk, false, h->nl.n_proj) > 160 * 1024)
      continue;
    tys.push_back(t);
  }
  if (tys.empty()) return set_err(RPA_E_STATE, "no tile shape fits");

  // fixed-work probe: one-hot start vectors through nu^1/2, omega = 0.69,
  // exactly K COCG iterations per system (tolerance out of reach)
  const Geom g0 = h->geom;
  const int blk0 = h->block, slots0 = h->slots_per_cu;
  const double tol0 = h->tol;
  const int maxit0 = h->maxit;
  auto restore = [&]() {
    h->geom = g0; h->block = blk0; h->slots_per_cu = slots0; h->tol = tol0; h->maxit = maxit0;
  };
  const int Bp = (int)std::min<long long>(64, std::max<long long>(1, (2LL * h->num_cu * 2 + nocc - 1) / nocc));
  rpa_status r = begin_stats(h, s, std::vector<double>(), Bp);
  if (r != RPA_OK) return r;
  ENSURE(h, h->Q, (size_t)Bp * N * sizeof(double));
  ENSURE(h, h->u64, (size_t)Bp * N * sizeof(double));
  ENSURE(h, h->omega_b, (size_t)Bp * sizeof(double));
  ENSURE(h, h->idx_b, (size_t)Bp * sizeof(long long));
  std::vector<double> om(Bp, 0.69);
  std::vector<long long> idx(Bp);
  for (int b = 0; b < Bp; ++b) idx[b] = (long long)((N - 1) * (double)b / std::max(1, Bp - 1));
  HIPCHK(h, hipMemcpyAsync(h->omega_b.p, om.data(), Bp * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->idx_b.p, idx.data(), Bp * sizeof(long long), hipMemcpyHostToDevice, s));
  HIPCHK(h, launch_fill_d(P<double>(h->Q), 0.0, (long long)Bp * N, s));
  HIPCHK(h, launch_set_onehot(P<double>(h->Q), N, P<long long>(h->idx_b), Bp, s));
  r = coulomb(h, 1, Bp, P<double>(h->Q), P<double>(h->u64), s);
  if (r != RPA_OK) return r;
  HIPCHK(h, hipStreamSynchronize(s));

  double best = -1.0;
  int best_ty = g0.ty, best_slots = 1;
  h->tol = 1e-300;
  h->maxit = K;
  for (int t : tys) {
    h->geom.ty = t;
    h->geom.ntiles = ny / t;
    h->block = ((t * nz + 63) / 64) * 64;
    const int occ = cocg_blocks_per_cu(h->geom, h->block, refine, h->nl.n_proj);
    for (int slots = 1; slots <= std::min(2, occ); ++slots) {
      h->slots_per_cu = slots;
      float ms = 0.f;
      for (int rep = 0; rep < 3; ++rep) {   // first run warms up
        if (rep == 1) HIPCHK(h, hipEventRecord(h->ev0, s));
        r = sternheimer_batch(h, Bp, om, nullptr, s, true, false);
        if (r != RPA_OK) { restore(); return r; }
      }
      HIPCHK(h, hipEventRecord(h->ev1, s));
      HIPCHK(h, hipStreamSynchronize(s));
      if (hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess) { restore(); return set_err(RPA_E_HIP, "timing failed"); }
      const double rate = 2.0 * Bp * nocc * K / (ms * 1e-3);   // system-iterations per s
      ++out->n_tried;
      if (rate > best) { best = rate; best_ty = t; best_slots = slots; }
    }
  }
  restore();
  h->geom.ty = best_ty;
  h->geom.ntiles = ny / best_ty;
  h->block = ((best_ty * nz + 63) / 64) * 64;
  h->slots_per_cu = best_slots;
  drop_graphs(h);
  h->warm_B = 0;
  h->warm_m = 0;
  ++h->alloc_epoch;

  // start vectors per launch: as many as fit (at most 64) in the budget, or
  // in 80% of the free device memory, next to what is allocated already
  const size_t per_vec = (size_t)nocc * N * sizeof(double2) + (size_t)n_lanczos * N * sizeof(double) +
                         6 * (size_t)N * sizeof(double);
  size_t avail = 0;
  if (h->budget) {
    avail = h->budget > h->allocated ? h->budget - h->allocated : 0;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); fr = 0; }
    avail = (size_t)(0.8 * (double)fr);
  }
  const int grid_slots = best_slots * h->num_cu;
  const size_t slots_bytes = (size_t)grid_slots * cocg_slot_bytes(h->geom, refine);
  avail = avail > slots_bytes ? avail - slots_bytes : 0;
  h->batch = (int)std::max<size_t>(1, std::min<size_t>(64, avail / per_vec));
  out->tile_y = best_ty;
  out->slots_per_cu = best_slots;
  out->batch = h->batch;
  out->system_iters_per_s = best;
  return RPA_OK;
}

rpa_status rpa_last_iteration_stats(rpa_handle h, int32_t cap, double* omega, int64_t* count,
                                    double* mean, double* stdev, int64_t* min_iters,
                                    int64_t* max_iters, int64_t* refine_cycles, int32_t* n_out) {
  if (!h) return set_err(RPA_E_ARG, "null handle");
  ARG_CHECK(cap >= 0, "cap must be >= 0");
  const int nb = h->stat_host.empty() ? 0 : h->stat_bins;
  if (n_out) *n_out = nb;
  const unsigned long long* o = h->stat_host.data();
  for (int i = 0; i < std::min(nb, (int)cap); ++i) {
    const double c = (double)o[i];
    const double m = c > 0 ? (double)o[nb + i] / c : 0.0;
    const double var = c > 0 ? std::max(0.0, (double)o[2 * nb + i] / c - m * m) : 0.0;
    if (omega) omega[i] = h->stat_omega[i];
    if (count) count[i] = (int64_t)o[i];
    if (mean) mean[i] = m;
    if (stdev) stdev[i] = std::sqrt(var);
    if (min_iters) min_iters[i] = c > 0 ? (int64_t)o[3 * nb + i] : 0;
    if (max_iters) max_iters[i] = (int64_t)o[4 * nb + i];
    if (refine_cycles) refine_cycles[i] = (int64_t)o[5 * nb + i];
  }
  return RPA_OK;
}

rpa_status rpa_last_cocg_split(rpa_handle h, double* ms_plain, double* ms_prec, double* ms_followup) {
  if (!h) return set_err(RPA_E_ARG, "null handle");
  if (ms_plain) *ms_plain = h->cocg_ms_kind[0];
  if (ms_prec) *ms_prec = h->cocg_ms_kind[1];
  if (ms_followup) *ms_followup = h->cocg_ms_kind[2];
  return RPA_OK;
}

rpa_status rpa_last_cocg_timing(rpa_handle h, double* ms, int32_t* launches, int32_t* grid,
                                int32_t* block, int32_t* tile_y) {
  if (!h) return set_err(RPA_E_ARG, "null handle");
  if (ms) *ms = h->cocg_ms_total;
  if (launches) *launches = h->cocg_launches;
  if (grid) *grid = h->last_grid;
  if (block) *block = h->block;
  if (tile_y) *tile_y = h->geom.ty;
  return RPA_OK;
}

}  // extern "C"
