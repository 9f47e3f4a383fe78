// Batched Sternheimer solves (paper: Eq. 4, COCG with Galerkin initial guess,
// Implementation section) as one persistent launch.
//
// Design (gfx950, wave64):
//  * One workgroup owns one complex-symmetric system (H - eps_n - i omega) x = b
//    at a time and runs COCG to convergence with no grid-wide synchronisation;
//    workgroups take systems from an atomic work counter (longest-first order
//    is chosen by the host), so per-system iteration counts that differ by
//    10x across omega do not idle the chip.
//  * The 37-point stencil of the 12th-order FD Hamiltonian marches along x:
//    each thread owns one (y, z) column of a tile of ty rows x nz columns and
//    keeps the 13 planes x-6..x+6 of its column in registers; the current
//    plane (plus 6 halo rows on each side in y) sits in LDS, double
//    buffered, so each step needs a single barrier.  Every vector element is
//    read from HBM once per sweep (plus the y halo and the periodic x wrap).
//  * COCG per iteration: sweep A forms p = r + beta p_old on load, writes p
//    and q = A p and reduces mu = p^T q (p is double buffered because
//    neighbouring planes and halo rows still need p_old); sweep B updates
//    x, r and reduces r^T r and ||r||^2.  All reductions are per workgroup in
//    a fixed order, so results do not depend on scheduling.
//  * FP32_REFINE: COCG in FP32 with reliable updates: the FP32 correction is
//    folded into the FP64 solution and the residual replaced by the FP64
//    residual r = b - A x (an FP64 stencil sweep) whenever the recursive
//    residual has dropped by a fixed factor; the search direction is kept.
//    b = -psi_n (.) u is formed on the fly in FP64 and never stored.
#pragma once

#include "internal.h"

namespace rpa {

namespace {

template <typename T> struct V2;
template <> struct V2<float> { typedef float2 t; };
template <> struct V2<double> { typedef double2 t; };

}  // namespace
}  // namespace rpa

#include "precond_impl.h"

namespace rpa {

namespace {

constexpr int R = kRadius;
constexpr int QN = 2 * R + 1;
constexpr int kMinGap = 4;     // fewest FP32 iterations between reliable updates
constexpr int kMaxGap = 100;   // most FP32 iterations between true-residual checks

__device__ __forceinline__ float2 mk2(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ double2 mk2(double a, double b) { return make_double2(a, b); }

template <typename T2>
__device__ __forceinline__ T2 zero2() { T2 z; z.x = 0; z.y = 0; return z; }

// Every value that steers control flow around a barrier is broadcast from
// lane 0 into a scalar register, so the compiler sees wave-uniform branches
// (values read back from LDS are otherwise treated as divergent, which puts
// __syncthreads() into divergent control flow).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---------------------------------------------------------------------------
// Workgroup reduction of K doubles, fixed order, result broadcast to all.
// red must hold (nwaves + 1) * K doubles.
template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* red) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[k] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w * K + k];
      red[nw * K + k] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = uni(red[nw * K + k]);
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <typename T>
__device__ __forceinline__ const T* nl_pick(const float* a, const double* b) {
  if constexpr (sizeof(T) == 4) return a;
  else return b;
}

// Nonlocal projections of one vector x (Background section, separable V_nl):
// c_p = chi_p^T x for every projector.  Each wave takes whole support groups
// (the projectors of a group share their support, so x is gathered once per
// group); lane 0 stores w_p = gamma_p h^3 c_p into coef (LDS) and adds
// sum_p w_p c_p = x^T V_nl x (unconjugated) to mu.  The caller synchronises
// before coef is read.
template <typename T, typename XT>
__device__ void nl_project(const NlArgs& nl, const typename V2<XT>::t* x,
                           typename V2<T>::t* coef, double& mu_re, double& mu_im) {
  const int lane = threadIdx.x & 63;
  const int wave = uni((int)(threadIdx.x >> 6));
  const int nw = (int)(blockDim.x >> 6);
  const T* bv = nl_pick<T>(nl.bv32, nl.bv64);
  for (int gi = wave; gi < nl.n_groups; gi += nw) {
    const int4 G = nl.ginfo[gi];
    const int s0 = uni(G.x), S = uni(G.y) - s0, p0 = uni(G.z), np = uni(G.w);
    const T* val = bv + uni(nl.gvoff[gi]);
    const int* idx = nl.bidx + s0;
    T ar[kMaxGroup], ai[kMaxGroup];
#pragma unroll
    for (int k = 0; k < kMaxGroup; ++k) { ar[k] = 0; ai[k] = 0; }
    for (int j = lane; j < S; j += 64) {
      const typename V2<XT>::t v = x[idx[j]];
      const T vr = (T)v.x, vi = (T)v.y;
#pragma unroll
      for (int k = 0; k < kMaxGroup; ++k) {
        if (k < np) {
          const T c = val[k * S + j];
          ar[k] += c * vr;
          ai[k] += c * vi;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxGroup; ++k) {
      if (k < np) {
        ar[k] = wave_sum(ar[k]);
        ai[k] = wave_sum(ai[k]);
        if (lane == 0) {
          const double gd = nl.gdv[p0 + k];
          const double cr = (double)ar[k], ci = (double)ai[k];
          const double wr = gd * cr, wi = gd * ci;
          typename V2<T>::t w;
          w.x = (T)wr;
          w.y = (T)wi;
          coef[p0 + k] = w;
          mu_re += wr * cr - wi * ci;
          mu_im += wr * ci + wi * cr;
        }
      }
    }
  }
}

// (V_nl x)_i = sum over the entries of point i of w_p chi_p(i), added to (ar, ai).
template <typename T>
__device__ __forceinline__ void nl_point(const int* pm_ptr, const int* pm_proj, const T* pm_v,
                                         const typename V2<T>::t* coef, long long i, T& ar,
                                         T& ai) {
  const int e1 = pm_ptr[i + 1];
  for (int e = pm_ptr[i]; e < e1; ++e) {
    const T c = pm_v[e];
    const typename V2<T>::t w = coef[pm_proj[e]];
    ar += c * w.x;
    ai += c * w.y;
  }
}

// ---------------------------------------------------------------------------
// x-marching stencil sweep over all tiles of one system.
//
// Pol provides (po = uniform plane offset, c = per-lane offset in the plane):
//   T2 load(size_t po, int c)  -- operand value at a point
//   Aux aux(size_t po, int c)  -- centre-only data (potential, right-hand side)
//   void center(size_t po, int c, T2 val, T2 nbr, const Aux&) -- nbr is the
//   sum of the off-centre stencil terms.
//
// Each thread keeps planes x-R .. x+R+PF of its column in a register FIFO
// whose slots rotate by compile-time phase (the x loop is unrolled by the
// FIFO length U), so no register moves are needed; planes are loaded PF steps
// before their first use.  The current plane sits in LDS with a compile-time
// row pitch PITCH, padded with R periodic copies on each side in z (and in y
// when one tile covers the whole plane), so all 24 in-plane neighbour reads
// are immediate offsets from one per-thread base address.
template <typename T> struct V2;

template <typename T, bool FULL, int HS, int PITCH, class Pol, int PPS>
struct Marcher {
  typedef typename V2<T>::t T2;
  typedef typename Pol::Aux AuxT;
  static constexpr int PF = Pol::kPF;
  static constexpr int U = QN + PF;   // FIFO: planes x-R .. x+R+PF
  static constexpr int PA = PF + 1;   // aux/halo pipelines: planes x .. x+PF
  // The x loop is unrolled by U, so a slot index (phase within the block) of
  // a pipeline of period PA equals x mod PA only if PA divides U
  // (PF in {1, 2, 3, 5} for the 13-plane stencil).
  static_assert(U % PA == 0, "prefetch depth must make PF+1 divide 2R+1+PF");

  static_assert(PPS == 1 || PPS == 2, "one or two planes per barrier");
  static_assert(U % PPS == 0, "plane pairs must not straddle the unrolled block");

  const Geom& g;
  const StencilCoef<T>& cf;
  Pol& pol;
  T2* buf0;            // plane buffers: 2 * PPS of them, bufs apart
  size_t bufs;         // elements per buffer
  size_t plane;
  int nx;
  bool own;
  int col;            // own column offset in the plane (gy*nz + z)
  int wbase;          // LDS index of the thread's stencil window (row rc-R, col z)
  int ci;             // LDS index of the own point
  int zpl, zpr;       // LDS indices of periodic copies in z (-1: none)
  int ypl, ypr;       // ... and in y (whole-plane tiles only)
  bool hv[HS];
  int hl[HS];         // LDS index of halo points
  int hcol[HS];       // halo column offsets in the plane
  T2 fifo[U];
  AuxT ax[PA];
  T2 hq[HS][PA];

  __device__ __forceinline__ static int wrapx(int p, int n) { return p >= n ? p - n : p; }

  // store plane x (FIFO phase PH) into buf
  template <int PH>
  __device__ __forceinline__ void put(T2* buf) {
    const T2 c = fifo[(PH + R) % U];
    if (own) {
      buf[ci] = c;
      if (zpl >= 0) buf[zpl] = c;
      if (zpr >= 0) buf[zpr] = c;
      if (FULL) {
        if (ypl >= 0) buf[ypl] = c;
        if (ypr >= 0) buf[ypr] = c;
      }
    }
#pragma unroll
    for (int h = 0; h < HS; ++h)
      if (hv[h]) buf[hl[h]] = hq[h][PH % PA];
  }

  // PPS consecutive planes x, x+1 share one barrier: both are stored into
  // their own buffers of the current set, then both are computed.  TAIL: the
  // block may end inside the pair (only the last block of a march).
  template <int PH, bool TAIL>
  __device__ __forceinline__ void step(int x) {
    T2* set = buf0 + (size_t)(((x / PPS) & 1) * PPS) * bufs;
    const bool second = PPS == 2 && (!TAIL || x + 1 < nx);
    put<PH>(set);
    if (second) put<PH + 1>(set + bufs);
    __syncthreads();
    point<PH>(x, set);
    if (second) point<PH + 1>(x + 1, set + bufs);
  }

  template <int PH>
  __device__ __forceinline__ void point(int x, const T2* buf) {
    const T2 c = fifo[(PH + R) % U];
    if (own) {
      const T2* w = buf + wbase;
      T xr = 0, xi = 0, yr = 0, yi = 0, zr = 0, zi = 0;
#pragma unroll
      for (int k = 1; k <= R; ++k) {
        const T2 a = fifo[(PH + R - k) % U];
        const T2 b = fifo[(PH + R + k) % U];
        xr += cf.w[k] * (a.x + b.x);
        xi += cf.w[k] * (a.y + b.y);
      }
#pragma unroll
      for (int k = 1; k <= R; ++k) {
        const T2 a = w[(R - k) * PITCH + R];
        const T2 b = w[(R + k) * PITCH + R];
        yr += cf.w[k] * (a.x + b.x);
        yi += cf.w[k] * (a.y + b.y);
      }
#pragma unroll
      for (int k = 1; k <= R; ++k) {
        const T2 a = w[R * PITCH + R - k];
        const T2 b = w[R * PITCH + R + k];
        zr += cf.w[k] * (a.x + b.x);
        zi += cf.w[k] * (a.y + b.y);
      }
      const T sx = cf.sx * xr + cf.sy * yr + cf.sz * zr;
      const T sy = cf.sx * xi + cf.sy * yi + cf.sz * zi;
      pol.center((size_t)x * plane, col, c, mk2(sx, sy), ax[PH % PA]);
    }
    // refill the pipelines: the FIFO slot of plane x-R takes plane x+R+PF+1,
    // the aux/halo slot of plane x takes plane x+PF+1.  The loads are issued
    // unconditionally (past the last plane they re-read plane nx-1, and
    // threads without a column read valid addresses whose values are never
    // used): with no branch around them the compiler can count the loads in
    // flight and wait only for the one a value comes from.
    const int xn = x + PF + 1;
    const int xc = xn < nx ? xn : nx - 1;
    fifo[PH % U] = pol.load((size_t)wrapx(xc + R, nx) * plane, col);
    ax[PH % PA] = pol.aux((size_t)xc * plane, col);
#pragma unroll
    for (int h = 0; h < HS; ++h) hq[h][PH % PA] = pol.load((size_t)xc * plane, hcol[h]);
  }

  // U planes from x; full blocks need no bounds checks between steps
  template <int PH>
  __device__ __forceinline__ void block_full(int x) {
    if constexpr (PH < U) {
      step<PH, false>(x);
      block_full<PH + PPS>(x + PPS);
    }
  }

  template <int PH>
  __device__ __forceinline__ void block(int x) {
    if constexpr (PH < U) {
      if (x < nx) {
        step<PH, true>(x);
        block<PH + PPS>(x + PPS);
      }
    }
  }

  __device__ __forceinline__ void run(int t_begin, int t_end) {
    const int tid = threadIdx.x;
    const int ny = g.ny, nz = g.nz, ty = g.ty;
    own = tid < ty * nz;
    const int ly = own ? tid / nz : 0;
    const int z = own ? tid - ly * nz : 0;
    const int nhalo = FULL ? 0 : 2 * R * nz;
    int hrow[HS], hz[HS];
#pragma unroll
    for (int h = 0; h < HS; ++h) {
      const int hid = tid + h * (int)blockDim.x;
      hv[h] = hid < nhalo;
      const int hr = hv[h] ? hid / nz : 0;
      hz[h] = hv[h] ? hid - hr * nz : 0;
      hrow[h] = hr;
      hl[h] = (hr < R ? hr : ty + hr) * PITCH + hz[h] + R;
    }
    for (int t = t_begin; t < t_end; ++t) {
      const int y0 = t * ty;
      const int gy = y0 + ly;
      col = gy * nz + z;
      const int rc = (FULL ? gy : ly) + R;
      ci = rc * PITCH + z + R;
      wbase = (rc - R) * PITCH + z;
      // a point is copied into the left pad if it is among the last R of the
      // row and into the right pad if among the first R (both when nz < 2R)
      zpl = z >= nz - R ? rc * PITCH + z + R - nz : -1;
      zpr = z < R ? rc * PITCH + z + R + nz : -1;
      ypl = -1;
      ypr = -1;
      if (FULL) {
        ypl = gy >= ny - R ? (gy + R - ny) * PITCH + z + R : -1;
        ypr = gy < R ? (gy + R + ny) * PITCH + z + R : -1;
      }
#pragma unroll
      for (int h = 0; h < HS; ++h) {
        int gr = hrow[h] < R ? y0 - R + hrow[h] : y0 + ty + (hrow[h] - R);
        gr = gr < 0 ? gr + ny : (gr >= ny ? gr - ny : gr);
        hcol[h] = gr * nz + hz[h];
      }
      // prologue: FIFO slot j holds plane j - R (phase 0); aux/halo slot j plane j
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int px = ((j - R) % nx + nx) % nx;
        fifo[j] = own ? pol.load((size_t)px * plane, col) : zero2<T2>();
      }
#pragma unroll
      for (int j = 0; j < PA; ++j) {
        ax[j] = own ? pol.aux((size_t)j * plane, col) : AuxT();
#pragma unroll
        for (int h = 0; h < HS; ++h)
          hq[h][j] = hv[h] ? pol.load((size_t)j * plane, hcol[h]) : zero2<T2>();
      }
      int x = 0;
      for (; x + U <= nx; x += U) block_full<0>(x);
      if (x < nx) block<0>(x);
      __syncthreads();
    }
  }
};

// FP32 sweeps march two planes per barrier (four plane buffers), FP64 ones one.
template <typename T>
constexpr int planes_per_step() { return sizeof(T) == 4 ? 2 : 1; }

template <typename T, bool FULL, int HS, int PITCH, class Pol>
__device__ __forceinline__ void march(const Geom& g, const StencilCoef<T>& cf, Pol& pol,
                                      typename V2<T>::t* lds, int t_begin, int t_end) {
  const int rows = (FULL ? g.ny : g.ty) + 2 * R;
  Marcher<T, FULL, HS, PITCH, Pol, planes_per_step<T>()> m{g, cf, pol};
  m.buf0 = lds;
  m.bufs = (size_t)rows * PITCH;
  m.plane = (size_t)g.ny * g.nz;
  m.nx = g.nx;
  m.run(t_begin, t_end);
}

// Register-light variant for the occasional FP64 residual sweep: no x queue;
// the 12 x neighbours are read through the caches (they were read moments
// before by the neighbouring planes' steps), y/z neighbours from the LDS plane.
template <typename T, bool FULL, int HS, class Pol>
__device__ __forceinline__ void march_light(const Geom& g, const StencilCoef<T>& cf, Pol& pol,
                                            typename V2<T>::t* lds, int t_begin, int t_end) {
  typedef typename V2<T>::t T2;
  typedef typename Pol::Aux AuxT;
  const int tid = threadIdx.x;
  const int nx = g.nx, ny = g.ny, nz = g.nz, ty = g.ty;
  const int ncol = ty * nz;
  const bool own = tid < ncol;
  const int ly = own ? tid / nz : 0;
  const int z = own ? tid - ly * nz : 0;
  const int rows = FULL ? ny : ty + 2 * R;
  const size_t plane = (size_t)ny * nz;
  const int nhalo = FULL ? 0 : 2 * R * nz;
  int hl[HS], hoff_r[HS], hz[HS];
  bool hv[HS];
#pragma unroll
  for (int j = 0; j < HS; ++j) {
    const int hid = tid + j * (int)blockDim.x;
    hv[j] = hid < nhalo;
    const int hr = hv[j] ? hid / nz : 0;
    hz[j] = hv[j] ? hid - hr * nz : 0;
    hoff_r[j] = hr;
    hl[j] = (hr < R ? hr : ty + hr) * nz + hz[j];
  }
  for (int t = t_begin; t < t_end; ++t) {
    const int y0 = t * ty;
    const int gy = y0 + ly;
    const size_t col = (size_t)gy * nz + z;
    int hrowoff[HS];
#pragma unroll
    for (int j = 0; j < HS; ++j) {
      int gr = hoff_r[j] < R ? y0 - R + hoff_r[j] : y0 + ty + (hoff_r[j] - R);
      gr = gr < 0 ? gr + ny : (gr >= ny ? gr - ny : gr);
      hrowoff[j] = gr * nz + hz[j];
    }
    const int rc = FULL ? gy : ly + R;
    for (int x = 0; x < nx; ++x) {
      T2* buf = lds + (x & 1) * rows * nz;
      const size_t po = (size_t)x * plane;
      const T2 c = own ? pol.load(po, (int)col) : zero2<T2>();
      if (own) buf[rc * nz + z] = c;
#pragma unroll
      for (int h = 0; h < HS; ++h)
        if (hv[h]) buf[hl[h]] = pol.load(po, hrowoff[h]);
      __syncthreads();
      if (own) {
        const AuxT axv = pol.aux(po, (int)col);
        T xr = 0, xi = 0, yr = 0, yi = 0, zr = 0, zi = 0;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          int xp = x + k, xm = x - k;
          xp -= xp >= nx ? nx : 0;
          xm += xm < 0 ? nx : 0;
          const T2 a = pol.load((size_t)xp * plane, (int)col);
          const T2 b = pol.load((size_t)xm * plane, (int)col);
          xr += cf.w[k] * (a.x + b.x);
          xi += cf.w[k] * (a.y + b.y);
        }
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          int up = rc + k, dn = rc - k;
          if (FULL) { up -= up >= ny ? ny : 0; dn += dn < 0 ? ny : 0; }
          const T2 a = buf[up * nz + z];
          const T2 b = buf[dn * nz + z];
          yr += cf.w[k] * (a.x + b.x);
          yi += cf.w[k] * (a.y + b.y);
        }
        const int rz = rc * nz;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          int zp = z + k, zm = z - k;
          zp -= zp >= nz ? nz : 0;
          zm += zm < 0 ? nz : 0;
          const T2 a = buf[rz + zp];
          const T2 b = buf[rz + zm];
          zr += cf.w[k] * (a.x + b.x);
          zi += cf.w[k] * (a.y + b.y);
        }
        const T sx = cf.sx * xr + cf.sy * yr + cf.sz * zr;
        const T sy = cf.sx * xi + cf.sy * yi + cf.sz * zi;
        pol.center(po, (int)col, c, mk2(sx, sy), axv);
      }
    }
    __syncthreads();
  }
}

// Bytes of LDS used by the plane buffers: the largest of the FIFO march (T of
// the COCG iterations, padded pitch) and the FP64 light march (unpadded).
__host__ __device__ inline size_t lds_plane_bytes(const Geom& g, int pitch, bool fp32_iter) {
  const bool full = g.ty == g.ny;
  const size_t rows_pad = (size_t)(full ? g.ny : g.ty) + 2 * R;
  const size_t rows_light = full ? (size_t)g.ny : (size_t)g.ty + 2 * R;
  const size_t main = fp32_iter ? 2 * planes_per_step<float>() * rows_pad * pitch * sizeof(float2)
                                : 2 * planes_per_step<double>() * rows_pad * pitch * sizeof(double2);
  const size_t light = 2 * rows_light * g.nz * sizeof(double2);
  size_t b = main > light ? main : light;
  if (g.prec) {
    // the preconditioner's planes (FP64 for the FP64 solver, which the FP32
    // path also launches for the systems it hands over)
    const size_t pb = prec_lds_bytes(g, fp32_iter ? sizeof(float) : sizeof(double));
    b = b > pb ? b : pb;
  }
  return (b + 255) & ~(size_t)255;
}

// Bytes of LDS for the reductions (4 doubles per wave plus the result).
__host__ __device__ inline size_t red_bytes(int block) {
  const size_t nw = (size_t)(block + 63) / 64;
  return ((nw + 1) * 4 * sizeof(double) + 255) & ~(size_t)255;
}

// ---------------------------------------------------------------------------
// Policies

// FP64 residual r = b - (H - sigma) x with b = -psi_n (.) u; stores r in TI.
template <typename TI, bool NL>
struct ResidPol {
  typedef typename V2<TI>::t TI2;
  const double2* x;
  const double* v;
  const double* psi;
  const double* u;
  TI2* r;
  double c0, eps, om;
  double rr, bb, rho_re, rho_im;
  const int* pm_ptr;              // point-major projector entries (NL)
  const int* pm_proj;
  const double* pm_v;
  const double2* coef;            // w_p of x (LDS)
  static constexpr int kPF = 1;   // runs a few times per solve: keep registers low
  struct Aux { double v, b; };
  __device__ double2 load(size_t po, int c) const { return (x + po)[c]; }
  __device__ Aux aux(size_t po, int c) const {
    Aux a;
    a.v = (v + po)[c];
    a.b = -(psi + po)[c] * (u + po)[c];
    return a;
  }
  __device__ void center(size_t po, int c, double2 xv, double2 nb, const Aux& ax) {
    const double a = c0 + ax.v - eps;
    double axr = a * xv.x + om * xv.y + nb.x;
    double axi = a * xv.y - om * xv.x + nb.y;
    if constexpr (NL) nl_point<double>(pm_ptr, pm_proj, pm_v, coef, (long long)po + c, axr, axi);
    const double bval = ax.b;
    const double rx = bval - axr;
    const double ry = -axi;
    TI2 rs; rs.x = (TI)rx; rs.y = (TI)ry;
    (r + po)[c] = rs;
    rr += rx * rx + ry * ry;
    bb += bval * bval;
    const double sx = (double)rs.x, sy = (double)rs.y;
    rho_re += sx * sx - sy * sy;
    rho_im += 2.0 * sx * sy;
  }
};

// COCG sweep A: p = r + beta p_old (formed on load), q = (H - sigma) p.
template <typename T>
struct ApplyPol {
  typedef typename V2<T>::t T2;
  const T2* r;
  const T2* pold;
  T2* pnew;
  T2* q;
  const T* v;
  T c0, eps, om;
  T br, bi;
  bool first;
  double mu_re, mu_im;
  // FP32: two planes per barrier already give the loads a plane of slack
  static constexpr int kPF = sizeof(T) == 4 ? 1 : 2;
  typedef T Aux;
  __device__ T aux(size_t po, int c) const { return (v + po)[c]; }
  __device__ T2 load(size_t po, int c) const {
    T2 rv = (r + po)[c];
    if (first) return rv;
    const T2 pv = (pold + po)[c];
    rv.x += br * pv.x - bi * pv.y;
    rv.y += br * pv.y + bi * pv.x;
    return rv;
  }
  __device__ void center(size_t po, int c, T2 pv, T2 nb, const T& vv) {
    const T a = c0 + vv - eps;
    T2 h;
    h.x = a * pv.x + om * pv.y + nb.x;
    h.y = a * pv.y - om * pv.x + nb.y;
    (pnew + po)[c] = pv;
    (q + po)[c] = h;
    mu_re += (double)(pv.x * h.x - pv.y * h.y);
    mu_im += (double)(pv.x * h.y + pv.y * h.x);
  }
};

// COCG sweep A without forming p as planes arrive: the stencil acts on r
// only, and since A is linear, q = A p = A r + beta q_old with q_old = A p_old;
// p = r + beta p_old and q are formed at the centre point from p_old and
// q_old, which come through the centre pipeline like V.  Nothing is computed
// from a value as soon as it is loaded, so the loads of later planes stay in
// flight across steps.  q is updated in place (only its centre point is read).
template <typename T>
struct RecurPol {
  typedef typename V2<T>::t T2;
  const T2* r;
  const T2* pold;
  T2* pnew;
  T2* q;
  const T* v;
  T c0, eps, om;
  T br, bi;
  bool first;                     // p = r, q = A r (p_old and q_old are not used)
  double mu_re, mu_im;
  static constexpr int kPF = 1;
  struct Aux { T v; T2 p, q; };
  __device__ Aux aux(size_t po, int c) const {
    Aux a;
    a.v = (v + po)[c];
    a.p = (pold + po)[c];
    a.q = (q + po)[c];
    return a;
  }
  __device__ T2 load(size_t po, int c) const { return (r + po)[c]; }
  __device__ void center(size_t po, int c, T2 rv, T2 nb, const Aux& ax) {
    const T a = c0 + ax.v - eps;
    T2 w, pv, qv;
    w.x = a * rv.x + om * rv.y + nb.x;
    w.y = a * rv.y - om * rv.x + nb.y;
    pv.x = rv.x + br * ax.p.x - bi * ax.p.y;
    pv.y = rv.y + br * ax.p.y + bi * ax.p.x;
    qv.x = w.x + br * ax.q.x - bi * ax.q.y;
    qv.y = w.y + br * ax.q.y + bi * ax.q.x;
    if (first) { pv = rv; qv = w; }
    (pnew + po)[c] = pv;
    (q + po)[c] = qv;
    mu_re += (double)(pv.x * qv.x - pv.y * qv.y);
    mu_im += (double)(pv.x * qv.y + pv.y * qv.x);
  }
};

// Plain operator application (test hook and stencil measurement); the
// vectors are stored in the compute precision.
template <typename T>
struct HPol {
  typedef typename V2<T>::t T2;
  const T2* x;
  T2* y;
  const T* v;
  T c0, sr, si;
  static constexpr int kPF = sizeof(T) == 4 ? 3 : 2;
  typedef T Aux;
  __device__ T aux(size_t po, int c) const { return (v + po)[c]; }
  __device__ T2 load(size_t po, int c) const { return (x + po)[c]; }
  __device__ void center(size_t po, int c, T2 xv, T2 nb, const T& vv) {
    const T a = c0 + vv - sr;
    T2 o;
    o.x = a * xv.x + si * xv.y + nb.x;
    o.y = a * xv.y - si * xv.x + nb.y;
    (y + po)[c] = o;
  }
};

// ---------------------------------------------------------------------------
// Streaming passes of one system (whole workgroup).

// Point-major nonlocal entries and the coefficients w_p of p (null: none).
template <typename T>
struct NlPoint {
  const int* ptr;
  const int* proj;
  const T* v;
  const typename V2<T>::t* coef;
};

// x (XT) = first ? alpha p : x + alpha p;  r -= alpha q;  returns ||r||^2, r^T r.
// With a nonlocal term, q holds (H_loc - sigma) p and V_nl p is added here.
// Four elements per thread per trip, all loads issued before the arithmetic.
template <typename T, typename XT, bool NL>
__device__ __forceinline__ void update_sweep(long long N, typename V2<XT>::t* x,
                                             const typename V2<T>::t* p, typename V2<T>::t* r,
                                             const typename V2<T>::t* q, T ar, T ai, bool first,
                                             const NlPoint<T>& nl, double& rr, double& rho_re,
                                             double& rho_im) {
  typedef typename V2<T>::t T2;
  typedef typename V2<XT>::t X2;
  constexpr int U = 4;
  const long long st = blockDim.x;
  long long i0 = threadIdx.x;
  for (; i0 + (U - 1) * st < N; i0 += U * st) {
    T2 pv[U], qv[U], rv[U];
    X2 xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * st;
      pv[u] = p[i];
      qv[u] = q[i];
      rv[u] = r[i];
      if (!first) xv[u] = x[i];
    }
    if constexpr (NL) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        nl_point<T>(nl.ptr, nl.proj, nl.v, nl.coef, i0 + u * st, qv[u].x, qv[u].y);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * st;
      const T dx = ar * pv[u].x - ai * pv[u].y;
      const T dy = ar * pv[u].y + ai * pv[u].x;
      if (first) { xv[u].x = (XT)dx; xv[u].y = (XT)dy; }
      else { xv[u].x += (XT)dx; xv[u].y += (XT)dy; }
      x[i] = xv[u];
      rv[u].x -= ar * qv[u].x - ai * qv[u].y;
      rv[u].y -= ar * qv[u].y + ai * qv[u].x;
      r[i] = rv[u];
      const double sx = (double)rv[u].x, sy = (double)rv[u].y;
      rr += sx * sx + sy * sy;
      rho_re += sx * sx - sy * sy;
      rho_im += 2.0 * sx * sy;
    }
  }
  for (long long i = i0; i < N; i += st) {
    const T2 pv = p[i];
    T2 qv = q[i];
    T2 rv = r[i];
    if constexpr (NL) nl_point<T>(nl.ptr, nl.proj, nl.v, nl.coef, i, qv.x, qv.y);
    const T dx = ar * pv.x - ai * pv.y;
    const T dy = ar * pv.y + ai * pv.x;
    X2 xv;
    if (first) { xv.x = (XT)dx; xv.y = (XT)dy; }
    else { xv = x[i]; xv.x += (XT)dx; xv.y += (XT)dy; }
    x[i] = xv;
    rv.x -= ar * qv.x - ai * qv.y;
    rv.y -= ar * qv.y + ai * qv.x;
    r[i] = rv;
    const double sx = (double)rv.x, sy = (double)rv.y;
    rr += sx * sx + sy * sy;
    rho_re += sx * sx - sy * sy;
    rho_im += 2.0 * sx * sy;
  }
}

__device__ __forceinline__ void fold_sweep(long long N, double2* x, const float2* d) {
  for (long long i = threadIdx.x; i < N; i += blockDim.x) {
    double2 a = x[i];
    const float2 b = d[i];
    a.x += (double)b.x; a.y += (double)b.y;
    x[i] = a;
  }
}

__device__ __forceinline__ void zero_sweep(long long N, double2* x) {
  for (long long i = threadIdx.x; i < N; i += blockDim.x) x[i] = make_double2(0.0, 0.0);
}

// complex division a / b
__device__ __forceinline__ void cdiv(double ar, double ai, double br, double bi, double& cr,
                                     double& ci) {
  const double den = br * br + bi * bi;
  cr = (ar * br + ai * bi) / den;
  ci = (ai * br - ar * bi) / den;
}

__device__ __forceinline__ void record(const CocgArgs& a, int s, int its, int cycles, int status) {
  // per-frequency statistics of finished solves; a solve the FP32 launch hands
  // over (status 3) is counted once, by the FP64 launch, with the FP32
  // iterations (still in out_iters) added; reliable updates are summed per bin
  if (a.ostats != nullptr && status != 3) {
    unsigned long long tot = (unsigned long long)its, cyc = (unsigned long long)cycles;
    if (a.is_followup) {
      tot += (unsigned long long)a.out_iters[s];
      cyc += (unsigned long long)a.out_cycles[s];
    }
    const int nb = a.n_bins;
    const int bin = a.obin[s / a.n_occ];
    atomicAdd(&a.ostats[bin], 1ULL);
    atomicAdd(&a.ostats[nb + bin], tot);
    atomicAdd(&a.ostats[2 * nb + bin], tot * tot);
    atomicMin(&a.ostats[3 * nb + bin], tot);
    atomicMax(&a.ostats[4 * nb + bin], tot);
    atomicAdd(&a.ostats[5 * nb + bin], cyc);
  }
  a.out_iters[s] = its;
  a.out_cycles[s] = cycles;
  a.out_status[s] = status;
  atomicAdd(&a.stats[0], (unsigned long long)its);
  atomicMax(&a.stats[1], (unsigned long long)its);
  atomicAdd(&a.stats[2], (unsigned long long)cycles);
  if (status == 1) atomicAdd(&a.stats[3], 1ULL);
  if (status == 2) atomicAdd(&a.stats[4], 1ULL);
  if (status == 3) atomicAdd(&a.stats[5], 1ULL);
}

// ---------------------------------------------------------------------------
// One system, FP64 throughout.
template <bool FULL, int HS, int PITCH, bool NL, bool PC>
__device__ void solve_fp64(const CocgArgs& a, int s, char* smem, double* red, char* nlc) {
  const Geom& g = a.g;
  const long long N = g.N;
  const int b = s / a.n_occ;
  const int n = s - b * a.n_occ;
  double2* lds = reinterpret_cast<double2*>(smem);
  double2* ws = reinterpret_cast<double2*>(a.slot_ws + (size_t)blockIdx.x * a.slot_bytes);
  double2* r = ws;
  double2* q = ws + N;
  double2* pa = ws + 2 * N;
  double2* pb = ws + 3 * N;
  double2* x = a.x64 + (size_t)s * N;
  const double eps = a.eps[n];
  const double om = a.omega[b];
  // preconditioned COCG: z = M^-1 r is the stencil operand and rho = r^T z
  constexpr bool pc = PC;
  double2* z = pc ? ws + 4 * N : r;
  double2* tt = ws + 5 * N;
  const double psr = pc ? fmax(a.prec->vbar - eps, a.prec->floor) : 0.0, psi = -om;

  double2* coef = reinterpret_cast<double2*>(nlc);
  NlPoint<double> nlp{a.nl.pm_ptr, a.nl.pm_proj, a.nl.pm_v64, coef};

  ResidPol<double, NL> rp;
  rp.x = x; rp.v = a.v64; rp.psi = a.psi64 + (size_t)n * N; rp.u = a.u64 + (size_t)b * N;
  rp.r = r; rp.c0 = a.c64.c0; rp.eps = eps; rp.om = om;
  rp.rr = rp.bb = rp.rho_re = rp.rho_im = 0.0;
  rp.pm_ptr = a.nl.pm_ptr; rp.pm_proj = a.nl.pm_proj; rp.pm_v = a.nl.pm_v64;
  rp.coef = coef;
  if constexpr (NL) {
    double d0 = 0.0, d1 = 0.0;
    nl_project<double, double>(a.nl, x, coef, d0, d1);
    __syncthreads();
  }
  march_light<double, FULL, HS>(g, a.c64, rp, lds, 0, g.ntiles);
  double v4[4] = {rp.rr, rp.bb, rp.rho_re, rp.rho_im};
  block_reduce<4>(v4, red);
  const double bnorm = sqrt(v4[1]);
  double rnorm = sqrt(v4[0]);
  double rho_r = v4[2], rho_i = v4[3];
  int its = 0, status = 0;
  if (bnorm == 0.0) {
    zero_sweep(N, x);
  } else {
    const double thr = a.tol * bnorm;
    if constexpr (PC) {
      if (rnorm > thr) {
        double q2[2] = {0.0, 0.0};
        precond_apply<double>(g, a.prec, r, tt, z, psr, psi, smem, q2[0], q2[1]);
        block_reduce<2>(q2, red);
        rho_r = q2[0];
        rho_i = q2[1];
      }
    }
    double br = 0.0, bi = 0.0;
    bool first = true;
    double2* pold = pa;
    double2* pnew = pb;
    while (rnorm > thr) {
      if (its >= a.maxit) { status = 1; break; }
      ApplyPol<double> ap;
      ap.r = z; ap.pold = pold; ap.pnew = pnew; ap.q = q; ap.v = a.v64;
      ap.c0 = a.c64.c0; ap.eps = eps; ap.om = om; ap.br = br; ap.bi = bi; ap.first = first;
      ap.mu_re = ap.mu_im = 0.0;
      march<double, FULL, HS, PITCH>(g, a.c64, ap, lds, 0, g.ntiles);
      double m2[2] = {ap.mu_re, ap.mu_im};
      if constexpr (NL) nl_project<double, double>(a.nl, pnew, coef, m2[0], m2[1]);
      block_reduce<2>(m2, red);
      if (fabs(m2[0]) + fabs(m2[1]) < 1e-300) { status = 2; break; }
      double al_r, al_i;
      cdiv(rho_r, rho_i, m2[0], m2[1], al_r, al_i);
      double rr = 0.0, nr = 0.0, ni = 0.0;
      update_sweep<double, double, NL>(N, x, pnew, r, q, al_r, al_i, false, nlp, rr, nr, ni);
      double u3[3] = {rr, nr, ni};
      block_reduce<3>(u3, red);
      ++its;
      rnorm = sqrt(u3[0]);
      if constexpr (PC) {
        if (rnorm > thr) {
          double q2[2] = {0.0, 0.0};
          precond_apply<double>(g, a.prec, r, tt, z, psr, psi, smem, q2[0], q2[1]);
          block_reduce<2>(q2, red);
          u3[1] = q2[0];
          u3[2] = q2[1];
          if (fabs(u3[1]) + fabs(u3[2]) < 1e-300) { status = 2; break; }
        }
      }
      cdiv(u3[1], u3[2], rho_r, rho_i, br, bi);
      rho_r = u3[1]; rho_i = u3[2];
      first = false;
      double2* t = pold; pold = pnew; pnew = t;
    }
    if (status == 0 && !(rnorm <= thr)) status = 1;   // NaN residual is not convergence
  }
  if (threadIdx.x == 0) record(a, s, its, 0, status);
}

// One system, FP32 COCG with reliable updates (Sleijpen and van der Vorst,
// 1996): the search direction is kept for the whole solve, while every time
// the FP32 recursive residual has dropped by the factor delta (inner_tol) the
// FP32 correction d is folded into the FP64 solution and the residual is
// replaced by the true FP64 residual b - A x64.  Convergence is declared on
// the FP64 residual only.
template <bool FULL, int HS, int PITCH, bool NL, bool PC>
__device__ void solve_refine(const CocgArgs& a, int s, char* smem, double* red, char* nlc) {
  const Geom& g = a.g;
  const long long N = g.N;
  const int b = s / a.n_occ;
  const int n = s - b * a.n_occ;
  float2* ws = reinterpret_cast<float2*>(a.slot_ws + (size_t)blockIdx.x * a.slot_bytes);
  float2* r = ws;
  float2* q = ws + N;
  float2* pa = ws + 2 * N;
  float2* pb = ws + 3 * N;
  float2* d = ws + 4 * N;
  double2* x = a.x64 + (size_t)s * N;
  const double eps = a.eps[n];
  const double om = a.omega[b];
  // preconditioned COCG: z = M^-1 r is the stencil operand and rho = r^T z
  constexpr bool pc = PC;
  float2* z = pc ? ws + 5 * N : r;
  float2* tt = ws + 6 * N;
  const float psr = pc ? (float)fmax(a.prec->vbar - eps, a.prec->floor) : 0.f, psi = (float)(-om);

  // nonlocal coefficients: FP64 for the residual sweeps, FP32 for the inner
  // iterations (same LDS region, never live at the same time)
  double2* coef64 = reinterpret_cast<double2*>(nlc);
  float2* coef32 = reinterpret_cast<float2*>(nlc);
  NlPoint<float> nlp{a.nl.pm_ptr, a.nl.pm_proj, a.nl.pm_v32, coef32};

  ResidPol<float, NL> rp;
  rp.x = x; rp.v = a.v64; rp.psi = a.psi64 + (size_t)n * N; rp.u = a.u64 + (size_t)b * N;
  rp.r = r; rp.c0 = a.c64.c0; rp.eps = eps; rp.om = om;
  rp.rr = rp.bb = rp.rho_re = rp.rho_im = 0.0;
  rp.pm_ptr = a.nl.pm_ptr; rp.pm_proj = a.nl.pm_proj; rp.pm_v = a.nl.pm_v64;
  rp.coef = coef64;
  if constexpr (NL) {
    double d0 = 0.0, d1 = 0.0;
    nl_project<double, double>(a.nl, x, coef64, d0, d1);
    __syncthreads();
  }
  march_light<double, FULL, HS>(g, a.c64, rp, reinterpret_cast<double2*>(smem), 0, g.ntiles);
  double v4[4] = {rp.rr, rp.bb, rp.rho_re, rp.rho_im};
  block_reduce<4>(v4, red);
  const double bnorm = sqrt(v4[1]);
  double rnorm = sqrt(v4[0]);      // current residual estimate
  double rho_r = v4[2], rho_i = v4[3];
  int its = 0, updates = 0, status = 0;
  bool failed = false;             // FP32 iteration produced a non-finite value
  if (bnorm == 0.0) {
    zero_sweep(N, x);
  } else {
    const double thr = a.tol * bnorm;
    const double delta = a.inner_tol;
    double rmax = rnorm;           // true residual at the last update
    double best_true = rnorm;      // smallest true residual seen
    int no_gain = 0;               // updates in a row without progress
    int last_upd = 0;              // iteration of the last update
    double br = 0.0, bi = 0.0;
    bool first = true;             // p = r (no previous direction)
    bool dfresh = true;            // d holds nothing yet
    bool exact_q = false;          // q = A p directly (after a residual replacement)
    float2* pold = pa;
    float2* pnew = pb;
    if constexpr (PC) {
      if (rnorm > thr) {
        double q2[2] = {0.0, 0.0};
        precond_apply<float>(g, a.prec, r, tt, z, psr, psi, smem, q2[0], q2[1]);
        block_reduce<2>(q2, red);
        rho_r = q2[0];
        rho_i = q2[1];
      }
    }
    while (rnorm > thr) {
      if (its >= a.maxit32) { status = 1; break; }
      double m2[2];
      // the direct form also serves tiles with two halo slots per thread, and
      // the preconditioned solver: there the recurrence form's larger centre
      // pipeline is kept in scratch memory
      if (exact_q || HS == 2 || PC) {
        // bound the drift of the q recurrence: one sweep with p formed on load
        ApplyPol<float> ap;
        ap.r = z; ap.pold = pold; ap.pnew = pnew; ap.q = q; ap.v = a.v32;
        ap.c0 = a.c32.c0; ap.eps = (float)eps; ap.om = (float)om; ap.br = (float)br;
        ap.bi = (float)bi; ap.first = first;
        ap.mu_re = ap.mu_im = 0.0;
        march<float, FULL, HS, PITCH>(g, a.c32, ap, reinterpret_cast<float2*>(smem), 0, g.ntiles);
        m2[0] = ap.mu_re; m2[1] = ap.mu_im;
        exact_q = false;
      } else {
        RecurPol<float> ap;
        ap.r = z; ap.pold = pold; ap.pnew = pnew; ap.q = q; ap.v = a.v32;
        ap.c0 = a.c32.c0; ap.eps = (float)eps; ap.om = (float)om; ap.br = (float)br;
        ap.bi = (float)bi; ap.first = first;
        ap.mu_re = ap.mu_im = 0.0;
        march<float, FULL, HS, PITCH>(g, a.c32, ap, reinterpret_cast<float2*>(smem), 0, g.ntiles);
        m2[0] = ap.mu_re; m2[1] = ap.mu_im;
      }
      if constexpr (NL) nl_project<float, float>(a.nl, pnew, coef32, m2[0], m2[1]);
      block_reduce<2>(m2, red);
      if (!isfinite(m2[0]) || !isfinite(m2[1])) { failed = true; break; }
      if (fabs(m2[0]) + fabs(m2[1]) < 1e-300) { status = 2; break; }
      double al_r, al_i;
      cdiv(rho_r, rho_i, m2[0], m2[1], al_r, al_i);
      double rr = 0.0, nr = 0.0, ni = 0.0;
      update_sweep<float, float, NL>(N, d, pnew, r, q, (float)al_r, (float)al_i, dfresh, nlp, rr,
                                     nr, ni);
      double u3[3] = {rr, nr, ni};
      block_reduce<3>(u3, red);
      ++its;
      dfresh = false;
      double rn = sqrt(u3[0]);
      double rho_nr = u3[1], rho_ni = u3[2];
      if (!isfinite(rn) || !isfinite(rho_nr) || !isfinite(rho_ni)) { failed = true; break; }
      // reliable update when the recursive residual has dropped by delta, on
      // apparent convergence, and at least every kMaxGap iterations (an FP32
      // recursion that stalls above delta * rmax is caught there)
      if ((rn < delta * rmax && its - last_upd >= kMinGap) || rn <= thr ||
          its - last_upd >= kMaxGap) {
        // reliable update: x64 += d; r = b - A x64 in FP64 (stored rounded to FP32)
        fold_sweep(N, x, d);
        __syncthreads();
        dfresh = true;
        ++updates;
        last_upd = its;
        rp.rr = rp.bb = rp.rho_re = rp.rho_im = 0.0;
        if constexpr (NL) {
          double d0 = 0.0, d1 = 0.0;
          nl_project<double, double>(a.nl, x, coef64, d0, d1);
          __syncthreads();
        }
        march_light<double, FULL, HS>(g, a.c64, rp, reinterpret_cast<double2*>(smem), 0, g.ntiles);
        double w4[4] = {rp.rr, rp.bb, rp.rho_re, rp.rho_im};
        block_reduce<4>(w4, red);
        rn = sqrt(w4[0]);
        rho_nr = w4[2];
        rho_ni = w4[3];
        rmax = rn;
        exact_q = true;
        if (rn < 0.5 * best_true) { best_true = rn; no_gain = 0; }
        else if (++no_gain >= 4) { rnorm = rn; status = 1; break; }   // FP32 stagnation
      }
      if constexpr (PC) {
        if (rn > thr) {
          double q2[2] = {0.0, 0.0};
          precond_apply<float>(g, a.prec, r, tt, z, psr, psi, smem, q2[0], q2[1]);
          block_reduce<2>(q2, red);
          rho_nr = q2[0];
          rho_ni = q2[1];
          if (!isfinite(rho_nr) || !isfinite(rho_ni)) { failed = true; break; }
          if (fabs(rho_nr) + fabs(rho_ni) < 1e-300) { status = 2; break; }
        }
      }
      cdiv(rho_nr, rho_ni, rho_r, rho_i, br, bi);
      rho_r = rho_nr; rho_i = rho_ni;
      rnorm = rn;
      first = false;
      float2* t = pold; pold = pnew; pnew = t;
    }
    if (!dfresh && !failed) {      // fold a pending correction (maxit / breakdown exits)
      fold_sweep(N, x, d);
      __syncthreads();
    }
    // not converged in FP32 (maxit, stagnation, breakdown, non-finite values):
    // x64 holds the last folded solution, which the FP64 launch continues from
    if (failed || status != 0 || !(rnorm <= thr)) status = a.fail_list ? 3 : (status ? status : 1);
  }
  if (threadIdx.x == 0) {
    record(a, s, its, updates, status);
    if (status == 3) a.fail_list[atomicAdd(a.fail_count, 1)] = s;
  }
}

// M: 0 = tile covers the whole plane, 1 = y halo with one slot per thread,
// 2 = y halo with two slots per thread.  PITCH: LDS row pitch (>= nz + 2R).
// NL: with the nonlocal projector term (a separate kernel, so the
// projector-free kernels carry none of its code or registers).
// V: bit 0 = nonlocal projector term, bit 1 = preconditioned solves.
template <bool REFINE, int M, int PITCH, int V>
__global__ void __launch_bounds__(kMaxBlock) k_cocg(CocgArgs a) {
  constexpr bool NL = (V & 1) != 0;
  constexpr bool PC = (V & 2) != 0;
  constexpr bool FULL = M == 0;
  constexpr int HS = M == 2 ? 2 : 1;
  extern __shared__ double smem_d[];
  char* smem = reinterpret_cast<char*>(smem_d);
  const Geom& g = a.g;
  double* red = reinterpret_cast<double*>(smem + lds_plane_bytes(g, PITCH, REFINE));
  char* nlc = smem + lds_plane_bytes(g, PITCH, REFINE) + red_bytes(blockDim.x);
  __shared__ int s_item;
  int item = 0;
  // the FP64 launch after an FP32 one takes the systems the latter handed over
  const int n_items = a.n_items_dev ? uni(*a.n_items_dev) : a.n_items;
  if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
  __syncthreads();
  item = uni(s_item);
  __syncthreads();
  while (item < n_items) {
    const int s = uni(a.order[item]);
    const int b = s / a.n_occ;
    const int live = a.active == nullptr ? 1 : uni(a.active[b]);
    if (live) {
      if (REFINE) solve_refine<FULL, HS, PITCH, NL, PC>(a, s, smem, red, nlc);
      else solve_fp64<FULL, HS, PITCH, NL, PC>(a, s, smem, red, nlc);
    } else if (threadIdx.x == 0) {
      a.out_iters[s] = 0;
      a.out_cycles[s] = 0;
      a.out_status[s] = 0;
    }
    if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    item = uni(s_item);
    __syncthreads();
  }
}

int tile_mode(const Geom& g, int block) {
  if (g.ty == g.ny) return 0;
  return block >= 2 * R * g.nz ? 1 : 2;
}
int pitch_for(const Geom& g) { return g.nz + 2 * R <= 64 ? 64 : 128; }

template <bool REFINE, int M, int V>
const void* cocg_fn_p(int pitch) {
  return pitch == 64 ? reinterpret_cast<const void*>(&k_cocg<REFINE, M, 64, V>)
                     : reinterpret_cast<const void*>(&k_cocg<REFINE, M, 128, V>);
}
template <int V>
const void* cocg_fn_t(bool refine, int m, int pitch) {
  if (refine) {
    if (m == 0) return cocg_fn_p<true, 0, V>(pitch);
    if (m == 1) return cocg_fn_p<true, 1, V>(pitch);
    return cocg_fn_p<true, 2, V>(pitch);
  }
  if (m == 0) return cocg_fn_p<false, 0, V>(pitch);
  if (m == 1) return cocg_fn_p<false, 1, V>(pitch);
  return cocg_fn_p<false, 2, V>(pitch);
}

template <bool REFINE, int M, int P, int V>
hipError_t launch_c(const CocgArgs& a, int grid, int block, size_t shmem, hipStream_t s) {
  hipLaunchKernelGGL((k_cocg<REFINE, M, P, V>), dim3(grid), dim3(block), shmem, s, a);
  return hipGetLastError();
}
template <bool REFINE, int M, int V>
hipError_t launch_cm(const CocgArgs& a, int pitch, int grid, int block, size_t shmem, hipStream_t s) {
  return pitch == 64 ? launch_c<REFINE, M, 64, V>(a, grid, block, shmem, s)
                     : launch_c<REFINE, M, 128, V>(a, grid, block, shmem, s);
}
template <int V>
hipError_t launch_cocg_t(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                         hipStream_t s) {
  const int m = tile_mode(a.g, block);
  const int pitch = pitch_for(a.g);
  if (fp32_refine) {
    if (m == 0) return launch_cm<true, 0, V>(a, pitch, grid, block, shmem, s);
    if (m == 1) return launch_cm<true, 1, V>(a, pitch, grid, block, shmem, s);
    return launch_cm<true, 2, V>(a, pitch, grid, block, shmem, s);
  }
  if (m == 0) return launch_cm<false, 0, V>(a, pitch, grid, block, shmem, s);
  if (m == 1) return launch_cm<false, 1, V>(a, pitch, grid, block, shmem, s);
  return launch_cm<false, 2, V>(a, pitch, grid, block, shmem, s);
}

}  // namespace
}  // namespace rpa
