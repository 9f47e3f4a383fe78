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
//  * FP32_REFINE: inner COCG in FP32 on the residual system, FP64 residual
//    r = b - A x recomputed by an FP64 stencil sweep after each cycle, the FP32
//    correction folded into the FP64 solution.  b = -psi_n (.) u is formed on
//    the fly in FP64 and never stored.
#include "internal.h"

namespace rpa {

namespace {

constexpr int R = kRadius;
constexpr int QN = 2 * R + 1;

template <typename T> struct V2;
template <> struct V2<float> { typedef float2 t; };
template <> struct V2<double> { typedef double2 t; };

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

// ---------------------------------------------------------------------------
// x-marching stencil sweep over all tiles of one system.
// Pol provides:  T2 load(size_t off)  -- value of the operand at a point
//                void center(size_t off, T2 val, T2 nbr)  -- nbr = sum of
//                the off-centre stencil terms; the policy adds the diagonal.
template <typename T, bool FULL, class Pol>
__device__ __forceinline__ void march(const Geom& g, const StencilCoef<T>& cf, Pol& pol,
                                      typename V2<T>::t* lds, int t_begin, int t_end) {
  typedef typename V2<T>::t T2;
  const int tid = threadIdx.x;
  const int nx = g.nx, ny = g.ny, nz = g.nz, ty = g.ty;
  const int ncol = ty * nz;
  const bool own = tid < ncol;
  const int ly = own ? tid / nz : 0;
  const int z = own ? tid - ly * nz : 0;
  const int rows = FULL ? ny : ty + 2 * R;
  const size_t plane = (size_t)ny * nz;


  // halo points (only when the tile does not cover the whole plane): each
  // thread loads at most two of the 2R*nz halo values per plane (ty >= R).
  const int nhalo = FULL ? 0 : 2 * R * nz;
  int hl[2];      // LDS element index
  int hoff_r[2];  // halo row index in [0, 2R)
  int hz[2];
  bool hv[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
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
    int hrowoff[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      int gr = hoff_r[j] < R ? y0 - R + hoff_r[j] : y0 + ty + (hoff_r[j] - R);
      gr = gr < 0 ? gr + ny : (gr >= ny ? gr - ny : gr);
      hrowoff[j] = gr * nz + hz[j];
    }
    // LDS row of the own point; y neighbours at rows rc +- k (wrapped when FULL)
    const int rc = FULL ? gy : ly + R;

    T2 q[QN];
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      int px = i - R; px = px < 0 ? px + nx : (px >= nx ? px - nx : px);
      q[i] = own ? pol.load(px * plane + col) : zero2<T2>();
    }
    int pn = R + 1; pn = pn >= nx ? pn - nx : pn;
    T2 nxt = own ? pol.load(pn * plane + col) : zero2<T2>();
    T2 hcur[2], hnxt[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      hcur[j] = hv[j] ? pol.load(hrowoff[j]) : zero2<T2>();
      hnxt[j] = (hv[j] && nx > 1) ? pol.load(plane + hrowoff[j]) : zero2<T2>();
    }

    for (int x = 0; x < nx; ++x) {
      T2* buf = lds + (x & 1) * rows * nz;
      if (own) buf[rc * nz + z] = q[R];
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (hv[j]) buf[hl[j]] = hcur[j];
      __syncthreads();
      if (own) {
        T ax = 0, ay = 0;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          ax += cf.cx[k] * (q[R - k].x + q[R + k].x);
          ay += cf.cx[k] * (q[R - k].y + q[R + k].y);
        }
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          int up = rc + k, dn = rc - k;
          if (FULL) { up -= up >= ny ? ny : 0; dn += dn < 0 ? ny : 0; }
          const T2 a = buf[up * nz + z];
          const T2 b = buf[dn * nz + z];
          ax += cf.cy[k] * (a.x + b.x);
          ay += cf.cy[k] * (a.y + b.y);
        }
        const int rz = rc * nz;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          int zp = z + k, zm = z - k;
          zp -= zp >= nz ? nz : 0;
          zm += zm < 0 ? nz : 0;
          const T2 a = buf[rz + zp];
          const T2 b = buf[rz + zm];
          ax += cf.cz[k] * (a.x + b.x);
          ay += cf.cz[k] * (a.y + b.y);
        }
        pol.center(x * plane + col, q[R], mk2(ax, ay));
      }
#pragma unroll
      for (int i = 0; i < QN - 1; ++i) q[i] = q[i + 1];
      q[QN - 1] = nxt;
      if (x + 1 < nx) {
        int px = x + R + 2; px = px >= nx ? px - nx : px;
        px = px >= nx ? px - nx : px;
        if (own) nxt = pol.load(px * plane + col);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        hcur[j] = hnxt[j];
        if (hv[j] && x + 2 < nx) hnxt[j] = pol.load((size_t)(x + 2) * plane + hrowoff[j]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Policies

// FP64 residual r = b - (H - sigma) x with b = -psi_n (.) u; stores r in TI.
template <typename TI>
struct ResidPol {
  typedef typename V2<TI>::t TI2;
  const double2* x;
  const double* v;
  const double* psi;
  const double* u;
  TI2* r;
  double c0, eps, om;
  double rr, bb, rho_re, rho_im;
  __device__ double2 load(size_t off) const { return x[off]; }
  __device__ void center(size_t off, double2 xv, double2 nb) {
    const double a = c0 + v[off] - eps;
    const double axr = a * xv.x + om * xv.y + nb.x;
    const double axi = a * xv.y - om * xv.x + nb.y;
    const double bval = -psi[off] * u[off];
    const double rx = bval - axr;
    const double ry = -axi;
    TI2 rs; rs.x = (TI)rx; rs.y = (TI)ry;
    r[off] = rs;
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
  __device__ T2 load(size_t off) const {
    T2 rv = r[off];
    if (first) return rv;
    const T2 pv = pold[off];
    rv.x += br * pv.x - bi * pv.y;
    rv.y += br * pv.y + bi * pv.x;
    return rv;
  }
  __device__ void center(size_t off, T2 pv, T2 nb) {
    const T a = c0 + v[off] - eps;
    T2 h;
    h.x = a * pv.x + om * pv.y + nb.x;
    h.y = a * pv.y - om * pv.x + nb.y;
    pnew[off] = pv;
    q[off] = h;
    mu_re += (double)(pv.x * h.x - pv.y * h.y);
    mu_im += (double)(pv.x * h.y + pv.y * h.x);
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
  __device__ T2 load(size_t off) const { return x[off]; }
  __device__ void center(size_t off, T2 xv, T2 nb) {
    const T a = c0 + v[off] - sr;
    T2 o;
    o.x = a * xv.x + si * xv.y + nb.x;
    o.y = a * xv.y - si * xv.x + nb.y;
    y[off] = o;
  }
};

// ---------------------------------------------------------------------------
// Streaming passes of one system (whole workgroup).

// x (XT) = first ? alpha p : x + alpha p;  r -= alpha q;  returns ||r||^2, r^T r.
template <typename T, typename XT>
__device__ __forceinline__ void update_sweep(long long N, typename V2<XT>::t* x,
                                             const typename V2<T>::t* p, typename V2<T>::t* r,
                                             const typename V2<T>::t* q, T ar, T ai, bool first,
                                             double& rr, double& rho_re, double& rho_im) {
  typedef typename V2<T>::t T2;
  typedef typename V2<XT>::t X2;
  for (long long i = threadIdx.x; i < N; i += blockDim.x) {
    const T2 pv = p[i];
    const T2 qv = q[i];
    T2 rv = r[i];
    const T dx = ar * pv.x - ai * pv.y;
    const T dy = ar * pv.y + ai * pv.x;
    X2 xv;
    if (first) {
      xv.x = (XT)dx; xv.y = (XT)dy;
    } else {
      xv = x[i];
      xv.x += (XT)dx; xv.y += (XT)dy;
    }
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
  a.out_iters[s] = its;
  a.out_cycles[s] = cycles;
  a.out_status[s] = status;
  atomicAdd(&a.stats[0], (unsigned long long)its);
  atomicMax(&a.stats[1], (unsigned long long)its);
  atomicAdd(&a.stats[2], (unsigned long long)cycles);
  if (status == 1) atomicAdd(&a.stats[3], 1ULL);
  if (status == 2) atomicAdd(&a.stats[4], 1ULL);
}

// ---------------------------------------------------------------------------
// One system, FP64 throughout.
template <bool FULL>
__device__ void solve_fp64(const CocgArgs& a, int s, char* smem, double* red) {
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

  ResidPol<double> rp;
  rp.x = x; rp.v = a.v64; rp.psi = a.psi64 + (size_t)n * N; rp.u = a.u64 + (size_t)b * N;
  rp.r = r; rp.c0 = a.c64.c0; rp.eps = eps; rp.om = om;
  rp.rr = rp.bb = rp.rho_re = rp.rho_im = 0.0;
  march<double, FULL>(g, a.c64, rp, lds, 0, g.ntiles);
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
    double br = 0.0, bi = 0.0;
    bool first = true;
    double2* pold = pa;
    double2* pnew = pb;
    while (rnorm > thr) {
      if (its >= a.maxit) { status = 1; break; }
      ApplyPol<double> ap;
      ap.r = r; ap.pold = pold; ap.pnew = pnew; ap.q = q; ap.v = a.v64;
      ap.c0 = a.c64.c0; ap.eps = eps; ap.om = om; ap.br = br; ap.bi = bi; ap.first = first;
      ap.mu_re = ap.mu_im = 0.0;
      march<double, FULL>(g, a.c64, ap, lds, 0, g.ntiles);
      double m2[2] = {ap.mu_re, ap.mu_im};
      block_reduce<2>(m2, red);
      if (fabs(m2[0]) + fabs(m2[1]) < 1e-300) { status = 2; break; }
      double al_r, al_i;
      cdiv(rho_r, rho_i, m2[0], m2[1], al_r, al_i);
      double rr = 0.0, nr = 0.0, ni = 0.0;
      update_sweep<double, double>(N, x, pnew, r, q, al_r, al_i, false, rr, nr, ni);
      double u3[3] = {rr, nr, ni};
      block_reduce<3>(u3, red);
      ++its;
      rnorm = sqrt(u3[0]);
      cdiv(u3[1], u3[2], rho_r, rho_i, br, bi);
      rho_r = u3[1]; rho_i = u3[2];
      first = false;
      double2* t = pold; pold = pnew; pnew = t;
    }
    if (status == 0 && !(rnorm <= thr)) status = 1;   // NaN residual is not convergence
  }
  if (threadIdx.x == 0) record(a, s, its, 0, status);
}

// One system, FP32 inner COCG + FP64 residual refinement.
template <bool FULL>
__device__ void solve_refine(const CocgArgs& a, int s, char* smem, double* red) {
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

  ResidPol<float> rp;
  rp.x = x; rp.v = a.v64; rp.psi = a.psi64 + (size_t)n * N; rp.u = a.u64 + (size_t)b * N;
  rp.r = r; rp.c0 = a.c64.c0; rp.eps = eps; rp.om = om;
  rp.rr = rp.bb = rp.rho_re = rp.rho_im = 0.0;
  march<double, FULL>(g, a.c64, rp, reinterpret_cast<double2*>(smem), 0, g.ntiles);
  double v4[4] = {rp.rr, rp.bb, rp.rho_re, rp.rho_im};
  block_reduce<4>(v4, red);
  const double bnorm = sqrt(v4[1]);
  double rnorm = sqrt(v4[0]);
  double rho_r = v4[2], rho_i = v4[3];
  int its = 0, cycles = 0, status = 0;
  if (bnorm == 0.0) {
    zero_sweep(N, x);
  } else {
    const double thr = a.tol * bnorm;
    while (rnorm > thr) {
      if (its >= a.maxit || cycles >= a.max_cycles) { status = 1; break; }
      // inner FP32 COCG on A d = r (d0 = 0): stop at ||r_in|| <= max(inner_tol*||r||, thr/2)
      const double in_thr = fmax(a.inner_tol * rnorm, 0.5 * thr);
      double br = 0.0, bi = 0.0;
      bool first = true;
      float2* pold = pa;
      float2* pnew = pb;
      double rin = rnorm;
      bool broke = false;
      while (rin > in_thr && its < a.maxit) {
        ApplyPol<float> ap;
        ap.r = r; ap.pold = pold; ap.pnew = pnew; ap.q = q; ap.v = a.v32;
        ap.c0 = a.c32.c0; ap.eps = (float)eps; ap.om = (float)om; ap.br = (float)br;
        ap.bi = (float)bi; ap.first = first;
        ap.mu_re = ap.mu_im = 0.0;
        march<float, FULL>(g, a.c32, ap, reinterpret_cast<float2*>(smem), 0, g.ntiles);
        double m2[2] = {ap.mu_re, ap.mu_im};
        block_reduce<2>(m2, red);
        if (fabs(m2[0]) + fabs(m2[1]) < 1e-300) { broke = true; break; }
        double al_r, al_i;
        cdiv(rho_r, rho_i, m2[0], m2[1], al_r, al_i);
        double rr = 0.0, nr = 0.0, ni = 0.0;
        update_sweep<float, float>(N, d, pnew, r, q, (float)al_r, (float)al_i, first, rr, nr, ni);
        double u3[3] = {rr, nr, ni};
        block_reduce<3>(u3, red);
        ++its;
        rin = sqrt(u3[0]);
        cdiv(u3[1], u3[2], rho_r, rho_i, br, bi);
        rho_r = u3[1]; rho_i = u3[2];
        first = false;
        float2* t = pold; pold = pnew; pnew = t;
      }
      if (!first) fold_sweep(N, x, d);   // x64 += d
      __syncthreads();
      ++cycles;
      rp.rr = rp.bb = rp.rho_re = rp.rho_im = 0.0;
      march<double, FULL>(g, a.c64, rp, reinterpret_cast<double2*>(smem), 0, g.ntiles);
      double w4[4] = {rp.rr, rp.bb, rp.rho_re, rp.rho_im};
      block_reduce<4>(w4, red);
      rnorm = sqrt(w4[0]);
      rho_r = w4[2]; rho_i = w4[3];
      if (broke && rnorm > thr) { status = 2; break; }
    }
    if (status == 0 && !(rnorm <= thr)) status = 1;   // NaN residual is not convergence
  }
  if (threadIdx.x == 0) record(a, s, its, cycles, status);
}

template <bool REFINE, bool FULL>
__global__ void __launch_bounds__(kMaxBlock) k_cocg(CocgArgs a) {
  extern __shared__ double smem_d[];
  char* smem = reinterpret_cast<char*>(smem_d);
  const Geom& g = a.g;
  const int rows = FULL ? g.ny : g.ty + 2 * R;
  double* red = reinterpret_cast<double*>(smem + (size_t)2 * rows * g.nz * sizeof(double2));
  __shared__ int s_item;
  int item = 0;
  if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
  __syncthreads();
  item = uni(s_item);
  __syncthreads();
  while (item < a.n_items) {
    const int s = uni(a.order[item]);
    const int b = s / a.n_occ;
    const int live = a.active == nullptr ? 1 : uni(a.active[b]);
    if (live) {
      if (REFINE) solve_refine<FULL>(a, s, smem, red);
      else solve_fp64<FULL>(a, s, smem, red);
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

template <bool FULL>
__global__ void __launch_bounds__(kMaxBlock) k_happly(Geom g, StencilCoef<double> c64,
                                                       StencilCoef<float> c32, const double* v64,
                                                       const float* v32, const double* sr,
                                                       const double* si, const void* x, void* y,
                                                       int fp32) {
  extern __shared__ double smem_d[];
  const int vec = blockIdx.y;
  const size_t base = (size_t)vec * g.N;
  if (fp32) {
    HPol<float> p;
    p.x = reinterpret_cast<const float2*>(x) + base;
    p.y = reinterpret_cast<float2*>(y) + base;
    p.v = v32; p.c0 = c32.c0;
    p.sr = (float)sr[vec]; p.si = (float)si[vec];
    march<float, FULL>(g, c32, p, reinterpret_cast<float2*>(smem_d), blockIdx.x, blockIdx.x + 1);
  } else {
    HPol<double> p;
    p.x = reinterpret_cast<const double2*>(x) + base;
    p.y = reinterpret_cast<double2*>(y) + base;
    p.v = v64; p.c0 = c64.c0; p.sr = sr[vec]; p.si = si[vec];
    march<double, FULL>(g, c64, p, reinterpret_cast<double2*>(smem_d), blockIdx.x,
                        blockIdx.x + 1);
  }
}

}  // namespace

size_t cocg_shmem_bytes(const Geom& g, int block, bool /*fp32_refine*/) {
  const bool full = g.ty == g.ny;
  const int rows = full ? g.ny : g.ty + 2 * R;
  const int nw = (block + 63) / 64;
  return (size_t)2 * rows * g.nz * sizeof(double2) + (size_t)(nw + 1) * 4 * sizeof(double);
}

int cocg_blocks_per_cu(const Geom& g, int block, bool fp32_refine) {
  const bool full = g.ty == g.ny;
  const size_t shmem = cocg_shmem_bytes(g, block, fp32_refine);
  int nb = 0;
  hipError_t e;
  if (fp32_refine)
    e = full ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cocg<true, true>, block, shmem)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cocg<true, false>, block, shmem);
  else
    e = full ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cocg<false, true>, block, shmem)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cocg<false, false>, block, shmem);
  if (e != hipSuccess || nb < 1) return 1;
  return nb;
}

long long cocg_slot_bytes(const Geom& g, bool fp32_refine) {
  return fp32_refine ? 5LL * g.N * (long long)sizeof(float2) : 4LL * g.N * (long long)sizeof(double2);
}

hipError_t launch_cocg(const CocgArgs& a, bool fp32_refine, int grid, int block, size_t shmem,
                       hipStream_t s) {
  const bool full = a.g.ty == a.g.ny;
  if (fp32_refine) {
    if (full) hipLaunchKernelGGL((k_cocg<true, true>), dim3(grid), dim3(block), shmem, s, a);
    else hipLaunchKernelGGL((k_cocg<true, false>), dim3(grid), dim3(block), shmem, s, a);
  } else {
    if (full) hipLaunchKernelGGL((k_cocg<false, true>), dim3(grid), dim3(block), shmem, s, a);
    else hipLaunchKernelGGL((k_cocg<false, false>), dim3(grid), dim3(block), shmem, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_happly(const Geom& g, const StencilCoef<double>& c64, const StencilCoef<float>& c32,
                         const double* v64, const float* v32, int nvec, const double* shift_re,
                         const double* shift_im, const void* x, void* y, bool fp32,
                         int block, hipStream_t s) {
  const bool full = g.ty == g.ny;
  const size_t shmem = cocg_shmem_bytes(g, block, false);
  dim3 grid(g.ntiles, nvec);
  if (full)
    hipLaunchKernelGGL((k_happly<true>), grid, dim3(block), shmem, s, g, c64, c32, v64, v32,
                       shift_re, shift_im, x, y, fp32 ? 1 : 0);
  else
    hipLaunchKernelGGL((k_happly<false>), grid, dim3(block), shmem, s, g, c64, c32, v64, v32,
                       shift_re, shift_im, x, y, fp32 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace rpa
