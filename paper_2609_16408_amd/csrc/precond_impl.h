// Shifted kinetic preconditioner inside the persistent COCG workgroup
// (preconditioned Sternheimer solves, named in the Conclusions and Future
// Work section; the operator is M = -1/2 Lap_h + sigma with the same
// 12th-order FD Laplacian as in H, inverted exactly in its per-axis
// eigenbasis):
//
//   z = M^-1 r = (Vx (x) Vy (x) Vz) diag(1 / (kx_a + ky_b + kz_c + sigma)) (Vx (x) Vy (x) Vz)^T r
//
// One workgroup applies it to its own system in three passes over the grid:
//   P1  per x-plane i:   S_i = Vy^T R_i Vz                       r -> t
//   P2  per y-mode b:    T_b = Vx diag(scale) Vx^T T_b           t -> t (in place)
//   P3  per x-plane i:   Z_i = Vy S_i Vz^T                       t -> z
// and rho = r^T z = sum over modes of c s c (c = (Vx (x) Vy (x) Vz)^T r the
// forward coefficients, s the diagonal; the basis is real orthogonal), taken
// in P2 where the coefficients are at hand.
// Every contraction is a small GEMM (dimensions padded to multiples of 16,
// at most 64) on the 16x16x4 matrix-core instructions: the plane or slab
// sits in LDS as separate real and imaginary arrays, the basis comes from
// global memory (a few KiB, cache-resident), and each wave computes whole
// 16x16 output tiles for both components.
#pragma once

#include "internal.h"

namespace rpa {

namespace {

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef mf4 acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator v of lane l holds output row 4 (l / 16) + v, column l % 16
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mma<double> {
  typedef md4 acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator v of lane l holds output row l / 16 + 4 v, column l % 16
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename T>
__device__ __forceinline__ const T* prec_pick(const float* a, const double* b) {
  if constexpr (sizeof(T) == 4) return a;
  else return b;
}

// Output tiles of D = A B (M x N, both multiples of 16; K a multiple of 4)
// for a complex operand X stored as real and imaginary LDS arrays with row
// stride ldx, and a real basis W, also in LDS (row stride ldw):
//   LEFT:  D = X W,    A(m, k) = X[m][k], B(k, n) = W[k][n]
//   !LEFT: D = W^T X,  A(m, k) = W[k][m], B(k, n) = X[k][n]
// Each wave takes whole tiles (both components); epi(m, n, re, im) receives
// every output element of the padded range.
template <typename T, bool LEFT, class Epi>
__device__ __forceinline__ void lds_gemm(int M, int N, int K, const T* Xr, const T* Xi, int ldx,
                                         const T* W, int ldw, Epi& epi) {
  typedef typename Mma<T>::acc acc;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nw = (int)(blockDim.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int ntn = N >> 4;
  const int njobs = (M >> 4) * ntn;
  for (int job = wave; job < njobs; job += nw) {
    const int m0 = (job / ntn) << 4, n0 = (job % ntn) << 4;
    acc cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + lk;
      if constexpr (LEFT) {
        const T w = W[k * ldw + n0 + li];
        const int xa = (m0 + li) * ldx + k;
        cr = Mma<T>::step(Xr[xa], w, cr);
        ci = Mma<T>::step(Xi[xa], w, ci);
      } else {
        const T w = W[k * ldw + m0 + li];
        const int xa = k * ldx + n0 + li;
        cr = Mma<T>::step(w, Xr[xa], cr);
        ci = Mma<T>::step(w, Xi[xa], ci);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) epi(m0 + Mma<T>::row(lane, v), n0 + li, (T)cr[v], (T)ci[v]);
  }
}

// Registers of the prefetched plane or slab: element e = tid + k * blockDim
// of the padded rows x cols array, k < kPrecRegs (the host checks the count).
constexpr int kPrecRegs = 4;

template <typename T2>
struct Stage {
  T2 v[kPrecRegs];
  // load rows x cols (padded: zero beyond nrow x ncol) from src[row * rstride + col]
  __device__ __forceinline__ void load(const T2* src, long long rstride, int rows, int cols, int nrow,
                                       int ncol) {
    const int tid = threadIdx.x, bs = blockDim.x;
#pragma unroll
    for (int k = 0; k < kPrecRegs; ++k) {
      const int e = tid + k * bs;
      const int i = e / cols, j = e - i * cols;
      T2 x;
      x.x = 0;
      x.y = 0;
      if (e < rows * cols && i < nrow && j < ncol) x = src[(long long)i * rstride + j];
      v[k] = x;
    }
  }
  template <typename T>
  __device__ __forceinline__ void put(T* dr, T* di, int ld, int rows, int cols) const {
    const int tid = threadIdx.x, bs = blockDim.x;
#pragma unroll
    for (int k = 0; k < kPrecRegs; ++k) {
      const int e = tid + k * bs;
      if (e < rows * cols) {
        const int i = e / cols, j = e - i * cols;
        dr[i * ld + j] = v[k].x;
        di[i * ld + j] = v[k].y;
      }
    }
  }
};

// Copy a P x P basis (global, row stride P) into LDS with row stride P + 1.
template <typename T>
__device__ __forceinline__ void stage_basis(T* dst, const T* src, int P) {
  for (int e = threadIdx.x; e < P * P; e += blockDim.x) {
    const int i = e / P, j = e - i * P;
    dst[i * (P + 1) + j] = src[e];
  }
}

// Epilogues --------------------------------------------------------------

template <typename T>
struct EpiLds {                  // into LDS
  T* dr;
  T* di;
  int ld;
  __device__ __forceinline__ void operator()(int m, int n, T re, T im) {
    dr[m * ld + n] = re;
    di[m * ld + n] = im;
  }
};

template <typename T>
struct EpiScale {                // x-mode a = m, z-mode c = n: times 1 / (kin + sigma), into LDS;
  T* dr;                         // also rho += c s c (c the forward coefficient, s the scale):
  T* di;                         // r^T M^-1 r = sum over modes of s c^2, the basis being real
  int ld;                        // orthogonal
  const T* kx;
  const T* kz;
  T kyb, sr, si;                 // sigma = sr + i si
  double rho_re, rho_im;
  __device__ __forceinline__ void operator()(int m, int n, T re, T im) {
    const T x = kx[m] + kyb + kz[n] + sr;
    const T den = x * x + si * si;
    // (re + i im) (x - i si) / den
    const T zr = (re * x + im * si) / den;
    const T zi = (im * x - re * si) / den;
    dr[m * ld + n] = zr;
    di[m * ld + n] = zi;
    rho_re += (double)re * (double)zr - (double)im * (double)zi;
    rho_im += (double)re * (double)zi + (double)im * (double)zr;
  }
};

template <typename T>
struct EpiStore {                // into the grid vector: row m, column n of a plane or slab
  typename V2<T>::t* out;
  long long rstride;             // elements between rows m
  int mlim, nlim;
  __device__ __forceinline__ void operator()(int m, int n, T re, T im) {
    if (m < mlim && n < nlim) {
      typename V2<T>::t o;
      o.x = re;
      o.y = im;
      out[(long long)m * rstride + n] = o;
    }
  }
};

// Bytes of LDS the preconditioner uses: two complex planes (real and
// imaginary arrays) of the padded size with an odd row stride, and the two
// bases of the current pass.
__host__ __device__ inline int prec_pad(int n) { return (n + 15) & ~15; }
__host__ __device__ inline size_t prec_lds_bytes(const Geom& g, size_t elem) {
  const int px = prec_pad(g.nx), py = prec_pad(g.ny), pz = prec_pad(g.nz);
  const int rows = px > py ? px : py;
  const int pm = rows > pz ? rows : pz;
  const size_t ld = (size_t)pz + 1;
  const size_t bas = 2 * (size_t)pm * (pm + 1);
  return ((4 * (size_t)rows * ld + bas) * elem + 255) & ~(size_t)255;
}
// Registers per thread the prefetched planes and slabs need (at most kPrecRegs).
__host__ __device__ inline int prec_regs(const Geom& g, int block) {
  const int px = prec_pad(g.nx), py = prec_pad(g.ny), pz = prec_pad(g.nz);
  const int e = (px > py ? px : py) * pz;
  return (e + block - 1) / block;
}

// z = M^-1 r with sigma = sr + i si; t is a scratch vector of the system;
// adds this thread's part of rho = r^T z to (rho_re, rho_im) (the caller
// reduces over the workgroup).  All threads of the
// workgroup call it; it leaves LDS free for the caller.  The tables are
// read through one pointer here, so that the solver's stencil sweeps do not
// keep eighteen table addresses live.
template <typename T>
__device__ __forceinline__ void precond_apply(const Geom& g, const PrecArgs* pap, const typename V2<T>::t* r,
                              typename V2<T>::t* t, typename V2<T>::t* z, T sr, T si,
                              char* smem, double& rho_re, double& rho_im) {
  typedef typename V2<T>::t T2;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int px = prec_pad(nx), py = prec_pad(ny), pz = prec_pad(nz);
  const int ld = pz + 1;
  const int rows = px > py ? px : py;
  const int pm = rows > pz ? rows : pz;
  T* D0r = reinterpret_cast<T*>(smem);
  T* D0i = D0r + rows * ld;
  T* D1r = D0i + rows * ld;
  T* D1i = D1r + rows * ld;
  T* W0 = D1i + rows * ld;       // the two bases of the current pass
  T* W1 = W0 + pm * (pm + 1);
  const PrecArgs& pa = *pap;
  const T* kx = prec_pick<T>(pa.k32[0], pa.k64[0]);
  const T* ky = prec_pick<T>(pa.k32[1], pa.k64[1]);
  const T* kz = prec_pick<T>(pa.k32[2], pa.k64[2]);
  const long long plane = (long long)ny * nz;
  Stage<T2> st;

  // P1: S_i = Vy^T R_i Vz per x-plane (the next plane's loads are in flight
  // during the current plane's products)
  stage_basis<T>(W0, prec_pick<T>(pa.v32[2], pa.v64[2]), pz);   // Vz
  stage_basis<T>(W1, prec_pick<T>(pa.v32[1], pa.v64[1]), py);   // Vy
  st.load(r, nz, py, pz, ny, nz);
  for (int i = 0; i < nx; ++i) {
    st.put(D0r, D0i, ld, py, pz);
    __syncthreads();
    if (i + 1 < nx) st.load(r + (long long)(i + 1) * plane, nz, py, pz, ny, nz);
    EpiLds<T> e1{D1r, D1i, ld};
    lds_gemm<T, true>(py, pz, pz, D0r, D0i, ld, W0, pz + 1, e1);
    __syncthreads();
    EpiStore<T> e2{t + (long long)i * plane, nz, ny, nz};
    lds_gemm<T, false>(py, pz, py, D1r, D1i, ld, W1, py + 1, e2);
  }
  __syncthreads();
  // P2: per y-mode b, the x contraction, the diagonal, the inverse x contraction
  stage_basis<T>(W0, prec_pick<T>(pa.v32[0], pa.v64[0]), px);   // Vx
  stage_basis<T>(W1, prec_pick<T>(pa.vt32[0], pa.vt64[0]), px); // Vx^T
  st.load(t, plane, px, pz, nx, nz);
  for (int b = 0; b < ny; ++b) {
    T2* tb = t + (long long)b * nz;
    st.put(D0r, D0i, ld, px, pz);
    __syncthreads();
    if (b + 1 < ny) st.load(tb + nz, plane, px, pz, nx, nz);
    EpiScale<T> e3{D1r, D1i, ld, kx, kz, ky[b], sr, si, 0.0, 0.0};
    lds_gemm<T, false>(px, pz, px, D0r, D0i, ld, W0, px + 1, e3);
    rho_re += e3.rho_re;
    rho_im += e3.rho_im;
    __syncthreads();
    EpiStore<T> e4{tb, plane, nx, nz};
    lds_gemm<T, false>(px, pz, px, D1r, D1i, ld, W1, px + 1, e4);
  }
  __syncthreads();
  // P3: Z_i = Vy S_i Vz^T per x-plane
  stage_basis<T>(W0, prec_pick<T>(pa.vt32[1], pa.vt64[1]), py); // Vy^T
  stage_basis<T>(W1, prec_pick<T>(pa.vt32[2], pa.vt64[2]), pz); // Vz^T
  st.load(t, nz, py, pz, ny, nz);
  for (int i = 0; i < nx; ++i) {
    st.put(D0r, D0i, ld, py, pz);
    __syncthreads();
    if (i + 1 < nx) st.load(t + (long long)(i + 1) * plane, nz, py, pz, ny, nz);
    EpiLds<T> e5{D1r, D1i, ld};
    lds_gemm<T, false>(py, pz, py, D0r, D0i, ld, W0, py + 1, e5);
    __syncthreads();
    EpiStore<T> e6{z + (long long)i * plane, nz, ny, nz};
    lds_gemm<T, true>(py, pz, pz, D1r, D1i, ld, W1, pz + 1, e6);
  }
  __syncthreads();
}

}  // namespace
}  // namespace rpa
