// Block Lanczos quadrature over groups of grid points: the block operations
// over several points that the Conclusions and Future Work section proposes
// for the diagonal estimates e_j^T f(A) e_j of Algorithm 1.
//
// A group of b points at one frequency starts from Q_1 = [e_j1 ... e_jb] and
// runs the block three-term recurrence
//   A Q_k = Q_{k-1} B_{k-1}^T + Q_k A_k + Q_{k+1} B_k,
// A_k = sym(Q_k^T A Q_k), full reorthogonalisation (two classical
// Gram-Schmidt passes against every stored block) and Q_{k+1} B_k the thin QR
// of the remainder, column by column with a second projection pass.  The
// block Gauss rule gives d_i = sum_l U_il^2 f(lambda_l) for the first b rows
// of the eigenvectors U of the block tridiagonal T (Jacobi eigensolver).
//
// Every group of a batch advances together, one kernel per stage; the
// vectors of a group are columns of the engine's Lanczos basis (layout
// [block k][batch column][N]).  The contractions with the stored blocks are
// tall-skinny products with K = N and at most 64 x 8 outputs per group: at
// about one flop per byte they are bound by HBM, so they run on vector FP64
// as chunked partial dot products with a fixed-order reduction (results do
// not depend on the launch shape).
#include "internal.h"

namespace rpa {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double* vec_ptr(const BVSet& s, int i, int ncol, int gcol, int B,
                                           long long N) {
  const int l = i / ncol, c = i - l * ncol;
  return s.base + ((size_t)(s.blk0 + l) * B + gcol + s.c0 + c) * (size_t)N;
}

// columns of the set that exist in a group of bg columns (<= 0: none)
__device__ __forceinline__ int set_cols(const BVSet& s, int bg) {
  const int avail = bg - s.c0;
  return s.ncol > 0 ? (s.ncol < avail ? s.ncol : avail) : avail;
}

// part[g][i][j][chunk] = sum over the chunk's rows of X_i[r] Y_j[r]
__global__ void __launch_bounds__(kThreads) k_bgram(BVSet X, BVSet Y, int B, long long N, int chunk,
                                                    int nchunks, const int* __restrict__ gcol,
                                                    const int* __restrict__ gsz,
                                                    const int* __restrict__ gact, int pmax,
                                                    double* __restrict__ part) {
  __shared__ double red[kThreads / 64][kMaxLzBlock];
  const int g = blockIdx.z, i = blockIdx.y, c = blockIdx.x;
  if (!gact[g]) return;
  const int bg = gsz[g];
  const int xn = set_cols(X, bg), yn = set_cols(Y, bg);
  if (xn <= 0 || yn <= 0 || i >= X.n_blk * xn) return;
  const double* x = vec_ptr(X, i, xn, gcol[g], B, N);
  const double* y[kMaxLzBlock];
#pragma unroll
  for (int j = 0; j < kMaxLzBlock; ++j) y[j] = j < yn ? vec_ptr(Y, j, yn, gcol[g], B, N) : x;
  double s[kMaxLzBlock];
#pragma unroll
  for (int j = 0; j < kMaxLzBlock; ++j) s[j] = 0.0;
  const long long r0 = (long long)c * chunk;
  const long long r1 = r0 + chunk < N ? r0 + chunk : N;
  for (long long r = r0 + threadIdx.x; r < r1; r += kThreads) {
    const double xv = x[r];
#pragma unroll
    for (int j = 0; j < kMaxLzBlock; ++j)
      if (j < yn) s[j] += xv * y[j][r];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kMaxLzBlock; ++j) {
    if (j < yn) {
      double v = s[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wave][j] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < yn) {
    double v = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) v += red[w][threadIdx.x];
    part[(((size_t)g * pmax + i) * kMaxLzBlock + threadIdx.x) * nchunks + c] = v;
  }
}

// C[g][i][j] = sum over chunks (in order) of part[g][i][j][chunk]
__global__ void k_bgram_reduce(BVSet X, BVSet Y, int G, int nchunks, const int* __restrict__ gsz,
                               const int* __restrict__ gact, int pmax, const double* __restrict__ part,
                               double* __restrict__ C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = t % kMaxLzBlock, i = (t / kMaxLzBlock) % pmax, g = t / (kMaxLzBlock * pmax);
  if (g >= G || !gact[g]) return;
  const int bg = gsz[g];
  const int xn = set_cols(X, bg), yn = set_cols(Y, bg);
  if (xn <= 0 || j >= yn || i >= X.n_blk * xn) return;
  const double* p = part + (((size_t)g * pmax + i) * kMaxLzBlock + j) * nchunks;
  double v = 0.0;
  for (int c = 0; c < nchunks; ++c) v += p[c];
  C[((size_t)g * pmax + i) * kMaxLzBlock + j] = v;
}

// Y_j[r] -= sum_i X_i[r] C[g][i][j]
__global__ void __launch_bounds__(kThreads) k_bcombine(BVSet X, BVSet Y, int B, long long N,
                                                       const int* __restrict__ gcol,
                                                       const int* __restrict__ gsz,
                                                       const int* __restrict__ gact, int pmax,
                                                       const double* __restrict__ C) {
  const int g = blockIdx.y;
  if (!gact[g]) return;
  const long long r = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (r >= N) return;
  const int bg = gsz[g];
  const int xn = set_cols(X, bg), yn = set_cols(Y, bg);
  if (xn <= 0 || yn <= 0) return;
  const int p = X.n_blk * xn;
  const double* Cg = C + (size_t)g * pmax * kMaxLzBlock;
  double acc[kMaxLzBlock];
#pragma unroll
  for (int j = 0; j < kMaxLzBlock; ++j) acc[j] = j < yn ? vec_ptr(Y, j, yn, gcol[g], B, N)[r] : 0.0;
  for (int i = 0; i < p; ++i) {
    const double xv = vec_ptr(X, i, xn, gcol[g], B, N)[r];
#pragma unroll
    for (int j = 0; j < kMaxLzBlock; ++j)
      if (j < yn) acc[j] -= xv * Cg[(size_t)i * kMaxLzBlock + j];
  }
#pragma unroll
  for (int j = 0; j < kMaxLzBlock; ++j)
    if (j < yn) vec_ptr(Y, j, yn, gcol[g], B, N)[r] = acc[j];
}

// After C = Q_k^T W: A_k = (C + C^T) / 2 into Ablk[g][k]; the coefficients
// of W -= Q_{k-1} B_{k-1}^T + Q_k A_k for the stacked set [Q_{k-1}, Q_k]
// (just Q_k when k = 0) into C; the running max |A| entry; the block count.
__global__ void k_bstep_diag(int G, int k, int m, const int* __restrict__ gsz,
                             const int* __restrict__ gact, int pmax, double* __restrict__ C,
                             double* __restrict__ Ablk, const double* __restrict__ Bblk,
                             double* __restrict__ amax, int* __restrict__ gm) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G || !gact[g]) return;
  const int b = gsz[g];
  constexpr int S = kMaxLzBlock * kMaxLzBlock;
  double* Cg = C + (size_t)g * pmax * kMaxLzBlock;
  double* Ak = Ablk + ((size_t)g * m + k) * S;
  double a = amax[g];
  for (int i = 0; i < b; ++i)
    for (int j = 0; j < b; ++j) {
      const double v = 0.5 * (Cg[i * kMaxLzBlock + j] + Cg[j * kMaxLzBlock + i]);
      Ak[i * kMaxLzBlock + j] = v;
      a = fmax(a, fabs(v));
    }
  amax[g] = a;
  gm[g] = k + 1;
  const int off = k > 0 ? b : 0;
  if (k > 0) {
    const double* Bp = Bblk + ((size_t)g * m + k - 1) * S;
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) Cg[i * kMaxLzBlock + j] = Bp[j * kMaxLzBlock + i];
  }
  for (int i = 0; i < b; ++i)
    for (int j = 0; j < b; ++j) Cg[(off + i) * kMaxLzBlock + j] = Ak[i * kMaxLzBlock + j];
}

// Thin QR of the remainder, column j: after a projection pass (C holds the
// coefficients against q_0..q_{j-1}) add them to R's column j.
__global__ void k_bqr_acc(int G, int k, int m, int j, const int* __restrict__ gsz,
                          const int* __restrict__ gact, int pmax, const double* __restrict__ C,
                          double* __restrict__ Bblk) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G || !gact[g] || j >= gsz[g]) return;
  constexpr int S = kMaxLzBlock * kMaxLzBlock;
  double* R = Bblk + ((size_t)g * m + k) * S;
  const double* Cg = C + (size_t)g * pmax * kMaxLzBlock;
  for (int i = 0; i < j; ++i) R[i * kMaxLzBlock + j] += Cg[i * kMaxLzBlock];
}

// Column j's norm (C[g][0][0] = w_j^T w_j): R_jj, or breakdown when it is at
// most brk times the largest |A| entry so far (the group stops; T keeps the
// k + 1 diagonal blocks it has).  scale[g] = 1 / R_jj for the normalisation.
__global__ void k_bqr_norm(int G, int k, int m, int j, const int* __restrict__ gcol,
                           const int* __restrict__ gsz, int* __restrict__ gact, int pmax,
                           const double* __restrict__ C, double* __restrict__ Bblk,
                           const double* __restrict__ amax, double brk, double* __restrict__ scale,
                           int* __restrict__ active) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G || !gact[g] || j >= gsz[g]) return;
  constexpr int S = kMaxLzBlock * kMaxLzBlock;
  const double r = sqrt(C[(size_t)g * pmax * kMaxLzBlock]);
  if (!(r > brk * amax[g])) {
    gact[g] = 0;
    for (int c = 0; c < gsz[g]; ++c) active[gcol[g] + c] = 0;
    return;
  }
  Bblk[((size_t)g * m + k) * S + j * kMaxLzBlock + j] = r;
  scale[g] = 1.0 / r;
}

// q_{k+1, j} = w_j * scale[g]
__global__ void __launch_bounds__(kThreads) k_bqr_scale(double* __restrict__ Q, const double* __restrict__ W,
                                                        int B, long long N, int k, int j,
                                                        const int* __restrict__ gcol,
                                                        const int* __restrict__ gsz,
                                                        const int* __restrict__ gact,
                                                        const double* __restrict__ scale) {
  const int g = blockIdx.y;
  if (!gact[g] || j >= gsz[g]) return;
  const long long r = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (r >= N) return;
  const size_t col = (size_t)gcol[g] + j;
  Q[((size_t)(k + 1) * B + col) * N + r] = W[col * N + r] * scale[g];
}

// Block Gauss rule per group (one wave): T from the blocks, cyclic Jacobi
// rotations T <- J^T T J tracking the first b rows of the eigenvector
// matrix, then d_i = sum_l U_il^2 f(lambda_l), f(x) = log(1 - x) + x,
// written to dout[pos[gcol + i]].
__global__ void __launch_bounds__(64) k_block_quad(int m, const int* __restrict__ gcol,
                                                   const int* __restrict__ gsz,
                                                   const int* __restrict__ gm,
                                                   const double* __restrict__ Ablk,
                                                   const double* __restrict__ Bblk,
                                                   const long long* __restrict__ pos,
                                                   double* __restrict__ dout, int* __restrict__ fail) {
  __shared__ double T[kMaxLanczos][kMaxLanczos + 1];
  __shared__ double V[kMaxLzBlock][kMaxLanczos + 1];
  __shared__ double red[2];
  const int g = blockIdx.x, l = threadIdx.x;
  const int b = gsz[g], nb = gm[g];
  const int n = nb * b;
  constexpr int S = kMaxLzBlock * kMaxLzBlock;
  for (int r = 0; r < n; ++r) T[r][l] = 0.0;
  __syncthreads();
  if (l < n) {
    const int kb = l / b, i = l % b;
    const double* Ak = Ablk + ((size_t)g * m + kb) * S;
    for (int j = 0; j < b; ++j) T[kb * b + i][kb * b + j] = Ak[i * kMaxLzBlock + j];
    if (kb + 1 < nb) {
      const double* Bk = Bblk + ((size_t)g * m + kb) * S;
      for (int j = 0; j < b; ++j) {
        // T[(kb+1) b + j][kb b + i] = B_kb[j][i] and its transpose
        T[(kb + 1) * b + j][kb * b + i] = Bk[j * kMaxLzBlock + i];
        T[kb * b + i][(kb + 1) * b + j] = Bk[j * kMaxLzBlock + i];
      }
    }
  }
  for (int i = 0; i < b; ++i) V[i][l] = (i == l) ? 1.0 : 0.0;
  __syncthreads();
  bool converged = n <= 1;
  for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double tpq = T[p][q];
        if (tpq == 0.0) continue;
        const double tau = (T[q][q] - T[p][p]) / (2.0 * tpq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        __syncthreads();
        if (l < n) {
          const double a = T[l][p], bq = T[l][q];
          T[l][p] = c * a - s * bq;
          T[l][q] = s * a + c * bq;
        }
        if (l < b) {
          const double a = V[l][p], bq = V[l][q];
          V[l][p] = c * a - s * bq;
          V[l][q] = s * a + c * bq;
        }
        __syncthreads();
        if (l < n) {
          const double a = T[p][l], bq = T[q][l];
          T[p][l] = c * a - s * bq;
          T[q][l] = s * a + c * bq;
        }
        __syncthreads();
        // the rotation annihilates T_pq; drop its rounding residue
        if (l == 0) { T[p][q] = 0.0; T[q][p] = 0.0; }
        __syncthreads();
      }
    }
    // off-diagonal mass against the diagonal
    double off = 0.0, dia = 0.0;
    if (l < n) {
      for (int r = 0; r < n; ++r) {
        const double v = T[l][r];
        if (r == l) dia += v * v;
        else off += v * v;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if (l == 0) { red[0] = off; red[1] = dia; }
    __syncthreads();
    converged = red[0] <= 1e-30 * red[1];
    __syncthreads();
  }
  if (l < b) {
    double acc = 0.0;
    for (int r = 0; r < n; ++r) {
      const double lam = T[r][r];
      acc += V[l][r] * V[l][r] * (log1p(-lam) + lam);
    }
    dout[pos[gcol[g] + l]] = acc;
  }
  if (l == 0) {
    if (!converged) atomicAdd(&fail[0], 1);
    if (nb < m) atomicAdd(&fail[1], 1);
  }
}

}  // namespace

int bgram_chunks(long long N) { return (int)((N + kBgramChunk - 1) / kBgramChunk); }

hipError_t launch_bgram(const BVSet& X, const BVSet& Y, int max_x, int B, long long N, int G,
                        const int* gcol, const int* gsz, const int* gact, int pmax, double* part,
                        double* C, hipStream_t s) {
  if (max_x <= 0 || G <= 0) return hipSuccess;
  const int nc = bgram_chunks(N);
  hipLaunchKernelGGL(k_bgram, dim3(nc, max_x, G), dim3(kThreads), 0, s, X, Y, B, N, kBgramChunk, nc,
                     gcol, gsz, gact, pmax, part);
  const int tot = G * pmax * kMaxLzBlock;
  hipLaunchKernelGGL(k_bgram_reduce, dim3((tot + 255) / 256), dim3(256), 0, s, X, Y, G, nc, gsz, gact,
                     pmax, part, C);
  return hipGetLastError();
}

hipError_t launch_bcombine(const BVSet& X, const BVSet& Y, int B, long long N, int G, const int* gcol,
                           const int* gsz, const int* gact, int pmax, const double* C, hipStream_t s) {
  if (G <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bcombine, dim3((unsigned)((N + kThreads - 1) / kThreads), G), dim3(kThreads), 0,
                     s, X, Y, B, N, gcol, gsz, gact, pmax, C);
  return hipGetLastError();
}

hipError_t launch_bstep_diag(int G, int k, int m, const int* gsz, const int* gact, int pmax, double* C,
                             double* Ablk, const double* Bblk, double* amax, int* gm, hipStream_t s) {
  hipLaunchKernelGGL(k_bstep_diag, dim3((G + 63) / 64), dim3(64), 0, s, G, k, m, gsz, gact, pmax, C,
                     Ablk, Bblk, amax, gm);
  return hipGetLastError();
}

hipError_t launch_bqr_acc(int G, int k, int m, int j, const int* gsz, const int* gact, int pmax,
                          const double* C, double* Bblk, hipStream_t s) {
  hipLaunchKernelGGL(k_bqr_acc, dim3((G + 63) / 64), dim3(64), 0, s, G, k, m, j, gsz, gact, pmax, C,
                     Bblk);
  return hipGetLastError();
}

hipError_t launch_bqr_norm(int G, int k, int m, int j, const int* gcol, const int* gsz, int* gact,
                           int pmax, const double* C, double* Bblk, const double* amax, double brk,
                           double* scale, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_bqr_norm, dim3((G + 63) / 64), dim3(64), 0, s, G, k, m, j, gcol, gsz, gact, pmax,
                     C, Bblk, amax, brk, scale, active);
  return hipGetLastError();
}

hipError_t launch_bqr_scale(double* Q, const double* W, int B, long long N, int G, int k, int j,
                            const int* gcol, const int* gsz, const int* gact, const double* scale,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_bqr_scale, dim3((unsigned)((N + kThreads - 1) / kThreads), G), dim3(kThreads), 0,
                     s, Q, W, B, N, k, j, gcol, gsz, gact, scale);
  return hipGetLastError();
}

hipError_t launch_block_quad(int G, int m, const int* gcol, const int* gsz, const int* gm,
                             const double* Ablk, const double* Bblk, const long long* pos, double* dout,
                             int* fail, hipStream_t s) {
  hipLaunchKernelGGL(k_block_quad, dim3(G), dim3(64), 0, s, m, gcol, gsz, gm, Ablk, Bblk, pos, dout,
                     fail);
  return hipGetLastError();
}

}  // namespace rpa
