// Kernels around the Sternheimer solve: Kronecker-form nu^1/2 and the
// separable interpolants (per-axis transforms), Galerkin initial guess,
// density accumulation, Lanczos recurrence with full reorthogonalisation,
// tridiagonal Gauss quadrature and frequency integration.
#include "internal.h"

namespace rpa {

namespace {

// ---------------------------------------------------------------------------
__global__ void k_fill_d(double* p, double v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i(int* p, int v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}
__global__ void k_set_onehot(double* q, long long stride, const long long* idx, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) q[(size_t)b * stride + idx[b]] = 1.0;
}

// ---------------------------------------------------------------------------
// Per-axis transform: out[b, ..., i, ...] = sum_k M(i, k) in[b, ..., k, ...]
__global__ void k_axis(const double* __restrict__ in, double* __restrict__ out, int B, int d0,
                       int d1, int d2, int axis, int n_out, const double* __restrict__ M,
                       int trans, const double* __restrict__ scale) {
  int od0 = d0, od1 = d1, od2 = d2;
  if (axis == 0) od0 = n_out; else if (axis == 1) od1 = n_out; else od2 = n_out;
  const long long osz = (long long)od0 * od1 * od2;
  const long long isz = (long long)d0 * d1 * d2;
  const long long total = osz * B;
  const int n_in = axis == 0 ? d0 : (axis == 1 ? d1 : d2);
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long b = t / osz;
    const long long o = t - b * osz;
    const int i2 = (int)(o % od2);
    const long long o01 = o / od2;
    const int i1 = (int)(o01 % od1);
    const int i0 = (int)(o01 / od1);
    const double* src = in + b * isz;
    long long base, stride;
    int i;
    if (axis == 0) { i = i0; base = (long long)i1 * d2 + i2; stride = (long long)d1 * d2; }
    else if (axis == 1) { i = i1; base = (long long)i0 * d1 * d2 + i2; stride = d2; }
    else { i = i2; base = ((long long)i0 * d1 + i1) * d2; stride = 1; }
    double acc = 0.0;
    if (trans) {
      for (int k = 0; k < n_in; ++k) acc += M[(long long)k * n_out + i] * src[base + k * stride];
    } else {
      const double* row = M + (long long)i * n_in;
      for (int k = 0; k < n_in; ++k) acc += row[k] * src[base + k * stride];
    }
    if (scale) acc *= scale[o];
    out[t] = acc;
  }
}

// ---------------------------------------------------------------------------
// Complex diagonal solve in the eigenbasis of the FD Laplacian, the middle
// step of the shifted kinetic preconditioner: vector b is stored planar
// (N real parts, then N imaginary parts) and each mode o is divided by
// kin[o] + sigma_b, kin >= 0 the kinetic eigenvalue, Re(sigma_b) > 0.
__global__ void k_kin_scale(double* __restrict__ a, const double* __restrict__ kin,
                            const double* __restrict__ sig_re, const double* __restrict__ sig_im,
                            int B, long long N) {
  const long long total = (long long)B * N;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long b = t / N;
    const long long o = t - b * N;
    double* re = a + b * 2 * N;
    double* im = re + N;
    const double dr = kin[o] + sig_re[b];
    const double di = sig_im[b];
    const double den = dr * dr + di * di;
    const double xr = re[o], xi = im[o];
    re[o] = (xr * dr + xi * di) / den;
    im[o] = (xi * dr - xr * di) / den;
  }
}

// ---------------------------------------------------------------------------
// Galerkin projection, part 1: part[b][c][m][n] = sum_{r in chunk c} psi_m psi_n u_b,
// a contraction over grid points on the FP64 matrix cores.  A 256-thread
// workgroup owns a 128 x 128 output tile; each wave a 64 x 64 quadrant as
// 4 x 4 MFMA tiles (v_mfma_f64_16x16x4: A lane l = row l%16, k l/16; B lane
// l = column l%16, k l/16; D register v of lane l = row l/16 + 4v, column
// l%16).  GK grid
// points of the 128 rows of each operand are staged in LDS per step (the
// psi_m u_b rows and the psi_n rows), zero beyond n_occ and the chunk end.
constexpr int GT = 128;   // output tile
constexpr int GK = 16;    // r-block staged in LDS

typedef double d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gram(const double* __restrict__ psi,
                                              const double* __restrict__ u, int n_occ, int ng,
                                              long long N, int n_chunks, int ntn,
                                              double* __restrict__ part) {
  __shared__ double sA[GK][GT + 2];
  __shared__ double sB[GK][GT + 2];
  const int c = blockIdx.x;
  const int b = blockIdx.y;
  const int tm = blockIdx.z / ntn, tn = blockIdx.z % ntn;
  const int m0 = tm * GT, n0 = tn * GT;
  const long long clen = (N + n_chunks - 1) / n_chunks;
  const long long r0 = c * clen;
  const long long r1 = r0 + clen < N ? r0 + clen : N;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int qm = (wave >> 1) * 64, qn = (wave & 1) * 64;   // quadrant of the tile
  const int li = lane & 15, lk = lane >> 4;
  const double* ub = u + (size_t)b * N;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  for (long long rb = r0; rb < r1; rb += GK) {
    for (int e = threadIdx.x; e < GK * GT; e += 256) {
      const int k = e % GK, i = e / GK;
      const long long r = rb + k;
      double a = 0.0, bb = 0.0;
      if (r < r1) {
        const double uu = ub[r];
        if (m0 + i < ng) a = psi[(size_t)(m0 + i) * N + r] * uu;
        if (n0 + i < n_occ) bb = psi[(size_t)(n0 + i) * N + r];
      }
      sA[k][i] = a;
      sB[k][i] = bb;
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < GK; k0 += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        av[t] = sA[k0 + lk][qm + t * 16 + li];
        bv[t] = sB[k0 + lk][qn + t * 16 + li];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = part + ((size_t)b * n_chunks + c) * ng * n_occ;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + qn + j * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + qm + i * 16 + lk + 4 * v;
        if (m < ng && n < n_occ) out[(size_t)m * n_occ + n] = acc[i][j][v];
      }
    }
  }
}

// part 2: G[b][m][n] = (-dV sum_c part) / (eps_m - eps_n - i omega_b), m over the
// ng Galerkin states (occupied first), n over the occupied ones
__global__ void k_gram_finish(const double* __restrict__ part, int B, int n_occ, int ng, int n_chunks,
                              double dV, const double* __restrict__ eps,
                              const double* __restrict__ omega, double2* __restrict__ G) {
  const long long total = (long long)B * ng * n_occ;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / ((long long)ng * n_occ));
    const long long mn = t - (long long)b * ng * n_occ;
    const int m = (int)(mn / n_occ), n = (int)(mn % n_occ);
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += part[((size_t)b * n_chunks + c) * ng * n_occ + mn];
    const double cm = -dV * s;
    const double dr = eps[m] - eps[n];
    const double di = -omega[b];
    const double den = dr * dr + di * di;
    G[t] = make_double2(cm * dr / den, -cm * di / den);
  }
}

// part 3: x64[(b*n_occ + n)][r] = sum_m psi_m(r) G[b][m][n], m over the ng states
// tile 64 r x 64 n; thread (rl = t%16, nl = t/16) owns r = r0+rl+16i, n = n0+nl+16j
__global__ void __launch_bounds__(256) k_expand(const double* __restrict__ psi,
                                                const double2* __restrict__ G, int n_occ, int ng,
                                                long long N, double2* __restrict__ x64) {
  __shared__ double sP[16][64 + 1];
  __shared__ double2 sG[16][64 + 1];
  const long long r0 = (long long)blockIdx.x * 64;
  const int n0 = blockIdx.y * 64;
  const int b = blockIdx.z;
  const int rl = threadIdx.x & 15, nl = threadIdx.x >> 4;
  const double2* Gb = G + (size_t)b * ng * n_occ;
  double ar[4][4], ai[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) { ar[i][j] = 0.0; ai[i][j] = 0.0; }
  for (int mb = 0; mb < ng; mb += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int k = e / 64, i = e % 64;
      const int m = mb + k;
      const long long r = r0 + i;
      sP[k][i] = (m < ng && r < N) ? psi[(size_t)m * N + r] : 0.0;
      sG[k][i] = (m < ng && n0 + i < n_occ) ? Gb[(size_t)m * n_occ + n0 + i] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      double pv[4];
      double2 gv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) pv[i] = sP[k][rl + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) gv[j] = sG[k][nl + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) { ar[i][j] += pv[i] * gv[j].x; ai[i][j] += pv[i] * gv[j].y; }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + nl + 16 * j;
    if (n >= n_occ) continue;
    double2* dst = x64 + ((size_t)b * n_occ + n) * N;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long r = r0 + rl + 16 * i;
      if (r < N) dst[r] = make_double2(ar[i][j], ai[i][j]);
    }
  }
}

// racc[b][r] = 4 sum_n psi_n(r) Re x64[b][n][r]
__global__ void k_accumulate(const double* __restrict__ psi, const double2* __restrict__ x64,
                             int B, int n_occ, long long N, const int* __restrict__ active,
                             double* __restrict__ racc) {
  const long long total = (long long)B * N;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / N);
    const long long r = t - (long long)b * N;
    double s = 0.0;
    if (active == nullptr || active[b]) {
      const double2* xb = x64 + (size_t)b * n_occ * N;
      for (int n = 0; n < n_occ; ++n) s += psi[(size_t)n * N + r] * xb[(size_t)n * N + r].x;
    }
    racc[t] = 4.0 * s;
  }
}

// ---------------------------------------------------------------------------
// Lanczos step k for start vector b = blockIdx.x (one workgroup each):
//   alpha_k = q_k^T v;  v -= alpha_k q_k + beta_{k-1} q_{k-1};
//   two classical Gram-Schmidt passes against q_0..q_k;
//   if k < m-1: beta_k = ||v||, breakdown if beta_k <= brk * max|alpha|,
//   else q_{k+1} = v / beta_k.
// lane-0 broadcast into scalar registers: wave-uniform control flow around barriers
__device__ __forceinline__ int uni_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ double lz_block_sum(double x, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if (lane == 0) red[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    red[64] = s;
  }
  __syncthreads();
  const double r = uni_d(red[64]);
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(1024) k_lanczos_step(int k, int m_total, int B, long long N,
                                                       double* __restrict__ Q,
                                                       double* __restrict__ v,
                                                       double* __restrict__ alpha,
                                                       double* __restrict__ beta,
                                                       int* __restrict__ mlen,
                                                       int* __restrict__ active, double brk) {
  __shared__ double red[72];
  __shared__ double coef[kMaxLanczos];
  const int b = blockIdx.x;
  if (!uni_i(active[b])) return;
  // Q layout [m_total][B][N]: q_j of start vector b at Q + (j*B + b)*N
  const size_t qs = (size_t)B * N;
  double* Qb = Q + (size_t)b * N;
  double* vb = v + (size_t)b * N;
  const double* qk = Qb + (size_t)k * qs;
  double s = 0.0;
  for (long long i = threadIdx.x; i < N; i += blockDim.x) s += qk[i] * vb[i];
  const double a = lz_block_sum(s, red);
  const double bprev = k > 0 ? beta[(size_t)b * m_total + k - 1] : 0.0;
  const double* qkm = k > 0 ? Qb + (size_t)(k - 1) * qs : nullptr;
  for (long long i = threadIdx.x; i < N; i += blockDim.x) {
    double t = vb[i] - a * qk[i];
    if (k > 0) t -= bprev * qkm[i];
    vb[i] = t;
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j <= k; ++j) {
      const double* qj = Qb + (size_t)j * qs;
      double sj = 0.0;
      for (long long i = threadIdx.x; i < N; i += blockDim.x) sj += qj[i] * vb[i];
      const double cj = lz_block_sum(sj, red);
      if (threadIdx.x == 0) coef[j] = cj;
    }
    __syncthreads();
    for (long long i = threadIdx.x; i < N; i += blockDim.x) {
      double t = vb[i];
      for (int j = 0; j <= k; ++j) t -= coef[j] * Qb[(size_t)j * qs + i];
      vb[i] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) alpha[(size_t)b * m_total + k] = a;
  if (k < m_total - 1) {
    double s2 = 0.0;
    for (long long i = threadIdx.x; i < N; i += blockDim.x) s2 += vb[i] * vb[i];
    const double bk = sqrt(lz_block_sum(s2, red));
    double amax = 0.0;
    for (int j = 0; j < k; ++j) amax = fmax(amax, fabs(alpha[(size_t)b * m_total + j]));
    amax = uni_d(fmax(amax, fabs(a)));
    if (bk <= brk * amax) {
      if (threadIdx.x == 0) { mlen[b] = k + 1; active[b] = 0; }
      return;
    }
    const double inv = 1.0 / bk;
    double* qn = Qb + (size_t)(k + 1) * qs;
    for (long long i = threadIdx.x; i < N; i += blockDim.x) qn[i] = vb[i] * inv;
    if (threadIdx.x == 0) { beta[(size_t)b * m_total + k] = bk; mlen[b] = k + 2; }
  } else {
    if (threadIdx.x == 0) mlen[b] = k + 1;
  }
}

// ---------------------------------------------------------------------------
// Symmetric tridiagonal eigenproblem by the implicit-shift QL iteration
// (Bowdler, Martin, Reinsch and Wilkinson, 1968), tracking only the first
// row of the eigenvector matrix; then [f(T)]_11 = sum_i z_i^2 f(lambda_i).
__device__ __host__ inline int ql_first_row(int n, double* d, double* e, double* z) {
  for (int i = 0; i < n; ++i) z[i] = (i == 0) ? 1.0 : 0.0;
  if (n == 1) return 0;
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    int m;
    for (;;) {
      for (m = l; m < n - 1; ++m) {
        const double dd = fabs(d[m]) + fabs(d[m + 1]);
        if (fabs(e[m]) <= 2.2e-16 * dd) break;
      }
      if (m == l) break;
      if (++iter > 100) return 1;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
      double s = 1.0, c = 1.0, p = 0.0;
      int i;
      bool underflow = false;
      for (i = m - 1; i >= l; --i) {
        double f = s * e[i];
        const double bb = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          underflow = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * bb;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - bb;
        f = z[i + 1];
        z[i + 1] = s * z[i] + c * f;
        z[i] = c * z[i] - s * f;
      }
      if (underflow) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return 0;
}

__global__ void k_tridiag_quad(int B, int m_total, const double* __restrict__ alpha,
                               const double* __restrict__ beta, const int* __restrict__ mlen,
                               const long long* __restrict__ out_pos, double* __restrict__ dout,
                               int* __restrict__ fail) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double d[kMaxLanczos], e[kMaxLanczos], z[kMaxLanczos];
  const int m = mlen[b];
  for (int i = 0; i < m; ++i) d[i] = alpha[(size_t)b * m_total + i];
  for (int i = 0; i + 1 < m; ++i) e[i] = beta[(size_t)b * m_total + i];
  const int bad = ql_first_row(m, d, e, z);
  double acc = 0.0;
  for (int i = 0; i < m; ++i) acc += z[i] * z[i] * (log1p(-d[i]) + d[i]);
  dout[out_pos ? out_pos[b] : b] = acc;
  if (bad) atomicAdd(&fail[0], 1);
  if (m < m_total) atomicAdd(&fail[1], 1);
}

__global__ void k_scatter(const double* __restrict__ src, const long long* __restrict__ pos, int n,
                          double* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[pos[i]] = src[i];
}

// ---------------------------------------------------------------------------
// e_fine[j] = scale_fine * sum_k w_k dhat_k[j];  partials[block] = sum_j sum_k w_k dhat_k[j]
__global__ void __launch_bounds__(256) k_weighted_sum(const double* __restrict__ dhat,
                                                     const double* __restrict__ w, int n_omega,
                                                     long long N, double scale_fine,
                                                     double* __restrict__ e_fine,
                                                     double* __restrict__ partials) {
  __shared__ double red[8];
  const long long per = (N + gridDim.x - 1) / gridDim.x;
  const long long j0 = blockIdx.x * per;
  const long long j1 = j0 + per < N ? j0 + per : N;
  double s = 0.0;
  for (long long j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    double t = 0.0;
    for (int k = 0; k < n_omega; ++k) t += w[k] * dhat[(size_t)k * N + j];
    s += t;
    if (e_fine) e_fine[j] = scale_fine * t;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    partials[blockIdx.x] = t;
  }
}

int grid_for(long long n, int block) {
  long long g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_fill_d(double* p, double v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_d, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_i(int* p, int v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_d2f(const double* a, float* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_d2f, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}
hipError_t launch_set_onehot(double* q, long long stride, const long long* idx, int B, hipStream_t s) {
  hipLaunchKernelGGL(k_set_onehot, dim3((B + 63) / 64), dim3(64), 0, s, q, stride, idx, B);
  return hipGetLastError();
}

hipError_t launch_axis(const double* in, double* out, int B, int d0, int d1, int d2, int axis,
                       int n_out, const double* M, bool trans, const double* scale, hipStream_t s) {
  long long osz = (long long)d0 * d1 * d2;
  const int nin = axis == 0 ? d0 : (axis == 1 ? d1 : d2);
  osz = osz / nin * n_out;
  hipLaunchKernelGGL(k_axis, dim3(grid_for(osz * B, 256)), dim3(256), 0, s, in, out, B, d0, d1,
                     d2, axis, n_out, M, trans ? 1 : 0, scale);
  return hipGetLastError();
}

hipError_t launch_kin_scale(double* a, const double* kin, const double* sig_re,
                            const double* sig_im, int B, long long N, hipStream_t s) {
  hipLaunchKernelGGL(k_kin_scale, dim3(grid_for((long long)B * N, 256)), dim3(256), 0, s, a, kin,
                     sig_re, sig_im, B, N);
  return hipGetLastError();
}
hipError_t launch_gram(const double* psi, const double* u, int B, int n_occ, int ng, long long N,
                       int n_chunks, double* part, hipStream_t s) {
  const int ntm = (ng + GT - 1) / GT, ntn = (n_occ + GT - 1) / GT;
  hipLaunchKernelGGL(k_gram, dim3(n_chunks, B, ntm * ntn), dim3(256), 0, s, psi, u, n_occ, ng, N,
                     n_chunks, ntn, part);
  return hipGetLastError();
}
hipError_t launch_gram_finish(const double* part, int B, int n_occ, int ng, int n_chunks, double dV,
                              const double* eps, const double* omega, double2* G, hipStream_t s) {
  const long long total = (long long)B * ng * n_occ;
  hipLaunchKernelGGL(k_gram_finish, dim3(grid_for(total, 256)), dim3(256), 0, s, part, B, n_occ, ng,
                     n_chunks, dV, eps, omega, G);
  return hipGetLastError();
}
hipError_t launch_expand(const double* psi, const double2* G, int B, int n_occ, int ng, long long N,
                         double2* x64, hipStream_t s) {
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((n_occ + 63) / 64), (unsigned)B);
  hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, s, psi, G, n_occ, ng, N, x64);
  return hipGetLastError();
}
hipError_t launch_accumulate(const double* psi, const double2* x64, int B, int n_occ, long long N,
                             const int* active, double* racc, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate, dim3(grid_for((long long)B * N, 256)), dim3(256), 0, s, psi,
                     x64, B, n_occ, N, active, racc);
  return hipGetLastError();
}
hipError_t launch_lanczos_step(int k, int m_total, int B, long long N, double* Q, double* v,
                               double* alpha, double* beta, int* mlen, int* active, double brk,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_step, dim3(B), dim3(1024), 0, s, k, m_total, B, N, Q, v, alpha, beta,
                     mlen, active, brk);
  return hipGetLastError();
}
hipError_t launch_tridiag_quad(int B, int m_total, const double* alpha, const double* beta,
                                const int* mlen, const long long* out_pos, double* d, int* fail,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_quad, dim3((B + 63) / 64), dim3(64), 0, s, B, m_total, alpha, beta,
                     mlen, out_pos, d, fail);
  return hipGetLastError();
}

hipError_t launch_scatter(const double* src, const long long* pos, int n, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, src, pos, n, dst);
  return hipGetLastError();
}

hipError_t launch_weighted_sum(const double* dhat, const double* w, int n_omega, long long N,
                               double scale_fine, double* e_fine, double* partials, int nblocks,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_weighted_sum, dim3(nblocks), dim3(256), 0, s, dhat, w, n_omega, N,
                     scale_fine, e_fine, partials);
  return hipGetLastError();
}

}  // namespace rpa
