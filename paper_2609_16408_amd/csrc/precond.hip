// Shifted kinetic preconditioner (rpa_kinetic_precond_* in rpa.h).
//
// M = -1/2 Lap_h + sigma is inverted exactly in the eigenbasis of the FD
// Laplacian, which factorises per axis: forward transforms along x, y, z
// (k_axis with the transposed 1D basis), a complex divide by kin + sigma per
// mode (k_kin_scale), and the inverse transforms.  A plan owns the three 1D
// bases, the kinetic diagonal and its transform workspaces; it is separate
// from the problem handle so that applying it leaves the handle untouched.
// Errors are reported by status only.
#include "rpa.h"
#include "internal.h"

#include <cmath>
#include <vector>

struct rpa_kinetic_precond_s {
  int n[3] = {0, 0, 0};
  long long N = 0;
  double* V[3] = {nullptr, nullptr, nullptr};  // [grid point][mode], orthonormal
  double* kin = nullptr;                       // -1/2 (lam_x + lam_y + lam_z) per mode
  double* ws[2] = {nullptr, nullptr};          // transform workspaces
  size_t ws_bytes = 0;
  double* sig = nullptr;                       // [2][cap] shifts on the device
  int sig_cap = 0;
};

namespace {

// Weights of the 12th-order central second derivative (Fornberg's closed
// form for order 2R): w_k = 2 (-1)^(k+1) (R!)^2 / (k^2 (R-k)! (R+k)!),
// w_0 = -2 sum_k w_k.
void second_derivative_weights(double* w) {
  const int R = rpa::kRadius;
  auto fact = [](int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; };
  double s = 0.0;
  for (int k = 1; k <= R; ++k) {
    w[k] = 2.0 * ((k % 2) ? 1.0 : -1.0) * fact(R) * fact(R) /
           ((double)k * k * fact(R - k) * fact(R + k));
    s += w[k];
  }
  w[0] = -2.0 * s;
}

// The periodic 1D second-derivative matrix is circulant, so the real Fourier
// modes diagonalise it: mode 0 is constant, modes 2m-1 and 2m are cos and
// sin of wavenumber m, and for even n the last mode alternates in sign.
// V[i * n + j] is mode j at point i; lam[j] its eigenvalue.
void fourier_basis(int n, double h, const double* w, std::vector<double>& V,
                   std::vector<double>& lam) {
  V.assign((size_t)n * n, 0.0);
  lam.assign(n, 0.0);
  auto eig = [&](int m) {
    double s = w[0];
    for (int p = 1; p <= rpa::kRadius; ++p) s += 2.0 * w[p] * std::cos(2.0 * M_PI * m * p / n);
    return s / (h * h);
  };
  for (int i = 0; i < n; ++i) V[(size_t)i * n] = 1.0 / std::sqrt((double)n);
  int j = 1;
  for (int m = 1; 2 * m < n; ++m, j += 2) {
    for (int i = 0; i < n; ++i) {
      V[(size_t)i * n + j] = std::sqrt(2.0 / n) * std::cos(2.0 * M_PI * m * i / n);
      V[(size_t)i * n + j + 1] = std::sqrt(2.0 / n) * std::sin(2.0 * M_PI * m * i / n);
    }
    lam[j] = lam[j + 1] = eig(m);
  }
  if (n % 2 == 0) {
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = ((i % 2) ? -1.0 : 1.0) / std::sqrt((double)n);
    lam[j] = eig(n / 2);
  }
}

void release(rpa_kinetic_precond p) {
  if (!p) return;
  for (double* v : p->V) if (v) (void)hipFree(v);
  for (double* v : p->ws) if (v) (void)hipFree(v);
  if (p->kin) (void)hipFree(p->kin);
  if (p->sig) (void)hipFree(p->sig);
  delete p;
}

}  // namespace

rpa_status rpa_kinetic_precond_create(const int32_t* n, const double* L, void* stream,
                                      rpa_kinetic_precond* out) {
  if (!n || !L || !out) return RPA_E_ARG;
  *out = nullptr;
  for (int d = 0; d < 3; ++d)
    if (n[d] < 7 || n[d] > 4096 || !std::isfinite(L[d]) || !(L[d] > 0.0)) return RPA_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  auto* p = new rpa_kinetic_precond_s;
  p->N = (long long)n[0] * n[1] * n[2];
  double w[rpa::kRadius + 1];
  second_derivative_weights(w);
  std::vector<double> V[3], lam[3];
  for (int d = 0; d < 3; ++d) {
    p->n[d] = n[d];
    fourier_basis(n[d], L[d] / n[d], w, V[d], lam[d]);
  }
  std::vector<double> kin((size_t)p->N);
  for (int i = 0; i < n[0]; ++i)
    for (int j = 0; j < n[1]; ++j)
      for (int k = 0; k < n[2]; ++k)
        kin[((size_t)i * n[1] + j) * n[2] + k] = -0.5 * (lam[0][i] + lam[1][j] + lam[2][k]);
  bool ok = hipMalloc((void**)&p->kin, (size_t)p->N * sizeof(double)) == hipSuccess;
  for (int d = 0; d < 3 && ok; ++d)
    ok = hipMalloc((void**)&p->V[d], V[d].size() * sizeof(double)) == hipSuccess;
  if (!ok) { (void)hipGetLastError(); release(p); return RPA_E_OOM; }
  hipError_t e = hipMemcpyAsync(p->kin, kin.data(), kin.size() * sizeof(double),
                                hipMemcpyHostToDevice, s);
  for (int d = 0; d < 3 && e == hipSuccess; ++d)
    e = hipMemcpyAsync(p->V[d], V[d].data(), V[d].size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host tables go out of scope
  if (e != hipSuccess) { (void)hipGetLastError(); release(p); return RPA_E_HIP; }
  *out = p;
  return RPA_OK;
}

rpa_status rpa_kinetic_precond_apply(rpa_kinetic_precond p, int32_t nvec, const double* sigma_re,
                                     const double* sigma_im, const double* x, double* y,
                                     void* stream) {
  if (!p || nvec < 1 || nvec > (1 << 24) || !sigma_re || !sigma_im || !x || !y) return RPA_E_ARG;
  for (int b = 0; b < nvec; ++b)
    if (!std::isfinite(sigma_re[b]) || !std::isfinite(sigma_im[b]) || !(sigma_re[b] > 0.0))
      return RPA_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int B = 2 * nvec;  // the real and imaginary halves transform as separate real fields
  const size_t bytes = (size_t)B * p->N * sizeof(double);
  if (bytes > p->ws_bytes) {
    // hipFree waits for the device, so no earlier apply still uses the old buffers
    for (double*& v : p->ws) { if (v) (void)hipFree(v); v = nullptr; }
    p->ws_bytes = 0;
    for (double*& v : p->ws)
      if (hipMalloc((void**)&v, bytes) != hipSuccess) { (void)hipGetLastError(); return RPA_E_OOM; }
    p->ws_bytes = bytes;
  }
  if (nvec > p->sig_cap) {
    if (p->sig) (void)hipFree(p->sig);
    p->sig = nullptr;
    p->sig_cap = 0;
    if (hipMalloc((void**)&p->sig, 2 * (size_t)nvec * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return RPA_E_OOM;
    }
    p->sig_cap = nvec;
  }
  double* a = p->ws[0];
  double* b = p->ws[1];
  const int* n = p->n;
  hipError_t e = hipMemcpyAsync(p->sig, sigma_re, nvec * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->sig + nvec, sigma_im, nvec * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = rpa::launch_axis(x, a, B, n[0], n[1], n[2], 0, n[0], p->V[0], true, nullptr, s);
  if (e == hipSuccess) e = rpa::launch_axis(a, b, B, n[0], n[1], n[2], 1, n[1], p->V[1], true, nullptr, s);
  if (e == hipSuccess) e = rpa::launch_axis(b, a, B, n[0], n[1], n[2], 2, n[2], p->V[2], true, nullptr, s);
  if (e == hipSuccess) e = rpa::launch_kin_scale(a, p->kin, p->sig, p->sig + nvec, nvec, p->N, s);
  if (e == hipSuccess) e = rpa::launch_axis(a, b, B, n[0], n[1], n[2], 2, n[2], p->V[2], false, nullptr, s);
  if (e == hipSuccess) e = rpa::launch_axis(b, a, B, n[0], n[1], n[2], 1, n[1], p->V[1], false, nullptr, s);
  if (e == hipSuccess) e = rpa::launch_axis(a, y, B, n[0], n[1], n[2], 0, n[0], p->V[0], false, nullptr, s);
  if (e != hipSuccess) { (void)hipGetLastError(); return RPA_E_HIP; }
  return RPA_OK;
}

rpa_status rpa_kinetic_precond_destroy(rpa_kinetic_precond p) {
  if (!p) return RPA_OK;
  (void)hipDeviceSynchronize();
  release(p);
  return RPA_OK;
}
