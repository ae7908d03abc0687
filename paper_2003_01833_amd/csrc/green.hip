// One block step of Green Iteration (the body of Algorithm 2 applied to every
// wavefunction of a block) around the batched treecode convolution:
//   f_o = V_eff psi_o;  psi'_o = -(1/2 pi) conv_{Yukawa-SS}(f_o; kappa_o = sqrt(-2 eps_o))
//     (Eqs. integral_operator and Hemlholtz_Greens_Function with the Section 4.3
//      subtraction);
//   eps'_o = eps_o - <V psi_o, psi_o - psi'_o> / <psi'_o, psi'_o>   (Eq. gradient-free);
//   psi'_o orthogonalized against psi'_j, j < o (classical Gram-Schmidt, twice)
//   and normalized; residual_o = ||psi'_o - psi_o||.
// Inner products use the quadrature weights. Every reduction is a fixed grid of
// block partial sums added on the host in block order, so the step is bitwise
// repeatable.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.hpp"

namespace tagi {
namespace {

constexpr int kRedBlocks = 256;   // partial sums per reduced quantity
constexpr int kRedThreads = 256;

// f[o][i] = V[i] psi[o][i]
__global__ void k_vpsi(const double* __restrict__ v, const double* __restrict__ psi, int64_t n,
                       int n_orb, double* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double vi = v[i];
  for (int o = 0; o < n_orb; ++o) f[(int64_t)o * n + i] = vi * psi[(int64_t)o * n + i];
}

// sum of one value over the block, in a fixed order
__device__ double block_sum(double v) {
  __shared__ double red[kRedThreads / kWave];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < kRedThreads / kWave; ++k) s += red[k];
  return s;
}

// blockIdx.y = orbital o: psi'[o] = -phi[o] / (2 pi), and the update's sums
//   num_o = sum w f_o (psi_o - psi'_o)  -> part[(2 o) kRedBlocks + block]
//   den_o = sum w psi'_o^2              -> part[(2 o + 1) kRedBlocks + block]
__global__ __launch_bounds__(kRedThreads) void k_update_sums(
    const double* __restrict__ w, const double* __restrict__ f, const double* __restrict__ psi,
    const double* __restrict__ phi, int64_t n, double* __restrict__ psi_new,
    double* __restrict__ part) {
  const int o = blockIdx.y;
  const double c = -1.0 / (2.0 * M_PI);
  double num = 0.0, den = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = (int64_t)o * n + i;
    const double p = c * phi[j];
    psi_new[j] = p;
    num += w[i] * f[j] * (psi[j] - p);
    den += w[i] * p * p;
  }
  num = block_sum(num);
  den = block_sum(den);
  if (threadIdx.x == 0) {
    part[(int64_t)(2 * o) * kRedBlocks + blockIdx.x] = num;
    part[(int64_t)(2 * o + 1) * kRedBlocks + blockIdx.x] = den;
  }
}

// blockIdx.y = k < o: sum_i w_i x[k][i] x[o][i]
__global__ __launch_bounds__(kRedThreads) void k_dots(const double* __restrict__ w,
                                                      const double* __restrict__ x, int64_t n,
                                                      int o, double* __restrict__ part) {
  const int k = blockIdx.y;
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v += w[i] * x[(int64_t)k * n + i] * x[(int64_t)o * n + i];
  v = block_sum(v);
  if (threadIdx.x == 0) part[(int64_t)k * kRedBlocks + blockIdx.x] = v;
}

// squared norm of row o -> part[block]
__global__ __launch_bounds__(kRedThreads) void k_norm(const double* __restrict__ w,
                                                      const double* __restrict__ x, int64_t n,
                                                      int o, double* __restrict__ part) {
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double xi = x[(int64_t)o * n + i];
    v += w[i] * xi * xi;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// x[o] = (x[o] - sum_{j<m} c_j x[j]) * scale
struct Axpy {
  int o, m;
  double c[kMaxOrb];
  double scale;
};

__global__ void k_axpy(double* __restrict__ x, int64_t n, Axpy a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = x[(int64_t)a.o * n + i];
  for (int j = 0; j < a.m; ++j) s -= a.c[j] * x[(int64_t)j * n + i];
  x[(int64_t)a.o * n + i] = s * a.scale;
}

// blockIdx.y = o: sum w (a_o - b_o)^2
__global__ __launch_bounds__(kRedThreads) void k_resid(const double* __restrict__ w,
                                                       const double* __restrict__ a,
                                                       const double* __restrict__ b, int64_t n,
                                                       double* __restrict__ part) {
  const int o = blockIdx.y;
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = a[(int64_t)o * n + i] - b[(int64_t)o * n + i];
    v += w[i] * d * d;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) part[(int64_t)o * kRedBlocks + blockIdx.x] = v;
}

// host sums of m quantities' block partials, each in block order
int gather_sums(const DBuf& part, int m, std::vector<double>& out, hipStream_t s) {
  std::vector<double> h((size_t)m * kRedBlocks);
  TAGI_HIP(hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  out.assign(m, 0.0);
  for (int k = 0; k < m; ++k)
    for (int b = 0; b < kRedBlocks; ++b) out[k] += h[(size_t)k * kRedBlocks + b];
  return TAGI_OK;
}

// f_o = V psi_o into the tree's Green buffers; kappa_o = sqrt(-2 eps_o)
int green_prepare(tagi_tree* t, const double* psi, const double* veff, int n_orb,
                  const double* eps, std::vector<double>& kappa, hipStream_t s) {
  const int64_t n = t->n;
  TAGI_TRY(t->green_f.ensure((size_t)n_orb * n * sizeof(double)));
  TAGI_TRY(t->green_phi.ensure((size_t)n_orb * n * sizeof(double)));
  TAGI_TRY(t->green_part.ensure((size_t)2 * kMaxOrb * kRedBlocks * sizeof(double)));
  hipLaunchKernelGGL(k_vpsi, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, veff, psi, n,
                     n_orb, t->green_f.as<double>());
  TAGI_HIP(hipGetLastError());
  kappa.resize(n_orb);
  for (int o = 0; o < n_orb; ++o) kappa[o] = std::sqrt(-2.0 * eps[o]);
  // the convolution's upward pass replaces the tree's charges
  ++t->charges_gen;
  return TAGI_OK;
}

// everything after the convolution phi_o = conv(f_o): psi' = -phi / (2 pi), the
// eigenvalue update, Gram-Schmidt, normalization and the residual
int green_finish(tagi_tree* t, const double* psi, const double* w, int n_orb, double* eps,
                 double* psi_out, double* resid, hipStream_t s) {
  const int64_t n = t->n;
  const int grid = (int)((n + 255) / 256);
  const double* f = t->green_f.as<double>();
  const double* phi = t->green_phi.as<double>();
  double* part = t->green_part.as<double>();
  // scale, and the eigenvalue update from psi' before orthogonalization
  hipLaunchKernelGGL(k_update_sums, dim3(kRedBlocks, n_orb), dim3(kRedThreads), 0, s, w, f, psi,
                     phi, n, psi_out, part);
  TAGI_HIP(hipGetLastError());
  std::vector<double> sums;
  TAGI_TRY(gather_sums(t->green_part, 2 * n_orb, sums, s));
  std::vector<double> eps_new(n_orb);
  for (int o = 0; o < n_orb; ++o) {
    if (!(sums[2 * o + 1] > 0.0)) {
      set_error("green step: wavefunction %d vanished after the convolution", o);
      return TAGI_E_ARG;
    }
    eps_new[o] = eps[o] - sums[2 * o] / sums[2 * o + 1];
  }
  // Gram-Schmidt in block order: two projection passes, then normalization
  for (int o = 0; o < n_orb; ++o) {
    for (int pass = 0; pass < 2 && o > 0; ++pass) {
      hipLaunchKernelGGL(k_dots, dim3(kRedBlocks, o), dim3(kRedThreads), 0, s, w, psi_out, n, o,
                         part);
      TAGI_HIP(hipGetLastError());
      std::vector<double> c;
      TAGI_TRY(gather_sums(t->green_part, o, c, s));
      Axpy a{};
      a.o = o;
      a.m = o;
      for (int j = 0; j < o; ++j) a.c[j] = c[j];
      a.scale = 1.0;
      hipLaunchKernelGGL(k_axpy, dim3(grid), dim3(256), 0, s, psi_out, n, a);
      TAGI_HIP(hipGetLastError());
    }
    // squared norm of row o: the dot of row o with itself (grid.y = 1, k = o)
    hipLaunchKernelGGL(k_norm, dim3(kRedBlocks), dim3(kRedThreads), 0, s, w, psi_out, n, o, part);
    TAGI_HIP(hipGetLastError());
    std::vector<double> nn;
    TAGI_TRY(gather_sums(t->green_part, 1, nn, s));
    if (!(nn[0] > 0.0)) {
      set_error("green step: wavefunction %d is linearly dependent on the earlier ones", o);
      return TAGI_E_ARG;
    }
    Axpy a{};
    a.o = o;
    a.m = 0;
    a.scale = 1.0 / std::sqrt(nn[0]);
    hipLaunchKernelGGL(k_axpy, dim3(grid), dim3(256), 0, s, psi_out, n, a);
    TAGI_HIP(hipGetLastError());
  }
  if (resid) {
    hipLaunchKernelGGL(k_resid, dim3(kRedBlocks, n_orb), dim3(kRedThreads), 0, s, w, psi_out, psi,
                       n, part);
    TAGI_HIP(hipGetLastError());
    std::vector<double> r;
    TAGI_TRY(gather_sums(t->green_part, n_orb, r, s));
    for (int o = 0; o < n_orb; ++o) resid[o] = std::sqrt(r[o]);
  }
  for (int o = 0; o < n_orb; ++o) eps[o] = eps_new[o];
  return TAGI_OK;
}

}  // namespace

int green_step(tagi_tree* t, const double* psi, const double* veff, const double* w, int n_orb,
               double* eps, double theta, int degree, int precision, double* psi_out,
               double* resid, hipStream_t s) {
  std::vector<double> kappa;
  TAGI_TRY(green_prepare(t, psi, veff, n_orb, eps, kappa, s));
  // psi'_o = G(eps_o) psi_o through the batched treecode
  TAGI_TRY(upward(t, t->green_f.as<double>(), w, n_orb, degree, s));
  const int ob = orbital_block_of(t, TAGI_YUKAWA_SS, precision);
  if (!lists_current(t, theta, degree) ||
      !(t->items_orb_block == ob && t->items_n_orb == n_orb && t->n_items > 0)) {
    phase_begin(t, kPhaseLists, s);
    int st = ensure_lists(t, theta, degree, s);
    if (st == TAGI_OK) st = ensure_schedule(t, ob, s);
    phase_end(t, kPhaseLists, s);
    if (st != TAGI_OK) return st;
  }
  TAGI_TRY(order_schedule(t, far_weight(TAGI_YUKAWA_SS, precision, false), s));
  TAGI_TRY(convolve(t, TAGI_YUKAWA_SS, kappa.data(), 1.0, precision, t->green_phi.as<double>(),
                    s));
  return green_finish(t, psi, w, n_orb, eps, psi_out, resid, s);
}

int green_step_learned(tagi_tree* t, const double* psi, const double* veff, const double* w,
                       int n_orb, double* eps, const float* params, const float* norm,
                       const double* tol, double theta_max, double theta_fb, int degree_fb,
                       int precision, double* psi_out, double* resid, hipStream_t s) {
  std::vector<double> kappa;
  TAGI_TRY(green_prepare(t, psi, veff, n_orb, eps, kappa, s));
  // the learned path forms its own per-degree proxy charges: the upward pass
  // stages f and w (lowest degree), and the lists follow the new charges
  TAGI_TRY(upward(t, t->green_f.as<double>(), w, n_orb, 1, s));
  learned_follow_charges(t);
  TAGI_TRY(convolve_learned(t, TAGI_YUKAWA_SS, kappa.data(), 1.0, params, norm, tol, theta_max,
                            theta_fb, degree_fb, precision, t->green_phi.as<double>(), s));
  return green_finish(t, psi, w, n_orb, eps, psi_out, resid, s);
}

}  // namespace tagi
