// Learned degree/MAC selector: training data from the method itself, and the
// network's training kernels.
//
// Samples. For a candidate batch-cluster pair (B, C) and a degree n, the label is
// the largest absolute error, over up to kSampleT targets spread evenly over B
// (all of them when B holds at most kSampleT), of the
// particle-cluster approximation of Eq. particle-cluster-approx-rearranged against
// the direct sum of Eq. direct-sum_2 (both with the Section 4.3 subtraction, i.e.
// the pair's contribution a1 - f_i a2). Features: cluster radius r_C, distance
// from the batch's bounding sphere to the cluster centre R - r_B, the decay rate
// (kappa, or 0 for Coulomb), N_S and l1 = |q^_C|_1 + g max_B |f| |w^_C|_1 from the
// degree-4 proxy charges: the size of the charges q^ - f_i w^ the pair's far field
// carries, the subtracted ones weighted by g = 1 (Yukawa-SS) or the Gaussian at
// the least batch-cluster distance max(R - r_B - r_C, 0) (Coulomb-SS).
//
// Network (FP32): 5 inputs, three tanh layers of 64, 9 linear outputs (the
// log10 errors at degrees 4..12). Training is mini-batch Adam with one kernel per
// dense layer in each direction; every reduction runs in a fixed order, so
// training is repeatable bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "interact_impl.hpp"
#include "internal.hpp"

namespace tagi {
namespace {

using namespace ik;

constexpr int kSelIn = 5, kSelH = 64, kSelOut = 9;

// ---------------------------------------------------------------------------
// sample generation

constexpr int kSampleT = 256;  // targets per pair a label is taken over

// k-th sampled target of a batch [tb, tb + nb): evenly spread, all when nb <= kSampleT
__device__ inline int sample_target(int tb, int nb, int k) {
  const int nt = min(nb, kSampleT);
  return tb + (int)(((int64_t)k * nb) / nt);
}

// exact (direct) contribution of cluster C to the sampled targets of batch B;
// KER is TAGI_YUKAWA_SS (decay kappa) or TAGI_COULOMB_SS (Gaussian 1/a^2 = A.ia2)
template <int KER>
__global__ __launch_bounds__(256) void k_pair_exact(const int2* __restrict__ pairs, int n_pairs,
                                                    InteractArgs A, double kappa,
                                                    double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int p = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + threadIdx.x / kWave));
  if (p >= n_pairs) return;
  const int2 pr = pairs[p];
  const int B = pr.x, C = pr.y;
  const int tb = A.nbeg[B], nb = A.nend[B] - tb;
  const int nt = min(nb, kSampleT);
  const double kl2[1] = {-kappa * kLog2e};
  const double* qr[1] = {A.qs};
  for (int k0 = 0; k0 < nt; k0 += kWave) {
    const bool live = k0 + lane < nt;
    const int i = sample_target(tb, nb, live ? k0 + lane : 0);
    double a1[1] = {0.0}, a2[1] = {0.0};
    near_range<KER, 1>(A.xs[i], A.ys[i], A.zs[i], A.nbeg[C], A.nend[C], A.xs, A.ys, A.zs, A.ws,
                       qr, kl2, -A.ia2 * kLog2e, a1, a2);
    if (live) out[(int64_t)p * kSampleT + k0 + lane] = __builtin_fma(-A.fs[i], a2[0], a1[0]);
  }
}

// approximated contribution at the degree of the current upward pass, its largest
// error over the sampled targets; pairs without proxies at this degree write NaN
template <int KER>
__global__ __launch_bounds__(256) void k_pair_approx(const int2* __restrict__ pairs, int n_pairs,
                                                     InteractArgs A, double kappa,
                                                     const double* __restrict__ exact,
                                                     float* __restrict__ err) {
  const int lane = threadIdx.x % kWave;
  const int p = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + threadIdx.x / kWave));
  if (p >= n_pairs) return;
  const int2 pr = pairs[p];
  const int B = pr.x, C = pr.y;
  const int slot = A.slot_of[C];
  const int tb = A.nbeg[B], nb = A.nend[B] - tb;
  const int nt = min(nb, kSampleT);
  double e = 0.0;
  if (slot >= 0) {
    const int np1 = A.degree + 1;
    const int K = np1 * np1 * np1;
    const double kl2[1] = {-kappa * kLog2e};
    const double* qk[1] = {A.qhat + (int64_t)slot * K};
    for (int k0 = 0; k0 < nt; k0 += kWave) {
      const bool live = k0 + lane < nt;
      const int i = sample_target(tb, nb, live ? k0 + lane : 0);
      double a1[1] = {0.0}, a2[1] = {0.0};
      far_cluster<KER, 1, 0>(A.xs[i], A.ys[i], A.zs[i], np1, A.pnodes + (int64_t)slot * 3 * np1,
                             A.what + (int64_t)slot * K, qk, kl2, -A.ia2 * kLog2e, a1, a2);
      const double u = __builtin_fma(-A.fs[i], a2[0], a1[0]);
      if (live) e = fmax(e, fabs(u - exact[(int64_t)p * kSampleT + k0 + lane]));
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) e = fmax(e, __shfl_xor(e, off));
  if (lane == 0) err[p] = slot >= 0 ? (float)e : NAN;
}

// l1 norm of each slot's charges (q points at one charge set, [n_approx][K]),
// scattered to a per-node array
__global__ void k_l1_scatter(const double* __restrict__ q, const int32_t* __restrict__ node,
                             int K, float* __restrict__ out) {
  const int slot = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < K; k += kWave) s += fabs(q[(int64_t)slot * K + k]);
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (threadIdx.x == 0) out[node[slot]] = (float)s;
}

// max |f| over each batch's targets, per orbital: out[o][leaf]
__global__ void k_leaf_fmax(const int32_t* __restrict__ leaf_node,
                            const int32_t* __restrict__ nbeg, const int32_t* __restrict__ nend,
                            const double* __restrict__ fs, int64_t n, int n_leaves,
                            float* __restrict__ out) {
  const int b = blockIdx.x, o = blockIdx.y;
  const int c = leaf_node[b];
  double m = 0.0;
  for (int i = nbeg[c] + threadIdx.x; i < nend[c]; i += kWave) m = fmax(m, fabs(fs[(int64_t)o * n + i]));
  for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (threadIdx.x == 0) out[(int64_t)o * n_leaves + b] = (float)m;
}

InteractArgs args_of(tagi_tree* t) {
  InteractArgs A{};
  A.nbeg = t->nd_begin.as<int32_t>();
  A.nend = t->nd_end.as<int32_t>();
  A.slot_of = t->px.slot_of.as<int32_t>();
  A.xs = t->xs.as<double>();
  A.ys = t->ys.as<double>();
  A.zs = t->zs.as<double>();
  A.qs = t->qs.as<double>();
  A.ws = t->ws.as<double>();
  A.fs = t->fs.as<double>();
  A.pnodes = t->px.pnodes.as<double>();
  A.qhat = t->px.qhat.as<double>();
  A.what = t->px.what.as<double>();
  A.geom = t->nd_geom.as<double>();
  A.n = t->n;
  A.n_orb = t->n_orb;
  A.n_approx = t->px.n_approx;
  A.degree = t->degree;
  targets_are_sources(A);
  return A;
}

// ---------------------------------------------------------------------------
// network training (FP32)

// H[b][o] = act(sum_i W[o][i] X[b][i] + bias[o]), act = tanh or identity
__global__ void k_dense_fwd(const float* __restrict__ X, int nin, const float* __restrict__ W,
                            const float* __restrict__ bias, int nout, int m, int act,
                            float* __restrict__ H) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)m * nout) return;
  const int b = (int)(id / nout), o = (int)(id % nout);
  float s = bias[o];
  for (int i = 0; i < nin; ++i) s = __builtin_fmaf(W[o * nin + i], X[(int64_t)b * nin + i], s);
  H[id] = act ? tanhf(s) : s;
}

// Asymmetric squared loss: residual r = out - y, weight a = 1 for r >= 0 and
// kUnder for r < 0 (a prediction below the observed error costs kUnder times
// more, which keeps the selector on the safe side);
// G[b][k] = mask a r / count, loss partial per block = sum mask a r^2 / (2 count)
constexpr float kUnder = 4.0f;
__global__ void k_out_grad(const float* __restrict__ out, const float* __restrict__ Y,
                           const float* __restrict__ M, int64_t total, float inv_cnt,
                           float* __restrict__ G, float* __restrict__ loss_part) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (id < total) {
    const float r = (out[id] - Y[id]) * M[id];
    const float a = r < 0.0f ? kUnder : 1.0f;
    G[id] = a * r * inv_cnt;
    l = 0.5f * a * r * r * inv_cnt;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) l += __shfl_xor(l, off);
  __shared__ float red[4];
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// dW[o][i] = sum_b G[b][o] H[b][i];  db[o] = sum_b G[b][o]  (thread per weight)
__global__ void k_dense_wgrad(const float* __restrict__ G, int nout, const float* __restrict__ H,
                              int nin, int m, float* __restrict__ dW, float* __restrict__ db) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nout * (nin + 1)) return;
  const int o = id / (nin + 1), i = id % (nin + 1);
  float s = 0.0f;
  if (i < nin) {
    for (int b = 0; b < m; ++b) s = __builtin_fmaf(G[(int64_t)b * nout + o], H[(int64_t)b * nin + i], s);
    dW[o * nin + i] = s;
  } else {
    for (int b = 0; b < m; ++b) s += G[(int64_t)b * nout + o];
    db[o] = s;
  }
}

// Gin[b][i] = (sum_o G[b][o] W[o][i]) (1 - H[b][i]^2)   (back through tanh)
__global__ void k_dense_bgrad(const float* __restrict__ G, int nout, const float* __restrict__ W,
                              const float* __restrict__ H, int nin, int m,
                              float* __restrict__ Gin) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)m * nin) return;
  const int b = (int)(id / nin), i = (int)(id % nin);
  float s = 0.0f;
  for (int o = 0; o < nout; ++o) s = __builtin_fmaf(G[(int64_t)b * nout + o], W[o * nin + i], s);
  const float h = H[id];
  Gin[id] = s * (1.0f - h * h);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const float gi = g[id];
  const float mi = b1 * m[id] + (1.0f - b1) * gi;
  const float vi = b2 * v[id] + (1.0f - b2) * gi * gi;
  m[id] = mi;
  v[id] = vi;
  p[id] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather_rows(const float* __restrict__ src, const int32_t* __restrict__ idx,
                              int width, int m, float* __restrict__ dst) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)m * width) return;
  const int r = (int)(id / width), c = (int)(id % width);
  dst[id] = src[(int64_t)idx[r] * width + c];
}

int grid_of(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

}  // namespace

int selector_param_count() {
  return (kSelIn * kSelH + kSelH) + 2 * (kSelH * kSelH + kSelH) + (kSelH * kSelOut + kSelOut);
}

int l1_to_nodes(const ProxySet& ps, int set, float* out, hipStream_t s) {
  if (ps.n_approx == 0) return TAGI_OK;
  const int np1 = ps.degree + 1;
  const int64_t K = (int64_t)np1 * np1 * np1;
  const double* q = set < ps.n_orb ? ps.qhat.as<double>() + (int64_t)set * ps.n_approx * K
                                   : ps.what.as<double>();
  hipLaunchKernelGGL(k_l1_scatter, dim3(ps.n_approx), dim3(kWave), 0, s, q,
                     ps.node.as<int32_t>(), (int)K, out);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

int leaf_fmax(tagi_tree* t, float* out, hipStream_t s) {
  const int nl = (int)t->leaves.size();
  hipLaunchKernelGGL(k_leaf_fmax, dim3(nl, t->n_orb), dim3(kWave), 0, s, t->leaf_node.as<int32_t>(),
                     t->nd_begin.as<int32_t>(), t->nd_end.as<int32_t>(), t->fs.as<double>(), t->n,
                     nl, out);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

// Forward, loss gradient and backward of one mini-batch; fills grads (same layout
// as params) and returns the loss. Buffers: acts = 4 * m * 64 floats, g = 2 * m * 64.
static int mlp_batch_grad(const float* params, const float* X, const float* Y, const float* M,
                          int m, float inv_cnt, float* acts, float* gbuf, float* grads,
                          float* loss_part, int* n_loss_part, hipStream_t s) {
  const int sizes[5] = {kSelIn, kSelH, kSelH, kSelH, kSelOut};
  const float* W[4];
  const float* Bv[4];
  float* dW[4];
  float* dB[4];
  int off = 0;
  for (int l = 0; l < 4; ++l) {
    W[l] = params + off;
    dW[l] = grads + off;
    off += sizes[l] * sizes[l + 1];
    Bv[l] = params + off;
    dB[l] = grads + off;
    off += sizes[l + 1];
  }
  float* H[5];
  H[0] = const_cast<float*>(X);
  for (int l = 1; l <= 4; ++l) H[l] = acts + (int64_t)(l - 1) * m * kSelH;
  for (int l = 0; l < 4; ++l) {
    hipLaunchKernelGGL(k_dense_fwd, dim3(grid_of((int64_t)m * sizes[l + 1])), dim3(256), 0, s, H[l],
                       sizes[l], W[l], Bv[l], sizes[l + 1], m, l < 3 ? 1 : 0, H[l + 1]);
  }
  float* G = gbuf;
  float* G2 = gbuf + (int64_t)m * kSelH;
  const int64_t tot = (int64_t)m * kSelOut;
  *n_loss_part = grid_of(tot);
  hipLaunchKernelGGL(k_out_grad, dim3(*n_loss_part), dim3(256), 0, s, H[4], Y, M, tot, inv_cnt, G,
                     loss_part);
  for (int l = 3; l >= 0; --l) {
    hipLaunchKernelGGL(k_dense_wgrad, dim3(grid_of(sizes[l + 1] * (sizes[l] + 1))), dim3(256), 0,
                       s, G, sizes[l + 1], H[l], sizes[l], m, dW[l], dB[l]);
    if (l > 0) {
      hipLaunchKernelGGL(k_dense_bgrad, dim3(grid_of((int64_t)m * sizes[l])), dim3(256), 0, s, G,
                         sizes[l + 1], W[l], H[l], sizes[l], m, G2);
      std::swap(G, G2);
    }
  }
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

int selector_grad(const float* params, const float* X, const float* Y, const float* M, int64_t m,
                  float* grads, float* loss, hipStream_t s) {
  StreamScratch scratch(s);
  float *acts = nullptr, *gbuf = nullptr, *lp = nullptr;
  TAGI_TRY(scratch.alloc(&acts, (size_t)4 * m * kSelH));
  TAGI_TRY(scratch.alloc(&gbuf, (size_t)2 * m * kSelH));
  TAGI_TRY(scratch.alloc(&lp, (size_t)grid_of(m * kSelOut)));
  std::vector<float> hm(m * kSelOut);
  TAGI_HIP(hipMemcpyAsync(hm.data(), M, hm.size() * sizeof(float), hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  double cnt = 0.0;
  for (float v : hm) cnt += v;
  int nlp = 0;
  int st = mlp_batch_grad(params, X, Y, M, (int)m, (float)(1.0 / std::max(cnt, 1.0)), acts, gbuf,
                          grads, lp, &nlp, s);
  if (st == TAGI_OK && loss) {
    std::vector<float> h(nlp);
    TAGI_HIP(hipMemcpyAsync(h.data(), lp, nlp * sizeof(float), hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipStreamSynchronize(s));
    double l = 0.0;
    for (float v : h) l += v;
    *loss = (float)l;
  }
  return st;
}

int selector_train(float* params, const float* X, const float* Y, const float* M, int64_t m,
                   const int32_t* order, int epochs, int batch, float lr, float* loss_hist,
                   hipStream_t s) {
  if (m < batch) {
    set_error("selector_train: %lld samples are fewer than one mini-batch of %d", (long long)m, batch);
    return TAGI_E_ARG;
  }
  const int np = selector_param_count();
  StreamScratch scratch(s);
  float *acts, *gbuf, *lp, *grads, *mom, *vel, *bx, *by, *bm;
  int32_t* didx;
  TAGI_TRY(scratch.alloc(&acts, (size_t)4 * batch * kSelH));
  TAGI_TRY(scratch.alloc(&gbuf, (size_t)2 * batch * kSelH));
  TAGI_TRY(scratch.alloc(&lp, (size_t)grid_of((int64_t)batch * kSelOut)));
  TAGI_TRY(scratch.alloc(&grads, (size_t)np));
  TAGI_TRY(scratch.alloc(&mom, (size_t)np));
  TAGI_TRY(scratch.alloc(&vel, (size_t)np));
  TAGI_TRY(scratch.alloc(&bx, (size_t)batch * kSelIn));
  TAGI_TRY(scratch.alloc(&by, (size_t)batch * kSelOut));
  TAGI_TRY(scratch.alloc(&bm, (size_t)batch * kSelOut));
  TAGI_TRY(scratch.alloc(&didx, (size_t)(m + batch)));
  TAGI_HIP(hipMemsetAsync(mom, 0, np * sizeof(float), s));
  TAGI_HIP(hipMemsetAsync(vel, 0, np * sizeof(float), s));
  // the order, followed by its first `batch` entries, so any window of `batch`
  // consecutive rows starting below m is contiguous
  std::vector<int32_t> hord((size_t)(m + batch));
  for (int64_t r = 0; r < m + batch; ++r) hord[r] = order[r % m];
  TAGI_HIP(hipMemcpyAsync(didx, hord.data(), hord.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  std::vector<float> hm((size_t)m * kSelOut);
  TAGI_HIP(hipMemcpyAsync(hm.data(), M, hm.size() * sizeof(float), hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int64_t nb = m / batch;        // mini-batches per epoch
  const int64_t shift = batch / 3 + 1; // epochs start at shifted windows of the order
  int step = 0, st = TAGI_OK;
  std::vector<float> hl;
  for (int ep = 0; ep < epochs && st == TAGI_OK; ++ep) {
    double ep_loss = 0.0;
    for (int64_t bi = 0; bi < nb; ++bi) {
      const int64_t base = (bi * batch + ep * shift) % m;
      double cnt = 0.0;
      for (int r = 0; r < batch; ++r)
        for (int k = 0; k < kSelOut; ++k) cnt += hm[(size_t)hord[base + r] * kSelOut + k];
      const int32_t* rows = didx + base;
      hipLaunchKernelGGL(k_gather_rows, dim3(grid_of((int64_t)batch * kSelIn)), dim3(256), 0, s, X, rows, kSelIn, batch, bx);
      hipLaunchKernelGGL(k_gather_rows, dim3(grid_of((int64_t)batch * kSelOut)), dim3(256), 0, s, Y, rows, kSelOut, batch, by);
      hipLaunchKernelGGL(k_gather_rows, dim3(grid_of((int64_t)batch * kSelOut)), dim3(256), 0, s, M, rows, kSelOut, batch, bm);
      int nlp = 0;
      st = mlp_batch_grad(params, bx, by, bm, batch, (float)(1.0 / std::max(cnt, 1.0)), acts, gbuf,
                          grads, lp, &nlp, s);
      if (st != TAGI_OK) break;
      ++step;
      const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
      hipLaunchKernelGGL(k_adam, dim3(grid_of(np)), dim3(256), 0, s, params, grads, mom, vel, np,
                         lr, b1, b2, eps, c1, c2);
      if (loss_hist) {
        hl.resize(nlp);
        TAGI_HIP(hipMemcpyAsync(hl.data(), lp, nlp * sizeof(float), hipMemcpyDeviceToHost, s));
        TAGI_HIP(hipStreamSynchronize(s));
        for (float v : hl) ep_loss += v;
      }
    }
    if (loss_hist) loss_hist[ep] = (float)(ep_loss / std::max<int64_t>(nb, 1));
  }
  TAGI_HIP(hipGetLastError());
  TAGI_HIP(hipStreamSynchronize(s));
  return st;
}

int selector_samples(tagi_tree* t, const double* f, const double* w, int kernel, double kappa,
                     double alpha, double theta_max, int64_t max_pairs, float* feat, float* err,
                     int32_t* pair_ids, int64_t* n_out, hipStream_t s) {
  const bool coul = kernel == TAGI_COULOMB_SS;
  if (coul) kappa = 0.0;  // the decay rate of 1/r
  // candidate pairs: the far pairs of the lists at (theta_max, degree 4)
  const int d0 = 4;
  ++t->charges_gen;
  TAGI_TRY(upward(t, f, w, 1, d0, s));
  TAGI_TRY(ensure_lists(t, theta_max, d0, s));
  const int nl = (int)t->leaves.size();
  std::vector<int32_t> fid(std::max<int64_t>(t->n_far, 1));
  if (t->n_far)
    TAGI_HIP(hipMemcpyAsync(fid.data(), t->far_id.p, t->n_far * 4, hipMemcpyDeviceToHost, s));
  // l1 norms of the degree-4 proxy charges of f w and of w per node, and max |f|
  // per batch: the pair's feature is ||q^||_1 + max_B |f| ||w^||_1, which bounds
  // the l1 norm of the subtracted charges q^ - f_i w^ seen by any target of B
  const int nn = (int)t->nodes.size();
  std::vector<float> l1f(nn, 0.0f), l1w(nn, 0.0f), fmaxb(nl, 0.0f);
  {
    StreamScratch scratch(s);
    float* dbuf;
    TAGI_TRY(scratch.alloc(&dbuf, (size_t)(2 * nn + nl)));
    TAGI_HIP(hipMemsetAsync(dbuf, 0, (size_t)(2 * nn + nl) * sizeof(float), s));
    TAGI_TRY(l1_to_nodes(t->px, 0, dbuf, s));
    TAGI_TRY(l1_to_nodes(t->px, 1, dbuf + nn, s));
    TAGI_TRY(leaf_fmax(t, dbuf + 2 * nn, s));
    TAGI_HIP(hipMemcpyAsync(l1f.data(), dbuf, nn * sizeof(float), hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipMemcpyAsync(l1w.data(), dbuf + nn, nn * sizeof(float), hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipMemcpyAsync(fmaxb.data(), dbuf + 2 * nn, nl * sizeof(float), hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipStreamSynchronize(s));
  }
  std::vector<int32_t> leaf_index(nn, -1);
  for (int b = 0; b < nl; ++b) leaf_index[t->leaves[b]] = b;
  TAGI_HIP(hipStreamSynchronize(s));
  // evenly strided subset of the far pairs, in list order
  std::vector<int2> pairs;
  const int64_t nf = t->n_far;
  const int64_t want = std::min<int64_t>(max_pairs, nf);
  if (want > 0) {
    pairs.reserve(want);
    int b = 0;
    for (int64_t k = 0; k < want; ++k) {
      const int64_t e = k * nf / want;
      while (t->h_far_off[b + 1] <= e) ++b;
      pairs.push_back({t->leaves[b], fid[e]});
    }
  }
  const int np = (int)pairs.size();
  *n_out = np;
  if (np == 0) return TAGI_OK;
  for (int p = 0; p < np; ++p) {
    const HostNode& B = t->nodes[pairs[p].x];
    const HostNode& C = t->nodes[pairs[p].y];
    double cb[3], cc[3], hb[3], hc[3];
    for (int k = 0; k < 3; ++k) {
      cb[k] = 0.5 * (B.lo[k] + B.hi[k]);
      cc[k] = 0.5 * (C.lo[k] + C.hi[k]);
      hb[k] = 0.5 * (B.hi[k] - B.lo[k]);
      hc[k] = 0.5 * (C.hi[k] - C.lo[k]);
    }
    const double rb = std::sqrt(hb[0] * hb[0] + hb[1] * hb[1] + hb[2] * hb[2]);
    const double rc = std::sqrt(hc[0] * hc[0] + hc[1] * hc[1] + hc[2] * hc[2]);
    const double R = std::sqrt((cb[0] - cc[0]) * (cb[0] - cc[0]) + (cb[1] - cc[1]) * (cb[1] - cc[1]) +
                               (cb[2] - cc[2]) * (cb[2] - cc[2]));
    const int Cn = pairs[p].y;
    feat[p * 5 + 0] = (float)rc;
    feat[p * 5 + 1] = (float)(R - rb);
    feat[p * 5 + 2] = (float)kappa;  // decay rate: kappa, or 0 for Coulomb
    feat[p * 5 + 3] = (float)(C.end - C.begin);
    // subtracted charges weighted by their kernel relative to the first one's:
    // 1 for Yukawa-SS, the Gaussian at the least batch-cluster distance for
    // Coulomb-SS
    double gsub = 1.0;
    if (coul) {
      const double dm = std::max(R - rb - rc, 0.0);
      gsub = std::exp(-dm * dm / (alpha * alpha));
    }
    feat[p * 5 + 4] = (float)(l1f[Cn] + gsub * fmaxb[leaf_index[pairs[p].x]] * l1w[Cn]);
    if (pair_ids) {
      pair_ids[2 * p] = pairs[p].x;
      pair_ids[2 * p + 1] = pairs[p].y;
    }
  }
  StreamScratch scratch(s);
  int2* dp;
  double* exact;
  float* derr;
  TAGI_TRY(scratch.alloc(&dp, (size_t)np));
  TAGI_TRY(scratch.alloc(&exact, (size_t)np * kSampleT));
  TAGI_TRY(scratch.alloc(&derr, (size_t)np));
  TAGI_HIP(hipMemcpyAsync(dp, pairs.data(), np * sizeof(int2), hipMemcpyHostToDevice, s));
  const double ia2 = coul ? 1.0 / (alpha * alpha) : 0.0;
  InteractArgs A = args_of(t);
  A.ia2 = ia2;
  if (coul)
    hipLaunchKernelGGL(k_pair_exact<TAGI_COULOMB_SS>, dim3((np + 3) / 4), dim3(256), 0, s, dp, np,
                       A, kappa, exact);
  else
    hipLaunchKernelGGL(k_pair_exact<TAGI_YUKAWA_SS>, dim3((np + 3) / 4), dim3(256), 0, s, dp, np,
                       A, kappa, exact);
  TAGI_HIP(hipGetLastError());
  std::vector<float> e(np);
  for (int d = 4; d <= 12; ++d) {
    ++t->charges_gen;
    TAGI_TRY(upward(t, f, w, 1, d, s));
    A = args_of(t);
    A.ia2 = ia2;
    if (coul)
      hipLaunchKernelGGL(k_pair_approx<TAGI_COULOMB_SS>, dim3((np + 3) / 4), dim3(256), 0, s, dp,
                         np, A, kappa, exact, derr);
    else
      hipLaunchKernelGGL(k_pair_approx<TAGI_YUKAWA_SS>, dim3((np + 3) / 4), dim3(256), 0, s, dp,
                         np, A, kappa, exact, derr);
    TAGI_HIP(hipGetLastError());
    TAGI_HIP(hipMemcpyAsync(e.data(), derr, np * sizeof(float), hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < np; ++p) err[p * 9 + (d - 4)] = e[p];
  }
  (void)nl;
  return TAGI_OK;
}

}  // namespace tagi
