// Algorithm 3, proxy-charge step (Section 6.2): proxy charges of every source cluster that
// can be approximated ((n+1)^3 < N_S, Eq. MAC), by Eq.
// particle-cluster-approx-rearranged:
//
//     q^_{k1 k2 k3} = sum_{j in C} L_k1(x_j) L_k2(y_j) L_k3(z_j) q_j
//
// with Chebyshev points of the second kind s_k = c + h cos(pi k / n) mapped to the
// cluster's shrunk box (end points placed exactly on the faces) and the
// barycentric basis L_k(t) = (b_k/(t - s_k)) / sum_m b_m/(t - s_m),
// b_k = (-1)^k delta_k (Eqs. Lagrange_polynomials, barycentric_weights). A source
// that coincides with a node takes the Kronecker basis there; a zero-extent
// dimension puts all mass on node 0.
//
// Charge sets: q_j = f_j w_j for every orbital, plus q_j = w_j (orbital
// independent), which carries the singularity subtraction through the far field.
//
// Hermite charges (the Hermite treecode variant of the conclusions, Section 8):
// per dimension the interpolant matches values and first derivatives at the same
// nodes, with the basis A_k(t) = (1 - 2 c_k (t - s_k)) L_k(t)^2 for values and
// B_k(t) = (t - s_k) L_k(t)^2 for derivatives, c_k = L_k'(s_k) =
// sum_{m != k} 1/(s_k - s_m); the charge of node k and derivative pattern beta is
// q^_{k,beta} = sum_j prod_d H^{beta_d}_{k_d}(y_{j,d}) q_j (H^0 = A, H^1 = B),
// stored with the 8 patterns of one node adjacent. A source on a node has
// A_k = delta, B_k = 0; a zero-extent dimension puts all mass on A_0.
//
// GPU mapping: a work item is (cluster, range of at most kItemPts sources,
// block of charge sets). The block stages the basis values of 64 sources at a
// time in LDS. For Lagrange charges at degrees 4..12 each thread owns one
// (k1, k2) pair and every k3 for MB charge sets (k_upward_rb); otherwise each
// thread owns up to R coefficients and MB charge sets, with the charges q_j
// wave-uniform through scalar loads (k_upward). Items of one cluster write
// partial sums that a second kernel adds in a fixed order, so the result does
// not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace tagi {
namespace {

constexpr int kThreads = 256;
constexpr int kStage = 64;         // sources whose basis values sit in LDS at once
constexpr int kItemPts = 2048;     // sources per work item

struct UpItem {
  int32_t slot, p0, p1, part;  // part: index of this item's partial block
};

__global__ void k_gather(const int32_t* __restrict__ perm, const double* __restrict__ f,
                         const double* __restrict__ w, int64_t n, int n_orb,
                         double* __restrict__ fs, double* __restrict__ qs,
                         double* __restrict__ ws) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t src = perm[i];
  const double wi = w[src];
  ws[i] = wi;
  for (int o = 0; o < n_orb; ++o) {
    const double fi = f[(int64_t)o * n + src];
    fs[(int64_t)o * n + i] = fi;
    qs[(int64_t)o * n + i] = fi * wi;
  }
}

__device__ void cheb_nodes(double lo, double hi, int n, double* s) {
#pragma clang fp contract(off)
  const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
  for (int k = 0; k <= n; ++k) s[k] = c + h * cos(M_PI * k / n);
  s[0] = hi;
  s[n] = lo;
}

// Barycentric basis values of one coordinate t at the nodes s[0..degree]
// (weights b), written to L[0..degree]; HERM: Hermite value basis A_k in L[k] and
// derivative basis B_k in L[ld + k] (c = L_k'(s_k)). A coordinate on a node takes
// the Kronecker basis there (derivative part 0); a zero-extent dimension puts all
// mass on node 0; live == false writes zeros (padding rows of a stage).
template <bool HERM>
__device__ void basis_values(bool live, double t, const double* s, const double* b,
                             const double* c, int degree, int ld, double* L) {
  if (!live) {
    for (int k = 0; k <= degree; ++k) L[k] = 0.0;
    if (HERM)
      for (int k = 0; k <= degree; ++k) L[ld + k] = 0.0;
    return;
  }
  bool exact = true;  // Kronecker values, no derivative part
  if (s[0] == s[degree]) {  // zero-extent dimension
    for (int k = 0; k <= degree; ++k) L[k] = k == 0 ? 1.0 : 0.0;
  } else {
    int hit = -1;
    for (int k = 0; k <= degree; ++k)
      if (t == s[k]) hit = k;
    if (hit >= 0) {
      for (int k = 0; k <= degree; ++k) L[k] = k == hit ? 1.0 : 0.0;
    } else {
      exact = false;
      double sum = 0.0;
      for (int k = 0; k <= degree; ++k) {
        const double a = b[k] / (t - s[k]);
        L[k] = a;
        sum += a;
      }
      for (int k = 0; k <= degree; ++k) L[k] = L[k] / sum;
    }
  }
  if (HERM) {
    for (int k = 0; k <= degree; ++k) {
      if (exact) {
        L[ld + k] = 0.0;
      } else {
        const double dt = t - s[k];
        const double l2 = L[k] * L[k];
        L[ld + k] = dt * l2;
        L[k] = (1.0 - 2.0 * c[k] * dt) * l2;
      }
    }
  }
}

// R: coefficient rounds per thread (K <= R * kThreads); MB: charge sets per pass;
// HERM: Hermite charges (K = 8 (n+1)^3 coefficients, index 8 k + beta)
template <int R, int MB, bool HERM>
__global__ __launch_bounds__(kThreads) void k_upward(
    const UpItem* __restrict__ items, const int32_t* __restrict__ approx_node,
    const double* __restrict__ box, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ qs, const double* __restrict__ ws, int64_t n, int n_orb,
    int m0, int n_sets, int degree, double* __restrict__ partial,
    double* __restrict__ pnodes, float* __restrict__ pnodes32) {
  const UpItem it = items[blockIdx.x];
  constexpr int NB = HERM ? 2 : 1;  // basis families per dimension (values, derivatives)
  constexpr int kLd = kMaxDegree + 1;
  const int np1 = degree + 1;
  const int K = (HERM ? kHermPatterns : 1) * np1 * np1 * np1;
  __shared__ double s_nodes[3][kLd];
  __shared__ double s_b[kLd];
  __shared__ double s_c[3][kLd];  // Hermite: L_k'(s_k)
  __shared__ double s_L[3][kStage][NB * kLd];
  const int c = approx_node[it.slot];
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    cheb_nodes(box[c * 6 + d], box[c * 6 + 3 + d], degree, s_nodes[d]);
  }
  if (threadIdx.x <= degree) {
    double b = (threadIdx.x & 1) ? -1.0 : 1.0;
    if (threadIdx.x == 0 || threadIdx.x == degree) b *= 0.5;
    s_b[threadIdx.x] = b;
  }
  __syncthreads();
  if (HERM && threadIdx.x < 3 * np1) {
    const int d = threadIdx.x / np1, k = threadIdx.x % np1;
    const double* s = s_nodes[d];
    double ck = 0.0;
    if (s[0] != s[degree])
      for (int m = 0; m <= degree; ++m)
        if (m != k) ck += 1.0 / (s[k] - s[m]);
    s_c[d][k] = ck;
  }
  __syncthreads();
  // the first item of each cluster publishes the node coordinates
  if (m0 == 0 && it.part == it.slot && threadIdx.x < 3 * np1) {
    const int d = threadIdx.x / np1, k = threadIdx.x % np1;
    const double v = s_nodes[d][k];
    pnodes[((int64_t)it.slot * 3 + d) * np1 + k] = v;
    const double ctr = 0.5 * (box[c * 6 + d] + box[c * 6 + 3 + d]);
    pnodes32[((int64_t)it.slot * 3 + d) * np1 + k] = (float)(v - ctr);
  }
  // per coefficient: offsets of its three basis values within a staged row
  int k1[R], k2[R], k3[R];
  for (int r = 0; r < R; ++r) {
    const int k = threadIdx.x + r * kThreads;
    const int kc = k < K ? k : 0;
    const int kk = HERM ? kc / kHermPatterns : kc;
    const int beta = HERM ? kc % kHermPatterns : 0;
    k1[r] = kk / (np1 * np1) + ((beta >> 0) & 1) * kLd;
    k2[r] = (kk / np1) % np1 + ((beta >> 1) & 1) * kLd;
    k3[r] = kk % np1 + ((beta >> 2) & 1) * kLd;
  }
  double acc[R][MB];
  for (int r = 0; r < R; ++r)
    for (int m = 0; m < MB; ++m) acc[r][m] = 0.0;

  for (int p0 = it.p0; p0 < it.p1; p0 += kStage) {
    const int cnt = min(kStage, it.p1 - p0);
    if (threadIdx.x < 3 * kStage) {
      const int d = threadIdx.x / kStage, p = threadIdx.x % kStage;
      const double* cp = d == 0 ? xs : (d == 1 ? ys : zs);
      basis_values<HERM>(p < cnt, p < cnt ? cp[p0 + p] : 0.0, s_nodes[d], s_b, s_c[d], degree,
                         kLd, s_L[d][p]);
    }
    __syncthreads();
#pragma unroll 4
    for (int p = 0; p < cnt; ++p) {
      const int64_t j = p0 + p;
      double q[MB];
      for (int m = 0; m < MB; ++m) {
        const int set = m0 + m;
        q[m] = set < n_orb ? qs[(int64_t)set * n + j] : (set == n_orb ? ws[j] : 0.0);
      }
      for (int r = 0; r < R; ++r) {
        const double phi = s_L[0][p][k1[r]] * s_L[1][p][k2[r]] * s_L[2][p][k3[r]];
        for (int m = 0; m < MB; ++m) acc[r][m] = fma(phi, q[m], acc[r][m]);
      }
    }
    __syncthreads();
  }
  for (int r = 0; r < R; ++r) {
    const int k = threadIdx.x + r * kThreads;
    if (k >= K) continue;
    for (int m = 0; m < MB; ++m)
      if (m < n_sets) partial[((int64_t)blockIdx.x * MB + m) * K + k] = acc[r][m];
  }
}

// Lagrange charges with the k3 direction in registers. Thread (k1, k2, group g)
// holds acc[m][k3] for MB charge sets and every k3. Per staged source it forms
// c = L_k1(x) L_k2(y) once and c q_m once per set, then (n+1) MB multiply-adds
// with the values L_k3(z), which every thread of a group reads at one LDS address
// (a broadcast). The G = 256 / (n+1)^2 groups of a block take interleaved sources
// of each stage; at the end their sums are added in LDS in group order. Per
// source and thread: 2 + (n+1) + MB LDS reads against 1 + MB + (n+1) MB VALU
// operations (the coefficient-per-thread form above reads 3 values per 2 + MB).
template <int NP1, int MB>
__global__ __launch_bounds__(kThreads) void k_upward_rb(
    const UpItem* __restrict__ items, const int32_t* __restrict__ approx_node,
    const double* __restrict__ box, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ qs, const double* __restrict__ ws, int64_t n, int n_orb,
    int m0, int n_sets, double* __restrict__ partial, double* __restrict__ pnodes,
    float* __restrict__ pnodes32) {
  constexpr int P = NP1 * NP1;
  static_assert(P <= kThreads, "one (k1, k2) pair per thread");
  constexpr int G = kThreads / P;                  // source groups per block
  constexpr int LD = NP1 % 2 ? NP1 + 1 : NP1;      // even row stride: 16-byte aligned rows
  constexpr int K = NP1 * NP1 * NP1;
  constexpr int degree = NP1 - 1;
  constexpr int RED = (G - 1) * P * NP1 > 0 ? (G - 1) * P * NP1 : 1;
  const UpItem it = items[blockIdx.x];
  __shared__ double s_nodes[3][NP1];
  __shared__ double s_b[NP1];
  __shared__ __align__(16) double s_L[3][kStage][LD];
  __shared__ double s_q[MB][kStage];
  __shared__ double s_red[RED];
  const int c = approx_node[it.slot];
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    cheb_nodes(box[c * 6 + d], box[c * 6 + 3 + d], degree, s_nodes[d]);
  }
  if (threadIdx.x <= degree) {
    double b = (threadIdx.x & 1) ? -1.0 : 1.0;
    if (threadIdx.x == 0 || threadIdx.x == degree) b *= 0.5;
    s_b[threadIdx.x] = b;
  }
  __syncthreads();
  if (m0 == 0 && it.part == it.slot && threadIdx.x < 3 * NP1) {
    const int d = threadIdx.x / NP1, k = threadIdx.x % NP1;
    const double v = s_nodes[d][k];
    pnodes[((int64_t)it.slot * 3 + d) * NP1 + k] = v;
    const double ctr = 0.5 * (box[c * 6 + d] + box[c * 6 + 3 + d]);
    pnodes32[((int64_t)it.slot * 3 + d) * NP1 + k] = (float)(v - ctr);
  }
  const int g = threadIdx.x / P, pr = threadIdx.x % P;
  const bool active = g < G;
  const int k1 = pr / NP1, k2 = pr % NP1;
  double acc[MB][NP1];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int k = 0; k < NP1; ++k) acc[m][k] = 0.0;

  for (int p0 = it.p0; p0 < it.p1; p0 += kStage) {
    const int cnt = min(kStage, it.p1 - p0);
    if (threadIdx.x < 3 * kStage) {
      const int d = threadIdx.x / kStage, pp = threadIdx.x % kStage;
      const double* cp = d == 0 ? xs : (d == 1 ? ys : zs);
      basis_values<false>(pp < cnt, pp < cnt ? cp[p0 + pp] : 0.0, s_nodes[d], s_b, nullptr,
                          degree, 0, s_L[d][pp]);
    }
    for (int e = threadIdx.x; e < MB * kStage; e += kThreads) {
      const int m = e / kStage, pp = e % kStage;
      const int set = m0 + m;
      const int64_t j = p0 + pp;
      s_q[m][pp] = pp >= cnt ? 0.0 : (set < n_orb ? qs[(int64_t)set * n + j]
                                                   : (set == n_orb ? ws[j] : 0.0));
    }
    __syncthreads();
    if (active) {
      for (int pp = g; pp < cnt; pp += G) {
        const double cxy = s_L[0][pp][k1] * s_L[1][pp][k2];
        double cq[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) cq[m] = cxy * s_q[m][pp];
#pragma unroll
        for (int k = 0; k < NP1; ++k) {
          const double z = s_L[2][pp][k];
#pragma unroll
          for (int m = 0; m < MB; ++m) acc[m][k] = fma(cq[m], z, acc[m][k]);
        }
      }
    }
    __syncthreads();
  }
  // groups 1 .. G-1 hand their sums to group 0, one charge set at a time
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    if (G > 1) {
      if (active && g > 0)
#pragma unroll
        for (int k = 0; k < NP1; ++k) s_red[((g - 1) * P + pr) * NP1 + k] = acc[m][k];
      __syncthreads();
      if (g == 0)
        for (int gg = 1; gg < G; ++gg)
#pragma unroll
          for (int k = 0; k < NP1; ++k) acc[m][k] += s_red[((gg - 1) * P + pr) * NP1 + k];
      __syncthreads();
    }
    if (g == 0 && m < n_sets) {
      double* out = partial + ((int64_t)blockIdx.x * MB + m) * K + pr * NP1;
#pragma unroll
      for (int k = 0; k < NP1; ++k) out[k] = acc[m][k];
    }
  }
}

// charge sets per pass of k_upward_rb for n+1 = np1 (its accumulators: MB (n+1)
// doubles per thread)
constexpr int rb_sets(int np1) { return np1 <= 9 ? 8 : 4; }
constexpr bool rb_supported(int np1) { return np1 >= 5 && np1 <= 13; }

// sum the partial charges of each cluster's items in item order
__global__ void k_upward_reduce(const int32_t* __restrict__ slot_first,
                                const double* __restrict__ partial, int n_approx, int K, int MB,
                                int m0, int n_sets, int n_orb, double* __restrict__ qhat,
                                double* __restrict__ what) {
  const int slot = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_sets * K) return;
  const int m = (int)(idx / K), k = (int)(idx % K);
  double s = 0.0;
  for (int i = slot_first[slot]; i < slot_first[slot + 1]; ++i)
    s += partial[((int64_t)i * MB + m) * K + k];
  const int set = m0 + m;
  if (set < n_orb)
    qhat[((int64_t)set * n_approx + slot) * K + k] = s;
  else
    what[(int64_t)slot * K + k] = s;
}

template <int R, int MB>
void launch_upward(hipStream_t s, tagi_tree* t, ProxySet& ps, int m0, int n_sets) {
  auto kern = ps.herm ? k_upward<R, MB, true> : k_upward<R, MB, false>;
  hipLaunchKernelGGL(kern, dim3(ps.n_items), dim3(kThreads), 0, s,
                     ps.items.as<UpItem>(), ps.node.as<int32_t>(), t->nd_box.as<double>(),
                     t->xs.as<double>(), t->ys.as<double>(), t->zs.as<double>(),
                     t->qs.as<double>(), t->ws.as<double>(), t->n, ps.n_orb, m0, n_sets,
                     ps.degree, ps.partial.as<double>(), ps.pnodes.as<double>(),
                     ps.pnodes32.as<float>());
}

// charge sets per pass that R coefficient rounds leave registers for
constexpr int max_sets(int R) { return R <= 3 ? 8 : (R <= 6 ? 4 : (R <= 10 ? 2 : 1)); }

int charge_blocking(int K, int* R_out) {
  const int R = (K + kThreads - 1) / kThreads;
  *R_out = R;
  return max_sets(R);
}

// charge sets per pass for n_sets sets in all: no wider than the sets present
int charge_block(int K, int n_sets, int* R_out) {
  int mb = charge_blocking(K, R_out);
  while (mb > 1 && mb / 2 >= n_sets) mb /= 2;
  return mb;
}

template <int NP1, int MB>
void launch_upward_rb(hipStream_t s, tagi_tree* t, ProxySet& ps, int m0, int n_sets) {
  hipLaunchKernelGGL((k_upward_rb<NP1, MB>), dim3(ps.n_items), dim3(kThreads), 0, s,
                     ps.items.as<UpItem>(), ps.node.as<int32_t>(), t->nd_box.as<double>(),
                     t->xs.as<double>(), t->ys.as<double>(), t->zs.as<double>(),
                     t->qs.as<double>(), t->ws.as<double>(), t->n, ps.n_orb, m0, n_sets,
                     ps.partial.as<double>(), ps.pnodes.as<double>(), ps.pnodes32.as<float>());
}

template <int NP1>
void launch_upward_rb_mb(int MB, hipStream_t s, tagi_tree* t, ProxySet& ps, int m0, int n_sets) {
  if constexpr (rb_sets(NP1) >= 8)
    if (MB == 8) return launch_upward_rb<NP1, 8>(s, t, ps, m0, n_sets);
  if (MB == 4) return launch_upward_rb<NP1, 4>(s, t, ps, m0, n_sets);
  launch_upward_rb<NP1, 2>(s, t, ps, m0, n_sets);
}

template <int R>
void launch_upward_r(int MB, hipStream_t s, tagi_tree* t, ProxySet& ps, int m0, int n_sets) {
  if constexpr (max_sets(R) >= 8)
    if (MB == 8) return launch_upward<R, 8>(s, t, ps, m0, n_sets);
  if constexpr (max_sets(R) >= 4)
    if (MB == 4) return launch_upward<R, 4>(s, t, ps, m0, n_sets);
  if constexpr (max_sets(R) >= 2)
    if (MB == 2) return launch_upward<R, 2>(s, t, ps, m0, n_sets);
  launch_upward<R, 1>(s, t, ps, m0, n_sets);
}

}  // namespace

// Host plan of the proxy charges of `nodes` at `degree`: slots, work items and
// device buffers. Built once per (set, degree, n_orb) and reused, so a repeated
// upward pass only launches kernels (and can be captured in a HIP graph).
int prepare_proxies(tagi_tree* t, ProxySet& ps, const std::vector<int32_t>& nodes, int degree,
                    int n_orb, hipStream_t s, bool herm) {
  ps.degree = ps.n_orb = 0;
  const int np1 = degree + 1;
  const int K = (herm ? kHermPatterns : 1) * np1 * np1 * np1;
  ps.nodes = nodes;
  ps.h_slot_of.assign(t->nodes.size(), -1);
  for (size_t sl = 0; sl < nodes.size(); ++sl) ps.h_slot_of[nodes[sl]] = (int32_t)sl;
  const int na = (int)nodes.size();
  ps.n_approx = na;
  TAGI_TRY(ps.slot_of.ensure(ps.h_slot_of.size() * 4));
  TAGI_HIP(hipMemcpyAsync(ps.slot_of.p, ps.h_slot_of.data(), ps.h_slot_of.size() * 4,
                          hipMemcpyHostToDevice, s));
  std::vector<UpItem> items;
  std::vector<int32_t> slot_first(na + 1, 0);
  for (int sl = 0; sl < na; ++sl) {
    slot_first[sl] = (int32_t)items.size();
    const HostNode& q = t->nodes[nodes[sl]];
    for (int32_t p = q.begin; p < q.end; p += kItemPts)
      items.push_back({sl, p, std::min(q.end, p + kItemPts), 0});
  }
  slot_first[na] = (int32_t)items.size();
  // `part` marks the first item of each cluster (it publishes the node coordinates)
  for (int sl = 0; sl < na; ++sl)
    for (int i = slot_first[sl]; i < slot_first[sl + 1]; ++i)
      items[i].part = i == slot_first[sl] ? sl : -1;
  ps.n_items = (int)items.size();
  if (na > 0) {
    TAGI_TRY(ps.node.ensure(na * 4));
    TAGI_HIP(hipMemcpyAsync(ps.node.p, ps.nodes.data(), na * 4, hipMemcpyHostToDevice, s));
    // host staging lives in the set so the asynchronous uploads never outlive it
    ps.h_items.resize(items.size() * 4);
    std::memcpy(ps.h_items.data(), items.data(), items.size() * sizeof(UpItem));
    ps.h_slot_first = slot_first;
    TAGI_TRY(ps.items.ensure(items.size() * sizeof(UpItem) + (na + 1) * 4));
    TAGI_HIP(hipMemcpyAsync(ps.items.p, ps.h_items.data(), items.size() * sizeof(UpItem),
                            hipMemcpyHostToDevice, s));
    TAGI_HIP(hipMemcpyAsync(ps.items.as<char>() + items.size() * sizeof(UpItem),
                            ps.h_slot_first.data(), (na + 1) * 4, hipMemcpyHostToDevice, s));
    TAGI_TRY(ps.pnodes.ensure((size_t)na * 3 * np1 * sizeof(double)));
    TAGI_TRY(ps.pnodes32.ensure((size_t)na * 3 * np1 * sizeof(float)));
    TAGI_TRY(ps.qhat.ensure((size_t)n_orb * na * K * sizeof(double)));
    TAGI_TRY(ps.what.ensure((size_t)na * K * sizeof(double)));
    int R;
    const int MB = std::max(charge_blocking(K, &R), herm ? 1 : rb_sets(np1));
    TAGI_TRY(ps.partial.ensure((size_t)ps.n_items * MB * K * sizeof(double)));
  }
  ps.degree = degree;
  ps.n_orb = n_orb;
  ps.herm = herm;
  return TAGI_OK;
}

int compute_proxies(tagi_tree* t, ProxySet& ps, hipStream_t s) {
  const int na = ps.n_approx;
  if (na == 0) return TAGI_OK;
  const int np1 = ps.degree + 1;
  const int K = (ps.herm ? kHermPatterns : 1) * np1 * np1 * np1;
  const int n_sets_total = ps.n_orb + 1;
  const int32_t* d_slot_first =
      reinterpret_cast<const int32_t*>(ps.items.as<char>() + (size_t)ps.n_items * sizeof(UpItem));
  if (!ps.herm && rb_supported(np1)) {
    // k3 in registers: as many sets per pass as there are, up to rb_sets
    int MB = 2;
    while (MB < n_sets_total && MB < rb_sets(np1)) MB *= 2;
    for (int m0 = 0; m0 < n_sets_total; m0 += MB) {
      const int n_sets = std::min(MB, n_sets_total - m0);
      switch (np1) {
        case 5: launch_upward_rb_mb<5>(MB, s, t, ps, m0, n_sets); break;
        case 6: launch_upward_rb_mb<6>(MB, s, t, ps, m0, n_sets); break;
        case 7: launch_upward_rb_mb<7>(MB, s, t, ps, m0, n_sets); break;
        case 8: launch_upward_rb_mb<8>(MB, s, t, ps, m0, n_sets); break;
        case 9: launch_upward_rb_mb<9>(MB, s, t, ps, m0, n_sets); break;
        case 10: launch_upward_rb_mb<10>(MB, s, t, ps, m0, n_sets); break;
        case 11: launch_upward_rb_mb<11>(MB, s, t, ps, m0, n_sets); break;
        case 12: launch_upward_rb_mb<12>(MB, s, t, ps, m0, n_sets); break;
        default: launch_upward_rb_mb<13>(MB, s, t, ps, m0, n_sets); break;
      }
      TAGI_HIP(hipGetLastError());
      const int64_t tot = (int64_t)n_sets * K;
      hipLaunchKernelGGL(k_upward_reduce, dim3((tot + 255) / 256, na), dim3(256), 0, s,
                         d_slot_first, ps.partial.as<double>(), na, K, MB, m0, n_sets, ps.n_orb,
                         ps.qhat.as<double>(), ps.what.as<double>());
      TAGI_HIP(hipGetLastError());
    }
    return TAGI_OK;
  }
  int R;
  const int MB = charge_block(K, n_sets_total, &R);
  for (int m0 = 0; m0 < n_sets_total; m0 += MB) {
    const int n_sets = std::min(MB, n_sets_total - m0);
    switch (R) {
      case 1: launch_upward_r<1>(MB, s, t, ps, m0, n_sets); break;
      case 2: launch_upward_r<2>(MB, s, t, ps, m0, n_sets); break;
      case 3: launch_upward_r<3>(MB, s, t, ps, m0, n_sets); break;
      case 4: launch_upward_r<4>(MB, s, t, ps, m0, n_sets); break;
      case 5: launch_upward_r<5>(MB, s, t, ps, m0, n_sets); break;
      case 6: launch_upward_r<6>(MB, s, t, ps, m0, n_sets); break;
      case 7: launch_upward_r<7>(MB, s, t, ps, m0, n_sets); break;
      case 8: launch_upward_r<8>(MB, s, t, ps, m0, n_sets); break;
      case 9: launch_upward_r<9>(MB, s, t, ps, m0, n_sets); break;
      case 10: launch_upward_r<10>(MB, s, t, ps, m0, n_sets); break;
      case 11: case 12: launch_upward_r<12>(MB, s, t, ps, m0, n_sets); break;
      case 13: case 14: launch_upward_r<14>(MB, s, t, ps, m0, n_sets); break;
      case 15: case 16: launch_upward_r<16>(MB, s, t, ps, m0, n_sets); break;
      default: launch_upward_r<20>(MB, s, t, ps, m0, n_sets); break;
    }
    TAGI_HIP(hipGetLastError());
    const int64_t tot = (int64_t)n_sets * K;
    hipLaunchKernelGGL(k_upward_reduce, dim3((tot + 255) / 256, na), dim3(256), 0, s,
                       d_slot_first, ps.partial.as<double>(), na, K, MB, m0, n_sets, ps.n_orb,
                       ps.qhat.as<double>(), ps.what.as<double>());
    TAGI_HIP(hipGetLastError());
  }
  return TAGI_OK;
}

int upward(tagi_tree* t, const double* f, const double* w, int n_orb, int degree,
           hipStream_t s, bool herm) {
  const int64_t n = t->n;
  t->degree = 0;  // invalid until complete
  phase_begin(t, kPhaseUpward, s);
  if (!(t->px.degree == degree && t->px.n_orb == n_orb && t->px.herm == herm)) {
    t->px.degree = t->px.n_orb = 0;  // invalid until the plan is complete
    TAGI_TRY(t->ws.ensure(n * sizeof(double)));
    TAGI_TRY(t->fs.ensure((size_t)n_orb * n * sizeof(double)));
    TAGI_TRY(t->qs.ensure((size_t)n_orb * n * sizeof(double)));
    // approximable clusters: more sources than charges ((n+1)^3, Hermite 8 (n+1)^3);
    // the root is skipped because every batch centre lies inside it, so the
    // distance test can never accept it
    const int K = (herm ? kHermPatterns : 1) * (degree + 1) * (degree + 1) * (degree + 1);
    std::vector<int32_t> nodes;
    for (size_t c = 1; c < t->nodes.size(); ++c)
      if (t->nodes[c].end - t->nodes[c].begin > K) nodes.push_back((int32_t)c);
    TAGI_TRY(prepare_proxies(t, t->px, nodes, degree, n_orb, s, herm));
  }
  hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, s, t->perm.as<int32_t>(), f,
                     w, n, n_orb, t->fs.as<double>(), t->qs.as<double>(), t->ws.as<double>());
  TAGI_HIP(hipGetLastError());
  TAGI_TRY(compute_proxies(t, t->px, s));
  t->n_orb = n_orb;
  t->degree = degree;
  phase_end(t, kPhaseUpward, s);
  return TAGI_OK;
}

}  // namespace tagi
