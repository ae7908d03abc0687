// Learned degree/MAC selection (a project addition on Algorithm 3): the
// interaction lists are built by the same per-batch ComputePotential traversal,
// but for a pair that passes a permissive geometric test (r_B + r_C) < theta_max R
// the selector network predicts the approximation error at every degree 4..12
// from (r_C, R - r_B, c, N_S, l1 bound of the cluster's subtracted degree-4
// proxy charges), one orbital at a time, as a residual over the scale
// l1 exp(-c (R - r_B)) / (R - r_B) of the pair's far field; c is the kernel's
// decay rate (kappa for Yukawa, 0 for Coulomb, the kappa -> 0 limit), which enters
// the network as ln(c + 0.25). The pair is approximated at the lowest degree
// whose predicted error meets the pair budget for every orbital (and whose
// (n+1)^3 is below N_S); if no degree does, the cluster is opened (a leaf is
// summed directly). The pair budget of batch B is the caller's per-target budget
// divided by M_B, M_B = the far pairs of B in the fixed-MAC lists at
// (theta_max, degree 4): a target's far-field error is at most the sum of its
// pairs' errors, whatever their signs. Where any feature lies outside
// the range the network was trained on, the pair falls back to the fixed MAC
// (theta_fb, degree_fb).
//
// Far entries are written grouped by degree within each batch; every degree in
// use gets its own proxy set (only the clusters used at that degree), and the
// far field is launched once per degree with the degree's compiled kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "interact_impl.hpp"
#include "internal.hpp"

namespace tagi {
namespace ik {
extern template void launch_interact_ob<TAGI_YUKAWA_SS>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_ob<TAGI_YUKAWA>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_ob<TAGI_COULOMB_SS>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_ob<TAGI_COULOMB>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
}  // namespace ik

namespace {
using namespace ik;

constexpr int kDegMin = kLearnDegMin, kDegMax = kLearnDegMax, kNDeg = kDegMax - kDegMin + 1;
constexpr int kSlots = kNDeg + 1;  // per batch: far entries per degree, then near entries
constexpr int kH = 64, kIn = 5, kOut = 9;
constexpr int kNParam = (kIn * kH + kH) + 2 * (kH * kH + kH) + (kH * kOut + kOut);
// added to the decay rate before its logarithm (c = 0 for the Coulomb kernels)
constexpr float kDecayOffset = 0.25f;

struct LearnArgs {
  int n_leaves, n_nodes, n_orb;
  const int32_t *leaf_node, *nbeg, *nend, *first_child, *n_child;
  const double* geom;
  const float* l1n;        // [n_orb][n_nodes] l1 norm of the degree-4 charges of f w
  const float* l1w;        // [n_nodes] l1 norm of the degree-4 charges of w
  const float* fmax;       // [n_orb][n_leaves] max |f| over each batch
  const int64_t* mb;       // [n_leaves] far pairs of each batch at (theta_max, degree 4)
  int sub_kind;            // subtracted charges in the l1 feature: 0 none, 1 Yukawa, 2 Gaussian
  float ia2;               // 1 / alpha^2 of the Gaussian
  const float* params;
  double theta_max, theta_fb;
  int degree_fb;
  float log_tol[kMaxOrb];  // per orbital: log10 of the per-target error budget
  float shift[kIn], scale[kIn], lo[kIn], hi[kIn];
  float logc[kMaxOrb];     // per orbital: ln(decay rate + kDecayOffset)
  float kap[kMaxOrb];      // per orbital: decay rate (kappa, or 0 for Coulomb)
  int64_t* cnt;        // [n_leaves][kSlots] entries per slot
  int64_t* nlog;       // [n_leaves] entries visited (may exceed cap)
  int32_t* log;        // [n_leaves][cap] (C << 4) | slot in traversal order
  int64_t cap;
  int32_t* overflow;   // traversal stack overflow
};

// Offsets of the layers in the parameter vector: W0 [64][5], b0 [64], W1 [64][64],
// b1 [64], W2 [64][64], b2 [64], W3 [9][64], b3 [9] (row-major, out x in).
constexpr int kOffW0 = 0, kOffB0 = kOffW0 + kH * kIn, kOffW1 = kOffB0 + kH;
constexpr int kOffB1 = kOffW1 + kH * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kOut * kH;
constexpr int kW3Stride = kH + 1;  // LDS row stride of W3: the 9 rows fall in distinct banks

// The network for one orbital with the wave's 64 lanes as the 64 hidden units:
// lane j holds row j of W0, W1 and W2 in registers (w0, w1, w2, and the biases
// bj), each layer's input is read from LDS as a broadcast, and each unit's sum
// runs over its inputs in order, so every output has the bits of the plain
// per-unit loop. x: the orbital's normalised features (LDS); hx: three [64] LDS
// buffers; w3: W3 in LDS with row stride kW3Stride; b3: the output biases;
// out: the 9 outputs, written to LDS by lanes 0..8.
__device__ void mlp_units(const float* w0, const float* w1, const float* w2, const float* bj,
                          const float* x, float* hx, const float* w3, const float* b3, int lane,
                          float* out) {
  float s = bj[0];
#pragma unroll
  for (int i = 0; i < kIn; ++i) s = __builtin_fmaf(w0[i], x[i], s);
  hx[lane] = tanhf(s);
  __syncthreads();
  s = bj[1];
#pragma unroll
  for (int i = 0; i < kH; ++i) s = __builtin_fmaf(w1[i], hx[i], s);
  hx[kH + lane] = tanhf(s);
  __syncthreads();
  s = bj[2];
#pragma unroll
  for (int i = 0; i < kH; ++i) s = __builtin_fmaf(w2[i], hx[kH + i], s);
  hx[2 * kH + lane] = tanhf(s);
  __syncthreads();
  if (lane < kOut) {
    s = b3[lane];
    for (int i = 0; i < kH; ++i) s = __builtin_fmaf(w3[lane * kW3Stride + i], hx[2 * kH + i], s);
    out[lane] = s;
  }
  __syncthreads();
}

constexpr int kStack = 512;  // traversal stack entries

// One wave per batch: the ComputePotential traversal is wave-uniform; at a
// candidate pair lane o forms the features of orbital o, then the wave evaluates
// the network for each orbital in turn (lanes = hidden units), and lane o picks
// its orbital's degree. Every visited pair's outcome goes to the batch's log in
// traversal order as (C << 4) | slot (slot 0..8: far at degree 4 + slot, 9:
// near); entries beyond `cap` are counted but not written.
__global__ __launch_bounds__(64) void k_lists_learned(LearnArgs L) {
  __shared__ float sW3[kOut * kW3Stride + kOut];
  __shared__ float sx[kMaxOrb * kIn];      // normalised features per orbital
  __shared__ float spred[kMaxOrb * kOut];  // network outputs per orbital
  __shared__ float hx[3 * kH];             // layer outputs (broadcast buffers)
  __shared__ int stk[kStack];
  const int lane = threadIdx.x;
  for (int i = lane; i < kOut * kH; i += blockDim.x)
    sW3[(i / kH) * kW3Stride + i % kH] = L.params[kOffW3 + i];
  if (lane < kOut) sW3[kOut * kW3Stride + lane] = L.params[kOffB3 + lane];
  // this lane's hidden unit: its rows of W0, W1, W2 and its biases
  float w0[kIn], w1[kH], w2[kH], bj[3];
#pragma unroll
  for (int i = 0; i < kIn; ++i) w0[i] = L.params[kOffW0 + lane * kIn + i];
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    w1[i] = L.params[kOffW1 + lane * kH + i];
    w2[i] = L.params[kOffW2 + lane * kH + i];
  }
  bj[0] = L.params[kOffB0 + lane];
  bj[1] = L.params[kOffB1 + lane];
  bj[2] = L.params[kOffB2 + lane];
  const int b = blockIdx.x;
  const int B = L.leaf_node[b];
  const double rB = L.geom[B * 4 + 3];
  // this lane's orbital's pair budget: log10(tol_o / M_B)
  const float pair_log_tol = lane < L.n_orb
                                 ? L.log_tol[lane] - log10f((float)max(L.mb[b], (int64_t)1))
                                 : 0.0f;
  int32_t* blog = L.log + (int64_t)b * L.cap;
  int64_t c[kSlots];
  for (int k = 0; k < kSlots; ++k) c[k] = 0;
  int64_t nlog = 0;
  if (lane == 0) stk[0] = 0;
  int sp = 1;
  bool over = false;
  while (sp > 0) {
    __syncthreads();
    const int C = stk[--sp];
    const int cnt = L.nend[C] - L.nbeg[C];
    const bool leaf = L.n_child[C] == 0;
    double R, rC;
    {
#pragma clang fp contract(off)
      const double dx = L.geom[B * 4 + 0] - L.geom[C * 4 + 0];
      const double dy = L.geom[B * 4 + 1] - L.geom[C * 4 + 1];
      const double dz = L.geom[B * 4 + 2] - L.geom[C * 4 + 2];
      R = sqrt(dx * dx + dy * dy + dz * dz);
      rC = L.geom[C * 4 + 3];
    }
    int kind;  // 0 far (at degree deg), 1 near, 2 open
    int deg = 0;
    if (!((rB + rC) < L.theta_max * R)) {
      kind = leaf ? 1 : 2;
    } else if (cnt <= (kDegMin + 1) * (kDegMin + 1) * (kDegMin + 1)) {
      kind = 1;  // too few sources for any degree: direct, as a size-rejected pair
    } else {
      bool fb = false;
      int d_o = 0;  // this lane's orbital: lowest acceptable degree, -1 if none
      float l1_o = 1.0f;
      // weight of the subtracted charges: 1 (Yukawa-SS), the Gaussian at the
      // least batch-cluster distance (Coulomb-SS), 0 (plain kernels)
      float gsub = L.sub_kind == 1 ? 1.0f : 0.0f;
      if (L.sub_kind == 2) {
        const float dm = (float)fmax(R - rB - rC, 0.0);
        gsub = expf(-dm * dm * L.ia2);
      }
      if (lane < L.n_orb) {
        const int o = lane;
        float raw[kIn];
        raw[0] = logf((float)rC);
        raw[1] = logf((float)fmax(R - rB, 1e-12));
        raw[2] = L.logc[o];
        raw[3] = logf((float)cnt);
        // size of the charges q^ - f_i w^ the pair's far field carries, the
        // subtracted ones weighted by their kernel relative to the first one's
        const float l1 = fmaxf(L.l1n[(int64_t)o * L.n_nodes + C] +
                                   gsub * L.fmax[(int64_t)o * L.n_leaves + b] * L.l1w[C],
                               1e-30f);
        raw[4] = logf(l1);
        for (int k = 0; k < kIn; ++k) {
          if (!(raw[k] >= L.lo[k] && raw[k] <= L.hi[k])) fb = true;
          sx[o * kIn + k] = (raw[k] - L.shift[k]) * L.scale[k];
        }
        l1_o = l1;
      }
      const bool fallback = __builtin_amdgcn_ballot_w64(fb) != 0;
      if (!fallback) {
        __syncthreads();  // the features are in LDS
        for (int o = 0; o < L.n_orb; ++o)
          mlp_units(w0, w1, w2, bj, sx + o * kIn, hx, sW3, sW3 + kOut * kW3Stride, lane,
                    spred + o * kOut);
        if (lane < L.n_orb) {
          const int o = lane;
          // the network predicts the error relative to the magnitude scale
          // l1 exp(-c d) / d of the pair, d = R - r_B
          const float dd = (float)fmax(R - rB, 1e-12);
          const float scl = log10f(l1_o) - 0.43429448f * L.kap[o] * dd - log10f(dd);
          d_o = -1;
          for (int d = kDegMin; d <= kDegMax; ++d) {
            if ((d + 1) * (d + 1) * (d + 1) >= cnt) break;
            if (spred[o * kOut + d - kDegMin] + scl <= pair_log_tol) {
              d_o = d;
              break;
            }
          }
        }
      }
      const bool ok = __builtin_amdgcn_ballot_w64(d_o < 0) == 0;
      int dmax = d_o;
      for (int off = kWave / 2; off > 0; off >>= 1) dmax = max(dmax, __shfl_xor(dmax, off));
      if (fallback) {
        const int nf = L.degree_fb + 1;
        const bool dist = (rB + rC) < L.theta_fb * R;
        if (dist && nf * nf * nf < cnt) {
          kind = 0;
          deg = L.degree_fb;
        } else if (!dist) {
          kind = leaf ? 1 : 2;
        } else {
          kind = 1;
        }
      } else if (ok) {
        kind = 0;
        deg = max(dmax, kDegMin);
      } else {
        kind = leaf ? 1 : 2;
      }
    }
    kind = __builtin_amdgcn_readfirstlane(kind);
    deg = __builtin_amdgcn_readfirstlane(deg);
    if (kind == 2) {
      const int fc = L.first_child[C], nc = L.n_child[C];
      if (sp + nc > kStack) {
        over = true;
        break;
      }
      __syncthreads();  // every lane has read stk[sp] before it is overwritten
      if (lane < nc) stk[sp + nc - 1 - lane] = fc + lane;
      sp += nc;
    } else {
      const int slot = kind == 0 ? deg - kDegMin : kNDeg;
      if (lane == 0 && nlog < L.cap) blog[nlog] = (C << 4) | slot;
      ++nlog;
      ++c[slot];
    }
  }
  if (lane == 0) {
    for (int k = 0; k < kSlots; ++k) L.cnt[(int64_t)b * kSlots + k] = c[k];
    L.nlog[b] = nlog;
    if (over) atomicExch(L.overflow, 1);
  }
}

// Scatters each batch's log into the far list (grouped by degree, traversal
// order within a degree) and the near list, at the host-computed offsets.
__global__ void k_lists_scatter(int n_leaves, int64_t cap, const int32_t* __restrict__ log,
                                const int64_t* __restrict__ nlog, const int64_t* __restrict__ off,
                                int32_t* __restrict__ far_id, int32_t* __restrict__ near_id) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_leaves) return;
  int64_t pos[kSlots];
  for (int k = 0; k < kSlots; ++k) pos[k] = off[(int64_t)b * kSlots + k];
  const int32_t* lg = log + (int64_t)b * cap;
  for (int64_t i = 0; i < nlog[b]; ++i) {
    const int32_t e = lg[i];
    const int slot = e & 15, C = e >> 4;
    if (slot < kNDeg) far_id[pos[slot]++] = C;
    else near_id[pos[kNDeg]++] = C;
  }
}

}  // namespace

int convolve_learned(tagi_tree* t, int kernel, const double* kappa, double alpha,
                     const float* params, const float* norm, const double* tol, double theta_max,
                     double theta_fb, int degree_fb, int precision, double* out, hipStream_t s) {
  LearnedState& S = t->learned;
  const int n_orb = t->n_orb;
  const int nl = (int)t->leaves.size();
  const int nn = (int)t->nodes.size();
  // cache key: everything the lists depend on
  std::vector<double> key = {(double)n_orb, theta_max, theta_fb, (double)degree_fb,
                             (double)kernel, kernel == TAGI_COULOMB_SS ? alpha : 0.0,
                             (double)schedule_items(t)};
  const bool yuk_kernel = kernel == TAGI_YUKAWA_SS || kernel == TAGI_YUKAWA;
  for (int o = 0; o < n_orb; ++o) key.push_back(yuk_kernel ? kappa[o] : 0.0);
  for (int o = 0; o < n_orb; ++o) key.push_back(tol[o]);
  for (int k = 0; k < 4 * kIn; ++k) key.push_back(norm[k]);
  for (int k = 0; k < kNParam; ++k) key.push_back(params[k]);
  const int ob = orbital_block_of(t, kernel, precision, true);
  if (key != S.key) {
    phase_begin(t, kPhaseLists, s);
    S.key.clear();
    // features: l1 norms of the degree-4 charges of every cluster that could be approximated
    std::vector<int32_t> cand;
    const int K4 = (kDegMin + 1) * (kDegMin + 1) * (kDegMin + 1);
    for (int c = 1; c < nn; ++c)
      if (t->nodes[c].end - t->nodes[c].begin > K4) cand.push_back(c);
    TAGI_TRY(prepare_proxies(t, S.l1set, cand, kDegMin, n_orb, s));
    TAGI_TRY(compute_proxies(t, S.l1set, s));
    // per node: l1 of each orbital's charges, then of w's; per batch: max |f|
    TAGI_TRY(S.l1n.ensure((size_t)((n_orb + 1) * nn + n_orb * nl) * sizeof(float)));
    TAGI_HIP(hipMemsetAsync(S.l1n.p, 0, (size_t)((n_orb + 1) * nn + n_orb * nl) * sizeof(float), s));
    float* d_l1w = S.l1n.as<float>() + (size_t)n_orb * nn;
    float* d_fmax = d_l1w + nn;
    for (int o = 0; o <= n_orb; ++o)
      TAGI_TRY(l1_to_nodes(S.l1set, o, S.l1n.as<float>() + (size_t)o * nn, s));
    TAGI_TRY(leaf_fmax(t, d_fmax, s));
    TAGI_TRY(S.params.ensure(kNParam * sizeof(float)));
    TAGI_HIP(hipMemcpyAsync(S.params.p, params, kNParam * sizeof(float), hipMemcpyHostToDevice, s));
    // M_B: far pairs per batch of the fixed-MAC lists at (theta_max, degree 4)
    TAGI_TRY(S.mb.ensure((size_t)nl * 3 * sizeof(int64_t) + sizeof(int32_t)));
    TAGI_TRY(count_far_pairs(t, theta_max, (kDegMin + 1) * (kDegMin + 1) * (kDegMin + 1),
                             S.mb.as<int64_t>(), S.mb.as<int64_t>() + nl, s));
    // lists: count, offsets, fill
    LearnArgs L{};
    L.n_leaves = nl;
    L.n_nodes = nn;
    L.n_orb = n_orb;
    L.leaf_node = t->leaf_node.as<int32_t>();
    L.nbeg = t->nd_begin.as<int32_t>();
    L.nend = t->nd_end.as<int32_t>();
    L.first_child = t->nd_first_child.as<int32_t>();
    L.n_child = t->nd_n_child.as<int32_t>();
    L.geom = t->nd_geom.as<double>();
    L.l1n = S.l1n.as<float>();
    L.l1w = d_l1w;
    L.fmax = d_fmax;
    L.mb = S.mb.as<int64_t>();
    L.sub_kind = kernel == TAGI_YUKAWA_SS ? 1 : (kernel == TAGI_COULOMB_SS ? 2 : 0);
    L.ia2 = kernel == TAGI_COULOMB_SS ? (float)(1.0 / (alpha * alpha)) : 0.0f;
    L.params = S.params.as<float>();
    L.theta_max = theta_max;
    L.theta_fb = theta_fb;
    L.degree_fb = degree_fb;
    for (int o = 0; o < n_orb; ++o) L.log_tol[o] = (float)std::log10(tol[o]);
    for (int k = 0; k < kIn; ++k) {
      L.shift[k] = norm[k];
      L.scale[k] = norm[kIn + k];
      L.lo[k] = norm[2 * kIn + k];
      L.hi[k] = norm[3 * kIn + k];
    }
    const bool yuk = kernel == TAGI_YUKAWA_SS || kernel == TAGI_YUKAWA;
    for (int o = 0; o < n_orb; ++o) {
      const double c = yuk ? kappa[o] : 0.0;  // decay rate
      L.logc[o] = (float)std::log(c + (double)kDecayOffset);
      L.kap[o] = (float)c;
    }
    // one wave per batch; the per-batch logs are scattered into grouped lists
    TAGI_TRY(S.cnt.ensure((size_t)nl * (2 * kSlots + 1) * sizeof(int64_t) + 4));
    int64_t* d_cnt = S.cnt.as<int64_t>();
    int64_t* d_off = d_cnt + (size_t)nl * kSlots;
    int64_t* d_nlog = d_off + (size_t)nl * kSlots;
    int32_t* d_over = reinterpret_cast<int32_t*>(d_nlog + nl);
    L.cnt = d_cnt;
    L.nlog = d_nlog;
    L.overflow = d_over;
    std::vector<int64_t> h((size_t)nl * kSlots), hlog(nl);
    int64_t cap = std::max<int64_t>(S.log_cap, 2048);
    for (int attempt = 0; attempt < 2; ++attempt) {
      TAGI_TRY(S.log.ensure((size_t)nl * cap * sizeof(int32_t)));
      TAGI_HIP(hipMemsetAsync(d_over, 0, 4, s));
      L.log = S.log.as<int32_t>();
      L.cap = cap;
      hipLaunchKernelGGL(k_lists_learned, dim3(nl), dim3(64), 0, s, L);
      TAGI_HIP(hipGetLastError());
      int32_t over = 0;
      TAGI_HIP(hipMemcpyAsync(h.data(), d_cnt, h.size() * 8, hipMemcpyDeviceToHost, s));
      TAGI_HIP(hipMemcpyAsync(hlog.data(), d_nlog, hlog.size() * 8, hipMemcpyDeviceToHost, s));
      TAGI_HIP(hipMemcpyAsync(&over, d_over, 4, hipMemcpyDeviceToHost, s));
      TAGI_HIP(hipStreamSynchronize(s));
      if (over) {
        set_error("learned lists: traversal stack overflow");
        return TAGI_E_UNSUPPORTED;
      }
      const int64_t need = *std::max_element(hlog.begin(), hlog.end());
      if (need <= cap) break;
      if (attempt == 1 || need >= INT32_MAX / 16) {
        set_error("learned lists: per-batch log of %lld entries", (long long)need);
        return TAGI_E_UNSUPPORTED;
      }
      cap = need;  // a second traversal with room for every batch
    }
    S.log_cap = cap;
    std::vector<int64_t> off(h.size());
    int64_t nf = 0, nnear = 0;
    for (int b = 0; b < nl; ++b) {
      for (int k = 0; k < kNDeg; ++k) {
        off[(size_t)b * kSlots + k] = nf;
        nf += h[(size_t)b * kSlots + k];
      }
      off[(size_t)b * kSlots + kNDeg] = nnear;
      nnear += h[(size_t)b * kSlots + kNDeg];
    }
    if (nf >= INT32_MAX || nnear >= INT32_MAX) {
      set_error("learned lists exceed 2^31 entries");
      return TAGI_E_UNSUPPORTED;
    }
    S.n_far = nf;
    S.n_near = nnear;
    TAGI_TRY(S.far_id.ensure(std::max<int64_t>(nf, 1) * 4));
    TAGI_TRY(S.near_id.ensure(std::max<int64_t>(nnear, 1) * 4));
    TAGI_HIP(hipMemcpyAsync(d_off, off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_lists_scatter, dim3((nl + 127) / 128), dim3(128), 0, s, nl, cap,
                       S.log.as<int32_t>(), d_nlog, d_off, S.far_id.as<int32_t>(),
                       S.near_id.as<int32_t>());
    TAGI_HIP(hipGetLastError());
    std::vector<int32_t>& fid = S.h_fid;
    std::vector<int32_t>& nid = S.h_nid;
    fid.assign(std::max<int64_t>(nf, 1), 0);
    nid.assign(std::max<int64_t>(nnear, 1), 0);
    S.h_cnt = h;
    if (nf) TAGI_HIP(hipMemcpyAsync(fid.data(), S.far_id.p, nf * 4, hipMemcpyDeviceToHost, s));
    if (nnear) TAGI_HIP(hipMemcpyAsync(nid.data(), S.near_id.p, nnear * 4, hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipStreamSynchronize(s));
    // proxy sets per degree: the clusters used at that degree
    for (int d = 0; d <= kMaxDegree; ++d) S.far_by_degree[d] = 0;
    S.far_inter = S.near_inter = 0;
    for (int k = 0; k < kNDeg; ++k) {
      const int d = kDegMin + k;
      std::vector<char> used(nn, 0);
      for (int b = 0; b < nl; ++b) {
        const int64_t e0 = off[(size_t)b * kSlots + k], e1 = e0 + h[(size_t)b * kSlots + k];
        const HostNode& q = t->nodes[t->leaves[b]];
        S.far_by_degree[d] += e1 - e0;
        S.far_inter += (int64_t)(q.end - q.begin) * (e1 - e0) * (d + 1) * (d + 1) * (d + 1);
        for (int64_t e = e0; e < e1; ++e) used[fid[e]] = 1;
      }
      std::vector<int32_t> nodes;
      for (int c = 0; c < nn; ++c)
        if (used[c]) nodes.push_back(c);
      if (nodes.empty()) {
        t->lx[d].release();
      } else {
        TAGI_TRY(prepare_proxies(t, t->lx[d], nodes, d, n_orb, s));
      }
    }
    // chunks (host): far segments per degree, then the near list, each cut by cost
    // (kernel evaluations per target lane), at most 1/schedule_items of the whole
    S.h_chunks.clear();
    std::vector<int32_t> bfirst(nl), bcount(nl);
    int64_t lane_cost = 0;
    for (int b = 0; b < nl; ++b) {
      const HostNode& q = t->nodes[t->leaves[b]];
      const int64_t nb = q.end - q.begin;
      for (int k = 0; k < kNDeg; ++k)
        lane_cost += h[(size_t)b * kSlots + k] * (kDegMin + k + 1) * (kDegMin + k + 1) * (kDegMin + k + 1);
      for (int64_t e = off[(size_t)b * kSlots + kNDeg]; e < off[(size_t)b * kSlots + kNDeg] + h[(size_t)b * kSlots + kNDeg]; ++e) {
        const int64_t ns = t->nodes[nid[e]].end - t->nodes[nid[e]].begin;
        S.near_inter += nb * ns;
        lane_cost += ns;
      }
    }
    const int64_t ccap = std::max<int64_t>(lane_cost / schedule_items(t), 4096);
    for (int b = 0; b < nl; ++b) {
      bfirst[b] = (int32_t)(S.h_chunks.size() / 4);
      for (int k = 0; k <= kNDeg; ++k) {
        const int64_t e0 = off[(size_t)b * kSlots + k], e1 = e0 + h[(size_t)b * kSlots + k];
        const int kindv = k < kNDeg ? 16 + kDegMin + k : 1;
        int64_t start = e0, cost = 0;
        for (int64_t e = e0; e < e1; ++e) {
          const int64_t cst = k < kNDeg ? (int64_t)(kDegMin + k + 1) * (kDegMin + k + 1) * (kDegMin + k + 1)
                                        : (int64_t)(t->nodes[nid[e]].end - t->nodes[nid[e]].begin);
          if (cost > 0 && cost + cst > ccap) {
            S.h_chunks.insert(S.h_chunks.end(), {kindv, (int32_t)start, (int32_t)e, (int32_t)std::min<int64_t>(cost, INT32_MAX)});
            start = e;
            cost = 0;
          }
          cost += cst;
        }
        if (e1 > start)
          S.h_chunks.insert(S.h_chunks.end(), {kindv, (int32_t)start, (int32_t)e1, (int32_t)std::min<int64_t>(cost, INT32_MAX)});
      }
      bcount[b] = (int32_t)(S.h_chunks.size() / 4) - bfirst[b];
    }
    S.h_batch_chunks.assign(2 * (size_t)nl, 0);
    for (int b = 0; b < nl; ++b) {
      S.h_batch_chunks[2 * b] = bfirst[b];
      S.h_batch_chunks[2 * b + 1] = bcount[b];
    }
    auto up = [&](DBuf& buf, const std::vector<int32_t>& v) -> int {
      TAGI_TRY(buf.ensure(std::max<size_t>(v.size(), 1) * 4));
      if (!v.empty()) TAGI_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
      return TAGI_OK;
    };
    TAGI_TRY(up(S.chunks, S.h_chunks));
    TAGI_TRY(up(S.batch_chunks, S.h_batch_chunks));
    TAGI_HIP(hipStreamSynchronize(s));
    S.key = key;
    S.ob = 0;  // the items below depend on the orbital block
    phase_end(t, kPhaseLists, s);
  }
  if (S.ob != ob) {
    // items (batch, group, orbital block, chunk); launch lists per degree and near
    S.ob = 0;  // invalid until every buffer below is in place
    const int n_ob = (n_orb + ob - 1) / ob;
    S.h_items.clear();
    S.h_group_first.clear();
    S.h_group_base.assign(nl, 0);
    std::vector<std::vector<int32_t>> per(kNDeg + 1);
    std::vector<std::vector<WaveRun>> per_runs(kNDeg + 1);
    for (int b = 0; b < nl; ++b) {
      const HostNode& q = t->nodes[t->leaves[b]];
      const int ng = (q.end - q.begin + kWave - 1) / kWave;
      const int32_t* bch = S.h_batch_chunks.data();  // {first chunk, n chunks} per batch
      S.h_group_base[b] = (int32_t)S.h_group_first.size();
      const int bf = bch[2 * b], bc = bch[2 * b + 1];
      for (int g = 0; g < ng; ++g) {
        S.h_group_first.push_back((int32_t)(S.h_items.size() / 4));
        for (int o = 0; o < n_ob; ++o)
          for (int cidx = 0; cidx < bc; ++cidx)
            S.h_items.insert(S.h_items.end(), {b, g, o, bf + cidx});
      }
      // launch order within the batch: chunk-major, the target groups that read
      // the same sources side by side
      for (int o = 0; o < n_ob; ++o)
        for (int cidx = 0; cidx < bc; ++cidx) {
          const int kindv = S.h_chunks[(size_t)(bf + cidx) * 4];
          const int slot = kindv == 1 ? kNDeg : kindv - 16 - kDegMin;
          per_runs[slot].push_back({(int32_t)per[slot].size(), ng,
                                    (double)S.h_chunks[(size_t)(bf + cidx) * 4 + 3]});
          for (int g = 0; g < ng; ++g)
            per[slot].push_back(S.h_group_first[S.h_group_base[b] + g] + o * bc + cidx);
        }
    }
    S.n_items = (int64_t)S.h_items.size() / 4;
    S.h_lists.clear();
    S.list_begin.clear();
    S.list_degree.clear();
    for (int k = 0; k <= kNDeg; ++k) {
      if (per[k].empty()) continue;
      // one launch per list: its chunks are all of one kind, so their costs
      // compare directly
      TAGI_TRY(balance_runs_per_xcd(per[k], per_runs[k], true));
      S.list_begin.push_back((int64_t)S.h_lists.size());
      S.list_degree.push_back(k < kNDeg ? kDegMin + k : 0);
      S.h_lists.insert(S.h_lists.end(), per[k].begin(), per[k].end());
    }
    S.list_begin.push_back((int64_t)S.h_lists.size());
    auto up = [&](DBuf& buf, const std::vector<int32_t>& v) -> int {
      TAGI_TRY(buf.ensure(std::max<size_t>(v.size(), 1) * 4));
      if (!v.empty()) TAGI_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
      return TAGI_OK;
    };
    TAGI_TRY(up(S.items, S.h_items));
    TAGI_TRY(up(S.group_first, S.h_group_first));
    TAGI_TRY(up(S.group_base, S.h_group_base));
    TAGI_TRY(up(S.item_lists, S.h_lists));
    TAGI_TRY(S.partial.ensure(std::max<int64_t>(S.n_items, 1) * ob * 2 * kWave * sizeof(double)));
    TAGI_HIP(hipStreamSynchronize(s));
    S.ob = ob;
  }
  const bool mix = precision == TAGI_MIXED;
  if (mix) {  // FP32 copies of the proxy charges (allocation before the fork)
    for (size_t li = 0; li + 1 < S.list_begin.size(); ++li) {
      const int d = S.list_degree[li];
      if (d == 0) continue;
      ProxySet& ps = t->lx[d];
      const int64_t K = (int64_t)(d + 1) * (d + 1) * (d + 1);
      TAGI_TRY(ps.qhat32.ensure((size_t)n_orb * ps.n_approx * K * sizeof(float)));
      TAGI_TRY(ps.what32.ensure((size_t)ps.n_approx * K * sizeof(float)));
    }
  }
  const OrbArg orb = make_orb(kernel, n_orb, kappa, alpha);
  phase_begin(t, kPhaseInteract, s);
  // The launches (one per degree, one for the near items) touch disjoint items
  // and partial sums, so they run side by side on S.kStreams streams, each after
  // its degree's proxy charges on the same stream: the small high-degree
  // launches cannot fill the GPU on their own. Largest first, each to the stream
  // with the least work so far; all are forked from s and joined back to it.
  const int n_launch = (int)S.list_begin.size() - 1;
  std::vector<int> by_size(std::max(n_launch, 0));
  for (int li = 0; li < n_launch; ++li) by_size[li] = li;
  std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int b) {
    return S.list_begin[a + 1] - S.list_begin[a] > S.list_begin[b + 1] - S.list_begin[b];
  });
  std::vector<int> stream_of(std::max(n_launch, 0), 0);
  {
    int64_t load[LearnedState::kStreams] = {};
    for (int li : by_size) {
      int k = 0;
      for (int j = 1; j < LearnedState::kStreams; ++j)
        if (load[j] < load[k]) k = j;
      stream_of[li] = k;
      load[k] += S.list_begin[li + 1] - S.list_begin[li];
    }
  }
  TAGI_TRY(S.ensure_streams());
  TAGI_HIP(hipEventRecord(S.fork, s));
  for (int k = 0; k < LearnedState::kStreams; ++k)
    TAGI_HIP(hipStreamWaitEvent(S.streams[k], S.fork, 0));
  for (size_t li = 0; li + 1 < S.list_begin.size(); ++li) {
    const int d = S.list_degree[li];
    hipStream_t ls = S.streams[stream_of[li]];
    if (d > 0) {
      // this degree's proxy charges, from the current tree-ordered values, on
      // the stream of the launch that reads them
      ProxySet& ps = t->lx[d];
      TAGI_TRY(compute_proxies(t, ps, ls));
      if (mix) {
        const int64_t K = (int64_t)(d + 1) * (d + 1) * (d + 1);
        TAGI_TRY(launch_to_f32(ps.qhat.as<double>(), ps.qhat32.as<float>(), n_orb * ps.n_approx * K, ls));
        TAGI_TRY(launch_to_f32(ps.what.as<double>(), ps.what32.as<float>(), ps.n_approx * K, ls));
      }
    }
    InteractArgs A{};
    A.items = S.items.as<int4>();
    A.n_items = S.n_items;
    A.chunks = reinterpret_cast<const Chunk*>(S.chunks.p);
    A.leaf_node = t->leaf_node.as<int32_t>();
    A.nbeg = t->nd_begin.as<int32_t>();
    A.nend = t->nd_end.as<int32_t>();
    A.far_id = S.far_id.as<int32_t>();
    A.near_id = S.near_id.as<int32_t>();
    A.xs = t->xs.as<double>();
    A.ys = t->ys.as<double>();
    A.zs = t->zs.as<double>();
    A.qs = t->qs.as<double>();
    A.ws = t->ws.as<double>();
    A.fs = t->fs.as<double>();
    A.geom = t->nd_geom.as<double>();
    A.box = t->nd_box.as<double>();
    A.n = t->n;
    A.n_orb = n_orb;
    A.partial = S.partial.as<double>();
    A.item_list = S.item_lists.as<int32_t>() + S.list_begin[li];
    A.n_list = S.list_begin[li + 1] - S.list_begin[li];
    targets_are_sources(A);
    if (d > 0) {
      const ProxySet& ps = t->lx[d];
      A.slot_of = ps.slot_of.as<int32_t>();
      A.pnodes = ps.pnodes.as<double>();
      A.qhat = ps.qhat.as<double>();
      A.what = ps.what.as<double>();
      A.pnodes32 = ps.pnodes32.as<float>();
      A.qhat32 = ps.qhat32.as<float>();
      A.what32 = ps.what32.as<float>();
      A.n_approx = ps.n_approx;
      A.degree = d;
    } else {
      A.degree = 0;  // near items only: any compiled variant
    }
    A.ia2 = kernel == TAGI_COULOMB_SS ? 1.0 / (alpha * alpha) : 0.0;
    ++t->interact_launches;
    phase_begin(t, kLaunchInteract, ls);
    switch (kernel) {
      case TAGI_YUKAWA_SS: launch_interact_ob<TAGI_YUKAWA_SS>(ob, t, mix, A, orb, ls); break;
      case TAGI_COULOMB_SS: launch_interact_ob<TAGI_COULOMB_SS>(ob, t, mix, A, orb, ls); break;
      case TAGI_YUKAWA: launch_interact_ob<TAGI_YUKAWA>(ob, t, mix, A, orb, ls); break;
      default: launch_interact_ob<TAGI_COULOMB>(ob, t, mix, A, orb, ls); break;
    }
    phase_end(t, kLaunchInteract, ls);
    TAGI_HIP(hipGetLastError());
  }
  for (int k = 0; k < LearnedState::kStreams; ++k) {
    TAGI_HIP(hipEventRecord(S.join[k], S.streams[k]));
    TAGI_HIP(hipStreamWaitEvent(s, S.join[k], 0));
  }
  phase_end(t, kPhaseInteract, s);
  phase_begin(t, kPhaseCombine, s);
  TAGI_TRY(launch_combine(t, ob, kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS,
                          S.group_base.as<int32_t>(),
                          S.group_first.as<int32_t>(), S.batch_chunks.as<int2>(),
                          S.partial.as<double>(), orb, out, s));
  phase_end(t, kPhaseCombine, s);
  return TAGI_OK;
}

}  // namespace tagi
