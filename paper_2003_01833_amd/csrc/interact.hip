// Batch-cluster interactions (Algorithm 3, ComputePotential step; Eqs. direct-sum_2 and
// particle-cluster-approx-rearranged) with the singularity subtraction of
// Section 4.3, the combine step, and the plain direct sum (Eq. direct-sum).
// This file: combine, direct sum and the host side of the convolution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "interact_impl.hpp"

namespace tagi {
namespace ik {
extern template void launch_interact_ob<TAGI_YUKAWA_SS>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_ob<TAGI_COULOMB_SS>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_ob<TAGI_YUKAWA>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_ob<TAGI_COULOMB>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_herm_ob<TAGI_YUKAWA_SS>(int, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_herm_ob<TAGI_COULOMB_SS>(int, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_herm_ob<TAGI_YUKAWA>(int, const InteractArgs&, const OrbArg&, hipStream_t);
extern template void launch_interact_herm_ob<TAGI_COULOMB>(int, const InteractArgs&, const OrbArg&, hipStream_t);
}  // namespace ik

namespace {
using namespace ik;

// out[o][i] = f[o][perm[i]]: caller-order values into a tree's order
__global__ void k_gather_values(const int32_t* __restrict__ perm, const double* __restrict__ f,
                                int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = blockIdx.y;
  if (i < n) out[o * n + i] = f[o * n + perm[i]];
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_combine(int64_t n, int n_orb, int OB, int ss, const int32_t* __restrict__ perm,
                          const int32_t* __restrict__ leaf_of_pos,
                          const int32_t* __restrict__ leaf_node, const int32_t* __restrict__ nbeg,
                          const int32_t* __restrict__ group_base,
                          const int32_t* __restrict__ group_first,
                          const int2* __restrict__ batch_chunks, const double* __restrict__ fs,
                          const double* __restrict__ partial, OrbArg orb,
                          double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int o = blockIdx.y;
  if (i >= n) return;
  const int b = leaf_of_pos[i];
  const int rel = (int)(i - nbeg[leaf_node[b]]);
  const int g = rel / kWave, lane = rel % kWave;
  const int nch = batch_chunks[b].y;
  const int64_t first = group_first[group_base[b] + g] + (int64_t)(o / OB) * nch;
  const int oo = o % OB;
  double a1 = 0.0, a2 = 0.0;
  for (int c = 0; c < nch; ++c) {
    const double* p = partial + (first + c) * OB * 2 * kWave;
    a1 += p[(oo * 2 + 0) * kWave + lane];
    a2 += p[(oo * 2 + 1) * kWave + lane];
  }
  double u = a1;
  if (ss) {
    const double f = fs[(int64_t)o * n + i];
    u = fma(-f, a2, a1) + orb.self[o] * f;
  }
  out[(int64_t)o * n + perm[i]] = u;
}

// ---------------------------------------------------------------------------
// direct sum: wave = (64-target group, source chunk)

__global__ void k_charge(const double* __restrict__ sf, const double* __restrict__ sw, int64_t ns,
                         double* __restrict__ q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < ns) q[j] = sf[j] * sw[j];
}

template <int KER>
__global__ __launch_bounds__(kBlock) void k_direct(
    const double* __restrict__ sx, const double* __restrict__ sy, const double* __restrict__ sz,
    const double* __restrict__ sq, const double* __restrict__ sw, int64_t ns,
    const double* __restrict__ tx, const double* __restrict__ ty, const double* __restrict__ tz,
    int64_t nt, int n_sc, int64_t sc_len, double kappa, double ia2, double* __restrict__ partial) {
  const int lane = threadIdx.x % kWave;
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave));
  const int64_t n_groups = (nt + kWave - 1) / kWave;
  if (w >= n_groups * n_sc) return;
  const int64_t g = w / n_sc;
  const int sc = w % n_sc;
  const int64_t t = g * kWave + lane < nt ? g * kWave + lane : g * kWave;
  const double xi = tx[t], yi = ty[t], zi = tz[t];
  const int j0 = (int)(sc * sc_len), j1 = (int)min(ns, j0 + sc_len);
  double a1[1] = {0.0}, a2[1] = {0.0};
  const double kl2[1] = {-kappa * kLog2e};
  const double* qr[1] = {sq};
  near_range<KER, 1>(xi, yi, zi, j0, j1, sx, sy, sz, sw, qr, kl2, -ia2 * kLog2e, a1, a2);
  double* out = partial + (int64_t)w * 2 * kWave;
  out[lane] = a1[0];
  out[kWave + lane] = a2[0];
}

__global__ void k_direct_combine(int64_t nt, int n_sc, int ss, double self,
                                 const double* __restrict__ tf, const double* __restrict__ partial,
                                 double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int64_t g = t / kWave;
  const int lane = (int)(t % kWave);
  double a1 = 0.0, a2 = 0.0;
  for (int c = 0; c < n_sc; ++c) {
    const double* p = partial + ((g * n_sc) + c) * 2 * kWave;
    a1 += p[lane];
    a2 += p[kWave + lane];
  }
  double u = a1;
  if (ss) {
    const double f = tf[t];
    u = fma(-f, a2, a1) + self * f;
  }
  out[t] = u;
}

}  // namespace

int convolve(tagi_tree* t, tagi_tree* bt, const double* tfs, int kernel, const double* kappa,
             double alpha, int precision, double* out, hipStream_t s) {
  // t: source tree (particles, proxy charges); bt: batch tree (targets, lists,
  // schedule); bt == t when the targets are the sources
  const int n_orb = t->n_orb;
  const int ob = orbital_block_of(t, kernel, precision);
  if (bt->items_orb_block != ob || bt->items_n_orb != n_orb || bt->n_items == 0) {
    set_error("convolve: the compute schedule was not prepared");
    return TAGI_E_STATE;
  }
  OrbArg orb{};
  for (int o = 0; o < n_orb; ++o) {
    const bool yuk = kernel == TAGI_YUKAWA_SS || kernel == TAGI_YUKAWA;
    orb.kappa[o] = yuk ? kappa[o] : 0.0;
    orb.self[o] = kernel == TAGI_YUKAWA_SS ? 4.0 * M_PI / (kappa[o] * kappa[o])
                                           : (kernel == TAGI_COULOMB_SS ? 2.0 * M_PI * alpha * alpha : 0.0);
  }
  const double ia2 = kernel == TAGI_COULOMB_SS ? 1.0 / (alpha * alpha) : 0.0;
  const bool mix = precision == TAGI_MIXED;
  if (mix && t->px.herm) {
    set_error("convolve: the mixed-precision far field takes Lagrange charges (tagi_upward)");
    return TAGI_E_UNSUPPORTED;
  }
  const int np1 = t->degree + 1;
  const int64_t K = (int64_t)np1 * np1 * np1;
  if (mix && t->px.n_approx > 0) {
    // FP32 copies of the FP64 proxy charges for the FP32 far-field tiles
    const int64_t nq = (int64_t)n_orb * t->px.n_approx * K, nw = (int64_t)t->px.n_approx * K;
    TAGI_TRY(t->px.qhat32.ensure(nq * sizeof(float)));
    TAGI_TRY(t->px.what32.ensure(nw * sizeof(float)));
    hipLaunchKernelGGL(k_to_f32, dim3((nq + 255) / 256), dim3(256), 0, s, t->px.qhat.as<double>(),
                       t->px.qhat32.as<float>(), nq);
    hipLaunchKernelGGL(k_to_f32, dim3((nw + 255) / 256), dim3(256), 0, s, t->px.what.as<double>(),
                       t->px.what32.as<float>(), nw);
    TAGI_HIP(hipGetLastError());
  }
  InteractArgs A{};
  A.items = bt->items.as<int4>();
  A.n_items = bt->n_items;
  A.chunks = bt->chunks.as<Chunk>();
  A.leaf_node = bt->leaf_node.as<int32_t>();
  A.nbeg = t->nd_begin.as<int32_t>();
  A.nend = t->nd_end.as<int32_t>();
  A.far_id = bt->far_id.as<int32_t>();
  A.near_id = bt->near_id.as<int32_t>();
  A.slot_of = t->px.slot_of.as<int32_t>();
  A.xs = t->xs.as<double>();
  A.ys = t->ys.as<double>();
  A.zs = t->zs.as<double>();
  A.qs = t->qs.as<double>();
  A.fs = t->fs.as<double>();
  A.ws = t->ws.as<double>();
  A.pnodes = t->px.pnodes.as<double>();
  A.qhat = t->px.qhat.as<double>();
  A.what = t->px.what.as<double>();
  A.geom = t->nd_geom.as<double>();
  A.box = t->nd_box.as<double>();
  A.pnodes32 = t->px.pnodes32.as<float>();
  A.qhat32 = t->px.qhat32.as<float>();
  A.what32 = t->px.what32.as<float>();
  A.n = t->n;
  A.n_orb = n_orb;
  A.n_approx = t->px.n_approx;
  A.degree = t->degree;
  A.ia2 = ia2;
  A.partial = bt->partial.as<double>();
  A.item_list = bt->item_order.as<int32_t>();
  A.n_list = (int64_t)bt->h_order.size();
  A.bbeg = bt->nd_begin.as<int32_t>();
  A.bend = bt->nd_end.as<int32_t>();
  A.bbox = bt->nd_box.as<double>();
  A.txs = bt->xs.as<double>();
  A.tys = bt->ys.as<double>();
  A.tzs = bt->zs.as<double>();
  A.tfs = tfs;
  A.tn = bt->n;
  if (bt->n_items > 0) {
    phase_begin(t, kPhaseInteract, s);
    phase_begin(t, kLaunchInteract, s);
    ++t->interact_launches;
    if (t->px.herm) {
      switch (kernel) {
        case TAGI_YUKAWA_SS: launch_interact_herm_ob<TAGI_YUKAWA_SS>(ob, A, orb, s); break;
        case TAGI_COULOMB_SS: launch_interact_herm_ob<TAGI_COULOMB_SS>(ob, A, orb, s); break;
        case TAGI_YUKAWA: launch_interact_herm_ob<TAGI_YUKAWA>(ob, A, orb, s); break;
        default: launch_interact_herm_ob<TAGI_COULOMB>(ob, A, orb, s); break;
      }
    } else {
      switch (kernel) {
        case TAGI_YUKAWA_SS: launch_interact_ob<TAGI_YUKAWA_SS>(ob, t, mix, A, orb, s); break;
        case TAGI_COULOMB_SS: launch_interact_ob<TAGI_COULOMB_SS>(ob, t, mix, A, orb, s); break;
        case TAGI_YUKAWA: launch_interact_ob<TAGI_YUKAWA>(ob, t, mix, A, orb, s); break;
        default: launch_interact_ob<TAGI_COULOMB>(ob, t, mix, A, orb, s); break;
      }
    }
    phase_end(t, kLaunchInteract, s);
    phase_end(t, kPhaseInteract, s);
    TAGI_HIP(hipGetLastError());
  }
  phase_begin(t, kPhaseCombine, s);
  const int ss = kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS;
  hipLaunchKernelGGL(k_combine, dim3((bt->n + 255) / 256, n_orb), dim3(256), 0, s, bt->n, n_orb,
                     ob, ss, bt->perm.as<int32_t>(), bt->leaf_of_pos.as<int32_t>(),
                     bt->leaf_node.as<int32_t>(), bt->nd_begin.as<int32_t>(),
                     bt->batch_group_base.as<int32_t>(), bt->group_first_item.as<int32_t>(),
                     bt->batch_chunks.as<int2>(), tfs, bt->partial.as<double>(), orb, out);
  phase_end(t, kPhaseCombine, s);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

namespace ik {

int launch_combine(tagi_tree* t, int ob, int ss, const int32_t* group_base,
                   const int32_t* group_first, const int2* batch_chunks, const double* partial,
                   const OrbArg& orb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3((t->n + 255) / 256, t->n_orb), dim3(256), 0, s, t->n,
                     t->n_orb, ob, ss, t->perm.as<int32_t>(), t->leaf_of_pos.as<int32_t>(),
                     t->leaf_node.as<int32_t>(), t->nd_begin.as<int32_t>(), group_base, group_first,
                     batch_chunks, t->fs.as<double>(), partial, orb, out);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

int launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s) {
  if (n <= 0) return TAGI_OK;
  hipLaunchKernelGGL(k_to_f32, dim3((n + 255) / 256), dim3(256), 0, s, a, b, n);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

OrbArg make_orb(int kernel, int n_orb, const double* kappa, double alpha) {
  OrbArg orb{};
  for (int o = 0; o < n_orb; ++o) {
    const bool yuk = kernel == TAGI_YUKAWA_SS || kernel == TAGI_YUKAWA;
    orb.kappa[o] = yuk ? kappa[o] : 0.0;
    orb.self[o] = kernel == TAGI_YUKAWA_SS ? 4.0 * M_PI / (kappa[o] * kappa[o])
                                           : (kernel == TAGI_COULOMB_SS ? 2.0 * M_PI * alpha * alpha : 0.0);
  }
  return orb;
}

}  // namespace ik

int gather_values(const tagi_tree* t, const double* f, int n_orb, double* out, hipStream_t s) {
  if (t->n == 0) return TAGI_OK;
  hipLaunchKernelGGL(k_gather_values, dim3((t->n + 255) / 256, n_orb), dim3(256), 0, s,
                     t->perm.as<int32_t>(), f, t->n, out);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

int orbital_block_of(const tagi_tree* t, int kernel, int precision, bool learned) {
  const int ob =
      t->ob_override ? t->ob_override : orbital_block(kernel, t->n_orb, precision, learned);
  // the Hermite far field reads 8 charges per proxy point and set: at most 4 orbitals
  return t->px.herm ? std::min(ob, 4) : ob;
}

int orbital_block(int kernel, int n_orb, int precision, bool learned) {
  // The widest block that the orbitals fill: a pair's geometry is then shared by
  // more orbitals. Measured on 21 orbitals (benzene): FP64 Yukawa tiles are 9%
  // faster at 8 than at 4. The fixed-MAC mixed launch is 6% faster at 4 (at 8
  // its FP32 tiles hold 4 waves per SIMD instead of 6); the learned lists' mixed
  // launches are 3% faster at 8, where their separate FP64 near launch gains
  // from sharing a pair's geometry over more orbitals.
  const int cap = (precision == TAGI_MIXED && !learned &&
                   (kernel == TAGI_YUKAWA_SS || kernel == TAGI_YUKAWA))
                      ? 4
                      : 8;
  int ob = 1;
  while (ob * 2 <= n_orb && ob * 2 <= cap) ob *= 2;
  return ob;
}

namespace {

// source chunks per 64-target group of the direct sum: enough waves to fill the
// machine, chunks of at least 512 sources
void direct_chunks(int64_t ns, int64_t nt, int64_t* n_sc_out, int64_t* sc_len_out) {
  const int64_t n_groups = (nt + kWave - 1) / kWave;
  int64_t n_sc = std::max<int64_t>(1, 16384 / n_groups);
  n_sc = std::min<int64_t>(n_sc, std::max<int64_t>(1, ns / 512));
  const int64_t sc_len = (ns + n_sc - 1) / n_sc;
  *n_sc_out = (ns + sc_len - 1) / sc_len;
  *sc_len_out = sc_len;
}

// the direct-sum kernels with the charges q [ns] and partial sums
// part [n_groups * n_sc][2][64] in caller-provided device memory
int direct_launch(const double* sx, const double* sy, const double* sz, const double* sf,
                  const double* sw, int64_t ns, const double* tx, const double* ty,
                  const double* tz, const double* tf, int64_t nt, int kernel, double kappa,
                  double alpha, double* out, int64_t n_sc, int64_t sc_len, double* q,
                  double* part, hipStream_t s) {
  const int64_t n_groups = (nt + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_charge, dim3((ns + 255) / 256), dim3(256), 0, s, sf, sw, ns, q);
  const double ia2 = kernel == TAGI_COULOMB_SS ? 1.0 / (alpha * alpha) : 0.0;
  const int64_t waves = n_groups * n_sc;
  const dim3 grid((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock));
#define TAGI_DIRECT(K)                                                                          \
  hipLaunchKernelGGL(k_direct<K>, grid, dim3(kBlock), 0, s, sx, sy, sz, q, sw, ns, tx, ty, tz, \
                     nt, (int)n_sc, sc_len, kappa, ia2, part)
  switch (kernel) {
    case TAGI_YUKAWA_SS: TAGI_DIRECT(TAGI_YUKAWA_SS); break;
    case TAGI_COULOMB_SS: TAGI_DIRECT(TAGI_COULOMB_SS); break;
    case TAGI_YUKAWA: TAGI_DIRECT(TAGI_YUKAWA); break;
    default: TAGI_DIRECT(TAGI_COULOMB); break;
  }
#undef TAGI_DIRECT
  TAGI_HIP(hipGetLastError());
  const int ss = kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS;
  const double self = kernel == TAGI_YUKAWA_SS ? 4.0 * M_PI / (kappa * kappa)
                                               : (kernel == TAGI_COULOMB_SS ? 2.0 * M_PI * alpha * alpha : 0.0);
  hipLaunchKernelGGL(k_direct_combine, dim3((nt + 255) / 256), dim3(256), 0, s, nt, (int)n_sc, ss,
                     self, tf, part, out);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

// Device scratch of the allocation-free direct sum (tagi_direct_noalloc): the
// charges q and the partial sums. Every GPU the library runs on holds its own
// copy until the process ends. In host code `scratch` names a host-side stand-in,
// not device memory: kernels get the per-device address from
// hipGetSymbolAddress, taken once per device.
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's address of `scratch`
int scratch_address(void** out) {
  int dev = 0;
  TAGI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("tagi_direct_noalloc: device %d beyond the %d this library tracks", dev, kMaxDevices);
    return TAGI_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    TAGI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TAGI_OK;
}

}  // namespace

int direct(const double* sx, const double* sy, const double* sz, const double* sf,
           const double* sw, int64_t ns, const double* tx, const double* ty, const double* tz,
           const double* tf, int64_t nt, int kernel, double kappa, double alpha, double* out,
           hipStream_t s) {
  const int64_t n_groups = (nt + kWave - 1) / kWave;
  int64_t n_sc, sc_len;
  direct_chunks(ns, nt, &n_sc, &sc_len);
  // stream-ordered scratch: allocated and freed on `s`, so no host synchronisation
  StreamScratch scr(s);
  double* part = nullptr;
  double* q = nullptr;
  TAGI_TRY(scr.alloc(&part, (size_t)n_groups * n_sc * 2 * kWave));
  TAGI_TRY(scr.alloc(&q, (size_t)ns));
  return direct_launch(sx, sy, sz, sf, sw, ns, tx, ty, tz, tf, nt, kernel, kappa, alpha, out,
                       n_sc, sc_len, q, part, s);
}

size_t direct_noalloc_bytes(int64_t ns, int64_t nt) {
  const int64_t n_groups = (nt + kWave - 1) / kWave;
  int64_t n_sc, sc_len;
  direct_chunks(ns, nt, &n_sc, &sc_len);
  const size_t q_bytes = ((size_t)ns * sizeof(double) + 255) / 256 * 256;
  return q_bytes + (size_t)n_groups * n_sc * 2 * kWave * sizeof(double);
}

size_t direct_noalloc_limit() { return kScratchBytes; }

int direct_noalloc(const double* sx, const double* sy, const double* sz, const double* sf,
                   const double* sw, int64_t ns, const double* tx, const double* ty,
                   const double* tz, const double* tf, int64_t nt, int kernel, double kappa,
                   double alpha, double* out, hipStream_t s) {
  if (direct_noalloc_bytes(ns, nt) > kScratchBytes) {
    set_error("tagi_direct_noalloc: ns = %lld and nt = %lld need %zu bytes of scratch, more than "
              "its %zu",
              (long long)ns, (long long)nt, direct_noalloc_bytes(ns, nt), kScratchBytes);
    return TAGI_E_ARG;
  }
  void* base = nullptr;
  TAGI_TRY(scratch_address(&base));
  int64_t n_sc, sc_len;
  direct_chunks(ns, nt, &n_sc, &sc_len);
  double* q = static_cast<double*>(base);
  double* part = reinterpret_cast<double*>(static_cast<unsigned char*>(base) +
                                           ((size_t)ns * sizeof(double) + 255) / 256 * 256);
  return direct_launch(sx, sy, sz, sf, sw, ns, tx, ty, tz, tf, nt, kernel, kappa, alpha, out,
                       n_sc, sc_len, q, part, s);
}

}  // namespace tagi
