// Batch-cluster interactions (Algorithm 3, line 3; Eqs. direct-sum_2 and
// particle-cluster-approx-rearranged) with the singularity subtraction of
// Section 4.3, the combine step, and the plain direct sum (Eq. direct-sum).
//
// One wave processes one work item = (batch, group of <= 64 targets, block of
// OB orbitals, chunk of the batch's far or near list); lane l owns target l of the
// group. Sources (proxy points of a far cluster, or particles of a near cluster)
// are the same for every lane, so their coordinates and charges are wave-uniform
// and arrive through scalar loads; the kernel evaluation per pair is vector FP64.
// Per target the wave accumulates
//     a1 = sum K1(d) c      (c = proxy charge of f w, or f_j w_j)
//     a2 = sum K2(d) m      (m = proxy charge of w,   or w_j)
// and the combine kernel forms u_i = a1 - f_i a2 + s f_i with the analytic term
// s = 4 pi / k^2 (Yukawa) or 2 pi a^2 (Coulomb); for the plain kernels u_i = a1.
// Yukawa: K1 = K2 = exp(-k d)/d. Coulomb with Gaussian subtraction: K1 = 1/d,
// K2 = exp(-d^2/a^2)/d. Pairs at distance zero contribute nothing.
//
// Far pairs use the tensor structure of the proxy grid: d^2 is built from the
// per-dimension differences in three nested loops, so one pair costs one
// multiply-add for its squared distance. Items write partial sums per chunk;
// the combine adds them in chunk order, so results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace tagi {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

struct OrbArg {
  double kappa[kMaxOrb];  // Yukawa decay rate per orbital
  double self[kMaxOrb];   // analytic subtraction term per orbital
};

struct Chunk {
  int32_t kind, e0, e1, cost;
};

template <int KER>
struct Pair {
  // accumulate one source (charges c[o], m) at squared distance r2 > 0 with
  // inverse distance rinv, distance r
  template <int OB>
  __device__ __forceinline__ static void add(double r2, double r, double rinv, const double* c,
                                             double m, const double* kap, double ia2,
                                             double* a1, double* a2) {
    if constexpr (KER == TAGI_YUKAWA_SS) {
#pragma unroll
      for (int o = 0; o < OB; ++o) {
        const double g = exp(-kap[o] * r) * rinv;
        a1[o] = fma(g, c[o], a1[o]);
        a2[o] = fma(g, m, a2[o]);
      }
    } else if constexpr (KER == TAGI_YUKAWA) {
#pragma unroll
      for (int o = 0; o < OB; ++o) a1[o] = fma(exp(-kap[o] * r) * rinv, c[o], a1[o]);
    } else if constexpr (KER == TAGI_COULOMB_SS) {
      a2[0] = fma(exp(-r2 * ia2) * rinv, m, a2[0]);
#pragma unroll
      for (int o = 0; o < OB; ++o) a1[o] = fma(rinv, c[o], a1[o]);
    } else {
#pragma unroll
      for (int o = 0; o < OB; ++o) a1[o] = fma(rinv, c[o], a1[o]);
    }
  }
};

template <int KER, int OB>
__global__ __launch_bounds__(kBlock) void k_interact(
    const int4* __restrict__ items, int64_t n_items, const Chunk* __restrict__ chunks,
    const int32_t* __restrict__ leaf_node, const int32_t* __restrict__ nbeg,
    const int32_t* __restrict__ nend, const int32_t* __restrict__ far_id,
    const int32_t* __restrict__ near_id, const int32_t* __restrict__ slot_of,
    const double* __restrict__ xs, const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ qs, const double* __restrict__ ws,
    const double* __restrict__ pnodes, const double* __restrict__ qhat,
    const double* __restrict__ what, int64_t n, int n_orb, int n_approx, int degree,
    double ia2, OrbArg orb, double* __restrict__ partial) {
  const int lane = threadIdx.x % kWave;
  const int it = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave));
  if (it >= n_items) return;
  const int4 item = items[it];
  const int B = leaf_node[item.x];
  const int tb = nbeg[B] + item.y * kWave;
  const int te = min(nend[B], tb + kWave);
  const int i = tb + lane < te ? tb + lane : tb;
  const double xi = xs[i], yi = ys[i], zi = zs[i];
  const int o0 = item.z * OB;
  double kap[OB];
  int orb_row[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    orb_row[o] = min(o0 + o, n_orb - 1);
    kap[o] = orb.kappa[orb_row[o]];
  }
  double a1[OB], a2[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) a1[o] = a2[o] = 0.0;
  const Chunk ch = chunks[item.w];
  if (ch.kind == 0) {
    const int np1 = degree + 1;
    const int K = np1 * np1 * np1;
    for (int e = ch.e0; e < ch.e1; ++e) {
      const int slot = slot_of[far_id[e]];
      if (slot < 0) continue;  // never taken: far clusters always hold proxy charges
      const double* px = pnodes + (int64_t)slot * 3 * np1;
      const double* py = px + np1;
      const double* pz = py + np1;
      const double* wk = what + (int64_t)slot * K;
      const double* qk[OB];
#pragma unroll
      for (int o = 0; o < OB; ++o) qk[o] = qhat + ((int64_t)orb_row[o] * n_approx + slot) * K;
      int k = 0;
      for (int k1 = 0; k1 < np1; ++k1) {
        const double dx = xi - px[k1];
        const double dx2 = dx * dx;
        for (int k2 = 0; k2 < np1; ++k2) {
          const double dy = yi - py[k2];
          const double dxy = fma(dy, dy, dx2);
          for (int k3 = 0; k3 < np1; ++k3, ++k) {
            const double dz = zi - pz[k3];
            const double r2 = fma(dz, dz, dxy);
            const double rinv = rsqrt(r2);
            const double r = r2 * rinv;
            double c[OB];
#pragma unroll
            for (int o = 0; o < OB; ++o) c[o] = qk[o][k];
            Pair<KER>::template add<OB>(r2, r, rinv, c, wk[k], kap, ia2, a1, a2);
          }
        }
      }
    }
  } else {
    for (int e = ch.e0; e < ch.e1; ++e) {
      const int C = near_id[e];
      const int j1 = nend[C];
      for (int j = nbeg[C]; j < j1; ++j) {
        const double dx = xi - xs[j];
        const double dy = yi - ys[j];
        const double dz = zi - zs[j];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double rinv = r2 > 0.0 ? rsqrt(r2) : 0.0;
        const double r = r2 * rinv;
        double c[OB];
#pragma unroll
        for (int o = 0; o < OB; ++o) c[o] = qs[(int64_t)orb_row[o] * n + j];
        Pair<KER>::template add<OB>(r2, r, rinv, c, ws[j], kap, ia2, a1, a2);
      }
    }
  }
  double* out = partial + (int64_t)it * OB * 2 * kWave;
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    out[(o * 2 + 0) * kWave + lane] = a1[o];
    out[(o * 2 + 1) * kWave + lane] = KER == TAGI_COULOMB_SS ? a2[0] : a2[o];
  }
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

template <int KER, int OB>
void launch_interact(tagi_tree* t, double ia2, const OrbArg& orb, hipStream_t s) {
  const int64_t blocks = (t->n_items + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((k_interact<KER, OB>), dim3(blocks), dim3(kBlock), 0, s,
                     t->items.as<int4>(), t->n_items, t->chunks.as<Chunk>(),
                     t->leaf_node.as<int32_t>(), t->nd_begin.as<int32_t>(),
                     t->nd_end.as<int32_t>(), t->far_id.as<int32_t>(), t->near_id.as<int32_t>(),
                     t->slot_of_node.as<int32_t>(), t->xs.as<double>(), t->ys.as<double>(),
                     t->zs.as<double>(), t->qs.as<double>(), t->ws.as<double>(),
                     t->pnodes.as<double>(), t->qhat.as<double>(), t->what.as<double>(), t->n,
                     t->n_orb, t->n_approx, t->degree, ia2, orb, t->partial.as<double>());
}

template <int KER>
void launch_interact_ob(int ob, tagi_tree* t, double ia2, const OrbArg& orb, hipStream_t s) {
  switch (ob) {
    case 1: launch_interact<KER, 1>(t, ia2, orb, s); break;
    case 2: launch_interact<KER, 2>(t, ia2, orb, s); break;
    case 4: launch_interact<KER, 4>(t, ia2, orb, s); break;
    default: launch_interact<KER, 8>(t, ia2, orb, s); break;
  }
}

// ---------------------------------------------------------------------------
// direct sum: wave = (64-target group, source chunk)

template <int KER>
__global__ __launch_bounds__(kBlock) void k_direct(
    const double* __restrict__ sx, const double* __restrict__ sy, const double* __restrict__ sz,
    const double* __restrict__ sf, const double* __restrict__ sw, int64_t ns,
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
  const int64_t j0 = sc * sc_len, j1 = min(ns, j0 + sc_len);
  double a1[1] = {0.0}, a2[1] = {0.0};
  const double kap[1] = {kappa};
  for (int64_t j = j0; j < j1; ++j) {
    const double dx = xi - sx[j];
    const double dy = yi - sy[j];
    const double dz = zi - sz[j];
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double rinv = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double r = r2 * rinv;
    const double wj = sw[j];
    const double c[1] = {sf[j] * wj};
    Pair<KER>::template add<1>(r2, r, rinv, c, wj, kap, ia2, a1, a2);
  }
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

int convolve(tagi_tree* t, int kernel, const double* kappa, double alpha, int precision,
             double* out, hipStream_t s) {
  (void)precision;
  const int n_orb = t->n_orb;
  const int ob = orbital_block(kernel, n_orb);
  if (t->items_orb_block != ob || t->items_n_orb != n_orb || t->n_items == 0) {
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
  if (t->n_items > 0) {
    phase_begin(t, kPhaseInteract, s);
    ++t->interact_launches;
    switch (kernel) {
      case TAGI_YUKAWA_SS: launch_interact_ob<TAGI_YUKAWA_SS>(ob, t, ia2, orb, s); break;
      case TAGI_COULOMB_SS: launch_interact_ob<TAGI_COULOMB_SS>(ob, t, ia2, orb, s); break;
      case TAGI_YUKAWA: launch_interact_ob<TAGI_YUKAWA>(ob, t, ia2, orb, s); break;
      default: launch_interact_ob<TAGI_COULOMB>(ob, t, ia2, orb, s); break;
    }
    phase_end(t, kPhaseInteract, s);
    TAGI_HIP(hipGetLastError());
  }
  phase_begin(t, kPhaseCombine, s);
  const int ss = kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS;
  hipLaunchKernelGGL(k_combine, dim3((t->n + 255) / 256, n_orb), dim3(256), 0, s, t->n, n_orb,
                     ob, ss, t->perm.as<int32_t>(), t->leaf_of_pos.as<int32_t>(),
                     t->leaf_node.as<int32_t>(), t->nd_begin.as<int32_t>(),
                     t->batch_group_base.as<int32_t>(), t->group_first_item.as<int32_t>(),
                     t->batch_chunks.as<int2>(), t->fs.as<double>(), t->partial.as<double>(), orb,
                     out);
  phase_end(t, kPhaseCombine, s);
  TAGI_HIP(hipGetLastError());
  return TAGI_OK;
}

int orbital_block(int kernel, int n_orb) {
  // Coulomb kernels share all geometry across orbitals, so wider blocks pay off
  if (kernel == TAGI_COULOMB_SS || kernel == TAGI_COULOMB)
    return n_orb >= 8 ? 8 : (n_orb >= 4 ? 4 : (n_orb >= 2 ? 2 : 1));
  return n_orb >= 4 ? 4 : (n_orb >= 2 ? 2 : 1);
}

int direct(const double* sx, const double* sy, const double* sz, const double* sf,
           const double* sw, int64_t ns, const double* tx, const double* ty, const double* tz,
           const double* tf, int64_t nt, int kernel, double kappa, double alpha, double* out,
           hipStream_t s) {
  const int64_t n_groups = (nt + kWave - 1) / kWave;
  // enough waves to fill the machine, chunks of at least 512 sources
  int64_t n_sc = std::max<int64_t>(1, 16384 / n_groups);
  n_sc = std::min<int64_t>(n_sc, std::max<int64_t>(1, ns / 512));
  const int64_t sc_len = (ns + n_sc - 1) / n_sc;
  n_sc = (ns + sc_len - 1) / sc_len;
  // stream-ordered scratch: allocated and freed on `s`, so no host synchronisation
  DBuf part;
  TAGI_HIP(hipMallocAsync(&part.p, (size_t)n_groups * n_sc * 2 * kWave * sizeof(double), s));
  const double ia2 = kernel == TAGI_COULOMB_SS ? 1.0 / (alpha * alpha) : 0.0;
  const int64_t waves = n_groups * n_sc;
  const dim3 grid((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock));
  switch (kernel) {
    case TAGI_YUKAWA_SS:
      hipLaunchKernelGGL(k_direct<TAGI_YUKAWA_SS>, grid, dim3(kBlock), 0, s, sx, sy, sz, sf, sw, ns,
                         tx, ty, tz, nt, (int)n_sc, sc_len, kappa, ia2, part.as<double>());
      break;
    case TAGI_COULOMB_SS:
      hipLaunchKernelGGL(k_direct<TAGI_COULOMB_SS>, grid, dim3(kBlock), 0, s, sx, sy, sz, sf, sw,
                         ns, tx, ty, tz, nt, (int)n_sc, sc_len, kappa, ia2, part.as<double>());
      break;
    case TAGI_YUKAWA:
      hipLaunchKernelGGL(k_direct<TAGI_YUKAWA>, grid, dim3(kBlock), 0, s, sx, sy, sz, sf, sw, ns,
                         tx, ty, tz, nt, (int)n_sc, sc_len, kappa, ia2, part.as<double>());
      break;
    default:
      hipLaunchKernelGGL(k_direct<TAGI_COULOMB>, grid, dim3(kBlock), 0, s, sx, sy, sz, sf, sw, ns,
                         tx, ty, tz, nt, (int)n_sc, sc_len, kappa, ia2, part.as<double>());
      break;
  }
  TAGI_HIP(hipGetLastError());
  const int ss = kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS;
  const double self = kernel == TAGI_YUKAWA_SS ? 4.0 * M_PI / (kappa * kappa)
                                               : (kernel == TAGI_COULOMB_SS ? 2.0 * M_PI * alpha * alpha : 0.0);
  hipLaunchKernelGGL(k_direct_combine, dim3((nt + 255) / 256), dim3(256), 0, s, nt, (int)n_sc, ss,
                     self, tf, part.as<double>(), out);
  TAGI_HIP(hipGetLastError());
  TAGI_HIP(hipFreeAsync(part.p, s));
  return TAGI_OK;
}

}  // namespace tagi
