// Batch-cluster interactions (Algorithm 3, ComputePotential step; Eqs. direct-sum_2 and
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
// Templates of the batch-cluster interaction kernel, shared by the per-kernel
// translation units interact_*.hip (one per Green's function, compiled in
// parallel) and by the direct sum in interact.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "devmath.hpp"
#include "internal.hpp"

namespace tagi {
namespace ik {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

struct OrbArg {
  double kappa[kMaxOrb];  // Yukawa decay rate per orbital
  double self[kMaxOrb];   // analytic subtraction term per orbital
};

struct Chunk {
  int32_t kind, e0, e1, cost;
};

// Accumulates one source with charges c[o] (per orbital) and m (orbital
// independent) at squared distance r2 with inverse distance rinv (0 for a
// coincident pair, which then adds nothing).
template <int KER>
struct Pair {
  template <int OB>
  __device__ __forceinline__ static void add(double r2, double rinv, const double* c, double m,
                                             const double* nkap, double nia2, double* a1,
                                             double* a2) {
    if constexpr (KER == TAGI_YUKAWA_SS || KER == TAGI_YUKAWA) {
      const double r = r2 * rinv;
#pragma unroll
      for (int o = 0; o < OB; ++o) {
        const double g = exp_nonpos(nkap[o] * r) * rinv;
        a1[o] = __builtin_fma(g, c[o], a1[o]);
        if constexpr (KER == TAGI_YUKAWA_SS) a2[o] = __builtin_fma(g, m, a2[o]);
      }
    } else {
      if constexpr (KER == TAGI_COULOMB_SS)
        a2[0] = __builtin_fma(exp_nonpos(r2 * nia2) * rinv, m, a2[0]);
#pragma unroll
      for (int o = 0; o < OB; ++o) a1[o] = __builtin_fma(rinv, c[o], a1[o]);
    }
  }
};

// Proxy charges of a grid row arrive through scalar loads, (OB + 1) doubles per
// proxy point. A row is taken in steps of kRowStep points, with a scheduling
// barrier between steps, so that the loaded charges stay within the scalar
// register file instead of spilling into vector lanes.
template <int OB>
constexpr int kRowStep = 24 / (OB + 1) > 2 ? 24 / (OB + 1) : 2;

// Far pairs of one cluster: proxy points s_k on the tensor grid px x py x pz
// (NP1 = degree + 1 points per dimension; NP1 == 0 means a run-time degree).
template <int KER, int OB, int NP1>
__device__ __forceinline__ void far_cluster(double xi, double yi, double zi, int np1_rt,
                                            const double* __restrict__ px,
                                            const double* __restrict__ wk,
                                            const double* const* qk, const double* nkap,
                                            double nia2, double* a1, double* a2) {
  const int np1 = NP1 ? NP1 : np1_rt;
  const double* py = px + np1;
  const double* pz = py + np1;
  if constexpr (KER == TAGI_COULOMB_SS && NP1 > 0) {
    // The Gaussian of K2 separates over the tensor grid,
    //   exp(-d^2/a^2) = exp(-dx^2/a^2) exp(-dy^2/a^2) exp(-dz^2/a^2),
    // so the cluster needs 3 (n+1) exponentials per target instead of (n+1)^3.
    double dz[NP1], gz[NP1], gy[NP1];
#pragma unroll
    for (int k3 = 0; k3 < NP1; ++k3) {
      dz[k3] = zi - pz[k3];
      gz[k3] = exp_nonpos(dz[k3] * dz[k3] * nia2);
    }
#pragma unroll
    for (int k2 = 0; k2 < NP1; ++k2) {
      const double dy = yi - py[k2];
      gy[k2] = exp_nonpos(dy * dy * nia2);
    }
    int k = 0;
    for (int k1 = 0; k1 < NP1; ++k1) {
      const double dx = xi - px[k1];
      const double dx2 = dx * dx;
      const double gx = exp_nonpos(dx2 * nia2);
#pragma unroll
      for (int k2 = 0; k2 < NP1; ++k2) {
        const double dy = yi - py[k2];
        const double dxy = __builtin_fma(dy, dy, dx2);
        const double gxy = gx * gy[k2];
#pragma unroll
        for (int h = 0; h < NP1; h += kRowStep<OB>) {
#pragma unroll
          for (int k3 = h; k3 < (h + kRowStep<OB> < NP1 ? h + kRowStep<OB> : NP1); ++k3) {
            const double r2 = __builtin_fma(dz[k3], dz[k3], dxy);
            const double rinv = rsqrt_pos(r2);
            a2[0] = __builtin_fma(gxy * gz[k3] * rinv, wk[k + k3], a2[0]);
#pragma unroll
            for (int o = 0; o < OB; ++o) a1[o] = __builtin_fma(rinv, qk[o][k + k3], a1[o]);
          }
          if constexpr (kRowStep<OB> < NP1) __builtin_amdgcn_sched_barrier(0);
        }
        k += NP1;
      }
    }
    return;
  }
  int k = 0;
  for (int k1 = 0; k1 < np1; ++k1) {
    const double dx = xi - px[k1];
    const double dx2 = dx * dx;
    for (int k2 = 0; k2 < np1; ++k2) {
      const double dy = yi - py[k2];
      const double dxy = __builtin_fma(dy, dy, dx2);
      if constexpr (NP1 > 0) {
#pragma unroll
        for (int h = 0; h < NP1; h += kRowStep<OB>) {
#pragma unroll
          for (int k3 = h; k3 < (h + kRowStep<OB> < NP1 ? h + kRowStep<OB> : NP1); ++k3) {
            const double dz = zi - pz[k3];
            const double r2 = __builtin_fma(dz, dz, dxy);
            double c[OB];
#pragma unroll
            for (int o = 0; o < OB; ++o) c[o] = qk[o][k + k3];
            Pair<KER>::template add<OB>(r2, rsqrt_pos(r2), c, wk[k + k3], nkap, nia2, a1, a2);
          }
          if constexpr (kRowStep<OB> < NP1) __builtin_amdgcn_sched_barrier(0);
        }
        k += NP1;
      } else {
        for (int k3 = 0; k3 < np1; ++k3, ++k) {
          const double dz = zi - pz[k3];
          const double r2 = __builtin_fma(dz, dz, dxy);
          double c[OB];
#pragma unroll
          for (int o = 0; o < OB; ++o) c[o] = qk[o][k];
          Pair<KER>::template add<OB>(r2, rsqrt_pos(r2), c, wk[k], nkap, nia2, a1, a2);
        }
      }
    }
  }
}

// Far pairs of one cluster in FP32 (mixed precision): the target's offset from
// the cluster centre o = r_i - c_C is formed in FP64 and rounded once, the proxy
// points are stored as FP32 offsets from the same centre, so every difference
// o - (s_k - c_C) is taken between numbers no larger than the batch-cluster
// distance. Kernel values use the hardware v_rsq_f32 and v_exp_f32 (2^x, with the
// exponent pre-scaled by log2 e); the cluster's sums accumulate in FP32 and are
// added to the FP64 accumulators once per cluster.
// For the subtracted Yukawa kernel the per-proxy charge is formed in FP64 from
// the FP64 proxy charges, c_k = q^_k - f_i w^_k (one FP64 multiply-add), and only
// G c_k is summed in FP32: summing f_i G w^_k separately in FP32 would carry an
// error of the size of the analytic term 4 pi f_i / k^2, which can exceed u_i by
// orders of magnitude where f is peaked.
template <int KER, int OB, int NP1>
__device__ __forceinline__ void far_cluster32(float ox, float oy, float oz, int np1_rt,
                                              const float* __restrict__ px,
                                              const float* __restrict__ wk,
                                              const float* const* qk, const float* nkl2,
                                              float nial2, const double* __restrict__ wk64,
                                              const double* const* qk64, const double* fi,
                                              double* a1, double* a2) {
  const int np1 = NP1 ? NP1 : np1_rt;
  const float* py = px + np1;
  const float* pz = py + np1;
  float b1[OB], b2[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) b1[o] = b2[o] = 0.0f;
  if constexpr (KER == TAGI_COULOMB_SS && NP1 > 0) {
    // separable Gaussian, as in the FP64 far field
    float dz[NP1], gz[NP1], gy[NP1];
#pragma unroll
    for (int k3 = 0; k3 < NP1; ++k3) {
      dz[k3] = oz - pz[k3];
      gz[k3] = __builtin_amdgcn_exp2f(dz[k3] * dz[k3] * nial2);
    }
#pragma unroll
    for (int k2 = 0; k2 < NP1; ++k2) {
      const float dy = oy - py[k2];
      gy[k2] = __builtin_amdgcn_exp2f(dy * dy * nial2);
    }
    int k = 0;
    for (int k1 = 0; k1 < NP1; ++k1) {
      const float dx = ox - px[k1];
      const float dx2 = dx * dx;
      const float gx = __builtin_amdgcn_exp2f(dx2 * nial2);
#pragma unroll
      for (int k2 = 0; k2 < NP1; ++k2) {
        const float dy = oy - py[k2];
        const float dxy = __builtin_fmaf(dy, dy, dx2);
        const float gxy = gx * gy[k2];
#pragma unroll
        for (int k3 = 0; k3 < NP1; ++k3) {
          const float r2 = __builtin_fmaf(dz[k3], dz[k3], dxy);
          const float rinv = __builtin_amdgcn_rsqf(r2);
          b2[0] = __builtin_fmaf(gxy * gz[k3] * rinv, wk[k + k3], b2[0]);
#pragma unroll
          for (int o = 0; o < OB; ++o) b1[o] = __builtin_fmaf(rinv, qk[o][k + k3], b1[o]);
        }
        k += NP1;
      }
    }
#pragma unroll
    for (int o = 0; o < OB; ++o) {
      a1[o] += (double)b1[o];
      a2[o] += (double)b2[o];
    }
    return;
  }
  int k = 0;
  for (int k1 = 0; k1 < np1; ++k1) {
    const float dx = ox - px[k1];
    const float dx2 = dx * dx;
    for (int k2 = 0; k2 < np1; ++k2) {
      const float dy = oy - py[k2];
      const float dxy = __builtin_fmaf(dy, dy, dx2);
#pragma unroll(NP1 > 0 ? NP1 : 1)
      for (int k3 = 0; k3 < np1; ++k3) {
        const float dz = oz - pz[k3];
        const float r2 = __builtin_fmaf(dz, dz, dxy);
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float m = wk[k + k3];
        if constexpr (KER == TAGI_YUKAWA_SS || KER == TAGI_YUKAWA) {
          const float r = r2 * rinv;
#pragma unroll
          for (int o = 0; o < OB; ++o) {
            const float g = __builtin_amdgcn_exp2f(nkl2[o] * r) * rinv;
            if constexpr (KER == TAGI_YUKAWA_SS) {
              const float c = (float)__builtin_fma(-fi[o], wk64[k + k3], qk64[o][k + k3]);
              b1[o] = __builtin_fmaf(g, c, b1[o]);
            } else {
              b1[o] = __builtin_fmaf(g, qk[o][k + k3], b1[o]);
            }
          }
        } else {
          if constexpr (KER == TAGI_COULOMB_SS)
            b2[0] = __builtin_fmaf(__builtin_amdgcn_exp2f(r2 * nial2) * rinv, m, b2[0]);
#pragma unroll
          for (int o = 0; o < OB; ++o) b1[o] = __builtin_fmaf(rinv, qk[o][k + k3], b1[o]);
        }
      }
      k += np1;
    }
  }
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    a1[o] += (double)b1[o];
    a2[o] += (double)b2[o];
  }
}

// Near pairs with the particles [j0, j1): coincident points are masked out
// (MASK), or, where the caller has shown that no source coincides with a target
// of the wave, summed without the test.
template <int KER, int OB, bool MASK = true>
__device__ __forceinline__ void near_range(double xi, double yi, double zi, int j0, int j1,
                                           const double* __restrict__ xs,
                                           const double* __restrict__ ys,
                                           const double* __restrict__ zs,
                                           const double* __restrict__ ws,
                                           const double* const* qr, const double* nkap,
                                           double nia2, double* a1, double* a2) {
  // 4 sources per step; the masked form (rare: only where a target may coincide
  // with a source) takes 2, which keeps the kernel's scalar registers from
  // spilling into the unmasked loop
  constexpr int U = MASK ? 2 : 4;
  int j = j0;
  for (; j + U <= j1; j += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double dx = xi - xs[j + u];
      const double dy = yi - ys[j + u];
      const double dz = zi - zs[j + u];
      const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
      const double rinv = !MASK || r2 > 0.0 ? rsqrt_pos(r2) : 0.0;
      double c[OB];
#pragma unroll
      for (int o = 0; o < OB; ++o) c[o] = qr[o][j + u];
      Pair<KER>::template add<OB>(r2, rinv, c, ws[j + u], nkap, nia2, a1, a2);
    }
  }
  for (; j < j1; ++j) {
    const double dx = xi - xs[j];
    const double dy = yi - ys[j];
    const double dz = zi - zs[j];
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    const double rinv = !MASK || r2 > 0.0 ? rsqrt_pos(r2) : 0.0;
    double c[OB];
#pragma unroll
    for (int o = 0; o < OB; ++o) c[o] = qr[o][j];
    Pair<KER>::template add<OB>(r2, rinv, c, ws[j], nkap, nia2, a1, a2);
  }
}

// Everything the interaction kernel reads, passed by value.
struct InteractArgs {
  const int4* items;
  int64_t n_items;
  const Chunk* chunks;
  const int32_t *leaf_node, *nbeg, *nend, *far_id, *near_id, *slot_of;
  const double *xs, *ys, *zs, *qs, *ws, *fs;
  const double *pnodes, *qhat, *what, *geom;
  const double* box;  // optional: node bounding boxes [n_nodes][6] (lo xyz, hi xyz)
  const float *pnodes32, *qhat32, *what32;
  int64_t n;
  int n_orb, n_approx, degree;
  double ia2;
  double* partial;
  const int32_t* item_list;  // optional: this launch processes items item_list[0 .. n_list)
  int64_t n_list;
};

// Workgroups are handed to the 8 XCDs of the chip round-robin by their index, and
// every XCD has its own L2. Renumbering the workgroups so that each XCD runs one
// contiguous range of the launch order keeps items that read the same clusters
// (the groups of one chunk, neighbouring batches) on one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds;
  return x * q + min(x, r) + b / kXcds;
}

// Register budget in waves per SIMD: at least 5 for FP64 tiles and 6 for mixed
// ones (measured 1-7% faster than the compiler's own allocation, which held 4).
// The FP64 Coulomb far field (per-dimension Gaussian factors held in registers)
// and blocks of 8 orbitals keep the compiler's allocation (1 = no bound), which
// does not spill.
template <int KER, int OB, bool MIX>
constexpr int kWavesPerEu = (OB >= 8 || (KER == TAGI_COULOMB_SS && !MIX)) ? 1 : (MIX ? 6 : 5);

template <int KER, int OB, int NP1, bool MIX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<KER, OB, MIX>)))
void k_interact(InteractArgs A, OrbArg orb) {
  const int lane = threadIdx.x % kWave;
  const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
  const int wv = __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + (int)(threadIdx.x / kWave));
  if (A.item_list ? wv >= A.n_list : wv >= A.n_items) return;
  const int it = A.item_list ? __builtin_amdgcn_readfirstlane(A.item_list[wv]) : wv;
  const int4 item = A.items[it];
  const int B = A.leaf_node[item.x];
  const int tb = A.nbeg[B] + item.y * kWave;
  const int te = min(A.nend[B], tb + kWave);
  const int i = tb + lane < te ? tb + lane : tb;
  const double xi = A.xs[i], yi = A.ys[i], zi = A.zs[i];
  const int o0 = item.z * OB;
  double nkap[OB];
  int orb_row[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    orb_row[o] = min(o0 + o, A.n_orb - 1);
    nkap[o] = -orb.kappa[orb_row[o]];
  }
  const double nia2 = -A.ia2;
  double fi[OB];  // target values, for the FP64 subtracted charges of mixed tiles
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    if constexpr (MIX && KER == TAGI_YUKAWA_SS)
      fi[o] = A.fs[(int64_t)orb_row[o] * A.n + i];
    else
      fi[o] = 0.0;
  }
  double a1[OB], a2[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) a1[o] = a2[o] = 0.0;
  const Chunk ch = A.chunks[item.w];
  if (ch.kind != 1) {  // far chunk (kind 0, or 16 + degree in learned lists)
    const int np1 = A.degree + 1;
    const int K = np1 * np1 * np1;
    for (int e = ch.e0; e < ch.e1; ++e) {
      const int C = A.far_id[e];
      const int slot = A.slot_of[C];
      if (slot < 0) continue;  // never taken: far clusters always hold proxy charges
      if constexpr (MIX) {
        constexpr double kLog2e = 0x1.71547652b82fep+0;
        float nkl2[OB];
        const float* qk[OB];
        const double* qk64[OB];
#pragma unroll
        for (int o = 0; o < OB; ++o) {
          nkl2[o] = (float)(nkap[o] * kLog2e);
          qk[o] = A.qhat32 + ((int64_t)orb_row[o] * A.n_approx + slot) * K;
          qk64[o] = A.qhat + ((int64_t)orb_row[o] * A.n_approx + slot) * K;
        }
        const float ox = (float)(xi - A.geom[C * 4 + 0]);
        const float oy = (float)(yi - A.geom[C * 4 + 1]);
        const float oz = (float)(zi - A.geom[C * 4 + 2]);
        far_cluster32<KER, OB, NP1>(ox, oy, oz, np1, A.pnodes32 + (int64_t)slot * 3 * np1,
                                    A.what32 + (int64_t)slot * K, qk, nkl2,
                                    (float)(nia2 * kLog2e), A.what + (int64_t)slot * K, qk64,
                                    fi, a1, a2);
      } else {
        const double* qk[OB];
#pragma unroll
        for (int o = 0; o < OB; ++o) qk[o] = A.qhat + ((int64_t)orb_row[o] * A.n_approx + slot) * K;
        far_cluster<KER, OB, NP1>(xi, yi, zi, np1, A.pnodes + (int64_t)slot * 3 * np1,
                                  A.what + (int64_t)slot * K, qk, nkap, nia2, a1, a2);
      }
    }
  } else {
    const double* qr[OB];
#pragma unroll
    for (int o = 0; o < OB; ++o) qr[o] = A.qs + (int64_t)orb_row[o] * A.n;
    for (int e = ch.e0; e < ch.e1; ++e) {
      const int C = A.near_id[e];
      // A source can only coincide with a target inside the cluster's (closed)
      // bounding box; the coincidence test is needed only when some lane's target
      // lies in it.
      bool inside = true;
      if (A.box) {
        const double* bx = A.box + (int64_t)C * 6;
        inside = xi >= bx[0] && xi <= bx[3] && yi >= bx[1] && yi <= bx[4] && zi >= bx[2] &&
                 zi <= bx[5];
      }
      if (__builtin_amdgcn_ballot_w64(inside))
        near_range<KER, OB, true>(xi, yi, zi, A.nbeg[C], A.nend[C], A.xs, A.ys, A.zs, A.ws, qr,
                                  nkap, nia2, a1, a2);
      else
        near_range<KER, OB, false>(xi, yi, zi, A.nbeg[C], A.nend[C], A.xs, A.ys, A.zs, A.ws,
                                   qr, nkap, nia2, a1, a2);
    }
  }
  double* out = A.partial + (int64_t)it * OB * 2 * kWave;
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    out[(o * 2 + 0) * kWave + lane] = a1[o];
    out[(o * 2 + 1) * kWave + lane] = KER == TAGI_COULOMB_SS ? a2[0] : a2[o];
  }
}

template <int KER, int OB, int NP1>
void launch_interact(tagi_tree* t, bool mix, const InteractArgs& A, const OrbArg& orb,
                     hipStream_t s) {
  const int64_t waves = A.item_list ? A.n_list : A.n_items;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0) return;
  if (mix)
    hipLaunchKernelGGL((k_interact<KER, OB, NP1, true>), dim3(blocks), dim3(kBlock), 0, s, A, orb);
  else
    hipLaunchKernelGGL((k_interact<KER, OB, NP1, false>), dim3(blocks), dim3(kBlock), 0, s, A, orb);
}

template <int KER, int OB>
void launch_interact_np(tagi_tree* t, bool mix, const InteractArgs& A, const OrbArg& orb,
                        hipStream_t s) {
  switch (A.degree + 1) {
    case 5: launch_interact<KER, OB, 5>(t, mix, A, orb, s); break;
    case 6: launch_interact<KER, OB, 6>(t, mix, A, orb, s); break;
    case 7: launch_interact<KER, OB, 7>(t, mix, A, orb, s); break;
    case 8: launch_interact<KER, OB, 8>(t, mix, A, orb, s); break;
    case 9: launch_interact<KER, OB, 9>(t, mix, A, orb, s); break;
    case 10: launch_interact<KER, OB, 10>(t, mix, A, orb, s); break;
    case 11: launch_interact<KER, OB, 11>(t, mix, A, orb, s); break;
    default: launch_interact<KER, OB, 0>(t, mix, A, orb, s); break;
  }
}

template <int KER>
void launch_interact_ob(int ob, tagi_tree* t, bool mix, const InteractArgs& A, const OrbArg& orb,
                        hipStream_t s) {
  switch (ob) {
    case 1: launch_interact_np<KER, 1>(t, mix, A, orb, s); break;
    case 2: launch_interact_np<KER, 2>(t, mix, A, orb, s); break;
    case 4: launch_interact_np<KER, 4>(t, mix, A, orb, s); break;
    default: launch_interact_np<KER, 8>(t, mix, A, orb, s); break;
  }
}

// host helpers defined in interact.hip
int launch_combine(tagi_tree* t, int ob, int ss, const int32_t* group_base,
                   const int32_t* group_first, const int2* batch_chunks, const double* partial,
                   const OrbArg& orb, double* out, hipStream_t s);
int launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s);
OrbArg make_orb(int kernel, int n_orb, const double* kappa, double alpha);

}  // namespace ik
}  // namespace tagi
