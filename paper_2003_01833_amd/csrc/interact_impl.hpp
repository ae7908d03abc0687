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

// 1/d and, for the Yukawa kernels, d from the squared distance r2; with MASK,
// both are 0 for a coincident pair (r2 = 0), which then adds nothing. With X2
// both come out doubled (2/d, 2d; one operation fewer per pair): callers then
// pass the Yukawa decay constants halved and halve their sums once at the end.
template <int KER, bool MASK, bool X2 = false>
__device__ __forceinline__ void inv_dist(double r2, double& rinv, double& r) {
  if constexpr (KER == TAGI_YUKAWA_SS || KER == TAGI_YUKAWA) {
    if constexpr (X2)
      rsqrt_sqrt_x2(r2, rinv, r);
    else
      rsqrt_sqrt(r2, rinv, r);
  } else {
    rinv = X2 ? rsqrt_pos_x2(r2) : rsqrt_pos(r2);
    r = 0.0;
  }
  if constexpr (MASK) {
    if (!(r2 > 0.0)) rinv = r = 0.0;
  }
}

// Accumulates one source with charges c[o] (per orbital) and m (orbital
// independent) at squared distance r2, inverse distance rinv and distance r
// (Yukawa kernels only), as inv_dist gives them. kl2[o] = -k_o log2(e) and
// al2 = -log2(e) / a^2 are the decay constants in base 2.
template <int KER>
struct Pair {
  template <int OB>
  __device__ __forceinline__ static void add(double r2, double rinv, double r, const double* c,
                                             double m, const double* kl2, double al2,
                                             double* a1, double* a2) {
    if constexpr (KER == TAGI_YUKAWA_SS || KER == TAGI_YUKAWA) {
#pragma unroll
      for (int o = 0; o < OB; ++o) {
        const double g = exp2_scaled(r, kl2[o]) * rinv;
        a1[o] = __builtin_fma(g, c[o], a1[o]);
        if constexpr (KER == TAGI_YUKAWA_SS) a2[o] = __builtin_fma(g, m, a2[o]);
      }
    } else {
      if constexpr (KER == TAGI_COULOMB_SS)
        a2[0] = __builtin_fma(exp2_scaled(r2, al2) * rinv, m, a2[0]);
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
// X2 as for inv_dist: the sums come out doubled. RS: proxy points per step of a
// grid row (kRowStep by default).
template <int KER, int OB, int NP1, bool X2 = false, int RS = kRowStep<OB>>
__device__ __forceinline__ void far_cluster(double xi, double yi, double zi, int np1_rt,
                                            const double* __restrict__ px,
                                            const double* __restrict__ wk,
                                            const double* const* qk, const double* kl2,
                                            double al2, double* a1, double* a2) {
  const int np1 = NP1 ? NP1 : np1_rt;
  const double* py = px + np1;
  const double* pz = py + np1;
  if constexpr (KER == TAGI_COULOMB_SS && NP1 > 0) {
    // The Gaussian of K2 separates over the tensor grid,
    //   exp(-d^2/a^2) = exp(-dx^2/a^2) exp(-dy^2/a^2) exp(-dz^2/a^2),
    // so the cluster needs 3 (n+1) exponentials per target instead of (n+1)^3;
    // along a grid row (fixed x and y) the sum of exp(-dz^2/a^2) w^_k / d is
    // formed first and multiplied by the row's exp(-dx^2/a^2) exp(-dy^2/a^2) once.
    double dz[NP1], gz[NP1], gy[NP1];
#pragma unroll
    for (int k3 = 0; k3 < NP1; ++k3) {
      dz[k3] = zi - pz[k3];
      gz[k3] = exp2_scaled(dz[k3] * dz[k3], al2);
    }
#pragma unroll
    for (int k2 = 0; k2 < NP1; ++k2) {
      const double dy = yi - py[k2];
      gy[k2] = exp2_scaled(dy * dy, al2);
    }
    int k = 0;
    for (int k1 = 0; k1 < NP1; ++k1) {
      const double dx = xi - px[k1];
      const double dx2 = dx * dx;
      const double gx = exp2_scaled(dx2, al2);
#pragma unroll
      for (int k2 = 0; k2 < NP1; ++k2) {
        const double dy = yi - py[k2];
        const double dxy = __builtin_fma(dy, dy, dx2);
        double row = 0.0;
#pragma unroll
        for (int h = 0; h < NP1; h += RS) {
#pragma unroll
          for (int k3 = h; k3 < (h + RS < NP1 ? h + RS : NP1); ++k3) {
            const double r2 = __builtin_fma(dz[k3], dz[k3], dxy);
            const double rinv = X2 ? rsqrt_pos_x2(r2) : rsqrt_pos(r2);
            row = __builtin_fma(gz[k3] * wk[k + k3], rinv, row);
#pragma unroll
            for (int o = 0; o < OB; ++o) a1[o] = __builtin_fma(rinv, qk[o][k + k3], a1[o]);
          }
          if constexpr (RS < NP1) __builtin_amdgcn_sched_barrier(0);
        }
        a2[0] = __builtin_fma(gx * gy[k2], row, a2[0]);
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
        for (int h = 0; h < NP1; h += RS) {
#pragma unroll
          for (int k3 = h; k3 < (h + RS < NP1 ? h + RS : NP1); ++k3) {
            const double dz = zi - pz[k3];
            const double r2 = __builtin_fma(dz, dz, dxy);
            double c[OB];
#pragma unroll
            for (int o = 0; o < OB; ++o) c[o] = qk[o][k + k3];
            double rinv, r;
            inv_dist<KER, false, X2>(r2, rinv, r);
            Pair<KER>::template add<OB>(r2, rinv, r, c, wk[k + k3], kl2, al2, a1, a2);
          }
          if constexpr (RS < NP1) __builtin_amdgcn_sched_barrier(0);
        }
        k += NP1;
      } else {
        for (int k3 = 0; k3 < np1; ++k3, ++k) {
          const double dz = zi - pz[k3];
          const double r2 = __builtin_fma(dz, dz, dxy);
          double c[OB];
#pragma unroll
          for (int o = 0; o < OB; ++o) c[o] = qk[o][k];
          double rinv, r;
          inv_dist<KER, false, X2>(r2, rinv, r);
          Pair<KER>::template add<OB>(r2, rinv, r, c, wk[k], kl2, al2, a1, a2);
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
// Proxy points per step of a grid row in the FP32 far field: whole rows for up
// to 4 orbitals; 2 for 8, whose 9 scalar-loaded doubles per point would
// otherwise overflow the scalar register file.
template <int OB>
constexpr int kRowStep32 = OB >= 8 ? 2 : 16;

template <int KER, int OB, int NP1, bool X2 = false, int RS = kRowStep32<OB>>
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
  const double vzero = 0.0 * (double)ox;  // 0 in a vector register (ox is finite)
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
      a1[o] += (X2 ? 2.0 : 1.0) * (double)b1[o];
      a2[o] += (X2 ? 2.0 : 1.0) * (double)b2[o];
    }
    return;
  }
  // one proxy point k = k0 + k3 of the row whose squared (x, y) offset is dxy
  auto point = [&](int k0, int k3, float dxy) {
    const float dz = oz - pz[k3];
    const float r2 = __builtin_fmaf(dz, dz, dxy);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float m = wk[k0 + k3];
    if constexpr (KER == TAGI_YUKAWA_SS || KER == TAGI_YUKAWA) {
      // The charges of a proxy point arrive in scalar registers and one
      // instruction may read only one of them: the shared w^_k is copied to a
      // vector register once (added to a lane-varying zero), so that each
      // orbital's subtracted charge q^_k - f_i w^_k takes one multiply-add
      // instead of two vector moves and one.
      const double wv = KER == TAGI_YUKAWA_SS ? wk64[k0 + k3] + vzero : 0.0;
      const float r = r2 * rinv;
#pragma unroll
      for (int o = 0; o < OB; ++o) {
        const float g = __builtin_amdgcn_exp2f(nkl2[o] * r) * rinv;
        if constexpr (KER == TAGI_YUKAWA_SS) {
          const double c64 = __builtin_fma(-fi[o], wv, qk64[o][k0 + k3]);
          b1[o] = __builtin_fmaf(g, (float)c64, b1[o]);
        } else {
          b1[o] = __builtin_fmaf(g, qk[o][k0 + k3], b1[o]);
        }
      }
    } else {
      if constexpr (KER == TAGI_COULOMB_SS)
        b2[0] = __builtin_fmaf(__builtin_amdgcn_exp2f(r2 * nial2) * rinv, m, b2[0]);
#pragma unroll
      for (int o = 0; o < OB; ++o) b1[o] = __builtin_fmaf(rinv, qk[o][k0 + k3], b1[o]);
    }
  };
  int k = 0;
  for (int k1 = 0; k1 < np1; ++k1) {
    const float dx = ox - px[k1];
    const float dx2 = dx * dx;
    for (int k2 = 0; k2 < np1; ++k2) {
      const float dy = oy - py[k2];
      const float dxy = __builtin_fmaf(dy, dy, dx2);
      if constexpr (NP1 > 0) {
        // a row in steps of RS points, a scheduling barrier between steps, so
        // that the step's scalar-loaded charges fit the scalar register file
#pragma unroll
        for (int h = 0; h < NP1; h += RS) {
#pragma unroll
          for (int k3 = h; k3 < (h + RS < NP1 ? h + RS : NP1); ++k3) point(k, k3, dxy);
          if constexpr (RS < NP1) __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        for (int k3 = 0; k3 < np1; ++k3) point(k, k3, dxy);
      }
      k += np1;
    }
  }
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    a1[o] += (X2 ? 2.0 : 1.0) * (double)b1[o];
    a2[o] += (X2 ? 2.0 : 1.0) * (double)b2[o];
  }
}

// Near pairs with the particles [j0, j1): coincident points are masked out
// (MASK), or, where the caller has shown that no source coincides with a target
// of the wave, summed without the test. X2 as for inv_dist.
template <int KER, int OB, bool MASK = true, bool X2 = false, int UN = 0>
__device__ __forceinline__ void near_range(double xi, double yi, double zi, int j0, int j1,
                                           const double* __restrict__ xs,
                                           const double* __restrict__ ys,
                                           const double* __restrict__ zs,
                                           const double* __restrict__ ws,
                                           const double* const* qr, const double* kl2,
                                           double al2, double* a1, double* a2) {
  // 4 sources per step for blocks of one or two orbitals; 2 for the masked form
  // (rare: only where a target may coincide with a source) and for blocks of 4
  // or 8 orbitals, whose per-orbital charges of 4 sources overflow the scalar
  // register file (spill moves were a quarter of the 8-orbital loop). UN > 0
  // sets the unmasked step instead.
  constexpr int U = MASK ? 2 : (UN > 0 ? UN : (OB >= 4 ? 2 : 4));
  int j = j0;
  for (; j + U <= j1; j += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double dx = xi - xs[j + u];
      const double dy = yi - ys[j + u];
      const double dz = zi - zs[j + u];
      const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
      double rinv, r;
      inv_dist<KER, MASK, X2>(r2, rinv, r);
      double c[OB];
#pragma unroll
      for (int o = 0; o < OB; ++o) c[o] = qr[o][j + u];
      Pair<KER>::template add<OB>(r2, rinv, r, c, ws[j + u], kl2, al2, a1, a2);
    }
  }
  for (; j < j1; ++j) {
    const double dx = xi - xs[j];
    const double dy = yi - ys[j];
    const double dz = zi - zs[j];
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    double rinv, r;
    inv_dist<KER, MASK, X2>(r2, rinv, r);
    double c[OB];
#pragma unroll
    for (int o = 0; o < OB; ++o) c[o] = qr[o][j];
    Pair<KER>::template add<OB>(r2, rinv, r, c, ws[j], kl2, al2, a1, a2);
  }
}

// Far pairs of one cluster by Hermite interpolation (the Hermite treecode variant
// of the conclusions, Section 8): per proxy point s_k eight charges, one per
// derivative pattern beta of the source point, and
//     sum_k sum_beta d^beta_y G(|y - x_i|)|_{y = s_k} q^_{k,beta}.
// For a radial G and distinct coordinates d^beta_y G = D_|beta|(r) prod (s - x)_d
// with D_0 = G and D_{m+1} = (1/r) dD_m/dr:
//   e^{-k r}/r:     D_m = (-1)^m P_m(k r) e^{-k r} / r^{2m+1}, P_0 = 1, P_1 = 1 + p,
//                   P_2 = 3 + 3p + p^2, P_3 = 15 + 15p + 6p^2 + p^3;
//   1/r:            D_1 = -1/r^3, D_2 = 3/r^5, D_3 = -15/r^7;
//   e^{-b r^2}/r:   D_1 = -E (1/r^3 + 2b/r), D_2 = E (3/r^5 + 4b/r^3 + 4b^2/r),
//                   D_3 = -E (15/r^7 + 18b/r^5 + 12b^2/r^3 + 8b^3/r), b = 1/a^2.
// The charges of one proxy point, taken with the geometric factors of their
// patterns, reduce to four sums S_m (m = |beta|), so a set costs four FMAs with
// the D_m per pair.
template <int OB>
constexpr int kHermStep = 1;

struct HermGeo {
  double g1, g2, g4, g3, g5, g6, g7;  // factors of the patterns x, y, z, xy, xz, yz, xyz
};

__device__ __forceinline__ void herm_sums(const HermGeo& g, const double* __restrict__ c,
                                          double* S) {
  S[0] = c[0];
  S[1] = __builtin_fma(g.g1, c[1], __builtin_fma(g.g2, c[2], g.g4 * c[4]));
  S[2] = __builtin_fma(g.g3, c[3], __builtin_fma(g.g5, c[5], g.g6 * c[6]));
  S[3] = g.g7 * c[7];
}

__device__ __forceinline__ double herm_dot(const double* D, const double* S, double acc) {
  return __builtin_fma(D[0], S[0],
                       __builtin_fma(D[1], S[1], __builtin_fma(D[2], S[2], __builtin_fma(D[3], S[3], acc))));
}

template <int KER, int OB>
__device__ __forceinline__ void herm_point(const HermGeo& g, double r2, const double* __restrict__ m8,
                                           const double* const* q8, const double* kl2,
                                           const double* kap, double al2, double b,
                                           double* a1, double* a2) {
  double rinv, r;
  inv_dist<KER, false>(r2, rinv, r);
  const double ri2 = rinv * rinv;
  constexpr bool SS = KER == TAGI_YUKAWA_SS || KER == TAGI_COULOMB_SS;
  double W[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (SS) herm_sums(g, m8, W);
  if constexpr (KER == TAGI_YUKAWA_SS || KER == TAGI_YUKAWA) {
#pragma unroll
    for (int o = 0; o < OB; ++o) {
      const double p = kap[o] * r;  // k r
      double D[4];
      D[0] = exp2_scaled(r, kl2[o]) * rinv;
      const double t1 = D[0] * ri2;
      D[1] = -(p + 1.0) * t1;
      const double t2 = t1 * ri2;
      D[2] = __builtin_fma(p, p + 3.0, 3.0) * t2;
      D[3] = -__builtin_fma(__builtin_fma(p + 6.0, p, 15.0), p, 15.0) * (t2 * ri2);
      double S[4];
      herm_sums(g, q8[o], S);
      a1[o] = herm_dot(D, S, a1[o]);
      if constexpr (SS) a2[o] = herm_dot(D, W, a2[o]);
    }
  } else {
    const double t1 = rinv * ri2, t2 = t1 * ri2, t3 = t2 * ri2;
    const double D[4] = {rinv, -t1, 3.0 * t2, -15.0 * t3};
#pragma unroll
    for (int o = 0; o < OB; ++o) {
      double S[4];
      herm_sums(g, q8[o], S);
      a1[o] = herm_dot(D, S, a1[o]);
    }
    if constexpr (KER == TAGI_COULOMB_SS) {
      const double E = exp2_scaled(r2, al2);
      const double b2 = b * b;
      double G[4];
      G[0] = E * rinv;
      G[1] = -E * __builtin_fma(2.0 * b, rinv, t1);
      G[2] = E * __builtin_fma(3.0, t2, __builtin_fma(4.0 * b, t1, 4.0 * b2 * rinv));
      G[3] = -E * __builtin_fma(15.0, t3, __builtin_fma(18.0 * b, t2,
                                __builtin_fma(12.0 * b2, t1, 8.0 * b2 * b * rinv)));
      a2[0] = herm_dot(G, W, a2[0]);
    }
  }
}

template <int KER, int OB, int NP1>
__device__ __forceinline__ void far_cluster_herm(double xi, double yi, double zi, int np1_rt,
                                                 const double* __restrict__ px,
                                                 const double* __restrict__ wk,
                                                 const double* const* qk, const double* kl2,
                                                 double al2, double* a1, double* a2) {
  const int np1 = NP1 ? NP1 : np1_rt;
  // k and 1/a^2 for the derivative polynomials
  double kap[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) kap[o] = -kl2[o] * kLn2;
  const double b = -al2 * kLn2;
  const double* py = px + np1;
  const double* pz = py + np1;
  int k = 0;
  for (int k1 = 0; k1 < np1; ++k1) {
    const double dx = px[k1] - xi;
    for (int k2 = 0; k2 < np1; ++k2) {
      const double dy = py[k2] - yi;
      const double dxy2 = __builtin_fma(dy, dy, dx * dx);
      const double pxy = dx * dy;
      for (int h = 0; h < np1; h += kHermStep<OB>) {
#pragma unroll
        for (int u = 0; u < kHermStep<OB>; ++u) {
          const int k3 = h + u;
          if (kHermStep<OB> > 1 && k3 >= np1) break;
          const double dz = pz[k3] - zi;
          const HermGeo g{dx, dy, dz, pxy, dx * dz, dy * dz, pxy * dz};
          const int kk = (k + k3) * kHermPatterns;
          const double* q8[OB];
#pragma unroll
          for (int o = 0; o < OB; ++o) q8[o] = qk[o] + kk;
          herm_point<KER, OB>(g, __builtin_fma(dz, dz, dxy2), wk + kk, q8, kl2, kap, al2, b, a1,
                              a2);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      k += np1;
    }
  }
}

// Everything the interaction kernel reads, passed by value. Source side: the
// source tree's nodes (nbeg, nend, geom, box), sorted particles and proxy data.
// Target side: the batch tree's leaves, node ranges and boxes, and the sorted
// targets with their values (the same arrays as the source side when the
// targets are the sources; targets_are_sources() sets them so).
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
                             // (entries -1 are empty slots)
  int64_t n_list;
  // target side: batch-tree node ranges and boxes, targets [tn] and values [n_orb][tn]
  const int32_t *bbeg, *bend;
  const double* bbox;  // optional, as box
  const double *txs, *tys, *tzs, *tfs;
  int64_t tn;
};

inline void targets_are_sources(InteractArgs& A) {
  A.bbeg = A.nbeg;
  A.bend = A.nend;
  A.bbox = A.box;
  A.txs = A.xs;
  A.tys = A.ys;
  A.tzs = A.zs;
  A.tfs = A.fs;
  A.tn = A.n;
}

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

// the logical blocks [b0, b1) that XCD x runs under xcd_block
__host__ __device__ inline void xcd_range(int x, int nb, int& b0, int& b1) {
  const int q = nb / kXcds, r = nb % kXcds;
  b0 = x * q + (x < r ? x : r);
  b1 = b0 + q + (x < r ? 1 : 0);
}

// The Gaussian of the Coulomb-SS kernel, exp(-d^2/a^2), is below
// exp(-37.5) < 2^-54 for every pair between the boxes of nodes B and C when they
// lie at least 6.12 a apart: such terms are below the FP64 resolution of the
// subtracted sum. Proxy points lie in their cluster's box.
__device__ __forceinline__ bool gauss_negligible(const InteractArgs& A, int B, int C) {
  if (!A.box || !A.bbox) return false;
  const double* bb = A.bbox + (int64_t)B * 6;
  const double* bc = A.box + (int64_t)C * 6;
  double g2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double gap = fmax(0.0, fmax(bc[d] - bb[3 + d], bb[d] - bc[3 + d]));
    g2 = __builtin_fma(gap, gap, g2);
  }
  return g2 * A.ia2 > 37.5;
}

// Far-field forms of the interaction kernel
constexpr int kModeFp64 = 0, kModeMixed = 1, kModeHermite = 2;

// Register budget in waves per SIMD: at least 5 for FP64 tiles and 6 for mixed
// ones (measured 1-7% faster than the compiler's own allocation, which held 4).
// The FP64 Coulomb far field (per-dimension Gaussian factors held in registers),
// blocks of 8 orbitals and the Hermite far field keep the compiler's allocation
// (1 = no bound).
template <int KER, int OB, int MODE>
constexpr int kWavesPerEu =
    (OB >= 8 || MODE == kModeHermite || (KER == TAGI_COULOMB_SS && MODE == kModeFp64))
        ? 1
        : (MODE == kModeMixed ? 6 : 5);

// Launch variants the autotuner chooses between (tagi_tree_set_kernel_variant).
// None changes the arithmetic or its order, so all give the same bits:
//   0  the defaults above;
//   1  the other register budget (the bound where the default has none: 5 waves
//      per SIMD for FP64 tiles, 6 for mixed ones; none where it has one);
//   2  the other proxy-row step of the FP64 far field (whole rows where the
//      default splits them, half rows where it does not);
//   3  the other near-field step (4 sources where the default takes 2, and 2
//      where it takes 4).
// Compiled for the subtracted kernels, degrees 6 to 10 and blocks of 1, 4 and 8
// orbitals; elsewhere every variant runs the defaults. (kKernelVariants, the
// number of variants, is in internal.hpp.)
template <int KER, int OB, int NP1>
constexpr bool kHasVariants = (KER == TAGI_YUKAWA_SS || KER == TAGI_COULOMB_SS) && NP1 >= 7 &&
                              NP1 <= 11 && OB != 2;
template <int KER, int OB, int MODE, int VAR>
constexpr int kWavesPerEuV =
    VAR == 1 ? (kWavesPerEu<KER, OB, MODE> == 1 ? (MODE == kModeMixed ? 6 : 5) : 1)
             : kWavesPerEu<KER, OB, MODE>;
template <int OB, int NP1, int VAR>
constexpr int kRowStepV =
    VAR == 2 && NP1 > 0 ? (kRowStep<OB> < NP1 ? NP1 : (NP1 + 1) / 2) : kRowStep<OB>;
template <int OB, int VAR>
constexpr int kNearStepV = VAR == 3 ? (OB >= 4 ? 4 : 2) : (OB >= 4 ? 2 : 4);

template <int KER, int OB, int NP1, int MODE, int VAR = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWavesPerEuV<KER, OB, MODE, VAR>)))
void k_interact(InteractArgs A, OrbArg orb) {
  constexpr int RS = kRowStepV<OB, NP1, VAR>;
  constexpr int UN = kNearStepV<OB, VAR>;
  const int lane = threadIdx.x % kWave;
  const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
  const int wv = __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + (int)(threadIdx.x / kWave));
  if (A.item_list ? wv >= A.n_list : wv >= A.n_items) return;
  const int it = A.item_list ? __builtin_amdgcn_readfirstlane(A.item_list[wv]) : wv;
  if (it < 0) return;  // an empty slot of a cost-balanced launch order
  const int4 item = A.items[it];
  const int B = A.leaf_node[item.x];
  const int tb = A.bbeg[B] + item.y * kWave;
  const int te = min(A.bend[B], tb + kWave);
  const int i = tb + lane < te ? tb + lane : tb;
  const double xi = A.txs[i], yi = A.tys[i], zi = A.tzs[i];
  const int o0 = item.z * OB;
  // The FP64 and mixed forms sum doubled terms (inv_dist's X2: 2/d and 2d, one
  // operation fewer per pair) and halve the sums at the end; the Yukawa decay
  // constants they use with 2d are halved to match (kl2x). The Hermite form
  // takes powers of 1/d and keeps the plain terms.
  constexpr bool X2 = MODE != kModeHermite;
  double nkap[OB], kl2[OB], kl2x[OB];  // -k, -k log2(e) and its X2 form per orbital
  int orb_row[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    orb_row[o] = min(o0 + o, A.n_orb - 1);
    nkap[o] = -orb.kappa[orb_row[o]];
    kl2[o] = nkap[o] * kLog2e;
    kl2x[o] = X2 ? 0.5 * kl2[o] : kl2[o];
  }
  const double nia2 = -A.ia2;
  const double al2 = nia2 * kLog2e;
  double fi[OB];  // target values, for the FP64 subtracted charges of mixed tiles
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    if constexpr (MODE == kModeMixed && KER == TAGI_YUKAWA_SS)
      fi[o] = A.tfs[(int64_t)orb_row[o] * A.tn + i];
    else
      fi[o] = 0.0;
  }
  double a1[OB], a2[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) a1[o] = a2[o] = 0.0;
  const Chunk ch = A.chunks[item.w];
  if (ch.kind != 1) {  // far chunk (kind 0, or 16 + degree in learned lists)
    const int np1 = A.degree + 1;
    const int K = (MODE == kModeHermite ? kHermPatterns : 1) * np1 * np1 * np1;
    for (int e = ch.e0; e < ch.e1; ++e) {
      const int C = A.far_id[e];
      const int slot = A.slot_of[C];
      if (slot < 0) continue;  // never taken: far clusters always hold proxy charges
      if constexpr (MODE == kModeMixed) {
        float nkl2[OB];
        const float* qk[OB];
        const double* qk64[OB];
#pragma unroll
        for (int o = 0; o < OB; ++o) {
          nkl2[o] = (float)kl2[o];
          qk[o] = A.qhat32 + ((int64_t)orb_row[o] * A.n_approx + slot) * K;
          qk64[o] = A.qhat + ((int64_t)orb_row[o] * A.n_approx + slot) * K;
        }
        const float ox = (float)(xi - A.geom[C * 4 + 0]);
        const float oy = (float)(yi - A.geom[C * 4 + 1]);
        const float oz = (float)(zi - A.geom[C * 4 + 2]);
        far_cluster32<KER, OB, NP1, X2>(ox, oy, oz, np1, A.pnodes32 + (int64_t)slot * 3 * np1,
                                    A.what32 + (int64_t)slot * K, qk, nkl2,
                                    (float)al2, A.what + (int64_t)slot * K, qk64,
                                    fi, a1, a2);
      } else {
        const double* qk[OB];
#pragma unroll
        for (int o = 0; o < OB; ++o) qk[o] = A.qhat + ((int64_t)orb_row[o] * A.n_approx + slot) * K;
        if constexpr (MODE == kModeHermite) {
          far_cluster_herm<KER, OB, NP1>(xi, yi, zi, np1, A.pnodes + (int64_t)slot * 3 * np1,
                                         A.what + (int64_t)slot * K, qk, kl2, al2, a1, a2);
        } else {
          const double* pn = A.pnodes + (int64_t)slot * 3 * np1;
          const double* wk = A.what + (int64_t)slot * K;
          if constexpr (KER == TAGI_COULOMB_SS && OB <= 4) {
            // only the 1/d part where the Gaussian is negligible (not for blocks of
            // 8 orbitals: the second far loop makes their near loop spill)
            if (gauss_negligible(A, B, C))
              far_cluster<TAGI_COULOMB, OB, NP1, X2, RS>(xi, yi, zi, np1, pn, wk, qk, kl2x, al2,
                                                         a1, a2);
            else
              far_cluster<KER, OB, NP1, X2, RS>(xi, yi, zi, np1, pn, wk, qk, kl2x, al2, a1, a2);
          } else {
            far_cluster<KER, OB, NP1, X2, RS>(xi, yi, zi, np1, pn, wk, qk, kl2x, al2, a1, a2);
          }
        }
      }
    }
  } else {
    const double* qr[OB];
#pragma unroll
    for (int o = 0; o < OB; ++o) qr[o] = A.qs + (int64_t)orb_row[o] * A.n;
    for (int e = ch.e0; e < ch.e1; ++e) {
      const int C = A.near_id[e];
      if constexpr (KER == TAGI_COULOMB_SS) {
        // only the 1/d part where the Gaussian is negligible (such a cluster
        // cannot hold a target either)
        if (gauss_negligible(A, B, C)) {
          near_range<TAGI_COULOMB, OB, false, X2, UN>(xi, yi, zi, A.nbeg[C], A.nend[C], A.xs,
                                                      A.ys, A.zs, A.ws, qr, kl2x, al2, a1, a2);
          continue;
        }
      }
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
        near_range<KER, OB, true, X2>(xi, yi, zi, A.nbeg[C], A.nend[C], A.xs, A.ys, A.zs, A.ws,
                                      qr, kl2x, al2, a1, a2);
      else
        near_range<KER, OB, false, X2, UN>(xi, yi, zi, A.nbeg[C], A.nend[C], A.xs, A.ys, A.zs,
                                           A.ws, qr, kl2x, al2, a1, a2);
    }
  }
  double* out = A.partial + (int64_t)it * OB * 2 * kWave;
  constexpr double kScale = X2 ? 0.5 : 1.0;
#pragma unroll
  for (int o = 0; o < OB; ++o) {
    out[(o * 2 + 0) * kWave + lane] = kScale * a1[o];
    out[(o * 2 + 1) * kWave + lane] = kScale * (KER == TAGI_COULOMB_SS ? a2[0] : a2[o]);
  }
}

// The mixed Coulomb-SS far field for 8 orbitals at 12 or more proxy points per
// dimension keeps far more values live than the scalar register file holds
// (over a thousand spilled scalars); it takes the run-time-degree loop instead.
template <int KER, int OB, int NP1>
constexpr int kMixedNP1 = KER == TAGI_COULOMB_SS && OB == 8 && NP1 >= 12 ? 0 : NP1;

template <int KER, int OB, int NP1, int VAR>
void launch_interact_var(bool mix, const InteractArgs& A, const OrbArg& orb, int64_t blocks,
                         hipStream_t s) {
  if (mix)
    hipLaunchKernelGGL((k_interact<KER, OB, kMixedNP1<KER, OB, NP1>, kModeMixed, VAR>),
                       dim3(blocks), dim3(kBlock), 0, s, A, orb);
  else
    hipLaunchKernelGGL((k_interact<KER, OB, NP1, kModeFp64, VAR>), dim3(blocks), dim3(kBlock), 0,
                       s, A, orb);
}

template <int KER, int OB, int NP1>
void launch_interact(tagi_tree* t, bool mix, const InteractArgs& A, const OrbArg& orb,
                     hipStream_t s) {
  const int64_t waves = A.item_list ? A.n_list : A.n_items;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0) return;
  if constexpr (kHasVariants<KER, OB, NP1>) {
    switch (t ? t->kvariant : 0) {
      case 1: launch_interact_var<KER, OB, NP1, 1>(mix, A, orb, blocks, s); return;
      case 2: launch_interact_var<KER, OB, NP1, 2>(mix, A, orb, blocks, s); return;
      case 3: launch_interact_var<KER, OB, NP1, 3>(mix, A, orb, blocks, s); return;
      default: break;
    }
  }
  launch_interact_var<KER, OB, NP1, 0>(mix, A, orb, blocks, s);
}

// Hermite far field: degrees 1 .. kMaxHermDegree
template <int KER, int OB, int NP1>
void launch_interact_herm(const InteractArgs& A, const OrbArg& orb, hipStream_t s) {
  const int64_t waves = A.item_list ? A.n_list : A.n_items;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_interact<KER, OB, NP1, kModeHermite>), dim3(blocks), dim3(kBlock), 0, s, A,
                     orb);
}

template <int KER, int OB>
void launch_interact_herm_np(const InteractArgs& A, const OrbArg& orb, hipStream_t s) {
  switch (A.degree + 1) {
    case 3: launch_interact_herm<KER, OB, 3>(A, orb, s); break;
    case 4: launch_interact_herm<KER, OB, 4>(A, orb, s); break;
    case 5: launch_interact_herm<KER, OB, 5>(A, orb, s); break;
    case 6: launch_interact_herm<KER, OB, 6>(A, orb, s); break;
    default: launch_interact_herm<KER, OB, 0>(A, orb, s); break;
  }
}

template <int KER>
void launch_interact_herm_ob(int ob, const InteractArgs& A, const OrbArg& orb, hipStream_t s) {
  switch (ob) {
    case 1: launch_interact_herm_np<KER, 1>(A, orb, s); break;
    case 2: launch_interact_herm_np<KER, 2>(A, orb, s); break;
    default: launch_interact_herm_np<KER, 4>(A, orb, s); break;
  }
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
    case 12: launch_interact<KER, OB, 12>(t, mix, A, orb, s); break;
    case 13: launch_interact<KER, OB, 13>(t, mix, A, orb, s); break;
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
