// Adaptive cuboid cells with tensor Fejer quadrature (Section 4.2) on the GPU.
//
// Refinement (Eq. refinement_criterion): after `uniform_levels` bisection rounds,
// every cell C of a round is replaced by its eight children C_i iff
// |int_C t - sum_i int_{C_i} t| >= tol_m, both integrals by the Fejer rule on
// (p+1)^3 Chebyshev points of the first kind (Eq. Chebyshev_points). One
// work-group per cell evaluates the test function at the 9 (p+1)^3 points of the
// cell and its children; the host forms the next round's cells. Afterwards atoms
// are moved onto cell vertices and long cells are halved (aspect repair), and the
// cells are sorted (host). Point generation is one thread per point.
//
// Test functions: the sum of hydrogenic 1s densities Z^3/pi exp(-2 Z d), or
// Eq. test_function, sqrt(rho0) V_ext with that density as rho0 and
// V_ext = -sum_a Z_a / d_a.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <new>
#include <vector>

#include "internal.hpp"

namespace tagi {
namespace {

constexpr int kMaxAtoms = 64;
constexpr int kThreads = 256;

struct TestArgs {
  int kind, n_atoms, p;
  double ax[kMaxAtoms], ay[kMaxAtoms], az[kMaxAtoms], Z[kMaxAtoms];
  double nodes[kMeshMaxP + 1], weights[kMeshMaxP + 1];
};

__device__ double test_fn(const TestArgs& T, double x, double y, double z) {
#pragma clang fp contract(off)
  double rho = 0.0, v = 0.0;
  for (int a = 0; a < T.n_atoms; ++a) {
    const double dx = x - T.ax[a], dy = y - T.ay[a], dz = z - T.az[a];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double Za = T.Z[a];
    rho += Za * Za * Za / M_PI * exp(-2.0 * Za * d);
    v -= Za / d;
  }
  return T.kind == TAGI_TEST_DENSITY ? rho : sqrt(rho) * v;
}

// Fejer integral over [lo, hi] of the test function, one cell per block: each
// thread sums its points, then a fixed-order block reduction
__device__ double cell_integral(const TestArgs& T, const double* lo, const double* hi) {
#pragma clang fp contract(off)
  const int q = T.p + 1, q3 = q * q * q;
  double c[3], h[3];
  for (int d = 0; d < 3; ++d) {
    c[d] = 0.5 * (lo[d] + hi[d]);
    h[d] = 0.5 * (hi[d] - lo[d]);
  }
  double s = 0.0;
  for (int k = threadIdx.x; k < q3; k += blockDim.x) {
    const int i = k / (q * q), j = (k / q) % q, l = k % q;
    const double x = c[0] + h[0] * T.nodes[i];
    const double y = c[1] + h[1] * T.nodes[j];
    const double z = c[2] + h[2] * T.nodes[l];
    const double w = (h[0] * T.weights[i]) * (h[1] * T.weights[j]) * (h[2] * T.weights[l]);
    s += test_fn(T, x, y, z) * w;
  }
  __shared__ double red[kThreads / kWave];
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __syncthreads();
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < kThreads / kWave; ++w) tot += red[w];
  return tot;
}

// flag[c] = 1 iff cell c (boxes [n][6]: lo xyz, hi xyz) is to be split
__global__ __launch_bounds__(kThreads) void k_refine(TestArgs T, const double* __restrict__ box,
                                                     int n, int8_t* __restrict__ flag,
                                                     double tol) {
  const int c = blockIdx.x;
  if (c >= n) return;
  const double* lo = box + (int64_t)c * 6;
  const double* hi = lo + 3;
  const double whole = cell_integral(T, lo, hi);
  double parts = 0.0;
  for (int b = 0; b < 8; ++b) {
    double clo[3], chi[3];
    for (int d = 0; d < 3; ++d) {
      const double mid = 0.5 * (lo[d] + hi[d]);
      const bool up = (b >> (2 - d)) & 1;
      clo[d] = up ? mid : lo[d];
      chi[d] = up ? hi[d] : mid;
    }
    parts += cell_integral(T, clo, chi);
  }
  if (threadIdx.x == 0) flag[c] = fabs(whole - parts) >= tol ? 1 : 0;
}

// points and weights of every cell, x index slowest within a cell
__global__ void k_points(const double* __restrict__ box, int64_t n_points, int q,
                         const double* __restrict__ nodes, const double* __restrict__ weights,
                         double* __restrict__ x, double* __restrict__ y, double* __restrict__ z,
                         double* __restrict__ w) {
#pragma clang fp contract(off)
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_points) return;
  const int q3 = q * q * q;
  const int64_t c = k / q3;
  const int r = (int)(k % q3);
  const int i = r / (q * q), j = (r / q) % q, l = r % q;
  const double* lo = box + c * 6;
  const double* hi = lo + 3;
  double cc[3], h[3];
  for (int d = 0; d < 3; ++d) {
    cc[d] = 0.5 * (lo[d] + hi[d]);
    h[d] = 0.5 * (hi[d] - lo[d]);
  }
  x[k] = cc[0] + h[0] * nodes[i];
  y[k] = cc[1] + h[1] * nodes[j];
  z[k] = cc[2] + h[2] * nodes[l];
  w[k] = ((h[0] * weights[i]) * (h[1] * weights[j])) * (h[2] * weights[l]);
}

using Cell = std::array<double, 6>;  // lo xyz, hi xyz

void children(const Cell& c, std::vector<Cell>& out) {
  double mid[3];
  for (int d = 0; d < 3; ++d) mid[d] = 0.5 * (c[d] + c[3 + d]);
  for (int b = 0; b < 8; ++b) {
    Cell k;
    for (int d = 0; d < 3; ++d) {
      const bool up = (b >> (2 - d)) & 1;
      k[d] = up ? mid[d] : c[d];
      k[3 + d] = up ? c[3 + d] : mid[d];
    }
    out.push_back(k);
  }
}

}  // namespace

int mesh_build(const double* dlo, const double* dhi, int p, double tol, int uniform_levels,
               int max_level, const double* atoms, int n_atoms, int kind, double max_aspect,
               hipStream_t s, tagi_mesh** out) {
  tagi_mesh* m = new (std::nothrow) tagi_mesh();
  if (!m) {
    set_error("tagi_mesh_build: host allocation failed");
    return TAGI_E_OOM;
  }
  std::unique_ptr<tagi_mesh> guard(m);
  m->p = p;
  TestArgs T{};
  T.kind = kind;
  T.n_atoms = n_atoms;
  T.p = p;
  for (int a = 0; a < n_atoms; ++a) {
    T.ax[a] = atoms[4 * a + 0];
    T.ay[a] = atoms[4 * a + 1];
    T.az[a] = atoms[4 * a + 2];
    T.Z[a] = atoms[4 * a + 3];
  }
  // Chebyshev points of the first kind and Fejer's first-rule weights on [-1, 1]
  const int N = p + 1;
  for (int i = 0; i < N; ++i) {
    T.nodes[i] = std::cos((2 * i + 1) * M_PI / (2 * p + 2));
    const double t = (2 * i + 1) * M_PI / (2 * N);
    double acc = 0.0;
    for (int k = 1; k <= N / 2; ++k) acc += std::cos(2 * k * t) / (4 * k * k - 1);
    T.weights[i] = (2.0 / N) * (1.0 - 2.0 * acc);
    m->nodes[i] = T.nodes[i];
    m->weights[i] = T.weights[i];
  }
  std::vector<Cell> cur{{dlo[0], dlo[1], dlo[2], dhi[0], dhi[1], dhi[2]}};
  for (int l = 0; l < uniform_levels; ++l) {
    std::vector<Cell> nxt;
    nxt.reserve(cur.size() * 8);
    for (const Cell& c : cur) children(c, nxt);
    cur.swap(nxt);
  }
  std::vector<Cell> fin;
  DBuf dbox, dflag;
  struct Release {  // frees the round buffers on every return path
    DBuf& a;
    DBuf& b;
    ~Release() {
      a.release();
      b.release();
    }
  } release_bufs{dbox, dflag};
  std::vector<int8_t> flag;
  for (int level = uniform_levels; !cur.empty() && level < max_level; ++level) {
    const int n = (int)cur.size();
    TAGI_TRY(dbox.ensure((size_t)n * sizeof(Cell)));
    TAGI_TRY(dflag.ensure((size_t)n));
    TAGI_HIP(hipMemcpyAsync(dbox.p, cur.data(), (size_t)n * sizeof(Cell), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_refine, dim3(n), dim3(kThreads), 0, s, T, dbox.as<double>(), n,
                       dflag.as<int8_t>(), tol);
    TAGI_HIP(hipGetLastError());
    flag.resize(n);
    TAGI_HIP(hipMemcpyAsync(flag.data(), dflag.p, n, hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipStreamSynchronize(s));
    std::vector<Cell> nxt;
    for (int c = 0; c < n; ++c) {
      if (flag[c]) children(cur[c], nxt);
      else fin.push_back(cur[c]);
    }
    cur.swap(nxt);
  }
  fin.insert(fin.end(), cur.begin(), cur.end());
  // atoms onto vertices
  for (int a = 0; a < n_atoms; ++a) {
    const double A[3] = {atoms[4 * a], atoms[4 * a + 1], atoms[4 * a + 2]};
    std::vector<Cell> nxt;
    for (const Cell& c : fin) {
      bool inside = true;
      int dims[3], nd = 0;
      for (int d = 0; d < 3; ++d) {
        inside = inside && c[d] <= A[d] && A[d] <= c[3 + d];
        if (c[d] < A[d] && A[d] < c[3 + d]) dims[nd++] = d;
      }
      if (!inside || nd == 0) {
        nxt.push_back(c);
        continue;
      }
      for (int b = 0; b < (1 << nd); ++b) {
        Cell k = c;
        for (int j = 0; j < nd; ++j) {
          const int d = dims[j];
          if ((b >> j) & 1) k[d] = A[d];
          else k[3 + d] = A[d];
        }
        nxt.push_back(k);
      }
    }
    fin.swap(nxt);
  }
  // aspect repair
  for (bool changed = true; changed;) {
    changed = false;
    std::vector<Cell> nxt;
    for (const Cell& c : fin) {
      double ext[3];
      for (int d = 0; d < 3; ++d) ext[d] = c[3 + d] - c[d];
      const int dmax = (int)(std::max_element(ext, ext + 3) - ext);
      if (*std::max_element(ext, ext + 3) / *std::min_element(ext, ext + 3) > max_aspect) {
        const double mid = 0.5 * (c[dmax] + c[3 + dmax]);
        Cell a = c, b = c;
        a[3 + dmax] = mid;
        b[dmax] = mid;
        nxt.push_back(a);
        nxt.push_back(b);
        changed = true;
      } else {
        nxt.push_back(c);
      }
    }
    fin.swap(nxt);
  }
  std::sort(fin.begin(), fin.end());  // lexicographic: lo x, lo y, lo z, hi x, hi y, hi z
  m->lo.resize(fin.size() * 3);
  m->hi.resize(fin.size() * 3);
  for (size_t c = 0; c < fin.size(); ++c)
    for (int d = 0; d < 3; ++d) {
      m->lo[c * 3 + d] = fin[c][d];
      m->hi[c * 3 + d] = fin[c][3 + d];
    }
  *out = guard.release();
  return TAGI_OK;
}

int mesh_points(const tagi_mesh* m, double* x, double* y, double* z, double* w, hipStream_t s) {
  const int64_t nc = (int64_t)m->lo.size() / 3;
  const int q = m->p + 1;
  const int64_t np = nc * q * q * q;
  if (np == 0) return TAGI_OK;
  std::vector<double> h((size_t)nc * 6 + 2 * q);
  for (int64_t c = 0; c < nc; ++c)
    for (int d = 0; d < 3; ++d) {
      h[c * 6 + d] = m->lo[c * 3 + d];
      h[c * 6 + 3 + d] = m->hi[c * 3 + d];
    }
  for (int i = 0; i < q; ++i) {
    h[nc * 6 + i] = m->nodes[i];
    h[nc * 6 + q + i] = m->weights[i];
  }
  StreamScratch scratch(s);
  double* d = nullptr;
  TAGI_TRY(scratch.alloc(&d, h.size()));
  TAGI_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_points, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, d, np, q,
                     d + nc * 6, d + nc * 6 + q, x, y, z, w);
  TAGI_HIP(hipGetLastError());
  TAGI_HIP(hipStreamSynchronize(s));  // the host staging buffer goes out of scope
  return TAGI_OK;
}

}  // namespace tagi
