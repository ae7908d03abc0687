// Algorithm 3, tree step (Section 6.1): source clusters and target batches.
//
// The tree is built level by level on the GPU. At each level, every cluster with
// more than N_L sources is bisected at the midpoint of its box in the dimensions
// the aspect rule selects (extent >= 1/sqrt(2) of the largest), which gives each
// source a 3-bit child digit. A segmented, stable partition by that digit (count
// kernel, host prefix sums over tiles, scatter kernel) reorders the sources so
// that every child is a contiguous range; a tiled min/max reduction then shrinks
// each child to the bounding box of its sources. The host only keeps the node
// table (a few words per cluster) and does the per-level prefix sums, so the
// point data never leaves the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "internal.hpp"

namespace tagi {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kTilePts = kThreads * kPerThread;  // points per partition tile
constexpr double kSqrt1_2 = 0.70710678118654752440;

struct Tile {
  int32_t start, len, node, pad;
};
struct Split {
  double mid[3];
  int32_t mask;  // bit 2: x, bit 1: y, bit 0: z
  int32_t pad;
};

__global__ void k_iota(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// min/max of x, y, z over each tile's range: out[tile][6] = lo xyz, hi xyz
__global__ __launch_bounds__(kThreads) void k_bbox(const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ z,
                                                   const Tile* __restrict__ tiles,
                                                   double* __restrict__ out) {
  const Tile tl = tiles[blockIdx.x];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = threadIdx.x; i < tl.len; i += kThreads) {
    const int64_t p = (int64_t)tl.start + i;
    const double a = x[p], b = y[p], c = z[p];
    v[0] = fmin(v[0], a); v[1] = fmin(v[1], b); v[2] = fmin(v[2], c);
    v[3] = fmax(v[3], a); v[4] = fmax(v[4], b); v[5] = fmax(v[5], c);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    for (int k = 0; k < 3; ++k) v[k] = fmin(v[k], __shfl_xor(v[k], off));
    for (int k = 3; k < 6; ++k) v[k] = fmax(v[k], __shfl_xor(v[k], off));
  }
  __shared__ double red[kThreads / kWave][6];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0)
    for (int k = 0; k < 6; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    double r = red[0][k];
    for (int w = 1; w < kThreads / kWave; ++w) r = k < 3 ? fmin(r, red[w][k]) : fmax(r, red[w][k]);
    out[(int64_t)blockIdx.x * 6 + k] = r;
  }
}

__device__ __forceinline__ int child_digit(double a, double b, double c, const Split& s) {
  int d = 0;
  if ((s.mask & 4) && a >= s.mid[0]) d |= 4;
  if ((s.mask & 2) && b >= s.mid[1]) d |= 2;
  if ((s.mask & 1) && c >= s.mid[2]) d |= 1;
  return d;
}

__global__ __launch_bounds__(kThreads) void k_digit_count(const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ z,
                                                          const Tile* __restrict__ tiles,
                                                          const Split* __restrict__ splits,
                                                          int32_t* __restrict__ counts) {
  __shared__ int cnt[8];
  if (threadIdx.x < 8) cnt[threadIdx.x] = 0;
  __syncthreads();
  const Tile tl = tiles[blockIdx.x];
  const Split sp = splits[tl.node];
  for (int k = 0; k < kPerThread; ++k) {
    const int i = threadIdx.x * kPerThread + k;
    if (i < tl.len) {
      const int64_t p = (int64_t)tl.start + i;
      atomicAdd(&cnt[child_digit(x[p], y[p], z[p], sp)], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < 8) counts[(int64_t)blockIdx.x * 8 + threadIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: the k-th item (in source order) of digit d inside a tile goes to
// dest[tile][d] + (number of earlier items of digit d in the tile). Per-thread
// digit counts are packed 16 bits per digit into two words and prefix-summed
// across the block.
__global__ __launch_bounds__(kThreads) void k_scatter(
    const int32_t* __restrict__ sp_perm, const double* __restrict__ sx,
    const double* __restrict__ sy, const double* __restrict__ sz, int32_t* __restrict__ dp_perm,
    double* __restrict__ dx, double* __restrict__ dy, double* __restrict__ dz,
    const Tile* __restrict__ tiles, const Split* __restrict__ splits,
    const int32_t* __restrict__ dest) {
  const Tile tl = tiles[blockIdx.x];
  const Split sp = splits[tl.node];
  int dig[kPerThread];
  uint64_t pk[2] = {0, 0};
  for (int k = 0; k < kPerThread; ++k) {
    const int i = threadIdx.x * kPerThread + k;
    dig[k] = -1;
    if (i < tl.len) {
      const int64_t p = (int64_t)tl.start + i;
      dig[k] = child_digit(sx[p], sy[p], sz[p], sp);
      pk[dig[k] >> 2] += (uint64_t)1 << (16 * (dig[k] & 3));
    }
  }
  // inclusive wave scan
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  uint64_t inc0 = pk[0], inc1 = pk[1];
  for (int off = 1; off < kWave; off <<= 1) {
    const uint64_t a = __shfl_up(inc0, off), b = __shfl_up(inc1, off);
    if (lane >= off) {
      inc0 += a;
      inc1 += b;
    }
  }
  __shared__ uint64_t wsum[kThreads / kWave][2];
  if (lane == kWave - 1) {
    wsum[wave][0] = inc0;
    wsum[wave][1] = inc1;
  }
  __syncthreads();
  uint64_t ex0 = inc0 - pk[0], ex1 = inc1 - pk[1];
  for (int w = 0; w < wave; ++w) {
    ex0 += wsum[w][0];
    ex1 += wsum[w][1];
  }
  const int32_t* db = dest + (int64_t)blockIdx.x * 8;
  for (int k = 0; k < kPerThread; ++k) {
    if (dig[k] < 0) continue;
    const int d = dig[k];
    uint64_t& word = d < 4 ? ex0 : ex1;
    const int sh = 16 * (d & 3);
    const int rank = (int)((word >> sh) & 0xFFFF);
    word += (uint64_t)1 << sh;
    const int64_t src = (int64_t)tl.start + threadIdx.x * kPerThread + k;
    const int64_t dst = (int64_t)db[d] + rank;
    dp_perm[dst] = sp_perm[src];
    dx[dst] = sx[src];
    dy[dst] = sy[src];
    dz[dst] = sz[src];
  }
}

__global__ void k_leaf_of_pos(const int32_t* __restrict__ leaf_node,
                              const int32_t* __restrict__ nbeg, const int32_t* __restrict__ nend,
                              int32_t* __restrict__ out) {
  const int b = blockIdx.x;
  const int c = leaf_node[b];
  for (int i = nbeg[c] + threadIdx.x; i < nend[c]; i += blockDim.x) out[i] = b;
}

int upload(DBuf& buf, const void* host, size_t bytes, hipStream_t s) {
  TAGI_TRY(buf.ensure(bytes));
  if (bytes) TAGI_HIP(hipMemcpyAsync(buf.p, host, bytes, hipMemcpyHostToDevice, s));
  return TAGI_OK;
}

// bounding boxes of ranges [begin, end) via tiles; returns lo/hi per range
int range_bboxes(const double* x, const double* y, const double* z,
                 const std::vector<std::pair<int32_t, int32_t>>& ranges, DBuf& tiles_buf,
                 DBuf& out_buf, std::vector<double>& boxes, hipStream_t s) {
  std::vector<Tile> tiles;
  std::vector<int32_t> owner;
  const int32_t span = 16 * kTilePts;
  for (size_t r = 0; r < ranges.size(); ++r)
    for (int32_t b = ranges[r].first; b < ranges[r].second; b += span) {
      tiles.push_back({b, std::min(span, ranges[r].second - b), (int32_t)r, 0});
      owner.push_back((int32_t)r);
    }
  boxes.assign(ranges.size() * 6, 0.0);
  for (size_t r = 0; r < ranges.size(); ++r)
    for (int k = 0; k < 3; ++k) {
      boxes[r * 6 + k] = INFINITY;
      boxes[r * 6 + 3 + k] = -INFINITY;
    }
  if (tiles.empty()) return TAGI_OK;
  TAGI_TRY(upload(tiles_buf, tiles.data(), tiles.size() * sizeof(Tile), s));
  TAGI_TRY(out_buf.ensure(tiles.size() * 6 * sizeof(double)));
  hipLaunchKernelGGL(k_bbox, dim3(tiles.size()), dim3(kThreads), 0, s, x, y, z,
                     tiles_buf.as<Tile>(), out_buf.as<double>());
  TAGI_HIP(hipGetLastError());
  std::vector<double> part(tiles.size() * 6);
  TAGI_HIP(hipMemcpyAsync(part.data(), out_buf.p, part.size() * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  for (size_t t = 0; t < tiles.size(); ++t) {
    double* bx = &boxes[owner[t] * 6];
    for (int k = 0; k < 3; ++k) {
      bx[k] = std::min(bx[k], part[t * 6 + k]);
      bx[3 + k] = std::max(bx[3 + k], part[t * 6 + 3 + k]);
    }
  }
  return TAGI_OK;
}

}  // namespace

int build_tree(tagi_tree* t, const double* x, const double* y, const double* z,
               const double* box, hipStream_t s) {
  const int64_t n = t->n;
  const size_t nd = (size_t)n * sizeof(double), ni = (size_t)n * sizeof(int32_t);
  DBuf bperm, bx, by, bz, tiles_buf, split_buf, cnt_buf, dest_buf, part_buf;
  struct Guard {
    DBuf* b[9];
    ~Guard() {
      for (DBuf* p : b) p->release();
    }
  } guard{{&bperm, &bx, &by, &bz, &tiles_buf, &split_buf, &cnt_buf, &dest_buf, &part_buf}};
  TAGI_TRY(t->perm.ensure(ni));
  TAGI_TRY(t->xs.ensure(nd));
  TAGI_TRY(t->ys.ensure(nd));
  TAGI_TRY(t->zs.ensure(nd));
  TAGI_TRY(bperm.ensure(ni));
  TAGI_TRY(bx.ensure(nd));
  TAGI_TRY(by.ensure(nd));
  TAGI_TRY(bz.ensure(nd));
  DBuf* cur[4] = {&t->perm, &t->xs, &t->ys, &t->zs};
  DBuf* nxt[4] = {&bperm, &bx, &by, &bz};

  hipLaunchKernelGGL(k_iota, dim3((n + 255) / 256), dim3(256), 0, s, t->perm.as<int32_t>(), n);
  TAGI_HIP(hipGetLastError());
  TAGI_HIP(hipMemcpyAsync(t->xs.p, x, nd, hipMemcpyDeviceToDevice, s));
  TAGI_HIP(hipMemcpyAsync(t->ys.p, y, nd, hipMemcpyDeviceToDevice, s));
  TAGI_HIP(hipMemcpyAsync(t->zs.p, z, nd, hipMemcpyDeviceToDevice, s));

  // root: shrunk box of all sources; split box = the domain box if given
  std::vector<double> boxes;
  TAGI_TRY(range_bboxes(t->xs.as<double>(), t->ys.as<double>(), t->zs.as<double>(),
                        {{0, (int32_t)n}}, tiles_buf, part_buf, boxes, s));
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(boxes[k])) {
      set_error("tagi_tree_build: a source coordinate is not finite");
      return TAGI_E_ARG;
    }
  double root_split[6];
  if (box) {
    for (int k = 0; k < 3; ++k) {
      if (!(box[k] <= boxes[k]) || !(boxes[3 + k] <= box[3 + k])) {
        set_error("tagi_tree_build: sources lie outside the given box in dimension %d", k);
        return TAGI_E_ARG;
      }
    }
    std::memcpy(root_split, box, sizeof(root_split));
  } else {
    std::memcpy(root_split, boxes.data(), sizeof(root_split));
  }
  t->nodes.clear();
  HostNode root{0, (int32_t)n, -1, 0, -1, 0, {boxes[0], boxes[1], boxes[2]},
                {boxes[3], boxes[4], boxes[5]}};
  t->nodes.push_back(root);

  size_t lv_begin = 0, lv_end = 1;
  for (int level = 0;; ++level) {
    std::vector<int32_t> active;
    std::vector<Split> splits;
    for (size_t c = lv_begin; c < lv_end; ++c) {
      const HostNode& nd_ = t->nodes[c];
      if (nd_.end - nd_.begin <= t->leaf_size) continue;
      double lo[3], hi[3];
      for (int k = 0; k < 3; ++k) {
        lo[k] = c == 0 ? root_split[k] : nd_.lo[k];
        hi[k] = c == 0 ? root_split[3 + k] : nd_.hi[k];
      }
      double ext[3], lmax = 0.0;
      for (int k = 0; k < 3; ++k) {
        ext[k] = hi[k] - lo[k];
        lmax = std::max(lmax, ext[k]);
      }
      if (!(lmax > 0.0)) continue;
      Split sp{};
      for (int k = 0; k < 3; ++k) {
        sp.mid[k] = 0.5 * (lo[k] + hi[k]);
        if (ext[k] >= lmax * kSqrt1_2 && ext[k] > 0.0) sp.mask |= 4 >> k;
      }
      active.push_back((int32_t)c);
      splits.push_back(sp);
    }
    if (active.empty()) break;
    std::vector<Tile> tiles;
    std::vector<int32_t> tile_first(active.size() + 1);
    for (size_t a = 0; a < active.size(); ++a) {
      tile_first[a] = (int32_t)tiles.size();
      const HostNode& nd_ = t->nodes[active[a]];
      for (int32_t b = nd_.begin; b < nd_.end; b += kTilePts)
        tiles.push_back({b, std::min(kTilePts, nd_.end - b), (int32_t)a, 0});
    }
    tile_first[active.size()] = (int32_t)tiles.size();
    const size_t nt = tiles.size();
    TAGI_TRY(upload(tiles_buf, tiles.data(), nt * sizeof(Tile), s));
    TAGI_TRY(upload(split_buf, splits.data(), splits.size() * sizeof(Split), s));
    TAGI_TRY(cnt_buf.ensure(nt * 8 * sizeof(int32_t)));
    hipLaunchKernelGGL(k_digit_count, dim3(nt), dim3(kThreads), 0, s, cur[1]->as<double>(),
                       cur[2]->as<double>(), cur[3]->as<double>(), tiles_buf.as<Tile>(),
                       split_buf.as<Split>(), cnt_buf.as<int32_t>());
    TAGI_HIP(hipGetLastError());
    std::vector<int32_t> counts(nt * 8), dest(nt * 8);
    TAGI_HIP(hipMemcpyAsync(counts.data(), cnt_buf.p, counts.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    TAGI_HIP(hipStreamSynchronize(s));
    std::vector<std::pair<int32_t, int32_t>> child_ranges;
    for (size_t a = 0; a < active.size(); ++a) {
      int64_t tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int32_t tt = tile_first[a]; tt < tile_first[a + 1]; ++tt)
        for (int d = 0; d < 8; ++d) tot[d] += counts[tt * 8 + d];
      const int32_t c = active[a];
      int32_t base[8];
      int32_t off = t->nodes[c].begin;
      int nonempty = 0;
      for (int d = 0; d < 8; ++d) {
        base[d] = off;
        off += (int32_t)tot[d];
        nonempty += tot[d] > 0;
      }
      int32_t run[8];
      std::copy(base, base + 8, run);
      for (int32_t tt = tile_first[a]; tt < tile_first[a + 1]; ++tt)
        for (int d = 0; d < 8; ++d) {
          dest[tt * 8 + d] = run[d];
          run[d] += counts[tt * 8 + d];
        }
      if (nonempty < 2) continue;  // cannot be divided: stays a leaf (scatter is the identity)
      t->nodes[c].first_child = (int32_t)t->nodes.size();
      t->nodes[c].n_child = nonempty;
      for (int d = 0; d < 8; ++d) {
        if (!tot[d]) continue;
        HostNode ch{base[d], base[d] + (int32_t)tot[d], c, level + 1, -1, 0, {0, 0, 0}, {0, 0, 0}};
        t->nodes.push_back(ch);
        child_ranges.push_back({ch.begin, ch.end});
      }
    }
    TAGI_TRY(upload(dest_buf, dest.data(), dest.size() * sizeof(int32_t), s));
    TAGI_HIP(hipMemcpyAsync(nxt[0]->p, cur[0]->p, ni, hipMemcpyDeviceToDevice, s));
    for (int k = 1; k < 4; ++k)
      TAGI_HIP(hipMemcpyAsync(nxt[k]->p, cur[k]->p, nd, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_scatter, dim3(nt), dim3(kThreads), 0, s, cur[0]->as<int32_t>(),
                       cur[1]->as<double>(), cur[2]->as<double>(), cur[3]->as<double>(),
                       nxt[0]->as<int32_t>(), nxt[1]->as<double>(), nxt[2]->as<double>(),
                       nxt[3]->as<double>(), tiles_buf.as<Tile>(), split_buf.as<Split>(),
                       dest_buf.as<int32_t>());
    TAGI_HIP(hipGetLastError());
    std::swap(cur, nxt);
    TAGI_TRY(range_bboxes(cur[1]->as<double>(), cur[2]->as<double>(), cur[3]->as<double>(),
                          child_ranges, tiles_buf, part_buf, boxes, s));
    for (size_t r = 0, c = lv_end; c < t->nodes.size(); ++c, ++r)
      for (int k = 0; k < 3; ++k) {
        t->nodes[c].lo[k] = boxes[r * 6 + k];
        t->nodes[c].hi[k] = boxes[r * 6 + 3 + k];
      }
    lv_begin = lv_end;
    lv_end = t->nodes.size();
    if (lv_begin == lv_end) break;
  }
  // the sorted data must end in the tree's own buffers
  if (cur[0] != &t->perm) {
    std::swap(t->perm, bperm);
    std::swap(t->xs, bx);
    std::swap(t->ys, by);
    std::swap(t->zs, bz);
  }

  // node table on the device; centre = box midpoint, radius = half diagonal
  const size_t nn = t->nodes.size();
  std::vector<int32_t> hb(nn), he(nn), hf(nn), hc(nn);
  std::vector<double> geom(nn * 4), bxs(nn * 6);
  t->leaves.clear();
  t->max_level = 0;
  for (size_t c = 0; c < nn; ++c) {
    const HostNode& q = t->nodes[c];
    hb[c] = q.begin;
    he[c] = q.end;
    hf[c] = q.first_child;
    hc[c] = q.n_child;
    double h[3];
    for (int k = 0; k < 3; ++k) {
      geom[c * 4 + k] = 0.5 * (q.lo[k] + q.hi[k]);
      h[k] = 0.5 * (q.hi[k] - q.lo[k]);
      bxs[c * 6 + k] = q.lo[k];
      bxs[c * 6 + 3 + k] = q.hi[k];
    }
    volatile double r2 = h[0] * h[0];
    volatile double r2b = r2 + h[1] * h[1];
    volatile double r2c = r2b + h[2] * h[2];
    geom[c * 4 + 3] = std::sqrt((double)r2c);
    if (q.n_child == 0) t->leaves.push_back((int32_t)c);
    t->max_level = std::max(t->max_level, q.level);
  }
  TAGI_TRY(upload(t->nd_begin, hb.data(), nn * 4, s));
  TAGI_TRY(upload(t->nd_end, he.data(), nn * 4, s));
  TAGI_TRY(upload(t->nd_first_child, hf.data(), nn * 4, s));
  TAGI_TRY(upload(t->nd_n_child, hc.data(), nn * 4, s));
  TAGI_TRY(upload(t->nd_geom, geom.data(), nn * 4 * sizeof(double), s));
  TAGI_TRY(upload(t->nd_box, bxs.data(), nn * 6 * sizeof(double), s));
  TAGI_TRY(upload(t->leaf_node, t->leaves.data(), t->leaves.size() * 4, s));
  TAGI_TRY(t->leaf_of_pos.ensure(ni));
  hipLaunchKernelGGL(k_leaf_of_pos, dim3(t->leaves.size()), dim3(256), 0, s,
                     t->leaf_node.as<int32_t>(), t->nd_begin.as<int32_t>(),
                     t->nd_end.as<int32_t>(), t->leaf_of_pos.as<int32_t>());
  TAGI_HIP(hipGetLastError());
  TAGI_HIP(hipStreamSynchronize(s));
  return TAGI_OK;
}

}  // namespace tagi
