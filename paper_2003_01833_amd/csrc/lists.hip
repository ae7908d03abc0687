// Algorithm 3, ComputePotential step (Section 6.3): the interaction lists of every target batch,
// precomputed as the paper's GPU implementation does, and the compute schedule.
//
// One thread per batch runs ComputePotential(B, root) with an explicit stack
// (children pushed in reverse so they are visited in order, which reproduces the
// recursive visiting order). MAC (Eq. MAC): a pair is approximated iff
// (r_B + r_C) < theta R and (n+1)^3 < N_S; if the distance test fails, a leaf is
// summed directly and a non-leaf is opened; if only the size test fails, the
// whole cluster is summed directly. A count pass and a fill pass write CSR
// lists (far = approximated, near = direct).
//
// Schedule: each batch's far list and near list are cut into chunks of bounded
// cost (|B| (n+1)^3 per far pair, |B| N_S per near pair); a work item is
// (batch, 64-target group, orbital block, chunk) and is processed by one wave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "interact_impl.hpp"
#include "internal.hpp"

namespace tagi {
namespace {

constexpr int kStack = 512;
// One wave per block. Each lane's traversal stack lives in LDS, laid out
// [entry][lane] (128 KB per block), so every access by a lane falls in its own
// bank; a stack in a per-thread array with a dynamic index would go through
// scratch memory, one memory round trip per pop.
constexpr int kListBlock = 64;

// distance part of Eq. MAC for batch B (geometry bgeom) and cluster C (geom)
__device__ __forceinline__ bool distance_ok(const double* __restrict__ bgeom,
                                            const double* __restrict__ geom, int B, int C,
                                            double theta) {
#pragma clang fp contract(off)
  const double dx = bgeom[B * 4 + 0] - geom[C * 4 + 0];
  const double dy = bgeom[B * 4 + 1] - geom[C * 4 + 1];
  const double dz = bgeom[B * 4 + 2] - geom[C * 4 + 2];
  const double R = sqrt(dx * dx + dy * dy + dz * dz);
  return (bgeom[B * 4 + 3] + geom[C * 4 + 3]) < theta * R;
}

// fill == 0: write counts (far pairs, near pairs, near sources) per batch;
// fill == 1: write the ids at the given offsets. Batches are the leaves
// leaf_node[] of the batch tree (geometry bgeom); clusters are nodes of the
// source tree (geom, nbeg, ...).
__global__ __launch_bounds__(kListBlock) void k_lists(int n_leaves, const int32_t* __restrict__ leaf_node,
                        const double* __restrict__ bgeom,
                        const double* __restrict__ geom, const int32_t* __restrict__ nbeg,
                        const int32_t* __restrict__ nend, const int32_t* __restrict__ first_child,
                        const int32_t* __restrict__ n_child, double theta, int K, int fill,
                        int64_t* __restrict__ far_cnt, int64_t* __restrict__ near_cnt,
                        int64_t* __restrict__ near_src, const int64_t* __restrict__ far_off,
                        const int64_t* __restrict__ near_off, int32_t* __restrict__ far_id,
                        int32_t* __restrict__ near_id, int32_t* __restrict__ overflow,
                        int32_t* __restrict__ root_far) {
  __shared__ int32_t stack[kStack][kListBlock];
  const int lane = threadIdx.x;
  const int b = blockIdx.x * kListBlock + lane;
  if (b >= n_leaves) return;
  const int B = leaf_node[b];
  int sp = 0;
  stack[sp++][lane] = 0;
  int64_t nf = 0, nn = 0, ns = 0;
  int64_t fo = fill ? far_off[b] : 0, no = fill ? near_off[b] : 0;
  while (sp > 0) {
    const int C = stack[--sp][lane];
    const int cnt = nend[C] - nbeg[C];
    const bool dist = distance_ok(bgeom, geom, B, C, theta);
    const bool size = K < cnt;
    int kind;  // 0 far, 1 near, 2 open
    if (dist && size)
      kind = 0;
    else if (!dist)
      kind = n_child[C] == 0 ? 1 : 2;
    else
      kind = 1;
    if (kind == 0) {
      if (fill) far_id[fo + nf] = C;
      if (C == 0 && root_far) *root_far = 1;
      ++nf;
    } else if (kind == 1) {
      if (fill) near_id[no + nn] = C;
      ++nn;
      ns += cnt;
    } else {
      const int fc = first_child[C], nc = n_child[C];
      if (sp + nc > kStack) {
        atomicExch(overflow, 1);
        return;
      }
      for (int k = nc - 1; k >= 0; --k) stack[sp++][lane] = fc + k;
    }
  }
  if (!fill) {
    far_cnt[b] = nf;
    near_cnt[b] = nn;
    near_src[b] = ns;
  }
}

// chunks: per batch, cut the far and near lists into pieces of cost <= cap
struct Chunk {
  int32_t kind, e0, e1, cost;
};

__global__ void k_chunks(int n_leaves, const int32_t* __restrict__ nbeg,
                         const int32_t* __restrict__ nend, const int64_t* __restrict__ far_off,
                         const int64_t* __restrict__ near_off, const int32_t* __restrict__ near_id,
                         int K, int64_t cap, int fill, int32_t* __restrict__ n_chunks,
                         const int32_t* __restrict__ chunk_off, Chunk* __restrict__ chunks) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_leaves) return;
  int nc = 0;
  int32_t co = fill ? chunk_off[b] : 0;
  for (int kind = 0; kind < 2; ++kind) {
    const int64_t e0 = kind == 0 ? far_off[b] : near_off[b];
    const int64_t e1 = kind == 0 ? far_off[b + 1] : near_off[b + 1];
    int64_t start = e0, cost = 0;
    for (int64_t e = e0; e < e1; ++e) {
      const int64_t c = kind == 0 ? K : (int64_t)(nend[near_id[e]] - nbeg[near_id[e]]);
      if (cost > 0 && cost + c > cap) {
        if (fill) chunks[co + nc] = Chunk{kind, (int32_t)start, (int32_t)e, (int32_t)min(cost, (int64_t)INT32_MAX)};
        ++nc;
        start = e;
        cost = 0;
      }
      cost += c;
    }
    if (e1 > start) {
      if (fill) chunks[co + nc] = Chunk{kind, (int32_t)start, (int32_t)e1, (int32_t)min(cost, (int64_t)INT32_MAX)};
      ++nc;
    }
  }
  if (!fill) n_chunks[b] = nc;
}

}  // namespace

// Far-pair counts per batch of the fixed-MAC lists at (theta, size part K < N_S)
// into far_cnt[n_leaves] (device), by the count pass of the list traversal;
// `scratch` must hold 2 n_leaves int64 and one int32.
int count_far_pairs(tagi_tree* t, double theta, int K, int64_t* far_cnt, int64_t* scratch,
                    hipStream_t s) {
  const int nl = (int)t->leaves.size();
  int32_t* d_over = reinterpret_cast<int32_t*>(scratch + 2 * (size_t)nl);
  TAGI_HIP(hipMemsetAsync(d_over, 0, sizeof(int32_t), s));
  hipLaunchKernelGGL(k_lists, dim3((nl + kListBlock - 1) / kListBlock), dim3(kListBlock), 0, s,
                     nl, t->leaf_node.as<int32_t>(), t->nd_geom.as<double>(),
                     t->nd_geom.as<double>(), t->nd_begin.as<int32_t>(), t->nd_end.as<int32_t>(),
                     t->nd_first_child.as<int32_t>(), t->nd_n_child.as<int32_t>(), theta, K, 0,
                     far_cnt, scratch, scratch + nl, nullptr, nullptr, nullptr, nullptr, d_over,
                     nullptr);
  TAGI_HIP(hipGetLastError());
  int32_t over = 0;
  TAGI_HIP(hipMemcpyAsync(&over, d_over, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  if (over) {
    set_error("interaction-list traversal stack overflow (tree deeper than supported)");
    return TAGI_E_UNSUPPORTED;
  }
  return TAGI_OK;
}

int ensure_lists(tagi_tree* src, tagi_tree* bt, double theta, int degree, hipStream_t s,
                 bool* root_far) {
  if (root_far) *root_far = false;
  if (lists_current(src, bt, theta, degree) && !root_far) return TAGI_OK;
  bt->list_theta = -1.0;
  bt->list_degree = -1;
  bt->items_orb_block = 0;
  bt->n_items = 0;
  const int nl = (int)bt->leaves.size();
  const int np1 = degree + 1;
  const int K = np1 * np1 * np1;
  // size part of the MAC: charges per approximated cluster, 8 per point for Hermite
  const bool herm = src->px.herm;
  const int K_mac = (herm ? kHermPatterns : 1) * K;
  DBuf cnt;
  TAGI_TRY(cnt.ensure((size_t)nl * 3 * sizeof(int64_t) + 2 * sizeof(int32_t)));
  int64_t* d_far_cnt = cnt.as<int64_t>();
  int64_t* d_near_cnt = d_far_cnt + nl;
  int64_t* d_near_src = d_near_cnt + nl;
  int32_t* d_over = reinterpret_cast<int32_t*>(d_near_src + nl);
  int32_t* d_root = d_over + 1;
  TAGI_HIP(hipMemsetAsync(d_over, 0, 2 * sizeof(int32_t), s));
  const int blk = kListBlock, grid = (nl + blk - 1) / blk;
  hipLaunchKernelGGL(k_lists, dim3(grid), dim3(blk), 0, s, nl, bt->leaf_node.as<int32_t>(),
                     bt->nd_geom.as<double>(), src->nd_geom.as<double>(),
                     src->nd_begin.as<int32_t>(), src->nd_end.as<int32_t>(),
                     src->nd_first_child.as<int32_t>(), src->nd_n_child.as<int32_t>(), theta,
                     K_mac, 0, d_far_cnt, d_near_cnt, d_near_src, nullptr, nullptr, nullptr,
                     nullptr, d_over, d_root);
  TAGI_HIP(hipGetLastError());
  std::vector<int64_t> h(3 * (size_t)nl);
  int32_t flags[2] = {0, 0};
  TAGI_HIP(hipMemcpyAsync(h.data(), d_far_cnt, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipMemcpyAsync(flags, d_over, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  if (flags[0]) {
    cnt.release();
    set_error("interaction-list traversal stack overflow (tree deeper than supported)");
    return TAGI_E_UNSUPPORTED;
  }
  if (root_far) *root_far = flags[1] != 0;
  bt->h_far_off.assign(nl + 1, 0);
  bt->h_near_off.assign(nl + 1, 0);
  bt->far_inter = bt->near_inter = 0;
  for (int b = 0; b < nl; ++b) {
    bt->h_far_off[b + 1] = bt->h_far_off[b] + h[b];
    bt->h_near_off[b + 1] = bt->h_near_off[b] + h[nl + b];
    const HostNode& q = bt->nodes[bt->leaves[b]];
    const int64_t nb = q.end - q.begin;
    bt->far_inter += nb * h[b] * K;
    bt->near_inter += nb * h[2 * (size_t)nl + b];
  }
  bt->n_far = bt->h_far_off[nl];
  bt->n_near = bt->h_near_off[nl];
  if (bt->n_far >= INT32_MAX || bt->n_near >= INT32_MAX) {
    cnt.release();
    set_error("interaction lists exceed 2^31 entries");
    return TAGI_E_UNSUPPORTED;
  }
  TAGI_TRY(bt->far_off.ensure((nl + 1) * sizeof(int64_t)));
  TAGI_TRY(bt->near_off.ensure((nl + 1) * sizeof(int64_t)));
  TAGI_TRY(bt->far_id.ensure(std::max<int64_t>(bt->n_far, 1) * 4));
  TAGI_TRY(bt->near_id.ensure(std::max<int64_t>(bt->n_near, 1) * 4));
  TAGI_HIP(hipMemcpyAsync(bt->far_off.p, bt->h_far_off.data(), (nl + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  TAGI_HIP(hipMemcpyAsync(bt->near_off.p, bt->h_near_off.data(), (nl + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_lists, dim3(grid), dim3(blk), 0, s, nl, bt->leaf_node.as<int32_t>(),
                     bt->nd_geom.as<double>(), src->nd_geom.as<double>(),
                     src->nd_begin.as<int32_t>(), src->nd_end.as<int32_t>(),
                     src->nd_first_child.as<int32_t>(), src->nd_n_child.as<int32_t>(), theta,
                     K_mac, 1, nullptr, nullptr, nullptr, bt->far_off.as<int64_t>(),
                     bt->near_off.as<int64_t>(), bt->far_id.as<int32_t>(),
                     bt->near_id.as<int32_t>(), d_over, nullptr);
  TAGI_HIP(hipGetLastError());
  TAGI_HIP(hipStreamSynchronize(s));
  cnt.release();
  bt->list_theta = theta;
  bt->list_degree = degree;
  bt->list_herm = herm;
  return TAGI_OK;
}

int ensure_schedule(const tagi_tree* src, tagi_tree* t, int orb_block, hipStream_t s) {
  // t: the batch tree, which holds the lists and receives the schedule
  if (t->items_orb_block == orb_block && t->items_n_orb == src->n_orb && t->n_items > 0)
    return TAGI_OK;
  t->items_orb_block = 0;
  t->n_items = 0;
  const int nl = (int)t->leaves.size();
  const int np1 = t->list_degree + 1;
  // kernel evaluations per far pair and target; a Hermite point costs about two
  const int K = (t->list_herm ? 2 : 1) * np1 * np1 * np1;
  // cost cap per chunk (kernel evaluations per target lane): small enough to give
  // every SIMD several items, large enough to amortise the per-item overhead
  const int64_t total = (t->n_far * (int64_t)K) + t->near_inter / std::max<int64_t>(1, t->n / nl);
  int64_t cap = std::max<int64_t>(total / schedule_items(src), 16 * (int64_t)K);
  cap = std::max<int64_t>(cap, 4096);
  DBuf nch;
  TAGI_TRY(nch.ensure((size_t)(nl + 1) * 2 * sizeof(int32_t)));
  int32_t* d_nch = nch.as<int32_t>();
  int32_t* d_choff = d_nch + nl + 1;
  const int blk = 128, grid = (nl + blk - 1) / blk;
  hipLaunchKernelGGL(k_chunks, dim3(grid), dim3(blk), 0, s, nl, src->nd_begin.as<int32_t>(),
                     src->nd_end.as<int32_t>(), t->far_off.as<int64_t>(), t->near_off.as<int64_t>(),
                     t->near_id.as<int32_t>(), K, cap, 0, d_nch, nullptr, nullptr);
  TAGI_HIP(hipGetLastError());
  std::vector<int32_t> hn(nl);
  TAGI_HIP(hipMemcpyAsync(hn.data(), d_nch, nl * 4, hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> choff(nl + 1, 0);
  for (int b = 0; b < nl; ++b) choff[b + 1] = choff[b] + hn[b];
  const int64_t n_chunks = choff[nl];
  TAGI_TRY(t->chunks.ensure(std::max<int64_t>(n_chunks, 1) * sizeof(Chunk)));
  TAGI_HIP(hipMemcpyAsync(d_choff, choff.data(), nl * 4, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_chunks, dim3(grid), dim3(blk), 0, s, nl, src->nd_begin.as<int32_t>(),
                     src->nd_end.as<int32_t>(), t->far_off.as<int64_t>(), t->near_off.as<int64_t>(),
                     t->near_id.as<int32_t>(), K, cap, 1, d_nch, d_choff, t->chunks.as<Chunk>());
  TAGI_HIP(hipGetLastError());
  // items in (batch, group, orbital block, chunk) order
  const int n_ob = (src->n_orb + orb_block - 1) / orb_block;
  std::vector<int32_t> items;
  std::vector<int32_t> group_first;
  std::vector<int32_t> group_base(nl);
  std::vector<int32_t> bch(2 * (size_t)nl);
  for (int b = 0; b < nl; ++b) {
    const HostNode& q = t->nodes[t->leaves[b]];
    const int ng = (q.end - q.begin + kWave - 1) / kWave;
    group_base[b] = (int32_t)group_first.size();
    bch[2 * b] = choff[b];
    bch[2 * b + 1] = hn[b];
    for (int g = 0; g < ng; ++g) {
      group_first.push_back((int32_t)(items.size() / 4));
      for (int ob = 0; ob < n_ob; ++ob)
        for (int c = 0; c < hn[b]; ++c) {
          items.push_back(b);
          items.push_back(g);
          items.push_back(ob);
          items.push_back(choff[b] + c);
        }
    }
  }
  t->n_items = (int64_t)items.size() / 4;
  if (t->n_items >= INT32_MAX) {
    nch.release();
    set_error("compute schedule exceeds 2^31 work items");
    return TAGI_E_UNSUPPORTED;
  }
  // launch order: the waves of one chunk (same sources, different target groups)
  // run side by side
  std::vector<int32_t> order;
  order.reserve((size_t)t->n_items);
  for (int b = 0; b < nl; ++b) {
    const HostNode& q = t->nodes[t->leaves[b]];
    const int ng = (q.end - q.begin + kWave - 1) / kWave;
    for (int ob = 0; ob < n_ob; ++ob)
      for (int c = 0; c < hn[b]; ++c)
        for (int g = 0; g < ng; ++g)
          order.push_back(group_first[group_base[b] + g] + ob * hn[b] + c);
  }
  // host copies for order_schedule: the chunk-major order as runs of one chunk's
  // waves (start, length, chunk), and each chunk's cost and kind
  t->h_order_base = order;
  t->h_runs.clear();
  for (int b = 0; b < nl; ++b) {
    const HostNode& q = t->nodes[t->leaves[b]];
    const int ng = (q.end - q.begin + kWave - 1) / kWave;
    for (int ob = 0; ob < n_ob; ++ob)
      for (int c = 0; c < hn[b]; ++c) {
        const int32_t start = t->h_runs.empty() ? 0 : t->h_runs.back().start + t->h_runs.back().len;
        t->h_runs.push_back({start, ng, choff[b] + c});
      }
  }
  {
    std::vector<Chunk> hch((size_t)n_chunks);
    if (n_chunks > 0) {
      TAGI_HIP(hipMemcpyAsync(hch.data(), t->chunks.p, hch.size() * sizeof(Chunk),
                              hipMemcpyDeviceToHost, s));
      TAGI_HIP(hipStreamSynchronize(s));
    }
    t->h_chunk_cost.resize(hch.size());
    t->h_chunk_far.resize(hch.size());
    for (size_t c = 0; c < hch.size(); ++c) {
      t->h_chunk_cost[c] = hch[c].cost;
      t->h_chunk_far[c] = hch[c].kind != 1;
    }
  }
  t->items_far_w = -1.0;
  TAGI_TRY(t->items.ensure(std::max<size_t>(items.size(), 4) * 4));
  TAGI_TRY(t->item_order.ensure(std::max<size_t>(order.size(), 1) * 4));
  if (!order.empty())
    TAGI_HIP(hipMemcpyAsync(t->item_order.p, order.data(), order.size() * 4, hipMemcpyHostToDevice, s));
  TAGI_TRY(t->group_first_item.ensure(std::max<size_t>(group_first.size(), 1) * 4));
  TAGI_TRY(t->batch_group_base.ensure((size_t)nl * 4));
  TAGI_TRY(t->batch_chunks.ensure((size_t)nl * 8));
  if (!items.empty())
    TAGI_HIP(hipMemcpyAsync(t->items.p, items.data(), items.size() * 4, hipMemcpyHostToDevice, s));
  if (!group_first.empty())
    TAGI_HIP(hipMemcpyAsync(t->group_first_item.p, group_first.data(), group_first.size() * 4,
                            hipMemcpyHostToDevice, s));
  TAGI_HIP(hipMemcpyAsync(t->batch_group_base.p, group_base.data(), (size_t)nl * 4,
                          hipMemcpyHostToDevice, s));
  TAGI_HIP(hipMemcpyAsync(t->batch_chunks.p, bch.data(), (size_t)nl * 8, hipMemcpyHostToDevice, s));
  TAGI_TRY(t->partial.ensure(std::max<int64_t>(t->n_items, 1) * orb_block * 2 * kWave * sizeof(double)));
  TAGI_HIP(hipStreamSynchronize(s));
  nch.release();
  t->items_orb_block = orb_block;
  t->items_n_orb = src->n_orb;
  return TAGI_OK;
}

// Cost-balanced XCD pieces. Workgroups go to the XCDs round-robin, so each XCD
// runs an equal count of the launch's waves: the range xcd_range gives it. With
// the order cut into equal counts, an XCD whose range holds the costly chunks
// (the dense parts of a mesh come together in tree order) finishes last while
// the others idle. Here the order (runs of waves in list order, each with its
// cost per wave) is cut into kXcds contiguous pieces of equal total cost, the
// pieces keep their waves in order (or sort their runs longest first), and each
// is padded with empty slots (-1, a wave that returns at once) to the length of
// the longest, rounded up to whole workgroups, so that piece x is exactly XCD
// x's range. A run cut by a piece boundary is split.
int balance_runs_per_xcd(std::vector<int32_t>& list, const std::vector<WaveRun>& runs,
                         bool longest_first) {
  struct Piece {
    int32_t a, b;
    double cost;
  };
  const std::vector<int32_t> base = list;
  const int64_t n = (int64_t)base.size();
  if (n == 0) return TAGI_OK;
  double total = 0.0;
  int64_t covered = 0;
  for (const WaveRun& u : runs) {
    total += u.cost * u.len;
    covered += u.len;
  }
  if (covered != n) {
    set_error("internal: %lld run waves for a launch order of %lld", (long long)covered,
              (long long)n);
    return TAGI_E_STATE;
  }
  std::vector<WaveRun> unit;
  const std::vector<WaveRun>* rs = &runs;
  if (!(total > 0.0)) {  // no costs: every wave counts 1
    unit = runs;
    for (WaveRun& u : unit) u.cost = 1.0;
    total = (double)n;
    rs = &unit;
  }
  std::vector<std::vector<Piece>> parts(ik::kXcds);
  int x = 0;
  double acc = 0.0;  // cost assigned to pieces 0..x
  for (const WaveRun& u : *rs) {
    int32_t a = u.start;
    const int32_t e = u.start + u.len;
    while (a < e) {
      // waves of this run that still fit in piece x's share (all, for the last)
      int32_t take = e - a;
      if (x < ik::kXcds - 1 && u.cost > 0.0) {
        const double room = total * (x + 1) / ik::kXcds - acc;
        const int64_t fit = (int64_t)std::ceil(room / u.cost);
        take = (int32_t)std::max<int64_t>(0, std::min<int64_t>(take, fit));
      }
      if (take > 0) {
        parts[x].push_back({a, a + take, u.cost});
        acc += u.cost * take;
        a += take;
      }
      if (a < e && x < ik::kXcds - 1) ++x;
    }
  }
  int64_t len = 0;
  for (const auto& p : parts) {
    int64_t m = 0;
    for (const Piece& q : p) m += q.b - q.a;
    len = std::max(len, m);
  }
  len = (len + ik::kWavesPerBlock - 1) / ik::kWavesPerBlock * ik::kWavesPerBlock;
  list.assign((size_t)(len * ik::kXcds), -1);
  for (int k = 0; k < ik::kXcds; ++k) {
    if (longest_first)
      std::stable_sort(parts[k].begin(), parts[k].end(),
                       [](const Piece& p, const Piece& q) { return p.cost > q.cost; });
    int64_t pos = k * len;
    for (const Piece& q : parts[k])
      for (int32_t i = q.a; i < q.b; ++i) list[(size_t)pos++] = base[(size_t)i];
  }
  return TAGI_OK;
}

// Launch order of the schedule for far evaluations that cost far_w near ones:
// the chunk-major order cut into cost-balanced XCD pieces, each sorted longest
// first (balance_runs_per_xcd over the chunk runs); far_w = 0 keeps the
// chunk-major order cut into equal counts. Results do not depend on the order.
int order_schedule(tagi_tree* t, double far_w, hipStream_t s) {
  if (t->n_items == 0 || t->items_far_w == far_w) return TAGI_OK;
  t->items_far_w = -1.0;  // invalid until the order is on the device
  t->h_order = t->h_order_base;
  if (far_w != 0.0) {
    std::vector<WaveRun> runs(t->h_runs.size());
    for (size_t k = 0; k < runs.size(); ++k) {
      const tagi_tree::Run& u = t->h_runs[k];
      runs[k] = {u.start, u.len,
                 t->h_chunk_cost[u.chunk] * (t->h_chunk_far[u.chunk] ? far_w : 1.0)};
    }
    TAGI_TRY(balance_runs_per_xcd(t->h_order, runs, true));
  }
  TAGI_TRY(t->item_order.ensure(std::max<size_t>(t->h_order.size(), 1) * 4));
  TAGI_HIP(hipMemcpyAsync(t->item_order.p, t->h_order.data(), t->h_order.size() * 4,
                          hipMemcpyHostToDevice, s));
  TAGI_HIP(hipStreamSynchronize(s));  // the host order is reused by the next call
  t->items_far_w = far_w;
  return TAGI_OK;
}

// Far evaluation cost relative to a near one, from the instruction counts of the
// interaction loops: FP64 Yukawa far 23 vs near 28; Coulomb-SS far 10.5 (the
// Gaussian factors per dimension) vs 27; a Hermite point about 65. Mixed
// precision keeps the chunk-major order in equal counts (0): on the 21 benzene
// orbitals it ran 5% faster than the order cut into pieces of equal modelled
// cost (far weight 0.5), and sorting by cost had made it 7% slower, where the
// FP64 launches gain from both.
double far_weight(int kernel, int precision, bool herm) {
  const bool yuk = kernel == TAGI_YUKAWA_SS || kernel == TAGI_YUKAWA;
  if (herm) return 2.3;
  if (precision == TAGI_MIXED) return 0.0;
  return yuk ? 0.8 : 0.4;
}

}  // namespace tagi
