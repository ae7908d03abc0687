// Internal declarations shared by the HIP translation units of libtagi.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tagi.h"

namespace tagi {

// ---------------------------------------------------------------------------
// error state

void set_error(const char* fmt, ...);

#define TAGI_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::tagi::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                        __FILE__, __LINE__);                                        \
      return e_ == hipErrorOutOfMemory ? TAGI_E_OOM : TAGI_E_HIP;                   \
    }                                                                               \
  } while (0)

#define TAGI_TRY(expr)      \
  do {                      \
    int s_ = (expr);        \
    if (s_ != TAGI_OK) return s_; \
  } while (0)

// ---------------------------------------------------------------------------
// grow-only device buffer

// device memory the library holds: every DBuf and StreamScratch allocation is
// counted, and refused with TAGI_E_OOM beyond the TAGI_WORKSPACE_LIMIT
// environment variable (bytes, K/M/G suffixes; unset or 0: no limit), read at
// each allocation
int workspace_take(size_t bytes);   // TAGI_OK, or TAGI_E_OOM with the message set
void workspace_give(size_t bytes);

// one owned device allocation (freed when the holder goes away, early error
// returns included)
struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), cap(o.cap) {
    o.p = nullptr;
    o.cap = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      cap = o.cap;
      o.p = nullptr;
      o.cap = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  int ensure(size_t bytes);   // reallocates (contents lost) when too small
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// stream-ordered device scratch: allocated with hipMallocAsync and freed on the
// same stream when the holder goes out of scope, early error returns included

class StreamScratch {
 public:
  explicit StreamScratch(hipStream_t s) : s_(s) {}
  StreamScratch(const StreamScratch&) = delete;
  StreamScratch& operator=(const StreamScratch&) = delete;
  ~StreamScratch() {
    for (void* p : ptrs_) (void)hipFreeAsync(p, s_);
    workspace_give(held_);
  }
  template <class T>
  int alloc(T** out, size_t count) {
    const size_t bytes = count * sizeof(T) + (count == 0 ? 8 : 0);
    const int st = workspace_take(bytes);
    if (st != TAGI_OK) return st;
    void* p = nullptr;
    const hipError_t e = hipMallocAsync(&p, bytes, s_);
    if (e != hipSuccess) {
      workspace_give(bytes);
      set_error("hipMallocAsync(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
      (void)hipGetLastError();
      return e == hipErrorOutOfMemory ? TAGI_E_OOM : TAGI_E_HIP;
    }
    ptrs_.push_back(p);
    held_ += bytes;
    *out = static_cast<T*>(p);
    return TAGI_OK;
  }

 private:
  hipStream_t s_;
  std::vector<void*> ptrs_;
  size_t held_ = 0;
};

// ---------------------------------------------------------------------------
// tree handle

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxDegree = 16;
constexpr int kMaxOrb = 64;
constexpr int kLearnDegMin = 4, kLearnDegMax = 12;  // degrees the learned selector chooses from
constexpr int kMeshMaxP = 15;                        // largest Fejer order of a mesh cell
// Hermite proxy charges: per proxy point one charge per derivative pattern
// beta in {0,1}^3 (bit 0: d/dx, bit 1: d/dy, bit 2: d/dz of the source point)
constexpr int kHermPatterns = 8;
constexpr int kMaxHermDegree = 7;

struct HostNode {
  int32_t begin, end, parent, level, first_child, n_child;
  double lo[3], hi[3];
};

// Proxy data (Section 6.2) of a set of clusters at one degree.
struct ProxySet {
  int degree = 0;                   // degree of the plan (0 = none)
  int n_orb = 0;
  int n_approx = 0;                 // clusters ("slots") in the set
  int n_items = 0;                  // upward work items
  bool herm = false;                // Hermite charges: 8 per proxy point (see kHermPatterns)
  std::vector<int32_t> nodes;       // host: node id per slot
  std::vector<int32_t> h_slot_of, h_items, h_slot_first;  // host staging for uploads
  DBuf slot_of;                     // int32 [n_nodes], -1 if the node has no slot
  DBuf node;                        // int32 [n_approx]
  DBuf pnodes;                      // double [n_approx][3][degree+1]
  DBuf pnodes32;                    // float [n_approx][3][degree+1], offsets from the cluster centre
  DBuf qhat;                        // double [n_orb][n_approx][(degree+1)^3], Hermite: [..][(degree+1)^3][8]
  DBuf what;                        // double [n_approx][(degree+1)^3], Hermite: [..][(degree+1)^3][8]
  DBuf qhat32, what32;              // FP32 copies for mixed-precision tiles
  DBuf items, partial;              // upward work items (+ slot_first) and partial charges
  void release() {
    for (DBuf* b : {&slot_of, &node, &pnodes, &pnodes32, &qhat, &what, &qhat32, &what32, &items,
                    &partial})
      b->release();
    degree = n_orb = n_approx = n_items = 0;
    herm = false;
  }
};

// Cached state of the learned degree/MAC selection.
struct LearnedState {
  std::vector<double> key;          // arguments the cached lists were built for
  ProxySet l1set;                   // degree-4 charges of every candidate cluster (features)
  DBuf l1n;                         // float l1 norms of those charges: [n_orb][n_nodes] of f w,
                                    // [n_nodes] of w, then [n_orb][n_leaves] max |f| per batch
  DBuf params;                      // float network parameters
  DBuf mb;                          // int64 [n_leaves] far pairs per batch at (theta_max, 4), + scratch
  DBuf cnt;                         // int64 [n_leaves][kDegSlots] counts, offsets; [n_leaves] log sizes
  DBuf log;                         // int32 [n_leaves][log_cap] traversal logs
  int64_t log_cap = 0;
  DBuf far_id, near_id;             // int32 lists (far grouped by degree within a batch)
  DBuf chunks, items, group_first, group_base, batch_chunks, partial, item_lists;
  std::vector<int32_t> h_items, h_chunks, h_group_first, h_group_base, h_batch_chunks, h_lists;
  std::vector<int64_t> h_cnt;       // host copies of the lists: [n_leaves][kDegSlots] counts,
  std::vector<int32_t> h_fid, h_nid;  // far ids (grouped by degree per batch), near ids
  std::vector<int64_t> list_begin;  // per launch: offset into item_lists
  std::vector<int> list_degree;     // per launch: degree (0 = near items)
  int64_t n_items = 0;
  int ob = 0;
  int64_t n_far = 0, n_near = 0, far_inter = 0, near_inter = 0;
  int64_t far_by_degree[kMaxDegree + 1] = {};
  // streams (default priority) on which the per-degree launches run side by
  // side, forked from and joined back to the caller's stream by events
  static constexpr int kStreams = 4;
  hipStream_t streams[kStreams] = {};
  hipEvent_t fork = nullptr, join[kStreams] = {};
  int ensure_streams() {
    if (streams[0]) return TAGI_OK;
    for (int k = 0; k < kStreams; ++k)
      if (hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&join[k], hipEventDisableTiming) != hipSuccess) {
        release_streams();
        return TAGI_E_HIP;
      }
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
      release_streams();
      return TAGI_E_HIP;
    }
    return TAGI_OK;
  }
  void release_streams() {
    for (int k = 0; k < kStreams; ++k) {
      if (streams[k]) (void)hipStreamDestroy(streams[k]);
      if (join[k]) (void)hipEventDestroy(join[k]);
      streams[k] = nullptr;
      join[k] = nullptr;
    }
    if (fork) (void)hipEventDestroy(fork);
    fork = nullptr;
  }
  void release() {
    l1set.release();
    for (DBuf* b : {&l1n, &params, &mb, &cnt, &log, &far_id, &near_id, &chunks, &items, &group_first,
                    &group_base, &batch_chunks, &partial, &item_lists})
      b->release();
    release_streams();
    key.clear();
    n_items = 0;
    log_cap = 0;
  }
};

}  // namespace tagi

struct tagi_tree {
  int device = 0;
  int64_t n = 0;
  int leaf_size = 0;
  // host copy of the nodes (level order) and leaves
  std::vector<tagi::HostNode> nodes;
  std::vector<int32_t> leaves;   // node ids of the leaves, in node order
  int max_level = 0;

  // device: tree-ordered sources
  tagi::DBuf perm;                  // int32 [n]
  tagi::DBuf xs, ys, zs;            // double [n]
  tagi::DBuf leaf_of_pos;           // int32 [n] batch index of each tree position
  // device: nodes
  tagi::DBuf nd_begin, nd_end, nd_first_child, nd_n_child;  // int32 [n_nodes]
  tagi::DBuf nd_geom;               // double [n_nodes][4] centre xyz, radius
  tagi::DBuf nd_box;                // double [n_nodes][6] lo xyz, hi xyz
  tagi::DBuf leaf_node;             // int32 [n_leaves]

  // upward state: tree-ordered values and the proxy charges of the last upward
  int degree = 0;
  int n_orb = 0;
  tagi::DBuf ws;                    // double [n] tree-ordered weights
  tagi::DBuf fs;                    // double [n_orb][n] tree-ordered values
  tagi::DBuf qs;                    // double [n_orb][n] f*w tree-ordered
  tagi::ProxySet px;                // degree `degree`, every cluster with (n+1)^3 < N_S
  tagi::ProxySet lx[tagi::kMaxDegree + 1];  // learned path: per degree, clusters in use
  tagi::LearnedState learned;
  // charges generation: bumped before every upward pass (tagi_upward, its Hermite
  // form, graph capture, the Green step, selector sampling); the learned lists
  // take their features from the charges, so they are rebuilt when it moves
  uint64_t charges_gen = 0;
  uint64_t learned_gen = 0;         // charges generation the learned lists were built from

  // cached interaction lists and compute schedule
  double list_theta = -1.0;
  int list_degree = -1;
  bool list_herm = false;  // lists built with the Hermite size test 8 (n+1)^3 < N_S
  int64_t n_far = 0, n_near = 0;
  int64_t far_inter = 0, near_inter = 0;
  tagi::DBuf far_off, near_off;     // int64 [n_leaves+1]
  tagi::DBuf far_id, near_id;       // int32
  std::vector<int64_t> h_far_off, h_near_off;
  // schedule: chunks of (kind, begin, end) per batch, items, group table
  int64_t n_items = 0;
  int items_orb_block = 0;
  double items_far_w = -1.0;             // far weight the launch order was made for
  std::vector<int32_t> h_order_base;     // chunk-major launch order
  std::vector<int32_t> h_order;          // the order last uploaded (-1: an empty slot)
  struct Run {
    int32_t start, len, chunk;           // waves [start, start+len) of h_order_base
  };
  std::vector<Run> h_runs;               // runs of one chunk's waves
  std::vector<int32_t> h_chunk_cost;     // evaluations per target lane of each chunk
  std::vector<uint8_t> h_chunk_far;      // 1 for far chunks
  int ob_override = 0;              // orbital block set by the caller (0 = automatic)
  int sched_items = 0;              // work items a schedule aims at (0 = kDefaultScheduleItems)
  int kvariant = 0;                 // interaction-kernel launch variant (0 = defaults)
  int items_n_orb = 0;
  tagi::DBuf chunks;                // int4 {kind, e0, e1, cost}
  tagi::DBuf items;                 // int4 {batch, group, oblock, chunk}
  tagi::DBuf item_order;            // int32 launch order (h_order): per batch and orbital
                                    // block, chunk-major (the groups of a chunk adjacent)
  tagi::DBuf group_first_item;      // int32 per (batch, group)
  tagi::DBuf batch_group_base;      // int32 [n_leaves] first (batch, group) index
  tagi::DBuf batch_chunks;          // int2 [n_leaves] {first chunk, n chunks}
  tagi::DBuf partial;               // double partial sums per item
  tagi::DBuf kappa_dev;             // double [n_orb]
  // Green-iteration step: V psi, the convolution, reduction partials
  tagi::DBuf green_f, green_phi, green_part;
  // separate target set of the last tagi_convolve with targets: a tree on the
  // targets (its leaves are the batches; it also holds that call's lists and
  // schedule) and the target values in its order, [n_orb][n_targets]
  tagi_tree* tgt = nullptr;
  tagi::DBuf tgt_fs;

  // phase timing (HIP events on the calls' stream)
  bool timing = false;
  double build_ms = 0.0;
  // upward, lists, interact, combine, and each interaction launch on its own stream
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events[5];
  double phase_ms[5] = {0, 0, 0, 0, 0};
  int64_t interact_launches = 0;
};

// adaptive mesh: cells and the one-dimensional Fejer rule on [-1, 1]
struct tagi_mesh {
  int p = 0;
  std::vector<double> lo, hi;  // [n_cells][3]
  double nodes[tagi::kMeshMaxP + 1] = {};
  double weights[tagi::kMeshMaxP + 1] = {};
};

namespace tagi {

// Work items a compute schedule aims at: each batch's lists are cut into chunks
// of at most (total kernel evaluations per target lane) / items, so the launch
// has about that many waves (more where batches hold several 64-target groups).
constexpr int kDefaultScheduleItems = 16384;
// launch variants of the interaction kernel (tagi_tree_set_kernel_variant)
constexpr int kKernelVariants = 4;
inline int64_t schedule_items(const tagi_tree* t) {
  return t->sched_items > 0 ? t->sched_items : kDefaultScheduleItems;
}

// the interaction lists cached in the batch tree `bt` serve (theta, degree) with
// the size test of the source tree's current proxy charges
inline bool lists_current(const tagi_tree* src, const tagi_tree* bt, double theta, int degree) {
  return bt->list_theta == theta && bt->list_degree == degree && bt->list_herm == src->px.herm;
}
inline bool lists_current(const tagi_tree* t, double theta, int degree) {
  return lists_current(t, t, theta, degree);
}

enum Phase {
  kPhaseUpward = 0,
  kPhaseLists = 1,
  kPhaseInteract = 2,
  kPhaseCombine = 3,
  kLaunchInteract = 4  // one interaction launch, on the stream it runs on
};

// a roctx range over one API call on the calling thread (host time of the
// call; rocprofv3 --marker-trace lists it beside the kernels it launched)
struct CallRange {
  explicit CallRange(const char* name) { roctxRangePush(name); }
  ~CallRange() { roctxRangePop(); }
  CallRange(const CallRange&) = delete;
  CallRange& operator=(const CallRange&) = delete;
};

inline void phase_begin(tagi_tree* t, int ph, hipStream_t s) {
  if (!t->timing) return;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  (void)hipEventRecord(a, s);
  t->events[ph].push_back({a, b});
}

inline void phase_end(tagi_tree* t, int ph, hipStream_t s) {
  if (!t->timing || t->events[ph].empty()) return;
  (void)hipEventRecord(t->events[ph].back().second, s);
}

int build_tree(tagi_tree* t, const double* x, const double* y, const double* z,
               const double* box, hipStream_t s);
int upward(tagi_tree* t, const double* f, const double* w, int n_orb, int degree, hipStream_t s,
           bool herm = false);
// plan (host lists, uploads, buffers) of proxy charges at `degree` for `nodes`
int prepare_proxies(tagi_tree* t, ProxySet& ps, const std::vector<int32_t>& nodes, int degree,
                    int n_orb, hipStream_t s, bool herm = false);
// proxy charges of the planned set from the tree-ordered q = f w and w
int compute_proxies(tagi_tree* t, ProxySet& ps, hipStream_t s);
// Interaction lists of the batches (leaves) of `bt` against the clusters of the
// source tree `src`, and their compute schedule, both kept in `bt`; bt == src
// when the targets are the sources. `root_far` (may be NULL) receives whether
// some batch accepted the root cluster as far.
int ensure_lists(tagi_tree* src, tagi_tree* bt, double theta, int degree, hipStream_t s,
                 bool* root_far = nullptr);
int ensure_schedule(const tagi_tree* src, tagi_tree* bt, int orb_block, hipStream_t s);
int count_far_pairs(tagi_tree* t, double theta, int K, int64_t* far_cnt, int64_t* scratch,
                    hipStream_t s);
inline int ensure_lists(tagi_tree* t, double theta, int degree, hipStream_t s) {
  return ensure_lists(t, t, theta, degree, s);
}
inline int ensure_schedule(tagi_tree* t, int orb_block, hipStream_t s) {
  return ensure_schedule(t, t, orb_block, s);
}
// launch order of the schedule for far evaluations costing far_w near ones
int order_schedule(tagi_tree* t, double far_w, hipStream_t s);
// waves [start, start + len) of a launch list that read the same sources
struct WaveRun {
  int32_t start, len;
  double cost;
};
// the launch order cut into one contiguous piece of equal cost per XCD, each
// padded with empty slots (-1) to a common length; `longest_first` also sorts
// the runs of each piece by descending cost
int balance_runs_per_xcd(std::vector<int32_t>& list, const std::vector<WaveRun>& runs,
                         bool longest_first);
double far_weight(int kernel, int precision, bool herm);
int orbital_block(int kernel, int n_orb, int precision, bool learned = false);
// the tree's orbital block for a kernel: its override if set, else the default
// (`learned`: for tagi_convolve_learned's launches)
int orbital_block_of(const tagi_tree* t, int kernel, int precision, bool learned = false);
// The far and near sums of the batches of `bt` (lists and schedule prepared in
// it) against the source tree `src`, the combine and the scatter to the caller's
// target order; tfs = target values in bt's order, [n_orb][bt->n] (bt == src:
// the source tree's own values).
int convolve(tagi_tree* src, tagi_tree* bt, const double* tfs, int kernel, const double* kappa,
             double alpha, int precision, double* out, hipStream_t s);
inline int convolve(tagi_tree* t, int kernel, const double* kappa, double alpha, int precision,
                    double* out, hipStream_t s) {
  return convolve(t, t, t->fs.as<double>(), kernel, kappa, alpha, precision, out, s);
}
// gathers caller-order values [n_orb][n] into the order of tree t
int gather_values(const tagi_tree* t, const double* f, int n_orb, double* out, hipStream_t s);
int convolve_learned(tagi_tree* t, int kernel, const double* kappa, double alpha,
                     const float* params, const float* norm, const double* tol, double theta_max,
                     double theta_fb, int degree_fb, int precision, double* out, hipStream_t s);
// the learned lists' features come from the charges: forget the cached lists
// once an upward pass has run since they were built
inline void learned_follow_charges(tagi_tree* t) {
  if (t->learned_gen != t->charges_gen) {
    t->learned.key.clear();
    t->learned_gen = t->charges_gen;
  }
}
int mesh_build(const double* lo, const double* hi, int p, double tol, int uniform_levels,
               int max_level, const double* atoms, int n_atoms, int kind, double max_aspect,
               hipStream_t s, tagi_mesh** out);
int mesh_points(const tagi_mesh* m, double* x, double* y, double* z, double* w, hipStream_t s);
int green_step(tagi_tree* t, const double* psi, const double* veff, const double* w, int n_orb,
               double* eps, double theta, int degree, int precision, double* psi_out,
               double* resid, hipStream_t s);
int green_step_learned(tagi_tree* t, const double* psi, const double* veff, const double* w,
                       int n_orb, double* eps, const float* params, const float* norm,
                       const double* tol, double theta_max, double theta_fb, int degree_fb,
                       int precision, double* psi_out, double* resid, hipStream_t s);
int selector_param_count();
// l1 norms of one charge set of a proxy set (set < n_orb: orbital, set == n_orb:
// the weights' charges), written to out[node] for every slot's node
int l1_to_nodes(const ProxySet& ps, int set, float* out, hipStream_t s);
// max |f| over each batch's targets: out[o][leaf]
int leaf_fmax(tagi_tree* t, float* out, hipStream_t s);
int selector_samples(tagi_tree* t, const double* f, const double* w, int kernel, double kappa,
                     double alpha, double theta_max, int64_t max_pairs, float* feat, float* err,
                     int32_t* pair_ids, int64_t* n_out, hipStream_t s);
int selector_grad(const float* params, const float* X, const float* Y, const float* M, int64_t m,
                  float* grads, float* loss, hipStream_t s);
int selector_train(float* params, const float* X, const float* Y, const float* M, int64_t m,
                   const int32_t* order, int epochs, int batch, float lr, float* loss_hist,
                   hipStream_t s);
int direct(const double* sx, const double* sy, const double* sz, const double* sf,
           const double* sw, int64_t ns, const double* tx, const double* ty, const double* tz,
           const double* tf, int64_t nt, int kernel, double kappa, double alpha, double* out,
           hipStream_t s);
// the allocation-free direct sum: its scratch lives in a library-owned device
// array of direct_noalloc_limit() bytes; a call needs direct_noalloc_bytes(ns, nt)
int direct_noalloc(const double* sx, const double* sy, const double* sz, const double* sf,
                   const double* sw, int64_t ns, const double* tx, const double* ty,
                   const double* tz, const double* tf, int64_t nt, int kernel, double kappa,
                   double alpha, double* out, hipStream_t s);
size_t direct_noalloc_bytes(int64_t ns, int64_t nt);
size_t direct_noalloc_limit();

}  // namespace tagi
