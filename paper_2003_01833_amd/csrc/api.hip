// The C ABI declared in include/tagi.h: argument validation, error state, and
// dispatch to the tree, upward, list and interaction stages.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>

#include "internal.hpp"

namespace tagi {

namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

namespace {
std::atomic<size_t> g_held{0};

// TAGI_WORKSPACE_LIMIT in bytes (a K, M or G suffix multiplies by 2^10, 2^20,
// 2^30); 0 when unset, empty or not a number
size_t workspace_limit() {
  const char* v = std::getenv("TAGI_WORKSPACE_LIMIT");
  if (!v || !*v) return 0;
  char* end = nullptr;
  const unsigned long long n = std::strtoull(v, &end, 10);
  if (end == v) return 0;
  int shift = 0;
  if (*end == 'K' || *end == 'k') shift = 10;
  if (*end == 'M' || *end == 'm') shift = 20;
  if (*end == 'G' || *end == 'g') shift = 30;
  return (size_t)n << shift;
}
}  // namespace

int workspace_take(size_t bytes) {
  const size_t lim = workspace_limit();
  const size_t held = g_held.fetch_add(bytes) + bytes;
  if (lim && held > lim) {
    g_held.fetch_sub(bytes);
    set_error("device workspace limit (TAGI_WORKSPACE_LIMIT = %zu bytes): %zu held, %zu more "
              "requested", lim, held - bytes, bytes);
    return TAGI_E_OOM;
  }
  return TAGI_OK;
}

void workspace_give(size_t bytes) { g_held.fetch_sub(bytes); }

int DBuf::ensure(size_t bytes) {
  if (bytes <= cap && p) return TAGI_OK;
  release();
  if (bytes == 0) bytes = 8;
  TAGI_TRY(workspace_take(bytes));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    p = nullptr;
    workspace_give(bytes);
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? TAGI_E_OOM : TAGI_E_HIP;
  }
  cap = bytes;
  return TAGI_OK;
}

void DBuf::release() {
  if (p) {
    (void)hipFree(p);
    workspace_give(cap);
  }
  p = nullptr;
  cap = 0;
}

}  // namespace tagi

using namespace tagi;

#define REQUIRE(cond, ...)         \
  do {                             \
    if (!(cond)) {                 \
      set_error(__VA_ARGS__);      \
      return TAGI_E_ARG;           \
    }                              \
  } while (0)

static bool valid_kernel(int k) { return k >= TAGI_YUKAWA_SS && k <= TAGI_COULOMB; }
static bool is_yukawa(int k) { return k == TAGI_YUKAWA_SS || k == TAGI_YUKAWA; }

// tagi_convolve at a separate target set (arguments validated): the batches are
// the leaves of a tree on the targets (Section 6.1, N_B = N_L), kept in t->tgt
// with that call's lists and schedule.
static int convolve_targets(tagi_tree* t, const tagi_points* tp, int kernel, const double* kappa,
                            double alpha, double theta, int degree, int precision, double* out,
                            hipStream_t s) {
  if (!t->tgt) {
    t->tgt = new (std::nothrow) tagi_tree();
    if (!t->tgt) {
      set_error("tagi_convolve: host allocation failed");
      return TAGI_E_OOM;
    }
  }
  tagi_tree* bt = t->tgt;
  bt->device = t->device;
  bt->n = tp->n;
  bt->leaf_size = t->leaf_size;
  bt->list_theta = -1.0;
  bt->list_degree = -1;
  bt->n_items = 0;
  bt->items_orb_block = 0;
  bt->items_far_w = -1.0;
  phase_begin(t, kPhaseLists, s);
  int st = build_tree(bt, tp->x, tp->y, tp->z, nullptr, s);
  const bool ss = kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS;
  if (st == TAGI_OK && ss) {
    st = t->tgt_fs.ensure((size_t)t->n_orb * tp->n * sizeof(double));
    if (st == TAGI_OK) st = gather_values(bt, tp->f, t->n_orb, t->tgt_fs.as<double>(), s);
  }
  bool root_far = false;
  if (st == TAGI_OK) st = ensure_lists(t, bt, theta, degree, s, &root_far);
  if (st == TAGI_OK && root_far && t->px.h_slot_of[0] < 0) {
    // some batch accepts the root (targets away from the sources' box): add its
    // proxy charges, computed from the last upward pass's tree-ordered values
    std::vector<int32_t> nodes(1, 0);
    nodes.insert(nodes.end(), t->px.nodes.begin(), t->px.nodes.end());
    st = prepare_proxies(t, t->px, nodes, degree, t->n_orb, s, t->px.herm);
    if (st == TAGI_OK) st = compute_proxies(t, t->px, s);
    if (st != TAGI_OK) t->degree = 0;  // the proxy plan is incomplete: upward again
  }
  const int ob = orbital_block_of(t, kernel, precision);
  if (st == TAGI_OK) st = ensure_schedule(t, bt, ob, s);
  phase_end(t, kPhaseLists, s);
  if (st != TAGI_OK) return st;
  TAGI_TRY(order_schedule(bt, far_weight(kernel, precision, t->px.herm), s));
  return convolve(t, bt, ss ? t->tgt_fs.as<double>() : nullptr, kernel, kappa, alpha, precision,
                  out, s);
}

#pragma GCC visibility push(default)
extern "C" {

const char* tagi_last_error(void) { return g_err; }

int tagi_workspace_held(int64_t* bytes) {
  g_err[0] = 0;
  REQUIRE(bytes, "tagi_workspace_held: bytes is NULL");
  *bytes = (int64_t)g_held.load();
  return TAGI_OK;
}

int tagi_tree_build(const double* x, const double* y, const double* z, int64_t n,
                    const double* box, int leaf_size, void* stream, tagi_tree** out) {
  g_err[0] = 0;
  CallRange range_("tagi_tree_build");
  REQUIRE(out, "tagi_tree_build: out is NULL");
  *out = nullptr;
  REQUIRE(x && y && z, "tagi_tree_build: null coordinate array");
  REQUIRE(n >= 1 && n < (int64_t)INT32_MAX, "tagi_tree_build: n = %lld out of range [1, 2^31)",
          (long long)n);
  REQUIRE(leaf_size >= 1, "tagi_tree_build: leaf_size = %d must be >= 1", leaf_size);
  if (box) {
    for (int k = 0; k < 3; ++k)
      REQUIRE(std::isfinite(box[k]) && std::isfinite(box[3 + k]) && box[k] <= box[3 + k],
              "tagi_tree_build: box dimension %d is empty or not finite", k);
  }
  tagi_tree* t = new (std::nothrow) tagi_tree();
  if (!t) {
    set_error("tagi_tree_build: host allocation failed");
    return TAGI_E_OOM;
  }
  (void)hipGetDevice(&t->device);
  t->n = n;
  t->leaf_size = leaf_size;
  const auto t0 = std::chrono::steady_clock::now();
  const int st = build_tree(t, x, y, z, box, (hipStream_t)stream);
  t->build_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st != TAGI_OK) {
    char keep[1024];
    std::memcpy(keep, g_err, sizeof(keep));
    tagi_tree_destroy(t);
    std::memcpy(g_err, keep, sizeof(keep));
    return st;
  }
  *out = t;
  return TAGI_OK;
}

int tagi_upward(tagi_tree* t, const double* f, const double* w, int n_orb, int degree,
                void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_upward");
  REQUIRE(t, "tagi_upward: tree is NULL");
  REQUIRE(f && w, "tagi_upward: null f or w");
  REQUIRE(n_orb >= 1 && n_orb <= kMaxOrb, "tagi_upward: n_orb = %d out of range [1, %d]", n_orb,
          kMaxOrb);
  REQUIRE(degree >= 1 && degree <= kMaxDegree, "tagi_upward: degree = %d out of range [1, %d]",
          degree, kMaxDegree);
  ++t->charges_gen;
  return upward(t, f, w, n_orb, degree, (hipStream_t)stream);
}

int tagi_upward_hermite(tagi_tree* t, const double* f, const double* w, int n_orb, int degree,
                        void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_upward_hermite");
  REQUIRE(t, "tagi_upward_hermite: tree is NULL");
  REQUIRE(f && w, "tagi_upward_hermite: null f or w");
  REQUIRE(n_orb >= 1 && n_orb <= kMaxOrb, "tagi_upward_hermite: n_orb = %d out of range [1, %d]",
          n_orb, kMaxOrb);
  REQUIRE(degree >= 1 && degree <= kMaxHermDegree,
          "tagi_upward_hermite: degree = %d out of range [1, %d]", degree, kMaxHermDegree);
  ++t->charges_gen;
  return upward(t, f, w, n_orb, degree, (hipStream_t)stream, true);
}

int tagi_convolve(tagi_tree* t, const tagi_points* targets, int kernel, const double* kappa,
                  double alpha, double theta, int degree, int precision, double* out,
                  void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_convolve");
  REQUIRE(t, "tagi_convolve: tree is NULL");
  REQUIRE(out || (targets && targets->n == 0), "tagi_convolve: out is NULL");
  REQUIRE(valid_kernel(kernel), "tagi_convolve: unknown kernel %d", kernel);
  REQUIRE(precision == TAGI_FP64 || precision == TAGI_MIXED,
          "tagi_convolve: unknown precision %d", precision);
  REQUIRE(theta >= 0.0 && theta < 1.0, "tagi_convolve: theta = %g out of range [0, 1)", theta);
  REQUIRE(degree >= 1 && degree <= kMaxDegree, "tagi_convolve: degree = %d out of range", degree);
  if (targets) {
    REQUIRE(targets->n >= 0 && targets->n < (int64_t)INT32_MAX,
            "tagi_convolve: targets->n = %lld out of range [0, 2^31)", (long long)targets->n);
    REQUIRE(targets->n == 0 || (targets->x && targets->y && targets->z),
            "tagi_convolve: null target coordinate array");
    REQUIRE(targets->n == 0 || targets->f ||
                !(kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS),
            "tagi_convolve: targets->f is required for the subtracted kernels");
  }
  if (t->degree == 0) {
    set_error("tagi_convolve: tagi_upward has not run on this tree");
    return TAGI_E_STATE;
  }
  if (t->degree != degree) {
    set_error("tagi_convolve: degree %d differs from the upward pass degree %d", degree, t->degree);
    return TAGI_E_STATE;
  }
  if (is_yukawa(kernel)) {
    REQUIRE(kappa, "tagi_convolve: kappa is NULL for a Yukawa kernel");
    for (int o = 0; o < t->n_orb; ++o)
      REQUIRE(std::isfinite(kappa[o]) && kappa[o] > 0.0,
              "tagi_convolve: kappa[%d] = %g must be finite and > 0", o, kappa[o]);
  }
  if (kernel == TAGI_COULOMB_SS)
    REQUIRE(std::isfinite(alpha) && alpha > 0.0, "tagi_convolve: alpha = %g must be > 0", alpha);
  hipStream_t s = (hipStream_t)stream;
  if (targets) {
    if (targets->n == 0) return TAGI_OK;
    return convolve_targets(t, targets, kernel, kappa, alpha, theta, degree, precision, out, s);
  }
  const int ob = orbital_block_of(t, kernel, precision);
  const bool rebuild = !lists_current(t, theta, degree) ||
                       !(t->items_orb_block == ob && t->items_n_orb == t->n_orb && t->n_items > 0);
  if (rebuild) {
    phase_begin(t, kPhaseLists, s);
    int st = ensure_lists(t, theta, degree, s);
    if (st == TAGI_OK) st = ensure_schedule(t, ob, s);
    phase_end(t, kPhaseLists, s);
    if (st != TAGI_OK) return st;
  }
  TAGI_TRY(order_schedule(t, far_weight(kernel, precision, t->px.herm), s));
  return convolve(t, kernel, kappa, alpha, precision, out, s);
}

int tagi_direct(const double* sx, const double* sy, const double* sz, const double* sf,
                const double* sw, int64_t ns, const double* tx, const double* ty,
                const double* tz, const double* tf, int64_t nt, int kernel, double kappa,
                double alpha, double* out, void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_direct");
  REQUIRE(valid_kernel(kernel), "tagi_direct: unknown kernel %d", kernel);
  REQUIRE(sx && sy && sz && sf && sw, "tagi_direct: null source array");
  REQUIRE(tx && ty && tz && out, "tagi_direct: null target or output array");
  REQUIRE(ns >= 1 && ns < (int64_t)INT32_MAX, "tagi_direct: ns = %lld out of range", (long long)ns);
  REQUIRE(nt >= 1 && nt < (int64_t)INT32_MAX, "tagi_direct: nt = %lld out of range", (long long)nt);
  const bool ss = kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS;
  REQUIRE(!ss || tf, "tagi_direct: target values tf are required for subtracted kernels");
  if (is_yukawa(kernel))
    REQUIRE(std::isfinite(kappa) && kappa > 0.0, "tagi_direct: kappa = %g must be > 0", kappa);
  if (kernel == TAGI_COULOMB_SS)
    REQUIRE(std::isfinite(alpha) && alpha > 0.0, "tagi_direct: alpha = %g must be > 0", alpha);
  return direct(sx, sy, sz, sf, sw, ns, tx, ty, tz, tf, nt, kernel, kappa, alpha, out,
                (hipStream_t)stream);
}

int tagi_direct_noalloc(const double* sx, const double* sy, const double* sz, const double* sf,
                        const double* sw, int64_t ns, const double* tx, const double* ty,
                        const double* tz, const double* tf, int64_t nt, int kernel, double kappa,
                        double alpha, double* out, void* stream) {
  g_err[0] = 0;
  REQUIRE(valid_kernel(kernel), "tagi_direct_noalloc: unknown kernel %d", kernel);
  REQUIRE(sx && sy && sz && sf && sw, "tagi_direct_noalloc: null source array");
  REQUIRE(tx && ty && tz && out, "tagi_direct_noalloc: null target or output array");
  REQUIRE(ns >= 1 && ns < (int64_t)INT32_MAX, "tagi_direct_noalloc: ns = %lld out of range",
          (long long)ns);
  REQUIRE(nt >= 1 && nt < (int64_t)INT32_MAX, "tagi_direct_noalloc: nt = %lld out of range",
          (long long)nt);
  const bool ss = kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS;
  REQUIRE(!ss || tf, "tagi_direct_noalloc: target values tf are required for subtracted kernels");
  if (is_yukawa(kernel))
    REQUIRE(std::isfinite(kappa) && kappa > 0.0, "tagi_direct_noalloc: kappa = %g must be > 0",
            kappa);
  if (kernel == TAGI_COULOMB_SS)
    REQUIRE(std::isfinite(alpha) && alpha > 0.0, "tagi_direct_noalloc: alpha = %g must be > 0",
            alpha);
  return direct_noalloc(sx, sy, sz, sf, sw, ns, tx, ty, tz, tf, nt, kernel, kappa, alpha, out,
                        (hipStream_t)stream);
}

int tagi_tree_stats(const tagi_tree* t, tagi_stats* o) {
  g_err[0] = 0;
  REQUIRE(t && o, "tagi_tree_stats: null argument");
  std::memset(o, 0, sizeof(*o));
  o->n_points = t->n;
  o->n_nodes = (int32_t)t->nodes.size();
  o->n_leaves = (int32_t)t->leaves.size();
  o->max_level = t->max_level;
  o->leaf_size = t->leaf_size;
  o->degree = t->degree;
  o->n_orb = t->n_orb;
  o->n_approx = t->px.n_approx;
  o->theta = t->list_degree >= 0 ? t->list_theta : -1.0;
  o->n_far_pairs = t->list_degree >= 0 ? t->n_far : 0;
  o->n_near_pairs = t->list_degree >= 0 ? t->n_near : 0;
  o->far_interactions = t->list_degree >= 0 ? t->far_inter : 0;
  o->near_interactions = t->list_degree >= 0 ? t->near_inter : 0;
  o->n_work_items = t->n_items;
  for (int32_t c : t->px.nodes) o->upward_points += t->nodes[c].end - t->nodes[c].begin;
  return TAGI_OK;
}

int tagi_tree_export(const tagi_tree* t, int32_t* perm, int32_t* begin, int32_t* end,
                     int32_t* parent, int32_t* level, int32_t* n_child, double* lo, double* hi,
                     void* stream) {
  g_err[0] = 0;
  REQUIRE(t, "tagi_tree_export: tree is NULL");
  if (perm) {
    TAGI_HIP(hipMemcpyAsync(perm, t->perm.p, t->n * sizeof(int32_t), hipMemcpyDeviceToHost,
                            (hipStream_t)stream));
    TAGI_HIP(hipStreamSynchronize((hipStream_t)stream));
  }
  for (size_t c = 0; c < t->nodes.size(); ++c) {
    const HostNode& q = t->nodes[c];
    if (begin) begin[c] = q.begin;
    if (end) end[c] = q.end;
    if (parent) parent[c] = q.parent;
    if (level) level[c] = q.level;
    if (n_child) n_child[c] = q.n_child;
    for (int k = 0; k < 3; ++k) {
      if (lo) lo[c * 3 + k] = q.lo[k];
      if (hi) hi[c * 3 + k] = q.hi[k];
    }
  }
  return TAGI_OK;
}

int tagi_lists_export(tagi_tree* t, double theta, int degree, int64_t* far_off, int32_t* far_id,
                      int64_t* near_off, int32_t* near_id, int64_t* n_far, int64_t* n_near,
                      void* stream) {
  g_err[0] = 0;
  REQUIRE(t, "tagi_lists_export: tree is NULL");
  REQUIRE(theta >= 0.0 && theta < 1.0, "tagi_lists_export: theta out of range");
  REQUIRE(degree >= 1 && degree <= kMaxDegree, "tagi_lists_export: degree out of range");
  hipStream_t s = (hipStream_t)stream;
  int st = ensure_lists(t, theta, degree, s);
  if (st != TAGI_OK) return st;
  const size_t nl1 = t->leaves.size() + 1;
  if (n_far) *n_far = t->n_far;
  if (n_near) *n_near = t->n_near;
  if (far_off) std::memcpy(far_off, t->h_far_off.data(), nl1 * sizeof(int64_t));
  if (near_off) std::memcpy(near_off, t->h_near_off.data(), nl1 * sizeof(int64_t));
  if (far_id && t->n_far)
    TAGI_HIP(hipMemcpyAsync(far_id, t->far_id.p, t->n_far * 4, hipMemcpyDeviceToHost, s));
  if (near_id && t->n_near)
    TAGI_HIP(hipMemcpyAsync(near_id, t->near_id.p, t->n_near * 4, hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  return TAGI_OK;
}

int tagi_upward_export(const tagi_tree* t, int32_t* cluster, double* nodes, double* qhat,
                       double* what, void* stream) {
  g_err[0] = 0;
  REQUIRE(t, "tagi_upward_export: tree is NULL");
  if (t->degree == 0) {
    set_error("tagi_upward_export: tagi_upward has not run on this tree");
    return TAGI_E_STATE;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t na = t->px.n_approx, np1 = t->degree + 1;
  const size_t K = (t->px.herm ? kHermPatterns : 1) * np1 * np1 * np1;
  if (cluster && na) std::memcpy(cluster, t->px.nodes.data(), na * 4);
  if (nodes && na)
    TAGI_HIP(hipMemcpyAsync(nodes, t->px.pnodes.p, na * 3 * np1 * 8, hipMemcpyDeviceToHost, s));
  if (qhat && na)
    TAGI_HIP(hipMemcpyAsync(qhat, t->px.qhat.p, (size_t)t->n_orb * na * K * 8, hipMemcpyDeviceToHost, s));
  if (what && na)
    TAGI_HIP(hipMemcpyAsync(what, t->px.what.p, na * K * 8, hipMemcpyDeviceToHost, s));
  TAGI_HIP(hipStreamSynchronize(s));
  return TAGI_OK;
}

}  // extern "C"

struct tagi_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  tagi_tree* tree = nullptr;  // every replay runs an upward pass on it
};

extern "C" {

int tagi_graph_create(tagi_tree* t, const double* f, const double* w, int n_orb, int degree,
                      int kernel, const double* kappa, double alpha, double theta, int precision,
                      double* out, void* stream, tagi_graph** graph) {
  g_err[0] = 0;
  CallRange range_("tagi_graph_create");
  REQUIRE(graph, "tagi_graph_create: graph is NULL");
  *graph = nullptr;
  hipStream_t s = (hipStream_t)stream;
  int st = tagi_upward(t, f, w, n_orb, degree, stream);
  if (st == TAGI_OK)
    st = tagi_convolve(t, nullptr, kernel, kappa, alpha, theta, degree, precision, out, stream);
  if (st != TAGI_OK) return st;
  TAGI_HIP(hipStreamSynchronize(s));
  hipStream_t cs;
  TAGI_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  tagi_graph* g = new (std::nothrow) tagi_graph();
  if (!g) {
    (void)hipStreamDestroy(cs);
    set_error("tagi_graph_create: host allocation failed");
    return TAGI_E_OOM;
  }
  const bool timing = t->timing;
  t->timing = false;  // no event records inside the capture
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    ++t->charges_gen;
    st = upward(t, f, w, n_orb, degree, cs);
    if (st == TAGI_OK) st = convolve(t, kernel, kappa, alpha, precision, out, cs);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &gr);
    if (e2 != hipSuccess && st == TAGI_OK) {
      set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e2));
      st = TAGI_E_HIP;
    }
    g->graph = gr;
  } else {
    set_error("hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    st = TAGI_E_HIP;
  }
  t->timing = timing;
  if (st == TAGI_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
      st = TAGI_E_HIP;
    }
  }
  (void)hipStreamDestroy(cs);
  if (st != TAGI_OK) {
    char keep[1024];
    std::memcpy(keep, g_err, sizeof(keep));
    tagi_graph_destroy(g);
    std::memcpy(g_err, keep, sizeof(keep));
    return st;
  }
  g->tree = t;
  *graph = g;
  return TAGI_OK;
}

int tagi_convolve_learned(tagi_tree* t, int kernel, const double* kappa, double alpha,
                          const float* params, const float* norm, const double* tol,
                          double theta_max, double theta_fb, int degree_fb, int precision,
                          double* out, void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_convolve_learned");
  REQUIRE(t && params && norm && out && tol, "tagi_convolve_learned: null argument");
  REQUIRE(valid_kernel(kernel), "tagi_convolve_learned: unknown kernel %d", kernel);
  REQUIRE(kappa || !is_yukawa(kernel), "tagi_convolve_learned: kappa is NULL for a Yukawa kernel");
  if (kernel == TAGI_COULOMB_SS)
    REQUIRE(std::isfinite(alpha) && alpha > 0.0, "tagi_convolve_learned: alpha = %g must be > 0",
            alpha);
  REQUIRE(precision == TAGI_FP64 || precision == TAGI_MIXED, "tagi_convolve_learned: precision");
  REQUIRE(theta_max > 0.0 && theta_max < 1.0, "tagi_convolve_learned: theta_max out of (0, 1)");
  REQUIRE(theta_fb > 0.0 && theta_fb < 1.0, "tagi_convolve_learned: theta_fb out of (0, 1)");
  REQUIRE(degree_fb >= 4 && degree_fb <= 12, "tagi_convolve_learned: degree_fb out of [4, 12]");
  if (t->degree == 0) {
    set_error("tagi_convolve_learned: tagi_upward has not run on this tree");
    return TAGI_E_STATE;
  }
  for (int o = 0; o < t->n_orb; ++o) {
    REQUIRE(std::isfinite(tol[o]) && tol[o] > 0.0,
            "tagi_convolve_learned: tol[%d] = %g must be finite and > 0", o, tol[o]);
    if (is_yukawa(kernel))
      REQUIRE(std::isfinite(kappa[o]) && kappa[o] > 0.0,
              "tagi_convolve_learned: kappa[%d] = %g must be finite and > 0", o, kappa[o]);
  }
  for (int k = 0; k < selector_param_count(); ++k)
    REQUIRE(std::isfinite(params[k]), "tagi_convolve_learned: params[%d] not finite", k);
  learned_follow_charges(t);
  return convolve_learned(t, kernel, kappa, alpha, params, norm, tol, theta_max, theta_fb,
                          degree_fb, precision, out, (hipStream_t)stream);
}

int tagi_learned_stats(const tagi_tree* t, int64_t* o) {
  g_err[0] = 0;
  REQUIRE(t && o, "tagi_learned_stats: null argument");
  const LearnedState& S = t->learned;
  o[0] = S.n_far;
  o[1] = S.n_near;
  o[2] = S.far_inter;
  o[3] = S.near_inter;
  for (int d = 0; d <= kMaxDegree && d < 13; ++d) o[4 + d] = S.far_by_degree[d];
  return TAGI_OK;
}

int tagi_learned_lists_export(const tagi_tree* t, int64_t* far_off, int32_t* far_id,
                              int32_t* far_degree, int64_t* near_off, int32_t* near_id) {
  g_err[0] = 0;
  REQUIRE(t && far_off && near_off, "tagi_learned_lists_export: null argument");
  const LearnedState& S = t->learned;
  if (S.key.empty()) {
    set_error("tagi_learned_lists_export: no learned lists on this tree");
    return TAGI_E_STATE;
  }
  REQUIRE((far_id && far_degree) || S.n_far == 0, "tagi_learned_lists_export: null far arrays");
  REQUIRE(near_id || S.n_near == 0, "tagi_learned_lists_export: null near array");
  const int nl = (int)t->leaves.size();
  constexpr int kDegMin = kLearnDegMin, kNDeg = kLearnDegMax - kLearnDegMin + 1;
  constexpr int kSlots = kNDeg + 1;
  int64_t f = 0, nn = 0;
  for (int b = 0; b < nl; ++b) {
    far_off[b] = f;
    near_off[b] = nn;
    for (int k = 0; k < kNDeg; ++k)
      for (int64_t e = 0; e < S.h_cnt[(size_t)b * kSlots + k]; ++e, ++f) {
        far_id[f] = S.h_fid[f];
        far_degree[f] = kDegMin + k;
      }
    for (int64_t e = 0; e < S.h_cnt[(size_t)b * kSlots + kNDeg]; ++e, ++nn) near_id[nn] = S.h_nid[nn];
  }
  far_off[nl] = f;
  near_off[nl] = nn;
  return TAGI_OK;
}

int tagi_selector_param_count(void) { return selector_param_count(); }

int tagi_selector_samples(tagi_tree* t, const double* f, const double* w, int kernel,
                          double kappa, double alpha, double theta_max, int64_t max_pairs,
                          float* features, float* errors, int32_t* pair_ids, int64_t* n,
                          void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_selector_samples");
  REQUIRE(t && f && w && features && errors && n, "tagi_selector_samples: null argument");
  REQUIRE(kernel == TAGI_YUKAWA_SS || kernel == TAGI_COULOMB_SS,
          "tagi_selector_samples: kernel must be TAGI_YUKAWA_SS or TAGI_COULOMB_SS");
  if (kernel == TAGI_YUKAWA_SS)
    REQUIRE(std::isfinite(kappa) && kappa > 0.0, "tagi_selector_samples: kappa must be > 0");
  else
    REQUIRE(std::isfinite(alpha) && alpha > 0.0, "tagi_selector_samples: alpha must be > 0");
  REQUIRE(theta_max > 0.0 && theta_max < 1.0, "tagi_selector_samples: theta_max out of (0, 1)");
  REQUIRE(max_pairs >= 1 && max_pairs < (int64_t)INT32_MAX, "tagi_selector_samples: bad max_pairs");
  *n = 0;
  return selector_samples(t, f, w, kernel, kappa, alpha, theta_max, max_pairs, features, errors,
                          pair_ids, n, (hipStream_t)stream);
}

int tagi_selector_grad(const float* params, const float* X, const float* Y, const float* M,
                       int64_t m, float* grads, float* loss, void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_selector_grad");
  REQUIRE(params && X && Y && M && grads, "tagi_selector_grad: null argument");
  REQUIRE(m >= 1 && m < (int64_t)INT32_MAX, "tagi_selector_grad: bad m");
  return selector_grad(params, X, Y, M, m, grads, loss, (hipStream_t)stream);
}

int tagi_selector_train(float* params, const float* X, const float* Y, const float* M, int64_t m,
                        const int32_t* order, int epochs, int batch, float lr, float* loss_hist,
                        void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_selector_train");
  REQUIRE(params && X && Y && M && order, "tagi_selector_train: null argument");
  REQUIRE(m >= 1 && m < (int64_t)INT32_MAX, "tagi_selector_train: bad m");
  REQUIRE(batch >= 1 && epochs >= 0 && lr > 0.0f, "tagi_selector_train: bad batch/epochs/lr");
  for (int64_t r = 0; r < m; ++r)
    REQUIRE(order[r] >= 0 && order[r] < m, "tagi_selector_train: order[%lld] out of range",
            (long long)r);
  return selector_train(params, X, Y, M, m, order, epochs, batch, lr, loss_hist,
                        (hipStream_t)stream);
}

int tagi_graph_launch(tagi_graph* g, void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_graph_launch");
  REQUIRE(g && g->exec, "tagi_graph_launch: graph is NULL");
  TAGI_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  ++g->tree->charges_gen;
  return TAGI_OK;
}

int tagi_graph_destroy(tagi_graph* g) {
  if (!g) return TAGI_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return TAGI_OK;
}

static void drop_events(tagi_tree* t) {
  for (auto& v : t->events) {
    for (auto& e : v) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    v.clear();
  }
}

int tagi_tree_set_timing(tagi_tree* t, int enable) {
  g_err[0] = 0;
  REQUIRE(t, "tagi_tree_set_timing: tree is NULL");
  (void)hipDeviceSynchronize();
  drop_events(t);
  for (double& v : t->phase_ms) v = 0.0;
  t->interact_launches = 0;
  t->timing = enable != 0;
  return TAGI_OK;
}

int tagi_tree_timing(tagi_tree* t, tagi_timing* o) {
  g_err[0] = 0;
  REQUIRE(t && o, "tagi_tree_timing: null argument");
  for (int ph = 0; ph < 5; ++ph) {
    for (auto& e : t->events[ph]) {
      TAGI_HIP(hipEventSynchronize(e.second));
      float ms = 0.f;
      // a phase that ended in an error has no end event: it adds nothing
      if (hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      t->phase_ms[ph] += ms;
    }
  }
  drop_events(t);
  o->build_ms = t->build_ms;
  o->upward_ms = t->phase_ms[kPhaseUpward];
  o->lists_ms = t->phase_ms[kPhaseLists];
  o->interact_ms = t->phase_ms[kPhaseInteract];
  o->combine_ms = t->phase_ms[kPhaseCombine];
  o->interact_launches = t->interact_launches;
  o->interact_kernel_ms = t->phase_ms[kLaunchInteract];
  return TAGI_OK;
}

int tagi_green_step(tagi_tree* t, const double* psi, const double* veff, const double* w,
                    int n_orb, double* eps, double theta, int degree, int precision,
                    double* psi_out, double* resid, void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_green_step");
  REQUIRE(t, "tagi_green_step: tree is NULL");
  REQUIRE(psi && veff && w && psi_out && eps, "tagi_green_step: null argument");
  REQUIRE(psi_out != psi, "tagi_green_step: psi_out must not alias psi");
  REQUIRE(n_orb >= 1 && n_orb <= kMaxOrb, "tagi_green_step: n_orb = %d out of range [1, %d]",
          n_orb, kMaxOrb);
  for (int o = 0; o < n_orb; ++o)
    REQUIRE(std::isfinite(eps[o]) && eps[o] < 0.0,
            "tagi_green_step: eps[%d] = %g must be finite and < 0", o, eps[o]);
  REQUIRE(theta >= 0.0 && theta < 1.0, "tagi_green_step: theta = %g out of range [0, 1)", theta);
  REQUIRE(degree >= 1 && degree <= kMaxDegree, "tagi_green_step: degree = %d out of range",
          degree);
  REQUIRE(precision == TAGI_FP64 || precision == TAGI_MIXED,
          "tagi_green_step: unknown precision %d", precision);
  return green_step(t, psi, veff, w, n_orb, eps, theta, degree, precision, psi_out, resid,
                    (hipStream_t)stream);
}

int tagi_green_step_learned(tagi_tree* t, const double* psi, const double* veff, const double* w,
                            int n_orb, double* eps, const float* params, const float* norm,
                            const double* tol, double theta_max, double theta_fb, int degree_fb,
                            int precision, double* psi_out, double* resid, void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_green_step_learned");
  REQUIRE(t, "tagi_green_step_learned: tree is NULL");
  REQUIRE(psi && veff && w && psi_out && eps && params && norm && tol,
          "tagi_green_step_learned: null argument");
  REQUIRE(psi_out != psi, "tagi_green_step_learned: psi_out must not alias psi");
  REQUIRE(n_orb >= 1 && n_orb <= kMaxOrb,
          "tagi_green_step_learned: n_orb = %d out of range [1, %d]", n_orb, kMaxOrb);
  for (int o = 0; o < n_orb; ++o) {
    REQUIRE(std::isfinite(eps[o]) && eps[o] < 0.0,
            "tagi_green_step_learned: eps[%d] = %g must be finite and < 0", o, eps[o]);
    REQUIRE(std::isfinite(tol[o]) && tol[o] > 0.0,
            "tagi_green_step_learned: tol[%d] = %g must be finite and > 0", o, tol[o]);
  }
  REQUIRE(theta_max > 0.0 && theta_max < 1.0, "tagi_green_step_learned: theta_max out of (0, 1)");
  REQUIRE(theta_fb > 0.0 && theta_fb < 1.0, "tagi_green_step_learned: theta_fb out of (0, 1)");
  REQUIRE(degree_fb >= 4 && degree_fb <= 12,
          "tagi_green_step_learned: degree_fb out of [4, 12]");
  REQUIRE(precision == TAGI_FP64 || precision == TAGI_MIXED,
          "tagi_green_step_learned: unknown precision %d", precision);
  for (int k = 0; k < selector_param_count(); ++k)
    REQUIRE(std::isfinite(params[k]), "tagi_green_step_learned: params[%d] not finite", k);
  return green_step_learned(t, psi, veff, w, n_orb, eps, params, norm, tol, theta_max, theta_fb,
                            degree_fb, precision, psi_out, resid, (hipStream_t)stream);
}

int tagi_mesh_build(const double* lo3, const double* hi3, int p, double tol_m,
                    int uniform_levels, int max_level, const double* atoms, int n_atoms,
                    int test_fn, double max_aspect, void* stream, tagi_mesh** out) {
  g_err[0] = 0;
  CallRange range_("tagi_mesh_build");
  REQUIRE(out, "tagi_mesh_build: out is NULL");
  *out = nullptr;
  REQUIRE(lo3 && hi3, "tagi_mesh_build: null domain");
  for (int d = 0; d < 3; ++d)
    REQUIRE(std::isfinite(lo3[d]) && std::isfinite(hi3[d]) && lo3[d] < hi3[d],
            "tagi_mesh_build: domain dimension %d is empty or not finite", d);
  REQUIRE(p >= 1 && p <= kMeshMaxP, "tagi_mesh_build: p = %d out of range [1, %d]", p, kMeshMaxP);
  REQUIRE(std::isfinite(tol_m) && tol_m > 0.0, "tagi_mesh_build: tol_m = %g must be > 0", tol_m);
  REQUIRE(uniform_levels >= 0 && uniform_levels <= 6,
          "tagi_mesh_build: uniform_levels = %d out of range [0, 6]", uniform_levels);
  REQUIRE(max_level >= uniform_levels && max_level <= 40,
          "tagi_mesh_build: max_level = %d out of range [uniform_levels, 40]", max_level);
  REQUIRE(n_atoms >= 0 && n_atoms <= 64, "tagi_mesh_build: n_atoms = %d out of range [0, 64]",
          n_atoms);
  REQUIRE(n_atoms == 0 || atoms, "tagi_mesh_build: atoms is NULL");
  for (int a = 0; a < n_atoms; ++a)
    for (int k = 0; k < 4; ++k)
      REQUIRE(std::isfinite(atoms[4 * a + k]), "tagi_mesh_build: atom %d is not finite", a);
  REQUIRE(test_fn == TAGI_TEST_DENSITY || test_fn == TAGI_TEST_ROOT_DENSITY_VEXT,
          "tagi_mesh_build: unknown test function %d", test_fn);
  REQUIRE(max_aspect >= 1.0, "tagi_mesh_build: max_aspect = %g must be >= 1", max_aspect);
  tagi_mesh* m = nullptr;
  const int st = mesh_build(lo3, hi3, p, tol_m, uniform_levels, max_level, atoms, n_atoms,
                            test_fn, max_aspect, (hipStream_t)stream, &m);
  if (st != TAGI_OK) return st;
  const int64_t q = p + 1;
  if ((int64_t)(m->lo.size() / 3) * q * q * q >= (int64_t)INT32_MAX) {
    delete m;
    set_error("tagi_mesh_build: the mesh has 2^31 points or more");
    return TAGI_E_UNSUPPORTED;
  }
  *out = m;
  return TAGI_OK;
}

int tagi_mesh_info(const tagi_mesh* m, int64_t* n_cells, int64_t* n_points) {
  g_err[0] = 0;
  REQUIRE(m && n_cells && n_points, "tagi_mesh_info: null argument");
  const int64_t q = m->p + 1;
  *n_cells = (int64_t)m->lo.size() / 3;
  *n_points = *n_cells * q * q * q;
  return TAGI_OK;
}

int tagi_mesh_cells(const tagi_mesh* m, double* lo, double* hi) {
  g_err[0] = 0;
  REQUIRE(m, "tagi_mesh_cells: mesh is NULL");
  if (lo) std::memcpy(lo, m->lo.data(), m->lo.size() * sizeof(double));
  if (hi) std::memcpy(hi, m->hi.data(), m->hi.size() * sizeof(double));
  return TAGI_OK;
}

int tagi_mesh_points(const tagi_mesh* m, double* x, double* y, double* z, double* w,
                     void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_mesh_points");
  REQUIRE(m && x && y && z && w, "tagi_mesh_points: null argument");
  return mesh_points(m, x, y, z, w, (hipStream_t)stream);
}

int tagi_mesh_destroy(tagi_mesh* m) {
  delete m;
  return TAGI_OK;
}

int tagi_tree_set_schedule_items(tagi_tree* t, int items) {
  g_err[0] = 0;
  REQUIRE(t, "tagi_tree_set_schedule_items: tree is NULL");
  REQUIRE(items == 0 || (items >= 256 && items <= (1 << 22)),
          "tagi_tree_set_schedule_items: items = %d must be 0 or in [256, 2^22]", items);
  if (schedule_items(t) != (items > 0 ? items : kDefaultScheduleItems)) {
    t->n_items = 0;  // the next convolution rebuilds the schedule
    t->items_orb_block = 0;
  }
  t->sched_items = items;
  return TAGI_OK;
}

int tagi_tree_set_kernel_variant(tagi_tree* t, int variant) {
  g_err[0] = 0;
  REQUIRE(t, "tagi_tree_set_kernel_variant: tree is NULL");
  REQUIRE(variant >= 0 && variant < kKernelVariants,
          "tagi_tree_set_kernel_variant: variant = %d out of range [0, %d)", variant,
          kKernelVariants);
  t->kvariant = variant;
  return TAGI_OK;
}

int tagi_tree_set_orbital_block(tagi_tree* t, int ob) {
  g_err[0] = 0;
  REQUIRE(t, "tagi_tree_set_orbital_block: tree is NULL");
  REQUIRE(ob == 0 || ob == 1 || ob == 2 || ob == 4 || ob == 8,
          "tagi_tree_set_orbital_block: ob = %d must be 0, 1, 2, 4 or 8", ob);
  t->ob_override = ob;
  return TAGI_OK;
}

}  // extern "C"

// Candidate arguments shared by the autotuners, checked before any work.
static int autotune_check(const char* who, const double* x, const double* y, const double* z,
                          const double* w, const double* f, int64_t n, int n_orb,
                          const int* leaf_sizes, int n_leaf, const int* obs, int n_ob,
                          const int* items, int n_items, const int* variants, int n_var,
                          int reps, const int* best) {
  REQUIRE(x && y && z && w && f, "%s: null input array", who);
  REQUIRE(leaf_sizes && n_leaf >= 1, "%s: no leaf size candidates", who);
  REQUIRE(obs && n_ob >= 1, "%s: no orbital block candidates", who);
  REQUIRE(items && n_items >= 1, "%s: no schedule item candidates", who);
  REQUIRE(variants && n_var >= 1, "%s: no kernel variant candidates", who);
  for (int i = 0; i < n_var; ++i)
    REQUIRE(variants[i] >= 0 && variants[i] < kKernelVariants,
            "%s: variants[%d] = %d out of range [0, %d)", who, i, variants[i], kKernelVariants);
  for (int i = 0; i < n_items; ++i)
    REQUIRE(items[i] == 0 || (items[i] >= 256 && items[i] <= (1 << 22)),
            "%s: items[%d] = %d must be 0 or in [256, 2^22]", who, i, items[i]);
  REQUIRE(best, "%s: best is NULL", who);
  REQUIRE(reps >= 1 && reps <= 1000, "%s: reps = %d out of range [1, 1000]", who, reps);
  REQUIRE(n >= 1 && n < (int64_t)INT32_MAX, "%s: n = %lld out of range", who, (long long)n);
  REQUIRE(n_orb >= 1 && n_orb <= kMaxOrb, "%s: n_orb = %d out of range", who, n_orb);
  for (int i = 0; i < n_leaf; ++i)
    REQUIRE(leaf_sizes[i] >= 1, "%s: leaf_sizes[%d] = %d must be >= 1", who, i, leaf_sizes[i]);
  for (int i = 0; i < n_ob; ++i)
    REQUIRE(obs[i] == 0 || obs[i] == 1 || obs[i] == 2 || obs[i] == 4 || obs[i] == 8,
            "%s: obs[%d] = %d must be 0, 1, 2, 4 or 8", who, i, obs[i]);
  return TAGI_OK;
}

// The timing loop shared by the autotuners: for every leaf size a tree, and on
// it for every (orbital block, schedule items, launch variant) one untimed
// step and `reps` timed ones of `step` (which writes its result to `out`).
static int autotune_loop(const char* who, const double* x, const double* y, const double* z,
                         int64_t n, const double* box, int n_orb, const int* leaf_sizes,
                         int n_leaf, const int* obs, int n_ob, const int* items, int n_items,
                         const int* variants, int n_var, int reps, int* best, double* times,
                         void* stream, const std::function<int(tagi_tree*, double*)>& step) {
  hipStream_t s = (hipStream_t)stream;
  StreamScratch scratch(s);
  double* out = nullptr;
  TAGI_TRY(scratch.alloc(&out, (size_t)n_orb * n));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = TAGI_OK;
  double best_ms = INFINITY;
  best[0] = best[1] = best[2] = best[3] = 0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("%s: hipEventCreate failed", who);
    st = TAGI_E_HIP;
  }
  for (int li = 0; li < n_leaf && st == TAGI_OK; ++li) {
    tagi_tree* t = nullptr;
    st = tagi_tree_build(x, y, z, n, box, leaf_sizes[li], stream, &t);
    for (int ci = 0; ci < n_ob * n_items * n_var && st == TAGI_OK; ++ci) {
      const int oi = ci / (n_items * n_var), ii = ci / n_var % n_items, vi = ci % n_var;
      t->ob_override = obs[oi];
      st = tagi_tree_set_schedule_items(t, items[ii]);
      if (st != TAGI_OK) break;
      t->kvariant = variants[vi];
      st = step(t, out);
      if (st != TAGI_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) st = TAGI_E_HIP;
      for (int r = 0; r < reps && st == TAGI_OK; ++r) st = step(t, out);
      if (st != TAGI_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        set_error("%s: event timing failed", who);
        st = TAGI_E_HIP;
        break;
      }
      const double per = (double)ms / reps;
      if (times) times[(((size_t)li * n_ob + oi) * n_items + ii) * n_var + vi] = per;
      if (per < best_ms) {
        best_ms = per;
        best[0] = leaf_sizes[li];
        best[1] = obs[oi];
        best[2] = items[ii];
        best[3] = variants[vi];
      }
    }
    if (t) {
      char keep[1024];
      std::memcpy(keep, g_err, sizeof(keep));
      tagi_tree_destroy(t);
      std::memcpy(g_err, keep, sizeof(keep));
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  return st;
}

extern "C" {

int tagi_autotune(const double* x, const double* y, const double* z, const double* w, int64_t n,
                  const double* box, const double* f, int n_orb, int kernel, const double* kappa,
                  double alpha, double theta, int degree, int precision, const int* leaf_sizes,
                  int n_leaf, const int* obs, int n_ob, const int* items, int n_items,
                  const int* variants, int n_var, int reps, int* best, double* times,
                  void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_autotune");
  TAGI_TRY(autotune_check("tagi_autotune", x, y, z, w, f, n, n_orb, leaf_sizes, n_leaf, obs,
                          n_ob, items, n_items, variants, n_var, reps, best));
  return autotune_loop("tagi_autotune", x, y, z, n, box, n_orb, leaf_sizes, n_leaf, obs, n_ob,
                       items, n_items, variants, n_var, reps, best, times, stream,
                       [&](tagi_tree* t, double* out) {
                         int r = tagi_upward(t, f, w, n_orb, degree, stream);
                         if (r == TAGI_OK)
                           r = tagi_convolve(t, nullptr, kernel, kappa, alpha, theta, degree,
                                             precision, out, stream);
                         return r;
                       });
}

int tagi_autotune_learned(const double* x, const double* y, const double* z, const double* w,
                          int64_t n, const double* box, const double* f, int n_orb, int kernel,
                          const double* kappa, double alpha, const float* params,
                          const float* norm, const double* tol, double theta_max,
                          double theta_fb, int degree_fb, int precision, const int* leaf_sizes,
                          int n_leaf, const int* obs, int n_ob, const int* items, int n_items,
                          const int* variants, int n_var, int reps, int* best, double* times,
                          void* stream) {
  g_err[0] = 0;
  CallRange range_("tagi_autotune_learned");
  REQUIRE(params && norm && tol, "tagi_autotune_learned: null selector argument");
  TAGI_TRY(autotune_check("tagi_autotune_learned", x, y, z, w, f, n, n_orb, leaf_sizes, n_leaf,
                          obs, n_ob, items, n_items, variants, n_var, reps, best));
  // each step stages new charges, so the learned lists are rebuilt every time,
  // as in a Green iteration whose kappa and charges change from step to step
  return autotune_loop("tagi_autotune_learned", x, y, z, n, box, n_orb, leaf_sizes, n_leaf, obs,
                       n_ob, items, n_items, variants, n_var, reps, best, times, stream,
                       [&](tagi_tree* t, double* out) {
                         int r = tagi_upward(t, f, w, n_orb, 1, stream);
                         if (r == TAGI_OK)
                           r = tagi_convolve_learned(t, kernel, kappa, alpha, params, norm, tol,
                                                     theta_max, theta_fb, degree_fb, precision,
                                                     out, stream);
                         return r;
                       });
}

int tagi_tree_destroy(tagi_tree* t) {
  if (!t) return TAGI_OK;
  (void)hipDeviceSynchronize();
  drop_events(t);
  DBuf* bufs[] = {&t->perm, &t->xs, &t->ys, &t->zs, &t->leaf_of_pos, &t->nd_begin, &t->nd_end,
                  &t->nd_first_child, &t->nd_n_child, &t->nd_geom, &t->nd_box, &t->leaf_node,
                  &t->ws, &t->fs, &t->qs, &t->far_off, &t->near_off, &t->far_id, &t->near_id,
                  &t->chunks, &t->items, &t->item_order, &t->group_first_item, &t->batch_group_base,
                  &t->batch_chunks, &t->partial, &t->kappa_dev, &t->green_f, &t->green_phi,
                  &t->green_part, &t->tgt_fs};
  for (DBuf* b : bufs) b->release();
  if (t->tgt) tagi_tree_destroy(t->tgt);
  t->tgt = nullptr;
  t->px.release();
  for (ProxySet& ps : t->lx) ps.release();
  t->learned.release();
  delete t;
  return TAGI_OK;
}

}  // extern "C"
#pragma GCC visibility pop
