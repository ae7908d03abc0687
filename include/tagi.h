/*
 * tagi.h -- C ABI of the MI355X (gfx950) barycentric Lagrange treecode for the
 * Green-function convolution sums of treecode-accelerated Green Iteration
 * (Vaughn, Wilson, Krasny et al., arXiv 2003.01833).
 *
 * The library evaluates, for points r_i with values f_i and quadrature weights w_i,
 *
 *     u_i = sum_{j : |r_i - r_j| > 0} G(r_i, r_j) f_j w_j                (Section 6, Eq. direct-sum)
 *
 * with the Yukawa kernel G = exp(-k r)/r or the Coulomb kernel G = 1/r, and with
 * the singularity-subtracted forms of Section 4.3:
 *
 *   TAGI_YUKAWA_SS  (Eq. yukawa-conv-ss and the analytic term 4 pi f / k^2):
 *       u_i = sum_j (f_j - f_i) exp(-k d_ij)/d_ij w_j + 4 pi f_i / k^2
 *   TAGI_COULOMB_SS (Eqs. coulomb-conv-ss and correction_term, Gaussian width a):
 *       u_i = sum_j (f_j - f_i exp(-d_ij^2/a^2))/d_ij w_j + 2 pi a^2 f_i
 *
 * either exactly (tagi_direct) or by the barycentric Lagrange treecode of
 * Section 6 (tagi_tree_build + tagi_upward + tagi_convolve: Algorithm 3, lines
 * 1, 2 and 3). The kernels are not normalised: the Green-iteration prefactor
 * -1/(2 pi) and f = V_eff psi are the caller's.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays are FP64 (or int32 where stated), contiguous, and live in DEVICE
 *   memory of the current HIP device unless stated "host". The caller owns them.
 *   Multi-field arrays are row-major: f[n_orb][n] means orbital o's values are
 *   f + o * n.
 * - `stream` is a hipStream_t (NULL = the legacy default stream). Calls enqueue
 *   work on it; tagi_tree_build and the first tagi_convolve for a given (theta,
 *   degree) also synchronise it (they read sizes back to the host). Inputs must
 *   stay valid until the stream has passed the call; the tree copies what it
 *   keeps (sorted coordinates, weights, values), so after the call has completed
 *   the caller may overwrite its inputs.
 * - Every function returns TAGI_OK (0) or a negative status; nothing aborts or
 *   throws across the ABI. tagi_last_error() returns a thread-local message for
 *   the last failure on the calling thread. Arguments are validated before any
 *   work is enqueued.
 * - A tree handle may be used by one host thread at a time.
 * - Pairs at distance exactly zero contribute nothing (the "i != j" of Eq.
 *   direct-sum, generalised to any pair of coincident points).
 */
#ifndef TAGI_H
#define TAGI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tagi_tree tagi_tree;

/*
 * Device memory. The library allocates its own device buffers (trees, proxy
 * charges, lists, schedules, partial sums; stream-ordered scratch inside a
 * call) and keeps a tree's buffers until tagi_tree_destroy. The environment
 * variable TAGI_WORKSPACE_LIMIT (bytes, optionally with a K, M or G suffix for
 * 2^10, 2^20, 2^30; unset or 0 means no limit), read at every allocation,
 * caps the bytes the library holds at once over all trees: an allocation
 * beyond it fails with TAGI_E_OOM before anything is launched that needs it,
 * and a failed call leaves each tree usable (its caches are rebuilt on the
 * next call). Caller-owned arrays and tagi_direct_noalloc's array do not count.
 * tagi_workspace_held: HOST *bytes = the device bytes the library holds now
 * (all trees and meshes of the process). Errors: TAGI_E_ARG.
 */
int tagi_workspace_held(int64_t* bytes);

enum tagi_status {
  TAGI_OK = 0,
  TAGI_E_ARG = -1,         /* invalid argument (null pointer, size, range) */
  TAGI_E_STATE = -2,       /* call out of order (convolve before upward, degree mismatch) */
  TAGI_E_OOM = -3,         /* device allocation failed, or beyond TAGI_WORKSPACE_LIMIT */
  TAGI_E_HIP = -4,         /* a HIP runtime call failed; message in tagi_last_error() */
  TAGI_E_UNSUPPORTED = -5  /* valid request the library does not implement */
};

enum tagi_kernel {
  TAGI_YUKAWA_SS = 0,  /* exp(-k r)/r with singularity subtraction (Section 4.3) */
  TAGI_COULOMB_SS = 1, /* 1/r with Gaussian singularity subtraction (Section 4.3) */
  TAGI_YUKAWA = 2,     /* exp(-k r)/r, singular pair skipped (Eq. direct-sum) */
  TAGI_COULOMB = 3     /* 1/r, singular pair skipped (Eq. direct-sum) */
};

enum tagi_precision {
  TAGI_FP64 = 0,  /* every step in FP64 */
  TAGI_MIXED = 1  /* far-field (batch-proxy) kernel sums in FP32 per batch-cluster tile,
                     added into FP64; near field, proxy charges, combine stay FP64 */
};

/* A set of evaluation points (targets) distinct from the sources. */
typedef struct {
  const double* x;  /* DEVICE [n] target coordinates */
  const double* y;
  const double* z;
  const double* f;  /* DEVICE [n_orb][n] values f_i at the targets (the subtracted
                       kernels need them; may be NULL for TAGI_YUKAWA, TAGI_COULOMB) */
  int64_t n;        /* number of targets, 0 <= n < 2^31 */
} tagi_points;

typedef struct {
  int64_t n_points;      /* sources (= targets) */
  int32_t n_nodes;       /* clusters, root included */
  int32_t n_leaves;      /* leaves = target batches (Section 6.1, N_B = N_L) */
  int32_t max_level;     /* deepest level (root = 0) */
  int32_t leaf_size;     /* N_L */
  int32_t degree;        /* degree of the last tagi_upward (0 if none) */
  int32_t n_orb;         /* orbitals of the last tagi_upward */
  int32_t n_approx;      /* clusters holding proxy charges ((n+1)^3 < N_S) */
  double theta;          /* theta of the cached interaction lists (-1 if none) */
  int64_t n_far_pairs;   /* batch-cluster pairs evaluated by the approximation */
  int64_t n_near_pairs;  /* batch-cluster pairs evaluated directly */
  int64_t far_interactions;  /* sum over far pairs of |B| (n+1)^3, one orbital */
  int64_t near_interactions; /* sum over near pairs of |B| N_S, one orbital */
  int64_t n_work_items;  /* compute work items of the cached schedule */
  int64_t upward_points; /* sum of N_S over the clusters holding proxy charges: the
                            (source, cluster) pairs of the last tagi_upward */
} tagi_stats;

/*
 * Algorithm 3, tree step (Section 6.1): build the tree of source clusters and the
 * target batches.
 *   x, y, z    device [n] source coordinates.
 *   box        host double[6] = {lo_x, lo_y, lo_z, hi_x, hi_y, hi_z}: the domain
 *              box that the root cluster encloses, or NULL for the sources'
 *              bounding box. All sources must lie inside it.
 *   leaf_size  N_L >= 1: a cluster with more than N_L sources is divided.
 * Division (Section 6.1): a cluster is bisected at the midpoint of its box (the
 * root: of `box`; others: of their shrunk box) in every dimension whose extent
 * is at least 1/sqrt(2) of the largest extent, so into 8, 4 or 2 children;
 * every cluster is shrunk to the bounding box of its sources. The sources are
 * reordered so that every cluster is a contiguous range; batches are the leaves.
 * Synchronises `stream`. On success *out owns all device memory of the tree.
 * Errors: TAGI_E_ARG (null pointers, n < 1, n >= 2^31, leaf_size < 1, a source
 * outside `box` or not finite), TAGI_E_OOM, TAGI_E_HIP.
 */
int tagi_tree_build(const double* x, const double* y, const double* z, int64_t n,
                    const double* box, int leaf_size, void* stream, tagi_tree** out);

/*
 * Algorithm 3, proxy-charge step (Section 6.2, Eq. particle-cluster-approx-rearranged):
 * proxy charges of every cluster with more than (degree+1)^3 sources,
 *     q^_k = sum_{j in C} L_k1(x_j) L_k2(y_j) L_k3(z_j) q_j,
 * on the tensor grid of Chebyshev points of the second kind mapped to the
 * cluster's box, with the barycentric Lagrange basis (Eqs. Lagrange_polynomials,
 * barycentric_weights). Two charge sets per cluster: q_j = f_j w_j per orbital
 * and q_j = w_j (the latter carries the singularity subtraction through the far
 * field). Also stores the tree-ordered f and w for the near field.
 *   f       device [n_orb][n] values in the caller's point order.
 *   w       device [n] quadrature weights in the caller's point order.
 *   n_orb   1 <= n_orb <= 64.
 *   degree  interpolation degree n, 1 <= n <= 16.
 * Errors: TAGI_E_ARG, TAGI_E_OOM, TAGI_E_HIP.
 */
int tagi_upward(tagi_tree* tree, const double* f, const double* w, int n_orb, int degree,
                void* stream);

/*
 * Hermite proxy charges, for the barycentric Hermite treecode that the paper's
 * conclusions (Section 8) propose for the high-accuracy regime: the same
 * clusters, points and charge sets as tagi_upward, but per dimension the
 * interpolant matches values and first derivatives at the n+1 points, with
 * A_k(t) = (1 - 2 c_k (t - s_k)) L_k(t)^2, B_k(t) = (t - s_k) L_k(t)^2 and
 * c_k = sum_{m != k} 1/(s_k - s_m). Per point k and derivative pattern
 * beta in {0,1}^3 (bit 0: x, bit 1: y, bit 2: z)
 *     q^_{k,beta} = sum_{j in C} prod_d H^{beta_d}_{k_d}(y_{j,d}) q_j,  H^0 = A, H^1 = B,
 * which interpolates the kernel to degree 2n+1 per dimension. A following
 * tagi_convolve evaluates the far field as
 *     sum_k sum_beta d^beta_y G(|y - x_i|) at y = s_k, times q^_{k,beta}
 * (FP64 only: precision TAGI_MIXED then fails with TAGI_E_UNSUPPORTED), with the
 * same lists, near field and subtraction as the Lagrange form. The next
 * tagi_upward returns the tree to Lagrange charges.
 *   f, w, n_orb  as for tagi_upward.
 *   degree       1 <= n <= 7.
 * Errors: TAGI_E_ARG, TAGI_E_OOM, TAGI_E_HIP.
 */
int tagi_upward_hermite(tagi_tree* tree, const double* f, const double* w, int n_orb, int degree,
                        void* stream);

/*
 * Algorithm 3, ComputePotential step (Section 6.3): for every target batch, ComputePotential
 * from the root with the MAC of Eq. MAC, (r_B + r_C) < theta R and
 * (n+1)^3 < N_S (r = half the diagonal of a shrunk box, R = distance between box
 * midpoints); accepted pairs use the proxy charges, rejected leaves and
 * size-rejected clusters are summed directly (Eq. direct-sum_2). Then the
 * analytic subtraction term is added and the result is written in the caller's
 * point order. All n_orb orbitals of the last tagi_upward are evaluated in one
 * launch sequence (orbital o with kappa[o]).
 *   targets    NULL: the targets are the sources, and the batches are the source
 *              tree's leaves. Otherwise the evaluation points (Eq. direct-sum:
 *              targets x_i, sources y_j): the batches are then the leaves of a
 *              tree built on the targets by the rule of tagi_tree_build (Section
 *              6.1) with N_B = the tree's N_L and the targets' bounding box as
 *              root box. targets->f [n_orb][n] (caller order) gives f_i of the
 *              subtracted kernels and is required for them. A target that
 *              coincides with a source skips that pair (distance zero), as a
 *              source does with itself. n = 0 returns TAGI_OK with nothing done.
 *              The target tree, lists and schedule are rebuilt on every call
 *              with targets (which synchronises the stream); if some batch
 *              accepts the root cluster (targets outside the sources' box), the
 *              root's proxy charges are added to the tree's from the values of
 *              the last tagi_upward.
 *   kernel     enum tagi_kernel.
 *   kappa      HOST [n_orb] Yukawa decay rates, finite and > 0 (ignored for
 *              Coulomb kernels; may then be NULL).
 *   alpha      Gaussian width of TAGI_COULOMB_SS (> 0; the paper uses 1).
 *   theta      MAC parameter, 0 <= theta < 1 (0 gives the direct sum).
 *   degree     must equal the degree of the last tagi_upward.
 *   precision  enum tagi_precision.
 *   out        device [n_orb][n_t] (n_t = n, or targets->n), caller's target order.
 * Without targets the interaction lists and the work schedule are cached per
 * (theta, degree); rebuilding them synchronises the stream.
 * Errors: TAGI_E_ARG, TAGI_E_STATE (no upward yet, degree mismatch), TAGI_E_OOM,
 * TAGI_E_HIP, TAGI_E_UNSUPPORTED (a target tree deeper than the list traversal
 * supports).
 */
int tagi_convolve(tagi_tree* tree, const tagi_points* targets, int kernel, const double* kappa,
                  double alpha, double theta, int degree, int precision, double* out,
                  void* stream);

/*
 * Direct evaluation of Eq. direct-sum (with the Section 4.3 subtraction for the
 * *_SS kernels) at nt targets over ns sources, FP64.
 *   sx, sy, sz, sf, sw  device [ns] source coordinates, values, weights.
 *   tx, ty, tz          device [nt] target coordinates.
 *   tf                  device [nt] target values (required for *_SS kernels,
 *                       ignored otherwise; may be NULL then).
 *   out                 device [nt].
 * Errors: TAGI_E_ARG (null pointers, sizes < 1 or >= 2^31, kappa <= 0 for
 * Yukawa, alpha <= 0 for TAGI_COULOMB_SS), TAGI_E_OOM, TAGI_E_HIP.
 */
int tagi_direct(const double* sx, const double* sy, const double* sz, const double* sf,
                const double* sw, int64_t ns, const double* tx, const double* ty,
                const double* tz, const double* tf, int64_t nt, int kernel, double kappa,
                double alpha, double* out, void* stream);

/*
 * tagi_direct for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, kernels and summation order as tagi_direct, so the same results;
 * it calls no allocating routine. Its scratch (the charges f w and the partial
 * sums) lives in a device array of 33,554,432 bytes that the library holds on
 * every GPU it runs on until the process ends. A call needs
 *     ceil(8 ns / 256) * 256 + 1024 * ceil(nt / 64) * n_sc
 * bytes of it, n_sc = the source chunks per 64-target group that tagi_direct
 * also uses (max(1, min(16384 / ceil(nt / 64), ns / 512)), then adjusted to
 * cover ns); calls needing more fail with TAGI_E_ARG before any work is
 * enqueued (e.g. ns = 1,000,000 and nt = 100,000 need 24,005,120 bytes).
 * Every call on one GPU uses that GPU's one array: calls that overlap on one GPU
 * (other streams, other host threads) race and give wrong results; calls in
 * stream order on one stream are safe. Errors: as tagi_direct; TAGI_E_ARG also
 * for sizes beyond the scratch.
 */
int tagi_direct_noalloc(const double* sx, const double* sy, const double* sz, const double* sf,
                        const double* sw, int64_t ns, const double* tx, const double* ty,
                        const double* tz, const double* tf, int64_t nt, int kernel, double kappa,
                        double alpha, double* out, void* stream);

/* Sizes and interaction counts of the tree and its cached lists (host struct). */
int tagi_tree_stats(const tagi_tree* tree, tagi_stats* out);

/*
 * Copies the tree to HOST buffers for inspection (any pointer may be NULL):
 *   perm   int32 [n]       tree position -> caller index
 *   begin, end, parent, level, n_child  int32 [n_nodes]
 *   lo, hi double [n_nodes][3] shrunk boxes
 * Synchronises `stream`. Errors: TAGI_E_ARG, TAGI_E_HIP.
 */
int tagi_tree_export(const tagi_tree* tree, int32_t* perm, int32_t* begin, int32_t* end,
                     int32_t* parent, int32_t* level, int32_t* n_child, double* lo, double* hi,
                     void* stream);

/*
 * Copies the cached interaction lists of (theta, degree) to HOST buffers, built
 * first if needed: per batch b (leaf order), far clusters
 * far_id[far_off[b] .. far_off[b+1]) and near clusters likewise, in the order
 * ComputePotential visits them. Pass NULL id arrays to query the sizes, which are
 * written to *n_far and *n_near (host int64). Offsets are int64 [n_leaves+1].
 * Errors: TAGI_E_ARG, TAGI_E_STATE, TAGI_E_OOM, TAGI_E_HIP.
 */
int tagi_lists_export(tagi_tree* tree, double theta, int degree, int64_t* far_off,
                      int32_t* far_id, int64_t* near_off, int32_t* near_id, int64_t* n_far,
                      int64_t* n_near, void* stream);

/*
 * Copies the proxy data of the last tagi_upward or tagi_upward_hermite to HOST
 * buffers (NULL skips):
 *   cluster  int32 [n_approx]                     node id of each approximable cluster
 *   nodes    double [n_approx][3][degree+1]       Chebyshev points per dimension
 *   qhat     double [n_orb][n_approx][(degree+1)^3] proxy charges of f w (k1 slowest);
 *            Hermite: [n_orb][n_approx][(degree+1)^3][8], pattern beta fastest
 *   what     double [n_approx][(degree+1)^3]      proxy charges of w; Hermite: [..][8]
 * Errors: TAGI_E_ARG, TAGI_E_STATE, TAGI_E_HIP.
 */
int tagi_upward_export(const tagi_tree* tree, int32_t* cluster, double* nodes, double* qhat,
                       double* what, void* stream);

/*
 * One step of a Green iteration, captured once as a HIP graph and replayed: the
 * upward pass (Algorithm 3, proxy-charge step) and the convolution (ComputePotential step) for fixed
 * buffers, exactly as tagi_upward followed by tagi_convolve with the same
 * arguments. Intended for iterations where f is rewritten in place between
 * steps (f = V_eff psi): each replay reads the current contents of f and w and
 * writes out.
 *   tagi_graph_create runs the step once on `stream` (which prepares and caches
 *   every plan, list and buffer), synchronises, then captures the kernels of a
 *   second run on an internal stream. f, w, kappa values, out and every other
 *   argument are frozen into the graph; the tree must outlive the graph and must
 *   not be used with other arguments while the graph is in use.
 *   tagi_graph_launch enqueues one replay on `stream`.
 * Errors: as tagi_upward and tagi_convolve; TAGI_E_HIP if capture fails.
 */
typedef struct tagi_graph tagi_graph;
int tagi_graph_create(tagi_tree* tree, const double* f, const double* w, int n_orb, int degree,
                      int kernel, const double* kappa, double alpha, double theta, int precision,
                      double* out, void* stream, tagi_graph** graph);
int tagi_graph_launch(tagi_graph* graph, void* stream);
int tagi_graph_destroy(tagi_graph* graph);

/*
 * Adaptive cuboid mesh with tensor Fejer quadrature (Section 4.2), built on the
 * GPU. From the domain box [lo3, hi3], `uniform_levels` rounds bisect every cell
 * into eight; then each round replaces a cell C by its eight children C_i iff
 * |int_C t - sum_i int_{C_i} t| >= tol_m (Eq. refinement_criterion), both by the
 * Fejer rule on (p+1)^3 Chebyshev points of the first kind (Eq.
 * Chebyshev_points), until no cell splits or `max_level` is reached. Cells that
 * hold an atom strictly inside along some dimension are split there (atoms on
 * vertices), cells with longest/shortest side > max_aspect are halved along the
 * longest side, and the cells are sorted by (lo x, lo y, lo z, hi x, hi y, hi z).
 *   atoms    HOST double [n_atoms][4] = x, y, z, Z (0 <= n_atoms <= 64)
 *   test_fn  TAGI_TEST_DENSITY: t = sum_a Z_a^3/pi exp(-2 Z_a d_a) (hydrogenic
 *            1s densities); TAGI_TEST_ROOT_DENSITY_VEXT: Eq. test_function,
 *            t = sqrt(rho0) V_ext with that rho0 and V_ext = -sum_a Z_a / d_a
 *   1 <= p <= 15, tol_m > 0, 0 <= uniform_levels <= 6,
 *   uniform_levels <= max_level <= 40, max_aspect >= 1.
 * Synchronises the stream. Points of a cell are c + h s_i per dimension
 * (c, h: centre and half-width, s_i = cos((2i+1) pi / (2p+2))) with weights the
 * products of h v_i (Fejer's first rule, Waldvogel 2006), x index slowest; cells
 * in order. Errors: TAGI_E_ARG, TAGI_E_OOM, TAGI_E_HIP, TAGI_E_UNSUPPORTED
 * (more than 2^31 points).
 */
typedef struct tagi_mesh tagi_mesh;
enum tagi_mesh_test { TAGI_TEST_DENSITY = 0, TAGI_TEST_ROOT_DENSITY_VEXT = 1 };
int tagi_mesh_build(const double* lo3, const double* hi3, int p, double tol_m,
                    int uniform_levels, int max_level, const double* atoms, int n_atoms,
                    int test_fn, double max_aspect, void* stream, tagi_mesh** out);
/* HOST outputs: cells and points ((p+1)^3 per cell). */
int tagi_mesh_info(const tagi_mesh* mesh, int64_t* n_cells, int64_t* n_points);
/* HOST double [n_cells][3] each (NULL skips). */
int tagi_mesh_cells(const tagi_mesh* mesh, double* lo, double* hi);
/* DEVICE double [n_points] each: quadrature points and weights. */
int tagi_mesh_points(const tagi_mesh* mesh, double* x, double* y, double* z, double* w,
                     void* stream);
int tagi_mesh_destroy(tagi_mesh* mesh);

/*
 * One block step of Green Iteration (the iteration body of Algorithm 2, applied
 * to every wavefunction of the block at once) around the batched convolution:
 *   1. f_o = V_eff psi_o and psi'_o = G(eps_o) psi_o (Eqs. integral_operator,
 *      Hemlholtz_Greens_Function): -1/(2 pi) times the subtracted Yukawa sum
 *      (Section 4.3) of f_o with kappa_o = sqrt(-2 eps_o), by the treecode at
 *      (theta, degree) on the tree's points with quadrature weights w;
 *   2. the gradient-free eigenvalue update (Eq. gradient-free),
 *      eps'_o = eps_o - <V_eff psi_o, psi_o - psi'_o> / <psi'_o, psi'_o>,
 *      with psi'_o before orthogonalization;
 *   3. psi'_o orthogonalized against psi'_j, j < o (classical Gram-Schmidt,
 *      twice), in block order, then normalized;
 *   4. resid_o = ||psi'_o - psi_o||.
 * Inner products are sum_j w_j a_j b_j (the mesh quadrature).
 *   psi      DEVICE double [n_orb][n] current wavefunctions, caller order
 *   veff, w  DEVICE double [n] effective potential and quadrature weights
 *   eps      HOST double [n_orb] eigenvalues (< 0), replaced by the update
 *   psi_out  DEVICE double [n_orb][n] new wavefunctions (must not alias psi)
 *   resid    HOST double [n_orb] or NULL
 * Runs tagi_upward on the tree (its previous upward state is replaced).
 * Reductions are block sums added on the host in a fixed order: the step is
 * bitwise repeatable. Synchronises the stream.
 * Errors: TAGI_E_ARG (bad arguments, a wavefunction that vanishes or becomes
 * linearly dependent), TAGI_E_OOM, TAGI_E_HIP.
 */
int tagi_green_step(tagi_tree* tree, const double* psi, const double* veff, const double* w,
                    int n_orb, double* eps, double theta, int degree, int precision,
                    double* psi_out, double* resid, void* stream);

/*
 * tagi_green_step with the learned selector as its convolution (the project's
 * learned degree/MAC lists, as tagi_convolve_learned with TAGI_YUKAWA_SS and
 * kappa_o = sqrt(-2 eps_o)) in place of the fixed (theta, degree): steps 2-4
 * are the same. params, norm, theta_max, theta_fb, degree_fb as for
 * tagi_convolve_learned; tol HOST [n_orb] the absolute error budget of one
 * target's subtracted Yukawa sum of f_o = V_eff psi_o (psi'_o's error is
 * 1/(2 pi) of it). The lists are rebuilt whenever kappa or tol change, i.e.
 * on nearly every step of an iteration. Runs an upward pass on the tree (its
 * previous upward state is replaced). Synchronises the stream; bitwise
 * repeatable.
 * Errors: as tagi_green_step and tagi_convolve_learned.
 */
int tagi_green_step_learned(tagi_tree* tree, const double* psi, const double* veff,
                            const double* w, int n_orb, double* eps, const float* params,
                            const float* norm, const double* tol, double theta_max,
                            double theta_fb, int degree_fb, int precision, double* psi_out,
                            double* resid, void* stream);

/*
 * Orbital block of the batched launch (a project addition on the per-orbital
 * loop of Algorithm 2): the interaction kernel evaluates the geometry of a pair
 * once for `ob` orbitals. ob = 1, 2, 4 or 8 fixes the width for every later
 * tagi_convolve / tagi_convolve_learned on the tree (the schedule is rebuilt on
 * the next call); ob = 0 restores the automatic choice: the largest power of
 * two not above n_orb, capped at 4 for Yukawa kernels in mixed precision
 * under tagi_convolve (tagi_convolve_learned takes 8 there too) and at
 * 8 otherwise. Results do not depend on ob.
 * Errors: TAGI_E_ARG.
 */
int tagi_tree_set_orbital_block(tagi_tree* tree, int ob);

/*
 * Granularity of the compute schedule (a project addition): each batch's far
 * and near lists are cut into chunks of at most E / items kernel evaluations per
 * target lane (E = the whole convolution's), and a work item is one chunk for
 * one 64-target group and orbital block, so a launch holds about `items` waves
 * (more where batches hold several groups). Fewer, longer items cost less
 * per-item overhead; more, shorter ones balance the chip's 256 CUs better.
 * items = 0 restores the default (16384); otherwise 256 <= items <= 2^22. The
 * next tagi_convolve / tagi_convolve_learned on the tree rebuilds its schedule.
 * Results change only by the order of the partial sums (rounding).
 * Errors: TAGI_E_ARG.
 */
int tagi_tree_set_schedule_items(tagi_tree* tree, int items);

/*
 * Launch variant of the interaction kernel (a project addition; tile
 * parameters the autotuner chooses): 0 the defaults; 1 the other register
 * budget (waves per SIMD); 2 the other step along a proxy-grid row in the FP64
 * far field; 3 the other number of near-field sources per step. Compiled for
 * the subtracted kernels at degrees 6 to 10 and orbital blocks of 1, 4 and 8;
 * elsewhere every variant runs the defaults. No variant changes the arithmetic
 * or its order: results are bitwise the same. Applies to later tagi_convolve /
 * tagi_convolve_learned calls on the tree.
 * Errors: TAGI_E_ARG (variant outside 0..3).
 */
int tagi_tree_set_kernel_variant(tagi_tree* tree, int variant);

/*
 * Autotuner for the batched launch (a project addition): picks the leaf size
 * N_L (Section 6.1; batches are leaves, so it sets both N_L and N_B), the
 * orbital block width, the schedule granularity and the kernel launch variant
 * for one convolution by timing the candidates on the caller's data. For every
 * leaf size it builds a tree, and for every (orbital block, schedule items,
 * variant) triple it runs tagi_upward + tagi_convolve once untimed (plans,
 * lists and schedule), then `reps` times between HIP events on `stream`.
 *   x, y, z, w   DEVICE double [n] sources; f DEVICE double [n_orb][n]
 *   box          HOST double[6] root box or NULL, as tagi_tree_build
 *   kernel, kappa (HOST [n_orb]), alpha, theta, degree, precision: as tagi_convolve
 *   leaf_sizes   HOST int [n_leaf] candidates (>= 1)
 *   obs          HOST int [n_ob] candidates (0, 1, 2, 4 or 8)
 *   items        HOST int [n_items] candidates for tagi_tree_set_schedule_items
 *   variants     HOST int [n_var] candidates for tagi_tree_set_kernel_variant
 *   best         HOST int [4] receives {leaf size, orbital block, items, variant} of the fastest
 *   times        HOST double [n_leaf][n_ob][n_items][n_var] mean ms per step (may be NULL)
 * The accuracy at a fixed (theta, degree) changes slightly with N_L; checking
 * it is the caller's. Synchronises the stream; allocates and frees its own
 * scratch (one output array and the candidate trees).
 * Errors: as tagi_tree_build, tagi_upward and tagi_convolve; TAGI_E_ARG.
 */
int tagi_autotune(const double* x, const double* y, const double* z, const double* w, int64_t n,
                  const double* box, const double* f, int n_orb, int kernel, const double* kappa,
                  double alpha, double theta, int degree, int precision, const int* leaf_sizes,
                  int n_leaf, const int* obs, int n_ob, const int* items, int n_items,
                  const int* variants, int n_var, int reps, int* best, double* times,
                  void* stream);

/*
 * tagi_autotune for the learned lists (a project addition): the same
 * candidates, best[4] and times layout, with each step an upward pass (lowest
 * degree) and tagi_convolve_learned(kernel, kappa, alpha, params, norm, tol,
 * theta_max, theta_fb, degree_fb, precision) as documented there. Every step
 * stages its charges again, so the learned lists are rebuilt in each timed
 * step, as in a Green iteration. Results do not depend on the orbital block
 * or the launch variant; the schedule items regroup partial sums and the leaf
 * size changes the tree. Synchronises the stream; allocates and frees its own
 * scratch.
 * Errors: as tagi_autotune and tagi_convolve_learned.
 */
int tagi_autotune_learned(const double* x, const double* y, const double* z, const double* w,
                          int64_t n, const double* box, const double* f, int n_orb, int kernel,
                          const double* kappa, double alpha, const float* params,
                          const float* norm, const double* tol, double theta_max,
                          double theta_fb, int degree_fb, int precision, const int* leaf_sizes,
                          int n_leaf, const int* obs, int n_ob, const int* items, int n_items,
                          const int* variants, int n_var, int reps, int* best, double* times,
                          void* stream);

/*
 * Learned degree/MAC selector (a project addition on top of Section 6.2-6.3).
 *
 * Network: 5 inputs -> 3 hidden tanh layers of 64 -> 9 linear outputs, FP32.
 * Parameters are one flat array, layer by layer, each layer's weights W[out][in]
 * (row-major) followed by its biases: 5*64+64, 64*64+64, 64*64+64, 64*9+9
 * floats (tagi_selector_param_count()). Output k predicts log10 of the largest
 * absolute error of approximating a batch-cluster pair at degree 4 + k, minus
 * the pair scale s = log10(l1) - c d log10(e) - log10(d), d = R - r_B,
 * l1 = feature 5 below, c = the kernel's decay rate (kappa for the Yukawa
 * kernels, 0 for the Coulomb kernels): the error relative to the size of the
 * pair's far field.
 *
 * tagi_selector_samples: training data from the method itself. After an upward
 * pass at degree 4 with f (one orbital) and w, the far pairs of the lists at
 * (theta_max, degree 4) are the candidates; an evenly strided subset of at most
 * max_pairs is kept. kernel: TAGI_YUKAWA_SS (decay kappa > 0) or
 * TAGI_COULOMB_SS (Gaussian width alpha > 0; decay 0). For each pair, HOST
 * outputs:
 *   features [m][5] = {r_C, R - r_B, c, N_S, l1}, radii and R as in the MAC,
 *                      c the decay rate, l1 = |q^_C|_1 + g max_B |f| |w^_C|_1 from
 *                      C's degree-4 proxy charges of f w (q^) and of w (w^): the
 *                      size of the charges q^ - f_i w^ the pair's far field
 *                      carries, with g = 1 for TAGI_YUKAWA_SS, and for
 *                      TAGI_COULOMB_SS g = exp(-dm^2/alpha^2) at the least
 *                      distance dm = max(R - r_B - r_C, 0) of the pair (the
 *                      Gaussian's bound over it); tagi_convolve_learned takes
 *                      g = 0 for the plain kernels;
 *   errors   [m][9] = max over up to 256 of the batch's targets, spread
 *                      evenly (target begin + k nb / min(nb, 256), k < min(nb, 256),
 *                      nb = batch size), of |approximated - direct| pair
 *                      contribution (with the Section 4.3 subtraction of the
 *                      kernel) at degrees 4..12; NaN where the cluster holds
 *                      too few sources for that degree ((n+1)^3 >= N_S);
 *   pair_ids [m][2] = {batch leaf node id, cluster node id} (may be NULL).
 * *n receives m. Synchronises the stream; leaves the tree's upward state at
 * degree 12.
 *
 * tagi_selector_grad: loss and gradient of one batch (DEVICE X [m][5] inputs,
 * Y [m][9] targets, M [m][9] mask of existing targets; with r = out - Y and a(r) = 1 for
 * r >= 0, 4 for r < 0 (under-prediction costs more): loss = sum M a(r) r^2 /
 * (2 sum M)); grads DEVICE, same layout as params; *loss HOST.
 *
 * tagi_selector_train: mini-batch Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8)
 * updating DEVICE params in place; `order` (HOST [m]) is a permutation of the
 * rows, epoch e takes windows of `batch` consecutive rows of it starting at
 * (b * batch + e * (batch / 3 + 1)) mod m; loss_hist (HOST [epochs], may be NULL)
 * receives each epoch's mean mini-batch loss. Needs m >= batch.
 */
/*
 * tagi_convolve_learned: the far/near split of Algorithm 3 with the degree and acceptance of
 * every batch-cluster pair chosen by the selector network (any kernel;
 * requires a previous tagi_upward, whose f and w are used at every degree).
 * A pair with (r_B + r_C) < theta_max R is evaluated by the network once per
 * orbital on the features above, transformed as x_k = (ln(raw_k + o_k) - shift_k) *
 * scale_k with o = (0, 0, 0.25, 0, 0) (the decay rate may be 0); it is
 * approximated at the lowest degree n in 4..12 with (n+1)^3 < N_S whose
 * predicted log10 error (output + pair scale) is <= log10(tol[o] / M_B)
 * for every orbital o, M_B = the number of far pairs of the batch in the
 * fixed-MAC lists at (theta_max, degree 4) (tol: HOST [n_orb], absolute error
 * budget of one target's sum per orbital; a target's far-field error is at most
 * the sum of its pairs' errors); otherwise the cluster is opened (a
 * leaf, or a cluster of at most 125 sources, is summed directly). If any
 * ln(raw_k + o_k) lies outside [lo_k, hi_k] (the training range), the pair falls back
 * to the fixed MAC with (theta_fb, degree_fb). Pairs failing the theta_max test
 * are opened as in Algorithm 3.
 *   kappa   HOST [n_orb] for the Yukawa kernels (may be NULL for Coulomb)
 *   alpha   Gaussian width of TAGI_COULOMB_SS (> 0); it does not enter the
 *           features (the shipped network's Coulomb-SS samples use alpha = 1)
 *   params  HOST float [tagi_selector_param_count()]
 *   norm    HOST float [20] = shift[5], scale[5], lo[5], hi[5]
 *   0 < theta_fb, theta_max < 1; 4 <= degree_fb <= 12; tol[o] > 0.
 * Lists and per-degree plans are cached per argument set and are rebuilt
 * after every upward pass, whose charges give the features (rebuilding them
 * synchronises the stream); proxy charges are recomputed on every call.
 * Errors: TAGI_E_ARG, TAGI_E_STATE (no upward), TAGI_E_OOM, TAGI_E_HIP,
 * TAGI_E_UNSUPPORTED (lists beyond 2^31 entries, a tree deeper than the
 * traversal supports).
 *
 * tagi_learned_stats: HOST int64 out[17] = {far pairs, near pairs, far
 * evaluations, near evaluations (one orbital), far pairs at degree 0..12}.
 */
int tagi_convolve_learned(tagi_tree* tree, int kernel, const double* kappa, double alpha,
                          const float* params, const float* norm, const double* tol,
                          double theta_max, double theta_fb, int degree_fb, int precision,
                          double* out, void* stream);
int tagi_learned_stats(const tagi_tree* tree, int64_t* out);
/*
 * Copies the lists of the last tagi_convolve_learned to HOST buffers:
 *   far_off [n_leaves+1], far_id / far_degree [far pairs] (per batch, grouped by
 *   increasing degree, traversal order within a degree), near_off [n_leaves+1],
 *   near_id [near pairs] (traversal order); sizes from tagi_learned_stats.
 * Errors: TAGI_E_ARG, TAGI_E_STATE (no learned lists).
 */
int tagi_learned_lists_export(const tagi_tree* tree, int64_t* far_off, int32_t* far_id,
                              int32_t* far_degree, int64_t* near_off, int32_t* near_id);
int tagi_selector_param_count(void);
int tagi_selector_samples(tagi_tree* tree, const double* f, const double* w, int kernel,
                          double kappa, double alpha, double theta_max, int64_t max_pairs,
                          float* features, float* errors, int32_t* pair_ids, int64_t* n,
                          void* stream);
int tagi_selector_grad(const float* params, const float* X, const float* Y, const float* M,
                       int64_t m, float* grads, float* loss, void* stream);
int tagi_selector_train(float* params, const float* X, const float* Y, const float* M, int64_t m,
                        const int32_t* order, int epochs, int batch, float lr, float* loss_hist,
                        void* stream);

/* Per-phase device time of the calls made on a tree while timing is enabled,
 * measured with HIP events recorded on the calls' stream around each phase's
 * kernels (host-side work between kernels is not included). */
typedef struct {
  double build_ms;        /* tagi_tree_build (device work and host orchestration) */
  double upward_ms;       /* tagi_upward: gather + proxy charges */
  double lists_ms;        /* interaction lists and schedule (only when rebuilt) */
  double interact_ms;     /* batch-cluster interaction kernel (far + near fields) */
  double combine_ms;      /* partial-sum reduction, subtraction term, unpermute */
  int64_t interact_launches;
  double interact_kernel_ms; /* sum of the interaction launches' own durations (events on
                                each launch's stream around it alone): interact_ms when
                                they run one after another, more when they overlap (the
                                learned selection runs its per-degree launches side by
                                side on several streams) */
} tagi_timing;

/* Enables (1) or disables (0) phase timing on the tree; enabling resets the sums. */
int tagi_tree_set_timing(tagi_tree* tree, int enable);

/* Sums of the phase times since timing was enabled. Synchronises on the recorded
 * events. Errors: TAGI_E_ARG, TAGI_E_HIP. */
int tagi_tree_timing(tagi_tree* tree, tagi_timing* out);

/* Frees every device buffer of the tree (synchronises the device first). NULL is a no-op. */
int tagi_tree_destroy(tagi_tree* tree);

/* Thread-local message describing the last failure on this thread ("" if none). */
const char* tagi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TAGI_H */
