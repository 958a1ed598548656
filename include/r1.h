/*
 * r1.h -- C-ABI of libr1, an MI355X (gfx950) library that approximates the
 * rank-one convex envelope of the condensed incremental stress potential of a
 * finite-strain (1-D) damage model by successive lamination, one quadrature
 * point at a time.
 *
 * Method: Balzani, Koehler, Neumeier, Peter, Peterseim, "Multidimensional
 * rank-one convexification of incremental damage models at finite strains",
 * arXiv 2211.14318.
 *   - W(F): the condensed incremental potential of eq. 2.9 (Section 2) with the
 *     neo-Hooke psi0 of eq. 2.3 or the St. Venant-Kirchhoff psi0 of eq. 2.2
 *     (plane strain in 2D), damage D(beta) = D_inf (1 - exp(-beta/D0)) and
 *     beta = max(beta_n, psi0(F)); the constant -psi(F_k, D_k) of eq. 2.9 is
 *     dropped.  Neo-Hooke: W = +inf where det F <= 0.
 *   - W^k(F): successive lamination (eq. 3.3) evaluated along the discrete
 *     rank-one lines of Section 4.1 through F: for each direction R = a (x) b the
 *     line samples W^{k-1}(F + t_i R) are convexified (Algorithm 1) and the hull
 *     is read at t = 0; W^k(F) is the minimum over the directions.
 *   - P^k(F): the laminate-endpoint derivative of eq. 5.2 (first case),
 *     evaluated over the binary lamination tree (Algorithms 2 and 3).
 *
 * Conventions shared by every entry point
 *   - d = material->dim in {2, 3}.  Deformation gradients and stresses are
 *     structure-of-arrays, component-major: F[(i*d + j)*n + p] for point p.
 *   - Every data pointer (F, beta_n, W, P, A, tree, flags, lam_idx, X, Y) is caller-
 *     owned DEVICE memory on the handle's device; the library never frees it.
 *     r1_material / r1_lamination structs and the direction arrays they point
 *     to are HOST memory read during the call.
 *   - dtype selects the element type of F, beta_n, W and P (float or double) and
 *     the precision of the arithmetic.
 *   - Calls are stream-ordered and asynchronous on `stream` (a hipStream_t; NULL
 *     is the null stream).  A handle is not thread-safe: use one per host thread.
 *   - Grid of a level: t_i = tau*(2i - (n_t-1))/(n_t-1), i = 0..n_t-1, n_t odd,
 *     3 <= n_t <= 2049; the centre index c = (n_t-1)/2 has t_c = 0.
 *   - Errors: a negative r1_status for invalid arguments or device failures
 *     (nothing is launched on R1_EINVAL).  Conditions of single points do not
 *     fail the call; they are reported in the optional per-point flags.
 */
#ifndef R1_H
#define R1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t r1_status;
#define R1_OK 0
#define R1_EINVAL (-1)        /* null pointer, bad size, even or out-of-range n_t, depth > 2, ... */
#define R1_ENOMEM (-2)        /* device workspace could not be allocated */
#define R1_EDEVICE (-3)       /* a HIP call failed (message via r1_last_error) */
#define R1_ENOTTRAINED (-4)   /* surrogate used before training or loading */
#define R1_EUNSUPPORTED (-5)  /* valid request that this library does not implement */
#define R1_EIO (-6)           /* surrogate file could not be read or written */

typedef int32_t r1_dtype;
#define R1_F32 0
#define R1_F64 1

/* Material models */
#define R1_NEOHOOKE_DAMAGE 0  /* W of eq. 2.9 with psi0 of eq. 2.3 */
#define R1_TEST_DOUBLEWELL 1  /* test energy (F11^2-1)^2 + sum_{(i,j)!=(1,1)} (F_ij - delta_ij)^2 */
#define R1_STVK_DAMAGE 2      /* W of eq. 2.9 with the St. Venant-Kirchhoff psi0 of eq. 2.2
                                 (defined for every F: no det F constraint, flag R1_PT_DETLE0 unused) */

/* Per-point flags (bit set) */
#define R1_PT_DETLE0 1        /* neo-Hooke, det F <= 0: W = +inf, P = NaN */
#define R1_PT_NONFINITE 2     /* F or beta_n not finite: outputs NaN */
#define R1_PT_FALLBACK 4      /* surrogate inference answered by plain lamination */
#define R1_PT_ITERCAP 8       /* a hull bridge search hit its iteration cap (result still a valid upper bound) */
#define R1_PT_TIE 16          /* the laminate is ambiguous: a winning direction that laminates has a
                                 runner-up within 1e-10 (FP64) / 1e-5 (FP32) of max(|W|, 1e-3 / 1e-2),
                                 at the top level or (depth 2) at an endpoint's inner envelope; W is
                                 unaffected, the tree and P may be any of the tied laminates' */

#define R1_MAX_DEPTH 2
#define R1_TREE_NODES 3       /* nodes of a depth-2 binary lamination tree */
#define R1_MAX_NT 2049
#define R1_MAX_DIRS 4096

typedef struct r1_handle_s* r1_handle;

typedef struct {
    int32_t dim;      /* 2 (plane strain) or 3 */
    int32_t model;    /* R1_NEOHOOKE_DAMAGE, R1_STVK_DAMAGE or R1_TEST_DOUBLEWELL */
    double mu;        /* Lame parameters */
    double lambda;
    double D_inf;     /* asymptotic damage, in [0, 1) */
    double D0;        /* damage saturation, > 0 */
} r1_material;

/* One lamination level: n_dir rank-one directions a_m (x) b_m (host arrays,
 * n_dir x dim row-major doubles) and the line grid (n_t, tau). */
typedef struct {
    int32_t n_dir;
    const double* a;
    const double* b;
    int32_t n_t;
    double tau;
} r1_level;

/* depth k in {1, 2}; level[0] is the outermost lamination, level[k-1] the
 * innermost (its line samples are values of W). */
typedef struct {
    int32_t depth;
    r1_level level[R1_MAX_DEPTH];
} r1_lamination;

/* One node of the lamination tree, heap-numbered: node 0 is the laminate at F,
 * node 2k+1 the one at F^- of node k, node 2k+2 the one at F^+.  F^-/+ =
 * G + t_{i_minus/i_plus} (a_dir (x) b_dir) for the node's point G, with volume
 * fraction xi of F^+.  A node whose centre sample is a hull vertex has
 * i_minus = i_plus = c and xi = 1 (no lamination; both children sit at G).
 * Depth-1 results fill node 0 only. */
typedef struct {
    int32_t dir;
    int32_t i_minus;
    int32_t i_plus;
    float xi;
} r1_laminate;

/* ---- handle ---------------------------------------------------------------- */

/* Creates a handle bound to HIP device `device` (which becomes current). */
r1_status r1_create(r1_handle* handle, int32_t device);
r1_status r1_destroy(r1_handle handle);
const char* r1_status_string(r1_status status);
/* Text of the last device error seen by this handle ("" if none). */
const char* r1_last_error(r1_handle handle);

/* ---- plain lamination --------------------------------------------------------- */

/* W[p] = W^k(F_p) (eq. 3.3 on the given levels; Section 4).  flags: nullable
 * int32[n]. */
r1_status r1_envelope(r1_handle handle, const r1_material* material,
                      const r1_lamination* lamination, int64_t n, r1_dtype dtype,
                      const void* F, const void* beta_n, void* W, int32_t* flags,
                      void* stream);

/* As r1_envelope, plus the laminate-endpoint stress P (d*d x n SoA, eq. 5.2)
 * and, if tree != NULL, the lamination tree: R1_TREE_NODES r1_laminate per
 * point, tree[p*R1_TREE_NODES + node].  The outputs (W, P, tree, flags) must
 * not overlap the inputs or each other: at depth 1 the call keeps each point's
 * laminate in P's first rows until its stress replaces it. */
r1_status r1_envelope_stress(r1_handle handle, const r1_material* material,
                             const r1_lamination* lamination, int64_t n, r1_dtype dtype,
                             const void* F, const void* beta_n, void* W, void* P,
                             r1_laminate* tree, int32_t* flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): r1_envelope_stress (depth 1
 * or 2) with nothing allocated.  The levels' directions, and at depth 2 W^1 per
 * point and one hull result per (point, outer direction), are kept in a fixed
 * per-device workspace of 64 MiB that the library holds until the process ends
 * (looked up by r1_create); the caller passes inputs and outputs as for
 * r1_envelope_stress.  Needs 2*n_dir*dim*8 bytes per level (each rounded up
 * to 256) plus, at depth 2, n*sizeof(dtype) (rounded up to 256) + 16 (FP32) or
 * 24 (FP64) bytes per (point, outer direction); a larger request fails with
 * R1_EINVAL and the sizes in r1_last_error, nothing launched.  Every call on one
 * device shares that device's workspace: calls that overlap in time on one
 * device (different streams, threads or handles) race; calls on one stream are
 * ordered.  The directions are copied from host memory on `stream`. */
r1_status r1_envelope_stress_noalloc(r1_handle handle, const r1_material* material,
                                     const r1_lamination* lamination, int64_t n, r1_dtype dtype,
                                     const void* F, const void* beta_n, void* W, void* P,
                                     r1_laminate* tree, int32_t* flags, void* stream);

/* As r1_envelope_stress, plus the tangent moduli of the laminate (Algorithm 3,
 * third output; the consistent tangent of the relaxed stress used in Section 5):
 * A = dP^k/dF as the tree-weighted sum of the leaf moduli d^2W/dF dF of eq. 2.9,
 * with the weights of P.  A (device, non-null) is d^4 x n SoA in dtype:
 * A[((i*d + j)*d*d + k*d + l) * n + p] = dP_ij / dF_kl at point p.  P and tree
 * are nullable (tree == NULL: the tree lives in handle workspace).  A is NaN
 * where W is +inf or NaN (flags R1_PT_DETLE0, R1_PT_NONFINITE).  Where the
 * laminate is ambiguous (R1_PT_TIE) A belongs to the tree written, like P. */
r1_status r1_envelope_tangent(r1_handle handle, const r1_material* material,
                              const r1_lamination* lamination, int64_t n, r1_dtype dtype,
                              const void* F, const void* beta_n, void* W, void* P, void* A,
                              r1_laminate* tree, int32_t* flags, void* stream);

/* Relax-then-fix driver of quadrature points, one pseudo-time step (the procedure
 * of the biaxial test, Section 6.6, with the damage history of Section 2).  The
 * state of point p is its history beta[p] (device, dtype[n]: the largest psi0 it
 * has seen) and fixed[p] (device, int32[n]: 0 while its envelope is relaxed anew
 * in each step, 1 once it has been fixed).  The step's relaxed potential at F
 * is W^k(F) (eq. 3.3 on the given levels) with the history entering the step
 * as beta_n, written to W, P, tree and flags as by r1_envelope_stress (P, tree
 * and flags nullable; without a tree the library keeps one in workspace).  Then
 * for each point with fixed[p] == 0 and finite W: if the root laminate
 * laminates (i_minus != i_plus), the non-convex regime is reached and the
 * envelope is fixed with its history (fixed[p] = 1, beta[p] unchanged, reused
 * by every later step); otherwise (W^k = W at F, the convex regime) beta[p]
 * becomes max(beta[p], psi0(F)) (rounded to dtype; the double-well test energy
 * has no history).  Points with fixed[p] != 0 or W not finite keep their state.
 * beta and fixed are read and written in stream order. */
r1_status r1_path_step(r1_handle handle, const r1_material* material, const r1_lamination* lamination,
                       int64_t n, r1_dtype dtype, const void* F, void* beta, int32_t* fixed, void* W,
                       void* P, r1_laminate* tree, int32_t* flags, void* stream);

/* Tangent moduli A (layout of r1_envelope_tangent) of given lamination trees
 * (Algorithm 3 on tree[p*R1_TREE_NODES ..], nodes as written by the envelope
 * calls for the same lamination): leaves F^-/+ of each node rebuilt from its
 * direction and sample indices, weights xi = (c - i_minus)/(i_plus - i_minus)
 * (the stored float xi is not read).  W (device, dtype[n]) marks the points to
 * skip: A is NaN where W is not finite.  A node whose direction or indices do
 * not name a laminate of its level (dir outside [0, n_dir), not i_minus <= c <=
 * i_plus, indices outside [0, n_t)) gives NaN for its point; all device
 * buffers are read-only but A. */
r1_status r1_laminate_tangent(r1_handle handle, const r1_material* material,
                              const r1_lamination* lamination, int64_t n, r1_dtype dtype,
                              const void* F, const void* beta_n, const void* W,
                              const r1_laminate* tree, void* A, void* stream);

/* Uneven batch in one persistent launch (the per-point tasks of Section 5.5,
 * each point with its own lamination): point p uses table[lam_idx[p]]
 * (lam_idx: device int32[n], each in [0, n_table), else R1_EINVAL).  P and tree
 * are nullable (no stress when P == NULL).
 *
 * A plan is built once for a table and a set of table indices:
 * r1_batched_plan_create reads lam_idx (one device-to-host copy; synchronizes
 * `stream`), runs the built-in autotuner for grid sizes that have neither a
 * user setting nor a tuned value, orders the work (largest points first) and
 * keeps its own device copies of the work lists, the indices and the table's
 * directions, so later changes to lam_idx or to the direction arrays do not
 * affect it.  r1_batched_plan_execute replays the plan's launch sequence as one
 * HIP graph on `stream`; a graph is captured on first use of a set of buffers
 * (F, beta_n, W, P, tree, flags) and up to 4 such sets are kept per plan.
 * Replays of one plan must not overlap in time (they share its work queues and
 * partial results): issue them on one stream.  A plan is freed by
 * r1_batched_plan_destroy, or by r1_destroy of its handle (which frees every
 * plan left; their pointers are invalid afterwards). */
typedef struct r1_batched_plan_s* r1_batched_plan;
r1_status r1_batched_plan_create(r1_handle handle, const r1_material* material,
                                 const r1_lamination* table, int32_t n_table, int64_t n,
                                 const int32_t* lam_idx, r1_dtype dtype, void* stream,
                                 r1_batched_plan* plan);
r1_status r1_batched_plan_execute(r1_batched_plan plan, const void* F, const void* beta_n, void* W,
                                  void* P, r1_laminate* tree, int32_t* flags, void* stream);
r1_status r1_batched_plan_destroy(r1_batched_plan plan);

/* One-call form: reads lam_idx on every call (one device-to-host copy;
 * synchronizes `stream`), finds or builds the plan for the contents of the
 * table and the indices (up to 8 plans are kept per handle) and executes it. */
r1_status r1_envelope_batched(r1_handle handle, const r1_material* material,
                              const r1_lamination* table, int32_t n_table, int64_t n,
                              const int32_t* lam_idx, r1_dtype dtype, const void* F,
                              const void* beta_n, void* W, void* P, r1_laminate* tree,
                              int32_t* flags, void* stream);

/* Segment width (lanes per line, 8..64) the library uses for lines of n_t
 * points, one-level lines and inner levels of depth-2 laminations alike; 0
 * lets the autotuner decide (default).  Exposed for tests and tuning. */
r1_status r1_set_segment_width(r1_handle handle, int32_t n_t, int32_t lanes);
r1_status r1_get_segment_width(r1_handle handle, int32_t n_t, r1_dtype dtype, int32_t dim,
                               int32_t* lanes);
/* Lanes per line used for the inner level (grid size n_t) of depth-2 laminations. */
r1_status r1_get_inner_segment_width(r1_handle handle, int32_t n_t, r1_dtype dtype, int32_t dim,
                                     int32_t* lanes);

/* Autotuner: times every admissible segment width for lines of n_t points on a
 * synthetic one-level batch of 16384 points (32 directions) with the given
 * material and dtype on `stream` (synchronizes it), records the fastest for
 * one-level lines of (n_t, dtype, material->dim) in the handle and returns it
 * in *lanes (nullable).  r1_envelope_batched runs it on first use of each
 * depth-1 grid size that has neither a user setting nor a tuned value. */
r1_status r1_autotune(r1_handle handle, const r1_material* material, int32_t n_t, r1_dtype dtype,
                      void* stream, int32_t* lanes);

/* Same for the inner level of depth-2 laminations, whose lines are sampled
 * along outer lines (the bridge searches start from the previous outer
 * sample's result, which favours other widths than independent lines): times
 * the depth-2 path on a synthetic batch of 1024 points (outer level 8
 * directions x 129 points, inner level 32 directions x n_t points).  Used by
 * r1_envelope_stress at depth 2 and by r1_envelope_batched (which runs it on
 * first use of each inner grid size without a user setting or tuned value). */
r1_status r1_autotune_inner(r1_handle handle, const r1_material* material, int32_t n_t, r1_dtype dtype,
                            void* stream, int32_t* lanes);

/* Persisting the tuned segment widths (for a cache kept between runs; the
 * autotuner's results otherwise live as long as the handle).  A record is five
 * int32: n_t, dtype (r1_dtype), dim (2, 3), role (R1_TUNE_LEVEL: lines of
 * one-level envelopes; R1_TUNE_INNER: inner levels of depth-2 laminations) and
 * lanes (8, 16, 32 or 64).  r1_tuning_export writes up to `capacity` records
 * (host int32[5 * capacity], nullable when capacity is 0) in ascending key order
 * and sets *count (host) to the number the handle holds.  r1_tuning_import
 * checks every record (n_t odd in 3..R1_MAX_NT, known dtype, dim and role, lanes
 * a supported width whose layout covers the grid) and installs them all, or
 * none with R1_EINVAL.  Neither touches the device. */
#define R1_TUNE_LEVEL 0
#define R1_TUNE_INNER 1
r1_status r1_tuning_export(r1_handle handle, int32_t* records, int32_t capacity, int32_t* count);
r1_status r1_tuning_import(r1_handle handle, const int32_t* records, int32_t count);

/* ---- global lamination on a deformation-gradient mesh -------------------------
 *
 * The grid variant of Section 4.1: node values on the mesh of Section 5.2 (one
 * mesh width for every component, as in all the paper's examples), iterations
 * of eq. 4.3 -- every node takes the minimum over the directions of the lower
 * hull (Algorithm 1) of its line (eq. 4.4) through the previous iterate,
 * clipped to the mesh's box -- and off-mesh values by multilinear
 * interpolation.
 *
 * Component c = i*dim + j of node k_c takes the value lo[c] + k_c*delta,
 * k_c = 0..n[c]-1 (1 <= n[c] <= 512, at most 2^31 nodes).  Nodes are numbered
 * with component 0 varying slowest: p = ((k_0*n_1 + k_1)*n_2 + ...).  Node
 * arrays are dtype[nodes] on the device.  A direction is an integer step
 * s in Z^{dim x dim} (dim*dim int32, host, not all zero, |s_c| <= 512): the line
 * through node F holds the nodes F + l*delta*s, l integer, inside the box.
 * Non-finite node values are absent from every hull and stay as they are. */
typedef struct {
    int32_t dim;      /* 2 or 3 */
    int32_t n[9];     /* nodes per component (first dim*dim entries) */
    double lo[9];     /* first node value per component */
    double delta;     /* mesh width, > 0 */
} r1_grid;

/* The reduced direction set of eq. 5.1, a (x) b with a, b in {-1, 0, 1}^dim
 * non-zero, one step per line (s and -s are the same line; the kept one has a
 * positive first non-zero entry): 16 steps in 2D, 169 in 3D, written to steps
 * (host, capacity 169*9 int32) in a fixed order; *n_dir receives the count. */
r1_status r1_grid_r11(int32_t dim, int32_t* steps, int32_t* n_dir);

/* W^0: the material's W (eq. 2.9; neo-Hooke: +inf where det F <= 0) at every
 * node, with history beta_n shared by all nodes (material->dim == grid->dim);
 * P (nullable, device, dim*dim x nodes component-major) receives P^0 = dW/dF
 * (eq. 2.12); A (nullable, device, dim^4 x nodes, component (i*dim + j)*dim*dim
 * + k*dim + l) the moduli d^2W/dF_ij dF_kl; both NaN where W is +inf. */
r1_status r1_grid_energy(r1_handle handle, const r1_material* material, const r1_grid* grid, double beta_n,
                         r1_dtype dtype, void* W, void* P, void* A, void* stream);

/* Iterates eq. 4.3 in place on W (device node array) until the maximal decrease
 * max_F (W^k(F) - W^{k+1}(F)) over nodes with finite W^k of an iteration is at
 * most tol, or k_max iterations are done (Section 6).  iterations (host,
 * nullable) receives the count; decrease (host, nullable, k_max doubles) the
 * maximal decrease of each iteration.  P (nullable; node stresses as written by
 * r1_grid_energy) is carried along: a node lowered by the hull segment [F_a, F_b]
 * of its line takes the stress of that laminate with the weights of its value
 * (eq. 5.2, first case); A (nullable; node moduli as written by r1_grid_energy)
 * likewise, which makes A the tangent of Algorithm 3: the laminate-weighted
 * moduli of the mesh nodes whose values built the node's value (the derivative
 * of the carried stress with the laminates held fixed).  A laminate replaces a
 * node's value only when it is
 * lower by more than 4 units of rounding (of dtype) times max(|W|, 1e-3): a node
 * on a straight hull run reads its own value back up to rounding, and of
 * directions that tie to rounding the first in `steps` keeps the node.
 * Interpolating P or A (r1_grid_interpolate per component) gives eq. 5.2's
 * second case off the mesh.  Uses handle workspace of up to 17 node arrays of
 * dtype (the other iterate and the candidates of up to 16 directions); when P or
 * A is given, also one array like each, one uint32 per node and candidate slot
 * and two int32 per node for the laminates; and one uint32 mask per node on
 * meshes where the lines of at least 3 nodes are a minority.  Synchronizes
 * `stream` once per iteration. */
r1_status r1_grid_laminate(r1_handle handle, const r1_grid* grid, int32_t n_dir, const int32_t* steps,
                           r1_dtype dtype, void* W, void* P, void* A, int32_t k_max, double tol,
                           int32_t* iterations, double* decrease, void* stream);

/* out[p] = multilinear interpolation of the node values W at F_p (device, SoA
 * dim*dim x n, dtype); corners of zero weight do not take part; NaN outside the
 * box (beyond a rounding margin of 1e-9 mesh widths). */
r1_status r1_grid_interpolate(r1_handle handle, const r1_grid* grid, r1_dtype dtype, const void* W, int64_t n,
                              const void* F, void* out, void* stream);

/* ---- learned surrogate ---------------------------------------------------------
 *
 * A multilayer perceptron (F, beta_n) -> (W^k, P^k) trained on lamination
 * results; plain lamination is the fallback and the measure of its error.  Inputs x = (F_11 ..
 * F_dd, beta_n) (d_in = d*d + 1), standardized with training statistics.  The
 * network predicts the relaxation gap g = W(F) - W^k(F) >= 0 and dP = P0(F) -
 * P^k(F); inference returns W(F) - max(g, 0) and P0(F) - dP with W(F) and
 * P0(F) computed exactly, so W^k <= W holds by construction.  Hidden layers:
 * n_hidden layers of `width` SiLU units; the width x width layers run as BF16
 * MFMA with FP32 accumulation, the first layer (FP32 inputs) and the output
 * layer in FP32.  Training: mean squared error on standardized targets, Adam,
 * FP32 master weights, all on the device.
 *
 * A non-positive predicted gap means "no lamination": inference then returns
 * W(F) and P0(F) exactly; training uses a one-sided (hinge) loss for rows that
 * did not laminate and trains the stress outputs on laminating rows only.
 *
 * Routing at inference: a point goes to the fallback lamination when it lies
 * outside the training box (per-input min/max of the training rows, det F above
 * the smallest training det) or when its predicted gap exceeds the threshold
 * calibration set for its gate cell ((|F - I|, beta_n) bin).  Uncalibrated
 * surrogates route on the box only.
 *
 * Packed rows (device, FP32, row-major): X[p] = (F_11, .., F_dd, beta_n),
 * Y[p] = (W^k, P_11, .., P_dd).
 */
typedef struct r1_surrogate_s* r1_surrogate;

typedef struct {
    int32_t epochs;       /* passes over the training rows */
    int32_t batch;        /* rows per Adam step, a multiple of 64 */
    float lr;             /* Adam step size */
    float beta1, beta2;   /* Adam moment decay */
    float eps;            /* Adam denominator guard */
    float val_fraction;   /* trailing fraction of the rows held out for the report */
    float energy_weight;  /* weight of the energy output's squared error (stress outputs: 1) */
    uint64_t seed;        /* shuffling */
} r1_train_cfg;

typedef struct {
    int64_t steps;        /* Adam steps taken */
    float train_loss;     /* mean loss over the last epoch */
    float val_loss;       /* loss on the held-out rows */
    double ms;            /* device time of the training loop, milliseconds */
} r1_train_report;

/* New network for d = dim (2 or 3): n_hidden in [2, 8] hidden layers of width in
 * {32, 64, 128, 256}; weights drawn from a seeded uniform(-1/sqrt(fan_in), ..). */
r1_status r1_surrogate_create(r1_handle handle, r1_surrogate* surrogate, int32_t dim,
                              int32_t n_hidden, int32_t width, uint64_t seed);
r1_status r1_surrogate_destroy(r1_surrogate surrogate);

/* Packs lamination inputs/outputs (SoA, dtype) into rows X (n x (d*d+1)) and
 * Y (n x (d*d+1)). */
r1_status r1_surrogate_pack(r1_handle handle, int32_t dim, int64_t n, r1_dtype dtype,
                            const void* F, const void* beta_n, const void* W, const void* P,
                            float* X, float* Y, void* stream);

/* Trains on n packed rows (the last cfg->val_fraction held out): computes the
 * input and target statistics and the training box, then runs the epochs with
 * a cosine decay of the step size from cfg->lr to 0.02 cfg->lr.
 * Synchronizes `stream`; report (nullable) is host memory. */
r1_status r1_surrogate_train(r1_handle handle, r1_surrogate surrogate, const r1_material* material,
                             const float* X, const float* Y, int64_t n, const r1_train_cfg* cfg,
                             r1_train_report* report, void* stream);

/* Error gate: predicts n packed validation rows (X, Y from plain lamination)
 * and, per cell = (|F - I|, beta_n) bin, orders the rows by predicted gap g.
 * The cell's threshold is the largest g such that the rows with predicted gap
 * <= g number at least 16 and a fraction of at least `quantile` of them has
 * |W_pred - W^k| / max(|W^k|, 1e-2) <= tol; at inference a point is served by
 * the network when its predicted gap is at most its cell's threshold, and
 * falls back otherwise (cells without a threshold always fall back).
 * cells_allowed (nullable, host) receives the number of cells with a
 * threshold (of 16 x 8).  Synchronizes `stream`. */
r1_status r1_surrogate_calibrate(r1_handle handle, r1_surrogate surrogate,
                                 const r1_material* material, const float* X, const float* Y,
                                 int64_t n, float tol, float quantile, int32_t* cells_allowed,
                                 void* stream);

/* The network's raw prediction for n packed rows X (device, FP32, n x d_in), as
 * the gates see it: gate cell (device int32[n]: (|F - I|, beta_n) bin, -1 outside
 * the training box), predicted W^k (device float[n]: W(F) - max(g, 0)) and
 * predicted gap g (device float[n], before clamping).  No gate is applied. */
r1_status r1_surrogate_predict(r1_handle handle, r1_surrogate surrogate, const r1_material* material,
                               const float* X, int64_t n, int32_t* cell, float* W_pred, float* gap_pred,
                               void* stream);

/* A-posteriori check at inference (eps > 0; 0, the default, turns it off): a
 * value the network would serve at F is checked against lamination on a subset
 * of the fallback's outermost line samples -- every sample within 8 of the
 * centre, then offsets growing by about a third out to the line's ends.  Fewer
 * samples only raise a hull (Algorithm 1), so a chord of subset samples that
 * passes below the served value w at the centre shows W^k < w (eq. 3.3, any
 * depth); when one passes more than eps max(|w|, 0.01) below w, the point goes to
 * the fallback lamination instead.  Costs the W samples of the subset (about 17%
 * of the fallback's for 16 directions x 201 points) at each served point. */
r1_status r1_surrogate_set_check(r1_surrogate surrogate, float eps);
/* The check's sample offsets from the centre (indices on the level's grid, one
 * side; the check takes each at + and -) for lines of n_t points: at most 32
 * written to offsets (host), their number to *count (host). */
r1_status r1_surrogate_check_offsets(int32_t n_t, int32_t* offsets, int32_t* count);

/* W and P (SoA, dtype) for n points: the network where the gates accept, plain
 * lamination with `fallback` elsewhere (flag R1_PT_FALLBACK).  n_fallback
 * (nullable, host) receives the number of fallback points.  Synchronizes
 * `stream` once to size the fallback launch. */
r1_status r1_surrogate_infer(r1_handle handle, r1_surrogate surrogate, const r1_material* material,
                             const r1_lamination* fallback, int64_t n, r1_dtype dtype,
                             const void* F, const void* beta_n, void* W, void* P,
                             int32_t* flags, int64_t* n_fallback, void* stream);

/* Checks and persistence.  Parameters are the flat FP32 master weights in the
 * order W_0, b_0, .., W_{n_hidden-1}, b_{n_hidden-1}, W_out, b_out (row-major,
 * out x in), host memory.  loss_grad runs one forward and backward pass on n
 * already standardized rows (Xn: n x d_in, Yn: n x d_out, device) without
 * updating, writing the loss (host) and the gradient (device, same layout). */
r1_status r1_surrogate_param_count(r1_surrogate surrogate, int64_t* count);
r1_status r1_surrogate_get_params(r1_surrogate surrogate, float* params, int64_t count);
r1_status r1_surrogate_set_params(r1_surrogate surrogate, const float* params, int64_t count);
/* Standardization: x_mean, x_std (d_in), y_mean, y_std (d_out), host arrays. */
r1_status r1_surrogate_get_norm(r1_surrogate surrogate, float* x_mean, float* x_std,
                                float* y_mean, float* y_std);
r1_status r1_surrogate_loss_grad(r1_handle handle, r1_surrogate surrogate, const float* Xn,
                                 const float* Yn, int64_t n, float* grad, float* loss,
                                 void* stream);
r1_status r1_surrogate_save(r1_surrogate surrogate, const char* path);
r1_status r1_surrogate_load(r1_handle handle, r1_surrogate* surrogate, const char* path);

/* ---- measurement ---------------------------------------------------------------- */

/* When enabled, every kernel launch of the handle is bracketed by HIP events
 * recorded on its launch stream.  Kernel names: "depth1" (one-level envelope),
 * "depth2_centre", "outer", "finalize" (two-level envelope), "tangent" (tangent moduli),
 * "grid_lines" (the hulls of a group of up to 16
 * directions of a mesh iteration), "grid_pick" (the choice among them), "batched".
 * r1_timing_query waits for the recorded events and returns the summed elapsed
 * milliseconds and the launch count of `kernel` since the last reset. */
r1_status r1_timing_enable(r1_handle handle, int32_t on);
r1_status r1_timing_reset(r1_handle handle);
r1_status r1_timing_query(r1_handle handle, const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
