/*
 * r1_oracle.h -- reference oracle for the rank-one lamination method of
 * Balzani, Koehler, Neumeier, Peter, Peterseim, "Multidimensional rank-one
 * convexification of incremental damage models at finite strains",
 * arXiv 2211.14318.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, serial, double-precision CPU
 * implementation written to be checked against the paper by eye.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * Conventions
 *   - Matrices are d x d, row-major, d in {2, 3}.  In 2D the deformation is
 *     plane strain: the 3x3 gradient is embedded with F33 = 1.
 *   - A "level" is one lamination step (eq. 3.3): n_dir rank-one directions
 *     R_m = a_m (x) b_m and an equispaced line grid t_i = tau*(2i-(n_t-1))/(n_t-1),
 *     i = 0..n_t-1, n_t odd, so the centre index c = (n_t-1)/2 has t_c = 0.
 *   - depth k: level[0] is the outermost lamination, level[k-1] the innermost,
 *     whose line samples are values of the unrelaxed potential W.
 *   - W = +inf where det G <= 0.
 */
#ifndef R1_ORACLE_H
#define R1_ORACLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MODEL_NH_DAMAGE 0   /* neo-Hooke psi0 (eq. 2.3) with (1-D) damage, W of eq. 2.9 */
#define ORC_MODEL_DOUBLEWELL 1  /* test energy (G11^2-1)^2 + sum_{(i,j)!=(1,1)} (G_ij-delta_ij)^2 */
#define ORC_MODEL_STVK_DAMAGE 2 /* St. Venant-Kirchhoff psi0 (eq. 2.2) with (1-D) damage, W of eq. 2.9 */

#define ORC_MAX_DEPTH 2
#define ORC_TREE_NODES 3        /* 2^ORC_MAX_DEPTH - 1 */

/* malloc that reports the request and aborts when it cannot be met (the oracle
 * has no partial results to return). */
void* orc_alloc(size_t bytes);

typedef struct {
    int dim;       /* 2 or 3 */
    int model;     /* ORC_MODEL_* */
    double mu, lambda, D_inf, D0;
} orc_material;

typedef struct {
    int n_dir;
    const double* a;   /* n_dir x dim, row-major */
    const double* b;   /* n_dir x dim */
    int n_t;           /* odd, >= 3 */
    double tau;
} orc_level;

typedef struct {
    int depth;         /* 0, 1 or 2 */
    orc_level level[ORC_MAX_DEPTH];
} orc_lamination;

/* One node of the lamination tree (Algorithm 2 restricted to a binary tree).
 * Nodes are numbered heap-wise: node 0 is the laminate at F, node 2k+1 is the
 * laminate at F^- of node k and node 2k+2 the one at F^+.  A node without
 * lamination (the centre sample is a hull vertex) has i_minus = i_plus = c,
 * xi = 1, and both its children sit at the same point. */
typedef struct {
    int dir;            /* minimising direction index m* */
    int i_minus;        /* hull vertex left of (or at) the centre */
    int i_plus;         /* hull vertex right of (or at) the centre */
    double xi;          /* volume fraction of F^+ : (c - i_minus)/(i_plus - i_minus) */
    double value;       /* W^l at this node */
    double dir_gap;     /* runner-up direction value minus the minimum (+inf if one direction,
                           or if the node does not laminate) */
    double bridge_gap;  /* laminating node: distance of the nearest other sample above the
                           chosen hull segment; non-laminating node: the smallest margin, over
                           all directions, by which the centre sample stays a hull vertex */
} orc_laminate;

/* Section 2 */
double orc_psi0(const orc_material* mat, const double* G);
double orc_damage(const orc_material* mat, double beta);
double orc_energy(const orc_material* mat, const double* G, double beta_n);
int orc_stress0(const orc_material* mat, const double* G, double beta_n, double* P);
/* Tangent moduli d^2 W / dG dG (d^2 x d^2, A[(i*d+j)*d*d + k*d+l]); NaN where det G <= 0. */
int orc_tangent0(const orc_material* mat, const double* G, double beta_n, double* A);

/* Algorithm 1 (convexify): lower hull of (x_i, w_i), x strictly increasing.
 * Writes the indices (into x/w) of the hull vertices to vert and returns their count. */
int orc_convexify(int L, const double* x, const double* w, int* vert);

/* Value at the centre index c of the lower convex hull of the finite samples of
 * w[0..n-1] (the finite samples form one index range containing c).  Returns the
 * hull value and the bracketing vertices; bridge_gap as in orc_laminate (nullable). */
double orc_hull_at_centre(int n, const double* w, int c, int* i_minus, int* i_plus,
                          double* bridge_gap);

/* Grid point t_i of a level. */
double orc_tgrid(const orc_level* lv, int i);

/* W^k(F) by successive lamination (eq. 3.3 restricted to the level's lines).
 * P (d*d, nullable) receives the laminate stress (eq. 5.2, Algorithm 3); tree
 * (ORC_TREE_NODES entries, nullable) receives the lamination tree. */
double orc_envelope(const orc_material* mat, const orc_lamination* lam,
                    const double* F, double beta_n, double* P, orc_laminate* tree);

/* Energy and stress of a given lamination tree (Algorithm 3 on the tree whose
 * dir/i_minus/i_plus entries are given; value/xi/gaps are ignored).  Returns the
 * tree's energy; P (nullable) its stress.  Used to check a result that differs
 * from the oracle's own at a tie. */
double orc_eval_tree(const orc_material* mat, const orc_lamination* lam,
                     const double* F, double beta_n, const orc_laminate* tree, double* P);

/* The same with the tangent moduli of the laminate (Algorithm 3's third output:
 * the tree-weighted sum of the leaves' d^2 W / dG dG); A (d^4, nullable). */
double orc_envelope_tangent(const orc_material* mat, const orc_lamination* lam,
                            const double* F, double beta_n, double* P, double* A, orc_laminate* tree);
double orc_eval_tree_tangent(const orc_material* mat, const orc_lamination* lam,
                             const double* F, double beta_n, const orc_laminate* tree, double* P,
                             double* A);

/* Batched drivers over structure-of-arrays inputs F[(i*d+j)*n + p]. */
void orc_envelope_batch(const orc_material* mat, const orc_lamination* lam, long n,
                        const double* F, const double* beta_n, double* W, double* P,
                        orc_laminate* trees);
/* With the tangent moduli, SoA A[(ij*d*d + kl)*n + p] (nullable). */
void orc_envelope_batch_tangent(const orc_material* mat, const orc_lamination* lam, long n,
                                const double* F, const double* beta_n, double* W, double* P,
                                double* A, orc_laminate* trees);

/* Surrogate network oracle (mlp.c): FP64 MLP with SiLU hidden layers, flat
 * parameter layout W_0, b_0, ..., W_out, b_out (row-major, out x in). */
long orc_mlp_param_count(int d_in, int width, int n_hidden, int d_out);
double orc_mlp_forward(int d_in, int width, int n_hidden, int d_out, const double* params,
                       long B, const double* x, const double* y, double* out);
double orc_mlp_loss_grad(int d_in, int width, int n_hidden, int d_out, const double* params,
                         long B, const double* x, const double* y, double* grad);

/* ---- global lamination on a deformation-gradient mesh (grid.c) ---- */

/* Mesh of Section 5.2 with one mesh width for every component: component c =
 * i*d + j takes the values lo[c] + k delta, k = 0..n[c]-1.  Node p enumerates
 * the components with component 0 varying slowest. */
typedef struct {
    int dim;
    int n[9];
    double lo[9];
    double delta;
} orc_grid;

long orc_grid_size(const orc_grid* g);
void orc_grid_node(const orc_grid* g, long p, double* F);
int orc_grid_r11(int dim, int* steps);
void orc_grid_energy(const orc_material* mat, const orc_grid* g, double beta_n, double* W, double* P,
                     double* A);
double orc_grid_sweep(const orc_grid* g, int n_dir, const int* steps, const double* Win, double* Wout, int m,
                      const double* Cin, double* Cout);
double orc_grid_update_node(const orc_grid* g, int n_dir, const int* steps, const double* W, long p);
int orc_grid_laminate(const orc_grid* g, int n_dir, const int* steps, double* W, int m, double* C, int k_max,
                      double tol, double* hist);
double orc_grid_interpolate(const orc_grid* g, const double* W, const double* F);

/* Relax-then-fix driver of one point (Section 6.6, history of Section 2; see
 * path.c): n_steps gradients F_steps (step-major, d*d each), initial history
 * beta0 and status fixed0 (1: the envelope is already fixed with beta0).  Per
 * step: W[s], P[s*d*d ..] (nullable), the history after the step beta[s] and the
 * status fixed[s] (both nullable).  Returns the step at which the envelope was
 * fixed, or -1. */
int orc_path_relax(const orc_material* mat, const orc_lamination* lam, int n_steps, const double* F_steps,
                   double beta0, int fixed0, double* W, double* P, double* beta, int* fixed);

#ifdef __cplusplus
}
#endif
#endif
