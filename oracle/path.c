/*
 * Oracle, material-point driver of the relax-then-fix procedure of the biaxial
 * test (Section 6.6) with the damage history of Section 2.  Test infrastructure
 * only (see r1_oracle.h).
 *
 * One point is driven through prescribed deformation gradients F_0, F_1, ...
 * (pseudo-time steps).  Its state is the history beta (the largest psi0 seen,
 * Section 2: beta_t = max over s <= t of psi0(F_s)) and whether its envelope has
 * been fixed.  At step s the incremental potential of eq. 2.9 is taken with the
 * history entering the step, beta_{s-1}, and relaxed by lamination (eq. 3.3 on
 * the given levels):
 *   - not yet fixed, and the envelope at F_s does not laminate (the centre is a
 *     hull vertex for the winning direction: W^k(F_s) = W(F_s), the convex
 *     regime): the step is elastic or damaging as in the unrelaxed model, and the
 *     history becomes max(beta_{s-1}, psi0(F_s));
 *   - not yet fixed, and it laminates: the non-convex regime is reached; the
 *     envelope, i.e. the relaxed potential with history beta_{s-1}, is fixed from
 *     this step on;
 *   - fixed: the fixed envelope, W^k(F_s) with the frozen history, is reused.
 * W and P at each step are the relaxed potential and its laminate stress
 * (eq. 5.2).  Points with det F <= 0 give W = +inf and leave the state as it is.
 */
#include <math.h>
#include <string.h>
#include "r1_oracle.h"

int orc_path_relax(const orc_material* mat, const orc_lamination* lam, int n_steps, const double* F_steps,
                   double beta0, int fixed0, double* W, double* P, double* beta, int* fixed)
{
    int d = mat->dim, dd = d * d;
    double b = beta0;
    int fx = fixed0 ? 1 : 0;
    int first = -1;
    orc_laminate tree[ORC_TREE_NODES];
    for (int s = 0; s < n_steps; ++s) {
        const double* F = F_steps + (size_t)s * (size_t)dd;
        double Ps[9];
        double w = orc_envelope(mat, lam, F, b, Ps, tree);
        if (!fx && isfinite(w)) {
            if (tree[0].i_minus != tree[0].i_plus) {
                fx = 1;
                first = s;
            } else {
                double psi = orc_psi0(mat, F);
                if (psi > b)
                    b = psi;
            }
        }
        W[s] = w;
        if (P)
            memcpy(P + (size_t)s * (size_t)dd, Ps, sizeof(double) * (size_t)dd);
        if (beta)
            beta[s] = b;
        if (fixed)
            fixed[s] = fx;
    }
    return first;
}
