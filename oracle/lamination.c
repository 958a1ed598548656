/*
 * Oracle, successive lamination (Section 3.1, eq. 3.3) evaluated along the
 * discrete lines of Section 4.1 (eq. 4.4) through one point, with the
 * laminate-endpoint derivative of Section 5.3 (eq. 5.2, first case;
 * Algorithms 2 and 3 for a binary tree).  Test infrastructure only.
 *
 *   W^0 = W;   W^{l}(G) = min_m  hull_i[ W^{l-1}(G + t_i R_m) ](t = 0)
 *
 * where hull_i[.](t = 0) is the lower convex hull of the finite line samples
 * (Algorithm 1) read at the centre sample, and R_m = a_m (x) b_m.
 * Stress:  P^l(G) = xi P^{l-1}(G^+) + (1 - xi) P^{l-1}(G^-),  G^{+/-} = G + t_{i+/-} R_{m*},
 * xi = (c - i_minus)/(i_plus - i_minus), and P^0 = dW/dF; the tangent moduli
 * A^l follow the same recursion with A^0 = d^2 W / dF dF (Algorithm 3).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "r1_oracle.h"

double orc_tgrid(const orc_level* lv, int i)
{
    return lv->tau * (double)(2 * i - (lv->n_t - 1)) / (double)(lv->n_t - 1);
}

/* G + t * a (x) b */
static void line_point(int d, const double* G, const double* a, const double* b, double t, double* out)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            out[i * d + j] = G[i * d + j] + t * a[i] * b[j];
}

/* W^{depth - ell}(G) where ell counts levels from the outermost (0) and the
 * levels ell..depth-1 remain to be applied.  Fills node `node` of the tree and
 * its descendants when tree != NULL, the stress when P != NULL and the tangent
 * moduli when A != NULL. */
static double level_value(const orc_material* mat, const orc_lamination* lam, int ell,
                          const double* G, double beta_n, double* P, double* A, orc_laminate* tree,
                          int node)
{
    int d = mat->dim;
    if (ell == lam->depth) {
        if (P)
            orc_stress0(mat, G, beta_n, P);
        if (A)
            orc_tangent0(mat, G, beta_n, A);
        return orc_energy(mat, G, beta_n);
    }
    const orc_level* lv = &lam->level[ell];
    int n = lv->n_t, c = (n - 1) / 2;
    double* w = (double*)orc_alloc(sizeof(double) * (size_t)n);
    double Gi[9];
    double best = INFINITY, second = INFINITY, best_gap = INFINITY;
    double vertex_gap = INFINITY;   /* how close any direction is to laminating */
    int best_m = 0, best_im = c, best_ip = c;
    /* the centre sample is G itself for every direction */
    double wc = level_value(mat, lam, ell + 1, G, beta_n, NULL, NULL, NULL, 0);
    for (int m = 0; m < lv->n_dir; ++m) {
        const double* a = lv->a + m * d;
        const double* b = lv->b + m * d;
        for (int i = 0; i < n; ++i) {
            if (i == c) { w[i] = wc; continue; }
            line_point(d, G, a, b, orc_tgrid(lv, i), Gi);
            w[i] = level_value(mat, lam, ell + 1, Gi, beta_n, NULL, NULL, NULL, 0);
        }
        int im, ip;
        double gap;
        double h = orc_hull_at_centre(n, w, c, &im, &ip, tree ? &gap : NULL);
        if (tree && im == ip && gap < vertex_gap)
            vertex_gap = gap;
        if (h < best) {
            second = best;
            best = h; best_m = m; best_im = im; best_ip = ip;
            best_gap = tree ? gap : INFINITY;
        } else if (h < second) {
            second = h;
        }
    }
    free(w);
    if (!isfinite(best)) {
        /* det G <= 0: the whole line set is inadmissible */
        if (P) for (int i = 0; i < d * d; ++i) P[i] = NAN;
        if (A) for (int i = 0; i < d * d * d * d; ++i) A[i] = NAN;
        if (tree) {
            orc_laminate* t = &tree[node];
            t->dir = 0; t->i_minus = t->i_plus = c; t->xi = 1.0; t->value = INFINITY;
            t->dir_gap = INFINITY; t->bridge_gap = INFINITY;
        }
        return INFINITY;
    }
    double xi = (best_im == best_ip) ? 1.0 : (double)(c - best_im) / (double)(best_ip - best_im);
    if (tree) {
        orc_laminate* t = &tree[node];
        t->dir = best_m; t->i_minus = best_im; t->i_plus = best_ip; t->xi = xi;
        t->value = best;
        if (best_im == best_ip) {
            /* no lamination: every direction reads W(G) at its centre, so equal
             * runner-up values change nothing; the result is fragile only if some
             * direction's centre is close to losing its vertex status */
            t->dir_gap = INFINITY;
            t->bridge_gap = vertex_gap;
        } else {
            t->dir_gap = second - best;
            t->bridge_gap = best_gap;
        }
    }
    if (P || A || tree) {
        const double* a = lv->a + best_m * d;
        const double* b = lv->b + best_m * d;
        double Gm[9], Gp[9], Pm[9], Pp[9], Am[81], Ap[81];
        line_point(d, G, a, b, orc_tgrid(lv, best_im), Gm);
        line_point(d, G, a, b, orc_tgrid(lv, best_ip), Gp);
        level_value(mat, lam, ell + 1, Gm, beta_n, P ? Pm : NULL, A ? Am : NULL, tree, 2 * node + 1);
        level_value(mat, lam, ell + 1, Gp, beta_n, P ? Pp : NULL, A ? Ap : NULL, tree, 2 * node + 2);
        if (P)
            for (int i = 0; i < d * d; ++i)
                P[i] = xi * Pp[i] + (1.0 - xi) * Pm[i];
        if (A)
            for (int i = 0; i < d * d * d * d; ++i)
                A[i] = xi * Ap[i] + (1.0 - xi) * Am[i];
    }
    return best;
}

double orc_envelope(const orc_material* mat, const orc_lamination* lam,
                    const double* F, double beta_n, double* P, orc_laminate* tree)
{
    return level_value(mat, lam, 0, F, beta_n, P, NULL, tree, 0);
}

double orc_envelope_tangent(const orc_material* mat, const orc_lamination* lam,
                            const double* F, double beta_n, double* P, double* A, orc_laminate* tree)
{
    return level_value(mat, lam, 0, F, beta_n, P, A, tree, 0);
}

/* Algorithm 3 on a given binary lamination tree. */
static double tree_value(const orc_material* mat, const orc_lamination* lam, int ell,
                         const double* G, double beta_n, const orc_laminate* tree, int node, double* P,
                         double* A)
{
    int d = mat->dim;
    if (ell == lam->depth) {
        if (P)
            orc_stress0(mat, G, beta_n, P);
        if (A)
            orc_tangent0(mat, G, beta_n, A);
        return orc_energy(mat, G, beta_n);
    }
    const orc_level* lv = &lam->level[ell];
    int c = (lv->n_t - 1) / 2;
    const orc_laminate* t = &tree[node];
    const double* a = lv->a + t->dir * d;
    const double* b = lv->b + t->dir * d;
    int im = t->i_minus, ip = t->i_plus;
    double xi = (im == ip) ? 1.0 : (double)(c - im) / (double)(ip - im);
    double Gm[9], Gp[9], Pm[9], Pp[9], Am[81], Ap[81];
    line_point(d, G, a, b, orc_tgrid(lv, im), Gm);
    line_point(d, G, a, b, orc_tgrid(lv, ip), Gp);
    double wm = tree_value(mat, lam, ell + 1, Gm, beta_n, tree, 2 * node + 1, P ? Pm : NULL, A ? Am : NULL);
    double wp = tree_value(mat, lam, ell + 1, Gp, beta_n, tree, 2 * node + 2, P ? Pp : NULL, A ? Ap : NULL);
    if (P)
        for (int i = 0; i < d * d; ++i)
            P[i] = xi * Pp[i] + (1.0 - xi) * Pm[i];
    if (A)
        for (int i = 0; i < d * d * d * d; ++i)
            A[i] = xi * Ap[i] + (1.0 - xi) * Am[i];
    if (im == ip)
        return wp;
    return xi * wp + (1.0 - xi) * wm;
}

double orc_eval_tree(const orc_material* mat, const orc_lamination* lam,
                     const double* F, double beta_n, const orc_laminate* tree, double* P)
{
    return tree_value(mat, lam, 0, F, beta_n, tree, 0, P, NULL);
}

double orc_eval_tree_tangent(const orc_material* mat, const orc_lamination* lam,
                             const double* F, double beta_n, const orc_laminate* tree, double* P,
                             double* A)
{
    return tree_value(mat, lam, 0, F, beta_n, tree, 0, P, A);
}

void orc_envelope_batch(const orc_material* mat, const orc_lamination* lam, long n,
                        const double* F, const double* beta_n, double* W, double* P,
                        orc_laminate* trees)
{
    int d = mat->dim, dd = d * d;
    double G[9], Pp[9];
    for (long p = 0; p < n; ++p) {
        for (int k = 0; k < dd; ++k)
            G[k] = F[(long)k * n + p];
        W[p] = orc_envelope(mat, lam, G, beta_n[p], P ? Pp : NULL,
                            trees ? trees + p * ORC_TREE_NODES : NULL);
        if (P)
            for (int k = 0; k < dd; ++k)
                P[(long)k * n + p] = Pp[k];
    }
}

void orc_envelope_batch_tangent(const orc_material* mat, const orc_lamination* lam, long n,
                                const double* F, const double* beta_n, double* W, double* P,
                                double* A, orc_laminate* trees)
{
    int d = mat->dim, dd = d * d;
    double G[9], Pp[9], Ap[81];
    for (long p = 0; p < n; ++p) {
        for (int k = 0; k < dd; ++k)
            G[k] = F[(long)k * n + p];
        W[p] = orc_envelope_tangent(mat, lam, G, beta_n[p], P ? Pp : NULL, A ? Ap : NULL,
                                    trees ? trees + p * ORC_TREE_NODES : NULL);
        if (P)
            for (int k = 0; k < dd; ++k)
                P[(long)k * n + p] = Pp[k];
        if (A)
            for (int k = 0; k < dd * dd; ++k)
                A[(long)k * n + p] = Ap[k];
    }
}
