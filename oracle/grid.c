/*
 * Oracle, Section 4.1 of arXiv 2211.14318: global rank-one lamination on a
 * deformation-gradient mesh.  The mesh is the per-component cuboid of Section
 * 5.2 with one mesh width delta for every component (the setting of all the
 * paper's examples, Tables 6.1-6.3); the iteration is eq. 4.3: every node is
 * updated from the previous iterate by the 1D lower hull (Algorithm 1) of the
 * line through it (eq. 4.4, clipped to the mesh's box), minimised over the
 * directions; the stopping rule is that of Section 6.
 *
 * A direction is an integer step s in Z^{d x d} (s = a (x) b for the reduced set
 * of eq. 5.1, a, b in {-1, 0, 1}^d): the line through node F holds the nodes
 * F + l delta s, l integer, inside the box.  Non-finite node values are absent
 * from a hull; a node that is itself non-finite stays so.
 *
 * Test infrastructure only (see r1_oracle.h).
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "r1_oracle.h"

long orc_grid_size(const orc_grid* g)
{
    long n = 1;
    for (int c = 0; c < g->dim * g->dim; ++c)
        n *= g->n[c];
    return n;
}

/* Multi-index of node p: component 0 varies slowest. */
static void unflatten(const orc_grid* g, long p, int* I)
{
    for (int c = g->dim * g->dim - 1; c >= 0; --c) {
        I[c] = (int)(p % g->n[c]);
        p /= g->n[c];
    }
}

static long flatten(const orc_grid* g, const int* I)
{
    long p = 0;
    for (int c = 0; c < g->dim * g->dim; ++c)
        p = p * g->n[c] + I[c];
    return p;
}

void orc_grid_node(const orc_grid* g, long p, double* F)
{
    int I[9];
    unflatten(g, p, I);
    for (int c = 0; c < g->dim * g->dim; ++c)
        F[c] = g->lo[c] + I[c] * g->delta;
}

/* The reduced direction set of eq. 5.1: a (x) b for a, b in {-1, 0, 1}^d,
 * both non-zero; s and -s give the same line, so each pair is kept once (the
 * one whose first non-zero entry is positive), in the order of first
 * appearance.  Returns the count; steps holds count x d*d integers. */
int orc_grid_r11(int dim, int* steps)
{
    int dd = dim * dim, count = 0, na = 1;
    for (int i = 0; i < dim; ++i)
        na *= 3;
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < na; ++ib) {
            int a[3], b[3], r = ia, q = ib, az = 1, bz = 1;
            for (int i = dim - 1; i >= 0; --i) {
                a[i] = r % 3 - 1; r /= 3;
                b[i] = q % 3 - 1; q /= 3;
                az &= a[i] == 0;
                bz &= b[i] == 0;
            }
            if (az || bz)
                continue;
            int s[9], first = 0;
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j)
                    s[i * dim + j] = a[i] * b[j];
            for (int c = 0; c < dd && !first; ++c)
                first = s[c];
            if (first < 0)
                for (int c = 0; c < dd; ++c)
                    s[c] = -s[c];
            int dup = 0;
            for (int m = 0; m < count && !dup; ++m)
                dup = memcmp(steps + m * dd, s, sizeof(int) * (size_t)dd) == 0;
            if (!dup) {
                memcpy(steps + count * dd, s, sizeof(int) * (size_t)dd);
                ++count;
            }
        }
    return count;
}

/* W^0 = W at every node; if P != NULL, P^0 = dW/dF (eq. 2.12), component-major
 * P[c * nodes + p]; if A != NULL, the moduli d^2W/dF dF (orc_tangent0),
 * A[c * nodes + p] with c = (i*d + j)*d*d + k*d + l. */
void orc_grid_energy(const orc_material* mat, const orc_grid* g, double beta_n, double* W, double* P,
                     double* A)
{
    long n = orc_grid_size(g);
    int dd = g->dim * g->dim;
    double F[9], S[9], T[81];
    for (long p = 0; p < n; ++p) {
        orc_grid_node(g, p, F);
        W[p] = orc_energy(mat, F, beta_n);
        if (P) {
            orc_stress0(mat, F, beta_n, S);
            for (int c = 0; c < dd; ++c)
                P[c * n + p] = S[c];
        }
        if (A) {
            orc_tangent0(mat, F, beta_n, T);
            for (int c = 0; c < dd * dd; ++c)
                A[c * n + p] = T[c];
        }
    }
}

/* One iteration of eq. 4.3.  For each direction, every line of the mesh
 * (its nodes in order of l) is convexified by Algorithm 1 and each node of the
 * line reads the hull at its own position; Wout is the
 * minimum over directions, starting from Win (every node is a sample of each of
 * its lines; a non-finite node stays so).  Returns max over nodes with finite
 * Win of Win - Wout.
 *
 * A hull value replaces the node's current value only when it is lower by more
 * than four units of rounding, 4 eps max(|W|, 1e-3): a node on a straight hull
 * run reads its own value back up to rounding, which is no lamination, and of
 * directions that tie to rounding the first keeps the node.
 *
 * Cin/Cout (nullable) hold m per-node quantities, component-major C[c * nodes + p]
 * -- the stresses (eq. 5.2, first case) and the tangent moduli (Algorithm 3) --
 * that the laminate lowering a node carries: a node q inside the hull segment
 * [a, b] takes ((b - q) C_a + (q - a) C_b) / (b - a), the weights of its value. */
double orc_grid_sweep(const orc_grid* g, int n_dir, const int* steps, const double* Win, double* Wout, int m,
                      const double* Cin, double* Cout)
{
    const int dd = g->dim * g->dim;
    const long n = orc_grid_size(g);
    int maxlen = 1;
    for (int c = 0; c < dd; ++c)
        if (g->n[c] > maxlen)
            maxlen = g->n[c];
    long* node = (long*)orc_alloc(sizeof(long) * (size_t)maxlen);
    double* w = (double*)orc_alloc(sizeof(double) * (size_t)maxlen);
    double* x = (double*)orc_alloc(sizeof(double) * (size_t)maxlen);
    double* v = (double*)orc_alloc(sizeof(double) * (size_t)maxlen);
    int* vert = (int*)orc_alloc(sizeof(int) * (size_t)maxlen);
    memcpy(Wout, Win, sizeof(double) * (size_t)n);
    if (Cin && Cout)
        memcpy(Cout, Cin, sizeof(double) * (size_t)n * (size_t)m);
    for (int r = 0; r < n_dir; ++r) {
        const int* s = steps + r * dd;
        int zero = 1;
        for (int c = 0; c < dd; ++c)
            zero &= s[c] == 0;
        if (zero)
            continue;
        for (long p = 0; p < n; ++p) {
            int I[9], J[9], start = 0;
            unflatten(g, p, I);
            /* p starts a line when the node one step back lies outside the box */
            for (int c = 0; c < dd; ++c) {
                int y = I[c] - s[c];
                if (y < 0 || y >= g->n[c])
                    start = 1;
            }
            if (!start)
                continue;
            int L = 0;
            memcpy(J, I, sizeof(J));
            for (;;) {
                int inside = 1;
                for (int c = 0; c < dd; ++c)
                    if (J[c] < 0 || J[c] >= g->n[c])
                        inside = 0;
                if (!inside)
                    break;
                node[L] = flatten(g, J);
                w[L] = Win[node[L]];
                ++L;
                for (int c = 0; c < dd; ++c)
                    J[c] += s[c];
            }
            /* Algorithm 1 on the line's finite samples; a node strictly inside a
             * hull segment [a, b] reads ((b - q) w_a + (q - a) w_b) / (b - a) */
            int Lf = 0;
            for (int q = 0; q < L; ++q)
                if (isfinite(w[q])) {
                    x[Lf] = (double)q;
                    v[Lf] = w[q];
                    ++Lf;
                }
            int nv = orc_convexify(Lf, x, v, vert);
            for (int k = 0; k + 1 < nv; ++k) {
                int a = (int)x[vert[k]], b = (int)x[vert[k + 1]];
                for (int q = a + 1; q < b; ++q) {
                    if (!isfinite(w[q]))
                        continue;
                    double val = ((double)(b - q) * w[a] + (double)(q - a) * w[b]) / (double)(b - a);
                    double cur = Wout[node[q]];
                    if (val < cur - 4.0 * DBL_EPSILON * fmax(fabs(cur), 1e-3)) {
                        Wout[node[q]] = val;
                        if (Cin && Cout)
                            for (int c = 0; c < m; ++c)
                                Cout[c * n + node[q]] = ((double)(b - q) * Cin[c * n + node[a]] +
                                                         (double)(q - a) * Cin[c * n + node[b]]) / (double)(b - a);
                    }
                }
            }
        }
    }
    free(node);
    free(w);
    free(x);
    free(v);
    free(vert);
    double md = 0.0;
    for (long p = 0; p < n; ++p)
        if (isfinite(Win[p]) && Win[p] - Wout[p] > md)
            md = Win[p] - Wout[p];
    return md;
}

/* Eq. 4.3 at one node p: the minimum over directions of the lower hull of the
 * line through p read at p (orc_hull_at_centre), and W[p] itself. */
double orc_grid_update_node(const orc_grid* g, int n_dir, const int* steps, const double* W, long p)
{
    const int dd = g->dim * g->dim;
    int maxlen = 1;
    for (int c = 0; c < dd; ++c)
        if (g->n[c] > maxlen)
            maxlen = g->n[c];
    double* w = (double*)orc_alloc(sizeof(double) * (size_t)(2 * maxlen + 1));
    int I[9];
    unflatten(g, p, I);
    double best = W[p];
    for (int m = 0; m < n_dir && isfinite(best); ++m) {
        const int* s = steps + m * dd;
        int lo = -2 * maxlen, hi = 2 * maxlen;
        for (int c = 0; c < dd; ++c) {
            if (s[c] > 0) {
                int a = -I[c] / s[c], b = (g->n[c] - 1 - I[c]) / s[c];
                if (a > lo) lo = a;
                if (b < hi) hi = b;
            } else if (s[c] < 0) {
                int a = -(g->n[c] - 1 - I[c]) / (-s[c]), b = I[c] / (-s[c]);
                if (a > lo) lo = a;
                if (b < hi) hi = b;
            }
        }
        if (lo == -2 * maxlen)
            continue;                       /* the zero step */
        int L = 0, J[9];
        for (int l = lo; l <= hi; ++l) {
            for (int c = 0; c < dd; ++c)
                J[c] = I[c] + l * s[c];
            w[L++] = W[flatten(g, J)];
        }
        int im, ip;
        double v = orc_hull_at_centre(L, w, -lo, &im, &ip, NULL);
        if (v < best)
            best = v;
    }
    free(w);
    return best;
}

/* Iterates eq. 4.3 in place until the maximal decrease of an iteration is at
 * most tol or k_max iterations are done (Section 6).  hist[k-1] receives the
 * maximal decrease of iteration k.  C (nullable): m per-node quantities carried
 * along (see orc_grid_sweep).  Returns the number of iterations done. */
int orc_grid_laminate(const orc_grid* g, int n_dir, const int* steps, double* W, int m, double* C, int k_max,
                      double tol, double* hist)
{
    long n = orc_grid_size(g);
    size_t np = C ? (size_t)n * (size_t)m : 0;
    double* next = (double*)orc_alloc(sizeof(double) * (size_t)n);
    double* pnext = C ? (double*)orc_alloc(sizeof(double) * np) : NULL;
    int k = 0;
    while (k < k_max) {
        double md = orc_grid_sweep(g, n_dir, steps, W, next, m, C, pnext);
        memcpy(W, next, sizeof(double) * (size_t)n);
        if (C)
            memcpy(C, pnext, sizeof(double) * np);
        hist[k++] = md;
        if (md <= tol)
            break;
    }
    free(next);
    free(pnext);
    return k;
}

/* Off-mesh values by multilinear interpolation of the node values (Section 4.1):
 * the weights of the 2^{d*d} corners of F's cell are products of the per-
 * component fractions; corners of zero weight do not take part.  NaN outside
 * the box (beyond a rounding margin of 1e-9 mesh widths). */
double orc_grid_interpolate(const orc_grid* g, const double* W, const double* F)
{
    const int dd = g->dim * g->dim;
    int base[9];
    double frac[9];
    for (int c = 0; c < dd; ++c) {
        double u = (F[c] - g->lo[c]) / g->delta;
        /* points on the box's faces may round to just outside it */
        if (!(u >= -1e-9 && u <= (double)(g->n[c] - 1) + 1e-9))
            return NAN;
        u = u < 0.0 ? 0.0 : u > (double)(g->n[c] - 1) ? (double)(g->n[c] - 1) : u;
        int i = (int)floor(u);
        if (i > g->n[c] - 2)
            i = g->n[c] - 2;
        if (i < 0)
            i = 0;
        base[c] = i;
        frac[c] = g->n[c] > 1 ? u - i : 0.0;
    }
    double sum = 0.0;
    for (long corner = 0; corner < (1L << dd); ++corner) {
        double wgt = 1.0;
        int I[9];
        for (int c = 0; c < dd; ++c) {
            int up = (int)((corner >> (dd - 1 - c)) & 1);
            if (up && g->n[c] == 1) { wgt = 0.0; break; }
            I[c] = base[c] + up;
            wgt *= up ? frac[c] : 1.0 - frac[c];
        }
        if (wgt == 0.0)
            continue;
        sum += wgt * W[flatten(g, I)];
    }
    return sum;
}
