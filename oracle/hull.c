/*
 * Oracle, Section 4.2 of arXiv 2211.14318: one-dimensional convexification
 * (Algorithm 1, "convexify") and the value of the hull at the line's centre.
 * Test infrastructure only (see r1_oracle.h).
 *
 * Reading of the printed algorithm: its initialisation assigns w to y where x
 * is meant (y holds abscissae, c values); the loop guard must read "n >= 2"
 * and be tested before the orientation test (otherwise y[n-1] is read at
 * n = 1); arrays run over L entries.  The orientation test pops the last
 * vertex when the new point lies on or below the line through the last two
 * vertices, so collinear points are not kept and a flat hull segment is
 * represented by its outermost points.
 */
#include <math.h>
#include <stdlib.h>
#include "r1_oracle.h"

int orc_convexify(int L, const double* x, const double* w, int* vert)
{
    if (L <= 0)
        return 0;
    if (L == 1) {
        vert[0] = 0;
        return 1;
    }
    /* y[k], c[k]: abscissa and value of hull vertex k (0-based, n entries) */
    double* y = (double*)orc_alloc(sizeof(double) * (size_t)L);
    double* c = (double*)orc_alloc(sizeof(double) * (size_t)L);
    y[0] = x[0]; c[0] = w[0]; vert[0] = 0;
    y[1] = x[1]; c[1] = w[1]; vert[1] = 1;
    int n = 2;
    for (int i = 2; i < L; ++i) {
        while (n >= 2 &&
               (c[n - 1] - c[n - 2]) * (x[i] - y[n - 1]) >= (w[i] - c[n - 1]) * (y[n - 1] - y[n - 2]))
            n -= 1;
        y[n] = x[i]; c[n] = w[i]; vert[n] = i;
        n += 1;
    }
    free(y);
    free(c);
    return n;
}

/* Hull value at index c from the lower hull of the finite samples: linear
 * interpolation between the vertices that bracket c (Section 4.2, last
 * paragraph of the one-dimensional convexification). */
double orc_hull_at_centre(int n, const double* w, int c, int* i_minus, int* i_plus,
                          double* bridge_gap)
{
    int* idx = (int*)orc_alloc(sizeof(int) * (size_t)n);
    double* x = (double*)orc_alloc(sizeof(double) * (size_t)n);
    double* v = (double*)orc_alloc(sizeof(double) * (size_t)n);
    int* vert = (int*)orc_alloc(sizeof(int) * (size_t)n);
    int L = 0;
    for (int i = 0; i < n; ++i)
        if (isfinite(w[i])) {
            idx[L] = i; x[L] = (double)i; v[L] = w[i]; ++L;
        }
    double value = INFINITY;
    int im = c, ip = c;
    double gap = INFINITY;
    if (L > 0 && isfinite(w[c])) {
        int nv = orc_convexify(L, x, v, vert);
        /* the segment [vert[k], vert[k+1]] containing c, or the vertex at c */
        for (int k = 0; k < nv; ++k) {
            int ik = idx[vert[k]];
            if (ik == c) { im = ip = c; break; }
            if (k + 1 < nv && ik < c && idx[vert[k + 1]] > c) {
                im = ik; ip = idx[vert[k + 1]]; break;
            }
        }
        if (im == ip) {
            value = w[c];
            /* robustness of the vertex: hull value at c without sample c */
            if (bridge_gap) {
                int L2 = 0;
                for (int k = 0; k < L; ++k)
                    if (idx[k] != c) { x[L2] = (double)idx[k]; v[L2] = w[idx[k]]; ++L2; }
                if (L2 >= 2 && x[0] < c && x[L2 - 1] > c) {
                    int nv2 = orc_convexify(L2, x, v, vert);
                    for (int k = 0; k + 1 < nv2; ++k) {
                        double xa = x[vert[k]], xb = x[vert[k + 1]];
                        if (xa < c && xb > c) {
                            double hv = ((xb - c) * v[vert[k]] + (c - xa) * v[vert[k + 1]]) / (xb - xa);
                            gap = hv - w[c];
                            break;
                        }
                    }
                }
            }
        } else {
            double dx = (double)(ip - im);
            value = ((double)(ip - c) * w[im] + (double)(c - im) * w[ip]) / dx;
            if (bridge_gap) {
                double slope = (w[ip] - w[im]) / dx;
                for (int k = 0; k < L; ++k) {
                    int i = idx[k];
                    if (i == im || i == ip) continue;
                    double d = w[i] - (w[im] + slope * (double)(i - im));
                    if (d < gap) gap = d;
                }
            }
        }
    }
    if (i_minus) *i_minus = im;
    if (i_plus) *i_plus = ip;
    if (bridge_gap) *bridge_gap = gap;
    free(idx); free(x); free(v); free(vert);
    return value;
}
