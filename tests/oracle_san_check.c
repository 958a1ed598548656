/*
 * Host harness that drives every entry of the FP64 oracle (test infrastructure)
 * on small random inputs, built together with the oracle sources under
 * AddressSanitizer and UndefinedBehaviorSanitizer by the CPU tests: one-level
 * and two-level envelopes with stress, tree and tangent moduli in 2D and 3D for
 * both energies, tree evaluation, the hull routines on lines with inadmissible
 * samples, grid sweeps with carried quantities, interpolation, the
 * relax-then-fix driver and the MLP forward/backward.  Prints "ok" and a
 * checksum; any sanitizer report aborts.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include "r1_oracle.h"

static unsigned long long rs = 88172645463325252ull;
static double urand(void) {            /* uniform in [-1, 1) */
    rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
    return (double)(rs >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static void unit(int d, double* v) {
    double s = 0.0;
    for (int i = 0; i < d; ++i) { v[i] = urand(); s += v[i] * v[i]; }
    s = sqrt(s) + 1e-12;
    for (int i = 0; i < d; ++i) v[i] /= s;
}

static double sum = 0.0;
static long n_nonfinite = 0;
static void acc(double v) {            /* checksum of the finite results */
    if (isfinite(v)) sum += v; else ++n_nonfinite;
}

int main(void) {
    for (int dim = 2; dim <= 3; ++dim)
        for (int model = 0; model <= 2; model += 2) {
            orc_material mat = {dim, model, 1.0, 0.5, 0.9, 0.3};
            int nd0 = 5, nd1 = 3;
            double a0[5 * 3], b0[5 * 3], a1[3 * 3], b1[3 * 3];
            for (int m = 0; m < nd0; ++m) { unit(dim, a0 + m * dim); unit(dim, b0 + m * dim); }
            for (int m = 0; m < nd1; ++m) { unit(dim, a1 + m * dim); unit(dim, b1 + m * dim); }
            orc_lamination lam1 = {1, {{nd0, a0, b0, 21, 1.2}, {0, 0, 0, 3, 1.0}}};
            orc_lamination lam2 = {2, {{nd0, a0, b0, 9, 1.2}, {nd1, a1, b1, 11, 1.2}}};
            for (int p = 0; p < 6; ++p) {
                double F[9], P[9], A[81], P2[9], A2[81];
                for (int k = 0; k < dim * dim; ++k) F[k] = (k % (dim + 1) == 0 ? 1.0 : 0.0) + 0.35 * urand();
                if (p == 5) for (int k = 0; k < dim; ++k) F[k] = 0.0;   /* det F = 0 */
                double bn = 0.2 * (urand() + 1.0);
                orc_laminate tree[ORC_TREE_NODES];
                for (int depth = 1; depth <= 2; ++depth) {
                    const orc_lamination* lam = depth == 1 ? &lam1 : &lam2;
                    double W = orc_envelope_tangent(&mat, lam, F, bn, P, A, tree);
                    double We = orc_eval_tree_tangent(&mat, lam, F, bn, tree, P2, A2);
                    acc(W); acc(We); acc(P[0] + A[0] + P2[1] + A2[1]);
                }
                acc(orc_psi0(&mat, F));
            }
            /* batch and path driver */
            const int n = 7;
            double Fs[9 * 7], bns[7], Wb[7], Pb[9 * 7], Ab[81 * 7];
            orc_laminate trees[7 * ORC_TREE_NODES];
            for (int p = 0; p < n; ++p) {
                for (int k = 0; k < dim * dim; ++k) Fs[k * n + p] = (k % (dim + 1) == 0 ? 1.0 : 0.0) + 0.3 * urand();
                bns[p] = 0.1 * (urand() + 1.0);
            }
            orc_envelope_batch_tangent(&mat, &lam1, n, Fs, bns, Wb, Pb, Ab, trees);
            orc_envelope_batch(&mat, &lam2, n, Fs, bns, Wb, Pb, trees);
            for (int p = 0; p < n; ++p) acc(Wb[p]);
            double path[9 * 5], Wp[5], Pp[9 * 5], bp[5];
            int fx[5];
            for (int s = 0; s < 5; ++s)
                for (int k = 0; k < dim * dim; ++k) path[s * dim * dim + k] = (k % (dim + 1) == 0 ? 1.0 : 0.0) + 0.1 * s * urand();
            orc_path_relax(&mat, &lam1, 5, path, 0.01, 0, Wp, Pp, bp, fx);
            acc(Wp[0] + bp[4] + fx[4]);
        }
    /* hulls with inadmissible ends */
    for (int t = 0; t < 50; ++t) {
        int n = 3 + 2 * (t % 9), c = (n - 1) / 2, im, ip;
        double w[21], x[21], gap;
        int vert[21];
        for (int i = 0; i < n; ++i) { w[i] = urand(); x[i] = i; }
        if (t % 3 == 0) w[0] = INFINITY;
        if (t % 5 == 0) w[n - 1] = INFINITY;
        acc(orc_hull_at_centre(n, w, c, &im, &ip, &gap) + im + ip);
        acc(orc_convexify(n, x, w, vert));
    }
    /* grids */
    for (int dim = 2; dim <= 3; ++dim) {
        orc_grid g = {dim, {0}, {0}, 0.3};
        for (int k = 0; k < dim * dim; ++k) { g.n[k] = (dim == 2 ? 5 : 2) + (k % 2); g.lo[k] = (k % (dim + 1) == 0) ? 0.5 : -0.3; }
        long N = orc_grid_size(&g);
        int steps[169 * 9];
        int nd = orc_grid_r11(dim, steps);
        double* W = malloc(sizeof(double) * N);
        double* W2 = malloc(sizeof(double) * N);
        double* C = malloc(sizeof(double) * N * 3);
        double* C2 = malloc(sizeof(double) * N * 3);
        double hist[4];
        orc_material mat = {dim, 0, 1.0, 0.5, 0.9, 0.3};
        orc_grid_energy(&mat, &g, 0.04, W, NULL, NULL);
        for (long p = 0; p < N * 3; ++p) C[p] = urand();
        acc(orc_grid_sweep(&g, nd, steps, W, W2, 3, C, C2));
        acc(orc_grid_update_node(&g, nd, steps, W, N / 2));
        acc(orc_grid_laminate(&g, nd, steps, W, 3, C, 4, 0.0, hist));
        double F[9];
        orc_grid_node(&g, N / 3, F);
        F[0] += 0.1;
        double v = orc_grid_interpolate(&g, W, F);
        acc(v);
        free(W); free(W2); free(C); free(C2);
    }
    /* MLP */
    {
        int din = 5, w = 16, nh = 3, dout = 5;
        long np = orc_mlp_param_count(din, w, nh, dout);
        double* prm = malloc(sizeof(double) * np);
        double* grad = malloc(sizeof(double) * np);
        double x[4 * 5], y[4 * 5], out[4 * 5];
        for (long i = 0; i < np; ++i) prm[i] = 0.3 * urand();
        for (int i = 0; i < 20; ++i) { x[i] = urand(); y[i] = urand(); }
        acc(orc_mlp_forward(din, w, nh, dout, prm, 4, x, y, out));
        acc(orc_mlp_loss_grad(din, w, nh, dout, prm, 4, x, y, grad) + grad[0]);
        free(prm); free(grad);
    }
    printf("ok %.6e (%ld non-finite results)\n", sum, n_nonfinite);
    return 0;
}
