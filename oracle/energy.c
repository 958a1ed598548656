/*
 * Oracle, Section 2 of arXiv 2211.14318: the condensed incremental stress
 * potential W(F) of the (1-D) damage model and its derivative P = dW/dF.
 * Test infrastructure only (see r1_oracle.h).
 */
#include <math.h>
#include "r1_oracle.h"

/* Plane-strain embedding: the 3x3 gradient of a 2D state has G33 = 1. */
static void embed3(int d, const double* G, double F3[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            F3[i][j] = (i == j) ? 1.0 : 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            F3[i][j] = G[i * d + j];
}

/* Determinant of a 3x3 matrix by cofactor expansion along the first row. */
static double det3(double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* psi0_NH(C) = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2 with J = sqrt(I3)
 * (eq. 2.3, invariants of eq. 2.1).  W is taken as +inf where det F <= 0. */
double orc_psi0(const orc_material* mat, const double* G)
{
    double F3[3][3], C[3][3];
    embed3(mat->dim, G, F3);
    if (!(det3(F3) > 0.0))
        return INFINITY;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += F3[k][i] * F3[k][j];
            C[i][j] = s;
        }
    double I1 = C[0][0] + C[1][1] + C[2][2];
    double I3 = det3(C);
    double J = sqrt(I3);
    double lnJ = log(J);
    return 0.5 * mat->mu * (I1 - 3.0) - mat->mu * lnJ + 0.5 * mat->lambda * lnJ * lnJ;
}

/* D(beta) = D_inf (1 - exp(-beta/D0))  (Section 2, damage function). */
double orc_damage(const orc_material* mat, double beta)
{
    return mat->D_inf * (1.0 - exp(-beta / mat->D0));
}

/* Antiderivative of D: Dbar(beta) = D_inf (beta + D0 exp(-beta/D0)); its
 * constant of integration cancels in W. */
static double damage_antiderivative(const orc_material* mat, double beta)
{
    return mat->D_inf * (beta + mat->D0 * exp(-beta / mat->D0));
}

static double doublewell(int d, const double* G)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            if (i == 0 && j == 0) {
                double q = G[0] * G[0] - 1.0;
                s += q * q;
            } else {
                double e = G[i * d + j] - (i == j ? 1.0 : 0.0);
                s += e * e;
            }
        }
    return s;
}

/* Condensed incremental potential, eq. 2.9:
 *   W = psi(F, D) - psi(F_k, D_k) + beta D - beta_k D_k - Dbar + Dbar_k
 * with psi(F, D) = (1 - D(beta)) psi0(F) and beta = max(beta_k, psi0(F)), the
 * minimiser of eq. 2.8 for a non-decreasing D.  The F-independent constant
 * -psi(F_k, D_k) is dropped.  beta_n denotes beta_k, the previous step's value. */
double orc_energy(const orc_material* mat, const double* G, double beta_n)
{
    if (mat->model == ORC_MODEL_DOUBLEWELL)
        return doublewell(mat->dim, G);
    double p0 = orc_psi0(mat, G);
    if (isinf(p0))
        return INFINITY;
    double beta = p0 > beta_n ? p0 : beta_n;
    double D = orc_damage(mat, beta);
    double Dk = orc_damage(mat, beta_n);
    double psi = (1.0 - D) * p0;
    return psi + beta * D - beta_n * Dk
         - damage_antiderivative(mat, beta) + damage_antiderivative(mat, beta_n);
}

/* P = dW/dF (eq. 2.12).  dW/dpsi0 = 1 - D(max(beta_k, psi0)) on both branches of
 * the max, and d psi0/dF = mu F + (lambda ln J - mu) F^{-T}.  In 2D only the
 * in-plane block is returned (F33 = 1 is held fixed).  Returns 0, or -1 where
 * det F <= 0 (P is then filled with NaN). */
int orc_stress0(const orc_material* mat, const double* G, double beta_n, double* P)
{
    int d = mat->dim;
    if (mat->model == ORC_MODEL_DOUBLEWELL) {
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                if (i == 0 && j == 0)
                    P[0] = 4.0 * G[0] * (G[0] * G[0] - 1.0);
                else
                    P[i * d + j] = 2.0 * (G[i * d + j] - (i == j ? 1.0 : 0.0));
            }
        return 0;
    }
    double F3[3][3];
    embed3(d, G, F3);
    double J = det3(F3);
    if (!(J > 0.0)) {
        for (int i = 0; i < d * d; ++i)
            P[i] = NAN;
        return -1;
    }
    /* F^{-T}_{ij} = cof(F)_{ij} / J */
    double cof[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            cof[i][j] = F3[i1][j1] * F3[i2][j2] - F3[i1][j2] * F3[i2][j1];
        }
    double p0 = orc_psi0(mat, G);
    double beta = p0 > beta_n ? p0 : beta_n;
    double g = 1.0 - orc_damage(mat, beta);
    double lnJ = log(J);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            P[i * d + j] = g * (mat->mu * F3[i][j] + (mat->lambda * lnJ - mat->mu) * cof[i][j] / J);
    return 0;
}

/* A0 = d^2 W / dG dG, the nominal tangent moduli of Section 2 at a leaf of the
 * lamination tree (Algorithm 3 sums them like the stresses).  With W = g(psi0),
 * g'(psi) = 1 - D(max(beta_n, psi)) and g''(psi) = -D'(psi) while loading
 * (psi0 > beta_n, as in orc_stress0), 0 otherwise:
 *   A0_ijkl = g' d^2psi0/dG_ij dG_kl + g'' S_ij S_kl,
 *   S = dpsi0/dG = mu G + (lambda ln J - mu) G^{-T},
 *   d^2psi0/dG_ij dG_kl = mu d_ik d_jl + lambda G^{-T}_ij G^{-T}_kl
 *                         - (lambda ln J - mu) G^{-T}_il G^{-T}_kj
 * (d ln J / dG = G^{-T}, d G^{-T}_ij / dG_kl = -G^{-T}_il G^{-T}_kj).  In 2D the
 * indices run over the in-plane block of the plane-strain embedding.
 * A[(i*d+j)*d*d + k*d+l]; NaN where det G <= 0. */
int orc_tangent0(const orc_material* mat, const double* G, double beta_n, double* A)
{
    int d = mat->dim, dd = d * d;
    if (mat->model == ORC_MODEL_DOUBLEWELL) {
        for (int a = 0; a < dd * dd; ++a)
            A[a] = 0.0;
        for (int a = 0; a < dd; ++a)
            A[a * dd + a] = 2.0;
        A[0] = 12.0 * G[0] * G[0] - 4.0;
        return 0;
    }
    double F3[3][3];
    embed3(d, G, F3);
    double J = det3(F3);
    if (!(J > 0.0)) {
        for (int a = 0; a < dd * dd; ++a)
            A[a] = NAN;
        return -1;
    }
    double Finv_T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            Finv_T[i][j] = (F3[i1][j1] * F3[i2][j2] - F3[i1][j2] * F3[i2][j1]) / J;
        }
    double lnJ = log(J);
    double p0 = orc_psi0(mat, G);
    double beta = p0 > beta_n ? p0 : beta_n;
    double g1 = 1.0 - orc_damage(mat, beta);
    double g2 = p0 > beta_n ? -mat->D_inf / mat->D0 * exp(-p0 / mat->D0) : 0.0;
    double c = mat->lambda * lnJ - mat->mu;
    double S[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            S[i][j] = mat->mu * F3[i][j] + c * Finv_T[i][j];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            for (int k = 0; k < d; ++k)
                for (int l = 0; l < d; ++l) {
                    double h = (i == k && j == l ? mat->mu : 0.0)
                             + mat->lambda * Finv_T[i][j] * Finv_T[k][l]
                             - c * Finv_T[i][l] * Finv_T[k][j];
                    A[(i * d + j) * dd + k * d + l] = g1 * h + g2 * S[i][j] * S[k][l];
                }
    return 0;
}
