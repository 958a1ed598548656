/*
 * Oracle, Section 2 of arXiv 2211.14318: the condensed incremental stress
 * potential W(F) of the (1-D) damage model and its derivative P = dW/dF.
 * Test infrastructure only (see r1_oracle.h).
 */
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>
#include "r1_oracle.h"

void* orc_alloc(size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "oracle: cannot allocate %zu bytes\n", bytes);
        abort();
    }
    return p;
}

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

/* C = F^T F of the 3x3 embedding. */
static void right_cauchy_green(double F3[3][3], double C[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += F3[k][i] * F3[k][j];
            C[i][j] = s;
        }
}

/* I1 = tr C and I2 = tr Cof C = ((tr C)^2 - tr(C^2)) / 2 (eq. 2.1). */
static void invariants12(double C[3][3], double* I1, double* I2)
{
    double t = C[0][0] + C[1][1] + C[2][2], t2 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            t2 += C[i][j] * C[j][i];
    *I1 = t;
    *I2 = 0.5 * (t * t - t2);
}

/* St. Venant-Kirchhoff, eq. 2.2: psi0 = lambda/8 (I1 - 3)^2 + mu/4 (I1^2 - 2 I1 - 2 I2 + 3),
 * and its derivatives in the invariants: dpsi0/dI1 = lambda/4 (I1 - 3) + mu/2 (I1 - 1),
 * dpsi0/dI2 = -mu/2, d^2psi0/dI1^2 = lambda/4 + mu/2 (the others vanish).  Defined for
 * every F (no constraint on det F). */
static double stvk_psi0(const orc_material* mat, double I1, double I2)
{
    double a = I1 - 3.0;
    return mat->lambda / 8.0 * a * a + mat->mu / 4.0 * (I1 * I1 - 2.0 * I1 - 2.0 * I2 + 3.0);
}

/* psi0 of the material model.  Neo-Hooke (eq. 2.3): mu/2 (I1 - 3) - mu ln J +
 * lambda/2 (ln J)^2 with J = sqrt(I3); W is taken as +inf where det F <= 0.
 * St. Venant-Kirchhoff: eq. 2.2, finite everywhere. */
double orc_psi0(const orc_material* mat, const double* G)
{
    double F3[3][3], C[3][3];
    embed3(mat->dim, G, F3);
    if (mat->model == ORC_MODEL_STVK_DAMAGE) {
        double I1, I2;
        right_cauchy_green(F3, C);
        invariants12(C, &I1, &I2);
        return stvk_psi0(mat, I1, I2);
    }
    if (!(det3(F3) > 0.0))
        return INFINITY;
    right_cauchy_green(F3, C);
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

/* St. Venant-Kirchhoff: S = dpsi0/dF = psi_1 dI1/dF + psi_2 dI2/dF with
 * dI1/dF = 2F and dI2/dF = 2 (I1 F - F C) (psi_a = dpsi0/dI_a), and, if H != NULL,
 * H[(i*3+j)*9 + k*3+l] = d^2psi0/dF_ij dF_kl
 *   = 4 psi_11 F_ij F_kl + 2 psi_1 d_ik d_jl + psi_2 d^2I2/dF_ij dF_kl,
 *   d^2I2/dF_ij dF_kl = 2 (2 F_ij F_kl + I1 d_ik d_jl - d_ik C_lj - F_il F_kj - B_ik d_jl),
 * with B = F F^T, on the 3x3 embedding (2D takes the in-plane entries). */
static void stvk_dpsi0(const orc_material* mat, double F3[3][3], double S[3][3], double* H)
{
    double C[3][3], B[3][3], FC[3][3], I1, I2;
    right_cauchy_green(F3, C);
    invariants12(C, &I1, &I2);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double b = 0.0, fc = 0.0;
            for (int k = 0; k < 3; ++k) {
                b += F3[i][k] * F3[j][k];
                fc += F3[i][k] * C[k][j];
            }
            B[i][j] = b;
            FC[i][j] = fc;
        }
    double psi1 = mat->lambda / 4.0 * (I1 - 3.0) + mat->mu / 2.0 * (I1 - 1.0);
    double psi2 = -mat->mu / 2.0;
    double psi11 = mat->lambda / 4.0 + mat->mu / 2.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            S[i][j] = 2.0 * psi1 * F3[i][j] + psi2 * 2.0 * (I1 * F3[i][j] - FC[i][j]);
    if (!H)
        return;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double dik = i == k, djl = j == l;
                    double d2I2 = 2.0 * (2.0 * F3[i][j] * F3[k][l] + I1 * dik * djl - dik * C[l][j]
                                         - F3[i][l] * F3[k][j] - B[i][k] * djl);
                    H[(i * 3 + j) * 9 + k * 3 + l] = 4.0 * psi11 * F3[i][j] * F3[k][l]
                                                   + 2.0 * psi1 * dik * djl + psi2 * d2I2;
                }
}

/* P = dW/dF (eq. 2.12).  dW/dpsi0 = 1 - D(max(beta_k, psi0)) on both branches of
 * the max, and d psi0/dF = mu F + (lambda ln J - mu) F^{-T} (neo-Hooke; St.
 * Venant-Kirchhoff: stvk_dpsi0).  In 2D only the
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
    if (mat->model == ORC_MODEL_STVK_DAMAGE) {
        double S[3][3];
        stvk_dpsi0(mat, F3, S, NULL);
        double p0 = orc_psi0(mat, G);
        double g = 1.0 - orc_damage(mat, p0 > beta_n ? p0 : beta_n);
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                P[i * d + j] = g * S[i][j];
        return 0;
    }
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
 * (d ln J / dG = G^{-T}, d G^{-T}_ij / dG_kl = -G^{-T}_il G^{-T}_kj) for neo-Hooke;
 * St. Venant-Kirchhoff takes S and the second derivative from stvk_dpsi0.  In 2D the
 * indices run over the in-plane block of the plane-strain embedding.
 * A[(i*d+j)*d*d + k*d+l]; NaN where det G <= 0 (neo-Hooke only). */
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
    if (mat->model == ORC_MODEL_STVK_DAMAGE) {
        double S[3][3], H[81];
        stvk_dpsi0(mat, F3, S, H);
        double p0 = orc_psi0(mat, G);
        double g1 = 1.0 - orc_damage(mat, p0 > beta_n ? p0 : beta_n);
        double g2 = p0 > beta_n ? -mat->D_inf / mat->D0 * exp(-p0 / mat->D0) : 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                for (int k = 0; k < d; ++k)
                    for (int l = 0; l < d; ++l)
                        A[(i * d + j) * dd + k * d + l] = g1 * H[(i * 3 + j) * 9 + k * 3 + l]
                                                        + g2 * S[i][j] * S[k][l];
        return 0;
    }
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
