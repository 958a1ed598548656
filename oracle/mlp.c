/*
 * Oracle for the learned surrogate: a plain FP64 multilayer perceptron
 * (forward pass, mean-squared loss, backpropagation) used to check the GPU
 * training kernels' gradients and the GPU inference.  Test infrastructure only.
 *
 * Network: x (d_in) -> [Linear(width), SiLU] x n_hidden -> Linear(d_out).
 * SiLU(z) = z / (1 + e^{-z}).  Loss over a batch of B rows:
 *   L = 1/(B d_out) sum_b sum_j (out_bj - y_bj)^2.
 * Flat parameter layout (row-major weights, out x in):
 *   W_0 (width x d_in), b_0 (width), W_1 (width x width), b_1, ...,
 *   W_{n_hidden-1}, b_{n_hidden-1}, W_out (d_out x width), b_out (d_out).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "r1_oracle.h"

long orc_mlp_param_count(int d_in, int width, int n_hidden, int d_out)
{
    long n = (long)width * d_in + width;
    n += (long)(n_hidden - 1) * ((long)width * width + width);
    n += (long)d_out * width + d_out;
    return n;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }

static double silu_prime(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* Forward for B rows; out (B x d_out).  Returns the loss if y != NULL. */
double orc_mlp_forward(int d_in, int width, int n_hidden, int d_out, const double* params,
                       long B, const double* x, const double* y, double* out)
{
    double* h = (double*)orc_alloc(sizeof(double) * (size_t)width);
    double* hn = (double*)orc_alloc(sizeof(double) * (size_t)width);
    double loss = 0.0;
    for (long b = 0; b < B; ++b) {
        const double* p = params;
        const double* in = x + b * d_in;
        int n_in = d_in;
        for (int l = 0; l < n_hidden; ++l) {
            const double* W = p;
            const double* bias = p + (long)width * n_in;
            for (int o = 0; o < width; ++o) {
                double z = bias[o];
                for (int i = 0; i < n_in; ++i)
                    z += W[(long)o * n_in + i] * in[i];
                hn[o] = silu(z);
            }
            memcpy(h, hn, sizeof(double) * (size_t)width);
            in = h;
            p = bias + width;
            n_in = width;
        }
        const double* W = p;
        const double* bias = p + (long)d_out * width;
        for (int j = 0; j < d_out; ++j) {
            double o = bias[j];
            for (int i = 0; i < width; ++i)
                o += W[(long)j * width + i] * h[i];
            if (out)
                out[b * d_out + j] = o;
            if (y) {
                double e = o - y[b * d_out + j];
                loss += e * e;
            }
        }
    }
    free(h);
    free(hn);
    return y ? loss / ((double)B * d_out) : 0.0;
}

/* Loss and its gradient with respect to every parameter (grad: same layout). */
double orc_mlp_loss_grad(int d_in, int width, int n_hidden, int d_out, const double* params,
                         long B, const double* x, const double* y, double* grad)
{
    long np = orc_mlp_param_count(d_in, width, n_hidden, d_out);
    memset(grad, 0, sizeof(double) * (size_t)np);
    /* pre-activations and activations of every hidden layer for one row */
    double* z = (double*)orc_alloc(sizeof(double) * (size_t)width * n_hidden);
    double* a = (double*)orc_alloc(sizeof(double) * (size_t)width * n_hidden);
    double* delta = (double*)orc_alloc(sizeof(double) * (size_t)width);
    double* dprev = (double*)orc_alloc(sizeof(double) * (size_t)width);
    double* gout = (double*)orc_alloc(sizeof(double) * (size_t)d_out);
    long* off = (long*)orc_alloc(sizeof(long) * (size_t)(n_hidden + 1));
    /* offsets of W_l in the flat layout */
    long o = 0;
    for (int l = 0; l < n_hidden; ++l) {
        off[l] = o;
        int n_in = l == 0 ? d_in : width;
        o += (long)width * n_in + width;
    }
    off[n_hidden] = o;
    double loss = 0.0;
    const double scale = 2.0 / ((double)B * d_out);
    for (long b = 0; b < B; ++b) {
        const double* xb = x + b * d_in;
        for (int l = 0; l < n_hidden; ++l) {
            int n_in = l == 0 ? d_in : width;
            const double* in = l == 0 ? xb : a + (long)(l - 1) * width;
            const double* W = params + off[l];
            const double* bias = W + (long)width * n_in;
            for (int k = 0; k < width; ++k) {
                double s = bias[k];
                for (int i = 0; i < n_in; ++i)
                    s += W[(long)k * n_in + i] * in[i];
                z[(long)l * width + k] = s;
                a[(long)l * width + k] = silu(s);
            }
        }
        const double* hl = a + (long)(n_hidden - 1) * width;
        const double* Wo = params + off[n_hidden];
        const double* bo = Wo + (long)d_out * width;
        double* gWo = grad + off[n_hidden];
        double* gbo = gWo + (long)d_out * width;
        for (int j = 0; j < d_out; ++j) {
            double s = bo[j];
            for (int i = 0; i < width; ++i)
                s += Wo[(long)j * width + i] * hl[i];
            double e = s - y[b * d_out + j];
            loss += e * e;
            gout[j] = scale * e;
            gbo[j] += gout[j];
            for (int i = 0; i < width; ++i)
                gWo[(long)j * width + i] += gout[j] * hl[i];
        }
        /* dL/dh of the last hidden layer, then through SiLU */
        for (int i = 0; i < width; ++i) {
            double s = 0.0;
            for (int j = 0; j < d_out; ++j)
                s += gout[j] * Wo[(long)j * width + i];
            delta[i] = s * silu_prime(z[(long)(n_hidden - 1) * width + i]);
        }
        for (int l = n_hidden - 1; l >= 0; --l) {
            int n_in = l == 0 ? d_in : width;
            const double* in = l == 0 ? xb : a + (long)(l - 1) * width;
            const double* W = params + off[l];
            double* gW = grad + off[l];
            double* gb = gW + (long)width * n_in;
            for (int k = 0; k < width; ++k) {
                gb[k] += delta[k];
                for (int i = 0; i < n_in; ++i)
                    gW[(long)k * n_in + i] += delta[k] * in[i];
            }
            if (l > 0) {
                for (int i = 0; i < width; ++i) {
                    double s = 0.0;
                    for (int k = 0; k < width; ++k)
                        s += delta[k] * W[(long)k * width + i];
                    dprev[i] = s * silu_prime(z[(long)(l - 1) * width + i]);
                }
                memcpy(delta, dprev, sizeof(double) * (size_t)width);
            }
        }
    }
    free(z); free(a); free(delta); free(dprev); free(gout); free(off);
    return loss / ((double)B * d_out);
}
