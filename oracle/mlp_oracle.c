/*
 * mlp_oracle.c -- fp64 reference of the small network that proposes initial
 * multicanonical weights: inputs (1/L, e = E/N), two tanh layers of 64 units,
 * linear output f ~ ln g(E)/N (entropy per site).
 *
 * TEST INFRASTRUCTURE ONLY (see mc_oracle.c): plain loops, no blocking.
 *
 * Parameter layout (4417 values):
 *   W1[64][2] | b1[64] | W2[64][64] (row j = unit j of layer 2) | b2[64] | W3[64] | b3
 * Loss: weighted mean squared error  sum_i w_i (y_i - t_i)^2 / sum_i w_i
 * (w = NULL means every w_i = 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + H * 2)
#define OFF_W2 (OFF_B1 + H)
#define OFF_B2 (OFF_W2 + H * H)
#define OFF_W3 (OFF_B2 + H)
#define OFF_B3 (OFF_W3 + H)
#define N_PARAMS (OFF_B3 + 1)

int32_t orc_mlp_n_params(void) { return N_PARAMS; }

static void forward_one(const double *p, const double *x, double *h1, double *h2, double *y) {
    for (int i = 0; i < H; ++i) {
        double z = p[OFF_B1 + i] + p[OFF_W1 + 2 * i] * x[0] + p[OFF_W1 + 2 * i + 1] * x[1];
        h1[i] = tanh(z);
    }
    for (int j = 0; j < H; ++j) {
        double z = p[OFF_B2 + j];
        for (int i = 0; i < H; ++i) z += p[OFF_W2 + H * j + i] * h1[i];
        h2[j] = tanh(z);
    }
    double o = p[OFF_B3];
    for (int j = 0; j < H; ++j) o += p[OFF_W3 + j] * h2[j];
    *y = o;
}

void orc_mlp_forward(const double *p, const double *x, int32_t n, double *y) {
    double h1[H], h2[H];
    for (int s = 0; s < n; ++s) forward_one(p, x + 2 * s, h1, h2, y + s);
}

/* Loss and its gradient with respect to every parameter (backpropagation
   written out by the chain rule, layer by layer). */
double orc_mlp_loss_grad(const double *p, const double *x, const double *t, const double *w, int32_t n,
                         double *grad) {
    double h1[H], h2[H], d2[H], d1[H];
    memset(grad, 0, sizeof(double) * N_PARAMS);
    double wsum = 0.0;
    for (int s = 0; s < n; ++s) wsum += w ? w[s] : 1.0;
    double loss = 0.0;
    for (int s = 0; s < n; ++s) {
        const double *xs = x + 2 * s;
        double y;
        forward_one(p, xs, h1, h2, &y);
        const double ws = (w ? w[s] : 1.0) / wsum;
        const double r = y - t[s];
        loss += ws * r * r;
        const double dy = 2.0 * ws * r; /* d loss / d y */
        grad[OFF_B3] += dy;
        for (int j = 0; j < H; ++j) {
            grad[OFF_W3 + j] += dy * h2[j];
            d2[j] = dy * p[OFF_W3 + j] * (1.0 - h2[j] * h2[j]); /* d loss / d z2_j */
        }
        for (int j = 0; j < H; ++j) {
            grad[OFF_B2 + j] += d2[j];
            for (int i = 0; i < H; ++i) grad[OFF_W2 + H * j + i] += d2[j] * h1[i];
        }
        for (int i = 0; i < H; ++i) {
            double a = 0.0;
            for (int j = 0; j < H; ++j) a += d2[j] * p[OFF_W2 + H * j + i];
            d1[i] = a * (1.0 - h1[i] * h1[i]); /* d loss / d z1_i */
        }
        for (int i = 0; i < H; ++i) {
            grad[OFF_B1 + i] += d1[i];
            grad[OFF_W1 + 2 * i] += d1[i] * xs[0];
            grad[OFF_W1 + 2 * i + 1] += d1[i] * xs[1];
        }
    }
    return loss;
}
