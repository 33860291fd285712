/*
 * mlp_oracle.c -- plain FP64 CPU reference of the learned interface
 * estimator: a 27 -> 64 -> 64 -> 4 perceptron with tanh hidden layers that
 * maps the 3x3x3 fill-level stencil of an interface cell to its normal and
 * curvature, its loss gradient and the Adam update.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the GPU path
 * shares no code with it.
 *
 * The paper needs the local curvature kappa only inside the Laplace pressure
 * 2 sigma kappa (Section 2.1) and does not say how it is estimated; the
 * network is a learned alternative to the finite-difference estimate, not
 * part of the paper.
 *
 * Layout of the flat parameter vector (double, 6212 entries):
 *   W1[64][27], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]
 * Input x_k = clamp(phi_k, 0, 1) - 1/2 in direction order (k = a+3b+9c for
 * the offset (a-1, b-1, c-1)).  Output y[0..2] is the normal (trained
 * towards the unit normal, normalised when used), y[3] is 4 * kappa.  Loss
 * per sample: |y[0..2] - n*|^2 + (y[3] - 4 kappa*)^2, averaged over the
 * batch.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NIN 27
#define NH 64
#define NOUT 4
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NIN)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NOUT * NH)
#define NPARAM (OFF_B3 + NOUT)

int32_t ol_mlp_nparam(void) { return NPARAM; }

static void forward_one(const double *P, const double *x, double *h1, double *h2, double *y)
{
    const double *W1 = P + OFF_W1, *b1 = P + OFF_B1, *W2 = P + OFF_W2, *b2 = P + OFF_B2;
    const double *W3 = P + OFF_W3, *b3 = P + OFF_B3;
    for (int j = 0; j < NH; ++j) {
        double s = b1[j];
        for (int k = 0; k < NIN; ++k) s += W1[j * NIN + k] * x[k];
        h1[j] = tanh(s);
    }
    for (int j = 0; j < NH; ++j) {
        double s = b2[j];
        for (int k = 0; k < NH; ++k) s += W2[j * NH + k] * h1[k];
        h2[j] = tanh(s);
    }
    for (int j = 0; j < NOUT; ++j) {
        double s = b3[j];
        for (int k = 0; k < NH; ++k) s += W3[j * NH + k] * h2[k];
        y[j] = s;
    }
}

void ol_mlp_forward(const double *P, int32_t n, const double *x, double *y)
{
    double h1[NH], h2[NH];
    for (int32_t s = 0; s < n; ++s) forward_one(P, x + (size_t)s * NIN, h1, h2, y + (size_t)s * NOUT);
}

/* mean loss over n samples; grad (NPARAM) receives dL/dP when not NULL.
 * target: n x 4 = exact unit normal (3) and curvature kappa* (1). */
double ol_mlp_loss_grad(const double *P, int32_t n, const double *x, const double *target, double *grad)
{
    const double *W2 = P + OFF_W2, *W3 = P + OFF_W3;
    double h1[NH], h2[NH], y[NOUT], dy[NOUT], d2[NH], d1[NH];
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * NPARAM);
    for (int32_t s = 0; s < n; ++s) {
        const double *xs = x + (size_t)s * NIN, *t = target + (size_t)s * NOUT;
        forward_one(P, xs, h1, h2, y);
        double e[4];
        for (int a = 0; a < 3; ++a) e[a] = y[a] - t[a];
        e[3] = y[3] - 4.0 * t[3];
        loss += e[0] * e[0] + e[1] * e[1] + e[2] * e[2] + e[3] * e[3];
        if (!grad) continue;
        for (int a = 0; a < 4; ++a) dy[a] = 2.0 * e[a] / n;
        for (int j = 0; j < NOUT; ++j) {
            grad[OFF_B3 + j] += dy[j];
            for (int k = 0; k < NH; ++k) grad[OFF_W3 + j * NH + k] += dy[j] * h2[k];
        }
        for (int k = 0; k < NH; ++k) {
            double g = 0.0;
            for (int j = 0; j < NOUT; ++j) g += dy[j] * W3[j * NH + k];
            d2[k] = g * (1.0 - h2[k] * h2[k]);
        }
        for (int j = 0; j < NH; ++j) {
            grad[OFF_B2 + j] += d2[j];
            for (int k = 0; k < NH; ++k) grad[OFF_W2 + j * NH + k] += d2[j] * h1[k];
        }
        for (int k = 0; k < NH; ++k) {
            double g = 0.0;
            for (int j = 0; j < NH; ++j) g += d2[j] * W2[j * NH + k];
            d1[k] = g * (1.0 - h1[k] * h1[k]);
        }
        for (int j = 0; j < NH; ++j) {
            grad[OFF_B1 + j] += d1[j];
            for (int k = 0; k < NIN; ++k) grad[OFF_W1 + j * NIN + k] += d1[j] * xs[k];
        }
    }
    return loss / n;
}

/* Adam (Kingma & Ba 2015), step number t >= 1 */
void ol_mlp_adam(double *P, double *m, double *v, const double *g, int64_t t, double lr,
                 double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int i = 0; i < NPARAM; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        P[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
