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
 * the offset (a-1, b-1, c-1)).  Loss per sample against a target t:
 * |y[0..2] - t[0..2]|^2 + (y[3] - 4 t[3])^2, averaged over the batch.  In a
 * lattice the outputs correct the finite-difference estimate of the same
 * stencil (ol_estimator_compose), so the targets are t = (n* - n_fd,
 * kappa* - kappa_fd).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "fsl_oracle.h"

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

/* The estimator as a lattice uses it (O18, a reading: the paper needs the
 * curvature only in the Laplace pressure 2 sigma kappa of Section 2.1 and
 * names no estimator).  phi is the interface cell's 3x3x3 fill stencil as the
 * lattice builds it (liquid 1, gas 0, interface clamp(m/rho), solid or wall
 * the centre value); solid_nb says whether any of its 26 neighbours is solid
 * or lies beyond a wall.  In order:
 *   1. the finite-difference estimate (n_fd, kappa_fd) of the stencil;
 *   2. the network outputs y for the input phi - 1/2;
 *   3. n_raw = n_fd + y[0..2] and kappa = kappa_fd + y[3]/4;
 *   4. the finite-difference estimate is kept when the first of these holds:
 *      (1) a neighbour is solid, (2) |n_raw| lies outside [0.5, 2], (3) n_raw
 *      makes an angle of more than 30 degrees with n_fd, (4) |kappa| > 0.5;
 *      otherwise n = n_raw/|n_raw| with the composed kappa.
 * Returns 0 when the corrected estimate is used, else the number of the rule
 * that kept finite differences.  q (may be NULL) receives |n_raw|, the angle
 * in degrees and the composed kappa, whichever rule decided. */
int32_t ol_estimator_compose(const double *P, const double phi[27], int32_t solid_nb, double n[3],
                             double *kappa, double q[3])
{
    double nfd[3], kfd, x[NIN], h1[NH], h2[NH], y[NOUT];
    ol_normal_curvature(phi, nfd, &kfd);
    for (int k = 0; k < NIN; ++k) x[k] = phi[k] - 0.5;
    forward_one(P, x, h1, h2, y);
    double nr[3] = {nfd[0] + y[0], nfd[1] + y[1], nfd[2] + y[2]};
    const double rn = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
    const double kap = kfd + 0.25 * y[3];
    /* n_fd is a unit vector or zero (vanishing gradient: the angle is then
     * taken as 90 degrees) */
    double cosang = rn > 0.0 ? (nfd[0] * nr[0] + nfd[1] * nr[1] + nfd[2] * nr[2]) / rn : 0.0;
    if (cosang > 1.0) cosang = 1.0;
    if (cosang < -1.0) cosang = -1.0;
    const double angle = acos(cosang) * (180.0 / 3.14159265358979323846);
    if (q) {
        q[0] = rn;
        q[1] = angle;
        q[2] = kap;
    }
    int32_t rule = 0;
    if (solid_nb) rule = 1;
    else if (rn < 0.5 || rn > 2.0) rule = 2;
    else if (angle > 30.0) rule = 3;
    else if (fabs(kap) > 0.5) rule = 4;
    if (rule) {
        for (int d = 0; d < 3; ++d) n[d] = nfd[d];
        *kappa = kfd;
    } else {
        for (int d = 0; d < 3; ++d) n[d] = nr[d] / rn;
        *kappa = kap;
    }
    return rule;
}
