/*
 * fsl_oracle.c -- plain FP64 CPU oracle of the free-surface cumulant LBM step.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
 * CPU baseline.  It shares no code with the GPU path.  It is written for
 * clarity, not speed: full PDFs in double, one cell at a time, every rule in
 * the order the method states it.
 *
 * Paper passages followed (Schwarzmeier et al., "Particle-resolved simulation
 * of antidunes in free-surface flows"):
 *   Section 2.1: lattice units, D3Q27 cumulant collision with all rates 1 but
 *     omega, nu = (1/omega - 1/2)/3, bounce-back at solid obstacles, the
 *     volume-of-fluid free-surface model whose boundary condition carries the
 *     gas pressure and the Laplace pressure 2*sigma*kappa.
 *   Section 2.2: no-slip at particle surfaces.
 *   Section 3.1: periodic x and y, no-slip z boundaries, body force in x.
 * Where the paper delegates to cited methods, the readings used are:
 *   collision   -- Geier et al. 2015 cumulant transform (chimera passes,
 *                  cumulants with first-order central moments taken as zero),
 *                  Galilean correction terms only as a variant; force by shifting the
 *                  velocity by F/(2 rho) and negating the first-order central
 *                  moments in the collision;
 *   walls       -- halfway bounce-back, Ladd's moving-wall term with rho_w=1;
 *   particles   -- momentum exchange in the Galilean-invariant form of Wen
 *                  et al. 2014 at the link midpoints (ol_particle_forces);
 *   free surface-- Koerner et al. 2005 anti-bounce-back reconstruction of
 *                  PDFs coming from gas or from the gas side of the normal,
 *                  gas density rho_gas + 6 sigma kappa; mass flux weighted by
 *                  the mean fill level between two interface cells;
 *   conversion  -- thresholds (1+eps) rho and -eps rho, isolated-cell rules,
 *                  fill -> cancel -> empty order (Thuerey 2007); excess mass
 *                  shared evenly among interface neighbours, a pool otherwise;
 *   variants    -- (optional, OL_VAR_*) Thuerey's flux modifiers between
 *                  interface cells, his normal-weighted excess mass, and a
 *                  curvature from the divergence of corner normals
 *                  (Brackbill et al. 1992), and the Galilean-invariance
 *                  correction of the cumulant collision;
 *   geometry    -- Parker-Youngs normal, mean curvature from the finite-
 *                  difference Hessian of the same 3x3x3 fill stencil.
 * The two per-cell phases (stream-collide, geometry) may run their cells on
 * several threads (OpenMP): every cell reads the previous state and writes
 * only its own entries, so the result does not depend on the thread count.
 */
#include "fsl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 27
#define REST 13

static int CV[Q][3];
static double WT[Q];
static int tables_ready = 0;

static double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

static void tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) {
        CV[i][0] = i % 3 - 1;
        CV[i][1] = (i / 3) % 3 - 1;
        CV[i][2] = i / 9 - 1;
        WT[i] = w1(CV[i][0]) * w1(CV[i][1]) * w1(CV[i][2]);
    }
    tables_ready = 1;
}

static int opp(int i) { return Q - 1 - i; }
static int K(int a, int b, int c) { return a + 3 * b + 9 * c; }
static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

void ol_velocities(int32_t c[27][3], double w[27])
{
    tables();
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) c[i][d] = CV[i][d];
        w[i] = WT[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Collision (Geier et al. 2015 as used in Section 2.1)                      */
/* ------------------------------------------------------------------------ */

/* One forward chimera step on a triplet of values at velocities -1, 0, +1:
 * returns the central moments of order 0, 1, 2 about u. */
static void chimera_fwd(double *fm, double *f0, double *fp, double u)
{
    double k0 = *fm + *f0 + *fp;
    double k1 = (*fp - *fm) - u * k0;
    double k2 = (*fp + *fm) - 2.0 * u * (*fp - *fm) + u * u * k0;
    *fm = k0;
    *f0 = k1;
    *fp = k2;
}

/* Inverse of chimera_fwd: central moments of order 0,1,2 -> values at -1,0,+1 */
static void chimera_bwd(double *k0p, double *k1p, double *k2p, double u)
{
    double k0 = *k0p, k1 = *k1p, k2 = *k2p;
    double f0 = k0 * (1.0 - u * u) - 2.0 * u * k1 - k2;
    double fm = 0.5 * (k0 * (u * u - u) + k1 * (2.0 * u - 1.0) + k2);
    double fp = 0.5 * (k0 * (u * u + u) + k1 * (2.0 * u + 1.0) + k2);
    *k0p = fm;
    *k1p = f0;
    *k2p = fp;
}

/* PDFs (index a+3b+9c, a<->x) -> raw central moments kappa_{abc} about u.
 * Passes in z, then y, then x. */
static void central_moments(double M[Q], const double u[3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            chimera_fwd(&M[K(a, b, 0)], &M[K(a, b, 1)], &M[K(a, b, 2)], u[2]);
    for (int a = 0; a < 3; ++a)
        for (int g = 0; g < 3; ++g)
            chimera_fwd(&M[K(a, 0, g)], &M[K(a, 1, g)], &M[K(a, 2, g)], u[1]);
    for (int b = 0; b < 3; ++b)
        for (int g = 0; g < 3; ++g)
            chimera_fwd(&M[K(0, b, g)], &M[K(1, b, g)], &M[K(2, b, g)], u[0]);
}

static void central_to_pdf(double M[Q], const double u[3])
{
    for (int b = 0; b < 3; ++b)
        for (int g = 0; g < 3; ++g)
            chimera_bwd(&M[K(0, b, g)], &M[K(1, b, g)], &M[K(2, b, g)], u[0]);
    for (int a = 0; a < 3; ++a)
        for (int g = 0; g < 3; ++g)
            chimera_bwd(&M[K(a, 0, g)], &M[K(a, 1, g)], &M[K(a, 2, g)], u[1]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            chimera_bwd(&M[K(a, b, 0)], &M[K(a, b, 1)], &M[K(a, b, 2)], u[2]);
}

/* shorthand for normalised central moment / cumulant tables */
#define k_(a, b, c) k[K(a, b, c)]
#define C_(a, b, c) C[K(a, b, c)]

/* Cumulants of orders 2..6 from normalised central moments, with the
 * first-order central moments taken as zero (moment-cumulant relations
 * restricted to blocks of size >= 2). */
static void cumulants_from_central(const double k[Q], double C[Q])
{
    for (int i = 0; i < Q; ++i) C[i] = k[i]; /* orders 0..3 are unchanged */

    /* order 4 */
    C_(2, 2, 0) = k_(2, 2, 0) - k_(2, 0, 0) * k_(0, 2, 0) - 2.0 * k_(1, 1, 0) * k_(1, 1, 0);
    C_(2, 0, 2) = k_(2, 0, 2) - k_(2, 0, 0) * k_(0, 0, 2) - 2.0 * k_(1, 0, 1) * k_(1, 0, 1);
    C_(0, 2, 2) = k_(0, 2, 2) - k_(0, 2, 0) * k_(0, 0, 2) - 2.0 * k_(0, 1, 1) * k_(0, 1, 1);
    C_(2, 1, 1) = k_(2, 1, 1) - k_(2, 0, 0) * k_(0, 1, 1) - 2.0 * k_(1, 1, 0) * k_(1, 0, 1);
    C_(1, 2, 1) = k_(1, 2, 1) - k_(0, 2, 0) * k_(1, 0, 1) - 2.0 * k_(1, 1, 0) * k_(0, 1, 1);
    C_(1, 1, 2) = k_(1, 1, 2) - k_(0, 0, 2) * k_(1, 1, 0) - 2.0 * k_(1, 0, 1) * k_(0, 1, 1);

    /* order 5 */
    C_(2, 2, 1) = k_(2, 2, 1) - (k_(2, 0, 0) * k_(0, 2, 1) + k_(0, 2, 0) * k_(2, 0, 1)
                                 + 4.0 * k_(1, 1, 0) * k_(1, 1, 1) + 2.0 * k_(1, 0, 1) * k_(1, 2, 0)
                                 + 2.0 * k_(0, 1, 1) * k_(2, 1, 0));
    C_(2, 1, 2) = k_(2, 1, 2) - (k_(2, 0, 0) * k_(0, 1, 2) + k_(0, 0, 2) * k_(2, 1, 0)
                                 + 4.0 * k_(1, 0, 1) * k_(1, 1, 1) + 2.0 * k_(1, 1, 0) * k_(1, 0, 2)
                                 + 2.0 * k_(0, 1, 1) * k_(2, 0, 1));
    C_(1, 2, 2) = k_(1, 2, 2) - (k_(0, 2, 0) * k_(1, 0, 2) + k_(0, 0, 2) * k_(1, 2, 0)
                                 + 4.0 * k_(0, 1, 1) * k_(1, 1, 1) + 2.0 * k_(1, 1, 0) * k_(0, 1, 2)
                                 + 2.0 * k_(1, 0, 1) * k_(0, 2, 1));

    /* order 6: m6 - sum(m2 m4) - sum(m3 m3) + 2 sum(m2 m2 m2) */
    double s24 = k_(2, 0, 0) * k_(0, 2, 2) + k_(0, 2, 0) * k_(2, 0, 2) + k_(0, 0, 2) * k_(2, 2, 0)
                 + 4.0 * (k_(1, 1, 0) * k_(1, 1, 2) + k_(1, 0, 1) * k_(1, 2, 1)
                          + k_(0, 1, 1) * k_(2, 1, 1));
    double s33 = 2.0 * (k_(2, 1, 0) * k_(0, 1, 2) + k_(2, 0, 1) * k_(0, 2, 1)
                        + k_(1, 2, 0) * k_(1, 0, 2))
                 + 4.0 * k_(1, 1, 1) * k_(1, 1, 1);
    double s222 = k_(2, 0, 0) * k_(0, 2, 0) * k_(0, 0, 2)
                  + 2.0 * (k_(2, 0, 0) * k_(0, 1, 1) * k_(0, 1, 1)
                           + k_(0, 2, 0) * k_(1, 0, 1) * k_(1, 0, 1)
                           + k_(0, 0, 2) * k_(1, 1, 0) * k_(1, 1, 0))
                  + 8.0 * k_(1, 1, 0) * k_(1, 0, 1) * k_(0, 1, 1);
    C_(2, 2, 2) = k_(2, 2, 2) - s24 - s33 + 2.0 * s222;
}

/* Inverse of cumulants_from_central for orders 2..6 (rearranged relations,
 * using the already rebuilt lower-order moments). */
static void central_from_cumulants(const double C[Q], double k[Q])
{
    for (int i = 0; i < Q; ++i) k[i] = C[i];

    k_(2, 2, 0) = C_(2, 2, 0) + k_(2, 0, 0) * k_(0, 2, 0) + 2.0 * k_(1, 1, 0) * k_(1, 1, 0);
    k_(2, 0, 2) = C_(2, 0, 2) + k_(2, 0, 0) * k_(0, 0, 2) + 2.0 * k_(1, 0, 1) * k_(1, 0, 1);
    k_(0, 2, 2) = C_(0, 2, 2) + k_(0, 2, 0) * k_(0, 0, 2) + 2.0 * k_(0, 1, 1) * k_(0, 1, 1);
    k_(2, 1, 1) = C_(2, 1, 1) + k_(2, 0, 0) * k_(0, 1, 1) + 2.0 * k_(1, 1, 0) * k_(1, 0, 1);
    k_(1, 2, 1) = C_(1, 2, 1) + k_(0, 2, 0) * k_(1, 0, 1) + 2.0 * k_(1, 1, 0) * k_(0, 1, 1);
    k_(1, 1, 2) = C_(1, 1, 2) + k_(0, 0, 2) * k_(1, 1, 0) + 2.0 * k_(1, 0, 1) * k_(0, 1, 1);

    k_(2, 2, 1) = C_(2, 2, 1) + (k_(2, 0, 0) * k_(0, 2, 1) + k_(0, 2, 0) * k_(2, 0, 1)
                                 + 4.0 * k_(1, 1, 0) * k_(1, 1, 1) + 2.0 * k_(1, 0, 1) * k_(1, 2, 0)
                                 + 2.0 * k_(0, 1, 1) * k_(2, 1, 0));
    k_(2, 1, 2) = C_(2, 1, 2) + (k_(2, 0, 0) * k_(0, 1, 2) + k_(0, 0, 2) * k_(2, 1, 0)
                                 + 4.0 * k_(1, 0, 1) * k_(1, 1, 1) + 2.0 * k_(1, 1, 0) * k_(1, 0, 2)
                                 + 2.0 * k_(0, 1, 1) * k_(2, 0, 1));
    k_(1, 2, 2) = C_(1, 2, 2) + (k_(0, 2, 0) * k_(1, 0, 2) + k_(0, 0, 2) * k_(1, 2, 0)
                                 + 4.0 * k_(0, 1, 1) * k_(1, 1, 1) + 2.0 * k_(1, 1, 0) * k_(0, 1, 2)
                                 + 2.0 * k_(1, 0, 1) * k_(0, 2, 1));

    double s24 = k_(2, 0, 0) * k_(0, 2, 2) + k_(0, 2, 0) * k_(2, 0, 2) + k_(0, 0, 2) * k_(2, 2, 0)
                 + 4.0 * (k_(1, 1, 0) * k_(1, 1, 2) + k_(1, 0, 1) * k_(1, 2, 1)
                          + k_(0, 1, 1) * k_(2, 1, 1));
    double s33 = 2.0 * (k_(2, 1, 0) * k_(0, 1, 2) + k_(2, 0, 1) * k_(0, 2, 1)
                        + k_(1, 2, 0) * k_(1, 0, 2))
                 + 4.0 * k_(1, 1, 1) * k_(1, 1, 1);
    double s222 = k_(2, 0, 0) * k_(0, 2, 0) * k_(0, 0, 2)
                  + 2.0 * (k_(2, 0, 0) * k_(0, 1, 1) * k_(0, 1, 1)
                           + k_(0, 2, 0) * k_(1, 0, 1) * k_(1, 0, 1)
                           + k_(0, 0, 2) * k_(1, 1, 0) * k_(1, 1, 0))
                  + 8.0 * k_(1, 1, 0) * k_(1, 0, 1) * k_(0, 1, 1);
    k_(2, 2, 2) = C_(2, 2, 2) + s24 + s33 - 2.0 * s222;
}

static int order_of(int i) { return i % 3 + (i / 3) % 3 + i / 9; }

/* density, momentum, force-shifted velocity */
static void macro(const double f[Q], const double g[3], double *rho, double u[3])
{
    tables();
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        for (int d = 0; d < 3; ++d) j[d] += f[i] * CV[i][d];
    }
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * r * g[d]) / r;
    *rho = r;
}

void ol_cumulants(const double fin[27], const double g[3], double C[27])
{
    double rho, u[3], M[Q], k[Q];
    macro(fin, g, &rho, u);
    for (int i = 0; i < Q; ++i) M[i] = fin[i];
    central_moments(M, u);
    for (int i = 0; i < Q; ++i) k[i] = M[i] / rho;
    cumulants_from_central(k, C);
    C[0] = rho;
}

void ol_collide(const double fin[27], const double g[3], double omega,
                double omega_bulk, double omega_high, int32_t galilean, double fout[27])
{
    double rho, u[3], M[Q], k[Q], C[Q], Cs[Q], ks[Q];
    macro(fin, g, &rho, u);
    for (int i = 0; i < Q; ++i) M[i] = fin[i];
    central_moments(M, u);
    for (int i = 0; i < Q; ++i) k[i] = M[i] / rho;
    cumulants_from_central(k, C);

    /* relaxation */
    for (int i = 0; i < Q; ++i) Cs[i] = C[i];
    /* second order: off-diagonal and deviatoric parts with omega, trace with
     * omega_bulk towards its equilibrium 3 * c_s^2 = 1 */
    Cs[K(1, 1, 0)] = (1.0 - omega) * C_(1, 1, 0);
    Cs[K(1, 0, 1)] = (1.0 - omega) * C_(1, 0, 1);
    Cs[K(0, 1, 1)] = (1.0 - omega) * C_(0, 1, 1);
    double D1 = (1.0 - omega) * (C_(2, 0, 0) - C_(0, 2, 0));
    double D2 = (1.0 - omega) * (C_(2, 0, 0) - C_(0, 0, 2));
    double T = (1.0 - omega_bulk) * (C_(2, 0, 0) + C_(0, 2, 0) + C_(0, 0, 2)) + omega_bulk * 1.0;
    if (galilean) {
        /* Galilean-invariance correction (Geier et al. 2015).  The first-
         * order non-equilibrium of the second-order cumulants is
         * -(2/(3 w)) times the strain rate, w the rate of that part; solving
         * the deviator (rate omega) and the trace (rate omega_bulk) for the
         * normal strain rates gives d_a u_a.  The cubic moment the lattice
         * cannot hold would add 3 u_a^2 d_a u_a to the momentum flux; it is
         * removed as a source term with the usual (1 - w/2) factor. */
        const double trace_neq = C_(2, 0, 0) + C_(0, 2, 0) + C_(0, 0, 2) - 1.0;
        const double dxu = -0.5 * omega * (2.0 * C_(2, 0, 0) - C_(0, 2, 0) - C_(0, 0, 2)) - 0.5 * omega_bulk * trace_neq;
        const double dyv = -0.5 * omega * (2.0 * C_(0, 2, 0) - C_(2, 0, 0) - C_(0, 0, 2)) - 0.5 * omega_bulk * trace_neq;
        const double dzw = -0.5 * omega * (2.0 * C_(0, 0, 2) - C_(2, 0, 0) - C_(0, 2, 0)) - 0.5 * omega_bulk * trace_neq;
        const double ex = u[0] * u[0] * dxu, ey = u[1] * u[1] * dyv, ez = u[2] * u[2] * dzw;
        D1 -= 3.0 * (1.0 - 0.5 * omega) * (ex - ey);
        D2 -= 3.0 * (1.0 - 0.5 * omega) * (ex - ez);
        T -= 3.0 * (1.0 - 0.5 * omega_bulk) * (ex + ey + ez);
    }
    Cs[K(2, 0, 0)] = (T + D1 + D2) / 3.0;
    Cs[K(0, 2, 0)] = (T - 2.0 * D1 + D2) / 3.0;
    Cs[K(0, 0, 2)] = (T + D1 - 2.0 * D2) / 3.0;
    /* orders 3..6 relax to their equilibrium value 0 */
    for (int i = 0; i < Q; ++i)
        if (order_of(i) >= 3) Cs[i] = (1.0 - omega_high) * C[i];

    central_from_cumulants(Cs, ks);
    /* zeroth and first order: mass kept, first-order central moments negated
     * (the velocity shift by F/(2 rho) then adds exactly F to the momentum) */
    ks[K(0, 0, 0)] = 1.0;
    ks[K(1, 0, 0)] = -k_(1, 0, 0);
    ks[K(0, 1, 0)] = -k_(0, 1, 0);
    ks[K(0, 0, 1)] = -k_(0, 0, 1);

    for (int i = 0; i < Q; ++i) M[i] = rho * ks[i];
    central_to_pdf(M, u);
    for (int i = 0; i < Q; ++i) fout[i] = M[i];
}

#undef k_
#undef C_

void ol_feq(double rho, const double u[3], double feq[27])
{
    tables();
    for (int i = 0; i < Q; ++i) {
        double p = rho;
        for (int d = 0; d < 3; ++d) {
            double ud = u[d];
            int c = CV[i][d];
            double psi = (c == 0) ? (2.0 / 3.0 - ud * ud) : 0.5 * (1.0 / 3.0 + ud * ud + c * ud);
            p *= psi;
        }
        feq[i] = p;
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry: Parker-Youngs normal and finite-difference mean curvature      */
/* ------------------------------------------------------------------------ */

static double st(const double phi[27], int a, int b, int c)
{
    return phi[(a + 1) + 3 * (b + 1) + 9 * (c + 1)];
}

void ol_normal_curvature(const double phi[27], double n[3], double *kappa)
{
    static const double Wpy[3] = {1.0, 2.0, 1.0};
    double g[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            double wgt = Wpy[p] * Wpy[q];
            g[0] += wgt * (st(phi, 1, p - 1, q - 1) - st(phi, -1, p - 1, q - 1));
            g[1] += wgt * (st(phi, p - 1, 1, q - 1) - st(phi, p - 1, -1, q - 1));
            g[2] += wgt * (st(phi, p - 1, q - 1, 1) - st(phi, p - 1, q - 1, -1));
        }
    for (int d = 0; d < 3; ++d) g[d] /= 32.0;
    double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (gn < 1e-12) {
        n[0] = n[1] = n[2] = 0.0;
        *kappa = 0.0;
        return;
    }
    double gh[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
    for (int d = 0; d < 3; ++d) n[d] = -gh[d];

    double H[3][3];
    double c0 = st(phi, 0, 0, 0);
    H[0][0] = st(phi, 1, 0, 0) - 2.0 * c0 + st(phi, -1, 0, 0);
    H[1][1] = st(phi, 0, 1, 0) - 2.0 * c0 + st(phi, 0, -1, 0);
    H[2][2] = st(phi, 0, 0, 1) - 2.0 * c0 + st(phi, 0, 0, -1);
    H[0][1] = H[1][0] = 0.25 * (st(phi, 1, 1, 0) - st(phi, 1, -1, 0) - st(phi, -1, 1, 0) + st(phi, -1, -1, 0));
    H[0][2] = H[2][0] = 0.25 * (st(phi, 1, 0, 1) - st(phi, 1, 0, -1) - st(phi, -1, 0, 1) + st(phi, -1, 0, -1));
    H[1][2] = H[2][1] = 0.25 * (st(phi, 0, 1, 1) - st(phi, 0, 1, -1) - st(phi, 0, -1, 1) + st(phi, 0, -1, -1));
    double tr = H[0][0] + H[1][1] + H[2][2];
    double gHg = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) gHg += gh[a] * H[a][b] * gh[b];
    *kappa = -(tr - gHg) / (2.0 * gn);
}

/* ------------------------------------------------------------------------ */
/* Lattice                                                                  */
/* ------------------------------------------------------------------------ */

enum { MK_TO_LIQ = 1, MK_TO_GAS = 2, MK_EMPTY = 4, MK_NEW_FROM_GAS = 8,
       MK_NEW_FROM_LIQ = 16, MK_RULE_ISO = 32, MK_WEIGHTED = 64 };

struct OlLattice {
    OlParams p;
    int64_t N;
    double *f;        /* N*27 post-collision PDFs */
    double *m, *phi, *rho;
    uint8_t *type, *mark;
    int32_t *owner;
    double *n, *kappa;
    double *share;    /* excess share of a converted cell */
    double *est_P;    /* learned estimator weights (NULL: finite differences only) */
    uint8_t *est_rule;  /* per interface cell: 1 + the rule of ol_estimator_compose */
    double *est_q;    /* per cell: |n_raw|, angle (degrees), composed kappa */
    int32_t nsph;
    double *sph;      /* per sphere: X[3], r, U[3], Omega[3] */
    double pool;
    int64_t cnt[8];
    int64_t steps;
};

static int64_t cell_of(const OlLattice *L, int x, int y, int z)
{
    return (int64_t)x + (int64_t)L->p.nx * ((int64_t)y + (int64_t)L->p.ny * z);
}

/* neighbour cell + sign*c_i; periodic in x, y; returns -1 beyond the z walls */
static int64_t nbr(const OlLattice *L, int64_t cell, int i, int sign)
{
    int nx = L->p.nx, ny = L->p.ny, nz = L->p.nz;
    int x = (int)(cell % nx);
    int y = (int)((cell / nx) % ny);
    int z = (int)(cell / ((int64_t)nx * ny));
    x += sign * CV[i][0];
    y += sign * CV[i][1];
    z += sign * CV[i][2];
    if (z < 0 || z >= nz) return -1;
    x = (x + nx) % nx;
    y = (y + ny) % ny;
    return cell_of(L, x, y, z);
}

static void cell_xyz(const OlLattice *L, int64_t cell, int *x, int *y, int *z)
{
    *x = (int)(cell % L->p.nx);
    *y = (int)((cell / L->p.nx) % L->p.ny);
    *z = (int)(cell / ((int64_t)L->p.nx * L->p.ny));
}

/* minimum-image offset along a periodic axis of length n */
static double min_image(double d, int n)
{
    if (d > 0.5 * n) d -= n;
    else if (d < -0.5 * n) d += n;
    return d;
}

/* wall point of the link from fluid cell `cell` to the solid cell cell - c_j:
 * halfway along the link; returned as its offset from the centre of sphere p
 * (minimum image in x and y) */
static void link_offset(const OlLattice *L, int p, int64_t cell, int j, double r[3])
{
    const double *s = &L->sph[10 * p];
    int x, y, z;
    cell_xyz(L, cell, &x, &y, &z);
    r[0] = min_image((x + 0.5 - 0.5 * CV[j][0]) - s[0], L->p.nx);
    r[1] = min_image((y + 0.5 - 0.5 * CV[j][1]) - s[1], L->p.ny);
    r[2] = (z + 0.5 - 0.5 * CV[j][2]) - s[2];
}

/* rigid-body velocity of sphere p at the wall point of that link */
static void sphere_wall_velocity(const OlLattice *L, int p, int64_t cell, int j, double uw[3])
{
    const double *s = &L->sph[10 * p];
    double r[3];
    link_offset(L, p, cell, j, r);
    const double *U = s + 4, *Om = s + 7;
    uw[0] = U[0] + (Om[1] * r[2] - Om[2] * r[1]);
    uw[1] = U[1] + (Om[2] * r[0] - Om[0] * r[2]);
    uw[2] = U[2] + (Om[0] * r[1] - Om[1] * r[0]);
}

/* fill value a stencil sees at a neighbour; centre value for walls/solids */
static double stencil_phi(const OlLattice *L, int64_t y, double centre)
{
    if (y < 0) return centre;
    switch (L->type[y]) {
    case OL_LIQUID: return 1.0;
    case OL_GAS: return 0.0;
    case OL_INTERFACE: return clamp01(L->phi[y]);
    default: return centre;
    }
}

/* Curvature in the manner of Brackbill et al. 1992 (continuum surface
 * force): half the divergence of the unit normal n = -grad(phi)/|grad(phi)|,
 * with the gradient taken at the 8 corners of the cell (differences of the
 * 2x2x2 cells around each corner) and the divergence from the corner
 * normals (differences between the four corners on either side).  A corner
 * gradient below CSF_GMIN gets the shortened normal -grad/CSF_GMIN: the
 * unit normal of a vanishing gradient is undefined, and without the floor a
 * rounding-level change of one fill level would turn a corner's normal from
 * zero to a unit vector. */
#define CSF_GMIN 1e-2
void ol_csf_curvature(const double phi[27], double *kappa)
{
    double div = 0.0;
    double nc[2][2][2][3];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                const int sx = 2 * a - 1, sy = 2 * b - 1, sz = 2 * c - 1;
                double g[3] = {0.0, 0.0, 0.0};
                for (int p = 0; p < 2; ++p)
                    for (int q = 0; q < 2; ++q) {
                        /* across x: the cells at x-offset sx and 0, over the
                         * two y and two z layers next to the corner */
                        g[0] += st(phi, sx, p * sy, q * sz) - st(phi, 0, p * sy, q * sz);
                        g[1] += st(phi, p * sx, sy, q * sz) - st(phi, p * sx, 0, q * sz);
                        g[2] += st(phi, p * sx, q * sy, sz) - st(phi, p * sx, q * sy, 0);
                    }
                g[0] *= 0.25 * sx;
                g[1] *= 0.25 * sy;
                g[2] *= 0.25 * sz;
                const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                for (int d = 0; d < 3; ++d) nc[a][b][c][d] = -g[d] / (gn > CSF_GMIN ? gn : CSF_GMIN);
            }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                div += 0.25 * (2 * a - 1) * nc[a][b][c][0];
                div += 0.25 * (2 * b - 1) * nc[a][b][c][1];
                div += 0.25 * (2 * c - 1) * nc[a][b][c][2];
            }
    *kappa = 0.5 * div;
}

static void geometry_cell(OlLattice *L, int64_t c)
{
    double st27[Q];
    double centre = clamp01(L->phi[c]);
    for (int i = 0; i < Q; ++i)
        st27[i] = (i == REST) ? centre : stencil_phi(L, nbr(L, c, i, +1), centre);
    if (L->est_P) {
        /* learned estimator with its finite-difference fallback (O18) */
        int32_t solid_nb = 0;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y < 0 || L->type[y] == OL_SOLID) solid_nb = 1;
        }
        L->est_rule[c] = (uint8_t)(1 + ol_estimator_compose(L->est_P, st27, solid_nb, &L->n[3 * c],
                                                            &L->kappa[c], &L->est_q[3 * c]));
        return;
    }
    ol_normal_curvature(st27, &L->n[3 * c], &L->kappa[c]);
    if (L->p.variants & OL_VAR_CSF_CURVATURE) ol_csf_curvature(st27, &L->kappa[c]);
}

static void phase_geometry(OlLattice *L)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < L->N; ++c) {
        if (L->type[c] == OL_INTERFACE) {
            geometry_cell(L, c);
        } else {
            L->n[3 * c] = L->n[3 * c + 1] = L->n[3 * c + 2] = 0.0;
            L->kappa[c] = 0.0;
            if (L->est_P) {
                L->est_rule[c] = 0;
                L->est_q[3 * c] = L->est_q[3 * c + 1] = L->est_q[3 * c + 2] = 0.0;
            }
        }
    }
}

/* Nearest IEEE binary16 value: 11 significant bits for |x| >= 2^-14 (the
 * smallest normal), spacing 2^-24 below; ties to even (nearbyint in the
 * default rounding mode).  Deviations stay far below the FP16 maximum. */
double ol_round_half(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e); /* |x| in [2^(e-1), 2^e) */
    const double q = (e - 1 >= -14) ? ldexp(1.0, e - 11) : ldexp(1.0, -24);
    return nearbyint(x / q) * q;
}

/* the storage form: FP64 as is, or deviations from w rounded to FP32 (the
 * C conversion rounds to nearest even) or to FP16 */
static void store_form(const OlLattice *L, double *f)
{
    if (L->p.store == 1)
        for (int i = 0; i < Q; ++i) f[i] = WT[i] + (double)(float)(f[i] - WT[i]);
    else if (L->p.store == 2)
        for (int i = 0; i < Q; ++i) f[i] = WT[i] + ol_round_half(f[i] - WT[i]);
}

static double sum27(const double *f)
{
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += f[i];
    return s;
}

static void refresh_fill(OlLattice *L)
{
    for (int64_t c = 0; c < L->N; ++c) {
        switch (L->type[c]) {
        case OL_INTERFACE: L->phi[c] = L->m[c] / L->rho[c]; break;
        case OL_LIQUID: L->phi[c] = 1.0; break;
        default: L->phi[c] = 0.0; break;
        }
    }
}

OlLattice *ol_create(const OlParams *p, const double *fill, const double *rho,
                     const double *vel)
{
    tables();
    if (!p || !fill || !rho) return NULL;
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return NULL;
    if (!(p->omega > 0.0 && p->omega < 2.0)) return NULL;
    if (p->variants & ~(OL_VAR_FLUX_MODIFIERS | OL_VAR_NORMAL_EXCESS | OL_VAR_CSF_CURVATURE | OL_VAR_GALILEAN))
        return NULL;
    OlLattice *L = (OlLattice *)calloc(1, sizeof(OlLattice));
    L->p = *p;
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    L->N = N;
    L->f = (double *)calloc((size_t)N * Q, sizeof(double));
    L->m = (double *)calloc((size_t)N, sizeof(double));
    L->phi = (double *)calloc((size_t)N, sizeof(double));
    L->rho = (double *)calloc((size_t)N, sizeof(double));
    L->type = (uint8_t *)calloc((size_t)N, 1);
    L->mark = (uint8_t *)calloc((size_t)N, 1);
    L->owner = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    L->n = (double *)calloc((size_t)N * 3, sizeof(double));
    L->kappa = (double *)calloc((size_t)N, sizeof(double));
    L->share = (double *)calloc((size_t)N, sizeof(double));
    for (int64_t c = 0; c < N; ++c) L->owner[c] = -1;

    /* cell types from the fill level */
    for (int64_t c = 0; c < N; ++c) {
        double fl = fill[c];
        L->type[c] = fl >= 1.0 ? OL_LIQUID : (fl <= 0.0 ? OL_GAS : OL_INTERFACE);
    }
    /* closure: a liquid cell next to a gas cell becomes interface */
    uint8_t *t0 = (uint8_t *)malloc((size_t)N);
    memcpy(t0, L->type, (size_t)N);
    for (int64_t c = 0; c < N; ++c) {
        if (t0[c] != OL_LIQUID) continue;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y >= 0 && t0[y] == OL_GAS) {
                L->type[c] = OL_INTERFACE;
                break;
            }
        }
    }
    free(t0);
    /* mass, equilibrium PDFs */
    for (int64_t c = 0; c < N; ++c) {
        double u[3] = {0.0, 0.0, 0.0};
        if (vel)
            for (int d = 0; d < 3; ++d) u[d] = vel[(int64_t)d * N + c];
        ol_feq(rho[c], u, &L->f[c * Q]);
        store_form(L, &L->f[c * Q]);
        L->rho[c] = sum27(&L->f[c * Q]);
        L->m[c] = (L->type[c] == OL_GAS) ? 0.0 : clamp01(fill[c]) * rho[c];
    }
    refresh_fill(L);
    phase_geometry(L);
    return L;
}

void ol_destroy(OlLattice *L)
{
    if (!L) return;
    free(L->f); free(L->m); free(L->phi); free(L->rho); free(L->type);
    free(L->mark); free(L->owner); free(L->n); free(L->kappa); free(L->share);
    free(L->sph); free(L->est_P); free(L->est_rule); free(L->est_q);
    free(L);
}

int ol_set_particles(OlLattice *L, int32_t n, const double *centre,
                     const double *radius, const double *vel, const double *angvel)
{
    int nx = L->p.nx, ny = L->p.ny, nz = L->p.nz;
    for (int32_t q = 0; q < n; ++q)
        if (!(radius[q] > 0.0) || 2.0 * radius[q] >= (nx < ny ? nx : ny)) return -1;
    free(L->sph);
    L->nsph = n;
    L->sph = (double *)calloc((size_t)(n > 0 ? n : 1) * 10, sizeof(double));
    for (int32_t q = 0; q < n; ++q) {
        double *s = &L->sph[10 * q];
        s[0] = centre[3 * q] - nx * floor(centre[3 * q] / nx);
        s[1] = centre[3 * q + 1] - ny * floor(centre[3 * q + 1] / ny);
        s[2] = centre[3 * q + 2];
        s[3] = radius[q];
        for (int d = 0; d < 3; ++d) {
            s[4 + d] = vel ? vel[3 * q + d] : 0.0;
            s[7 + d] = angvel ? angvel[3 * q + d] : 0.0;
        }
    }
    for (int64_t c = 0; c < L->N; ++c) L->owner[c] = -1;
    for (int32_t q = 0; q < n; ++q) {
        const double *s = &L->sph[10 * q];
        double r = s[3];
        int x0 = (int)floor(s[0] - r) - 1, x1 = (int)floor(s[0] + r) + 1;
        int y0 = (int)floor(s[1] - r) - 1, y1 = (int)floor(s[1] + r) + 1;
        int z0 = (int)floor(s[2] - r) - 1, z1 = (int)floor(s[2] + r) + 1;
        if (z0 < 0) z0 = 0;
        if (z1 > nz - 1) z1 = nz - 1;
        for (int z = z0; z <= z1; ++z)
            for (int yy = y0; yy <= y1; ++yy)
                for (int xx = x0; xx <= x1; ++xx) {
                    int x = ((xx % nx) + nx) % nx, y = ((yy % ny) + ny) % ny;
                    int64_t c = cell_of(L, x, y, z);
                    if (L->owner[c] >= 0) continue;
                    double dx = min_image((x + 0.5) - s[0], nx);
                    double dy = min_image((y + 0.5) - s[1], ny);
                    double dz = (z + 0.5) - s[2];
                    if (dx * dx + dy * dy + dz * dz <= r * r) L->owner[c] = q;
                }
    }
    for (int64_t c = 0; c < L->N; ++c) {
        if (L->owner[c] >= 0) {
            L->type[c] = OL_SOLID;
            L->m[c] = 0.0;
            L->phi[c] = 0.0;
        }
    }
    phase_geometry(L);
    return 0;
}

void ol_set_state(OlLattice *L, const uint8_t *type, const double *m, const double *f)
{
    memcpy(L->type, type, (size_t)L->N);
    memcpy(L->m, m, (size_t)L->N * sizeof(double));
    memcpy(L->f, f, (size_t)L->N * Q * sizeof(double));
    for (int64_t c = 0; c < L->N; ++c) L->rho[c] = sum27(&L->f[c * Q]);
    refresh_fill(L);
    phase_geometry(L);
}

/* ---- phase 1: streaming, boundaries, mass flux, collision ---------------- */
static void phase_stream_collide(OlLattice *L)
{
    const int64_t N = L->N;
    const OlParams *p = &L->p;
    double *fnew = (double *)malloc((size_t)N * Q * sizeof(double));
    double *mnew = (double *)malloc((size_t)N * sizeof(double));
    /* cells that do not stream keep their state */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        memcpy(&fnew[c * Q], &L->f[c * Q], Q * sizeof(double));
        mnew[c] = L->m[c];
    }
    int64_t liquid_next_to_gas = 0;
    /* flux-modifier class of each interface cell from the types at the start
     * of the step: 0 with gas but no liquid neighbours (it may only lose mass
     * to other interface cells), 2 with liquid but no gas neighbours (it may
     * only gain), 1 otherwise */
    uint8_t *cls = NULL;
    if (p->variants & OL_VAR_FLUX_MODIFIERS) {
        cls = (uint8_t *)malloc((size_t)N);
        for (int64_t c = 0; c < N; ++c) {
            cls[c] = 1;
            if (L->type[c] != OL_INTERFACE) continue;
            int has_gas = 0, has_liq = 0;
            for (int i = 0; i < Q; ++i) {
                if (i == REST) continue;
                int64_t y = nbr(L, c, i, +1);
                if (y < 0) continue;
                if (L->type[y] == OL_GAS) has_gas = 1;
                if (L->type[y] == OL_LIQUID) has_liq = 1;
            }
            if (has_gas && !has_liq) cls[c] = 0;
            else if (has_liq && !has_gas) cls[c] = 2;
        }
    }

#pragma omp parallel for schedule(static) reduction(+ : liquid_next_to_gas)
    for (int64_t c = 0; c < N; ++c) {
        uint8_t t = L->type[c];
        if (t != OL_LIQUID && t != OL_INTERFACE) continue;
        const double *fo = &L->f[c * Q];
        double fin[Q], feqG[Q];

        if (t == OL_INTERFACE) {
            /* gas-side equilibrium: gas pressure plus Laplace pressure 2 sigma kappa,
             * i.e. rho_G = rho_gas + 6 sigma kappa, at the cell's own velocity */
            double rg = p->rho_gas + 6.0 * p->sigma * L->kappa[c];
            double r0 = 0.0, j[3] = {0.0, 0.0, 0.0}, uI[3];
            for (int i = 0; i < Q; ++i) {
                r0 += fo[i];
                for (int d = 0; d < 3; ++d) j[d] += fo[i] * CV[i][d];
            }
            for (int d = 0; d < 3; ++d) uI[d] = j[d] / r0;
            ol_feq(rg, uI, feqG);
        }

        fin[REST] = fo[REST];
        for (int j = 0; j < Q; ++j) {
            if (j == REST) continue;
            int64_t src = nbr(L, c, j, -1);
            if (src < 0 || L->type[src] == OL_SOLID) {
                double uw[3] = {0.0, 0.0, 0.0};
                if (src >= 0) sphere_wall_velocity(L, L->owner[src], c, j, uw);
                double cu = CV[j][0] * uw[0] + CV[j][1] * uw[1] + CV[j][2] * uw[2];
                fin[j] = fo[opp(j)] + 6.0 * WT[j] * 1.0 * cu;
                continue;
            }
            int recon = 0;
            if (t == OL_INTERFACE) {
                if (L->type[src] == OL_GAS) {
                    recon = 1;
                } else {
                    const double *nn = &L->n[3 * c];
                    double nc = nn[0] * CV[j][0] + nn[1] * CV[j][1] + nn[2] * CV[j][2];
                    if (nc < -p->normal_tie) recon = 1;
                }
            } else if (L->type[src] == OL_GAS) {
                liquid_next_to_gas++;
            }
            if (recon)
                fin[j] = feqG[j] + feqG[opp(j)] - fo[opp(j)];
            else
                fin[j] = L->f[src * Q + j];
        }

        /* mass exchange with every fluid neighbour, from stored post-collision PDFs */
        double dm = 0.0;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y < 0) continue;
            uint8_t ty = L->type[y];
            if (ty == OL_SOLID || ty == OL_GAS) continue;
            double s = (t == OL_INTERFACE && ty == OL_INTERFACE)
                           ? 0.5 * (clamp01(L->phi[c]) + clamp01(L->phi[y]))
                           : 1.0;
            double in = L->f[y * Q + opp(i)], out = fo[i];
            if (cls && t == OL_INTERFACE && ty == OL_INTERFACE) {
                /* between classes mass moves only from the lower to the higher */
                if (cls[c] < cls[y]) in = 0.0;
                else if (cls[c] > cls[y]) out = 0.0;
            }
            dm += s * (in - out);
        }
        mnew[c] = L->m[c] + dm;

        ol_collide(fin, p->accel, p->omega, p->omega_bulk, p->omega_high, (p->variants & OL_VAR_GALILEAN) != 0,
                   &fnew[c * Q]);
        store_form(L, &fnew[c * Q]);
        L->rho[c] = sum27(&fnew[c * Q]);
    }
    L->cnt[7] += liquid_next_to_gas;
    free(cls);
    free(L->f);
    free(L->m);
    L->f = fnew;
    L->m = mnew;
}

/* ---- phase 2: conversion marks ------------------------------------------ */
static void phase_marks(OlLattice *L)
{
    const double eps = L->p.conv_eps;
    memset(L->mark, 0, (size_t)L->N);
    for (int64_t c = 0; c < L->N; ++c) {
        if (L->type[c] != OL_INTERFACE) continue;
        double m = L->m[c], r = L->rho[c];
        if (m > (1.0 + eps) * r) {
            L->mark[c] = MK_TO_LIQ;
        } else if (m < -eps * r) {
            L->mark[c] = MK_TO_GAS;
        } else if (L->p.rule_isolated) {
            int has_gas = 0, has_liq = 0;
            for (int i = 0; i < Q; ++i) {
                if (i == REST) continue;
                int64_t y = nbr(L, c, i, +1);
                if (y < 0) continue;
                if (L->type[y] == OL_GAS) has_gas = 1;
                if (L->type[y] == OL_LIQUID) has_liq = 1;
            }
            if (!has_gas && has_liq) L->mark[c] = MK_TO_LIQ | MK_RULE_ISO;
            else if (!has_liq && has_gas) L->mark[c] = MK_TO_GAS | MK_RULE_ISO;
        }
    }
}

/* ---- phase 3: conversion processing ------------------------------------- */
static void phase_convert(OlLattice *L)
{
    const int64_t N = L->N;
    uint8_t *mk = L->mark;

    /* counters of the marks as set from the thresholds and neighbour rules */
    for (int64_t c = 0; c < N; ++c) {
        if (mk[c] & MK_TO_LIQ) L->cnt[(mk[c] & MK_RULE_ISO) ? 2 : 0]++;
    }

    /* 1. filling: gas neighbours of filled cells become interface cells */
    for (int64_t c = 0; c < N; ++c) {
        if (!(mk[c] & MK_TO_LIQ)) continue;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y >= 0 && L->type[y] == OL_GAS) mk[y] |= MK_NEW_FROM_GAS;
        }
    }
    /* their PDFs: equilibrium at the mean density and velocity of the liquid
     * and (old) interface neighbours that are not marked for emptying */
    for (int64_t c = 0; c < N; ++c) {
        if (!(mk[c] & MK_NEW_FROM_GAS)) continue;
        double rs = 0.0, us[3] = {0.0, 0.0, 0.0};
        int cnt = 0;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y < 0) continue;
            uint8_t ty = L->type[y];
            if (ty != OL_LIQUID && ty != OL_INTERFACE) continue;
            if (mk[y] & MK_TO_GAS) continue;
            const double *fy = &L->f[y * Q];
            double r = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < Q; ++k) {
                r += fy[k];
                for (int d = 0; d < 3; ++d) j[d] += fy[k] * CV[k][d];
            }
            rs += r;
            for (int d = 0; d < 3; ++d) us[d] += j[d] / r;
            cnt++;
        }
        /* a filled neighbour always qualifies, so cnt >= 1 */
        double rbar = rs / cnt, ubar[3];
        for (int d = 0; d < 3; ++d) ubar[d] = us[d] / cnt;
        ol_feq(rbar, ubar, &L->f[c * Q]);
        store_form(L, &L->f[c * Q]);
        L->rho[c] = sum27(&L->f[c * Q]);
        L->m[c] = 0.0;
        L->cnt[5]++;
    }
    /* 2. an emptying next to a filling cell is cancelled */
    for (int64_t c = 0; c < N; ++c) {
        if (!(mk[c] & MK_TO_GAS)) continue;
        int near_fill = 0;
        for (int i = 0; i < Q && !near_fill; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y >= 0 && (mk[y] & MK_TO_LIQ)) near_fill = 1;
        }
        if (near_fill) {
            L->cnt[4]++;
        } else {
            mk[c] |= MK_EMPTY;
            L->cnt[(mk[c] & MK_RULE_ISO) ? 3 : 1]++;
        }
    }
    /* 3. emptying: liquid neighbours of emptied cells become interface cells,
     * keeping their PDFs and mass */
    for (int64_t c = 0; c < N; ++c) {
        if (!(mk[c] & MK_EMPTY)) continue;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y >= 0 && L->type[y] == OL_LIQUID && !(mk[y] & MK_NEW_FROM_LIQ)) {
                mk[y] |= MK_NEW_FROM_LIQ;
                L->cnt[6]++;
            }
        }
    }
    /* commit the new cell types */
    for (int64_t c = 0; c < N; ++c) {
        if (mk[c] & MK_TO_LIQ) L->type[c] = OL_LIQUID;
        else if (mk[c] & MK_EMPTY) L->type[c] = OL_GAS;
        else if (mk[c] & (MK_NEW_FROM_GAS | MK_NEW_FROM_LIQ)) L->type[c] = OL_INTERFACE;
    }
}

/* ---- phase 4: excess mass ------------------------------------------------ */
/* weight of the link c_i from a converted cell with normal n (liquid to gas)
 * in the normal-weighted variant: a filled cell sends its excess along n, an
 * emptied one against it; projections up to the normal tie count as zero */
static double excess_weight(const OlLattice *L, const double n[3], int i, int filled)
{
    double nc = n[0] * CV[i][0] + n[1] * CV[i][1] + n[2] * CV[i][2];
    if (!filled) nc = -nc;
    return nc > L->p.normal_tie ? nc : 0.0;
}

static void phase_excess(OlLattice *L)
{
    const int64_t N = L->N;
    uint8_t *mk = L->mark;
    const int weighted = (L->p.variants & OL_VAR_NORMAL_EXCESS) != 0;
    for (int64_t c = 0; c < N; ++c) {
        L->share[c] = 0.0;
        mk[c] &= (uint8_t)~MK_WEIGHTED;
        int filled = (mk[c] & MK_TO_LIQ) != 0, emptied = (mk[c] & MK_EMPTY) != 0;
        if (!filled && !emptied) continue;
        double e;
        if (filled) {
            e = L->m[c] - L->rho[c];
            L->m[c] = L->rho[c];
        } else {
            e = L->m[c];
            L->m[c] = 0.0;
        }
        int recv = 0;
        double wsum = 0.0;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y >= 0 && L->type[y] == OL_INTERFACE) {
                recv++;
                if (weighted) wsum += excess_weight(L, &L->n[3 * c], i, filled);
            }
        }
        if (wsum > 0.0) {
            /* receiver y = c + c_i takes share * weight of c_i */
            L->share[c] = e / wsum;
            mk[c] |= MK_WEIGHTED;
        } else if (recv > 0) {
            L->share[c] = e / recv;
        } else {
            L->pool += e;
        }
    }
    /* every interface cell gathers the shares of its converted neighbours in
     * direction order; seen from the neighbour y = c + c_i, c lies along
     * -c_i */
    for (int64_t c = 0; c < N; ++c) {
        if (L->type[c] != OL_INTERFACE) continue;
        double add = 0.0;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            int64_t y = nbr(L, c, i, +1);
            if (y < 0 || !(mk[y] & (MK_TO_LIQ | MK_EMPTY))) continue;
            if (mk[y] & MK_WEIGHTED)
                add += L->share[y] * excess_weight(L, &L->n[3 * y], opp(i), (mk[y] & MK_TO_LIQ) != 0);
            else
                add += L->share[y];
        }
        L->m[c] += add;
    }
    refresh_fill(L);
}

void ol_phase(OlLattice *L, int32_t phase)
{
    tables();
    switch (phase) {
    case 1: phase_stream_collide(L); break;
    case 2: phase_marks(L); break;
    case 3: phase_convert(L); break;
    case 4: phase_excess(L); break;
    case 5: phase_geometry(L); break;
    default: break;
    }
}

void ol_step(OlLattice *L, int32_t nsteps)
{
    tables();
    for (int32_t s = 0; s < nsteps; ++s) {
        phase_stream_collide(L);
        phase_marks(L);
        phase_convert(L);
        phase_excess(L);
        phase_geometry(L);
        L->steps++;
    }
}

void ol_set_estimator(OlLattice *L, const double *P)
{
    free(L->est_P);
    free(L->est_rule);
    free(L->est_q);
    L->est_P = NULL;
    L->est_rule = NULL;
    L->est_q = NULL;
    if (P) {
        const int32_t np = ol_mlp_nparam();
        L->est_P = (double *)malloc((size_t)np * sizeof(double));
        memcpy(L->est_P, P, (size_t)np * sizeof(double));
        L->est_rule = (uint8_t *)calloc((size_t)L->N, 1);
        L->est_q = (double *)calloc((size_t)L->N * 3, sizeof(double));
    }
    phase_geometry(L);
}

void ol_read(const OlLattice *L, int32_t field, void *dst)
{
    const int64_t N = L->N;
    switch (field) {
    case OL_F_TYPE: memcpy(dst, L->type, (size_t)N); break;
    case OL_F_MASS: memcpy(dst, L->m, (size_t)N * sizeof(double)); break;
    case OL_F_FILL: memcpy(dst, L->phi, (size_t)N * sizeof(double)); break;
    case OL_F_RHO: memcpy(dst, L->rho, (size_t)N * sizeof(double)); break;
    case OL_F_VEL: {
        double *o = (double *)dst;
        for (int64_t c = 0; c < N; ++c) {
            const double *f = &L->f[c * Q];
            double r = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < Q; ++i) {
                r += f[i];
                for (int d = 0; d < 3; ++d) j[d] += f[i] * CV[i][d];
            }
            for (int d = 0; d < 3; ++d) o[d * N + c] = (j[d] - 0.5 * r * L->p.accel[d]) / r;
        }
        break;
    }
    case OL_F_PDF: {
        double *o = (double *)dst;
        for (int64_t c = 0; c < N; ++c)
            for (int i = 0; i < Q; ++i) o[(int64_t)i * N + c] = L->f[c * Q + i];
        break;
    }
    case OL_F_NORMAL: {
        double *o = (double *)dst;
        for (int64_t c = 0; c < N; ++c)
            for (int d = 0; d < 3; ++d) o[d * N + c] = L->n[3 * c + d];
        break;
    }
    case OL_F_CURV: memcpy(dst, L->kappa, (size_t)N * sizeof(double)); break;
    case OL_F_OWNER: memcpy(dst, L->owner, (size_t)N * sizeof(int32_t)); break;
    case OL_F_MARKS: memcpy(dst, L->mark, (size_t)N); break;
    case OL_F_EST_RULE:
        if (L->est_rule) memcpy(dst, L->est_rule, (size_t)N);
        else memset(dst, 0, (size_t)N);
        break;
    case OL_F_EST_Q: {
        double *o = (double *)dst;
        for (int64_t c = 0; c < N; ++c)
            for (int d = 0; d < 3; ++d) o[d * N + c] = L->est_q ? L->est_q[3 * c + d] : 0.0;
        break;
    }
    default: break;
    }
}

double ol_total_mass(const OlLattice *L)
{
    double s = 0.0;
    for (int64_t c = 0; c < L->N; ++c)
        if (L->type[c] == OL_LIQUID || L->type[c] == OL_INTERFACE) s += L->m[c];
    return s + L->pool;
}

double ol_pool(const OlLattice *L) { return L->pool; }

void ol_counters(const OlLattice *L, int64_t out[8])
{
    for (int i = 0; i < 8; ++i) out[i] = L->cnt[i];
}

int64_t ol_steps_done(const OlLattice *L) { return L->steps; }

/* Move the spheres to new centres with new velocities (radii and number
 * unchanged).  Section 2.2 resolves moving particles on the lattice; the
 * remapping rules are readings:
 *   - the owner map is rebuilt (a cell covered by several spheres belongs to
 *     the lowest index);
 *   - a fluid cell that a sphere now covers becomes solid and its mass goes
 *     to the pool, so the total stays exact;
 *   - a solid cell that no sphere covers any more is typed from its 26
 *     neighbours: with liquid or interface neighbours and no gas
 *     neighbour it becomes liquid, with both an interface cell of fill 0,
 *     with gas neighbours only gas.  Uncovered cells are typed in rounds:
 *     a round takes every open cell with a neighbour typed before it (the
 *     lattice after the covering, then earlier rounds) and looks only at
 *     those; cells no round reaches become gas.  Liquid and interface cells
 *     get f = f^eq(rho_n, u), rho_n the mean density of those liquid and
 *     interface neighbours (for cells typed in an earlier round: their
 *     rho_n), u the rigid velocity of the sphere that covered the cell, at
 *     its centre; a liquid cell takes its mass rho_n out of the pool.
 * Returns -1 when no spheres are mapped. */
int ol_move_particles(OlLattice *L, const double *centre, const double *vel, const double *angvel)
{
    const int nx = L->p.nx, ny = L->p.ny, nz = L->p.nz, n = L->nsph;
    if (n <= 0) return -1;
    for (int32_t q = 0; q < n; ++q) {
        double *s = &L->sph[10 * q];
        s[0] = centre[3 * q] - nx * floor(centre[3 * q] / nx);
        s[1] = centre[3 * q + 1] - ny * floor(centre[3 * q + 1] / ny);
        s[2] = centre[3 * q + 2];
        for (int d = 0; d < 3; ++d) {
            s[4 + d] = vel ? vel[3 * q + d] : 0.0;
            s[7 + d] = angvel ? angvel[3 * q + d] : 0.0;
        }
    }
    int32_t *own = (int32_t *)malloc((size_t)L->N * sizeof(int32_t));
    uint8_t *t0 = (uint8_t *)malloc((size_t)L->N);
    uint8_t *tn = (uint8_t *)malloc((size_t)L->N);
    double *rn = (double *)malloc((size_t)L->N * sizeof(double));
    for (int64_t c = 0; c < L->N; ++c) {
        own[c] = -1;
        t0[c] = L->type[c];
    }
    for (int32_t q = 0; q < n; ++q) {
        const double *s = &L->sph[10 * q];
        const double r = s[3];
        int x0 = (int)floor(s[0] - r) - 1, x1 = (int)floor(s[0] + r) + 1;
        int y0 = (int)floor(s[1] - r) - 1, y1 = (int)floor(s[1] + r) + 1;
        int z0 = (int)floor(s[2] - r) - 1, z1 = (int)floor(s[2] + r) + 1;
        if (z0 < 0) z0 = 0;
        if (z1 > nz - 1) z1 = nz - 1;
        for (int z = z0; z <= z1; ++z)
            for (int yy = y0; yy <= y1; ++yy)
                for (int xx = x0; xx <= x1; ++xx) {
                    const int x = ((xx % nx) + nx) % nx, y = ((yy % ny) + ny) % ny;
                    const int64_t c = cell_of(L, x, y, z);
                    if (own[c] >= 0) continue;
                    const double dx = min_image((x + 0.5) - s[0], nx);
                    const double dy = min_image((y + 0.5) - s[1], ny);
                    const double dz = (z + 0.5) - s[2];
                    if (dx * dx + dy * dy + dz * dz <= r * r) own[c] = q;
                }
    }
    /* covering */
    for (int64_t c = 0; c < L->N; ++c) {
        if (own[c] < 0 || t0[c] == OL_SOLID) continue;
        if (t0[c] == OL_LIQUID || t0[c] == OL_INTERFACE) L->pool += L->m[c];
        L->type[c] = OL_SOLID;
        L->m[c] = 0.0;
        L->phi[c] = 0.0;
    }
    /* uncovered cells, in rounds: a round types every open cell that has a
     * neighbour typed before the round (the covered lattice, then earlier
     * rounds), from those neighbours only */
    double *dens = (double *)malloc((size_t)L->N * sizeof(double));
    uint8_t *tv = (uint8_t *)malloc((size_t)L->N); /* types as seen by the round */
    for (int64_t c = 0; c < L->N; ++c) {
        const int open = own[c] < 0 && t0[c] == OL_SOLID;
        tv[c] = open ? 255 : L->type[c];
        tn[c] = tv[c];
        dens[c] = (tv[c] == OL_LIQUID || tv[c] == OL_INTERFACE) ? sum27(&L->f[c * Q]) : 0.0;
        rn[c] = 1.0;
    }
    for (;;) {
        int64_t typed = 0;
        for (int64_t c = 0; c < L->N; ++c) {
            if (tv[c] != 255) continue;
            int nfl = 0, ngas = 0;
            double rs = 0.0;
            for (int i = 0; i < Q; ++i) {
                if (i == REST) continue;
                const int64_t y = nbr(L, c, i, 1);
                if (y < 0) continue;
                if (tv[y] == OL_LIQUID || tv[y] == OL_INTERFACE) {
                    ++nfl;
                    rs += dens[y];
                } else if (tv[y] == OL_GAS) {
                    ++ngas;
                }
            }
            if (nfl + ngas == 0) continue;
            tn[c] = nfl > 0 ? (ngas > 0 ? OL_INTERFACE : OL_LIQUID) : OL_GAS;
            rn[c] = nfl > 0 ? rs / nfl : 1.0;
            ++typed;
        }
        if (typed == 0) break;
        for (int64_t c = 0; c < L->N; ++c)
            if (tv[c] == 255 && tn[c] != 255) {
                tv[c] = tn[c];
                dens[c] = rn[c];
            }
    }
    for (int64_t c = 0; c < L->N; ++c)
        if (tn[c] == 255) tn[c] = OL_GAS; /* enclosed by solid cells */
    /* closure of the surface: a cell typed liquid in the same round as a
     * neighbour typed gas would border gas; it is an interface cell of
     * fill 0 instead */
    for (int64_t c = 0; c < L->N; ++c) {
        if (own[c] >= 0 || t0[c] != OL_SOLID || tn[c] != OL_LIQUID) continue;
        for (int i = 0; i < Q; ++i) {
            if (i == REST) continue;
            const int64_t y = nbr(L, c, i, 1);
            if (y < 0) continue;
            const int ty = (own[y] < 0 && t0[y] == OL_SOLID) ? tn[y] : L->type[y];
            if (ty == OL_GAS) {
                tn[c] = OL_INTERFACE;
                break;
            }
        }
    }
    free(dens);
    free(tv);
    for (int64_t c = 0; c < L->N; ++c) {
        if (own[c] >= 0 || t0[c] != OL_SOLID) continue;
        L->type[c] = tn[c];
        L->m[c] = 0.0;
        L->phi[c] = 0.0;
        if (tn[c] == OL_GAS) continue;
        /* rigid velocity of the sphere that covered the cell, at its centre */
        const double *s = &L->sph[10 * L->owner[c]];
        int x, y, z;
        cell_xyz(L, c, &x, &y, &z);
        const double r[3] = {min_image((x + 0.5) - s[0], nx), min_image((y + 0.5) - s[1], ny), (z + 0.5) - s[2]};
        const double u[3] = {s[4] + (s[8] * r[2] - s[9] * r[1]), s[5] + (s[9] * r[0] - s[7] * r[2]),
                             s[6] + (s[7] * r[1] - s[8] * r[0])};
        ol_feq(rn[c], u, &L->f[c * Q]);
        store_form(L, &L->f[c * Q]);
        L->rho[c] = rn[c];
        if (tn[c] == OL_LIQUID) {
            L->m[c] = rn[c];
            L->phi[c] = 1.0;
            L->pool -= rn[c];
        }
    }
    for (int64_t c = 0; c < L->N; ++c) L->owner[c] = own[c];
    free(own);
    free(t0);
    free(tn);
    free(rn);
    phase_geometry(L);
    return 0;
}

void ol_set_accel(OlLattice *L, const double accel[3])
{
    for (int d = 0; d < 3; ++d) L->p.accel[d] = accel[d];
}

/* Hydrodynamic force and torque on each sphere by momentum exchange
 * (Section 2.2 couples fluid and particles this way and cites Aidun et al.
 * 1998 and Wen et al. 2014; the form here is Wen's Galilean-invariant one).
 * Evaluated on the stored state, i.e. for the streaming of the next step:
 * every liquid or interface cell x with a link j whose source x - c_j is a
 * sphere cell sends f*_{opp j}(x) towards the wall and gets back
 * f_j = f*_{opp j} + 6 w_j c_j.u_w; relative to the wall velocity u_w at the
 * link midpoint, the sphere gains
 *   F = (c_{opp j} - u_w) f*_{opp j} - (c_j - u_w) f_j
 * and the torque r x F, r the midpoint's offset from the sphere centre.
 * out: 6 values per sphere, force then torque, summed in cell order. */
void ol_particle_forces(const OlLattice *L, double *out)
{
    for (int64_t k = 0; k < 6 * (int64_t)L->nsph; ++k) out[k] = 0.0;
    for (int64_t c = 0; c < L->N; ++c) {
        const uint8_t t = L->type[c];
        if (t != OL_LIQUID && t != OL_INTERFACE) continue;
        for (int j = 0; j < Q; ++j) {
            if (j == REST) continue;
            const int64_t s = nbr(L, c, j, -1);
            if (s < 0 || L->type[s] != OL_SOLID) continue;
            const int p = L->owner[s];
            double r[3], uw[3], F[3];
            link_offset(L, p, c, j, r);
            sphere_wall_velocity(L, p, c, j, uw);
            const double fout = L->f[c * Q + opp(j)];
            const double cu = CV[j][0] * uw[0] + CV[j][1] * uw[1] + CV[j][2] * uw[2];
            const double fin = fout + 6.0 * WT[j] * cu;
            for (int d = 0; d < 3; ++d)
                F[d] = (-CV[j][d] - uw[d]) * fout - (CV[j][d] - uw[d]) * fin;
            double *o = out + 6 * (int64_t)p;
            for (int d = 0; d < 3; ++d) o[d] += F[d];
            o[3] += r[1] * F[2] - r[2] * F[1];
            o[4] += r[2] * F[0] - r[0] * F[2];
            o[5] += r[0] * F[1] - r[1] * F[0];
        }
    }
}

void ol_set_threads(int32_t n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

int32_t ol_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
