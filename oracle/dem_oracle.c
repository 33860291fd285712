/*
 * dem_oracle.c -- plain FP64 CPU oracle of the particle side of the coupled
 * method: rigid spheres under hydrodynamic load, gravity, collisions and
 * lubrication, advanced by sub-stepping within one lattice step.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
 * CPU baseline.  It shares no code with the GPU path.  Every pair of spheres
 * is examined every sub-step (no neighbour lists); contact histories live in
 * a per-sphere list.
 *
 * Section 2.2 of the paper (Schwarzmeier et al.) names the ingredients: the
 * Newton-Euler equations of each rigid particle, collisions by a discrete
 * element method parameterised by a dry restitution coefficient e_dry, a
 * collision time T_c, Poisson's ratio nu_p and a friction coefficient mu_p,
 * and lubrication corrections for gaps the lattice cannot resolve.  The model
 * details live in Rettinger and Ruede 2022, which is not available; the
 * readings used are published standard forms:
 *   normal contact  -- linear spring-dashpot on the overlap delta, with
 *                      stiffness k_n = m_eff (pi^2 + ln^2 e)/T_c^2 and damping
 *                      gamma_n = -2 m_eff ln(e)/T_c, which give a free binary
 *                      collision the restitution e and the duration T_c;
 *   tangential      -- a linear spring on the accumulated tangential
 *                      displacement plus a dashpot, capped by Coulomb
 *                      friction mu |F_n| (Cundall and Strack 1979); k_t =
 *                      kappa k_n with Mindlin's ratio kappa = 2(1-nu)/(2-nu)
 *                      for equal materials, gamma_t = sqrt(kappa) gamma_n;
 *                      forces act at the middle of the overlap;
 *   lubrication     -- the leading-order normal force between two spheres
 *                      (Brenner 1961): -6 pi mu R_eff^2 u_n / s with
 *                      R_eff = r1 r2/(r1 + r2), applied for gaps 0 < s < s_c
 *                      as -6 pi mu R_eff^2 u_n (1/s - 1/s_c) so that it
 *                      vanishes at the cut-off, s limited below by s_min;
 *                      and the leading tangential force -6 pi mu R_t
 *                      ln(1/s) v_t on the tangential slip v_t of the facing
 *                      surfaces, R_t = 4 r1 r2 (2 r1^2 + r1 r2 + 2 r2^2) /
 *                      (15 (r1 + r2)^3) (Jeffrey and Onishi 1984: r/6 for
 *                      equal spheres; 8 r/15 against a wall, Goldman, Cox
 *                      and Brenner 1967), applied as ln(s_c/s) at the
 *                      middle of the gap;
 *   integration     -- symplectic Euler per sub-step: forces from the state
 *                      at the start of the sub-step, then velocities, then
 *                      positions from the new velocities.
 * Walls: planes z = 0 and z = nz (where the lattice's bounce-back walls lie)
 * act as spheres of infinite radius and mass; x and y are periodic.
 */
#include "fsl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t other;    /* partner sphere of a contact of a lower-indexed sphere */
    double xi[3];     /* accumulated tangential displacement */
} Hist;

struct OlDem {
    OlDemParams p;
    int32_t n;
    double *x, *v, *w;     /* centre, velocity, angular velocity: 3 per sphere */
    double *r, *m, *inertia;
    uint8_t *fixed;
    Hist **hist;           /* per sphere: contacts with higher-indexed spheres */
    int32_t *nhist, *caph;
    double *wxi;           /* 2 walls x 3 per sphere: bottom, top */
};

static const double PI = 3.14159265358979323846;

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static double min_image(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

OlDem *ol_dem_create(const OlDemParams *p, int32_t n, const double *centre, const double *radius,
                     const double *vel, const double *angvel, const uint8_t *fixed)
{
    if (!p || n < 0 || (n > 0 && (!centre || !radius))) return NULL;
    if (!(p->density > 0.0 && p->restitution > 0.0 && p->restitution <= 1.0 && p->collision_time > 0.0 &&
          p->poisson >= 0.0 && p->poisson < 0.5 && p->friction >= 0.0 && p->viscosity >= 0.0 &&
          p->lub_cut >= 0.0 && p->lub_min > 0.0 && p->dt > 0.0 && p->substeps >= 1))
        return NULL;
    OlDem *D = (OlDem *)calloc(1, sizeof(OlDem));
    D->p = *p;
    D->n = n;
    size_t n3 = (size_t)(n > 0 ? n : 1) * 3;
    D->x = (double *)calloc(n3, sizeof(double));
    D->v = (double *)calloc(n3, sizeof(double));
    D->w = (double *)calloc(n3, sizeof(double));
    D->wxi = (double *)calloc(2 * n3, sizeof(double));
    D->r = (double *)calloc(n3, sizeof(double));
    D->m = (double *)calloc(n3, sizeof(double));
    D->inertia = (double *)calloc(n3, sizeof(double));
    D->fixed = (uint8_t *)calloc(n3, 1);
    D->hist = (Hist **)calloc(n3, sizeof(Hist *));
    D->nhist = (int32_t *)calloc(n3, sizeof(int32_t));
    D->caph = (int32_t *)calloc(n3, sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            D->x[3 * i + d] = centre[3 * i + d];
            D->v[3 * i + d] = vel ? vel[3 * i + d] : 0.0;
            D->w[3 * i + d] = angvel ? angvel[3 * i + d] : 0.0;
        }
        double r = radius[i];
        D->r[i] = r;
        D->m[i] = p->density * (4.0 / 3.0) * PI * r * r * r;
        D->inertia[i] = 0.4 * D->m[i] * r * r;
        D->fixed[i] = fixed ? fixed[i] : 0;
    }
    return D;
}

void ol_dem_destroy(OlDem *D)
{
    if (!D) return;
    for (int32_t i = 0; i < D->n; ++i) free(D->hist[i]);
    free(D->hist);
    free(D->nhist);
    free(D->caph);
    free(D->x);
    free(D->v);
    free(D->w);
    free(D->wxi);
    free(D->r);
    free(D->m);
    free(D->inertia);
    free(D->fixed);
    free(D);
}

/* tangential displacement record of the contact (lo, hi), created empty */
static double *history(OlDem *D, int32_t lo, int32_t hi)
{
    for (int32_t k = 0; k < D->nhist[lo]; ++k)
        if (D->hist[lo][k].other == hi) return D->hist[lo][k].xi;
    if (D->nhist[lo] == D->caph[lo]) {
        D->caph[lo] = D->caph[lo] ? 2 * D->caph[lo] : 8;
        D->hist[lo] = (Hist *)realloc(D->hist[lo], (size_t)D->caph[lo] * sizeof(Hist));
    }
    Hist *h = &D->hist[lo][D->nhist[lo]++];
    h->other = hi;
    h->xi[0] = h->xi[1] = h->xi[2] = 0.0;
    return h->xi;
}

static void forget(OlDem *D, int32_t lo, int32_t hi)
{
    for (int32_t k = 0; k < D->nhist[lo]; ++k)
        if (D->hist[lo][k].other == hi) {
            D->hist[lo][k] = D->hist[lo][D->nhist[lo] - 1];
            D->nhist[lo]--;
            return;
        }
}

/* Force on body a from a contact or a lubrication interaction with body b.
 *   n       unit normal from a towards b
 *   delta   overlap (> 0 in contact; -delta is the gap otherwise)
 *   vrel    velocity of a's surface point relative to b's, at the contact
 *   ucen    normal approach speed of the centres, (v_a - v_b) . n
 *   meff, reff   effective mass and radius (normal lubrication)
 *   rt      radius of the tangential lubrication force
 *   xi      tangential displacement record (updated), NULL for no contact
 * Returns the force on a in F and its tangential part in Ft (zero without
 * contact). */
static void pair_force(const OlDemParams *p, double h, const double n[3], double delta,
                       const double vrel[3], double ucen, double meff, double reff, double rt, double *xi,
                       double F[3], double Ft[3])
{
    F[0] = F[1] = F[2] = 0.0;
    Ft[0] = Ft[1] = Ft[2] = 0.0;
    if (delta > 0.0) {
        const double lne = log(p->restitution);
        const double kn = meff * (PI * PI + lne * lne) / (p->collision_time * p->collision_time);
        const double gn = -2.0 * meff * lne / p->collision_time;
        const double kappa = 2.0 * (1.0 - p->poisson) / (2.0 - p->poisson);
        const double kt = kappa * kn, gt = sqrt(kappa) * gn;
        const double un = dot3(vrel, n);
        const double fn = kn * delta + gn * un;          /* repulsive magnitude along -n */
        double vt[3];
        for (int d = 0; d < 3; ++d) vt[d] = vrel[d] - un * n[d];
        /* the spring stays in the current tangent plane */
        const double xn = dot3(xi, n);
        for (int d = 0; d < 3; ++d) xi[d] -= xn * n[d];
        for (int d = 0; d < 3; ++d) Ft[d] = -kt * xi[d] - gt * vt[d];
        const double ft = sqrt(dot3(Ft, Ft)), lim = p->friction * fabs(fn);
        if (ft > lim) {
            /* sliding: Coulomb force along the trial force; the spring is
             * reset to the length that produces it */
            for (int d = 0; d < 3; ++d) {
                Ft[d] = lim * Ft[d] / ft;
                xi[d] = -(Ft[d] + gt * vt[d]) / kt;
            }
        }
        for (int d = 0; d < 3; ++d) xi[d] += h * vt[d];
        for (int d = 0; d < 3; ++d) F[d] = -fn * n[d] + Ft[d];
    } else if (p->lub_cut > 0.0 && -delta < p->lub_cut) {
        double s = -delta;
        if (s < p->lub_min) s = p->lub_min;
        const double f = -6.0 * PI * p->viscosity * reff * reff * ucen * (1.0 / s - 1.0 / p->lub_cut);
        const double un = dot3(vrel, n);
        const double g = -6.0 * PI * p->viscosity * rt * log(p->lub_cut / s);
        for (int d = 0; d < 3; ++d) {
            Ft[d] = g * (vrel[d] - un * n[d]);
            F[d] = f * n[d] + Ft[d];
        }
    }
}

static void substep(OlDem *D, const double *hydro, double h)
{
    const OlDemParams *p = &D->p;
    const int32_t n = D->n;
    double *F = (double *)calloc((size_t)(n > 0 ? n : 1) * 3, sizeof(double));
    double *T = (double *)calloc((size_t)(n > 0 ? n : 1) * 3, sizeof(double));
    /* external load first: hydrodynamic force and torque, then gravity */
    for (int32_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            F[3 * i + d] = (hydro ? hydro[6 * i + d] : 0.0) + D->m[i] * p->accel[d];
            T[3 * i + d] = hydro ? hydro[6 * i + 3 + d] : 0.0;
        }
    /* pairs, lower index first; every body's sum runs over its partners in
     * index order */
    for (int32_t a = 0; a < n; ++a) {
        for (int32_t b = a + 1; b < n; ++b) {
            double dv[3];
            dv[0] = min_image(D->x[3 * b] - D->x[3 * a], (double)p->nx);
            dv[1] = min_image(D->x[3 * b + 1] - D->x[3 * a + 1], (double)p->ny);
            dv[2] = D->x[3 * b + 2] - D->x[3 * a + 2];
            const double dist = sqrt(dot3(dv, dv));
            const double ra = D->r[a], rb = D->r[b];
            const double delta = ra + rb - dist;
            if (delta <= -p->lub_cut || dist == 0.0) {
                forget(D, a, b);
                continue;
            }
            if (D->fixed[a] && D->fixed[b]) continue;
            double nv[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
            double meff;
            if (D->fixed[a]) meff = D->m[b];
            else if (D->fixed[b]) meff = D->m[a];
            else meff = D->m[a] * D->m[b] / (D->m[a] + D->m[b]);
            const double reff = ra * rb / (ra + rb);
            const double rt = 4.0 * ra * rb * (2.0 * ra * ra + ra * rb + 2.0 * rb * rb) /
                              (15.0 * (ra + rb) * (ra + rb) * (ra + rb));
            /* contact point in the middle of the overlap */
            const double la = ra - 0.5 * delta, lb = rb - 0.5 * delta;
            double wa[3], wb[3], arm_a[3] = {la * nv[0], la * nv[1], la * nv[2]};
            double arm_b[3] = {-lb * nv[0], -lb * nv[1], -lb * nv[2]};
            cross3(&D->w[3 * a], arm_a, wa);
            cross3(&D->w[3 * b], arm_b, wb);
            double vrel[3], vc[3];
            for (int d = 0; d < 3; ++d) {
                vc[d] = D->v[3 * a + d] - D->v[3 * b + d];
                vrel[d] = (D->v[3 * a + d] + wa[d]) - (D->v[3 * b + d] + wb[d]);
            }
            const double ucen = dot3(vc, nv);
            double *xi = NULL;
            if (delta > 0.0) xi = history(D, a, b);
            else forget(D, a, b);
            double f[3], ft[3];
            pair_force(p, h, nv, delta, vrel, ucen, meff, reff, rt, xi, f, ft);
            /* b takes the opposite force; both torques come from the
             * tangential force at the common contact point (the normal part
             * has no lever about either centre) */
            double ta[3], tb[3], ftb[3] = {-ft[0], -ft[1], -ft[2]};
            cross3(arm_a, ft, ta);
            cross3(arm_b, ftb, tb);
            for (int d = 0; d < 3; ++d) {
                F[3 * a + d] += f[d];
                T[3 * a + d] += ta[d];
                F[3 * b + d] -= f[d];
                T[3 * b + d] += tb[d];
            }
        }
    }
    /* walls: bottom (normal -z), then top (normal +z) */
    for (int32_t i = 0; i < n; ++i) {
        if (D->fixed[i]) continue;
        for (int k = 0; k < 2; ++k) {
            const double gap = k == 0 ? D->x[3 * i + 2] : (double)p->nz - D->x[3 * i + 2];
            const double delta = D->r[i] - gap;
            double *xi = &D->wxi[6 * i + 3 * k];
            if (delta <= -p->lub_cut) {
                xi[0] = xi[1] = xi[2] = 0.0;
                continue;
            }
            const double nv[3] = {0.0, 0.0, k == 0 ? -1.0 : 1.0};
            const double la = D->r[i] - 0.5 * delta;
            double wa[3], arm[3] = {la * nv[0], la * nv[1], la * nv[2]};
            cross3(&D->w[3 * i], arm, wa);
            double vrel[3];
            for (int d = 0; d < 3; ++d) vrel[d] = D->v[3 * i + d] + wa[d];
            const double ucen = D->v[3 * i + 2] * nv[2];
            if (delta <= 0.0) xi[0] = xi[1] = xi[2] = 0.0;
            double f[3], ft[3], t[3];
            pair_force(p, h, nv, delta, vrel, ucen, D->m[i], D->r[i], 8.0 * D->r[i] / 15.0,
                       delta > 0.0 ? xi : NULL, f, ft);
            cross3(arm, ft, t);
            for (int d = 0; d < 3; ++d) {
                F[3 * i + d] += f[d];
                T[3 * i + d] += t[d];
            }
        }
    }
    /* symplectic Euler */
    for (int32_t i = 0; i < n; ++i) {
        if (D->fixed[i]) continue;
        for (int d = 0; d < 3; ++d) {
            D->v[3 * i + d] += h * F[3 * i + d] / D->m[i];
            D->w[3 * i + d] += h * T[3 * i + d] / D->inertia[i];
            D->x[3 * i + d] += h * D->v[3 * i + d];
        }
        D->x[3 * i] -= p->nx * floor(D->x[3 * i] / p->nx);
        D->x[3 * i + 1] -= p->ny * floor(D->x[3 * i + 1] / p->ny);
    }
    free(F);
    free(T);
}

void ol_dem_step(OlDem *D, const double *hydro)
{
    const double h = D->p.dt / D->p.substeps;
    for (int32_t k = 0; k < D->p.substeps; ++k) substep(D, hydro, h);
}

void ol_dem_read(const OlDem *D, double *centre, double *vel, double *angvel)
{
    size_t b = (size_t)D->n * 3 * sizeof(double);
    if (centre) memcpy(centre, D->x, b);
    if (vel) memcpy(vel, D->v, b);
    if (angvel) memcpy(angvel, D->w, b);
}

/* Bedload transport rate of Eq. (1): the sum over all particles of the
 * streamwise velocity times the particle volume, over the bed area Lx Ly. */
double ol_dem_bedload(const OlDem *D)
{
    double q = 0.0;
    for (int32_t i = 0; i < D->n; ++i) {
        const double r = D->r[i];
        q += D->v[3 * i] * ((4.0 / 3.0) * PI * r * r * r);
    }
    return q / ((double)D->p.nx * (double)D->p.ny);
}
