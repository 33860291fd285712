/*
 * fsl_oracle.h -- plain FP64 CPU oracle of one free-surface cumulant LBM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
 * baseline call this library; the GPU product path never includes, links or
 * calls it, and it shares no code with the GPU path.
 *
 * What it computes (paper: "Particle-resolved simulation of antidunes in
 * free-surface flows", Section 2.1, and the methods cited there):
 *   - D3Q27 lattice in lattice units, dx = dt = 1, reference density 1;
 *   - cumulant collision of Geier et al. (2015), shear rate omega, every other
 *     rate 1 (parameters omega_bulk / omega_high exist only so that tests can
 *     exercise the moment/cumulant transforms; the paper's choice is 1);
 *   - pull streaming, bounce-back at walls and (moving) sphere surfaces;
 *   - the free-surface model: fill level, mass flux, gas-side reconstruction
 *     with gas pressure plus Laplace pressure 2*sigma*kappa, conversion of
 *     interface cells and redistribution of excess mass;
 *   - Parker-Youngs normal and finite-difference mean curvature.
 *
 * Storage is deliberately naive: cell-major full PDFs f[cell*27 + i], all in
 * double, cell = x + nx*(y + ny*z).  Direction i = (cx+1) + 3(cy+1) + 9(cz+1).
 */
#ifndef FSL_ORACLE_H
#define FSL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OL_GAS = 0, OL_LIQUID = 1, OL_INTERFACE = 2, OL_SOLID = 3 };

typedef struct {
    int32_t nx, ny, nz;         /* x and y periodic; halfway bounce-back walls below z=0 and above z=nz-1 */
    double omega;               /* shear relaxation rate, nu = (1/omega - 1/2)/3 */
    double omega_bulk;          /* rate of the trace of the second-order cumulants (paper: 1) */
    double omega_high;          /* rate of every cumulant of order 3..6 (paper: 1) */
    double accel[3];            /* body acceleration g; force density F = rho*g */
    double sigma;               /* surface tension */
    double rho_gas;             /* gas density, p_g = rho_gas/3 */
    double conv_eps;            /* conversion threshold epsilon */
    double normal_tie;          /* n.c_j must be below -normal_tie to trigger reconstruction */
    int32_t rule_isolated;      /* 1: apply the no-gas-neighbour / no-liquid-neighbour conversion rules */
    int32_t store;              /* storage form: 0 FP64; 1 and 2: every stored PDF is
                                   w_i + (f_i - w_i) rounded to the nearest FP32 (1) or FP16 (2)
                                   value, as the reduced-precision forms store deviations */
    int32_t variants;           /* OL_VAR_* bits; 0 is the model described above */
} OlParams;

/* Free-surface variants of the cited method (Thuerey 2007):
 *   OL_VAR_FLUX_MODIFIERS  interface cells with no liquid neighbour only give
 *     mass to other interface cells, those with no gas neighbour only take
 *     it (the exchange between two interface cells of different classes
 *     keeps one of its two PDF terms);
 *   OL_VAR_NORMAL_EXCESS   a converted cell shares its excess mass among its
 *     interface neighbours in proportion to the projection of its normal on
 *     the link (along the normal when filled, against it when emptied),
 *     evenly when no link has a positive projection;
 *   OL_VAR_CSF_CURVATURE   the curvature is half the divergence of the unit
 *     normal, from normals at the 8 cell corners (Brackbill et al. 1992;
 *     corner gradients below 0.01 give shortened normals -grad/0.01),
 *     instead of the Hessian form; the normal stays Parker-Youngs.
 * And of the collision (Geier et al. 2015):
 *   OL_VAR_GALILEAN        Galilean-invariance correction of the second-order
 *     cumulants: D3Q27 cannot hold the cubic velocity moments, which leaves
 *     an error of 3 rho u_a^2 d_a u_a in the normal stresses; the correction
 *     subtracts 3 (1 - w/2) u_a^2 d_a u_a from the relaxed diagonal cumulants
 *     (w = omega for the deviator, omega_bulk for the trace), with the
 *     strain rates d_a u_a estimated from the cell's own non-equilibrium
 *     second-order cumulants. */
enum { OL_VAR_FLUX_MODIFIERS = 1, OL_VAR_NORMAL_EXCESS = 2, OL_VAR_CSF_CURVATURE = 4, OL_VAR_GALILEAN = 8 };

typedef struct OlLattice OlLattice;

/* lattice tables (so that tests can check them) */
void ol_velocities(int32_t c[27][3], double w[27]);

/* --- single-cell operators ------------------------------------------------ */
/* collision of one cell; g = body acceleration; galilean = 1 adds the
 * Galilean-invariance correction (OL_VAR_GALILEAN); returns post-collision f */
void ol_collide(const double fin[27], const double g[3], double omega,
                double omega_bulk, double omega_high, int32_t galilean, double fout[27]);
/* the normalised pre-collision cumulants of one cell (index a+3b+9c for
 * C_{abc}); entry 0 holds rho, entries 1,3,9 hold the first-order central
 * moments (which the higher cumulants treat as zero) */
void ol_cumulants(const double fin[27], const double g[3], double C[27]);
/* product-form equilibrium */
void ol_feq(double rho, const double u[3], double feq[27]);
/* Parker-Youngs normal and mean curvature from a 3x3x3 fill-level stencil in
 * direction order (entry i is the cell at offset c_i) */
void ol_normal_curvature(const double phi[27], double n[3], double *kappa);
/* curvature of the same stencil as half the divergence of corner normals */
void ol_csf_curvature(const double phi[27], double *kappa);

/* --- learned estimator (mlp_oracle.c) -------------------------------------- */
/* number of network parameters (6212) */
int32_t ol_mlp_nparam(void);
/* the estimator as the lattice uses it (reading O18: the network output y
 * corrects the finite-difference estimate of the same stencil, n_raw = n_fd +
 * y[0..2], kappa = kappa_fd + y[3]/4, with a per-cell fallback to finite
 * differences).  phi: the fill stencil in direction order; solid_nb: a
 * neighbour is solid or beyond a wall.  Returns 0 when the corrected
 * estimate is used, else the first rule that keeps finite differences:
 * 1 solid neighbour, 2 |n_raw| outside [0.5, 2], 3 angle to n_fd above 30
 * degrees, 4 |kappa| > 0.5.  q (may be NULL): |n_raw|, angle, kappa. */
int32_t ol_estimator_compose(const double *P, const double phi[27], int32_t solid_nb, double n[3],
                             double *kappa, double q[3]);

/* --- lattice -------------------------------------------------------------- */
/* fill, rho: nx*ny*nz values; vel: 3*nx*ny*nz values (component-major:
 * vel[d*N + cell]) or NULL for rest.  Returns NULL on bad arguments. */
OlLattice *ol_create(const OlParams *p, const double *fill, const double *rho,
                     const double *vel);
void ol_destroy(OlLattice *L);
/* spheres: centre[n*3], radius[n], vel[n*3], angvel[n*3] (may be NULL).
 * Cells with |x_c - X| <= r (minimum image in x and y) become solid; the
 * lowest sphere index owns a cell covered by several spheres. */
int ol_set_particles(OlLattice *L, int32_t n, const double *centre,
                     const double *radius, const double *vel,
                     const double *angvel);
/* replace the whole state (used by tests that build states by hand):
 * type[N], m[N], f[N*27] (cell-major), normal[N*3] may be NULL -> recomputed */
void ol_set_state(OlLattice *L, const uint8_t *type, const double *m,
                  const double *f);
/* attach network weights (ol_mlp_nparam() doubles, copied; NULL: back to
 * finite differences): from now on the geometry of every interface cell,
 * including the current ones, comes from ol_estimator_compose */
void ol_set_estimator(OlLattice *L, const double *P);
/* full time steps */
void ol_step(OlLattice *L, int32_t nsteps);
/* one phase of the step, for unit tests:
 *   1 stream/boundaries/mass flux/collide, 2 conversion flags,
 *   3 conversion processing, 4 excess mass + fill refresh, 5 geometry */
void ol_phase(OlLattice *L, int32_t phase);

/* --- read back ------------------------------------------------------------ */
enum {
    OL_F_TYPE = 0,   /* uint8 [N] */
    OL_F_MASS = 1,   /* double [N] */
    OL_F_FILL = 2,   /* double [N] */
    OL_F_RHO = 3,    /* double [N], post-collision density sum_i f_i */
    OL_F_VEL = 4,    /* double [3*N] component-major, (sum f c - F/2)/rho */
    OL_F_PDF = 5,    /* double [27*N] direction-major f[i*N + cell] */
    OL_F_NORMAL = 6, /* double [3*N] component-major */
    OL_F_CURV = 7,   /* double [N] */
    OL_F_OWNER = 8,  /* int32 [N], -1 if not inside a sphere */
    OL_F_MARKS = 9,  /* uint8 [N], conversion marks of the last phase 2/3 */
    OL_F_EST_RULE = 10,  /* uint8 [N], learned estimator: 0 not an interface cell (or no
                            estimator), 1 corrected estimate used, 2..5 finite differences
                            kept by rule 1..4 of ol_estimator_compose */
    OL_F_EST_Q = 11      /* double [3*N] component-major: |n_raw|, angle to n_fd in
                            degrees, composed kappa (learned estimator, interface cells) */
};
void ol_read(const OlLattice *L, int32_t field, void *dst);
double ol_total_mass(const OlLattice *L);   /* sum of m over liquid+interface cells + pool */
double ol_pool(const OlLattice *L);
/* counters: [0] filled by rule a, [1] emptied by rule b, [2] filled by rule c,
 * [3] emptied by rule d, [4] cancelled emptyings, [5] gas->interface,
 * [6] liquid->interface, [7] liquid cells found next to gas (must stay 0) */
void ol_counters(const OlLattice *L, int64_t out[8]);
int64_t ol_steps_done(const OlLattice *L);
/* move the spheres to new centres and velocities (radii and number kept):
 * the owner map is rebuilt; covered fluid cells turn solid and give their
 * mass to the pool; uncovered cells, typed in rounds from neighbours typed
 * in earlier rounds, become liquid (fluid and no gas neighbours), empty
 * interface (both) or gas (gas only, or never reached) -- a cell typed
 * liquid beside one typed gas in the same round is an empty interface
 * cell instead, so that no liquid cell borders gas --, fluid ones at the
 * equilibrium of their neighbours' mean density and the sphere's rigid
 * velocity, liquid ones taking that mass from the pool.  -1 when no spheres
 * are mapped. */
int ol_move_particles(OlLattice *L, const double *centre, const double *vel, const double *angvel);
/* change the body acceleration between steps (Section 3.1 drives the flow
 * by a body force controlled to hold the bulk flow rate) */
void ol_set_accel(OlLattice *L, const double accel[3]);
/* hydrodynamic force and torque on each sphere by momentum exchange
 * (Galilean-invariant form, link midpoints) for the streaming of the next
 * step; out[6*n]: per sphere Fx, Fy, Fz, Tx, Ty, Tz (torque about the
 * sphere centre) */
void ol_particle_forces(const OlLattice *L, double *out);
/* threads of the per-cell phases (n <= 0: all processors; results do not
 * depend on it) and the number in use */
void ol_set_threads(int32_t n);
/* nearest FP16 value of x (ties to even, subnormals kept), as a double */
double ol_round_half(double x);
int32_t ol_threads(void);

/* --- particles (dem_oracle.c) --------------------------------------------- */
typedef struct {
    int32_t nx, ny, nz;         /* periodic x in [0, nx), y in [0, ny); walls z = 0, z = nz */
    double density;             /* particle density over fluid density */
    double restitution;         /* dry coefficient of restitution, (0, 1] */
    double collision_time;      /* duration of a free binary collision */
    double poisson;             /* Poisson's ratio, [0, 0.5) */
    double friction;            /* Coulomb friction coefficient */
    double viscosity;           /* fluid kinematic viscosity (fluid density 1) */
    double lub_cut;             /* lubrication acts for gaps below this (0: off) */
    double lub_min;             /* smallest gap the lubrication force uses */
    double accel[3];            /* acceleration of every particle (gravity) */
    double dt;                  /* time advanced by one ol_dem_step */
    int32_t substeps;           /* sub-steps per ol_dem_step */
} OlDemParams;

typedef struct OlDem OlDem;

/* centre, vel, angvel: 3 per sphere (vel, angvel may be NULL: zero); fixed:
 * n flags (NULL: none; fixed spheres never move).  NULL on bad arguments. */
OlDem *ol_dem_create(const OlDemParams *p, int32_t n, const double *centre, const double *radius,
                     const double *vel, const double *angvel, const uint8_t *fixed);
void ol_dem_destroy(OlDem *D);
/* one lattice step of particle motion under hydro[6 n] (force, torque per
 * sphere, held over the sub-steps; NULL: none) */
void ol_dem_step(OlDem *D, const double *hydro);
void ol_dem_read(const OlDem *D, double *centre, double *vel, double *angvel);
/* bedload transport rate, Eq. (1): sum_i u_x,i V_i / (Lx Ly) */
double ol_dem_bedload(const OlDem *D);

#ifdef __cplusplus
}
#endif
#endif
