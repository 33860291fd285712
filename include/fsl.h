/*
 * fsl.h -- C-ABI of the MI355X free-surface cumulant lattice Boltzmann step.
 *
 * The library advances a D3Q27 free-surface lattice (Schwarzmeier et al.,
 * "Particle-resolved simulation of antidunes in free-surface flows",
 * Section 2.1 for the fluid model, Section 2.2 for no-slip particle surfaces,
 * Section 3.1 for the boundary conditions and the driving body force) on one
 * gfx950 GPU.  One time step is: pull streaming with bounce-back at walls and
 * (moving) sphere surfaces, reconstruction of PDFs arriving from the gas side
 * with the gas pressure plus the Laplace pressure 2*sigma*kappa, the
 * volume-of-fluid mass flux, the cumulant collision (Geier et al. 2015: shear
 * rate omega, every other rate 1), conversion of interface cells with excess
 * mass redistribution, and the interface normal / curvature update.
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, reference density 1 (Section 2.1).
 *   - Cells are indexed cell = x + nx*(y + ny*z); every per-cell host array
 *     passed in or out uses that order (x fastest).  Vector fields are
 *     component-major: v[d*ncells + cell].
 *   - x and y are periodic; halfway bounce-back walls lie below z = 0 and
 *     above z = nz-1 (Section 3.1).
 *   - Device memory: the caller allocates one workspace of
 *     fsl_workspace_bytes() bytes (for example a torch uint8 tensor) and
 *     keeps it alive until fsl_destroy().  The library never frees caller
 *     memory; it owns only internal buffers sized by the sphere geometry
 *     (the sphere table and the moving-wall bounce-back terms of the cells
 *     next to spheres), allocated in fsl_set_particles().
 *   - Streams: all device work of a lattice is enqueued on the HIP stream
 *     given to fsl_create_lattice().  fsl_read_fields() and fsl_total_mass()
 *     synchronise that stream; fsl_step() does not.
 *   - Errors: every call returns an FslStatus; no exception crosses the ABI.
 *     fsl_last_error() returns a thread-local text for the last failure.
 *   - Host input arrays are copied during the call and may be freed after.
 */
#ifndef FSL_H
#define FSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct FslLattice FslLattice;

typedef enum {
    FSL_OK = 0,
    FSL_ERR_ARG = 1,       /* invalid argument (sizes, rates, non-finite input) */
    FSL_ERR_STATE = 2,     /* call not allowed in the lattice's current state */
    FSL_ERR_DEVICE = 3,    /* a HIP runtime call failed */
    FSL_ERR_NOMEM = 4,     /* workspace too small, or an internal allocation failed */
    FSL_ERR_UNSTABLE = 5   /* watchdog: total mass non-finite or drifted, or a
                              density outside [0.5, 1.5] (see fsl_step) */
} FslStatus;

/* Storage precision of the PDFs.  Mass, fill level, excess mass and the
 * total mass are kept in FP64 in every form. */
typedef enum {
    FSL_FP64 = 0,          /* PDFs stored as f - w in FP64, FP64 collision */
    FSL_FP32 = 1,          /* PDFs stored as f - w in FP32, FP32 collision */
    FSL_FP16_STORE = 2     /* PDFs stored as f - w in FP16 (round to nearest
                              even, subnormals kept), FP32 collision */
} FslPrecision;

typedef struct {
    int32_t nx, ny, nz;     /* lattice size, each >= 3 */
    int32_t precision;      /* FslPrecision */
    double omega;           /* shear relaxation rate, 0 < omega < 2;
                               nu = (1/omega - 1/2)/3 (Section 2.1) */
    double accel[3];        /* body acceleration g; force density rho*g
                               (driving force in x and gravity, Section 3.1) */
    double sigma;           /* surface tension (Laplace pressure 2 sigma kappa) */
    double rho_gas;         /* gas density; gas pressure p_g = rho_gas/3 */
    double conv_eps;        /* conversion threshold: fill above (1+eps), empty below -eps */
    double normal_tie;      /* a direction c_j is reconstructed from the gas side
                               when n.c_j < -normal_tie */
    int32_t rule_isolated;  /* 1: convert interface cells without gas (liquid)
                               neighbours to liquid (gas) */
    int32_t normals;        /* 0: finite-difference normal and curvature,
                               1: learned estimator with finite-difference fallback */
    int32_t check_every;    /* watchdog interval in steps (0: never; see fsl_step) */
    int32_t variants;       /* FSL_VAR_* bits; 0 is the model of Section 2.1
                               as the cited FSLBM and collision define it */
    int32_t grid_blocks;    /* 0: launch geometry chosen from the lattice size;
                               otherwise 8..2048 workgroups for the dense pass and
                               the interface-list kernels.  Results do not depend
                               on it (every cell is updated on its own, every
                               reduction has a fixed order per geometry); it
                               exists to test that. */
} FslParams;

/* Optional variants of the free surface (Thuerey 2007) and of the collision
 * (Geier et al. 2015), bits of FslParams.variants:
 *   FSL_VAR_FLUX_MODIFIERS  between two interface cells, mass moves only
 *     from a cell with gas but no liquid neighbours (which may only lose)
 *     and towards a cell with liquid but no gas neighbours (which may only
 *     gain); the classes come from the cell types at the start of the step.
 *   FSL_VAR_NORMAL_EXCESS   a cell that fills (empties) shares its excess
 *     mass among its interface neighbours in proportion to the positive
 *     part of n . c_i (of -n . c_i), n its normal from liquid to gas,
 *     projections up to normal_tie counting as zero; evenly when no link
 *     has a positive weight, and the pool takes it when there is no
 *     interface neighbour at all.
 *   FSL_VAR_CSF_CURVATURE   the curvature of the finite-difference estimator
 *     is half the divergence of the unit normal, from normals at the 8 cell
 *     corners of the 3x3x3 fill stencil (Brackbill et al. 1992; a corner
 *     gradient g below 0.01 gives the shortened normal -g/0.01, so that the
 *     curvature is continuous in the fill levels), instead of the Hessian
 *     form; needs normals == 0.
 *   FSL_VAR_GALILEAN        Galilean-invariance correction of the cumulant
 *     collision: D3Q27 cannot hold the cubic velocity moments, which puts an
 *     error of 3 rho u_a^2 d_a u_a into the normal stresses; the relaxed
 *     diagonal second-order cumulants lose 3 (1 - w/2) u_a^2 d_a u_a
 *     (w = omega for the deviator, 1 for the trace), the strain rates d_a u_a
 *     estimated from the cell's non-equilibrium second-order cumulants.
 *     Applies to every fluid cell (liquid and interface).
 * Unknown bits make fsl_create_lattice fail with FSL_ERR_ARG. */
enum { FSL_VAR_FLUX_MODIFIERS = 1, FSL_VAR_NORMAL_EXCESS = 2, FSL_VAR_CSF_CURVATURE = 4, FSL_VAR_GALILEAN = 8 };

/* field ids for fsl_read_fields(); bit k of the mask selects field k */
enum {
    FSL_FIELD_TYPE = 0,     /* uint8 [n]: 0 gas, 1 liquid, 2 interface, 3 solid */
    FSL_FIELD_MASS = 1,     /* double [n]: liquid mass m (0 for gas and solid) */
    FSL_FIELD_FILL = 2,     /* double [n]: fill level m/rho (1 liquid, 0 gas/solid) */
    FSL_FIELD_RHO = 3,      /* double [n]: density sum_i f_i of the stored PDFs
                               (liquid and interface cells; 0 elsewhere) */
    FSL_FIELD_VEL = 4,      /* double [3n]: (sum_i f_i c_i - F/2)/rho (fluid cells) */
    FSL_FIELD_PDF = 5,      /* double [27n]: f_i, direction-major f[i*n + cell],
                               i = (cx+1) + 3(cy+1) + 9(cz+1) (fluid cells) */
    FSL_FIELD_NORMAL = 6,   /* double [3n]: interface normal, liquid -> gas */
    FSL_FIELD_CURV = 7,     /* double [n]: mean curvature (interface cells) */
    FSL_FIELD_OWNER = 8,    /* int32 [n]: owning sphere of a solid cell, -1 otherwise */
    FSL_FIELD_ESTIMATOR = 9,/* uint8 [n]: outcome of the learned estimator for the
                               current geometry of each interface cell: 1 the corrected
                               estimate is used; finite differences kept because
                               2 a neighbour is solid or beyond a wall, 3 |n_raw| lies
                               outside [0.5, 2], 4 the angle to the finite-difference
                               normal exceeds 30 degrees, 5 |kappa| > 0.5 (the first
                               that holds, see fsl_set_estimator); 0 for other cells and
                               when no network is attached */
    FSL_NFIELDS = 10
};

/* Bytes of device workspace the lattice needs (0 for invalid params). */
size_t fsl_workspace_bytes(const FslParams *params);

/* Create a lattice in the caller's workspace and initialise it (Section 3.1:
 * fill level, density and velocity per cell).
 *   params      lattice and model parameters (copied)
 *   dev_workspace, bytes   device memory of at least fsl_workspace_bytes()
 *   hip_stream  hipStream_t on which all work is enqueued (NULL: default)
 *   fill        host double [n]: fill level; >= 1 liquid, <= 0 gas,
 *               in between interface.  A liquid cell next to a gas cell
 *               becomes an interface cell.
 *   rho         host double [n]: density (> 0)
 *   vel         host double [3n] component-major, or NULL for rest
 *   out         receives the lattice handle
 * Mass is m = clamp(fill, 0, 1) * rho and the PDFs start at equilibrium. */
FslStatus fsl_create_lattice(const FslParams *params, void *dev_workspace,
                             size_t bytes, void *hip_stream,
                             const double *fill, const double *rho,
                             const double *vel, FslLattice **out);

/* Map resolved spheres onto the lattice (Section 2.2: no-slip on particle
 * surfaces via bounce-back).  A cell is solid when its centre lies within
 * radius of a sphere centre (minimum image in x and y); the lowest sphere
 * index owns a cell covered twice.  Wall velocity at a link is
 * vel + angvel x (link midpoint - centre).
 *   n           number of spheres (>= 0)
 *   centre      host double [3n]; x and y are wrapped into the box
 *   radius      host double [n], 0 < r < min(nx, ny)/2
 *   vel         host double [3n] or NULL (at rest)
 *   angvel      host double [3n] or NULL (not rotating)
 * The geometry is mapped by the first call, which must come before the
 * first fsl_step(); later calls may only change velocities (same n, centres
 * after wrapping, radii), else FSL_ERR_STATE.  Mass inside newly solid
 * cells leaves the system. */
FslStatus fsl_set_particles(FslLattice *lat, int32_t n, const double *centre,
                            const double *radius, const double *vel,
                            const double *angvel);

/* Advance nsteps time steps (asynchronous on the lattice's stream).  One
 * step is the fluid update of Section 2.1 (pull streaming with bounce-back,
 * gas-side reconstruction, mass flux, cumulant collision), then interface
 * conversion with excess-mass redistribution and the interface geometry.
 * Every step's kernels also leave per-block partials of the total mass
 * (liquid and interface mass before the step's conversions, which only
 * move mass) and of the range of the fluid cells' densities, and the
 * excess-mass pool before the conversions (Section 2.1's mass
 * conservation).  Watchdog: on every check_every-th step the partials are
 * reduced in one fixed-order pass and the step then synchronises and returns FSL_ERR_UNSTABLE when the mass is not
 * finite, when some density lies outside [0.5, 1.5] (or is not a number), or
 * when the mass differs from the reference mass (the exact total of
 * fsl_total_mass() after fsl_create_lattice() or fsl_set_particles()) by
 * more than 1e-10 relative.  The state then stays readable and
 * fsl_watchdog() gives the values found.  Steps without a check do not
 * synchronise. */
FslStatus fsl_step(FslLattice *lat, int32_t nsteps);

/* Values of the last watchdog check (zeros before the first): out[0] total
 * mass, out[1] reference mass, out[2] lowest and out[3] highest fluid
 * density, out[4] number of fluid cells with a density outside [0.5, 1.5].
 * Host memory; no device work.  FSL_ERR_STATE for a NULL lattice,
 * FSL_ERR_ARG for a NULL out. */
FslStatus fsl_watchdog(FslLattice *lat, double out[5]);

/* Copy fields out (the state after the last step; Section 2.1's fluid
 * fields plus the free-surface bookkeeping).  dst[k] is the destination of
 * field k when bit k of field_mask is set (entries of unselected fields are
 * ignored); sizes and types per field are listed with FSL_FIELD_*.  dst
 * points to host memory, or to device memory when dst_on_device != 0.  Host
 * output is staged on the device: in a buffer of 24 bytes per cell that the
 * lattice allocates on first need and keeps until fsl_destroy(), and for
 * FSL_FIELD_PDF in a temporary one.  FSL_ERR_ARG for NULL destinations,
 * FSL_ERR_DEVICE for a failed copy or allocation.  Synchronises the
 * lattice's stream. */
FslStatus fsl_read_fields(FslLattice *lat, uint32_t field_mask, void *const *dst,
                          int32_t dst_on_device);

/* Total liquid mass: sum of m over liquid and interface cells plus the pool
 * of excess mass that found no interface neighbour (FP64, fixed summation
 * order; Section 2.1's mass bookkeeping).  Right after fsl_step() it is the
 * fixed-order sum of the last step's partials (one small kernel); otherwise
 * (after set-up or a remap that changed cell types) a pass over the
 * lattice recomputes it from the stored masses and PDFs.  The two agree to
 * rounding (the step's conversions only move mass).  Synchronises the
 * lattice's stream. */
FslStatus fsl_total_mass(FslLattice *lat, double *mass);

/* Cumulative conversion counters since creation: [0] filled by the mass
 * threshold, [1] emptied by the mass threshold, [2] filled by the no-gas-
 * neighbour rule, [3] emptied by the no-liquid-neighbour rule, [4] cancelled
 * emptyings, [5] gas -> interface, [6] liquid -> interface, [7] reserved (0).
 * Synchronises the lattice's stream. */
FslStatus fsl_counters(FslLattice *lat, int64_t out[8]);

/* Steps done and current number of interface cells (synchronises). */
FslStatus fsl_info(FslLattice *lat, int64_t *steps, int64_t *interface_cells);

/* Per-launch timing of the dense stream-collide kernel with HIP events on
 * the lattice's stream.  enable=1 starts recording (and clears the sums),
 * enable=0 stops.  fsl_timing_read() synchronises and returns the summed
 * kernel time in milliseconds and the number of timed launches. */
FslStatus fsl_timing(FslLattice *lat, int32_t enable);
FslStatus fsl_timing_read(FslLattice *lat, double *ms_total, int64_t *launches);

/* ---- learned interface estimator -------------------------------------
 * The paper needs the local curvature kappa only inside the Laplace
 * pressure 2 sigma kappa (Section 2.1) and leaves its estimate open.  Besides
 * the finite-difference estimate (Parker-Youngs normal, Hessian curvature of
 * the 3x3x3 fill stencil) the library offers a small network: 27 fill levels
 * (input clamp(phi, 0, 1) - 1/2, stencil entry a + 3b + 9c = offset
 * (a-1, b-1, c-1)) -> 64 -> 64 -> 4 with tanh hidden layers.  Inside a
 * lattice its outputs y correct the finite-difference estimate (n_fd, k_fd)
 * of the same stencil: n = (n_fd + y[0..2]) / |n_fd + y[0..2]| (liquid ->
 * gas), kappa = k_fd + y[3] / 4.  Weights are 6212 floats: W1[64][27],
 * b1[64], W2[64][64], b2[64], W3[4][64], b3[4] (row-major, out x in).
 * Matrix products run in BF16 on the matrix cores with FP32 accumulation;
 * the master weights are FP32.  Loss per sample against targets t:
 * |y[0..2] - t[0..2]|^2 + (y[3] - 4 t[3])^2, mean over the batch (for use
 * in a lattice, t = (n* - n_fd, kappa* - k_fd)).  Host arrays: x float
 * [n][27] fill levels, y float [n][4] targets. */
typedef struct {
    int32_t epochs;         /* passes over the data (> 0) */
    int32_t batch;          /* samples per Adam step (>= 16) */
    double lr, beta1, beta2, eps;   /* Adam (Kingma & Ba 2015) */
    uint64_t seed;          /* seeds the per-epoch shuffles */
} FslTrainParams;

/* Train in place: weights (host, 6212 floats) hold the initial values and
 * receive the trained ones; epoch_loss (host, epochs floats, may be NULL)
 * receives the mean batch loss of each epoch.  Synchronous on hip_stream. */
FslStatus fsl_estimator_train(const float *x, const float *y, int64_t n,
                              const FslTrainParams *tp, float *weights,
                              float *epoch_loss, void *hip_stream);

/* Mean loss and its gradient (6212 floats) over n samples, one pass. */
FslStatus fsl_estimator_grad(const float *weights, const float *x, const float *y,
                             int64_t n, float *grad, double *loss, void *hip_stream);

/* For callers that cannot allocate memory -- code under HIP graph capture,
 * tight training loops, harnesses that forbid hipMalloc: the mean loss and
 * its gradient of fsl_estimator_grad with every array in device memory,
 * owned by the caller: weights float [6212], x float [n][27] fill levels,
 * y float [n][4] targets (inputs); grad float [6212] and loss float [1]
 * (outputs).  Enqueued on hip_stream (NULL: default) without synchronising.
 * Allocates nothing: the packed weights and the partial sums live in a
 * device array of the library, about 6.4 MB, one per GPU for the life of
 * the process, shared by every call on that GPU -- calls that overlap on
 * one GPU (other streams, other host threads) race and must be serialised
 * by the caller.  Partial sums are formed over groups of samples in a fixed
 * order, so the result equals fsl_estimator_grad's to FP32 rounding of the
 * summation order.  FSL_ERR_ARG for a NULL pointer or n outside [1, 2^24],
 * FSL_ERR_DEVICE for a failed launch or symbol lookup. */
FslStatus fsl_estimator_grad_device(const float *weights, const float *x, const float *y,
                                    int64_t n, float *grad, float *loss, void *hip_stream);

/* Network outputs y float [n][4] for n stencils x float [n][27]. */
FslStatus fsl_estimator_infer(const float *weights, const float *x, int64_t n,
                              float *y, void *hip_stream);

/* Training stencils of the learned estimator (Section 2.1's normal and
 * curvature; analytic shapes): fill levels x float [n][27] (entry
 * a + 3b + 9c = the cell at offset (a-1, b-1, c-1) from the centre cell)
 * of n analytic shapes by supersampling each cell on ss^3 points
 * (i + 1/2)/ss - 1/2 per axis around its centre.  params double [n][16]
 * per shape: [0] kind (0 sphere, 1 sinusoidal sheet), [1] nonzero to take
 * the outside (1 - fraction: a bubble); sphere: [2..4] centre, [5] radius,
 * a point is inside if |p - centre|^2 <= radius^2; sheet: [2..4] e1,
 * [5..7] e3, [8] A, [9] k, [10] psi, [11] s, inside if
 * p.e3 < A sin(k p.e1 + psi) + s; the other entries are ignored.  The
 * tests are evaluated in FP64, each product and sum rounded on its own in
 * the order written.  Host arrays, owned by the caller; FSL_ERR_ARG for
 * NULL, n outside [1, 2^26] or ss outside [1, 64], FSL_ERR_DEVICE for a
 * failed allocation or launch; synchronises hip_stream. */
FslStatus fsl_estimator_stencils(const double *params, int64_t n, int32_t ss, float *x, void *hip_stream);

/* Finite-difference geometry (Section 2.1 curvature; Parker-Youngs normal
 * and Hessian mean curvature, evaluated in FP64) of n stencils x float
 * [n][27] of fill levels (entry a + 3b + 9c = offset (a-1, b-1, c-1);
 * values are clamped to [0, 1]).  y float [n][4] receives the unit normal
 * pointing from liquid to gas and kappa (0 where the gradient vanishes).
 * Host arrays, owned by the caller; FSL_ERR_ARG for NULL or n outside
 * [1, 2^30]; synchronises hip_stream.  This is the estimate the learned
 * network is compared with and falls back to. */
FslStatus fsl_fd_geometry(const float *x, int64_t n, float *y, void *hip_stream);

/* Attach trained weights to a lattice (weights: 6212 host floats, copied;
 * the first call allocates the weights and their BF16 copies with hipMalloc,
 * kept until fsl_destroy).  With params.normals == 1 the geometry of every
 * interface cell, the current ones included, then comes from the corrected
 * estimate, except where (rules checked in this order) 1. a neighbour is
 * solid or beyond a wall, 2. |n_fd + y[0..2]| is outside [0.5, 2], 3. the
 * corrected normal differs from the finite-difference one by more than 30
 * degrees, or 4. |kappa| > 0.5: there the finite-difference estimate is kept
 * (FSL_FIELD_ESTIMATOR reports which).  The network stands in for the
 * curvature estimate of the Laplace pressure 2 sigma kappa (Section 2.1);
 * the paper names no estimator.  FSL_ERR_ARG for NULL or non-finite
 * weights; synchronises the lattice's stream. */
FslStatus fsl_set_estimator(FslLattice *lat, const float *weights);

/* Move the spheres of fsl_set_particles() to new centres with new
 * velocities (radii and count unchanged); centre, vel, angvel: 3 doubles
 * per sphere (vel/angvel may be NULL: zero).  Section 2.2 resolves moving
 * particles on the lattice; the remapping is a reading:
 *   - if no cell changes owner, only the moving-wall terms follow the
 *     spheres (the common case: particles cross a cell in many steps);
 *   - otherwise fluid cells now covered turn solid and give their mass to
 *     the excess-mass pool; uncovered cells are typed in rounds from
 *     neighbours typed before each round: liquid (liquid or interface
 *     neighbours, no gas), interface of fill 0 (both), gas (gas only, or
 *     never reached); a cell typed liquid beside one typed gas in the same
 *     round is an interface cell of fill 0 instead (no liquid cell borders
 *     gas); liquid and interface cells get the equilibrium at the
 *     mean density of those neighbours and the sphere's rigid velocity at
 *     the cell centre, liquid cells taking that mass from the pool, so the
 *     total of fsl_total_mass() is unchanged; everything derived from the
 *     cell types is rebuilt.
 * FSL_ERR_STATE when no spheres are mapped, FSL_ERR_ARG for a NULL centre or
 * non-finite values.  The first call allocates a scratch buffer of 25
 * bytes per cell, kept until fsl_destroy().  Synchronises the stream. */
FslStatus fsl_move_particles(FslLattice *lat, const double *centre, const double *vel,
                             const double *angvel);

/* The same move with centre, vel and angvel in device memory (3 doubles per
 * sphere; vel/angvel may be NULL: zero), e.g. the particle state of
 * fsl_dem_read(..., out_on_device = 1), so that a coupled step keeps the
 * sphere state on the GPU.  The values are checked on the device before
 * anything changes (FSL_ERR_ARG for a non-finite value); then as
 * fsl_move_particles.  Synchronises the stream. */
FslStatus fsl_move_particles_device(FslLattice *lat, const double *centre, const double *vel,
                                    const double *angvel);

/* Change the body acceleration g (force density rho g) from the next step
 * on.  Section 3.1 drives the flume by a body force F_x controlled to hold
 * the bulk flow rate; the control law is the caller's (see
 * fsl_bulk_velocity).  FSL_ERR_ARG for NULL or non-finite values. */
FslStatus fsl_set_accel(FslLattice *lat, const double accel[3]);

/* Bulk velocity of the liquid: the fill-weighted mean of the velocity
 * u = (sum_i c_i f*_i - rho g / 2) / rho over liquid (weight 1) and
 * interface cells (weight = fill level); u[0..2] on the host.  FP64 sums in
 * a fixed order; synchronises the lattice's stream. */
FslStatus fsl_bulk_velocity(FslLattice *lat, double u[3]);

/* Bed profile (Section 3.2): phi_b[z*nx + x] = solid cells of the column
 * (x, z) divided by ny (the y-averaged solid-volume fraction on the
 * lattice), nz*nx values; h_b[x] = the bed height, the uppermost z at which
 * phi_b equals 0.3, interpolated linearly between cell centres z + 1/2
 * (0 without solid cells, nz when the top cell is at or above 0.3), nx
 * values.  Host memory, or device memory when out_on_device != 0.
 * Synchronises the lattice's stream; do not call it while steps that were
 * enqueued on another stream still run (host output is staged in a
 * per-step scratch array of the workspace). */
FslStatus fsl_bed_profile(FslLattice *lat, double *phi_b, double *h_b, int32_t out_on_device);

/* Hydrodynamic force and torque on every sphere by momentum exchange
 * (Section 2.2 couples fluid and particles this way, citing Aidun et al.
 * 1998 and Wen et al. 2014; this is Wen's Galilean-invariant form).  It is
 * evaluated on the current state, i.e. for the streaming of the next step:
 * each liquid or interface cell x with a link j whose source x - c_j is a
 * cell of sphere q sends f*_{-j}(x) towards the wall and receives
 * f_j = f*_{-j} + 6 w_j c_j.u_w (u_w: the sphere's rigid-body velocity at the
 * link midpoint); q gains (c_{-j} - u_w) f*_{-j} - (c_j - u_w) f_j and the
 * torque r x that force, r the midpoint's offset from the sphere centre
 * (minimum image in x and y).
 * out: 6 doubles per sphere in the order given to fsl_set_particles():
 * Fx, Fy, Fz, Tx, Ty, Tz (lattice units); host memory, or device memory when
 * out_on_device != 0.  Sums run in FP64 in a fixed order (deterministic).
 * Nothing is written when no spheres are mapped; FSL_ERR_ARG for a NULL out
 * otherwise.  The first call after set-up builds per-sphere lists of the
 * cells with links into each sphere (in a library buffer that grows with
 * hipMalloc when needed and is kept until fsl_destroy); the first call after
 * moves refills the lists of the spheres whose cells or box changed, and
 * rebuilds them all when one has outgrown its slot.  The result does not
 * depend on which of these happened.  Synchronises the lattice's stream. */
FslStatus fsl_particle_forces(FslLattice *lat, double *out, int32_t out_on_device);

/* Interface-cell updates since creation that used the network / fell back. */
FslStatus fsl_estimator_stats(FslLattice *lat, int64_t *learned, int64_t *fallback);

/* ---- particle motion (Section 2.2) -------------------------------------
 * Rigid spheres advanced by the Newton-Euler equations under a hydrodynamic
 * load (e.g. fsl_particle_forces), gravity, collisions and lubrication, with
 * several sub-steps per lattice step.  Section 2.2 parameterises the
 * collision model by e_dry, T_c, nu_p and mu_p and adds lubrication
 * corrections; the model details are readings of the cited coupling paper:
 *   normal contact: linear spring-dashpot on the overlap delta with
 *     k_n = m_eff (pi^2 + ln^2 e)/T_c^2, gamma_n = -2 m_eff ln(e)/T_c
 *     (a free binary collision rebounds with restitution e after T_c);
 *     m_eff = m_i m_j/(m_i + m_j), the free sphere's mass against a fixed
 *     sphere or a wall;
 *   tangential: a spring on the accumulated tangential displacement plus a
 *     dashpot, k_t = kappa k_n, gamma_t = sqrt(kappa) gamma_n with
 *     kappa = 2(1 - nu)/(2 - nu), capped by Coulomb friction mu |F_n|;
 *     forces act at the middle of the overlap;
 *   lubrication: -6 pi nu_f R_eff^2 u_n (1/s - 1/s_c) along the line of
 *     centres for gaps 0 < s < s_c (s taken >= s_min), R_eff = r_i r_j /
 *     (r_i + r_j) (r_i against a wall), u_n the normal approach speed; and
 *     -6 pi nu_f R_t ln(s_c/s) v_t on the tangential slip v_t of the facing
 *     surfaces at the middle of the gap, R_t = 4 r_i r_j (2 r_i^2 + r_i r_j +
 *     2 r_j^2) / (15 (r_i + r_j)^3) (8 r_i/15 against a wall);
 *   time: symplectic Euler per sub-step (forces from the sub-step's start,
 *     then velocities, then positions); x and y periodic, walls z = 0 and
 *     z = nz (the lattice's bounce-back planes); m = density 4/3 pi r^3,
 *     I = 2/5 m r^2; fixed spheres never move. */
typedef struct {
    int32_t nx, ny, nz;     /* box: periodic x in [0, nx), y in [0, ny); walls at z = 0, nz */
    double density;         /* particle density over fluid density (> 0) */
    double restitution;     /* e_dry in (0, 1] */
    double collision_time;  /* T_c (> 0), time units of the lattice */
    double poisson;         /* nu_p in [0, 0.5) */
    double friction;        /* mu_p >= 0 */
    double viscosity;       /* fluid kinematic viscosity nu_f (lubrication; fluid density 1) */
    double lub_cut;         /* s_c: lubrication for gaps below it (0: off) */
    double lub_min;         /* s_min > 0 */
    double accel[3];        /* acceleration of every sphere (gravity) */
    double dt;              /* time per step (> 0; one lattice step: 1) */
    int32_t substeps;       /* sub-steps per step (>= 1) */
    double skin;            /* > 0: neighbour lists hold spheres within r_i + r_j + s_c + skin */
} FslDemParams;

typedef struct FslDem FslDem;  /* opaque */

/* Create the particle state for n >= 1 spheres: centre, vel, angvel are 3
 * host doubles per sphere (vel/angvel may be NULL: zero), radius n doubles
 * (> 0), fixed n bytes or NULL.  Allocates about (36 + 6*32) doubles and
 * 66 int32 per sphere of device memory with hipMalloc (freed by
 * fsl_dem_destroy); all work runs on hip_stream (NULL: default).
 * FSL_ERR_ARG for invalid parameters or state, FSL_ERR_NOMEM. */
FslStatus fsl_dem_create(const FslDemParams *params, void *hip_stream, int32_t n,
                         const double *centre, const double *radius, const double *vel,
                         const double *angvel, const uint8_t *fixed, FslDem **out);

/* Advance nsteps steps of dt, each in `substeps` sub-steps, under hydro:
 * 6 doubles per sphere (force, torque; the order of fsl_particle_forces),
 * held over all sub-steps; host memory, or device memory when
 * hydro_on_device != 0; NULL for none.  Each step rebuilds the neighbour
 * lists; a sphere with more than 32 spheres within reach gives
 * FSL_ERR_NOMEM, a sphere that moves more than skin/2 within one step
 * FSL_ERR_UNSTABLE (the state stays readable; later steps report the same
 * error).  Forces sum in a fixed order (deterministic).  Synchronises the
 * stream. */
FslStatus fsl_dem_step(FslDem *dem, const double *hydro, int32_t hydro_on_device, int32_t nsteps);

/* Copy the state out: 3 doubles per sphere each (any may be NULL), centres
 * wrapped into [0, nx) x [0, ny); host memory, or device memory when
 * out_on_device != 0.  Synchronises the stream. */
FslStatus fsl_dem_read(FslDem *dem, double *centre, double *vel, double *angvel, int32_t out_on_device);

/* Bedload transport rate of Eq. (1) (Section 3.2): the sum over all spheres
 * of the streamwise velocity times the sphere volume 4/3 pi r^3, over the
 * bed area nx * ny; one double on the host.  Fixed-order sum
 * (deterministic); synchronises the stream.  FSL_ERR_ARG for a NULL qb. */
FslStatus fsl_dem_bedload(FslDem *dem, double *qb);

void fsl_dem_destroy(FslDem *dem);

/* Thread-local text of the last error (never NULL). */
const char *fsl_last_error(void);

/* Release the lattice's host state and internal buffers (not the workspace). */
void fsl_destroy(FslLattice *lat);

#ifdef __cplusplus
}
#endif
#endif
