"""ctypes wrapper of the plain FP64 CPU oracle (``fsl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark.  The GPU product path never imports it.

The C source is compiled with gcc on first use (or by :func:`build`), with
``-O2 -ffp-contract=off`` and no fast-math, so every operation rounds as
written.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fsl_oracle.c")
MLP_SRC = os.path.join(HERE, "mlp_oracle.c")
DEM_SRC = os.path.join(HERE, "dem_oracle.c")
HDR = os.path.join(HERE, "fsl_oracle.h")
LIB = os.path.join(HERE, "liboracle.so")

GAS, LIQUID, INTERFACE, SOLID = 0, 1, 2, 3
F_TYPE, F_MASS, F_FILL, F_RHO, F_VEL, F_PDF, F_NORMAL, F_CURV, F_OWNER, F_MARKS, F_EST_RULE, F_EST_Q = range(12)
# learned estimator, per interface cell: 1 the corrected estimate is used; 2..5 finite
# differences kept by a solid neighbour, |n_raw| outside [0.5, 2], an angle above 30
# degrees, |kappa| > 0.5 (0 elsewhere)
EST_NETWORK, EST_SOLID, EST_NORM, EST_ANGLE, EST_KAPPA = 1, 2, 3, 4, 5
VAR_FLUX_MODIFIERS, VAR_NORMAL_EXCESS, VAR_CSF_CURVATURE, VAR_GALILEAN = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` next to its source."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
        os.path.getmtime(SRC), os.path.getmtime(HDR), os.path.getmtime(MLP_SRC), os.path.getmtime(DEM_SRC)
    ):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp, SRC, MLP_SRC, DEM_SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _DemParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("density", ctypes.c_double), ("restitution", ctypes.c_double),
        ("collision_time", ctypes.c_double), ("poisson", ctypes.c_double),
        ("friction", ctypes.c_double), ("viscosity", ctypes.c_double),
        ("lub_cut", ctypes.c_double), ("lub_min", ctypes.c_double),
        ("accel", ctypes.c_double * 3), ("dt", ctypes.c_double), ("substeps", ctypes.c_int32),
    ]


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("omega", ctypes.c_double), ("omega_bulk", ctypes.c_double),
        ("omega_high", ctypes.c_double), ("accel", ctypes.c_double * 3),
        ("sigma", ctypes.c_double), ("rho_gas", ctypes.c_double),
        ("conv_eps", ctypes.c_double), ("normal_tie", ctypes.c_double),
        ("rule_isolated", ctypes.c_int32), ("store", ctypes.c_int32),
        ("variants", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # FSL_ORACLE_LIB points the pins at another build of the oracle (the
        # mutation test uses it to check that planted mistakes are caught)
        path = os.environ.get("FSL_ORACLE_LIB") or build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ol_create.restype = ctypes.c_void_p
        L.ol_create.argtypes = [ctypes.POINTER(_Params), dp, dp, dp]
        L.ol_destroy.argtypes = [ctypes.c_void_p]
        L.ol_set_particles.restype = ctypes.c_int
        L.ol_set_particles.argtypes = [ctypes.c_void_p, ctypes.c_int32, dp, dp, dp, dp]
        L.ol_set_state.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, dp]
        L.ol_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.ol_phase.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.ol_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.ol_total_mass.restype = ctypes.c_double
        L.ol_total_mass.argtypes = [ctypes.c_void_p]
        L.ol_pool.restype = ctypes.c_double
        L.ol_pool.argtypes = [ctypes.c_void_p]
        L.ol_counters.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        L.ol_steps_done.restype = ctypes.c_int64
        L.ol_steps_done.argtypes = [ctypes.c_void_p]
        L.ol_particle_forces.argtypes = [ctypes.c_void_p, dp]
        L.ol_set_accel.argtypes = [ctypes.c_void_p, dp]
        L.ol_move_particles.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.ol_move_particles.restype = ctypes.c_int
        L.ol_set_threads.argtypes = [ctypes.c_int32]
        L.ol_round_half.restype = ctypes.c_double
        L.ol_round_half.argtypes = [ctypes.c_double]
        L.ol_threads.restype = ctypes.c_int32
        L.ol_collide.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32, dp]
        L.ol_cumulants.argtypes = [dp, dp, dp]
        L.ol_feq.argtypes = [ctypes.c_double, dp, dp]
        L.ol_normal_curvature.argtypes = [dp, dp, dp]
        L.ol_csf_curvature.argtypes = [dp, dp]
        L.ol_velocities.argtypes = [ctypes.c_void_p, dp]
        L.ol_mlp_nparam.restype = ctypes.c_int32
        L.ol_mlp_forward.argtypes = [dp, ctypes.c_int32, dp, dp]
        L.ol_mlp_loss_grad.restype = ctypes.c_double
        L.ol_mlp_loss_grad.argtypes = [dp, ctypes.c_int32, dp, dp, dp]
        L.ol_mlp_adam.argtypes = [dp, dp, dp, dp, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.ol_estimator_compose.restype = ctypes.c_int32
        L.ol_estimator_compose.argtypes = [dp, dp, ctypes.c_int32, dp, dp, dp]
        L.ol_set_estimator.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.ol_dem_create.restype = ctypes.c_void_p
        L.ol_dem_create.argtypes = [ctypes.POINTER(_DemParams), ctypes.c_int32, dp, dp, dp, dp, ctypes.c_void_p]
        L.ol_dem_destroy.argtypes = [ctypes.c_void_p]
        L.ol_dem_step.argtypes = [ctypes.c_void_p, dp]
        L.ol_dem_read.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.ol_dem_bedload.restype = ctypes.c_double
        L.ol_dem_bedload.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def round_half(x: float) -> float:
    """Nearest FP16 value of x (ties to even), as the oracle's FP16 storage
    form rounds the stored deviations."""
    return float(lib().ol_round_half(float(x)))


def set_threads(n: int) -> int:
    """Threads of the per-cell phases (n <= 0: all processors); returns the
    number in use.  Results do not depend on it."""
    lib().ol_set_threads(int(n))
    return int(lib().ol_threads())


# ---------------------------------------------------------------- operators
def velocities():
    c = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    lib().ol_velocities(c.ctypes.data, _dp(w))
    return c, w


def collide(f, g=(0.0, 0.0, 0.0), omega=1.0, omega_bulk=1.0, omega_high=1.0, galilean=False):
    f = _f64(f)
    g = _f64(g)
    out = np.zeros(27)
    lib().ol_collide(_dp(f), _dp(g), omega, omega_bulk, omega_high, int(bool(galilean)), _dp(out))
    return out


def cumulants(f, g=(0.0, 0.0, 0.0)):
    f = _f64(f)
    g = _f64(g)
    out = np.zeros(27)
    lib().ol_cumulants(_dp(f), _dp(g), _dp(out))
    return out


def feq(rho, u):
    u = _f64(u)
    out = np.zeros(27)
    lib().ol_feq(float(rho), _dp(u), _dp(out))
    return out


def csf_curvature(phi27):
    """Curvature of a 3x3x3 stencil as half the divergence of the unit
    normals at the cell corners (Brackbill et al. 1992)."""
    p = _f64(phi27).reshape(27)
    k = np.zeros(1)
    lib().ol_csf_curvature(_dp(p), _dp(k))
    return float(k[0])


def normal_curvature(phi27):
    phi = _f64(phi27)
    n = np.zeros(3)
    k = np.zeros(1)
    lib().ol_normal_curvature(_dp(phi), _dp(n), _dp(k))
    return n, float(k[0])


# ------------------------------------------------------------------ lattice
class OracleLattice:
    """FP64 reference lattice.  Fields are (nz, ny, nx) arrays, x fastest."""

    def __init__(self, shape, omega, accel=(0.0, 0.0, 0.0), sigma=0.0, rho_gas=1.0,
                 conv_eps=1e-2, normal_tie=1e-6, rule_isolated=True,
                 omega_bulk=1.0, omega_high=1.0, fill=None, rho=None, vel=None, store="fp64",
                 flux_modifiers=False, normal_excess=False, csf_curvature=False, galilean=False):
        nx, ny, nz = shape
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        p = _Params()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.omega, p.omega_bulk, p.omega_high = omega, omega_bulk, omega_high
        for d in range(3):
            p.accel[d] = accel[d]
        p.sigma, p.rho_gas, p.conv_eps, p.normal_tie = sigma, rho_gas, conv_eps, normal_tie
        p.rule_isolated = 1 if rule_isolated else 0
        p.store = {"fp64": 0, "fp32": 1, "fp16": 2}[store]
        # variants of the free-surface model and of the collision (bits of the C header)
        p.variants = (VAR_FLUX_MODIFIERS if flux_modifiers else 0) | (VAR_NORMAL_EXCESS if normal_excess else 0) | \
            (VAR_CSF_CURVATURE if csf_curvature else 0) | (VAR_GALILEAN if galilean else 0)
        self._p = p
        fill = _f64(np.ones((nz, ny, nx)) if fill is None else fill).reshape(-1)
        rho = _f64(np.ones((nz, ny, nx)) if rho is None else rho).reshape(-1)
        vp = None
        if vel is not None:
            self._vel = _f64(vel).reshape(-1)
            vp = _dp(self._vel)
        h = lib().ol_create(ctypes.byref(p), _dp(fill), _dp(rho), vp)
        if not h:
            raise ValueError("oracle rejected the lattice parameters")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ol_destroy(h)
            self.h = None

    def set_particles(self, centre, radius, vel=None, angvel=None):
        centre = _f64(centre).reshape(-1)
        radius = _f64(radius).reshape(-1)
        n = radius.size
        v = _f64(np.zeros((n, 3)) if vel is None else vel).reshape(-1)
        w = _f64(np.zeros((n, 3)) if angvel is None else angvel).reshape(-1)
        rc = lib().ol_set_particles(self.h, n, _dp(centre), _dp(radius), _dp(v), _dp(w))
        if rc != 0:
            raise ValueError("oracle rejected the particles")
        self.nsph = n

    def set_state(self, type_, m, f_cellmajor):
        t = np.ascontiguousarray(type_, dtype=np.uint8).reshape(-1)
        m = _f64(m).reshape(-1)
        f = _f64(f_cellmajor).reshape(-1)
        assert t.size == self.N and m.size == self.N and f.size == 27 * self.N
        lib().ol_set_state(self.h, t.ctypes.data, _dp(m), _dp(f))

    def set_estimator(self, params):
        """Learned estimator with finite-difference fallback for the geometry
        of every interface cell from now on (params: 6212 values; None: finite
        differences only).  The current interface cells are re-evaluated."""
        if params is None:
            lib().ol_set_estimator(self.h, None)
            return
        self._est = _f64(params).reshape(-1)
        assert self._est.size == mlp_nparam()
        lib().ol_set_estimator(self.h, self._est.ctypes.data)

    def step(self, n=1):
        lib().ol_step(self.h, int(n))

    def phase(self, k):
        lib().ol_phase(self.h, int(k))

    def read(self, field):
        nx, ny, nz = self.shape
        N = self.N
        if field in (F_TYPE, F_MARKS, F_EST_RULE):
            out = np.zeros(N, dtype=np.uint8)
        elif field == F_OWNER:
            out = np.zeros(N, dtype=np.int32)
        elif field in (F_VEL, F_NORMAL, F_EST_Q):
            out = np.zeros(3 * N)
        elif field == F_PDF:
            out = np.zeros(27 * N)
        else:
            out = np.zeros(N)
        lib().ol_read(self.h, field, out.ctypes.data)
        if field in (F_VEL, F_NORMAL, F_EST_Q):
            return out.reshape(3, nz, ny, nx)
        if field == F_PDF:
            return out.reshape(27, nz, ny, nx)
        return out.reshape(nz, ny, nx)

    def total_mass(self):
        return lib().ol_total_mass(self.h)

    def pool(self):
        return lib().ol_pool(self.h)

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        lib().ol_counters(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return out

    @property
    def steps_done(self):
        return lib().ol_steps_done(self.h)

    def move_particles(self, centre, vel=None, angvel=None):
        n = getattr(self, "nsph", 0)
        centre = _f64(centre).reshape(-1)
        assert centre.size == 3 * n
        v = _f64(np.zeros((n, 3)) if vel is None else vel).reshape(-1)
        w = _f64(np.zeros((n, 3)) if angvel is None else angvel).reshape(-1)
        if lib().ol_move_particles(self.h, _dp(centre), _dp(v), _dp(w)) != 0:
            raise ValueError("no spheres to move")

    def set_accel(self, accel):
        a = _f64(accel).reshape(3)
        lib().ol_set_accel(self.h, _dp(a))

    def particle_forces(self):
        """(n, 6): force and torque on each sphere by momentum exchange for
        the streaming of the next step."""
        n = getattr(self, "nsph", 0)
        out = np.zeros(6 * max(n, 1))
        lib().ol_particle_forces(self.h, _dp(out))
        return out[:6 * n].reshape(n, 6)


# ------------------------------------------------------------------ estimator
MLP_SHAPES = (("W1", (64, 27)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (4, 64)), ("b3", (4,)))


def mlp_nparam():
    return int(lib().ol_mlp_nparam())


def mlp_forward(params, x):
    params = _f64(params)
    x = _f64(x).reshape(-1, 27)
    y = np.zeros((x.shape[0], 4))
    lib().ol_mlp_forward(_dp(params), x.shape[0], _dp(x), _dp(y))
    return y


def mlp_loss_grad(params, x, target, want_grad=True):
    params = _f64(params)
    x = _f64(x).reshape(-1, 27)
    target = _f64(target).reshape(-1, 4)
    g = np.zeros(params.size) if want_grad else None
    loss = lib().ol_mlp_loss_grad(_dp(params), x.shape[0], _dp(x), _dp(target),
                                  _dp(g) if want_grad else None)
    return loss, g


def mlp_adam(params, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    lib().ol_mlp_adam(_dp(params), _dp(m), _dp(v), _dp(_f64(grad)), int(t), lr, beta1, beta2, eps)


# ------------------------------------------------------------------ flume diagnostics
def bed_profile(type_field, threshold=0.3):
    """Section 3.2: the y-averaged solid-volume fraction phi_b(x, z) of every
    cell column (solid cells over ny) and the bed height h_b(x), the z at
    which phi_b equals the threshold, interpolated linearly between cell
    centres (z + 1/2).  The uppermost crossing counts; h_b = 0 without solid
    cells, nz when the top cell is still at or above the threshold.
    type_field: (nz, ny, nx).  Returns phi_b (nz, nx), h_b (nx)."""
    nz, ny, nx = type_field.shape
    phi = (type_field == SOLID).sum(axis=1) / float(ny)
    h = np.zeros(nx)
    for x in range(nx):
        k = -1
        for z in range(nz - 1, -1, -1):
            if phi[z, x] >= threshold:
                k = z
                break
        if k < 0:
            h[x] = 0.0
        elif k == nz - 1:
            h[x] = float(nz)
        else:
            h[x] = (k + 0.5) + (phi[k, x] - threshold) / (phi[k, x] - phi[k + 1, x])
    return phi, h


def bulk_velocity(o):
    """Section 3.1 holds the mean fluid velocity U_x,l at its target: here the
    fill-weighted mean of the velocity over liquid (fill 1) and interface
    cells, sum(fill * u) / sum(fill), all three components."""
    t = o.read(F_TYPE)
    fill = o.read(F_FILL)
    vel = o.read(F_VEL)
    w = np.where((t == LIQUID) | (t == INTERFACE), np.where(t == LIQUID, 1.0, fill), 0.0)
    return np.array([(w * vel[a]).sum() for a in range(3)]) / w.sum()


class FlowController:
    """Proportional-integral control of the body acceleration a_x so that the
    bulk velocity reaches `target` (Section 3.1 controls F_x to hold the bulk
    flow rate; the control law is a reading): every `every` steps,
    e = target - U_x, I += e, a_x = a0 + kp e + ki I."""

    def __init__(self, target, a0, kp, ki, every):
        self.target, self.a0, self.kp, self.ki, self.every = target, a0, kp, ki, every
        self.integral = 0.0

    def run(self, o, steps):
        ax = self.a0
        for s in range(0, steps, self.every):
            o.step(min(self.every, steps - s))
            e = self.target - bulk_velocity(o)[0]
            self.integral += e
            ax = self.a0 + self.kp * e + self.ki * self.integral
            o.set_accel((ax, 0.0, 0.0))
        return ax


# ------------------------------------------------------------------ particles
class OracleDem:
    """FP64 reference of the particle motion (dem_oracle.c): rigid spheres
    with contacts, lubrication, gravity and a given hydrodynamic load."""

    def __init__(self, box, centre, radius, vel=None, angvel=None, fixed=None, density=2.5,
                 restitution=0.97, collision_time=40.0, poisson=0.22, friction=0.5, viscosity=0.0,
                 lub_cut=0.0, lub_min=1e-3, accel=(0.0, 0.0, 0.0), dt=1.0, substeps=10):
        p = _DemParams()
        p.nx, p.ny, p.nz = (int(v) for v in box)
        p.density, p.restitution, p.collision_time = density, restitution, collision_time
        p.poisson, p.friction, p.viscosity = poisson, friction, viscosity
        p.lub_cut, p.lub_min, p.dt, p.substeps = lub_cut, lub_min, dt, int(substeps)
        for d in range(3):
            p.accel[d] = accel[d]
        centre = _f64(centre).reshape(-1, 3)
        self.n = n = centre.shape[0]
        self._keep = [_f64(centre).reshape(-1), _f64(radius).reshape(-1)]
        v = None if vel is None else _f64(vel).reshape(-1)
        w = None if angvel is None else _f64(angvel).reshape(-1)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8).reshape(-1)
        self._keep += [v, w, fx]
        L = lib()
        h = L.ol_dem_create(ctypes.byref(p), n, _dp(self._keep[0]), _dp(self._keep[1]),
                            _dp(v) if v is not None else None, _dp(w) if w is not None else None,
                            fx.ctypes.data if fx is not None else None)
        if not h:
            raise ValueError("oracle rejected the particle parameters")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ol_dem_destroy(h)
            self.h = None

    def step(self, hydro=None, n=1):
        hp = None
        if hydro is not None:
            self._hydro = _f64(hydro).reshape(-1)
            assert self._hydro.size == 6 * self.n
            hp = _dp(self._hydro)
        for _ in range(int(n)):
            lib().ol_dem_step(self.h, hp)

    def state(self):
        out = [np.zeros((self.n, 3)) for _ in range(3)]
        lib().ol_dem_read(self.h, *[_dp(o) for o in out])
        return out

    def bedload(self):
        """bedload transport rate q_b of Eq. (1)"""
        return lib().ol_dem_bedload(self.h)


def estimator_compose(params, phi27, solid_nb=False):
    """The learned estimator as a lattice applies it to one fill stencil
    (phi27 in direction order; solid_nb: a neighbour is solid or beyond a
    wall): returns (normal, kappa, rule, q) with rule 0 when the corrected
    estimate is used, else the first fallback rule (1 solid neighbour,
    2 |n_raw| outside [0.5, 2], 3 angle above 30 degrees, 4 |kappa| > 0.5),
    and q = (|n_raw|, angle in degrees, composed kappa)."""
    p = _f64(params)
    phi = _f64(phi27).reshape(27)
    n = np.zeros(3)
    k = np.zeros(1)
    q = np.zeros(3)
    rule = lib().ol_estimator_compose(_dp(p), _dp(phi), int(bool(solid_nb)), _dp(n), _dp(k), _dp(q))
    return n, float(k[0]), int(rule), q
