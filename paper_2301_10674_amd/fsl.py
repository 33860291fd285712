"""Python binding of the C-ABI in ``include/fsl.h``.

Argument marshalling only: every step of the method runs in the HIP library
``libfsl.so`` built next to this file.  PyTorch provides the device workspace
and the stream.  There is no fallback: if the library is missing, every call
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsl.so")

FSL_OK, FSL_ERR_ARG, FSL_ERR_STATE, FSL_ERR_DEVICE, FSL_ERR_NOMEM, FSL_ERR_UNSTABLE = range(6)
FP64, FP32, FP16_STORE = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16_STORE}
FSL_VAR_FLUX_MODIFIERS, FSL_VAR_NORMAL_EXCESS, FSL_VAR_CSF_CURVATURE, FSL_VAR_GALILEAN = 1, 2, 4, 8  # variants bits
(FIELD_TYPE, FIELD_MASS, FIELD_FILL, FIELD_RHO, FIELD_VEL, FIELD_PDF, FIELD_NORMAL,
 FIELD_CURV, FIELD_OWNER, FIELD_ESTIMATOR) = range(10)
NFIELDS = 10
# FIELD_ESTIMATOR values: corrected estimate used, or finite differences kept
# because of a solid neighbour, |n_raw|, the angle, |kappa|
EST_NETWORK, EST_SOLID, EST_LENGTH, EST_ANGLE, EST_KAPPA = 1, 2, 3, 4, 5
GAS, LIQUID, INTERFACE, SOLID = 0, 1, 2, 3

# every symbol declared in include/fsl.h
EXPORTS = ("fsl_workspace_bytes", "fsl_create_lattice", "fsl_set_particles", "fsl_step",
           "fsl_read_fields", "fsl_total_mass", "fsl_counters", "fsl_info", "fsl_timing",
           "fsl_timing_read", "fsl_estimator_train", "fsl_estimator_grad", "fsl_estimator_infer",
           "fsl_fd_geometry", "fsl_estimator_stencils", "fsl_particle_forces", "fsl_set_accel", "fsl_bulk_velocity",
           "fsl_bed_profile", "fsl_move_particles", "fsl_move_particles_device",
           "fsl_set_estimator", "fsl_estimator_stats", "fsl_dem_create", "fsl_dem_step",
           "fsl_dem_read", "fsl_dem_bedload", "fsl_dem_destroy", "fsl_last_error", "fsl_destroy",
           "fsl_watchdog", "fsl_estimator_grad_device")
MLP_NPARAM = 6212


class FslError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fsl status %d: %s" % (status, msg))
        self.status = status


class FslParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("omega", ctypes.c_double),
        ("accel", ctypes.c_double * 3), ("sigma", ctypes.c_double),
        ("rho_gas", ctypes.c_double), ("conv_eps", ctypes.c_double),
        ("normal_tie", ctypes.c_double), ("rule_isolated", ctypes.c_int32),
        ("normals", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("variants", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
    ]


class FslDemParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("density", ctypes.c_double), ("restitution", ctypes.c_double),
        ("collision_time", ctypes.c_double), ("poisson", ctypes.c_double),
        ("friction", ctypes.c_double), ("viscosity", ctypes.c_double),
        ("lub_cut", ctypes.c_double), ("lub_min", ctypes.c_double),
        ("accel", ctypes.c_double * 3), ("dt", ctypes.c_double), ("substeps", ctypes.c_int32),
        ("skin", ctypes.c_double),
    ]


class FslTrainParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


def make_params(shape, precision="fp64", omega=1.0, accel=(0.0, 0.0, 0.0), sigma=0.0,
                rho_gas=1.0, conv_eps=1e-2, normal_tie=1e-6, rule_isolated=True,
                normals=0, check_every=0, flux_modifiers=False, normal_excess=False, csf_curvature=False,
                galilean=False, grid_blocks=0):
    p = FslParams()
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.omega = float(omega)
    for d in range(3):
        p.accel[d] = float(accel[d])
    p.sigma, p.rho_gas = float(sigma), float(rho_gas)
    p.conv_eps, p.normal_tie = float(conv_eps), float(normal_tie)
    p.rule_isolated = 1 if rule_isolated else 0
    p.normals, p.check_every = int(normals), int(check_every)
    p.variants = (FSL_VAR_FLUX_MODIFIERS if flux_modifiers else 0) | \
        (FSL_VAR_NORMAL_EXCESS if normal_excess else 0) | (FSL_VAR_CSF_CURVATURE if csf_curvature else 0) | \
        (FSL_VAR_GALILEAN if galilean else 0)
    p.grid_blocks = int(grid_blocks)
    return p


_lib = None


def lib():
    """Load libfsl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfsl.so is not built; run `python -m paper_2301_10674_amd.build`")
        # torch provides the device memory and streams: bring its HIP runtime
        # up first so the library binds to the same, initialised runtime
        import torch

        if torch.cuda.is_available():
            torch.cuda.init()
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32
        L.fsl_workspace_bytes.restype = ctypes.c_size_t
        L.fsl_workspace_bytes.argtypes = [ctypes.POINTER(FslParams)]
        L.fsl_create_lattice.restype = ctypes.c_int
        L.fsl_create_lattice.argtypes = [ctypes.POINTER(FslParams), vp, ctypes.c_size_t, vp,
                                         dp, dp, dp, ctypes.POINTER(vp)]
        L.fsl_set_particles.restype = ctypes.c_int
        L.fsl_set_particles.argtypes = [vp, i32, dp, dp, dp, dp]
        L.fsl_step.restype = ctypes.c_int
        L.fsl_step.argtypes = [vp, i32]
        L.fsl_read_fields.restype = ctypes.c_int
        L.fsl_read_fields.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(vp), i32]
        L.fsl_total_mass.restype = ctypes.c_int
        L.fsl_total_mass.argtypes = [vp, dp]
        L.fsl_watchdog.restype = ctypes.c_int
        L.fsl_watchdog.argtypes = [vp, dp]
        L.fsl_counters.restype = ctypes.c_int
        L.fsl_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.fsl_info.restype = ctypes.c_int
        L.fsl_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.fsl_timing.restype = ctypes.c_int
        L.fsl_timing.argtypes = [vp, i32]
        L.fsl_timing_read.restype = ctypes.c_int
        L.fsl_timing_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
        fp = ctypes.POINTER(ctypes.c_float)
        L.fsl_estimator_train.restype = ctypes.c_int
        L.fsl_estimator_train.argtypes = [fp, fp, ctypes.c_int64, ctypes.POINTER(FslTrainParams), fp, fp, vp]
        L.fsl_estimator_grad.restype = ctypes.c_int
        L.fsl_estimator_grad.argtypes = [fp, fp, fp, ctypes.c_int64, fp, dp, vp]
        L.fsl_estimator_grad_device.restype = ctypes.c_int
        L.fsl_estimator_grad_device.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp]
        L.fsl_estimator_infer.restype = ctypes.c_int
        L.fsl_estimator_infer.argtypes = [fp, fp, ctypes.c_int64, fp, vp]
        L.fsl_fd_geometry.restype = ctypes.c_int
        L.fsl_fd_geometry.argtypes = [fp, ctypes.c_int64, fp, vp]
        L.fsl_estimator_stencils.restype = ctypes.c_int
        L.fsl_estimator_stencils.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, fp, vp]
        L.fsl_set_estimator.restype = ctypes.c_int
        L.fsl_particle_forces.argtypes = [vp, dp, i32]
        L.fsl_set_accel.argtypes = [vp, dp]
        L.fsl_move_particles.argtypes = [vp, dp, dp, dp]
        L.fsl_move_particles_device.argtypes = [vp, vp, vp, vp]
        L.fsl_bulk_velocity.argtypes = [vp, dp]
        L.fsl_bed_profile.argtypes = [vp, dp, dp, i32]
        L.fsl_set_estimator.argtypes = [vp, fp]
        L.fsl_estimator_stats.restype = ctypes.c_int
        L.fsl_estimator_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.fsl_dem_create.restype = ctypes.c_int
        L.fsl_dem_create.argtypes = [ctypes.POINTER(FslDemParams), vp, i32, dp, dp, dp, dp, vp,
                                     ctypes.POINTER(vp)]
        L.fsl_dem_step.restype = ctypes.c_int
        L.fsl_dem_step.argtypes = [vp, vp, i32, i32]
        L.fsl_dem_read.restype = ctypes.c_int
        L.fsl_dem_read.argtypes = [vp, dp, dp, dp, i32]
        L.fsl_dem_bedload.restype = ctypes.c_int
        L.fsl_dem_bedload.argtypes = [vp, dp]
        L.fsl_dem_destroy.restype = None
        L.fsl_dem_destroy.argtypes = [vp]
        L.fsl_last_error.restype = ctypes.c_char_p
        L.fsl_last_error.argtypes = []
        L.fsl_destroy.restype = None
        L.fsl_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _check(status):
    if status != FSL_OK:
        raise FslError(status, lib().fsl_last_error().decode())


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32).reshape(-1)


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def workspace_bytes(params: FslParams) -> int:
    return int(lib().fsl_workspace_bytes(ctypes.byref(params)))


class Lattice:
    """A lattice living in a torch device workspace."""

    def __init__(self, params: FslParams, fill, rho, vel=None, device="cuda"):
        import torch

        self.params = params
        self.shape = (params.nx, params.ny, params.nz)
        self.nsph = 0
        self.N = params.nx * params.ny * params.nz
        nbytes = workspace_bytes(params)
        if nbytes == 0:
            raise FslError(FSL_ERR_ARG, lib().fsl_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.workspace.device)
        fill, rho, vel = _f64(fill), _f64(rho), _f64(vel)
        assert fill.size == self.N and rho.size == self.N
        assert vel is None or vel.size == 3 * self.N
        h = ctypes.c_void_p()
        _check(lib().fsl_create_lattice(ctypes.byref(params), ctypes.c_void_p(self.workspace.data_ptr()),
                                        nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                        _dp(fill), _dp(rho), _dp(vel), ctypes.byref(h)))
        self.h = h

    def __del__(self):
        self.destroy()

    def destroy(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().fsl_destroy(h)
        self.h = None

    def set_particles(self, centre, radius, vel=None, angvel=None):
        centre, radius = _f64(centre), _f64(radius)
        n = radius.size
        assert centre.size == 3 * n
        vel, angvel = _f64(vel), _f64(angvel)
        _check(lib().fsl_set_particles(self.h, n, _dp(centre), _dp(radius), _dp(vel), _dp(angvel)))
        self.nsph = n

    def step(self, n=1):
        _check(lib().fsl_step(self.h, int(n)))

    def read_fields(self, fields):
        """Read the given field ids into new host arrays shaped (.., nz, ny, nx)."""
        nx, ny, nz = self.shape
        N = self.N
        outs = {}
        ptrs = (ctypes.c_void_p * NFIELDS)()
        mask = 0
        for f in fields:
            if f in (FIELD_TYPE, FIELD_ESTIMATOR):
                a = np.zeros(N, dtype=np.uint8)
            elif f == FIELD_OWNER:
                a = np.zeros(N, dtype=np.int32)
            elif f in (FIELD_VEL, FIELD_NORMAL):
                a = np.zeros(3 * N)
            elif f == FIELD_PDF:
                a = np.zeros(27 * N)
            else:
                a = np.zeros(N)
            outs[f] = a
            ptrs[f] = a.ctypes.data
            mask |= 1 << f
        _check(lib().fsl_read_fields(self.h, mask, ptrs, 0))
        res = {}
        for f, a in outs.items():
            if f in (FIELD_VEL, FIELD_NORMAL):
                res[f] = a.reshape(3, nz, ny, nx)
            elif f == FIELD_PDF:
                res[f] = a.reshape(27, nz, ny, nx)
            else:
                res[f] = a.reshape(nz, ny, nx)
        return res

    def read(self, field):
        return self.read_fields([field])[field]

    def total_mass(self):
        m = ctypes.c_double()
        _check(lib().fsl_total_mass(self.h, ctypes.byref(m)))
        return m.value

    def counters(self):
        out = (ctypes.c_int64 * 8)()
        _check(lib().fsl_counters(self.h, out))
        return np.array(out[:], dtype=np.int64)

    def info(self):
        s, n = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fsl_info(self.h, ctypes.byref(s), ctypes.byref(n)))
        return s.value, n.value

    def timing(self, enable):
        _check(lib().fsl_timing(self.h, 1 if enable else 0))

    def move_particles(self, centre, vel=None, angvel=None):
        centre = _f64(centre)
        assert centre.size == 3 * self.nsph
        vel, angvel = _f64(vel), _f64(angvel)
        _check(lib().fsl_move_particles(self.h, _dp(centre), _dp(vel), _dp(angvel)))

    def move_particles_device(self, centre, vel=None, angvel=None):
        """the same with CUDA float64 tensors of 3 values per sphere"""
        def ptr(t):
            if t is None:
                return None
            assert t.is_cuda and t.dtype == _torch().float64 and t.is_contiguous() and t.numel() == 3 * self.nsph
            return ctypes.c_void_p(t.data_ptr())
        _check(lib().fsl_move_particles_device(self.h, ptr(centre), ptr(vel), ptr(angvel)))

    def set_accel(self, accel):
        a = _f64(accel).reshape(3)
        _check(lib().fsl_set_accel(self.h, _dp(a)))

    def bulk_velocity(self):
        u = np.zeros(3)
        _check(lib().fsl_bulk_velocity(self.h, _dp(u)))
        return u

    def bed_profile(self):
        """(phi_b (nz, nx), h_b (nx)): y-averaged solid fraction and bed height."""
        nx, ny, nz = self.shape
        phi, h = np.zeros(nz * nx), np.zeros(nx)
        _check(lib().fsl_bed_profile(self.h, _dp(phi), _dp(h), 0))
        return phi.reshape(nz, nx), h

    def particle_forces(self):
        """(n, 6) array: force and torque on each sphere by momentum
        exchange for the streaming of the next step (fsl_particle_forces)."""
        n = self.nsph
        out = np.zeros(6 * max(n, 1))
        _check(lib().fsl_particle_forces(self.h, _dp(out), 0))
        return out[:6 * n].reshape(n, 6)

    def particle_forces_device(self):
        """(n, 6) CUDA float64 tensor of the same force and torque"""
        torch = _torch()
        out = torch.empty((max(self.nsph, 1), 6), dtype=torch.float64, device="cuda")
        _check(lib().fsl_particle_forces(self.h, ctypes.cast(out.data_ptr(), ctypes.POINTER(ctypes.c_double)), 1))
        return out[:self.nsph]

    def set_estimator(self, weights):
        w = _f32(weights)
        assert w.size == MLP_NPARAM
        _check(lib().fsl_set_estimator(self.h, _fp(w)))

    def watchdog(self):
        """Last watchdog check: dict of mass, reference mass, lowest and
        highest fluid density, cells outside [0.5, 1.5]."""
        out = np.zeros(5)
        _check(lib().fsl_watchdog(self.h, _dp(out)))
        return dict(zip(("mass", "mass_ref", "rho_min", "rho_max", "cells_out"), out.tolist()))

    def estimator_stats(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fsl_estimator_stats(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def timing_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().fsl_timing_read(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def create_lattice(params, fill, rho, vel=None, device="cuda"):
    return Lattice(params, fill, rho, vel, device=device)


def lattice_from_workload(w, precision="fp64", check_every=0, **overrides):
    """Create a lattice from a seeded workload (``inputs.Workload``) and map
    its spheres."""
    kw = dict(shape=w.shape, precision=precision, omega=w.omega, accel=w.accel,
              sigma=w.sigma, rho_gas=w.rho_gas, conv_eps=w.conv_eps, check_every=check_every)
    kw.update(overrides)
    lat = Lattice(make_params(**kw), w.fill, w.rho, w.vel)
    if len(w.radius):
        lat.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    return lat


# ---------------------------------------------------------------- estimator
def estimator_train(x, y, weights, epochs=10, batch=1024, lr=1e-3, beta1=0.9, beta2=0.999,
                    eps=1e-8, seed=0):
    """Train the interface estimator on the GPU; returns (weights, epoch losses)."""
    x, y, w = _f32(x), _f32(y), _f32(weights).copy()
    n = x.size // 27
    assert x.size == 27 * n and y.size == 4 * n and w.size == MLP_NPARAM
    tp = FslTrainParams(int(epochs), int(batch), lr, beta1, beta2, eps, int(seed))
    losses = np.zeros(int(epochs), dtype=np.float32)
    _check(lib().fsl_estimator_train(_fp(x), _fp(y), n, ctypes.byref(tp), _fp(w), _fp(losses), _stream()))
    return w, losses


def estimator_grad_device(weights, x, y, grad, loss, n=None):
    """The loss gradient with every array a torch device tensor (float32:
    weights [6212], x [n, 27], y [n, 4], grad [6212] and loss [1] written);
    enqueued on the current stream, nothing allocated by the library."""
    n = x.shape[0] if n is None else int(n)
    _check(lib().fsl_estimator_grad_device(ctypes.c_void_p(weights.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), n, ctypes.c_void_p(grad.data_ptr()),
                                           ctypes.c_void_p(loss.data_ptr()), _stream()))


def estimator_grad(weights, x, y):
    x, y, w = _f32(x), _f32(y), _f32(weights)
    n = x.size // 27
    g = np.zeros(MLP_NPARAM, dtype=np.float32)
    loss = ctypes.c_double()
    _check(lib().fsl_estimator_grad(_fp(w), _fp(x), _fp(y), n, _fp(g), ctypes.byref(loss), _stream()))
    return g, loss.value


def estimator_infer(weights, x):
    x, w = _f32(x), _f32(weights)
    n = x.size // 27
    y = np.zeros(4 * n, dtype=np.float32)
    _check(lib().fsl_estimator_infer(_fp(w), _fp(x), n, _fp(y), _stream()))
    return y.reshape(n, 4)


def estimator_stencils(params, ss):
    """Fill levels (n, 27) of analytic shapes params (n, 16) supersampled
    on ss^3 points per cell (fsl_estimator_stencils)."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    n = params.shape[0]
    x = np.zeros(27 * n, dtype=np.float32)
    _check(lib().fsl_estimator_stencils(_dp(params), n, int(ss), _fp(x), _stream()))
    return x.reshape(n, 27)


def fd_geometry(x):
    """Finite-difference normal and curvature of stencils x (n, 27) -> (n, 4)."""
    x = _f32(x)
    n = x.size // 27
    y = np.zeros(4 * n, dtype=np.float32)
    _check(lib().fsl_fd_geometry(_fp(x), n, _fp(y), _stream()))
    return y.reshape(n, 4)


class Dem:
    """Rigid spheres on the GPU (fsl_dem_*): Newton-Euler motion under a
    hydrodynamic load, gravity, collisions and lubrication, sub-stepped per
    lattice step.  Defaults are the paper's collision parameters (e_dry 0.97,
    T_c = 4 d50 for d50 = 10 cells, nu_p 0.22, mu_p 0.5) and the density
    ratio of its gravel (2.55)."""

    def __init__(self, box, centre, radius, vel=None, angvel=None, fixed=None, density=2.55,
                 restitution=0.97, collision_time=40.0, poisson=0.22, friction=0.5, viscosity=0.0,
                 lub_cut=0.0, lub_min=1e-3, accel=(0.0, 0.0, 0.0), dt=1.0, substeps=10, skin=1.0,
                 stream=None):
        p = FslDemParams()
        p.nx, p.ny, p.nz = (int(v) for v in box)
        p.density, p.restitution, p.collision_time = density, restitution, collision_time
        p.poisson, p.friction, p.viscosity = poisson, friction, viscosity
        p.lub_cut, p.lub_min, p.dt, p.substeps, p.skin = lub_cut, lub_min, dt, int(substeps), skin
        for d in range(3):
            p.accel[d] = float(accel[d])
        c = _f64(centre)
        self.n = n = c.size // 3
        r, v, w = _f64(radius), _f64(vel), _f64(angvel)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8).reshape(-1)
        h = ctypes.c_void_p()
        _check(lib().fsl_dem_create(ctypes.byref(p), stream, n, _dp(c), _dp(r), _dp(v), _dp(w),
                                    None if fx is None else fx.ctypes.data, ctypes.byref(h)))
        self.h = h

    def step(self, hydro=None, n=1):
        """hydro: (n, 6) host array, a CUDA tensor of 6 n float64, or None"""
        if hydro is None:
            _check(lib().fsl_dem_step(self.h, None, 0, int(n)))
        elif hasattr(hydro, "data_ptr"):
            assert hydro.is_cuda and hydro.numel() == 6 * self.n and hydro.is_contiguous()
            _check(lib().fsl_dem_step(self.h, ctypes.c_void_p(hydro.data_ptr()), 1, int(n)))
        else:
            a = _f64(hydro)
            assert a.size == 6 * self.n
            _check(lib().fsl_dem_step(self.h, a.ctypes.data, 0, int(n)))

    def state(self):
        """(centre, vel, angvel), each (n, 3) host arrays"""
        out = [np.zeros(3 * self.n) for _ in range(3)]
        _check(lib().fsl_dem_read(self.h, *[_dp(o) for o in out], 0))
        return [o.reshape(self.n, 3) for o in out]

    def state_device(self):
        """(centre, vel, angvel) as (n, 3) CUDA float64 tensors"""
        torch = _torch()
        out = [torch.empty((self.n, 3), dtype=torch.float64, device="cuda") for _ in range(3)]
        _check(lib().fsl_dem_read(self.h, *[ctypes.cast(o.data_ptr(), ctypes.POINTER(ctypes.c_double)) for o in out], 1))
        return out

    def bedload(self):
        """bedload transport rate q_b of Eq. (1)"""
        q = np.zeros(1)
        _check(lib().fsl_dem_bedload(self.h, _dp(q)))
        return float(q[0])

    def destroy(self):
        if self.h:
            lib().fsl_dem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
