"""ctypes driver of ``libfsl_emu.so``: the library's kernels built as host
code (tests/hostemu/build.py), run on the CPU against the oracle.

Same C-ABI as libfsl.so; the "device" workspace is host memory from the
emulation's allocator, and the stream is NULL.
"""
from __future__ import annotations

import ctypes
import glob
import os

import numpy as np

from paper_2301_10674_amd import fsl as F

HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _stale(p):
    """The library is missing or older than a source it is built from."""
    if not os.path.exists(p):
        return True
    root = os.path.dirname(os.path.dirname(HERE))
    srcs = glob.glob(os.path.join(root, "paper_2301_10674_amd", "csrc", "*"))
    srcs += glob.glob(os.path.join(HERE, "hip", "*")) + [os.path.join(HERE, f) for f in ("hostemu.cpp", "build.py")]
    srcs.append(os.path.join(root, "include", "fsl.h"))
    t = os.path.getmtime(p)
    return any(os.path.getmtime(f) > t for f in srcs if os.path.isfile(f))


def lib(path=None):
    global _lib
    if _lib is None:
        p = path or os.path.join(HERE, "_build", "libfsl_emu.so")
        if path is None and _stale(p):
            import importlib.util
            spec = importlib.util.spec_from_file_location("hostemu_build", os.path.join(HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            p = mod.build()
        L = ctypes.CDLL(p)
        vp, dp, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32
        L.hipemu_alloc.restype = vp
        L.hipemu_alloc.argtypes = [ctypes.c_size_t]
        L.hipemu_free.argtypes = [vp]
        L.fsl_workspace_bytes.restype = ctypes.c_size_t
        L.fsl_workspace_bytes.argtypes = [ctypes.POINTER(F.FslParams)]
        L.fsl_create_lattice.argtypes = [ctypes.POINTER(F.FslParams), vp, ctypes.c_size_t, vp,
                                         dp, dp, dp, ctypes.POINTER(vp)]
        L.fsl_set_particles.argtypes = [vp, i32, dp, dp, dp, dp]
        L.fsl_step.argtypes = [vp, i32]
        L.fsl_read_fields.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(vp), i32]
        L.fsl_total_mass.argtypes = [vp, dp]
        L.fsl_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.fsl_move_particles.argtypes = [vp, dp, dp, dp]
        L.fsl_particle_forces.argtypes = [vp, dp, i32]
        L.fsl_last_error.restype = ctypes.c_char_p
        L.fsl_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(s):
    if s != 0:
        raise F.FslError(s, lib().fsl_last_error().decode())


class EmuLattice:
    def __init__(self, w, precision="fp64", **overrides):
        kw = dict(shape=w.shape, precision=precision, omega=w.omega, accel=w.accel, sigma=w.sigma,
                  rho_gas=w.rho_gas, conv_eps=w.conv_eps)
        kw.update(overrides)
        self.params = F.make_params(**kw)
        self.shape = w.shape
        self.N = int(np.prod(w.shape))
        nbytes = int(lib().fsl_workspace_bytes(ctypes.byref(self.params)))
        if nbytes == 0:
            raise F.FslError(1, lib().fsl_last_error().decode())
        self.ws = lib().hipemu_alloc(nbytes)
        fill = np.ascontiguousarray(w.fill, dtype=np.float64)
        rho = np.ascontiguousarray(w.rho, dtype=np.float64)
        vel = np.ascontiguousarray(w.vel, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().fsl_create_lattice(ctypes.byref(self.params), ctypes.c_void_p(self.ws), nbytes, None,
                                        _dp(fill), _dp(rho), _dp(vel), ctypes.byref(h)))
        self.h = h
        if len(w.radius):
            c = np.ascontiguousarray(w.centre, dtype=np.float64)
            r = np.ascontiguousarray(w.radius, dtype=np.float64)
            v = np.ascontiguousarray(w.sphere_vel, dtype=np.float64)
            a = np.ascontiguousarray(w.sphere_angvel, dtype=np.float64)
            _check(lib().fsl_set_particles(self.h, len(r), _dp(c), _dp(r), _dp(v), _dp(a)))

    def step(self, n=1):
        _check(lib().fsl_step(self.h, int(n)))

    def read(self, f):
        nx, ny, nz = self.shape
        N = self.N
        if f in (F.FIELD_TYPE, F.FIELD_ESTIMATOR):
            a = np.zeros(N, dtype=np.uint8)
        elif f == F.FIELD_OWNER:
            a = np.zeros(N, dtype=np.int32)
        elif f in (F.FIELD_VEL, F.FIELD_NORMAL):
            a = np.zeros(3 * N)
        elif f == F.FIELD_PDF:
            a = np.zeros(27 * N)
        else:
            a = np.zeros(N)
        ptrs = (ctypes.c_void_p * F.NFIELDS)()
        ptrs[f] = a.ctypes.data
        _check(lib().fsl_read_fields(self.h, 1 << f, ptrs, 0))
        if f in (F.FIELD_VEL, F.FIELD_NORMAL):
            return a.reshape(3, nz, ny, nx)
        if f == F.FIELD_PDF:
            return a.reshape(27, nz, ny, nx)
        return a.reshape(nz, ny, nx)

    def move_particles(self, centre, vel=None, angvel=None):
        c = np.ascontiguousarray(centre, dtype=np.float64)
        v = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64)
        a = None if angvel is None else np.ascontiguousarray(angvel, dtype=np.float64)
        _check(lib().fsl_move_particles(self.h, _dp(c), _dp(v), _dp(a)))

    def particle_forces(self, nsph):
        out = np.zeros((nsph, 6))
        _check(lib().fsl_particle_forces(self.h, _dp(out), 0))
        return out

    def total_mass(self):
        m = ctypes.c_double()
        _check(lib().fsl_total_mass(self.h, ctypes.byref(m)))
        return m.value

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        _check(lib().fsl_counters(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return out

    def destroy(self):
        if getattr(self, "h", None):
            lib().fsl_destroy(self.h)
            self.h = None
        if getattr(self, "ws", None):
            lib().hipemu_free(self.ws)
            self.ws = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
