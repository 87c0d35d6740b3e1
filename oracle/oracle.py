"""ctypes wrapper around the FP64 CPU oracle (oracle/ibm_oracle.c).

TEST INFRASTRUCTURE ONLY: the plain reference implementation that the HIP
library is checked against.  Only tests/, the smoke check and the CPU-baseline
leg of bench.py may import this module; the library never does.

Every array is float64 (int32 for triangles), C-contiguous.  Populations are
[19, nz, ny, nx] unshifted post-streaming values; positions are unwrapped
lattice coordinates [n, 3].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_ERR_WALL = -4


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no target-specific
    flags so that no fused multiply-add changes its rounding)."""
    cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        d, i, v = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.orc_lattice_constants.argtypes = [v, v, v]
        L.orc_equilibrium.argtypes = [d, v, v]
        L.orc_equilibrium_linear.argtypes = [d, v, v]
        L.orc_guo_source.argtypes = [d, v, v, v]
        L.orc_lbm_step.argtypes = [i, i, i, d, d, i, v, v, v, i]
        L.orc_lbm_step.restype = i
        L.orc_velocity_field.argtypes = [i, i, i, v, v, v, v, i]
        L.orc_phi.argtypes = [i, d]
        L.orc_phi.restype = d
        L.orc_spread.argtypes = [i, i, i, i, i, v, v, v]
        L.orc_spread.restype = i
        L.orc_interpolate.argtypes = [i, i, i, i, i, v, v, v]
        L.orc_interpolate.restype = i
        L.orc_membrane_energy.argtypes = [i, i, v, v, v, v, v]
        L.orc_membrane_energy.restype = d
        L.orc_membrane_forces.argtypes = [i, i, v, v, v, v, v, v]
        L.orc_icosphere_size.argtypes = [i, v, v]
        L.orc_icosphere.argtypes = [i, d, d, d, d, v, v]
        L.orc_icosphere.restype = i
        L.orc_capsule_observables.argtypes = [i, i, v, v, v]
        L.orc_run.argtypes = [i, i, i, d, d, i, i, i, i, i, v, v, v, v, v, v,
                              v, v, v, v, i, i]
        L.orc_run.restype = i
        L.orc_max_threads.restype = i
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice_constants():
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().orc_lattice_constants(_p(c), _p(w), _p(opp))
    return c, w, opp


def equilibrium(rho, u, linear=False):
    u = _f64(u)
    out = np.zeros(19)
    fn = lib().orc_equilibrium_linear if linear else lib().orc_equilibrium
    fn(float(rho), _p(u), _p(out))
    return out


def guo_source(tau, u, g):
    u, g = _f64(u), _f64(g)
    out = np.zeros(19)
    lib().orc_guo_source(float(tau), _p(u), _p(g), _p(out))
    return out


def phi(m, r):
    return lib().orc_phi(int(m), float(r))


def lbm_step(f, g, tau, uw, linear=False, nthreads=0):
    f = _f64(f)
    _, nz, ny, nx = f.shape
    out = np.empty_like(f)
    gg = None if g is None else _f64(g)
    rc = lib().orc_lbm_step(nx, ny, nz, float(tau), float(uw), int(linear),
                            _p(f), _p(gg), _p(out), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_lbm_step failed: {rc}")
    return out


def velocity_field(f, g=None, nthreads=0):
    f = _f64(f)
    _, nz, ny, nx = f.shape
    rho = np.empty((nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    gg = None if g is None else _f64(g)
    lib().orc_velocity_field(nx, ny, nz, _p(f), _p(gg), _p(rho), _p(u), int(nthreads))
    return rho, u


def spread(shape, m, x, F, g=None):
    """Adds the spread force density of nodes x with forces F to g (new zero
    field if None).  shape = (nz, ny, nx).  Returns (g, rc)."""
    nz, ny, nx = shape
    x, F = _f64(x), _f64(F)
    if g is None:
        g = np.zeros((3, nz, ny, nx))
    rc = lib().orc_spread(nx, ny, nz, int(m), x.shape[0], _p(x), _p(F), _p(g))
    return g, rc


def interpolate(m, x, u):
    x, u = _f64(x), _f64(u)
    _, nz, ny, nx = u.shape
    un = np.zeros((x.shape[0], 3))
    rc = lib().orc_interpolate(nx, ny, nz, int(m), x.shape[0], _p(x), _p(u), _p(un))
    return un, rc


def _per_face(v, nf):
    a = np.asarray(v, dtype=np.float64)
    if a.ndim == 0:
        a = np.full(nf, float(a))
    return _f64(a)


def membrane_energy(x, xref, tri, ks, ka):
    x, xref = _f64(x), _f64(xref)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    nf = tri.shape[0]
    return lib().orc_membrane_energy(x.shape[0], nf, _p(x), _p(xref), _p(tri),
                                     _p(_per_face(ks, nf)), _p(_per_face(ka, nf)))


def membrane_forces(x, xref, tri, ks, ka):
    x, xref = _f64(x), _f64(xref)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    nf = tri.shape[0]
    F = np.zeros_like(x)
    lib().orc_membrane_forces(x.shape[0], nf, _p(x), _p(xref), _p(tri),
                              _p(_per_face(ks, nf)), _p(_per_face(ka, nf)), _p(F))
    return F


def icosphere(level, r=1.0, center=(0.0, 0.0, 0.0)):
    nn, nf = ctypes.c_int(), ctypes.c_int()
    lib().orc_icosphere_size(int(level), ctypes.byref(nn), ctypes.byref(nf))
    xyz = np.zeros((nn.value, 3))
    tri = np.zeros((nf.value, 3), dtype=np.int32)
    rc = lib().orc_icosphere(int(level), float(r), float(center[0]), float(center[1]),
                             float(center[2]), _p(xyz), _p(tri))
    if rc != 0:
        raise ValueError("icosphere failed")
    return xyz, tri


OBS_FIELDS = ("V", "cx", "cy", "cz", "Ixx", "Iyy", "Izz", "Ixy", "Ixz", "Iyz",
              "E1", "E2", "E3", "ra", "rb", "rc", "D", "theta", "area")


def capsule_observables(x, tri):
    x = _f64(x)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    out = np.zeros(len(OBS_FIELDS))
    lib().orc_capsule_observables(x.shape[0], tri.shape[0], _p(x), _p(tri), _p(out))
    return dict(zip(OBS_FIELDS, out.tolist()))


def max_threads():
    return lib().orc_max_threads()


class Simulation:
    """Whole coupled state advanced by orc_run (Sec. II.C, sub-steps 1-5).

    tri holds global node indices over all capsules; ks, ka are per face."""

    def __init__(self, f, x, xref, tri, ks, ka, tau, uw, m, linear_eq=False,
                 ab2=False, nthreads=0):
        self.f = _f64(f).copy()
        self.x = _f64(x).copy()
        self.xref = _f64(xref).copy()
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        nf = self.tri.shape[0]
        self.ks = _per_face(ks, nf)
        self.ka = _per_face(ka, nf)
        self.tau, self.uw, self.m = float(tau), float(uw), int(m)
        self.linear_eq, self.ab2 = int(linear_eq), int(ab2)
        self.nthreads = int(nthreads)
        nn = self.x.shape[0]
        self.un_prev = np.zeros((max(nn, 1), 3))
        self.F = np.zeros((max(nn, 1), 3))
        self.un = np.zeros((max(nn, 1), 3))
        _, nz, ny, nx = self.f.shape
        self.g = np.zeros((3, nz, ny, nx))
        self.t = 0
        self.have_prev = False

    def run(self, nsteps):
        _, nz, ny, nx = self.f.shape
        nn, nf = self.x.shape[0], self.tri.shape[0]
        mode = 0
        if self.ab2:
            mode = 1 if self.have_prev else 2
            self.have_prev = self.have_prev or nsteps > 0
        rc = lib().orc_run(nx, ny, nz, self.tau, self.uw, self.m, self.linear_eq,
                           mode, nn, nf, _p(self.tri), _p(self.xref), _p(self.ks),
                           _p(self.ka), _p(self.f), _p(self.x), _p(self.un_prev),
                           _p(self.F), _p(self.un), _p(self.g), int(nsteps),
                           self.nthreads)
        self.t += nsteps
        return rc
