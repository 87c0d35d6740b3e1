"""Thin ctypes binding of libibmlbm.so (declared in include/ibm_lbm.h).

Argument marshalling only: every step of the timestep runs in the library's
HIP kernels.  PyTorch provides the device buffers the library works in and
the stream it enqueues on.  Importing this module fails if the library has
not been built (paper_1004_2416_amd/build.py); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libibmlbm.so")

IBM_OK = 0
ERRORS = {
    -1: "IBM_ERR_INVALID_ARG",
    -2: "IBM_ERR_BAD_STATE",
    -3: "IBM_ERR_HIP",
    -4: "IBM_ERR_STENCIL_HITS_WALL",
    -5: "IBM_ERR_NONFINITE",
    -6: "IBM_ERR_INVERTED_FACE",
    -7: "IBM_ERR_OUTSIDE_SLAB",
}
STORAGE = {"fp32": 0, "fp16": 1}
STORAGE_ONE_BUFFER = 4
FIELD_POPS, FIELD_RHO, FIELD_U, FIELD_FORCE = 0, 1, 2, 3
OPT_GRAPH, OPT_EQUILIBRIUM, OPT_ADVECTION, OPT_RECENTER, OPT_LBM_VARIANT = 0, 1, 2, 3, 4
OPT_STENCIL_BOX, OPT_OVERLAP, OPT_STREAMING, OPT_FP16_MASS = 6, 7, 8, 9
STREAM_TWO_BUFFERS, STREAM_AA = 0, 1
PHASES = ("forces", "spread", "lbm", "interp")
OBS_FIELDS = ("V", "cx", "cy", "cz", "D", "theta", "ra", "rb", "rc", "area",
              "Ixx", "Iyy", "Izz", "Ixy", "Ixz", "Iyz")
OBS_N = 16


class IBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _load():
    # PyTorch ships its own HIP runtime; the library must bind to that same
    # runtime (one per process), so torch is imported before the library is
    # loaded.  Loaded the other way round (the system runtime first), the
    # library's first call on the device failed with "no ROCm-capable device".
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_1004_2416_amd/build.py` "
            "(hipcc, gfx950); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    i, d, v, sz = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    i64 = ctypes.c_int64
    sig = {
        "ibm_lattice_bytes": ([i, i, i, i, ctypes.POINTER(sz)], i),
        "ibm_lattice_create": ([i, i, i, d, i, v, sz, v, ctypes.POINTER(v)], i),
        "ibm_set_shear": ([v, d, i], i),
        "ibm_membrane_bytes": ([i, v, v, ctypes.POINTER(sz)], i),
        "ibm_membrane_create": ([v, i, v, v, v, v, v, v, i, v, sz], i),
        "ibm_step": ([v, i64], i),
        "ibm_step_count": ([v], i64),
        "ibm_get_fields": ([v, i, v], i),
        "ibm_set_fields": ([v, i, v], i),
        "ibm_get_mesh": ([v, v, v, v], i),
        "ibm_set_mesh": ([v, v], i),
        "ibm_observables": ([v, v], i),
        "ibm_synchronize": ([v], i),
        "ibm_totals_bytes": ([v, ctypes.POINTER(sz)], i),
        "ibm_deformation_gradient": ([v, i, v], i),
        "ibm_lattice_totals": ([v, v, sz, v], i),
        "ibm_lattice_totals_noalloc": ([v, v], i),
        "ibm_set_option": ([v, i, i], i),
        "ibm_split_box": ([v, ctypes.POINTER(i)], i),
        "ibm_profile_step": ([v, i64, v], i),
        "ibm_profile_lattice_kernel": ([v, i64, v], i),
        "ibm_autotune": ([v, i, v], i),
        "ibm_batch_autotune": ([v, i, v], i),
        "ibm_batch_set_persistent": ([v, i], i),
        "ibm_destroy": ([v], i),
        "ibm_last_error": ([], ctypes.c_char_p),
        "ibm_icosphere_size": ([i, ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "ibm_icosphere": ([i, d, d, d, d, v, v], i),
        "ibm_tangent_bytes": ([v, ctypes.POINTER(sz)], i),
        "ibm_tangent_attach": ([v, v, v, d, i, v, sz], i),
        "ibm_tangent_detach": ([v], i),
        "ibm_tangent_get_pops": ([v, v], i),
        "ibm_tangent_get_mesh": ([v, v, v], i),
        "ibm_tangent_observables": ([v, d, v], i),
        "ibm_adjoint_bytes": ([v, i64, i, ctypes.POINTER(sz)], i),
        "ibm_adjoint_gradient": ([v, i64, i, i, i, v, sz, v, v, v, v], i),
        "ibm_batch_bytes": ([i, v, ctypes.POINTER(sz)], i),
        "ibm_batch_create": ([i, v, v, sz, ctypes.POINTER(v)], i),
        "ibm_batch_step": ([v, i64], i),
        "ibm_batch_profile_step": ([v, i64, v], i),
        "ibm_batch_profile_lattice_kernel": ([v, i64, v], i),
        "ibm_batch_destroy": ([v], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def _check(rc: int):
    if rc != IBM_OK:
        raise IBMError(rc, lib.ibm_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def icosphere(level: int, r: float = 1.0, center=(0.0, 0.0, 0.0)):
    """The library's icosahedron subdivision mesh (Sec. II.D)."""
    nn, nf = ctypes.c_int(), ctypes.c_int()
    _check(lib.ibm_icosphere_size(int(level), ctypes.byref(nn), ctypes.byref(nf)))
    xyz = np.zeros((nn.value, 3))
    tri = np.zeros((nf.value, 3), dtype=np.int32)
    _check(lib.ibm_icosphere(int(level), float(r), float(center[0]), float(center[1]),
                             float(center[2]), _ptr(xyz), _ptr(tri)))
    return xyz, tri


def _torch():
    import torch
    return torch


def _aligned_buffer(nbytes: int, device):
    """A caller-owned device buffer (torch uint8), 256-byte aligned view."""
    torch = _torch()
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw[off:off + nbytes]


class Lattice:
    """A lattice (and optionally its capsules) living in torch device memory.

    nx, ny, nz   fluid nodes; walls at z = -1/2 and nz - 1/2 (Sec. II.A)
    tau          BGK relaxation time (> 1/2)
    storage      "fp32" or "fp16" (scaled deviations f_i - w_i)
    one_buffer   one population buffer, streamed with the AA pattern
    stream       torch.cuda.Stream to enqueue on (default: the current one)
    """

    def __init__(self, nx: int, ny: int, nz: int, tau: float = 1.0, storage: str = "fp32",
                 device="cuda", stream=None, one_buffer: bool = False):
        torch = _torch()
        self.shape = (int(nz), int(ny), int(nx))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = ctypes.c_size_t()
        code = STORAGE[storage] | (STORAGE_ONE_BUFFER if one_buffer else 0)
        _check(lib.ibm_lattice_bytes(nx, ny, nz, code, ctypes.byref(nbytes)))
        self._raw, self._state = _aligned_buffer(nbytes.value, self.device)
        h = ctypes.c_void_p()
        _check(lib.ibm_lattice_create(nx, ny, nz, float(tau), code,
                                      ctypes.c_void_p(self._state.data_ptr()), nbytes.value,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n_caps = 0
        self.nn = 0
        self.nf = 0
        self._mem = None

    # -- setup ---------------------------------------------------------------
    def set_shear(self, u_w: float, init_profile: bool = True):
        _check(lib.ibm_set_shear(self._h, float(u_w), int(bool(init_profile))))

    def add_capsules(self, meshes: Sequence, ks: Sequence[float], ka: Sequence[float], m: int):
        """meshes: list of (xyz [n, 3] float64, tri [f, 3] int) in lattice
        coordinates, each the stress-free reference and initial shape."""
        xyz = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64) for x, _ in meshes]))
        tri = np.ascontiguousarray(np.concatenate([np.asarray(t, np.int32) for _, t in meshes]))
        nodes = np.array([len(x) for x, _ in meshes], dtype=np.int32)
        faces = np.array([len(t) for _, t in meshes], dtype=np.int32)
        ks = np.ascontiguousarray(ks, dtype=np.float64)
        ka = np.ascontiguousarray(ka, dtype=np.float64)
        nbytes = ctypes.c_size_t()
        _check(lib.ibm_membrane_bytes(len(meshes), _ptr(nodes), _ptr(faces), ctypes.byref(nbytes)))
        raw, buf = _aligned_buffer(nbytes.value, self.device)
        _check(lib.ibm_membrane_create(self._h, len(meshes), _ptr(nodes), _ptr(faces), _ptr(xyz),
                                       _ptr(tri), _ptr(ks), _ptr(ka), int(m),
                                       ctypes.c_void_p(buf.data_ptr()), nbytes.value))
        self._mem = (raw, buf)
        self.n_caps = len(meshes)
        self.nn = int(nodes.sum())
        self.nf = int(faces.sum())

    def set_option(self, option: int, value: int):
        _check(lib.ibm_set_option(self._h, int(option), int(value)))

    def split_box(self):
        """(zlo, zhi, ylo, yhi): the force box of the split lattice update
        (IBM_OPT_OVERLAP) the next graph steps use; the whole lattice when
        the update is not split."""
        box = (ctypes.c_int * 4)()
        _check(lib.ibm_split_box(self._h, box))
        return tuple(box)

    # -- stepping ------------------------------------------------------------
    def step(self, n: int = 1):
        _check(lib.ibm_step(self._h, int(n)))

    @property
    def steps(self) -> int:
        return int(lib.ibm_step_count(self._h))

    def synchronize(self):
        _check(lib.ibm_synchronize(self._h))

    def profile(self, n: int) -> dict:
        out = np.zeros(4)
        _check(lib.ibm_profile_step(self._h, int(n), _ptr(out)))
        return dict(zip(PHASES, out.tolist()))

    def lattice_kernel_ms(self, n: int) -> float:
        """Mean execution time (ms) of the collide-stream kernel over n plain
        steps, from its own dispatch timestamps (the run advances by n)."""
        out = np.zeros(1)
        _check(lib.ibm_profile_lattice_kernel(self._h, int(n), _ptr(out)))
        return float(out[0])

    def autotune(self, steps_per_trial: int = 64) -> dict:
        """Pick the fastest kernel forms by timing real steps (the run
        advances by them)."""
        out = np.zeros(2, dtype=np.int32)
        _check(lib.ibm_autotune(self._h, int(steps_per_trial), _ptr(out)))
        return {"lbm_variant": int(out[0]), "stencil_box": int(out[1])}

    # -- I/O -----------------------------------------------------------------
    def _field(self, what: int, comps: int):
        torch = _torch()
        nz, ny, nx = self.shape
        out = torch.empty((comps, nz, ny, nx), dtype=torch.float64, device=self.device)
        _check(lib.ibm_get_fields(self._h, what, ctypes.c_void_p(out.data_ptr())))
        return out

    def populations(self):
        return self._field(FIELD_POPS, 19)

    def density(self):
        return self._field(FIELD_RHO, 1)[0]

    def velocity(self):
        return self._field(FIELD_U, 3)

    def force_density(self):
        return self._field(FIELD_FORCE, 3)

    def set_populations(self, f):
        torch = _torch()
        t = torch.as_tensor(np.asarray(f, dtype=np.float64) if not torch.is_tensor(f) else f)
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(t.shape) == (19,) + self.shape
        _check(lib.ibm_set_fields(self._h, FIELD_POPS, ctypes.c_void_p(t.data_ptr())))
        self.synchronize()

    def mesh(self):
        """(positions, forces F(t), velocities u(t+1)) of the last step,
        float64 [nn, 3] device tensors."""
        torch = _torch()
        out = [torch.empty((self.nn, 3), dtype=torch.float64, device=self.device) for _ in range(3)]
        _check(lib.ibm_get_mesh(self._h, *[ctypes.c_void_p(o.data_ptr()) for o in out]))
        return tuple(out)

    def set_mesh(self, xyz):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        assert xyz.shape == (self.nn, 3)
        _check(lib.ibm_set_mesh(self._h, _ptr(xyz)))

    def deformation_gradient(self, capsule: int = 0) -> np.ndarray:
        """dD/dx [nn][3] of one capsule's Taylor deformation at the current
        node positions (zero rows for the other capsules)."""
        torch = _torch()
        out = torch.zeros((self.nn, 3), dtype=torch.float64, device=self.device)
        _check(lib.ibm_deformation_gradient(self._h, int(capsule), ctypes.c_void_p(out.data_ptr())))
        return out.cpu().numpy()

    def totals(self) -> np.ndarray:
        """FP64 (mass, momentum x, y, z) of the current populations, summed on
        the device (ibm_lattice_totals)."""
        torch = _torch()
        nb = ctypes.c_size_t()
        _check(lib.ibm_totals_bytes(self._h, ctypes.byref(nb)))
        work = torch.empty(max(nb.value // 8, 1), dtype=torch.float64, device=self.device)
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        _check(lib.ibm_lattice_totals(self._h, ctypes.c_void_p(work.data_ptr()), nb.value,
                                      ctypes.c_void_p(out.data_ptr())))
        self.synchronize()
        return out.cpu().numpy()

    def totals_noalloc(self, out):
        """ibm_lattice_totals_noalloc into the caller's float64 device tensor
        `out` (4 values); enqueued on the lattice's stream, no allocation."""
        _check(lib.ibm_lattice_totals_noalloc(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def observables(self) -> np.ndarray:
        out = np.zeros((self.n_caps, OBS_N))
        _check(lib.ibm_observables(self._h, _ptr(out)))
        return out

    # -- forward sensitivities ---------------------------------------------
    def attach_tangent(self, dks=None, dka=None, duw: float = 0.0, init_profile: bool = False):
        """Start a tangent along the parameter rates dks, dka (per capsule) and
        duw; every later step advances it."""
        nbytes = ctypes.c_size_t()
        _check(lib.ibm_tangent_bytes(self._h, ctypes.byref(nbytes)))
        self._tan = _aligned_buffer(nbytes.value, self.device)
        if self.n_caps:
            a = np.ascontiguousarray(np.broadcast_to(np.asarray(dks, np.float64), (self.n_caps,)))
            b = np.ascontiguousarray(np.broadcast_to(np.asarray(dka, np.float64), (self.n_caps,)))
            pa, pb = _ptr(a), _ptr(b)
        else:
            pa = pb = None
        _check(lib.ibm_tangent_attach(self._h, pa, pb, float(duw), int(bool(init_profile)),
                                      ctypes.c_void_p(self._tan[1].data_ptr()), nbytes.value))

    def detach_tangent(self):
        _check(lib.ibm_tangent_detach(self._h))
        self._tan = None

    def tangent_populations(self):
        torch = _torch()
        nz, ny, nx = self.shape
        out = torch.empty((19, nz, ny, nx), dtype=torch.float64, device=self.device)
        _check(lib.ibm_tangent_get_pops(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def tangent_mesh(self):
        """(d positions, d velocities), float64 [nn, 3] device tensors."""
        torch = _torch()
        out = [torch.empty((self.nn, 3), dtype=torch.float64, device=self.device) for _ in range(2)]
        _check(lib.ibm_tangent_get_mesh(self._h, *[ctypes.c_void_p(o.data_ptr()) for o in out]))
        return tuple(out)

    def tangent_observables(self, h: float) -> np.ndarray:
        out = np.zeros((self.n_caps, OBS_N))
        _check(lib.ibm_tangent_observables(self._h, float(h), _ptr(out)))
        return out

    # -- reverse-mode gradient ---------------------------------------------
    def adjoint_gradient(self, steps: int, checkpoint_every: int = 100, capsule: int = 0,
                         couette_start: bool = False) -> dict:
        """Run `steps` steps and return D(T) of `capsule` with its gradient
        with respect to k_s, k_alpha (per capsule) and u_w, by the adjoint."""
        nbytes = ctypes.c_size_t()
        _check(lib.ibm_adjoint_bytes(self._h, int(steps), int(checkpoint_every), ctypes.byref(nbytes)))
        raw, buf = _aligned_buffer(nbytes.value, self.device)
        D = np.zeros(1)
        dks, dka, duw = np.zeros(self.n_caps), np.zeros(self.n_caps), np.zeros(1)
        _check(lib.ibm_adjoint_gradient(self._h, int(steps), int(checkpoint_every), int(capsule),
                                        int(bool(couette_start)), ctypes.c_void_p(buf.data_ptr()),
                                        nbytes.value, _ptr(D), _ptr(dks), _ptr(dka), _ptr(duw)))
        del raw, buf
        return {"D": float(D[0]), "dks": dks, "dka": dka, "duw": float(duw[0])}

    def close(self):
        if getattr(self, "_h", None):
            lib.ibm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent runs (Lattice objects on one stream) advanced together:
    one launch per kernel of the step for all of them."""

    def __init__(self, lattices: Sequence[Lattice]):
        self.runs = list(lattices)
        n = len(self.runs)
        handles = (ctypes.c_void_p * n)(*[r._h.value for r in self.runs])
        nbytes = ctypes.c_size_t()
        _check(lib.ibm_batch_bytes(n, handles, ctypes.byref(nbytes)))
        self._raw, self._buf = _aligned_buffer(nbytes.value, self.runs[0].device)
        h = ctypes.c_void_p()
        _check(lib.ibm_batch_create(n, handles, ctypes.c_void_p(self._buf.data_ptr()), nbytes.value,
                                    ctypes.byref(h)))
        self._h = h

    def step(self, n: int = 1):
        _check(lib.ibm_batch_step(self._h, int(n)))

    def autotune(self, steps_per_trial: int = 64) -> dict:
        """ibm_batch_autotune: block shape, cached rows and the stencil-box
        mode per delta width, timed on the live batch."""
        out = (ctypes.c_int * 6)()
        _check(lib.ibm_batch_autotune(self._h, int(steps_per_trial), out))
        return {"waves_per_block": out[0], "cached_rows_div": out[1],
                "stencil_box": {m: out[m] for m in (2, 3, 4)}, "persistent": out[5]}

    def set_persistent(self, on: bool = True):
        _check(lib.ibm_batch_set_persistent(self._h, int(on)))

    def profile(self, n: int) -> dict:
        out = np.zeros(4)
        _check(lib.ibm_batch_profile_step(self._h, int(n), _ptr(out)))
        return dict(zip(PHASES, out.tolist()))

    def lattice_kernel_ms(self, n: int) -> float:
        """Mean execution time (ms) of the batched collide-stream kernel over
        n plain steps of every run, from its own dispatch timestamps."""
        out = np.zeros(1)
        _check(lib.ibm_batch_profile_lattice_kernel(self._h, int(n), _ptr(out)))
        return float(out[0])

    def close(self):
        if getattr(self, "_h", None):
            lib.ibm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- D(T) as a differentiable torch function --------------------------------
_DEFORMATION_FN = None


def _deformation_fn():
    global _DEFORMATION_FN
    if _DEFORMATION_FN is None:
        torch = _torch()

        class _Deformation(torch.autograd.Function):
            @staticmethod
            def forward(ctx, ks, ka, uw, make_lattice, steps, checkpoint_every, capsule):
                lat = make_lattice(ks.detach().cpu().tolist(), ka.detach().cpu().tolist(),
                                   float(uw))
                f64 = dict(dtype=torch.float64)
                try:
                    if not any(ctx.needs_input_grad[:3]):
                        # no gradient wanted: the forward run alone
                        lat.step(steps)
                        return torch.tensor(float(lat.observables()[capsule, 4]), **f64)
                    g = lat.adjoint_gradient(steps, checkpoint_every, capsule, couette_start=True)
                finally:
                    lat.close()
                ctx.save_for_backward(torch.as_tensor(g["dks"], **f64),
                                      torch.as_tensor(g["dka"], **f64),
                                      torch.tensor(g["duw"], **f64))
                return torch.tensor(g["D"], **f64)

            @staticmethod
            def backward(ctx, gD):
                dks, dka, duw = ctx.saved_tensors
                gD = gD.detach().to(torch.float64).cpu()
                return gD * dks, gD * dka, gD * duw, None, None, None, None

        _DEFORMATION_FN = _Deformation
    return _DEFORMATION_FN


def deformation(make_lattice, ks, ka, uw, steps: int, checkpoint_every: int = 100,
                capsule: int = 0):
    """D(T) of `capsule` after `steps` steps (Sec. III) as a torch function of
    the per-capsule moduli ks, ka (1-D float64 CPU tensors) and the wall
    speed uw (0-D tensor), differentiable by the discrete adjoint.

    make_lattice(ks, ka, uw) must return a new Lattice at t = 0 with its
    capsules added with these moduli and ibm_set_shear(uw, init_profile=1)
    applied, so that the start also depends on uw.  When a gradient is
    needed (an input requires grad and grad mode is on), the forward call
    runs ibm_adjoint_gradient once (forward sweep and reverse sweep) and
    keeps the gradient, and backward only scales it; otherwise it runs the
    steps alone."""
    return _deformation_fn().apply(ks, ka, uw, make_lattice, int(steps), int(checkpoint_every),
                                   int(capsule))
