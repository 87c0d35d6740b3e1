"""CPU checks of the C ABI: the shared library loads and exports every symbol
that include/ibm_lbm.h declares, and the host-side validation returns error
codes (no GPU call is made by any of these)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibm_lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ibm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def B():
    from paper_1004_2416_amd import binding
    return binding


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("ibm_lattice_create", "ibm_set_shear", "ibm_membrane_create", "ibm_step",
                 "ibm_get_fields", "ibm_get_mesh", "ibm_observables", "ibm_destroy"):
        assert want in names


def test_library_exports_every_declared_symbol(B):
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_size_queries_and_validation(B):
    n = ctypes.c_size_t()
    assert B.lib.ibm_lattice_bytes(128, 128, 128, 0, ctypes.byref(n)) == 0
    # per node: two population copies (2 x 19 x 4 B in FP32, 2 x 19 x 2 B in
    # FP16), two force-density fields (2 x 3 x 4 B), the velocity field
    # interpolation reads (16 B) and the node stamps (4 B); tile stamps and
    # the control block add little
    N = 128 ** 3
    per32, per16 = 2 * 19 * 4 + 24 + 16 + 4, 2 * 19 * 2 + 24 + 16 + 4
    assert per32 * N <= n.value < 1.02 * per32 * N
    m = ctypes.c_size_t()
    assert B.lib.ibm_lattice_bytes(128, 128, 128, 1, ctypes.byref(m)) == 0
    assert per16 * N <= m.value < 1.02 * per16 * N
    # one population buffer (the AA pattern): 19 x 4 B less per node in FP32,
    # 19 x 2 B in FP16; only for rows a multiple of 4 and at most 256 long
    for storage, pop in ((0, 76), (1, 38)):
        one, two = ctypes.c_size_t(), ctypes.c_size_t()
        assert B.lib.ibm_lattice_bytes(128, 128, 128, storage | 4, ctypes.byref(one)) == 0
        assert B.lib.ibm_lattice_bytes(128, 128, 128, storage, ctypes.byref(two)) == 0
        assert two.value - one.value == pop * N
    assert B.lib.ibm_lattice_bytes(30, 8, 8, 4, ctypes.byref(m)) == -1
    assert "multiple of 4" in B.lib.ibm_last_error().decode()
    assert B.lib.ibm_lattice_bytes(260, 8, 8, 4, ctypes.byref(m)) == -1
    assert B.lib.ibm_lattice_bytes(8, 8, 8, 2, ctypes.byref(m)) == -1
    assert B.lib.ibm_lattice_bytes(0, 4, 4, 0, ctypes.byref(n)) == -1
    assert "lattice size" in B.lib.ibm_last_error().decode()
    assert B.lib.ibm_lattice_bytes(4, 4, 4, 7, ctypes.byref(n)) == -1
    h = ctypes.c_void_p()
    # tau <= 1/2 and a NULL buffer are rejected before any device work
    assert B.lib.ibm_lattice_create(4, 4, 4, 0.5, 0, ctypes.c_void_p(256), 1 << 20, None,
                                    ctypes.byref(h)) == -1
    assert B.lib.ibm_lattice_create(4, 4, 4, 1.0, 0, None, 1 << 20, None, ctypes.byref(h)) == -1
    assert B.lib.ibm_lattice_create(4, 4, 4, 1.0, 0, ctypes.c_void_p(256), 16, None,
                                    ctypes.byref(h)) == -1
    assert B.lib.ibm_step(None, 1) == -1
    nodes = np.array([642, 642], dtype=np.int32)
    faces = np.array([1280, 1280], dtype=np.int32)
    assert B.lib.ibm_membrane_bytes(2, B._ptr(nodes), B._ptr(faces), ctypes.byref(n)) == 0
    assert n.value > 2 * (642 * 3 * 16 + 1280 * 64)
    bad = np.array([2, 642], dtype=np.int32)
    assert B.lib.ibm_membrane_bytes(2, B._ptr(bad), B._ptr(faces), ctypes.byref(n)) == -1
    # an empty membrane, a lattice beyond 2^31 nodes and a grid beyond the
    # launch limits are refused by the size queries themselves
    assert B.lib.ibm_membrane_bytes(0, B._ptr(nodes), B._ptr(faces), ctypes.byref(n)) == -1
    assert "n_caps" in B.lib.ibm_last_error().decode()
    assert B.lib.ibm_lattice_bytes(2048, 1024, 1025, 0, ctypes.byref(n)) == -1
    assert "2^31" in B.lib.ibm_last_error().decode()
    assert B.lib.ibm_lattice_bytes(4, 4, 65536, 0, ctypes.byref(n)) == -1
    assert B.lib.ibm_lattice_bytes(1024, 1024, 2048, 0, ctypes.byref(n)) == 0
    assert n.value > 2 * 19 * 4 * 2 ** 31


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_library_icosphere_matches_oracle_mesh(B, orc, level):
    """Both generators follow Sec. II.D from the same icosahedron, so they
    give the same nodes and the same oriented faces up to relabelling."""
    x, t = B.icosphere(level, 2.5, (1.0, 2.0, 3.0))
    xo, to = orc.icosphere(level, 2.5, (1.0, 2.0, 3.0))
    assert x.shape == xo.shape and t.shape == to.shape
    key = lambda a: np.round(a, 9)
    order = np.lexsort(key(x).T)
    order_o = np.lexsort(key(xo).T)
    assert np.abs(x[order] - xo[order_o]).max() < 1e-13
    relabel = np.empty(len(x), dtype=np.int64)
    relabel[order] = order_o
    canon = lambda f: tuple(np.roll(f, -int(np.argmin(f))))
    assert {canon(f) for f in relabel[t]} == {canon(f) for f in to}
    assert B.lib.ibm_icosphere(8, 1.0, 0, 0, 0, B._ptr(x), B._ptr(t)) == -1


def test_deformation_function_marshals_the_adjoint_gradient(B):
    """binding.deformation on the host side: the lattice factory receives the
    parameter values, the gradient the adjoint call returns reaches the
    parameters by the chain rule, and the lattice is closed.  A stand-in
    lattice returns D = a ks^2 + b ka + c uw^3 with its exact gradient (no GPU
    call)."""
    import torch

    made = []

    class Stand:
        def __init__(self, ks, ka, uw):
            self.p = (np.asarray(ks), np.asarray(ka), uw)
            self.closed = False

        def adjoint_gradient(self, steps, checkpoint_every, capsule, couette_start):
            assert (steps, checkpoint_every, capsule, couette_start) == (40, 8, 1, True)
            ks, ka, uw = self.p
            D = float(2.0 * np.sum(ks ** 2) + 3.0 * np.sum(ka) + 5.0 * uw ** 3)
            return {"D": D, "dks": 4.0 * ks, "dka": np.full_like(ka, 3.0), "duw": 15.0 * uw ** 2}

        def close(self):
            self.closed = True

    def make(ks, ka, uw):
        made.append(Stand(ks, ka, uw))
        return made[-1]

    f64 = dict(dtype=torch.float64)
    s = torch.tensor(1.5, requires_grad=True, **f64)
    uw = torch.tensor(0.02, requires_grad=True, **f64)
    ks0 = torch.tensor([0.01, 0.03], **f64)
    ks = ks0 * s
    ka = 0.5 * ks
    D = B.deformation(make, ks, ka, uw, 40, checkpoint_every=8, capsule=1)
    (7.0 * D).backward()
    assert len(made) == 1 and made[0].closed
    assert np.allclose(made[0].p[0], [0.015, 0.045]) and made[0].p[2] == pytest.approx(0.02)
    # dD/ds = sum(4 ks * ks0) + sum(3 * 0.5 ks0); dD/duw = 15 uw^2
    want_s = 7.0 * float(torch.sum(4.0 * ks0 * 1.5 * ks0) + torch.sum(1.5 * ks0))
    assert float(s.grad) == pytest.approx(want_s, rel=1e-12)
    assert float(uw.grad) == pytest.approx(7.0 * 15.0 * 0.02 ** 2, rel=1e-12)


def test_binding_constants_match_the_header(B):
    """Every error code, option, field selector, storage code and streaming
    pattern the header defines has the same value in the binding."""
    text = open(HEADER).read()
    defs = {k: int(v) for k, v in re.findall(r"#define (IBM_[A-Z0-9_]+) \(?(-?\d+)\)?", text)}
    errors = {v: k for k, v in defs.items() if k.startswith("IBM_ERR_")}
    assert errors == B.ERRORS
    for k, v in defs.items():
        for prefix in ("IBM_OPT_", "IBM_FIELD_", "IBM_STREAM_"):
            if k.startswith(prefix):
                assert getattr(B, k[4:]) == v, k
    assert B.STORAGE == {"fp32": defs["IBM_STORAGE_FP32"], "fp16": defs["IBM_STORAGE_FP16"]}
    assert B.STORAGE_ONE_BUFFER == defs["IBM_STORAGE_ONE_BUFFER"]
