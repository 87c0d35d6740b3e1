"""The AA streaming pattern (IBM_OPT_STREAMING = 1: one population buffer,
even steps collide in place into the opposite slots, odd steps gather from
the neighbours and push back) against the FP64 oracle: the lattice update
alone, coupled steps with each delta width and both interpolation forms
(which read the swapped state after even steps), FP16 storage, the device
totals and field read-back after odd step counts, and the refused
combinations."""
import sys

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W
from parity_helpers import Case, O, rel_err, scaled_err
from test_gpu_parity import W19, small_case

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1004_2416_amd import binding
    return binding


@pytest.mark.parametrize("shape,tau,linear", [((32, 20, 12), 1.0, False), ((64, 8, 6), 0.8, False),
                                              ((4, 3, 5), 1.7, True), ((256, 4, 4), 0.6, False)])
def test_aa_lattice_update(B, shape, tau, linear):
    """Five single steps (both kinds, the read-back after even and odd
    counts) and then 37 graph-replayed steps, walls moving."""
    nx, ny, nz = shape
    wl = W.Workload("lbm", nx, ny, nz, tau, 0.03, 2, 0, [])
    c = Case(wl, perturb=0.02, seed=3)
    lat = c.gpu(graph=True)
    lat.set_option(B.OPT_EQUILIBRIUM, int(linear))
    lat.set_option(B.OPT_STREAMING, B.STREAM_AA)
    f = c.f0
    for k in range(5):
        lat.step(1)
        f = O.lbm_step(f, None, tau, 0.03, linear=linear)
        assert rel_err(lat.populations().cpu().numpy(), f) < 1e-5, k
    lat.step(37)
    for _ in range(37):
        f = O.lbm_step(f, None, tau, 0.03, linear=linear)
    got = lat.populations().cpu().numpy()
    mass = lat.totals()[0]
    lat.close()
    say("  AA lattice %s: 42 steps, f %.2e, mass %.15g vs %.15g" % (shape, rel_err(got, f), mass,
                                                                    f.sum()))
    assert rel_err(got, f) < 1e-5
    assert abs(mass - f.sum()) < 1e-9 * f[0].size


@pytest.mark.parametrize("m,box,storage", [(2, 3, "fp32"), (3, 3, "fp32"), (4, 3, "fp32"),
                                           (2, 5, "fp32"), (3, 5, "fp32"), (3, 0, "fp32"),
                                           (3, 3, "fp16")])
def test_aa_coupled_steps(B, m, box, storage):
    """A capsule (and its stencils across the periodic x end): 1 step, then
    48 graph-replayed steps, populations, nodes and forces against the
    oracle.  After odd steps box 3 interpolates through LDS boxes, box 5 from
    the velocity field and box 0 per stencil node; after even steps all
    three go through the velocity field, which reads the swapped state."""
    c = small_case(n=(32, 20, 16), m=m, level=2, r=4.0, ca=0.02, uw=0.03,
                   center=(30.6, 9.3, 7.6))
    lat = c.gpu(storage=storage, graph=True)
    lat.set_option(B.OPT_STENCIL_BOX, box)
    lat.set_option(B.OPT_STREAMING, B.STREAM_AA)
    sim = c.oracle(f=lat.populations().cpu().numpy())
    for n in (1, 48):
        lat.step(n)
        assert sim.run(n) == 0
        f = lat.populations().cpu().numpy()
        xg, Fg, ug = [a.cpu().numpy() for a in lat.mesh()]
        ef, ex = rel_err(f, sim.f), float(np.max(np.abs(xg - sim.x)))
        eu = scaled_err(ug, sim.un)
        say("  AA m=%d box %d %s after %d: f %.2e  u %.2e  x %.2e" % (m, box, storage, sim.t, ef,
                                                                     eu, ex))
        if storage == "fp32":
            assert ef < 1e-5 and eu < 1e-4 and ex < 1e-4
        else:
            dev = np.max(np.abs(sim.f - W19))
            assert np.max(np.abs(f - sim.f)) < sim.t * 2.0 ** -11 * dev and ex < 1e-3
    lat.close()


def test_aa_matches_two_buffers(B):
    """The same coupled run with both streaming patterns: 33 steps (ending
    odd, the swapped state) and 64, then the fields and the totals."""
    c = small_case(n=(32, 20, 16), m=3, level=2, r=4.0, ca=0.02, uw=0.03)
    out = {}
    for pattern in (B.STREAM_TWO_BUFFERS, B.STREAM_AA):
        lat = c.gpu(graph=True)
        lat.set_option(B.OPT_STREAMING, pattern)
        res = []
        for n in (33, 31):
            lat.step(n)
            res.append((lat.populations().cpu().numpy(), lat.velocity().cpu().numpy(),
                        lat.mesh()[0].cpu().numpy(), lat.totals()))
        lat.close()
        out[pattern] = res
    for k in range(2):
        a, b = out[B.STREAM_TWO_BUFFERS][k], out[B.STREAM_AA][k]
        say("  AA vs two buffers, step %d: f %.2e  u %.2e  x %.2e  totals %.2e" % (
            (33, 64)[k], rel_err(b[0], a[0]), scaled_err(b[1], a[1]),
            float(np.max(np.abs(b[2] - a[2]))), float(np.max(np.abs(b[3] - a[3])))))
        assert rel_err(b[0], a[0]) < 1e-6
        assert scaled_err(b[1], a[1]) < 1e-5
        assert np.max(np.abs(b[2] - a[2])) < 1e-5
        assert np.max(np.abs(b[3] - a[3])) < 1e-9 * b[0][0].size


@pytest.mark.parametrize("ab2,linear,storage", [(True, False, "fp32"), (False, True, "fp32"),
                                                (True, True, "fp16")])
def test_aa_variants_against_oracle(B, ab2, linear, storage):
    """The paper's two variants (Adams-Bashforth advection, the linearised
    equilibrium) on a one-buffer lattice: 1 step, then 99 through the
    graphs, against the oracle (FP16: each step adds at most 2^-11 of the
    largest deviation)."""
    c = small_case(n=(32, 20, 16), m=3, level=2, r=4.0, ca=0.02, uw=0.03)
    wl = c.wl
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, storage=storage, one_buffer=True)
    lat.set_shear(wl.u_w, init_profile=False)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    lat.set_option(B.OPT_GRAPH, 1)
    lat.set_option(B.OPT_ADVECTION, int(ab2))
    lat.set_option(B.OPT_EQUILIBRIUM, int(linear))
    lat.set_populations(c.f0)
    sim = c.oracle(f=lat.populations().cpu().numpy(), ab2=ab2, linear=linear)
    lat.step(1)
    lat.step(99)
    assert sim.run(100) == 0
    f = lat.populations().cpu().numpy()
    xg = lat.mesh()[0].cpu().numpy()
    lat.close()
    ex = float(np.max(np.abs(xg - sim.x)))
    say("  AA ab2 %s linear %s %s, 100 steps: f %.2e  x %.2e" % (ab2, linear, storage,
                                                                rel_err(f, sim.f), ex))
    if storage == "fp32":
        assert rel_err(f, sim.f) < 1e-5 and ex < 1e-4
    else:
        dev = np.max(np.abs(sim.f - W19))
        assert np.max(np.abs(f - sim.f)) < 100 * 2.0 ** -11 * dev and ex < 1e-3


def test_aa_refused_combinations(B):
    c = small_case(n=(32, 20, 16), m=3)
    lat = c.gpu(graph=False)
    lat.set_option(B.OPT_STREAMING, B.STREAM_AA)
    lat.step(1)
    with pytest.raises(B.IBMError):
        lat.set_populations(c.f0)           # odd count: the swapped state
    with pytest.raises(B.IBMError):
        lat.set_option(B.OPT_STREAMING, 0)  # changes only at even counts
    lat.step(1)
    with pytest.raises(B.IBMError):
        lat.attach_tangent([1.0], [1.0], 0.0)
    lat.set_option(B.OPT_STREAMING, 0)
    lat.close()
    odd = Case(W.Workload("odd", 30, 8, 8, 1.0, 0.01, 2, 0, []))
    lat = odd.gpu(graph=False)
    with pytest.raises(B.IBMError):
        lat.set_option(B.OPT_STREAMING, B.STREAM_AA)  # nx not a multiple of 4
    lat.close()


def test_one_buffer_lattice(B):
    """IBM_STORAGE_ONE_BUFFER: the lattice holds one population array and
    streams with the AA pattern.  A coupled run (1 step, then 63 through the
    graphs, ending odd; then 1 more) against the oracle and against the same
    run on a two-buffer lattice with the AA pattern; the refused
    combinations."""
    c = small_case(n=(32, 20, 16), m=3, level=2, r=4.0, ca=0.02, uw=0.03)
    wl = c.wl

    def make(one_buffer):
        lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, one_buffer=one_buffer)
        lat.set_shear(wl.u_w, init_profile=False)
        lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
        lat.set_option(B.OPT_GRAPH, 1)
        if not one_buffer:
            lat.set_option(B.OPT_STREAMING, B.STREAM_AA)
        lat.set_populations(c.f0)
        return lat

    one, two = make(True), make(False)
    assert one._state.numel() < two._state.numel()
    sim = c.oracle()
    for n in (1, 63, 1):
        one.step(n)
        two.step(n)
        assert sim.run(n) == 0
        f1, f2 = one.populations().cpu().numpy(), two.populations().cpu().numpy()
        x1 = one.mesh()[0].cpu().numpy()
        x2 = two.mesh()[0].cpu().numpy()
        say("  one buffer after %d: f %.2e (two buffers %.2e)  x %.2e  vs two %.2e" % (
            sim.t, rel_err(f1, sim.f), rel_err(f2, sim.f), float(np.max(np.abs(x1 - sim.x))),
            float(np.max(np.abs(x1 - x2)))))
        assert rel_err(f1, sim.f) < 1e-5 and np.max(np.abs(x1 - sim.x)) < 1e-4
        assert rel_err(f1, f2) < 1e-6 and np.max(np.abs(x1 - x2)) < 1e-5
    assert abs(one.totals()[0] - sim.f.sum()) < 1e-9 * sim.f[0].size
    with pytest.raises(B.IBMError):
        one.set_option(B.OPT_STREAMING, B.STREAM_TWO_BUFFERS)
    one.step(1)  # even count again
    with pytest.raises(B.IBMError):
        one.set_option(B.OPT_STREAMING, B.STREAM_TWO_BUFFERS)
    with pytest.raises(B.IBMError):
        one.attach_tangent([1.0], [1.0], 0.0)
    with pytest.raises(B.IBMError):
        one.adjoint_gradient(4, 2)
    with pytest.raises(B.IBMError):
        B.Batch([one])
    one.close()
    two.close()
    with pytest.raises(B.IBMError):
        B.Lattice(30, 8, 8, 1.0, one_buffer=True)
