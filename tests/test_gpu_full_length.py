"""Full-length runs of the shear-flow workloads in the benchmark's launch
configuration (16-step graphs, split lattice update where it applies, the
default coupling kernels) against the FP64 oracle's trajectories stored in
tests/golden/ (written by tests/golden/make_trajectories.py, which runs only
the oracle):

  128^3, one r = 16 capsule, 4-point delta: 20,000 steps
  256 x 128 x 128, 200 r = 8 capsules, 2-point delta: 10,000 steps
  the batched sweep, 64 runs of 24^3..64^3 in one batch: 5000 steps

The Taylor deformation D (Sec. III) of every capsule, every 100 steps, must
stay within 1e-3 of that capsule's largest D over the run (FP32 storage).
With FP16 population storage the bound is stated separately (see each
test).  The 64^3 sensitivities of D after 2000 steps by the adjoint are
compared with the oracle's central differences to 1e-3."""
import os
import sys

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W
from parity_helpers import WEIGHTS as W19
from parity_helpers import Case

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1004_2416_amd import binding
    return binding


def golden_trajectory(name):
    path = os.path.join(GOLDEN, "trajectory_%s.txt" % name)
    if not os.path.exists(path):
        pytest.skip("oracle trajectory %s not written yet (make_trajectories.py)" % path)
    rows = np.loadtxt(path, comments="#", ndmin=2)
    return rows[:, 0].astype(int), rows[:, 1:]


def run_trajectory(B, name, storage, mass_fix=False):
    wl = W.config(name)
    steps, Do = golden_trajectory(name)
    assert steps[-1] == wl.steps and Do.shape[1] == len(wl.capsules)
    c = Case(wl)
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, storage=storage)
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    lat.set_option(B.OPT_OVERLAP, 1)
    if mass_fix:
        lat.set_option(B.OPT_FP16_MASS, 1)
    Dg = [lat.observables()[:, 4].copy()]
    for s0, s1 in zip(steps[:-1], steps[1:]):
        lat.step(int(s1 - s0))
        Dg.append(lat.observables()[:, 4].copy())
    mass = lat.totals()[0]
    # mean over the nodes of sum_i |f_i - w_i| in the final state (for the
    # rounding bound of FP16 storage)
    f = lat.populations()
    w = f.new_tensor(W19).reshape(19, 1, 1, 1)
    dev = float((f - w).abs().sum(dim=0).mean())
    dev0 = float((f[0] - w[0]).abs().mean())
    del f
    lat.close()
    Dg = np.array(Dg)
    eD = np.max(np.abs(Dg - Do), axis=0) / np.max(np.abs(Do), axis=0)
    worst = int(np.argmax(eD))
    say("  %s %s %d steps: worst capsule %d, D error %.2e of its max D (%.4f); "
        "median capsule %.2e; final D %.5f vs %.5f; mass %.12g" % (
            name, storage, steps[-1], worst, eD[worst], np.max(np.abs(Do[:, worst])),
            float(np.median(eD)), Dg[-1, worst], Do[-1, worst], mass))
    return eD, mass, wl, (dev, dev0)


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_length_trajectory_fp32(B, name):
    eD, mass, wl, _ = run_trajectory(B, name, "fp32")
    assert eD.max() < 1e-3
    N = wl.nx * wl.ny * wl.nz
    assert abs(mass / N - 1) < 1e-6


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_length_trajectory_fp16(B, name):
    """FP16 storage of the scaled deviations (16 (f_i - w_i) / w_i, 11
    significant bits): every stored population is rounded to within 2^-11
    of its deviation at every step.  The bound stated for the whole run is
    D within 2 % of each capsule's largest D.  The mass is not protected
    from those roundings: a node's stored mass moves by at most
    2^-11 sum_i |f_i - w_i| per step, and in a steady shear flow the same
    values are rounded the same way every step, so the drift grows linearly
    in time.  The stated mass bound is that worst case over the run,
    steps * 2^-11 * mean_nodes sum_i |f_i - w_i| (final state), relative to
    the initial mass; the observed drift is printed beside it."""
    eD, mass, wl, (dev, _) = run_trajectory(B, name, "fp16")
    assert eD.max() < 2e-2
    N = wl.nx * wl.ny * wl.nz
    bound = wl.steps * 2.0 ** -11 * dev
    say("  %s fp16 mass drift %.2e, worst-case rounding bound %.2e" % (name, abs(mass / N - 1),
                                                                          bound))
    assert abs(mass / N - 1) < bound


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_length_trajectory_fp16_mass_corrected(B, name):
    """FP16 storage with IBM_OPT_FP16_MASS: the rest population takes back
    the mass the other 18 values of its node lose to rounding, so only the
    rest populations' own rounding moves the mass, by at most
    2^-11 |f_0 - w_0| per node and step: the stated mass bound is
    steps * 2^-11 * mean_nodes |f_0 - w_0|; D as without the correction."""
    eD, mass, wl, (_, dev0) = run_trajectory(B, name, "fp16", mass_fix=True)
    assert eD.max() < 2e-2
    N = wl.nx * wl.ny * wl.nz
    bound = wl.steps * 2.0 ** -11 * dev0
    say("  %s fp16 with the mass correction: mass drift %.2e, bound %.2e" % (
        name, abs(mass / N - 1), bound))
    assert abs(mass / N - 1) < bound


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_full_length_batched_sweep(B, storage):
    """The 64 independent runs of the batched sweep (24^3..64^3, delta widths
    2-4) for their full 5000 steps as one batch in the benchmark's launch
    configuration (the batch's defaults, 16-step graphs), against the
    oracle's trajectories: D of every run every 100 steps within 1e-3 of that
    run's largest D (FP32 storage), within 2e-2 with FP16 storage."""
    path = os.path.join(GOLDEN, "trajectory_c4.txt")
    if not os.path.exists(path):
        pytest.skip("oracle trajectory %s not written yet (make_trajectories.py)" % path)
    rows = np.loadtxt(path, comments="#", ndmin=2)
    steps, Do = rows[:, 0].astype(int), rows[:, 1:]
    wls = W.sweep_workloads()
    assert Do.shape[1] == len(wls) and steps[-1] == wls[0].steps
    lats = [Case(wl).gpu(storage=storage, graph=True) for wl in wls]
    batch = B.Batch(lats)
    Dg = [[lat.observables()[0, 4] for lat in lats]]
    for s0, s1 in zip(steps[:-1], steps[1:]):
        batch.step(int(s1 - s0))
        Dg.append([lat.observables()[0, 4] for lat in lats])
    batch.close()
    for lat in lats:
        lat.close()
    Dg = np.array(Dg)
    eD = np.max(np.abs(Dg - Do), axis=0) / np.max(np.abs(Do), axis=0)
    worst = int(np.argmax(eD))
    say("  batched sweep %s %d steps: worst run %d (%s, m=%d), D error %.2e of its max D; "
        "median run %.2e" % (storage, steps[-1], worst, wls[worst].name, wls[worst].m,
                             eD[worst], float(np.median(eD))))
    assert eD.max() < (1e-3 if storage == "fp32" else 2e-2)


def test_full_length_adjoint_c5(B):
    """The 64^3 sensitivities of D after 2000 steps (checkpoints every 100)
    by one reverse sweep, against the oracle's central differences."""
    path = os.path.join(GOLDEN, "sensitivities_c5_2000.txt")
    gold = {}
    for line in open(path):
        if line.startswith("#"):
            continue
        k, p, dp, dm, d = line.split()
        gold[k] = float(d)
    wl = W.config("c5")
    c = Case(wl)
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    g = lat.adjoint_gradient(2000, checkpoint_every=100, couette_start=True)
    lat.close()
    ks, ka = c.ks[0], c.ka[0]
    adj = {"ks": g["dks"][0] + (ka / ks) * g["dka"][0], "C": ks * g["dka"][0],
           "gamma": 0.5 * wl.nz * g["duw"]}
    for k in ("ks", "C", "gamma"):
        say("  c5 2000 steps d D / d %s: adjoint %.8e  oracle FD %.8e  (%.2e)" % (
            k, adj[k], gold[k], abs(adj[k] - gold[k]) / abs(gold[k])))
        assert abs(adj[k] - gold[k]) < 1e-3 * abs(gold[k])
