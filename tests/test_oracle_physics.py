"""Physics pins of the whole oracle timestep (Sec. II.C) against results the
paper prints: the first row of Table 2 (deviation of the Taylor deformation
and of the inclination angle from the small-deformation theory at
kappa t = 120), the volume drift of Sec. IV.D, and exact kinematics of a
force-free membrane in the Couette profile."""
import os

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def couette_populations(orc, nz, ny, nx, uw, linear=False):
    f = np.empty((19, nz, ny, nx))
    for z in range(nz):
        ux = uw * (2 * z + 1 - nz) / nz
        f[:, z] = orc.equilibrium(1.0, [ux, 0.0, 0.0], linear=linear)[:, None, None]
    return f


def _table(name):
    rows = np.loadtxt(os.path.join(GOLDEN, name), comments="#")
    return {int(r[0]): r[1:] for r in rows}


_RUNS = {}


def paper_run(orc, m):
    """H = 35, r = 3.5, 1280 faces, G = 0.01, Re = 0.02, tau = 1, run to
    kappa t = 120 from the undeformed sphere in the linear shear profile."""
    if m not in _RUNS:
        wl = W.paper_case(35, 3.5, 3, m)
        cap = wl.capsules[0]
        x, t = orc.icosphere(cap.level, cap.r, cap.center)
        f = couette_populations(orc, wl.nz, wl.ny, wl.nx, wl.u_w)
        sim = orc.Simulation(f, x, x, t, cap.ks, cap.ka, wl.tau, wl.u_w, m)
        v0 = orc.capsule_observables(x, t)["V"]
        m0 = f.sum()
        assert sim.run(wl.steps) == 0
        o = orc.capsule_observables(sim.x, t)
        _RUNS[m] = (o, v0, m0, sim)
    return _RUNS[m]


@pytest.mark.slow
@pytest.mark.parametrize("m", [2, 3, 4])
def test_table2_first_row(orc, m):
    o, v0, m0, sim = paper_run(orc, m)
    G = 0.01
    Da = 25 / 4 * G                  # Sec. IV.A: D/G = 25/4 for Skalak, C = 1
    tha = np.pi * 15 / 8 * G         # Eq. (analyticangle)
    dD = 100 * (o["D"] - Da) / Da
    dth = 100 * ((np.pi / 4 - o["theta"]) - tha) / tha
    gold = _table("table2_H35.txt")[m]
    assert abs(dD - gold[0]) < 1.5, dD
    assert abs(dth - gold[1]) < 3.0, dth
    # D/G of order 7 instead of 6.25 (Sec. IV.A)
    assert 6.9 < o["D"] / G < 7.5


@pytest.mark.slow
@pytest.mark.parametrize("m", [2, 3, 4])
def test_volume_drift_and_mass(orc, m):
    o, v0, m0, sim = paper_run(orc, m)
    lo, hi = _table("volume_drift.txt")[m]
    drift = abs(o["V"] / v0 - 1)
    # same order of magnitude as quoted (within a factor 2 of the range)
    assert lo / 2 < drift < 2 * hi, drift
    assert abs(sim.f.sum() / m0 - 1) < 1e-12


def test_force_free_membrane_moves_with_couette_flow(orc):
    """With k_s = k_a = 0 the nodes are passive tracers; in the exactly
    steady linear profile (linearised equilibrium) each node moves with the
    Couette velocity u_w (2 z + 1 - nz)/nz of its own height, step by step."""
    nz, uw = 16, 0.01
    x, t = orc.icosphere(1, 3.0, (4.3, 5.1, 7.2))
    f = couette_populations(orc, nz, 10, 9, uw, linear=True)
    sim = orc.Simulation(f, x, x, t, 0.0, 0.0, 1.0, uw, 3, linear_eq=True)
    assert sim.run(25) == 0
    v = uw * (2 * x[:, 2] + 1 - nz) / nz
    want = x + 25 * np.stack([v, 0 * v, 0 * v], 1)
    assert np.allclose(sim.x, want, atol=1e-13)
