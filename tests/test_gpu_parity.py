"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Per step, from an identical injected state: populations within 1e-5
relative, nodal forces, force density and node velocities within 1e-5 of
their scale (FP32 arithmetic, errors ~1e-7).  Over many steps: the Taylor
deformation trajectory within 1e-3 of its maximum."""
import sys

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W
from parity_helpers import (Case, O, couette_populations, deformed_mesh, rel_err,
                            rep_populations, rep_positions, scaled_err)

pytestmark = pytest.mark.gpu

W19 = O.lattice_constants()[1][:, None, None, None]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1004_2416_amd import binding
    return binding


def small_case(n=(30, 20, 16), m=3, level=2, r=4.0, center=None, ca=0.05, uw=0.02, tau=1.0,
               perturb=0.0):
    nx, ny, nz = n
    c = center or ((nx - 1) / 2 + 0.3, (ny - 1) / 2 - 0.2, (nz - 1) / 2 + 0.1)
    ks = W.ks_from_capillary(ca, uw, nz, r, tau)
    wl = W.Workload("small", nx, ny, nz, tau, uw, m, 0, [W.CapsuleSpec(level, r, c, ks, ks)])
    return Case(wl, perturb=perturb, seed=5)


# ---------------------------------------------------------------------------
# lattice update alone
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,tau,linear", [((30, 20, 12), 1.0, False), ((64, 8, 6), 0.8, False),
                                              ((33, 7, 5), 1.7, True), ((1, 1, 2), 1.0, False),
                                              ((256, 4, 4), 0.6, False), ((300, 3, 4), 1.1, False),
                                              ((257, 2, 3), 0.9, True)])
def test_lbm_step_parity(B, shape, tau, linear):
    nx, ny, nz = shape
    say("lbm parity", shape, tau, linear)
    wl = W.Workload("lbm", nx, ny, nz, tau, 0.03, 2, 0, [])
    c = Case(wl, perturb=0.02, seed=1)
    lat = c.gpu(graph=False)
    lat.set_option(B.OPT_EQUILIBRIUM, int(linear))
    f = c.f0
    for k in range(3):
        lat.step(1)
        f = O.lbm_step(f, None, tau, 0.03, linear=linear)
        got = lat.populations().cpu().numpy()
        assert rel_err(got, f) < 1e-5, k
    rho = lat.density().cpu().numpy()
    rho_o, u_o = O.velocity_field(f)
    assert np.max(np.abs(rho - rho_o)) < 1e-5
    assert scaled_err(lat.velocity().cpu().numpy(), u_o) < 1e-4
    lat.close()


def test_couette_graph_run_matches_oracle(B):
    """500 steps from the linear profile through the captured graph."""
    nx, ny, nz, uw = 16, 8, 24, 0.05
    lat = B.Lattice(nx, ny, nz, 1.0)
    lat.set_shear(uw, init_profile=True)
    lat.step(500)
    f = rep_populations(couette_populations(nz, ny, nx, uw))
    for _ in range(500):
        f = O.lbm_step(f, None, 1.0, uw)
    got = lat.populations().cpu().numpy()
    assert rel_err(got, f) < 1e-5
    u = lat.velocity().cpu().numpy()[0].mean(axis=(1, 2))
    z = np.arange(nz)
    assert np.max(np.abs(u - uw * (2 * z + 1 - nz) / nz)) < 1e-3 * uw
    lat.close()


# ---------------------------------------------------------------------------
# one coupled step from an injected, deformed state
# ---------------------------------------------------------------------------
def deformed_state(c, steps):
    sim = c.oracle()
    assert sim.run(steps) == 0
    return rep_populations(sim.f), rep_positions(sim.x, c.node_counts)


def compare_one_step(B, c, f_s, x_s, tol_f=1e-5, tol_m=1e-5, opts=None):
    lat = c.gpu(graph=False)
    for k, v in (opts or {}).items():
        lat.set_option(k, v)
    lat.set_populations(f_s)
    lat.set_mesh(x_s)
    lat.step(1)
    sim = c.oracle(f=f_s, x=x_s)
    assert sim.run(1) == 0
    f_g = lat.populations().cpu().numpy()
    xg, Fg, ug = [a.cpu().numpy() for a in lat.mesh()]
    g_g = lat.force_density().cpu().numpy()
    errs = dict(f=rel_err(f_g, sim.f), F=scaled_err(Fg, sim.F), u=scaled_err(ug, sim.un),
                g=scaled_err(g_g, sim.g), x=float(np.max(np.abs(xg - sim.x))))
    say("  one-step errors", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["f"] < tol_f
    assert errs["F"] < tol_m
    assert errs["g"] < tol_m
    assert errs["u"] < tol_m
    assert errs["x"] < tol_m * np.max(np.abs(sim.un)) + 1e-6
    lat.close()
    return errs


@pytest.mark.parametrize("m", [2, 3, 4])
def test_coupled_step_parity(B, m):
    say("coupled step parity m =", m)
    c = small_case(m=m, level=2, r=4.0, ca=0.02, uw=0.03)
    f_s, x_s = deformed_state(c, 40)
    compare_one_step(B, c, f_s, x_s)


def test_c1_step_parity_at_sampled_steps(B):
    """The 32^3 single-capsule workload (642 nodes, 3-point delta): one step
    from the oracle's state after 1, 10, 100 and 999 steps (rounded to the
    FP32 storage), every population, force and node compared to the per-step
    bar.  (Step 0, the undeformed capsule, is its own test below.)"""
    c = Case(W.config("c1"))
    sim = c.oracle()
    done = 0
    for s in (1, 10, 100, 999):
        assert sim.run(s - done) == 0
        done = s
        say("c1 one step from step", s)
        compare_one_step(B, c, rep_populations(sim.f), rep_positions(sim.x, c.node_counts))


def test_coupled_step_parity_periodic_wrap(B):
    """A capsule straddling the periodic x and y ends, ragged lattice."""
    say("periodic wrap")
    c = small_case(n=(27, 19, 18), m=4, level=2, r=4.0, center=(0.4, 18.2, 8.6), ca=0.02)
    f_s, x_s = deformed_state(c, 30)
    compare_one_step(B, c, f_s, x_s)


@pytest.mark.parametrize("n,m", [((4, 4, 16), 2), ((6, 5, 16), 3), ((4, 6, 18), 4)])
def test_coupled_step_parity_capsule_wider_than_the_lattice(B, n, m):
    """A capsule of radius 3 on lattices 4 to 6 nodes wide in x and y: its
    stencils wrap onto its own periodic images, and a spreading box spans
    more than one period, so the box flush and the tile stamps take their
    general wrapped-index paths (nx not a multiple of 4 included)."""
    say("capsule wider than the lattice", n, "m", m)
    nx, ny, nz = n
    c = small_case(n=n, m=m, level=2, r=3.0, ca=0.02,
                   center=((nx - 1) / 2 + 0.3, (ny - 1) / 2 - 0.2, (nz - 1) / 2 + 0.1))
    f_s, x_s = deformed_state(c, 5)
    compare_one_step(B, c, f_s, x_s)


def test_coupled_step_parity_several_capsules(B):
    say("several capsules")
    nx, ny, nz, uw = 40, 24, 20, 0.02
    caps = []
    for k, (cen, lev, r) in enumerate([((8.3, 6.1, 9.7), 2, 3.5), ((25.0, 17.5, 10.2), 1, 3.0),
                                       ((38.7, 8.0, 9.1), 2, 3.2)]):
        ks = W.ks_from_capillary(0.02 + 0.01 * k, uw, nz, r)
        caps.append(W.CapsuleSpec(lev, r, cen, ks, 2.0 * ks))
    c = Case(W.Workload("three", nx, ny, nz, 1.0, uw, 3, 0, caps))
    f_s, x_s = deformed_state(c, 40)
    compare_one_step(B, c, f_s, x_s)


def test_coupled_step_parity_dense_mesh(B):
    """A 20480-face capsule of radius 6 with the 4-point delta: about a
    thousand membrane nodes reach each force tile near the membrane."""
    say("dense mesh")
    c = small_case(n=(24, 24, 24), m=4, level=5, r=6.0, ca=0.02)
    f_s, x_s = deformed_state(c, 3)
    compare_one_step(B, c, f_s, x_s)


def test_coupled_step_parity_crowded_overlapping_capsules(B):
    """Seventy small overlapping capsules around one point: hundreds of
    stencil contributions land on the same lattice nodes."""
    say("crowded tiles")
    nx = ny = nz = 16
    uw = 0.02
    rng = np.random.default_rng(8)
    caps = []
    for k in range(70):
        cen = tuple(7.5 + rng.uniform(-1.0, 1.0, 3))
        r = 2.0 + 0.5 * rng.uniform()
        ks = W.ks_from_capillary(0.05, uw, nz, r)
        caps.append(W.CapsuleSpec(0, r, cen, ks, ks))
    c = Case(W.Workload("crowded", nx, ny, nz, 1.0, uw, 2, 0, caps))
    f_s, x_s = deformed_state(c, 5)
    compare_one_step(B, c, f_s, x_s)


@pytest.mark.parametrize("m", [2, 3, 4])
@pytest.mark.parametrize("box", [1, 2, 3, 4, 5])
def test_stencil_box_modes(B, m, box):
    """Spreading and/or interpolation through per-block LDS boxes (bits 0, 1)
    or interpolation from the velocity field (bit 2) match the oracle
    like the direct per-lane form."""
    say("stencil box", box, "m", m)
    c = small_case(n=(40, 36, 30), m=m, level=3, r=8.0, ca=0.02, uw=0.03)
    f_s, x_s = deformed_state(c, 10)
    lat_opts = {B.OPT_STENCIL_BOX: box}
    compare_one_step(B, c, f_s, x_s, opts=lat_opts)


def test_autotune_keeps_the_run_on_the_oracle(B):
    """The autotuner times real steps of every candidate; afterwards the run
    is where the oracle is after the same number of steps."""
    c = small_case(m=3, ca=0.02, uw=0.03)
    lat = c.gpu(graph=True)
    chosen = lat.autotune(16)
    n = lat.steps
    say("  autotune chose", chosen, "after", n, "steps")
    assert 0 <= chosen["lbm_variant"] < 512 and 0 <= chosen["stencil_box"] < 6
    sim = c.oracle()
    assert sim.run(n) == 0
    f = lat.populations().cpu().numpy()
    xg = lat.mesh()[0].cpu().numpy()
    lat.close()
    assert rel_err(f, sim.f) < 1e-5
    assert np.max(np.abs(xg - sim.x)) < 1e-3


@pytest.mark.parametrize("box", [3, 5])
def test_coupling_box_too_large(B, box):
    """A coarse capsule (42 nodes, radius 14): the stencil box of every block
    exceeds the on-chip capacity, so the contributions go to and come from
    the global fields directly (with box 5 the nodes for the velocity field
    are then marked per stencil node)."""
    say("oversized boxes", box)
    c = small_case(n=(40, 40, 40), m=3, level=1, r=14.0, ca=0.02, uw=0.03)
    f_s, x_s = deformed_state(c, 10)
    compare_one_step(B, c, f_s, x_s, opts={B.OPT_STENCIL_BOX: box})


def test_undeformed_capsule_has_zero_force(B):
    c = small_case(m=2)
    lat = c.gpu(graph=False)
    _, F, _ = lat.mesh()
    lat.step(1)
    _, F, _ = lat.mesh()
    assert float(F.abs().max()) < 1e-12
    lat.close()


# ---------------------------------------------------------------------------
# trajectories
# ---------------------------------------------------------------------------
def trajectory(B, c, steps, every, graph=True, box=-1):
    lat = c.gpu(graph=graph)
    if box >= 0:
        lat.set_option(B.OPT_STENCIL_BOX, box)
    sim = c.oracle()
    Dg, Do = [], []
    for k in range(steps // every):
        lat.step(every)
        assert sim.run(every) == 0
        obs = lat.observables()
        Dg.append(obs[:, 4])
        Do.append([o["D"] for o in c.observables(sim.x)])
    xg = lat.mesh()[0].cpu().numpy()
    lat.close()
    return np.array(Dg), np.array(Do), xg, sim


def test_trajectory_c1(B):
    """The 32^3 single-capsule workload (r = 6, 1280 faces, 3-point delta,
    Ca = 0.05), its full 1000 steps through graphs, D every 50 steps."""
    say("trajectory c1 1000 steps")
    c = Case(W.config("c1"))
    Dg, Do, xg, sim = trajectory(B, c, 1000, 50)
    say("  D gpu", Dg[-1], "oracle", Do[-1], "max dev", np.max(np.abs(Dg - Do)))
    assert np.max(np.abs(Dg - Do)) < 1e-3 * np.max(np.abs(Do))
    assert np.max(np.abs(xg - sim.x)) < 1e-3


@pytest.mark.parametrize("nx,box", [(24, -1), (23, 5), (24, 4)])
def test_trajectory_drifting_capsule_wraps_and_recentres(B, nx, box):
    """An off-centre capsule carried 18 lattice spacings along x by the shear
    flow: crosses the periodic end and has its frame re-centred many times;
    with the velocity field (box 4, 5) also on a lattice whose x extent
    is not a multiple of the tile size (tiles straddling the periodic end)."""
    say("drifting capsule", nx, box)
    ny, nz, uw, r = 16, 24, 0.04, 3.0
    ks = W.ks_from_capillary(0.05, uw, nz, r)
    wl = W.Workload("drift", nx, ny, nz, 1.0, uw, 3, 0,
                    [W.CapsuleSpec(2, r, (12.2, 7.6, 17.0), ks, ks)])
    c = Case(wl)
    Dg, Do, xg, sim = trajectory(B, c, 1000, 100, box=box)
    assert np.mean(sim.x[:, 0]) - np.mean(c.xref[:, 0]) > 12.0
    assert np.max(np.abs(Dg - Do)) < 1e-3 * np.max(np.abs(Do))
    assert np.max(np.abs(xg - sim.x)) < 1e-3


def test_profiling_steps_are_ordinary_steps(B):
    """ibm_profile_step and ibm_profile_lattice_kernel advance the run by
    ordinary steps (plain launches; the second launches the collide-stream
    through hipExtLaunchKernel so that events take its dispatch's own
    timestamps): after 1 + 2 + 2 + 1 steps the run matches the oracle's six
    steps to the per-step bar, and the kernel's own duration is positive and
    within the lattice phase measured around it."""
    c = small_case(m=3, perturb=0.01)
    lat = c.gpu(graph=True)
    lat.step(1)
    phases = lat.profile(2)
    kms = lat.lattice_kernel_ms(2)
    lat.step(1)
    sim = c.oracle()
    assert sim.run(6) == 0
    f_g = lat.populations().cpu().numpy()
    xg = lat.mesh()[0].cpu().numpy()
    assert lat.steps == 6
    lat.close()
    say("  profiled steps: f %.2e  x %.2e  lattice phase %.4f ms  kernel %.4f ms"
        % (rel_err(f_g, sim.f), np.max(np.abs(xg - sim.x)), phases["lbm"], kms))
    assert rel_err(f_g, sim.f) < 1e-5
    assert np.max(np.abs(xg - sim.x)) < 1e-5
    assert 0.0 < kms < phases["lbm"] + 0.02

@pytest.mark.parametrize("box", [-1, 5])
def test_split_update_overlap(B, box):
    """IBM_OPT_OVERLAP on a tall lattice: the lattice update of graph steps is
    split into the slab of rows stencils can reach (after spreading) and the
    other rows (without force, inside the coupling launches).  192 steps with
    two re-centrings against the oracle, with the default interpolation and
    with the velocity field (box 5); then the option off goes back to
    the whole lattice."""
    nx, ny, nz, uw, r = 24, 40, 64, 0.02, 4.0
    ks = W.ks_from_capillary(0.05, uw, nz, r)
    c = Case(W.Workload("tall", nx, ny, nz, 1.0, uw, 3, 0,
                        [W.CapsuleSpec(2, r, (11.7, 19.6, 31.8), ks, ks)]), perturb=0.01, seed=5)
    lat = c.gpu(graph=True)
    if box >= 0:
        lat.set_option(B.OPT_STENCIL_BOX, box)
    lat.set_option(B.OPT_OVERLAP, 2)
    zlo, zhi, ylo, yhi = lat.split_box()
    say("  force box z", zlo, zhi, "y", ylo, yhi)
    # the capsule spans z 27.8..35.8; stencils reach 1 below and 2 above, the
    # margin is 4 + ceil(2 * 0.02 * 64) = 7, rounded out to multiples of 4
    assert (zlo, zhi, ylo, yhi) == (16, 48, 0, ny)
    sim = c.oracle()
    lat.step(192)
    assert sim.run(192) == 0
    lat.synchronize()
    f = lat.populations().cpu().numpy()
    xg = lat.mesh()[0].cpu().numpy()
    ef, ex = rel_err(f, sim.f), float(np.max(np.abs(xg - sim.x)))
    say("  overlap 192 steps: f %.2e  x %.2e" % (ef, ex))
    assert ef < 1e-5 and ex < 1e-4
    # value 1 splits only with 2^20 nodes outside the slab (here 40 k)
    lat.set_option(B.OPT_OVERLAP, 1)
    assert lat.split_box() == (0, nz, 0, ny)
    lat.set_option(B.OPT_OVERLAP, 0)
    assert lat.split_box() == (0, nz, 0, ny)
    lat.step(32)
    assert sim.run(32) == 0
    assert rel_err(lat.populations().cpu().numpy(), sim.f) < 1e-5
    lat.close()


def test_split_update_falls_back(B):
    """The whole lattice stays one update where the slab would hold more than
    three quarters of the rows; a capsule across the periodic y end."""
    short = small_case(m=3, ca=0.02, uw=0.03).gpu(graph=True)
    short.set_option(B.OPT_OVERLAP, 2)
    nz, ny, nx = short.shape
    assert short.split_box() == (0, nz, 0, ny)
    short.close()
    nx, ny, nz, uw, r = 24, 40, 64, 0.02, 4.0
    ks = W.ks_from_capillary(0.05, uw, nz, r)
    c = Case(W.Workload("tall", nx, ny, nz, 1.0, uw, 3, 0,
                        [W.CapsuleSpec(2, r, (11.7, 2.5, 31.8), ks, ks)]))
    lat = c.gpu(graph=True)
    lat.set_option(B.OPT_OVERLAP, 2)
    assert lat.split_box() == (16, 48, 0, ny)
    sim = c.oracle()
    lat.step(64)
    assert sim.run(64) == 0
    assert rel_err(lat.populations().cpu().numpy(), sim.f) < 1e-5
    lat.close()


def test_split_update_after_the_mesh_moves(B):
    """The split update with the membrane moved by ibm_set_mesh far enough
    that the force slab changes: the rows outside the new slab take the
    force-free update, so tiles the previous step stamped there must not keep
    their force field.  Move up by 14 lattice spacings, step, move back,
    step; the oracle makes the same moves."""
    nx, ny, nz, uw, r = 24, 40, 64, 0.02, 4.0
    ks = W.ks_from_capillary(0.05, uw, nz, r)
    c = Case(W.Workload("tall", nx, ny, nz, 1.0, uw, 3, 0,
                        [W.CapsuleSpec(2, r, (11.7, 19.6, 31.8), ks, ks)]), perturb=0.01, seed=5)
    lat = c.gpu(graph=True)
    lat.set_option(B.OPT_OVERLAP, 2)
    sim = c.oracle()
    lat.step(33)
    assert sim.run(33) == 0
    boxes = [lat.split_box()]
    for dz in (14.0, -14.0):
        xn = rep_positions(sim.x + np.array([0.0, 0.0, dz]), c.node_counts)
        lat.set_mesh(xn)
        sim.x[:] = xn
        lat.step(40)
        assert sim.run(40) == 0
        boxes.append(lat.split_box())
        f = lat.populations().cpu().numpy()
        xg = lat.mesh()[0].cpu().numpy()
        ef, ex = rel_err(f, sim.f), float(np.max(np.abs(xg - sim.x)))
        say("  moved by %+g: slab %s  f %.2e  x %.2e" % (dz, boxes[-1], ef, ex))
        assert ef < 1e-5 and ex < 1e-4
    # the slab did follow the membrane up and back
    assert boxes[1][0] > boxes[0][0] and boxes[2][0] < boxes[1][0]
    lat.close()


def test_adams_bashforth_and_linear_equilibrium(B):
    """The two variants of the method the paper tests: second-order
    advection (Sec. II.C) and the linearised equilibrium (Sec. IV.A)."""
    say("AB2 + linear equilibrium")
    c = small_case(m=3, ca=0.02, uw=0.03)
    for ab2, linear in ((True, False), (False, True), (True, True)):
        lat = c.gpu(graph=True)
        lat.set_option(B.OPT_ADVECTION, int(ab2))
        lat.set_option(B.OPT_EQUILIBRIUM, int(linear))
        sim = c.oracle(ab2=ab2, linear=linear)
        lat.step(1)
        assert sim.run(1) == 0
        lat.step(99)
        assert sim.run(99) == 0
        xg = lat.mesh()[0].cpu().numpy()
        f = lat.populations().cpu().numpy()
        lat.close()
        say("   ab2", ab2, "linear", linear, "x err %.2e" % np.max(np.abs(xg - sim.x)),
            "f err %.2e" % rel_err(f, sim.f))
        assert np.max(np.abs(xg - sim.x)) < 1e-4
        assert rel_err(f, sim.f) < 1e-5


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_size_step_parity(B, name):
    """The full-size workloads (128^3 with one 2562-node capsule and the
    4-point delta; 256x128x128 with 200 capsules and the 2-point delta) in the
    launch configuration the benchmark uses: one step from an identical
    injected state with every capsule deformed by ~2 %, every population,
    node and force compared; then two steps from the initial state."""
    say("full size", name)
    wl = W.config(name)
    c = Case(wl)
    from paper_1004_2416_amd import binding as Bm
    lat = Bm.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    x_s = deformed_mesh(c, 0.02, 11)
    lat.set_mesh(x_s)
    lat.step(1)
    sim = c.oracle(x=x_s)
    assert sim.run(1) == 0
    errs = dict(f=rel_err(lat.populations().cpu().numpy(), sim.f))
    xg, Fg, ug = [a.cpu().numpy() for a in lat.mesh()]
    errs.update(F=scaled_err(Fg, sim.F), u=scaled_err(ug, sim.un),
                g=scaled_err(lat.force_density().cpu().numpy(), sim.g),
                x=float(np.max(np.abs(xg - sim.x))))
    obs = lat.observables()
    Do = np.array([o["D"] for o in c.observables(sim.x)])
    lat.close()
    say("  one-step errors", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["f"] < 1e-5 and errs["F"] < 1e-5 and errs["u"] < 1e-5 and errs["g"] < 1e-5
    assert errs["x"] < 2e-6
    assert np.max(np.abs(obs[:, 4] - Do)) < 1e-5 * np.max(np.abs(Do))

    lat = Bm.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    lat.step(2)
    sim = c.oracle()
    assert sim.run(2) == 0
    ef = rel_err(lat.populations().cpu().numpy(), sim.f)
    xg, _, ug = [a.cpu().numpy() for a in lat.mesh()]
    lat.close()
    say("  two steps from rest: f %.2e  u %.2e  x %.2e" % (ef, scaled_err(ug, sim.un),
                                                          np.max(np.abs(xg - sim.x))))
    assert ef < 1e-5 and scaled_err(ug, sim.un) < 1e-5
    # FP32 node coordinates (|x - origin| <= 16): half an ulp of rounding per step
    assert np.max(np.abs(xg - sim.x)) < 4e-6


@pytest.mark.parametrize("name,steps,every", [("c2", 320, 40), ("c3", 96, 32)])
def test_trajectory_full_size(B, name, steps, every):
    """The full-size workloads as the benchmark runs them (16-step graphs,
    IBM_OPT_OVERLAP = 1: on 128^3 the lattice update is split at the force
    slab, re-centring every 64 steps) against the oracle from the same start:
    the Taylor deformation of every capsule within 1e-3 of its largest value
    over the run.  Node positions are FP32 offsets of up to 16 lattice
    spacings from each capsule's origin, so every step's x += u rounds by up
    to ~1e-6; they must stay within steps x 1e-6 of the oracle's."""
    wl = W.config(name)
    c = Case(wl)
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    lat.set_option(B.OPT_OVERLAP, 1)
    sim = c.oracle()
    Dg, Do = [], []
    for k in range(steps // every):
        lat.step(every)
        assert sim.run(every) == 0
        Dg.append(lat.observables()[:, 4].copy())
        Do.append([o["D"] for o in c.observables(sim.x)])
    say("  %s split box %s" % (name, lat.split_box()))
    xg = lat.mesh()[0].cpu().numpy()
    lat.close()
    Dg, Do = np.array(Dg), np.array(Do)
    eD = np.max(np.abs(Dg - Do), axis=0) / np.max(np.abs(Do), axis=0)
    ex = float(np.max(np.abs(xg - sim.x)))
    say("  %s %d steps: worst capsule D error %.2e of its max D, x %.2e" % (name, steps, eD.max(), ex))
    assert eD.max() < 1e-3
    assert ex < steps * 1e-6


# ---------------------------------------------------------------------------
# observables
# ---------------------------------------------------------------------------
def test_observables_match_oracle(B):
    c = small_case(n=(40, 40, 40), m=2, level=3, r=8.0)
    rng = np.random.default_rng(2)
    A = np.eye(3) + rng.uniform(-0.15, 0.15, (3, 3))
    cen = np.array(c.wl.capsules[0].center)
    x = rep_positions(cen + (c.xref - cen) @ A.T + rng.uniform(-0.02, 0.02, c.xref.shape),
                      c.node_counts)
    lat = c.gpu()
    lat.set_mesh(x)
    obs = lat.observables()[0]
    o = c.observables(x)[0]
    for k, name in enumerate(("V", "cx", "cy", "cz", "D", "theta", "ra", "rb", "rc", "area")):
        assert obs[k] == pytest.approx(o[name], rel=1e-9, abs=1e-12), name
    lat.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_lattice_totals(B, storage):
    """FP64 mass and momentum reductions on the device (Eqs. lbmmomenta0/1
    summed over the lattice): equal to the FP64 sums of the downloaded
    populations, and to the oracle's after 1 and 24 coupled steps.  Walls and
    forces conserve mass exactly, but every stored deviation f_i - w_i is
    rounded once per step (FP32: half an ulp, 2^-24 relative; FP16: 2^-11),
    so the library's totals may drift from the oracle's by at most
    steps x 4 x that rounding x sum |f_i - w_i| (the sum over the state)."""
    c = small_case(n=(37, 21, 18), m=3, ca=0.02, perturb=0.02)
    lat = c.gpu(storage=storage, graph=True)
    f_start = lat.populations().cpu().numpy()
    sim = c.oracle(f=f_start)
    cvec, _, _ = O.lattice_constants()
    for steps in (0, 1, 23):
        lat.step(steps)
        assert sim.run(steps) == 0
        tot = lat.totals()
        f = lat.populations().cpu().numpy()
        own = np.array([f.sum()] + [np.tensordot(cvec[:, a], f, axes=(0, 0)).sum()
                                    for a in range(3)])
        ref = np.array([sim.f.sum()] + [np.tensordot(cvec[:, a], sim.f, axes=(0, 0)).sum()
                                        for a in range(3)])
        N = f[0].size
        done = sim.t
        dev = float(np.sum(np.abs(f - W19)))
        bound = done * 4 * (2.0 ** -24 if storage == "fp32" else 2.0 ** -11) * dev + 1e-12 * N
        say("  %s after %d: mass %.15g (own %.3e, oracle %.3e, bound %.3e)  momentum err %.2e"
            % (storage, done, tot[0], abs(tot[0] - own[0]), abs(tot[0] - ref[0]), bound,
               np.max(np.abs(tot[1:] - ref[1:]))))
        assert abs(tot[0] - own[0]) < 1e-13 * N
        assert np.max(np.abs(tot[1:] - own[1:])) < 1e-13 * N
        assert abs(tot[0] - ref[0]) < bound
        assert np.max(np.abs(tot[1:] - ref[1:])) < bound
    lat.close()


def test_lattice_totals_full_size(B):
    """The dense-suspension lattice (4.2 M nodes, 1024 partial sums): the
    device totals of the Couette start equal the FP64 sums of the
    downloaded populations; the momentum of the linear profile vanishes."""
    wl = W.config("c3")
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
    lat.set_shear(wl.u_w, init_profile=True)
    tot = lat.totals()
    f = lat.populations()
    own = float(f.sum())
    N = wl.nx * wl.ny * wl.nz
    lat.close()
    say("  c3 totals", tot, "own mass", own)
    assert abs(tot[0] - own) < 1e-12 * N and abs(tot[0] - N) < 1e-6 * N
    assert np.max(np.abs(tot[1:])) < 1e-9 * N


# ---------------------------------------------------------------------------
# errors
# ---------------------------------------------------------------------------
def test_stencil_touching_wall_is_rejected(B):
    c = small_case(m=4)
    lat = c.gpu()
    x = c.xref.copy()
    x[:, 2] -= x[:, 2].min() - 0.9       # lowest node at z = 0.9: its 4-point stencil reaches z = -1
    with pytest.raises(B.IBMError) as e:
        lat.set_mesh(x)
    assert e.value.code == -4
    lat.step(2)                          # the handle stays usable
    lat.synchronize()
    lat.close()


def test_collapsed_face_is_reported(B):
    """A face whose current area vanishes (two corners on top of each other)
    makes det C = 0: the step reports IBM_ERR_INVERTED_FACE at the next
    synchronising call."""
    c = small_case(m=2)
    lat = c.gpu(graph=False)
    x = c.xref.copy()
    a, b, _ = c.tri[0]
    x[b] = x[a]
    lat.set_mesh(x)
    lat.step(1)
    with pytest.raises(B.IBMError) as e:
        lat.synchronize()
    assert e.value.code == -6
    lat.close()


def test_bad_arguments(B):
    lat = B.Lattice(8, 8, 8)
    with pytest.raises(B.IBMError):
        lat.set_shear(0.5)
    with pytest.raises(B.IBMError):
        lat.step(-1)
    with pytest.raises(B.IBMError):
        lat.mesh()
    lat.step(0)
    lat.close()


def test_collide_stream_variants_agree(B):
    """Every launch variant of the collide-stream kernel computes the
    oracle's update: the per-node forms (two nodes per thread, non-temporal
    accesses, 128-thread blocks) and the row form in 256-, 128- and 64-thread
    blocks (bits 6, 7) and with cached stores (bit 8), on padded and unpadded
    rows, each for six coupled steps from the same state as the oracle."""
    for shape in ((32, 20, 16), (30, 20, 16), (27, 19, 18)):
        c = small_case(n=shape, m=3, ca=0.02)
        sim = c.oracle()
        assert sim.run(6) == 0
        for v in list(range(8)) + [16, 80, 144, 87, 151, 272, 279]:
            lat = c.gpu(graph=False)
            lat.set_option(B.OPT_LBM_VARIANT, v)
            lat.step(6)
            f = lat.populations().cpu().numpy()
            x = lat.mesh()[0].cpu().numpy()
            lat.close()
            assert rel_err(f, sim.f) < 1e-5, v
            assert np.max(np.abs(x - sim.x)) < 1e-5, v
