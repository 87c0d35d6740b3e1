"""Batches of independent runs (lattices of different sizes, relaxation
times, wall speeds and delta widths, with and without capsules) advanced by
one launch per kernel: every run must match its own FP64 oracle run to the
per-step parity bar, through single steps and captured graphs."""
import sys

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W
from parity_helpers import Case, O, WEIGHTS, deformed_mesh, rel_err, rep_positions, scaled_err

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


def run_case(n, m, level, r, uw, tau=1.0, ca=0.02, off=(0.3, -0.2, 0.1), capsule=True):
    nx, ny, nz = n
    caps = []
    if capsule:
        c = ((nx - 1) / 2 + off[0], (ny - 1) / 2 + off[1], (nz - 1) / 2 + off[2])
        ks = W.ks_from_capillary(ca, uw, nz, r, tau)
        caps = [W.CapsuleSpec(level, r, c, ks, 0.5 * ks)]
    return Case(W.Workload("batch", nx, ny, nz, tau, uw, m, 0, caps), perturb=0.01, seed=nx)


CASES = [dict(n=(30, 20, 16), m=3, level=2, r=4.0, uw=0.03),
         dict(n=(24, 18, 21), m=2, level=2, r=3.5, uw=0.02, tau=0.8),
         dict(n=(20, 20, 12), m=2, level=1, r=3.0, uw=0.03, capsule=False),
         dict(n=(27, 22, 24), m=4, level=3, r=5.0, uw=0.015, tau=1.3),
         dict(n=(17, 13, 14), m=3, level=1, r=3.0, uw=0.025, tau=0.7)]


class Run:
    """One member of the batch and its oracle twin."""

    def __init__(self, B, spec, ab2=False, linear=False):
        self.case = run_case(**spec)
        self.has_caps = bool(self.case.wl.capsules)
        self.lat = self.case.gpu(graph=True)
        self.lat.set_option(B.OPT_ADVECTION, int(ab2))
        self.lat.set_option(B.OPT_EQUILIBRIUM, int(linear))
        self.linear = linear
        if self.has_caps:
            self.sim = self.case.oracle(ab2=ab2, linear=linear)
        else:
            self.f = self.case.f0

    def advance_oracle(self, n):
        wl = self.case.wl
        if self.has_caps:
            assert self.sim.run(n) == 0
        else:
            for _ in range(n):
                self.f = O.lbm_step(self.f, None, wl.tau, wl.u_w, linear=self.linear)

    def errors(self):
        f_g = self.lat.populations().cpu().numpy()
        if not self.has_caps:
            return dict(f=rel_err(f_g, self.f))
        xg, Fg, ug = [a.cpu().numpy() for a in self.lat.mesh()]
        # forces of the undeformed start are zero up to the oracle's rounding
        scale = max(float(np.max(np.abs(self.sim.F))), 1e-9)
        return dict(f=rel_err(f_g, self.sim.f), F=float(np.max(np.abs(Fg - self.sim.F))) / scale,
                    u=scaled_err(ug, self.sim.un), x=float(np.max(np.abs(xg - self.sim.x))))


def check(runs, tol_x, tol_F=1e-5, tol_u=1e-5):
    """Per-run errors.  After one step from identical states the bar is 1e-5;
    over several steps the FP32 positions drift by ~1e-6 lattice spacings,
    which moves the strain-sensitive nodal forces by ~1e-4 of their scale, so
    forces get tol_F there (populations and velocities keep 1e-5; over more
    than a thousand steps the velocities, which depend on the drifted
    positions, get tol_u)."""
    for k, r in enumerate(runs):
        e = r.errors()
        say("   run", k, {q: "%.2e" % v for q, v in e.items()})
        assert e["f"] < 1e-5, k
        if r.has_caps:
            assert e["F"] < tol_F and e["u"] < tol_u, k
            assert e["x"] < tol_x, k


def test_batch_autotune_keeps_runs_on_the_oracle(B):
    """ibm_batch_autotune times real batched steps of every candidate (row
    block shape, cached-row fraction, stencil-box mode per delta width);
    afterwards every run is where its oracle is after the same number of
    steps, and the chosen settings step on in agreement with the oracle."""
    runs = [Run(B, spec) for spec in CASES]
    batch = B.Batch([r.lat for r in runs])
    chosen = batch.autotune(16)
    n = runs[0].lat.steps
    say("  batch autotune chose", chosen, "after", n, "steps")
    assert chosen["waves_per_block"] in (1, 2, 4) and chosen["cached_rows_div"] in (0, 2, 4)
    assert all(chosen["stencil_box"][m] in (0, 1, 3, 5) for m in (2, 3, 4))
    assert chosen["persistent"] in (0, 1)
    for r in runs:
        assert r.lat.steps == n
        r.advance_oracle(n)
    check(runs, 1e-3, 1e-2, 1e-4)
    batch.step(33)
    for r in runs:
        r.advance_oracle(33)
    check(runs, 1e-3, 1e-2, 1e-4)
    batch.close()
    for r in runs:
        r.lat.close()


def test_batch_persistent_launch_matches_oracle(B):
    """The batched step as one cooperative launch per step (every phase of
    every run, grid barriers between the phases): five uneven runs against
    their oracles after 1 and 40 steps, with the velocity field for some
    delta widths and LDS boxes for others (autotuner-style per-width modes are
    exercised by the autotune test)."""
    runs = [Run(B, spec) for spec in CASES]
    batch = B.Batch([r.lat for r in runs])
    batch.set_persistent(True)
    batch.step(1)
    for r in runs:
        r.advance_oracle(1)
    check(runs, 1e-6)
    batch.step(40)
    for r in runs:
        r.advance_oracle(40)
    assert all(r.lat.steps == 41 for r in runs)
    check(runs, 2e-5, 1e-3)
    batch.close()
    for r in runs:
        r.lat.close()


def test_batch_matches_oracle_per_run(B):
    """Five uneven runs: 1 plain step, then 31 steps (graphs from step 2 on,
    one re-centring), every run against its own oracle."""
    runs = [Run(B, spec) for spec in CASES]
    batch = B.Batch([r.lat for r in runs])
    say("batch: 1 step")
    batch.step(1)
    for r in runs:
        r.advance_oracle(1)
    check(runs, 1e-6)
    say("batch: 31 more steps")
    batch.step(31)
    for r in runs:
        r.advance_oracle(31)
    assert all(r.lat.steps == 32 for r in runs)
    check(runs, 2e-5, 1e-3)
    say("batch: 70 more steps (crossing re-centring)")
    batch.step(70)
    for r in runs:
        r.advance_oracle(70)
    check(runs, 1e-4, 1e-3)
    batch.close()
    for r in runs:
        r.lat.synchronize()
        r.lat.close()


def test_batch_with_long_rows(B):
    """Runs whose rows are longer than 256 nodes take the per-node lattice
    update inside the batch while the others take the row form, and every
    run's coupling and velocity-pass work items still cover all of its
    nodes: three runs against their oracles after 1 and 24 steps (graphs)."""
    specs = [dict(n=(260, 10, 12), m=3, level=1, r=3.0, uw=0.02),
             dict(n=(257, 12, 11), m=4, level=1, r=2.5, uw=0.015, tau=0.9),
             dict(n=(27, 22, 24), m=4, level=3, r=5.0, uw=0.015, tau=1.3)]
    runs = [Run(B, spec) for spec in specs]
    batch = B.Batch([r.lat for r in runs])
    batch.step(1)
    for r in runs:
        r.advance_oracle(1)
    check(runs, 1e-6)
    batch.step(24)
    for r in runs:
        r.advance_oracle(24)
    assert all(r.lat.steps == 25 for r in runs)
    check(runs, 2e-5, 1e-3)
    batch.close()
    for r in runs:
        r.lat.close()


def test_batch_oversized_and_wrapping_boxes(B):
    """Runs whose spreading boxes exceed the LDS box (a 42-node capsule of
    radius 14: the per-lane path) or span more than one period (a radius-3
    capsule on a 4 x 4 lattice: the general wrapped indices), batched with
    an ordinary run: 1 step, then 16 graph-replayed steps, each run against
    its own oracle."""
    specs = [dict(n=(40, 40, 40), m=3, level=1, r=14.0, uw=0.03),
             dict(n=(4, 4, 16), m=2, level=2, r=3.0, uw=0.02),
             CASES[0]]
    runs = [Run(B, spec) for spec in specs]
    batch = B.Batch([r.lat for r in runs])
    say("oversized and wrapping boxes: 1 step")
    batch.step(1)
    for r in runs:
        r.advance_oracle(1)
    check(runs, 1e-6)
    say("oversized and wrapping boxes: 16 more steps")
    batch.step(16)
    for r in runs:
        r.advance_oracle(16)
    check(runs, 2e-5, 1e-3)
    batch.close()
    for r in runs:
        r.lat.synchronize()
        r.lat.close()


@pytest.mark.parametrize("box", [5, 4, 2])
def test_batch_interpolation_modes(B, box):
    """The batch's coupling kernels with the first run's stencil-box mode:
    interpolation from the runs' velocity fields (4, 5, the default of
    large batches) or through LDS boxes (2), over 40 steps."""
    runs = [Run(B, spec) for spec in CASES]
    runs[0].lat.set_option(B.OPT_STENCIL_BOX, box)
    batch = B.Batch([r.lat for r in runs])
    batch.step(1)
    batch.step(39)
    for r in runs:
        r.advance_oracle(40)
    check(runs, 1e-4, 1e-3)
    batch.close()
    for r in runs:
        r.lat.close()


def test_batch_profiling_steps_are_ordinary_steps(B):
    """ibm_batch_profile_step and ibm_batch_profile_lattice_kernel advance
    every run by ordinary steps (plain launches; the second times the batched
    collide-stream from its own dispatch timestamps): interleaved with
    ordinary steps, every run still follows its oracle, and the kernel's own
    duration is positive and within the lattice phase measured around it."""
    runs = [Run(B, spec) for spec in CASES]
    batch = B.Batch([r.lat for r in runs])
    batch.step(1)
    phases = batch.profile(3)
    kms = batch.lattice_kernel_ms(3)
    batch.step(3)
    for r in runs:
        r.advance_oracle(10)
    assert all(r.lat.steps == 10 for r in runs)
    say("batch: lattice phase %.4f ms, kernel %.4f ms" % (phases["lbm"], kms))
    check(runs, 1e-4, 1e-3)
    assert 0.0 < kms < phases["lbm"] + 0.02
    batch.close()
    for r in runs:
        r.lat.close()


def test_batch_adams_bashforth_linear_equilibrium(B):
    runs = [Run(B, spec, ab2=True, linear=True) for spec in CASES[:2]]
    batch = B.Batch([r.lat for r in runs])
    batch.step(1)
    batch.step(40)
    for r in runs:
        r.advance_oracle(41)
    check(runs, 1e-4, 1e-3)
    batch.close()
    for r in runs:
        r.lat.close()


def test_batch_and_single_runs_agree(B):
    """Runs stepped alone between batch steps stay consistent, and a batch of
    one run gives the run's own result."""
    runs = [Run(B, spec) for spec in CASES[:3]]
    batch = B.Batch([r.lat for r in runs])
    batch.step(16)
    for r in runs:
        r.lat.step(2)
        r.advance_oracle(18)
    batch.step(16)
    for r in runs:
        r.advance_oracle(16)
    check(runs, 1e-4, 1e-3)
    batch.close()
    for r in runs:
        r.lat.close()


def test_batch_fp16_mass_correction_per_run(B):
    """FP16 runs in one batch keep their own IBM_OPT_FP16_MASS.  Capsule-free
    runs (walls moving, no atomics): a run with the correction, its twin
    without it, and a run of another shape without it.  After one batched
    step each run lies within one FP16 unit of its largest deviation of the
    same run stepped alone (the batch and single kernels round alike up to
    the contraction of a few operations, and FP16 storage turns such
    differences into at most a unit).  After 400 more batched steps the
    corrected run's mass stays within the rounding budget of its rest
    populations, 400 * 2^-11 sum_X |f_0 - w_0|, and drifts less than its
    uncorrected twin's."""
    specs = [dict(n=(32, 12, 16), m=2, level=1, r=3.0, uw=0.03, capsule=False)] * 2 + \
        [dict(n=(24, 20, 14), m=2, level=1, r=3.0, uw=0.02, tau=0.8, capsule=False)]
    fixes = (1, 0, 0)

    def make(spec, fix):
        lat = run_case(**spec).gpu(storage="fp16", graph=True)
        lat.set_option(B.OPT_FP16_MASS, fix)
        return lat

    batched = [make(sp, fx) for sp, fx in zip(specs, fixes)]
    alone = [make(sp, fx) for sp, fx in zip(specs, fixes)]
    m0 = [float(lat.totals()[0]) for lat in batched]
    batch = B.Batch(batched)
    batch.step(1)
    for lat in alone:
        lat.step(1)
    w = WEIGHTS[:, None, None, None]
    for k, (a, b) in enumerate(zip(batched, alone)):
        fa, fb = a.populations().cpu().numpy(), b.populations().cpu().numpy()
        dev = float(np.max(np.abs(fb - w)))
        diff = float(np.max(np.abs(fa - fb)))
        say("   fp16 run %d (correction %d), one step: max |batch - alone| %.2e, max |f - w| %.2e"
            % (k, fixes[k], diff, dev))
        assert diff <= 2.0 ** -11 * dev
    batch.step(400)
    drift = [abs(float(lat.totals()[0]) - m) for lat, m in zip(batched, m0)]
    f_end = batched[0].populations().cpu().numpy()
    budget = 400 * 2.0 ** -11 * float(np.sum(np.abs(f_end[0] - w[0])))
    say("   400 more steps: mass drift %.2e with the correction (budget %.2e), %.2e without"
        % (drift[0], budget, drift[1]))
    assert drift[0] <= budget + 1e-9 * m0[0]
    assert drift[0] < drift[1]
    batch.close()
    for lat in batched + alone:
        lat.close()


def test_batch_rejects_inconsistent_runs(B):
    runs = [Run(B, spec) for spec in CASES[:2]]
    with pytest.raises(B.IBMError):
        B.Batch([runs[0].lat, runs[0].lat])
    batch = B.Batch([r.lat for r in runs])
    runs[0].lat.step(1)
    with pytest.raises(B.IBMError) as e:
        batch.step(1)
    assert e.value.code == -2
    runs[1].lat.step(1)
    batch.step(2)
    batch.close()
    half = B.Lattice(10, 10, 10, storage="fp16")
    with pytest.raises(B.IBMError):
        B.Batch([runs[0].lat, half])
    half.close()
    for r in runs:
        r.lat.close()


def test_full_size_batched_sweep(B):
    """The 64-run sweep at its full sizes (6.67 M lattice nodes, 78 k membrane
    nodes, delta widths 2-4) in the launch configuration the benchmark times:
    one batch with its default stencil-box mode (box spreading, interpolation
    from the velocity field), cached stores for the first quarter of each
    run's rows, 16-step graphs.  Every capsule is deformed by ~2 % and
    injected.  After one step every run's populations, forces, node
    velocities and positions meet the per-step bar against its own oracle.
    After 16 more (one graph) the populations and positions are compared
    along the trajectory (positions within one FP32 rounding per step); then
    each run's state is handed to a fresh oracle and the next step is held to
    the per-step bar again.  (Forces and node velocities are not compared
    along the trajectory: the fine meshes' forces move by ~1e-4 of their
    scale per FP32 rounding of a node position.)"""
    wls = W.sweep_workloads()
    say("full-size sweep: %d runs, %d lattice nodes" % (len(wls), sum(w.n_nodes_lattice for w in wls)))
    cases = [Case(wl) for wl in wls]
    lats, sims = [], []
    for k, c in enumerate(cases):
        lat = c.gpu(graph=True)
        x_s = deformed_mesh(c, 0.02, 300 + k)
        lat.set_mesh(x_s)
        lats.append(lat)
        sims.append(c.oracle(x=x_s))
    batch = B.Batch(lats)

    def compare(sims, steps, per_step, since_start=0):
        worst = dict(f=0.0, F=0.0, u=0.0, x=0.0)
        for k, (lat, sim) in enumerate(zip(lats, sims)):
            assert sim.run(steps) == 0
            xg, Fg, ug = [a.cpu().numpy() for a in lat.mesh()]
            e = dict(f=rel_err(lat.populations().cpu().numpy(), sim.f),
                     x=float(np.max(np.abs(xg - sim.x))),
                     F=scaled_err(Fg, sim.F) if per_step else 0.0,
                     u=scaled_err(ug, sim.un) if per_step else 0.0)
            worst = {q: max(worst[q], e[q]) for q in worst}
            assert e["f"] < 1e-5, (k, e)
            if per_step:
                assert e["F"] < 1e-5 and e["u"] < 1e-5 and e["x"] < 2e-6, (k, e)
            else:
                assert e["x"] < since_start * 1e-6, (k, e)
        say("   %d step(s), worst run:" % steps, {q: "%.2e" % v for q, v in worst.items()})

    batch.step(1)
    compare(sims, 1, True)
    batch.step(16)
    compare(sims, 16, False, since_start=17)
    state = [(lat.populations().cpu().numpy(), lat.mesh()[0].cpu().numpy()) for lat in lats]
    sims = [c.oracle(f=f, x=x) for c, (f, x) in zip(cases, state)]
    del state
    batch.step(1)
    compare(sims, 1, True)
    assert all(lat.steps == 18 for lat in lats)
    batch.close()
    for lat in lats:
        lat.synchronize()
        lat.close()
