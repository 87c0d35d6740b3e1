"""Accuracy of half-precision population storage against the FP64 oracle.

The library can keep each population as the FP16 number (f_i - w_i) 16/w_i
while computing in FP32.  Rounding that number to FP16 costs at most half an
ulp, 2^-11 of its value, so one step adds an error of at most 2^-11 max|f_i - w_i|
to any population; everything else in the step is the FP32 path.  The tests
state that error per result (populations, force density, node velocities,
positions, the Taylor deformation D(t) of a whole run, total mass) and bound
it."""
import sys

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W
from parity_helpers import Case, O, WEIGHTS, deformed_mesh, rep_positions, scaled_err

pytestmark = pytest.mark.gpu

HALF_ULP = 2.0 ** -11


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1004_2416_amd import binding
    return binding


def rep16(f):
    """What the FP16 store of f holds, as the library reports it:
    w + fp16(fp32(f - w) * s) / s with s = 16 / w (48, 288, 576: exact), where
    the product fp32(f - w) * s is rounded once, directly to FP16 (the
    kernels form it with a mixed-precision fused multiply-add), and the
    division is exact in FP64."""
    w = WEIGHTS[:, None, None, None]
    s = (16.0 / WEIGHTS).astype(np.float32)[:, None, None, None]
    exact = np.asarray(f - w, np.float32).astype(np.float64) * s.astype(np.float64)
    h = exact.astype(np.float16)
    return w + h.astype(np.float64) / s.astype(np.float64)


def dev_err(f_gpu, f_ref):
    """max |f_gpu - f_ref| over max |f_ref - w|: the error in units of the
    largest deviation from rest, which is what FP16 storage resolves."""
    w = WEIGHTS[:, None, None, None]
    return float(np.max(np.abs(f_gpu - f_ref)) / np.max(np.abs(f_ref - w)))


def u_bound(f_ref, u_ref):
    """Largest velocity error that FP16 rounding of the new populations can
    cause: |du| <= sum_i |c_i| |df_i| / rho <= 18 * 2^-11 max|f - w| (rho
    within 10 % of 1), plus the FP32 path's 1e-5 of max|u|."""
    w = WEIGHTS[:, None, None, None]
    return 1.1 * 18 * HALF_ULP * float(np.max(np.abs(f_ref - w))) + 1e-5 * float(np.max(np.abs(u_ref)))


def small_case(m=3, level=2, r=4.0, ca=0.02, uw=0.03, n=(30, 20, 16)):
    nx, ny, nz = n
    c = ((nx - 1) / 2 + 0.3, (ny - 1) / 2 - 0.2, (nz - 1) / 2 + 0.1)
    ks = W.ks_from_capillary(ca, uw, nz, r)
    return Case(W.Workload("small16", nx, ny, nz, 1.0, uw, m, 0,
                           [W.CapsuleSpec(level, r, c, ks, ks)]))


def test_fp16_store_is_the_stated_rounding(B):
    """set_populations followed by get_fields returns exactly rep16(f)."""
    c = small_case()
    sim = c.oracle()
    assert sim.run(20) == 0
    lat = c.gpu(storage="fp16", graph=False)
    lat.set_populations(sim.f)
    got = lat.populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, rep16(sim.f)), float(np.max(np.abs(got - rep16(sim.f))))


@pytest.mark.parametrize("m,n", [(2, (30, 20, 16)), (4, (30, 20, 16)), (3, (32, 20, 16))])
def test_fp16_one_step_error(B, m, n):
    """One coupled step from an identical (FP16-representable) deformed
    state: populations within 2^-11 (+ FP32 slack) of the largest
    deviation, force density as in FP32, node velocities and positions
    within the error the rounded populations carry.  nx = 30 runs the row
    form over padded rows, nx = 32 over unpadded ones."""
    c = small_case(m=m, n=n)
    sim = c.oracle()
    assert sim.run(40) == 0
    f_s = rep16(sim.f)
    x_s = rep_positions(sim.x, c.node_counts)
    lat = c.gpu(storage="fp16", graph=False)
    lat.set_populations(f_s)
    lat.set_mesh(x_s)
    lat.step(1)
    ref = c.oracle(f=f_s, x=x_s)
    assert ref.run(1) == 0
    f_g = lat.populations().cpu().numpy()
    xg, Fg, ug = [a.cpu().numpy() for a in lat.mesh()]
    g_g = lat.force_density().cpu().numpy()
    lat.close()
    errs = dict(f_dev=dev_err(f_g, ref.f), F=scaled_err(Fg, ref.F), g=scaled_err(g_g, ref.g),
                u_abs=float(np.max(np.abs(ug - ref.un))), x=float(np.max(np.abs(xg - ref.x))))
    ub = u_bound(ref.f, ref.un)
    say("  fp16 one-step errors m=%d" % m, {k: "%.2e" % v for k, v in errs.items()},
        "u bound %.2e" % ub)
    assert errs["f_dev"] < 1.05 * HALF_ULP
    assert errs["F"] < 1e-5 and errs["g"] < 1e-5
    assert errs["u_abs"] < ub
    assert errs["x"] < ub + 1e-6


def test_fp16_trajectory_c1(B):
    """The 32^3 single-capsule workload (r = 6, 1280 faces, 3-point delta,
    Ca = 0.05) for its full 1000 steps with FP16 storage: D(t) within 1 % of
    its maximum, node positions within 1e-2 lattice spacings, populations
    within 1e-2 of the largest deviation, mass within 1e-6."""
    c = Case(W.config("c1"))
    lat = c.gpu(storage="fp16", graph=True)
    sim = c.oracle()
    Dg, Do = [], []
    m0 = float(np.sum(rep16(c.f0)))
    for k in range(20):
        lat.step(50)
        assert sim.run(50) == 0
        Dg.append(lat.observables()[0, 4])
        Do.append(c.observables(sim.x)[0]["D"])
    Dg, Do = np.array(Dg), np.array(Do)
    xg = lat.mesh()[0].cpu().numpy()
    f_g = lat.populations().cpu().numpy()
    # the mass from the library's own FP64 reduction on the device, which
    # must also agree with the sum of the downloaded populations
    mass = float(lat.totals()[0])
    lat.close()
    assert abs(mass - float(np.sum(f_g))) < 1e-10 * m0
    eD = float(np.max(np.abs(Dg - Do)) / np.max(np.abs(Do)))
    ex = float(np.max(np.abs(xg - sim.x)))
    ef = dev_err(f_g, sim.f)
    em = abs(mass - m0) / m0
    say("  fp16 c1 1000 steps: D %.2e (D_end %.4f vs %.4f)  x %.2e  f_dev %.2e  mass %.2e"
        % (eD, Dg[-1], Do[-1], ex, ef, em))
    assert eD < 1e-2
    assert ex < 1e-2
    assert ef < 1e-2
    assert em < 1e-6


def test_fp16_full_size_step(B):
    """The 128^3 workload (one 2562-node capsule, 4-point delta) stored in
    FP16 at full size: one step from a deformed FP16-representable state."""
    wl = W.config("c2")
    c = Case(wl)
    from paper_1004_2416_amd import binding as Bm
    lat = Bm.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, storage="fp16")
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    x_s = deformed_mesh(c, 0.02, 11)
    lat.set_mesh(x_s)
    f_s = rep16(c.f0)
    lat.set_populations(f_s)
    lat.step(1)
    sim = c.oracle(f=f_s, x=x_s)
    assert sim.run(1) == 0
    f_g = lat.populations().cpu().numpy()
    xg, Fg, ug = [a.cpu().numpy() for a in lat.mesh()]
    g_g = lat.force_density().cpu().numpy()
    lat.close()
    errs = dict(f_dev=dev_err(f_g, sim.f), F=scaled_err(Fg, sim.F), g=scaled_err(g_g, sim.g),
                u_abs=float(np.max(np.abs(ug - sim.un))))
    ub = u_bound(sim.f, sim.un)
    say("  fp16 c2 one-step errors", {k: "%.2e" % v for k, v in errs.items()}, "u bound %.2e" % ub)
    assert errs["f_dev"] < 1.05 * HALF_ULP
    assert errs["F"] < 1e-5 and errs["g"] < 1e-5
    assert errs["u_abs"] < ub


def collide_stream_form(variant, nx):
    """The collide-stream form the library runs with FP16 storage for this
    IBM_OPT_LBM_VARIANT and row length (rows padded to a multiple of 4)."""
    return "rows4" if (variant & 16) and (nx + 3) // 4 <= 64 else "nodes"


def test_fp16_collide_stream_forms_agree(B):
    """The FP16 collide-stream forms on rows of 3 to 512 nodes (padded rows
    of 4 to 256 values run the row form: one lane per row up to a whole
    wavefront), with and without a capsule's forces, with wall bounce-back.  Each form's first step from an FP16-representable
    state is within 2^-11 of the largest deviation from the FP64 oracle's.
    The forms evaluate the same FP32 expressions, but the compiler may
    contract a product into a sum differently in each, and with a capsule
    the spreading's FP32 atomics sum in a varying order; a last-bit FP32
    difference can then round to the neighbouring FP16 value, so after five
    steps the forms agree within one FP16 ulp (2^-10) of the largest
    deviation."""
    forms = (23, 7, 0, 87, 151, 279)
    shapes = [((32, 20, 16), True), ((30, 20, 16), True), ((64, 12, 10), False),
              ((8, 6, 5), False), ((16, 10, 9), False), ((256, 6, 4), False),
              ((512, 4, 3), False), ((21, 9, 7), False), ((253, 4, 3), False),
              ((6, 5, 4), False), ((3, 4, 3), False)]
    for n, with_capsule in shapes:
        if with_capsule:
            c = small_case(n=n)
        else:
            c = Case(W.Workload("rows16", *n, 1.0, 0.03, 3, 0, []), perturb=0.01, seed=n[0])
            f_s = rep16(c.f0)
            one = O.lbm_step(f_s, None, c.wl.tau, c.wl.u_w)
        ref = None
        for v in forms:
            lat = c.gpu(storage="fp16", graph=False)
            lat.set_option(B.OPT_LBM_VARIANT, v)
            if not with_capsule:
                lat.set_populations(f_s)
                lat.step(1)
                e1 = dev_err(lat.populations().cpu().numpy(), one)
                assert e1 < 1.05 * HALF_ULP, (n, v, e1)
            lat.step(5)
            f = lat.populations().cpu().numpy()
            x = lat.mesh()[0].cpu().numpy() if with_capsule else None
            lat.close()
            form = collide_stream_form(v, n[0])
            if ref is None:
                ref = (f, x, form)
                continue
            e = dev_err(f, ref[0])
            say("  fp16 forms n=%s variant %d (%s vs %s): max |df| / max |f - w| %.2e"
                % (n, v, form, ref[2], e))
            assert e <= 2 * HALF_ULP, (n, v)
            if with_capsule:
                assert np.max(np.abs(x - ref[1])) < 1e-6, (n, v)
    lat = c.gpu(storage="fp16", graph=False)
    lat.set_option(B.OPT_LBM_VARIANT, 511)
    with pytest.raises(B.IBMError):
        lat.set_option(B.OPT_LBM_VARIANT, 512)
    lat.close()


def test_fp16_mass_correction(B):
    """IBM_OPT_FP16_MASS: the rest population takes back the mass the node's
    18 moving values lose to FP16 rounding.  One lattice step (walls moving,
    no capsule: deterministic) from an FP16-representable state: the moving
    populations are stored exactly as without the correction; the rest
    population is off the FP64 step by at most the node's rounding budget
    2^-11 sum_i |f_i - w_i|; the total mass is the FP32 step's, up to the
    rounding of the rest populations.  Then 2000 steps: the mass drifts by
    less than steps * 2^-11 * sum_X |f_0 - w_0|, the worst case of that
    rounding, while without the correction it drifts by more."""
    c = Case(W.Workload("mass16", 32, 12, 16, 1.0, 0.03, 2, 0, []), perturb=0.01, seed=7)
    f_s = rep16(c.f0)
    one = O.lbm_step(f_s, None, c.wl.tau, c.wl.u_w)
    w = WEIGHTS[:, None, None, None]
    res, mass = {}, {}
    for fix in (0, 1):
        lat = c.gpu(storage="fp16", graph=False)
        lat.set_option(B.OPT_FP16_MASS, fix)
        lat.set_populations(f_s)
        lat.step(1)
        res[fix] = lat.populations().cpu().numpy()
        lat.set_option(B.OPT_GRAPH, 1)
        lat.step(2000)
        mass[fix] = float(lat.totals()[0])
        f_end = lat.populations().cpu().numpy()
        lat.close()
    assert np.array_equal(res[0][1:], res[1][1:])
    budget = 2.0 ** -11 * np.sum(np.abs(one - w), axis=0)
    assert np.all(np.abs(res[1][0] - one[0]) <= 1.05 * budget + 1e-9)
    m0 = float(np.sum(f_s))
    m_rest = 2.0 ** -11 * float(np.sum(np.abs(one[0] - w[0])))
    e0, e1 = abs(res[0].sum() - one.sum()), abs(res[1].sum() - one.sum())
    say("  fp16 mass, one step: error %.2e without, %.2e with the correction (rest rounding %.2e)"
        % (e0, e1, m_rest))
    assert e1 <= 1.05 * m_rest + 1e-9 * m0
    drift0, drift1 = abs(mass[0] - m0) / m0, abs(mass[1] - m0) / m0
    bound = 2000 * 2.0 ** -11 * float(np.sum(np.abs(f_end[0] - w[0]))) / m0
    say("  fp16 mass, 2000 steps: drift %.2e without, %.2e with the correction (bound %.2e)"
        % (drift0, drift1, bound))
    assert drift1 < bound + 1e-9
    assert drift1 < drift0


def test_fp16_mass_correction_coupled_and_aa(B):
    """The correction with a capsule (forces in the collision), on a two-buffer
    lattice and on a one-buffer (AA) lattice: 100 steps against the oracle
    within the FP16 bars, mass drift within the rest populations' rounding
    budget."""
    c = small_case(m=3, n=(32, 20, 16))
    wl = c.wl
    w = WEIGHTS[:, None, None, None]
    for one_buffer in (False, True):
        lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, storage="fp16", one_buffer=one_buffer)
        lat.set_shear(wl.u_w, init_profile=False)
        lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
        lat.set_option(B.OPT_FP16_MASS, 1)
        lat.set_populations(c.f0)
        f0 = lat.populations().cpu().numpy()
        sim = c.oracle(f=f0)
        lat.step(1)
        lat.step(99)
        assert sim.run(100) == 0
        f = lat.populations().cpu().numpy()
        xg = lat.mesh()[0].cpu().numpy()
        mass = float(lat.totals()[0])
        lat.close()
        m0 = float(np.sum(f0))
        bound = 100 * 2.0 ** -11 * float(np.sum(np.abs(f[0] - w[0]))) / m0
        ef, ex = dev_err(f, sim.f), float(np.max(np.abs(xg - sim.x)))
        say("  fp16 mass correction, capsule, one buffer %s: f_dev %.2e  x %.2e  mass drift %.2e"
            " (bound %.2e)" % (one_buffer, ef, ex, abs(mass - m0) / m0, bound))
        assert ef < 100 * HALF_ULP and ex < 1e-3
        assert abs(mass - m0) / m0 < bound + 1e-9
    lat = Case(W.Workload("wide", 300, 4, 4, 1.0, 0.01, 2, 0, [])).gpu(storage="fp16", graph=False)
    with pytest.raises(B.IBMError):
        lat.set_option(B.OPT_FP16_MASS, 1)  # nx > 256: no row form
    lat.close()
    lat = c.gpu(storage="fp32", graph=False)
    with pytest.raises(B.IBMError):
        lat.set_option(B.OPT_FP16_MASS, 1)
    lat.close()
