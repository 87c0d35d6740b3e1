"""Forward sensitivities (tangent-linear model) of the timestep against central
finite differences of the FP64 oracle.

The parameters are the Skalak shear modulus k_s at fixed C = k_alpha / k_s,
the ratio C at fixed k_s, and the shear rate gamma = 2 u_w / nz, which enters
through the wall speed and the linear Couette start (Sec. II.A, Sec. III).
The oracle side is (D(p (1 + h)) - D(p (1 - h))) / (2 h p) from two full FP64
runs; the bar is 1e-3 of the derivative (the difference quotient itself is
good to ~1e-6 here, see the CPU test of its convergence)."""
import sys

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W
from parity_helpers import Case, O, couette_populations, rep_positions, scaled_err

pytestmark = pytest.mark.gpu

H_FD = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1004_2416_amd import binding
    return binding


def tangent_case(m=3):
    n, uw, r = (28, 24, 24), 0.02, 5.0
    ks = W.ks_from_capillary(0.05, uw, n[2], r)
    c = ((n[0] - 1) / 2 + 0.3, (n[1] - 1) / 2 - 0.2, (n[2] - 1) / 2 + 0.1)
    return Case(W.Workload("tangent", *n, 1.0, uw, m, 0, [W.CapsuleSpec(2, r, c, ks, 0.7 * ks)]))


def rates(c, which):
    """(dks, dka, duw) per unit of the parameter."""
    ks, ka, nz = c.ks[0], c.ka[0], c.wl.nz
    C = ka / ks
    if which == "ks":
        return np.array([1.0]), np.array([C]), 0.0
    if which == "C":
        return np.array([0.0]), np.array([ks]), 0.0
    return np.array([0.0]), np.array([0.0]), nz / 2.0   # gamma


def param_value(c, which):
    if which == "ks":
        return c.ks[0]
    if which == "C":
        return c.ka[0] / c.ks[0]
    return 2.0 * c.wl.u_w / c.wl.nz


def oracle_D(c, which, scale, steps):
    """D after `steps` oracle steps with the parameter multiplied by `scale`,
    from the exact FP64 Couette start and the undeformed capsule."""
    ks, ka, uw = c.ks_face.copy(), c.ka_face.copy(), c.wl.u_w
    if which == "ks":
        ks, ka = ks * scale, ka * scale
    elif which == "C":
        ka = ka * scale
    else:
        uw = uw * scale
    f0 = couette_populations(c.wl.nz, c.wl.ny, c.wl.nx, uw)
    sim = O.Simulation(f0, c.xref, c.xref, c.tri, ks, ka, c.wl.tau, uw, c.wl.m)
    assert sim.run(steps) == 0
    return c.observables(sim.x)[0]["D"], sim


@pytest.mark.parametrize("which", ["ks", "C", "gamma"])
def test_tangent_shape_derivative(B, which):
    """dD/dp after 300 steps (kappa t ~ 10) from the undeformed capsule in the
    linear Couette start: tangent model vs oracle central differences."""
    steps = 300
    c = tangent_case()
    p = param_value(c, which)
    d_plus, _ = oracle_D(c, which, 1 + H_FD, steps)
    d_minus, _ = oracle_D(c, which, 1 - H_FD, steps)
    fd = (d_plus - d_minus) / (2 * H_FD * p)
    lat = B.Lattice(c.wl.nx, c.wl.ny, c.wl.nz, c.wl.tau)
    lat.set_shear(c.wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, c.wl.m)
    dks, dka, duw = rates(c, which)
    lat.attach_tangent(dks, dka, duw, init_profile=(which == "gamma"))
    lat.step(steps)
    dobs = lat.tangent_observables(1e-6 * p)
    D = lat.observables()[0, 4]
    lat.close()
    say("  d D / d %s: tangent %.8e  oracle FD %.8e  (D = %.5f)" % (which, dobs[0, 4], fd, D))
    assert abs(dobs[0, 4] - fd) < 1e-3 * abs(fd)


def test_tangent_c5_workload(B):
    """The 64^3 single-capsule workload (r = 8, 1280 faces, 3-point delta,
    Ca = 0.05) for 500 steps: the three derivatives of D by the tangent model
    (one pass each) and by the adjoint (one reverse sweep), against oracle
    central differences at full size (six FP64 runs)."""
    steps = 500
    wl = W.config("c5")
    c = Case(wl)
    fds = {}
    for which in ("ks", "C", "gamma"):
        p = param_value(c, which)
        fd = (oracle_D(c, which, 1 + H_FD, steps)[0] - oracle_D(c, which, 1 - H_FD, steps)[0]) \
            / (2 * H_FD * p)
        lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
        lat.set_shear(wl.u_w, init_profile=True)
        lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
        dks, dka, duw = rates(c, which)
        lat.attach_tangent(dks, dka, duw, init_profile=(which == "gamma"))
        lat.step(steps)
        got = lat.tangent_observables(1e-6 * p)[0, 4]
        lat.close()
        say("  c5 d D / d %s: tangent %.8e  oracle FD %.8e" % (which, got, fd))
        assert abs(got - fd) < 1e-3 * abs(fd)
        fds[which] = fd
    # the reverse sweep gives all three at once
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules(c.meshes(), c.ks, c.ka, wl.m)
    g = lat.adjoint_gradient(steps, checkpoint_every=100, couette_start=True)
    lat.close()
    C = c.ka[0] / c.ks[0]
    adj = {"ks": g["dks"][0] + C * g["dka"][0], "C": c.ks[0] * g["dka"][0],
           "gamma": 0.5 * wl.nz * g["duw"]}
    for which, fd in fds.items():
        say("  c5 d D / d %s: adjoint %.8e" % (which, adj[which]))
        assert abs(adj[which] - fd) < 1e-3 * abs(fd)


def test_tangent_one_step_fields(B):
    """One step from a deformed injected state, direction k_s: tangent
    populations and node velocities against central differences of one
    oracle step (the injected state does not depend on k_s)."""
    c = tangent_case(m=4)
    sim = c.oracle()
    assert sim.run(30) == 0
    f_s = sim.f.copy()
    x_s = rep_positions(sim.x, c.node_counts)
    outs = []
    for s in (1 + H_FD, 1 - H_FD):
        o = O.Simulation(f_s, x_s, c.xref, c.tri, c.ks_face * s, c.ka_face * s, c.wl.tau,
                         c.wl.u_w, c.wl.m)
        assert o.run(1) == 0
        outs.append(o)
    p = c.ks[0]
    dfd = (outs[0].f - outs[1].f) / (2 * H_FD * p)
    dufd = (outs[0].un - outs[1].un) / (2 * H_FD * p)
    lat = c.gpu(graph=False)
    lat.set_populations(f_s)
    lat.set_mesh(x_s)
    dks, dka, _ = rates(c, "ks")
    lat.attach_tangent(dks, dka, 0.0)
    lat.step(1)
    tf = lat.tangent_populations().cpu().numpy()
    dx, du = [a.cpu().numpy() for a in lat.tangent_mesh()]
    lat.close()
    ef, eu = scaled_err(tf, dfd), scaled_err(du, dufd)
    say("  one-step tangent errors: pops %.2e  node velocities %.2e  (|dF scale| %.2e)"
        % (ef, eu, np.max(np.abs(dfd))))
    assert ef < 1e-3
    assert eu < 1e-3
    assert np.max(np.abs(dx - du)) == 0.0   # Euler: dx(1) = 0 + du


def test_tangent_rejected_combinations(B):
    c = tangent_case()
    half = B.Lattice(12, 12, 12, storage="fp16")
    with pytest.raises(B.IBMError):
        half.attach_tangent(duw=1.0)
    half.close()
    lat = c.gpu(graph=True)
    lat.attach_tangent([1.0], [0.7], 0.0)
    lat.set_option(B.OPT_ADVECTION, 1)
    with pytest.raises(B.IBMError):
        lat.step(1)
    lat.set_option(B.OPT_ADVECTION, 0)
    lat.step(2)
    with pytest.raises(B.IBMError):
        B.Batch([lat])
    lat.detach_tangent()
    lat.step(2)
    lat.close()
