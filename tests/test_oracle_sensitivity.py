"""The oracle side of the sensitivity parity tests: central differences of the
Taylor deformation D with respect to the model parameters.  Pins that the
difference quotient used there is in its asymptotic range (steps h and 2h
agree far inside the 1e-3 bar), and that it sees the one derivative known
in closed form: with the linearised equilibrium the Couette profile
u_x(z) = u_w (2 z + 1 - nz) / nz is an exact steady state (Sec. IV.A), so its
derivative with respect to u_w is the profile's shape."""
import numpy as np

from oracle import oracle as O
from paper_1004_2416_amd import workloads as W


def run_D(ks, ka, uw, steps=120, n=(18, 16, 16), m=3, r=3.5):
    nx, ny, nz = n
    c = ((nx - 1) / 2 + 0.3, (ny - 1) / 2 - 0.2, (nz - 1) / 2 + 0.1)
    x, t = O.icosphere(1, r, c)
    f = np.empty((19, nz, ny, nx))
    for z in range(nz):
        f[:, z] = O.equilibrium(1.0, [uw * (2 * z + 1 - nz) / nz, 0.0, 0.0])[:, None, None]
    nf = len(t)
    sim = O.Simulation(f, x, x, t, np.full(nf, ks), np.full(nf, ka), 1.0, uw, m)
    assert sim.run(steps) == 0
    return O.capsule_observables(sim.x, t)["D"]


def central(fun, p, h):
    return (fun(p * (1 + h)) - fun(p * (1 - h))) / (2 * h * p)


def test_difference_quotient_converged():
    uw = 0.03
    ks = W.ks_from_capillary(0.05, uw, 16, 3.5)
    for fun, p in ((lambda v: run_D(v, 0.7 * v, uw), ks),
                   (lambda v: run_D(ks, v * ks, uw), 0.7),
                   (lambda v: run_D(ks, 0.7 * ks, v), uw)):
        d1, d2 = central(fun, p, 1e-4), central(fun, p, 2e-4)
        assert d1 != 0.0
        assert abs(d1 - d2) < 1e-5 * abs(d1), (d1, d2)


def test_couette_profile_derivative_is_its_shape():
    nx, ny, nz = 4, 4, 12

    def ux(uw):
        f = np.empty((19, nz, ny, nx))
        for z in range(nz):
            f[:, z] = O.equilibrium(1.0, [uw * (2 * z + 1 - nz) / nz, 0.0, 0.0],
                                    linear=True)[:, None, None]
        for _ in range(40):
            f = O.lbm_step(f, None, 0.9, uw, linear=True)
        _, u = O.velocity_field(f)
        return u[0].mean(axis=(1, 2))

    d = (ux(0.02 * (1 + 1e-4)) - ux(0.02 * (1 - 1e-4))) / (2 * 1e-4 * 0.02)
    z = np.arange(nz)
    assert np.max(np.abs(d - (2 * z + 1 - nz) / nz)) < 1e-9
