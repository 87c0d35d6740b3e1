"""Pins of the oracle's lattice Boltzmann part (Sec. II.A) against what the
paper and the mathematics fix: the velocity set drawn in Fig. 1, the isotropy
the cited weights must give, the moments of the equilibrium and of the Guo
term, exact conservation, a closed-form forced start-up, pure streaming and
the Couette profile between the moving walls."""
import os

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_velocity_set_matches_fig1(orc):
    """Fig. 1 draws c_i as the arrow from v0 to v_i with v_i = 2 c_i in its
    TikZ coordinates (transcribed in golden/d3q19_fig1.txt)."""
    c, w, opp = orc.lattice_constants()
    gold = np.loadtxt(os.path.join(GOLDEN, "d3q19_fig1.txt"), dtype=int, comments="#")
    assert gold.shape == (19, 4)
    assert np.array_equal(gold[:, 0], np.arange(19))
    assert np.array_equal(c, gold[:, 1:] // 2)
    # caption: c_1..c_6 reach the next neighbours along the axes, c_7..c_18
    # the next-but-one neighbours; every vector lies in a coordinate plane
    n2 = (c * c).sum(1)
    assert n2[0] == 0 and np.all(n2[1:7] == 1) and np.all(n2[7:] == 2)
    assert np.all((c == 0).sum(1) >= 1)
    for i in range(1, 19):
        assert np.array_equal(c[opp[i]], -c[i])
        assert opp[i] == (i + 1 if i % 2 == 1 else i - 1)
    assert opp[0] == 0


def test_weights_isotropy(orc):
    """The D3Q19 weights must make the lattice moments isotropic up to fourth
    order: sum w = 1, sum w c = 0, sum w c_a c_b = d_ab/3,
    sum w c_a c_b c_c c_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9."""
    c, w, _ = orc.lattice_constants()
    c = c.astype(float)
    d = np.eye(3)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(w @ c, 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(orc, seed):
    """sum feq = rho, sum c feq = rho u, sum c c feq = rho (I/3 + u u)."""
    c, _, _ = orc.lattice_constants()
    c = c.astype(float)
    rng = np.random.default_rng(seed)
    rho = 1 + rng.uniform(-0.05, 0.05)
    u = rng.uniform(-0.05, 0.05, 3)
    feq = orc.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-14
    assert np.allclose(feq @ c, rho * u, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", feq, c, c),
                       rho * (np.eye(3) / 3 + np.outer(u, u)), atol=1e-15)
    lin = orc.equilibrium(rho, u, linear=True)
    assert abs(lin.sum() - rho) < 1e-14
    assert np.allclose(lin @ c, rho * u, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", lin, c, c), rho * np.eye(3) / 3, atol=1e-15)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_guo_moments(orc, tau):
    """Guo's term adds no mass, the momentum (1 - 1/(2 tau)) f and the second
    moment (1 - 1/(2 tau)) (u f + f u)."""
    c, _, _ = orc.lattice_constants()
    c = c.astype(float)
    rng = np.random.default_rng(7)
    u = rng.uniform(-0.05, 0.05, 3)
    g = rng.uniform(-1e-3, 1e-3, 3)
    S = orc.guo_source(tau, u, g)
    pre = 1 - 1 / (2 * tau)
    assert abs(S.sum()) < 1e-18
    assert np.allclose(S @ c, pre * g, rtol=1e-13, atol=1e-19)
    assert np.allclose(np.einsum("i,ia,ib->ab", S, c, c),
                       pre * (np.outer(u, g) + np.outer(g, u)), atol=1e-18)


def _eq_field(orc, rho, u):
    """f = feq(rho(X), u(X)) node by node. rho: [nz,ny,nx]; u: [3,nz,ny,nx]."""
    nz, ny, nx = rho.shape
    f = np.empty((19, nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                f[:, z, y, x] = orc.equilibrium(rho[z, y, x], u[:, z, y, x])
    return f


def test_rest_state_is_fixed_point(orc):
    _, w, _ = orc.lattice_constants()
    f = np.broadcast_to(1.03 * w[:, None, None, None], (19, 5, 4, 6)).copy()
    out = f
    for _ in range(3):
        out = orc.lbm_step(out, None, 1.0, 0.0)
    assert np.max(np.abs(out - f)) < 1e-15


def test_pure_streaming_and_wall_reflection(orc):
    """With tau -> infinity the collision does nothing and the update is pure
    streaming f_i(x + c_i, t + 1) = f_i(x, t), periodic in x and y; a
    population leaving through a resting wall comes back reversed."""
    c, w, opp = orc.lattice_constants()
    nz, ny, nx = 6, 5, 7
    f = np.broadcast_to(w[:, None, None, None], (19, nz, ny, nx)) * (
        1 + W.noise((19, nz, ny, nx), 0.1, 3))
    out = orc.lbm_step(f, None, 1e12, 0.0)
    for i in range(19):
        cx, cy, cz = c[i]
        moved = np.roll(np.roll(f[i], cx, axis=2), cy, axis=1)
        if cz == 0:
            assert np.allclose(out[i], moved, atol=1e-11)
        elif cz == 1:
            assert np.allclose(out[i][1:], moved[:-1], atol=1e-11)
            # arrivals at the bottom layer came from the wall: reversed opp(i)
            assert np.allclose(out[i][0], f[opp[i]][0], atol=1e-11)
        else:
            assert np.allclose(out[i][:-1], moved[1:], atol=1e-11)
            assert np.allclose(out[i][-1], f[opp[i]][-1], atol=1e-11)


@pytest.mark.parametrize("linear", [False, True])
def test_mass_conserved_with_moving_walls_and_force(orc, linear):
    _, w, _ = orc.lattice_constants()
    nz, ny, nx = 7, 6, 5
    f = np.broadcast_to(w[:, None, None, None], (19, nz, ny, nx)) * (
        1 + W.noise((19, nz, ny, nx), 0.05, 11))
    g = W.noise((3, nz, ny, nx), 1e-3, 12)
    m0 = f.sum()
    out = f
    for _ in range(5):
        out = orc.lbm_step(out, g, 0.8, 0.05, linear=linear)
    assert abs(out.sum() - m0) / m0 < 1e-14


def test_forced_startup_closed_form(orc):
    """From rest under a uniform body force g0, far from the walls the
    momentum density grows exactly as rho u(t) = (t + 1/2) g0 with rho = 1:
    the half-force velocity of Eq. (lbmmomenta1) plus Guo's momentum input."""
    c, w, _ = orc.lattice_constants()
    nz, ny, nx = 21, 4, 3
    g0 = np.array([1e-5, 2e-5, -1.5e-5])
    f = np.broadcast_to(w[:, None, None, None], (19, nz, ny, nx)).copy()
    g = np.broadcast_to(g0[:, None, None, None], (3, nz, ny, nx)).copy()
    for t in range(1, 9):
        f = orc.lbm_step(f, g, 1.0, 0.0)
        rho, u = orc.velocity_field(f, g)
        zc = nz // 2
        assert abs(rho[zc, 0, 0] - 1) < 1e-14
        assert np.allclose(rho[zc, 0, 0] * u[:, zc, 0, 0], (t + 0.5) * g0, rtol=1e-10)


def _couette(nz, uw):
    z = np.arange(nz)
    return uw * (2 * z + 1 - nz) / nz


def test_couette_linearised_equilibrium_is_exact(orc):
    """With the linearised equilibrium the linear shear profile between walls
    at z = -1/2 and nz - 1/2 moving with -+u_w is an exact steady state."""
    nz, ny, nx, uw = 12, 3, 4, 0.02
    ux = _couette(nz, uw)
    u = np.zeros((3, nz, ny, nx))
    u[0] = ux[:, None, None]
    f = _eq_field(orc, np.ones((nz, ny, nx)), u)
    out = f
    for _ in range(100):
        out = orc.lbm_step(out, None, 1.0, uw, linear=True)
    rho, v = orc.velocity_field(out)
    assert np.max(np.abs(v[0] - u[0])) < 1e-14
    assert np.max(np.abs(v[1:])) < 1e-15
    assert np.max(np.abs(rho - 1)) < 1e-14


@pytest.mark.parametrize("linear", [False, True])
def test_couette_from_rest_converges_to_linear_profile(orc, linear):
    """Whatever the start, the flow between the moving walls relaxes to the
    linear profile u_x(z) = u_w (2 z + 1 - nz)/nz, gamma_dot = 2 u_w / nz
    (Sec. II.A): fixes wall position, speed and direction."""
    nz, ny, nx, uw = 8, 2, 3, 0.01
    _, w, _ = orc.lattice_constants()
    f = np.broadcast_to(w[:, None, None, None], (19, nz, ny, nx)).copy()
    for _ in range(3000):
        f = orc.lbm_step(f, None, 1.0, uw, linear=linear)
    rho, v = orc.velocity_field(f)
    prof = v[0].mean(axis=(1, 2))
    assert np.max(np.abs(prof - _couette(nz, uw))) < 1e-3 * uw
    assert np.max(np.abs(v[1:])) < 1e-10


def test_velocity_field_half_force(orc):
    """rho u = sum_i c_i f_i + f/2 (Eq. lbmmomenta1, Delta t = 1)."""
    nz, ny, nx = 3, 2, 4
    rng = np.random.default_rng(5)
    rho0 = 1 + rng.uniform(-0.02, 0.02, (nz, ny, nx))
    ub = rng.uniform(-0.03, 0.03, (3, nz, ny, nx))
    g = rng.uniform(-1e-3, 1e-3, (3, nz, ny, nx))
    f = _eq_field(orc, rho0, ub)
    rho, u = orc.velocity_field(f, g)
    assert np.allclose(rho, rho0, atol=1e-15)
    assert np.allclose(u, ub + g / (2 * rho0), atol=1e-16)
