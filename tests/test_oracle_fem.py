"""Pins of the oracle's membrane model (Sec. II.B): Skalak's energy against
closed forms for homogeneous stretches, the virtual-work forces against
finite differences of the energy, invariance under rigid motions and corner
relabelling, and a scaling identity on the sphere."""
import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W


def _face():
    xr = np.array([[0.3, -0.2, 0.1], [1.4, 0.1, -0.2], [0.5, 1.2, 0.3]])
    return xr, np.array([[0, 1, 2]], dtype=np.int32)


def _area(x, t):
    return 0.5 * np.linalg.norm(np.cross(x[t[:, 1]] - x[t[:, 0]], x[t[:, 2]] - x[t[:, 0]]), axis=1).sum()


def _in_plane_map(xr, Dmat):
    """Apply the 2x2 in-plane map Dmat to a flat face, in an orthonormal
    frame of its plane (e1 along edge 1->2)."""
    o = xr[0]
    e1 = (xr[1] - o) / np.linalg.norm(xr[1] - o)
    n = np.cross(xr[1] - o, xr[2] - o)
    n /= np.linalg.norm(n)
    e2 = np.cross(n, e1)
    Bm = np.stack([e1, e2], 1)  # 3x2
    loc = (xr - o) @ Bm         # n x 2
    return o + (loc @ Dmat.T) @ Bm.T


@pytest.mark.parametrize("lam", [0.9, 1.0, 1.07, 1.3])
def test_equibiaxial_energy_closed_form(orc, lam):
    """lambda1 = lambda2 = lambda: I1 = 2 lambda^2 - 2, I2 = lambda^4 - 1, so
    w = (k_s/6)(lambda^2 - 1)^2 + (k_a/12)(lambda^4 - 1)^2."""
    xr, t = _face()
    ks, ka = 0.7, 1.9
    x = _in_plane_map(xr, lam * np.eye(2))
    w = ks / 6 * (lam ** 2 - 1) ** 2 + ka / 12 * (lam ** 4 - 1) ** 2
    assert orc.membrane_energy(x, xr, t, ks, ka) == pytest.approx(_area(xr, t) * w, rel=1e-12, abs=1e-18)


@pytest.mark.parametrize("lam", [0.8, 1.05, 1.4])
def test_uniaxial_energy_closed_form(orc, lam):
    """(lambda, 1): I1 = I2 = lambda^2 - 1, w = (k_s + k_a)/12 (lambda^2 - 1)^2,
    for the stretch along either in-plane axis."""
    xr, t = _face()
    ks, ka = 0.7, 1.9
    for D in (np.diag([lam, 1.0]), np.diag([1.0, lam])):
        x = _in_plane_map(xr, D)
        w = (ks + ka) / 12 * (lam ** 2 - 1) ** 2
        assert orc.membrane_energy(x, xr, t, ks, ka) == pytest.approx(_area(xr, t) * w, rel=1e-12)


@pytest.mark.parametrize("gam", [0.05, 0.3])
def test_simple_shear_energy_closed_form(orc, gam):
    """Area-preserving simple shear [[1, g], [0, 1]]: I1 = g^2, I2 = 0, so
    w = (k_s/12)(g^4 + 2 g^2) and the dilation modulus does not enter."""
    xr, t = _face()
    x = _in_plane_map(xr, np.array([[1.0, gam], [0.0, 1.0]]))
    w = 0.7 / 12 * (gam ** 4 + 2 * gam ** 2)
    assert orc.membrane_energy(x, xr, t, 0.7, 123.0) == pytest.approx(_area(xr, t) * w, rel=1e-11)


def test_rigid_motion_has_no_energy_or_force(orc):
    xr, t = orc.icosphere(2, 3.0, (5.0, 6.0, 7.0))
    R = W.random_rotation(4)
    x = (xr - 5.0) @ R.T + np.array([9.0, -1.0, 2.0])
    assert abs(orc.membrane_energy(x, xr, t, 0.1, 0.1)) < 1e-13
    assert np.max(np.abs(orc.membrane_forces(x, xr, t, 0.1, 0.1))) < 1e-13
    assert np.max(np.abs(orc.membrane_forces(xr, xr, t, 0.1, 0.1))) < 1e-15


def _deformed(orc, level=1, seed=0, amp=0.08):
    xr, t = orc.icosphere(level, 2.0, (3.0, 3.0, 3.0))
    x = xr + W.noise(xr.shape, amp, seed)
    return x, xr, t


@pytest.mark.parametrize("seed", [0, 1])
def test_forces_are_minus_energy_gradient(orc, seed):
    """F_n = -dW/dx_n (Eq. forcefromenergy) against central differences of the
    energy, h = 1e-6."""
    x, xr, t = _deformed(orc, 1, seed)
    ks, ka = 0.05, 0.11
    F = orc.membrane_forces(x, xr, t, ks, ka)
    h = 1e-6
    fd = np.zeros_like(x)
    for n in range(x.shape[0]):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[n, d] += h
            xm[n, d] -= h
            fd[n, d] = -(orc.membrane_energy(xp, xr, t, ks, ka)
                         - orc.membrane_energy(xm, xr, t, ks, ka)) / (2 * h)
    assert np.max(np.abs(F - fd)) < 1e-7 * np.max(np.abs(F))


def test_no_net_force_or_torque(orc):
    x, xr, t = _deformed(orc, 2, 5)
    F = orc.membrane_forces(x, xr, t, 0.03, 0.07)
    scale = np.abs(F).max()
    assert np.max(np.abs(F.sum(0))) < 1e-13 * scale * len(x)
    assert np.max(np.abs(np.cross(x, F).sum(0))) < 1e-12 * scale * len(x)


def test_rotation_covariance(orc):
    x, xr, t = _deformed(orc, 2, 6)
    R = W.random_rotation(8)
    F = orc.membrane_forces(x, xr, t, 0.03, 0.07)
    FR = orc.membrane_forces(x @ R.T + 4.0, xr, t, 0.03, 0.07)
    assert np.allclose(FR, F @ R.T, atol=1e-13 * np.abs(F).max())


def test_corner_relabelling_invariance(orc):
    """Which two edges define l, l' and phi is arbitrary (Sec. II.B): rotating
    the corner order of every face changes neither energy nor forces."""
    x, xr, t = _deformed(orc, 2, 9)
    t2 = np.ascontiguousarray(t[:, [1, 2, 0]])
    assert orc.membrane_energy(x, xr, t, 0.03, 0.07) == pytest.approx(
        orc.membrane_energy(x, xr, t2, 0.03, 0.07), rel=1e-12)
    F1 = orc.membrane_forces(x, xr, t, 0.03, 0.07)
    F2 = orc.membrane_forces(x, xr, t2, 0.03, 0.07)
    assert np.allclose(F1, F2, atol=1e-13 * np.abs(F1).max())


@pytest.mark.parametrize("s", [0.97, 1.02, 1.1])
def test_sphere_scaling_virial(orc, s):
    """Scaling the reference sphere by s about its centre stretches every face
    equibiaxially, W(s) = A0_total w(s), and sum_n F_n.(x_n - c) = -s W'(s)."""
    c = np.array([2.0, 2.0, 2.0])
    xr, t = orc.icosphere(3, 2.5, c)
    x = c + s * (xr - c)
    ks, ka = 0.02, 0.05
    A0 = _area(xr, t)
    W_ = A0 * (ks / 6 * (s ** 2 - 1) ** 2 + ka / 12 * (s ** 4 - 1) ** 2)
    dW = A0 * (ks / 6 * 2 * (s ** 2 - 1) * 2 * s + ka / 12 * 2 * (s ** 4 - 1) * 4 * s ** 3)
    assert orc.membrane_energy(x, xr, t, ks, ka) == pytest.approx(W_, rel=1e-11)
    F = orc.membrane_forces(x, xr, t, ks, ka)
    assert ((x - c) * F).sum() == pytest.approx(-s * dW, rel=1e-11)
