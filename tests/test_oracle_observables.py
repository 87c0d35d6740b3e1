"""Pins of the oracle's shape observables (Sec. III): the inertia-tensor
ellipsoid recovers D and theta exactly for affinely stretched icospheres,
with semiaxes underestimated by one common factor (as the paper remarks),
and the enclosed volume matches closed forms."""
import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W


def test_sphere_is_undeformed(orc):
    x, t = orc.icosphere(3, 6.0, (15.5, 15.5, 15.5))
    o = orc.capsule_observables(x, t)
    assert abs(o["D"]) < 1e-14
    assert np.isnan(o["theta"])  # no distinguished axis
    assert np.allclose([o["cx"], o["cy"], o["cz"]], 15.5, atol=1e-12)
    assert 0.97 * 4 / 3 * np.pi * 216 < o["V"] < 4 / 3 * np.pi * 216


@pytest.mark.parametrize("a,b,c,th", [(1.2, 1.0, 0.8, 0.3), (1.05, 1.0, 0.97, 0.7),
                                      (6.0, 5.0, 4.0, -0.4), (1.3, 0.9, 1.1, 1.2)])
def test_affine_ellipsoid_exact(orc, a, b, c, th):
    """Stretch the unit icosphere by diag(a, b, c), rotate by th about y and
    shift: D = (r_a - r_c)/(r_a + r_c) with the largest and smallest stretch,
    and theta = angle of the major axis in the xz plane (Sec. III)."""
    x, t = orc.icosphere(3, 1.0)
    R = np.array([[np.cos(th), 0, -np.sin(th)], [0, 1, 0], [np.sin(th), 0, np.cos(th)]])
    y = (x * [a, b, c]) @ R.T + [3.0, -4.0, 5.0]
    o = orc.capsule_observables(y, t)
    ax = sorted([a, b, c])
    assert o["D"] == pytest.approx((ax[2] - ax[0]) / (ax[2] + ax[0]), abs=1e-13)
    major = np.argmax([a, b, c])
    if major == 0:
        want = th
    elif major == 2:
        want = th + np.pi / 2
    else:
        want = None
    if want is not None:
        want = (want + np.pi / 2) % np.pi - np.pi / 2
        assert np.cos(o["theta"] - want) == pytest.approx(1.0, abs=1e-13)
    k = np.array([o["ra"], o["rb"], o["rc"]]) / np.array(ax[::-1])
    assert np.allclose(k, k[0], rtol=1e-12) and 0.99 < k[0] < 1.0


def test_affine_ellipsoid_any_rotation(orc):
    x, t = orc.icosphere(2, 1.0)
    R = W.random_rotation(21)
    o = orc.capsule_observables((x * [1.3, 1.1, 0.7]) @ R.T, t)
    assert o["D"] == pytest.approx(0.6 / 2.0, abs=1e-13)


def test_volume_closed_forms(orc):
    x0, t0 = orc.icosphere(0, 1.0)
    a = np.linalg.norm(x0[t0[0, 0]] - x0[t0[0, 1]])
    assert orc.capsule_observables(x0, t0)["V"] == pytest.approx(5 / 12 * (3 + 5 ** 0.5) * a ** 3, rel=1e-14)
    x, t = orc.icosphere(3, 2.0)
    v0 = orc.capsule_observables(x, t)["V"]
    assert orc.capsule_observables(x + [100.0, -7.0, 3.0], t)["V"] == pytest.approx(v0, rel=1e-12)
    assert orc.capsule_observables(x * [1.5, 1.0, 0.5], t)["V"] == pytest.approx(0.75 * v0, rel=1e-13)
