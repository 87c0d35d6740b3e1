"""Seeded synthetic workloads: the shear-flow capsule configurations, in
lattice units, and the random draws that set them up.

This module holds no arithmetic of the method itself: it states sizes and
parameters, converts the paper's dimensionless groups to lattice parameters,
places capsule centres and draws seeded random numbers.  Meshes are not made
here (each side builds its own icosphere).  Both the oracle-driven tests and
the HIP path take their inputs from here.

Lattice units throughout: Delta x = Delta t = 1, rho_0 = 1, tau = 1 so the
kinematic viscosity is nu = (tau - 1/2)/3 = 1/6 (Sec. II.A) and the dynamic
viscosity eta = rho_0 nu.  The walls are nz lattice spacings apart and move
with +-u_w, so the shear rate is gamma_dot = 2 u_w / nz (Sec. II.A).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

ICOSPHERE_FACES = {0: 20, 1: 80, 2: 320, 3: 1280, 4: 5120, 5: 20480}


def icosphere_counts(level: int) -> Tuple[int, int]:
    """(nodes, faces) of an icosahedron subdivided `level` times:
    N_f = 20 * 4^level and 2 N_n = N_f + 4 (Sec. II.D)."""
    nf = 20 * 4 ** level
    return (nf + 4) // 2, nf


def viscosity(tau: float) -> float:
    """nu = c_s^2 (tau - 1/2) with c_s^2 = 1/3 (Sec. II.A)."""
    return (tau - 0.5) / 3.0


def shear_rate(u_w: float, nz: int) -> float:
    """gamma_dot = 2 u_w / H with H = nz (Sec. II.A)."""
    return 2.0 * u_w / nz


def ks_from_capillary(ca: float, u_w: float, nz: int, r: float, tau: float = 1.0) -> float:
    """Membrane shear modulus from the reduced shear rate
    G = gamma_dot eta r / k_s (Sec. III, Eq. shearrate), eta = rho_0 nu."""
    return shear_rate(u_w, nz) * viscosity(tau) * r / ca


@dataclass
class CapsuleSpec:
    level: int
    r: float
    center: Tuple[float, float, float]
    ks: float
    ka: float


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    u_w: float
    m: int
    steps: int
    capsules: List[CapsuleSpec] = field(default_factory=list)

    @property
    def n_nodes_lattice(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_membrane_nodes(self) -> int:
        return sum(icosphere_counts(c.level)[0] for c in self.capsules)


def _centre(n: int) -> float:
    # midway between the walls and the periodic ends: where u_Couette = 0
    return (n - 1) / 2.0


def single_capsule(name, n, u_w, level, r, ca, m, steps, C=1.0, tau=1.0) -> Workload:
    ks = ks_from_capillary(ca, u_w, n, r, tau)
    cap = CapsuleSpec(level, r, (_centre(n),) * 3, ks, C * ks)
    return Workload(name, n, n, n, tau, u_w, m, steps, [cap])


def rsa_centres(count: int, r: float, box: Tuple[int, int, int], gap: float,
                wall_margin: float, seed: int, max_tries: int = 1_000_000):
    """Random sequential addition of `count` sphere centres in a box that is
    periodic in x and y: every pair is at least 2 r + gap apart (minimum image
    along x and y) and every centre keeps r + wall_margin from both walls."""
    nx, ny, nz = box
    rng = np.random.default_rng(seed)
    zlo = r + wall_margin
    zhi = (nz - 1) - r - wall_margin
    dmin2 = (2.0 * r + gap) ** 2
    out = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        c = np.array([rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(zlo, zhi)])
        ok = True
        for q in out:
            d = c - q
            d[0] -= nx * np.round(d[0] / nx)
            d[1] -= ny * np.round(d[1] / ny)
            if d @ d < dmin2:
                ok = False
                break
        if ok:
            out.append(c)
    return np.array(out)


def dense_suspension(count: int = 200, seed_place: int = 1004, seed_ca: int = 2416,
                     nx: int = 256, ny: int = 128, nz: int = 128, u_w: float = 0.02,
                     r: float = 8.0, level: int = 3, m: int = 2, steps: int = 10000,
                     ca_range=(0.01, 0.1)) -> Workload:
    """Dense suspension of identical icosphere capsules at random
    non-overlapping centres with uniform random capillary numbers."""
    centres = rsa_centres(count, r, (nx, ny, nz), gap=2.0, wall_margin=2.0, seed=seed_place)
    ca = np.random.default_rng(seed_ca).uniform(ca_range[0], ca_range[1], size=count)
    caps = []
    for c, a in zip(centres, ca):
        ks = ks_from_capillary(float(a), u_w, nz, r)
        caps.append(CapsuleSpec(level, r, tuple(float(v) for v in c), ks, ks))
    return Workload("dense_suspension_%dx%dx%d_%dcaps" % (nx, ny, nz, count),
                    nx, ny, nz, 1.0, u_w, m, steps, caps)


def config(name: str) -> Workload:
    """The five shear-flow workloads of this project (lattice units):
    c1  32^3 single capsule r=6, 1280 faces, Ca=0.05, 3-point delta
    c2  128^3 single capsule r=16, 5120 faces, Ca=0.0125, 4-point delta
    c3  256x128x128 dense suspension, 200 capsules r=8, 2-point delta
    c5  64^3 single capsule r=8, 1280 faces, Ca=0.05, 3-point delta
    paper35  the paper's convergence case H=35, r=3.5, N_f=1280, G=0.01,
             Re=0.02 (Sec. IV.C, Table 2, first row); m set by the caller."""
    if name == "c1":
        return single_capsule("c1_32cube_r6_l3_phi3", 32, 0.01, 3, 6.0, 0.05, 3, 1000)
    if name == "c2":
        return single_capsule("c2_128cube_r16_l4_phi4", 128, 0.01, 4, 16.0, 0.0125, 4, 20000)
    if name == "c3":
        return dense_suspension()
    if name == "c5":
        return single_capsule("c5_64cube_r8_l3_phi3", 64, 0.01, 3, 8.0, 0.05, 3, 2000)
    if name.startswith("paper35"):
        return paper_case(35, 3.5, 3, m=int(name[-1]) if name[-1].isdigit() else 4)
    raise KeyError(name)


def paper_case(H: int, r: float, level: int, m: int, G: float = 0.01, Re: float = 0.02,
               kappa_t: float = 120.0, tau: float = 1.0) -> Workload:
    """A cubic H^3 box with the capsule at its centre at the paper's reduced
    shear rate G and Reynolds number Re = rho gamma_dot r^2 / eta (Sec. III),
    run to reduced time kappa t = gamma_dot t / G (Sec. IV)."""
    nu = viscosity(tau)
    gamma = Re * nu / (r * r)
    u_w = gamma * H / 2.0
    ks = gamma * nu * r / G
    steps = int(round(kappa_t * G / gamma))
    cap = CapsuleSpec(level, r, (_centre(H),) * 3, ks, ks)
    return Workload("paper_H%d_r%g_phi%d" % (H, r, m), H, H, H, tau, u_w, m, steps, [cap])


@dataclass
class BatchRun:
    n: int
    r: float
    level: int
    ca: float
    m: int
    u_w: float = 0.01


def batched_sweep(count: int = 64, seed: int = 1004) -> List[BatchRun]:
    """Uneven independent shear runs: H ~ U{24..64}, (r, level) uniform from
    {(4.5, 2), (6, 3), (9, 4)}, Ca ~ U[0.003, 0.1], delta width ~ U{2, 3, 4}."""
    rng = np.random.default_rng(seed)
    shapes = [(4.5, 2), (6.0, 3), (9.0, 4)]
    runs = []
    for _ in range(count):
        n = int(rng.integers(24, 65))
        r, lev = shapes[int(rng.integers(0, 3))]
        ca = float(rng.uniform(0.003, 0.1))
        m = int(rng.integers(2, 5))
        # keep the capsule and its stencil clear of the walls
        n = max(n, int(np.ceil(2 * r + m + 6)))
        runs.append(BatchRun(n, r, lev, ca, m))
    return runs


def sweep_workloads(count: int = 64, seed: int = 1004, steps: int = 5000) -> List[Workload]:
    """The batched sweep as workloads: each run a centred single capsule in an
    n^3 box (Sec. IV's parameter studies run many such independent cases)."""
    return [single_capsule(f"sweep{k:02d}_{b.n}cube_r{b.r:g}_l{b.level}_phi{b.m}", b.n, b.u_w,
                           b.level, b.r, b.ca, b.m, steps)
            for k, b in enumerate(batched_sweep(count, seed))]


def noise(shape, amplitude: float, seed: int) -> np.ndarray:
    """Seeded uniform noise in [-amplitude, amplitude]."""
    return np.random.default_rng(seed).uniform(-amplitude, amplitude, size=shape)


def random_rotation(seed: int) -> np.ndarray:
    """Seeded uniformly random rotation matrix (QR of a Gaussian matrix)."""
    a = np.random.default_rng(seed).normal(size=(3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q
