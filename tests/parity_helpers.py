"""Helpers shared by the GPU parity tests: inputs in the precision both sides
represent exactly, oracle runs and error measures.  Inputs come from
paper_1004_2416_amd.workloads and the oracle; nothing here reads results of
the HIP path except the comparisons themselves."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1004_2416_amd import workloads as W

_, WEIGHTS, _ = O.lattice_constants()


def rep_populations(f):
    """Round f to what FP32 storage of f_i - w_i holds."""
    w = WEIGHTS[:, None, None, None]
    return w + (f - w).astype(np.float32).astype(np.float64)


def rep_positions(x, node_counts):
    """Round node positions to the library's frame: per capsule the integer
    origin floor(mean of its nodes) plus FP32 offsets.  The library takes
    that origin from the positions it is given, so the result must give back
    its own origin: a capsule centred on an integer has its mean within
    rounding of that integer, and rounding the offsets can move the mean
    across it; then the nodes are rounded again in the new frame."""
    out = np.empty_like(x)
    n0 = 0
    for n in node_counts:
        y = x[n0:n0 + n]
        for _ in range(8):
            o = np.floor(y.sum(axis=0) / n)
            y = o + (y - o).astype(np.float32).astype(np.float64)
            if np.array_equal(np.floor(y.sum(axis=0) / n), o):
                break
        else:
            raise RuntimeError("no FP32 frame reproduces its own origin")
        out[n0:n0 + n] = y
        n0 += n
    return out


def couette_populations(nz, ny, nx, uw, linear=False):
    f = np.empty((19, nz, ny, nx))
    for z in range(nz):
        ux = uw * (2 * z + 1 - nz) / nz
        f[:, z] = O.equilibrium(1.0, [ux, 0.0, 0.0], linear=linear)[:, None, None]
    return f


class Case:
    """A coupled configuration built from a workload, with representable
    inputs, ready for both the oracle and the library."""

    def __init__(self, wl: W.Workload, perturb: float = 0.0, seed: int = 0):
        self.wl = wl
        meshes = []
        for c in wl.capsules:
            x, t = O.icosphere(c.level, c.r, c.center)
            meshes.append((x, t))
        self.node_counts = [len(x) for x, _ in meshes]
        self.face_counts = [len(t) for _, t in meshes]
        x = np.concatenate([m[0] for m in meshes]) if meshes else np.zeros((0, 3))
        self.xref = rep_positions(x, self.node_counts) if meshes else x
        self.tri_local = [t for _, t in meshes]
        offs = np.cumsum([0] + self.node_counts[:-1]) if meshes else []
        self.tri = (np.concatenate([t + o for t, o in zip(self.tri_local, offs)])
                    if meshes else np.zeros((0, 3), np.int32)).astype(np.int32)
        self.ks = np.array([c.ks for c in wl.capsules])
        self.ka = np.array([c.ka for c in wl.capsules])
        self.ks_face = np.repeat(self.ks, self.face_counts) if meshes else np.zeros(0)
        self.ka_face = np.repeat(self.ka, self.face_counts) if meshes else np.zeros(0)
        f = couette_populations(wl.nz, wl.ny, wl.nx, wl.u_w)
        if perturb:
            f = f * (1 + W.noise(f.shape, perturb, seed))
        self.f0 = rep_populations(f)

    def meshes(self, x=None):
        x = self.xref if x is None else x
        out, n0 = [], 0
        for n, t in zip(self.node_counts, self.tri_local):
            out.append((x[n0:n0 + n], t))
            n0 += n
        return out

    def oracle(self, f=None, x=None, nthreads=0, linear=False, ab2=False):
        return O.Simulation(self.f0 if f is None else f, self.xref if x is None else x,
                            self.xref, self.tri, self.ks_face, self.ka_face, self.wl.tau,
                            self.wl.u_w, self.wl.m, linear_eq=linear, ab2=ab2, nthreads=nthreads)

    def gpu(self, storage="fp32", graph=True):
        from paper_1004_2416_amd import binding as B
        wl = self.wl
        lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, storage=storage)
        lat.set_shear(wl.u_w, init_profile=False)
        if wl.capsules:
            lat.add_capsules(self.meshes(), self.ks, self.ka, wl.m)
        lat.set_option(B.OPT_GRAPH, int(graph))
        lat.set_populations(self.f0)
        return lat

    def observables(self, x):
        out, n0, f0 = [], 0, 0
        for n, t in zip(self.node_counts, self.tri_local):
            out.append(O.capsule_observables(x[n0:n0 + n], t))
            n0 += n
        return out


def rel_err(a, b):
    """max |a - b| / |b| elementwise (b bounded away from 0)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def scaled_err(a, b):
    """max |a - b| / max |b|."""
    a, b = np.asarray(a), np.asarray(b)
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def deformed_mesh(c: Case, strain: float, seed: int):
    """Each capsule of case c stretched by a random symmetric map I + S
    (|S| ~ strain) about its centre, plus small node noise; rounded to the
    library frame."""
    rng = np.random.default_rng(seed)
    out, n0 = [], 0
    for n, cap in zip(c.node_counts, c.wl.capsules):
        S = rng.uniform(-strain, strain, (3, 3))
        A = np.eye(3) + 0.5 * (S + S.T)
        cen = np.array(cap.center)
        x = c.xref[n0:n0 + n]
        out.append(cen + (x - cen) @ A.T + rng.uniform(-0.05 * strain, 0.05 * strain, x.shape))
        n0 += n
    return rep_positions(np.concatenate(out), c.node_counts)
