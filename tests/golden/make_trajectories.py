"""Writes the oracle's reference results for the full-length parity tests.

Everything here comes from the FP64 CPU oracle (oracle/) started from the
same representable inputs the GPU tests use (tests/parity_helpers.Case: the
seeded workloads, Couette populations rounded to FP32 deviations, node
positions rounded to the library's FP32 frame).  Nothing reads the HIP path.

  trajectory_c2.txt   128^3, one r = 16 capsule (5120 faces), 4-point delta:
                      Taylor deformation D every 100 steps up to 20000
  trajectory_c3.txt   256 x 128 x 128 with 200 r = 8 capsules, 2-point delta:
                      D of every capsule every 100 steps up to 10000
  trajectory_c4.txt   the 64 independent runs of the batched sweep (24^3..64^3,
                      one capsule each, 2-, 3- and 4-point deltas): D of
                      every run every 100 steps up to 5000
  sensitivities_c5_2000.txt
                      64^3, one r = 8 capsule, 3-point delta: central
                      differences (h = 1e-4 relative) of D after 2000 steps
                      with respect to k_s (C fixed), C (k_s fixed) and the
                      shear rate 2 u_w / nz (through the walls and the
                      linear Couette start)

D is (r_a - r_c)/(r_a + r_c) from the inertia tensor of the closed mesh
(Sec. III).  The runs take hours of CPU; each file is written under a
'.partial' name row by row and renamed when complete.

usage: python tests/golden/make_trajectories.py {c2,c3,c4,c5} [--threads N]
(c4: N worker processes, one oracle thread each)
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

from parity_helpers import Case, O, couette_populations  # noqa: E402
from paper_1004_2416_amd import workloads as W  # noqa: E402

EVERY = 100
H_FD = 1e-4


def _open(path, header):
    fh = open(path + ".partial", "w")
    for line in header:
        fh.write("# " + line + "\n")
    fh.flush()
    return fh


def _finish(fh, path):
    fh.close()
    os.replace(path + ".partial", path)


def trajectory(name, threads, out_dir):
    wl = W.config(name)
    c = Case(wl)
    sim = c.oracle(nthreads=threads)
    path = os.path.join(out_dir, "trajectory_%s.txt" % name)
    fh = _open(path, [
        "oracle Taylor deformation D (Sec. III) of each capsule every %d steps" % EVERY,
        "workload %s: %dx%dx%d, tau %g, u_w %g, delta width %d, %d capsules, %d steps"
        % (wl.name, wl.nx, wl.ny, wl.nz, wl.tau, wl.u_w, wl.m, len(wl.capsules), wl.steps),
        "start: Couette equilibrium rounded to FP32 deviations, undeformed capsules in the"
        " library's FP32 frame (tests/parity_helpers.Case)",
        "written by: python tests/golden/make_trajectories.py %s" % name,
        "columns: step, D of capsule 0 .. %d" % (len(wl.capsules) - 1),
    ])
    t0 = time.time()
    fh.write("0 " + " ".join("%.12e" % o["D"] for o in c.observables(sim.x)) + "\n")
    for s in range(EVERY, wl.steps + 1, EVERY):
        rc = sim.run(EVERY)
        if rc != 0:
            raise RuntimeError("oracle run failed at step %d: %d" % (s, rc))
        fh.write("%d " % s + " ".join("%.12e" % o["D"] for o in c.observables(sim.x)) + "\n")
        fh.flush()
        print("%s step %d  %.0f s" % (name, s, time.time() - t0), flush=True)
    _finish(fh, path)


def _sweep_run(args):
    """D of one run of the batched sweep every EVERY steps (one oracle thread)."""
    k, wl, steps = args
    c = Case(wl)
    sim = c.oracle(nthreads=1)
    out = [c.observables(sim.x)[0]["D"]]
    for s in range(EVERY, steps + 1, EVERY):
        if sim.run(EVERY) != 0:
            raise RuntimeError("oracle run %d failed at step %d" % (k, s))
        out.append(c.observables(sim.x)[0]["D"])
    return k, out


def sweep_trajectories(processes, out_dir, steps=5000):
    from multiprocessing import Pool
    wls = W.sweep_workloads(steps=steps)
    path = os.path.join(out_dir, "trajectory_c4.txt")
    t0 = time.time()
    res = {}
    # the largest runs first, so that the pool ends evenly
    order = sorted(range(len(wls)), key=lambda k: -wls[k].n_nodes_lattice)
    with Pool(processes) as pool:
        for k, D in pool.imap_unordered(_sweep_run, [(k, wls[k], steps) for k in order]):
            res[k] = D
            print("c4 run %d done (%d of %d)  %.0f s" % (k, len(res), len(wls), time.time() - t0),
                  flush=True)
    fh = _open(path, [
        "oracle Taylor deformation D (Sec. III) of each run every %d steps" % EVERY,
        "workload batched_sweep_64runs: %d runs %s, %d steps" % (
            len(wls), " ".join("%dx%dx%d/m%d" % (w.nx, w.ny, w.nz, w.m) for w in wls), steps),
        "start: Couette equilibrium rounded to FP32 deviations, undeformed capsules in the"
        " library's FP32 frame (tests/parity_helpers.Case)",
        "written by: python tests/golden/make_trajectories.py c4",
        "columns: step, D of run 0 .. %d" % (len(wls) - 1),
    ])
    for j, s in enumerate(range(0, steps + 1, EVERY)):
        fh.write("%d " % s + " ".join("%.12e" % res[k][j] for k in range(len(wls))) + "\n")
    _finish(fh, path)


def sensitivities(threads, out_dir, steps=2000):
    wl = W.config("c5")
    c = Case(wl)
    nz = wl.nz

    def D(which, scale):
        ks, ka, uw = c.ks_face.copy(), c.ka_face.copy(), wl.u_w
        if which == "ks":
            ks, ka = ks * scale, ka * scale
        elif which == "C":
            ka = ka * scale
        else:
            uw = uw * scale
        f0 = couette_populations(wl.nz, wl.ny, wl.nx, uw)
        sim = O.Simulation(f0, c.xref, c.xref, c.tri, ks, ka, wl.tau, uw, wl.m,
                           nthreads=threads)
        if sim.run(steps) != 0:
            raise RuntimeError("oracle run failed")
        return c.observables(sim.x)[0]["D"]

    params = {"ks": c.ks[0], "C": c.ka[0] / c.ks[0], "gamma": 2.0 * wl.u_w / nz}
    path = os.path.join(out_dir, "sensitivities_c5_%d.txt" % steps)
    fh = _open(path, [
        "oracle central differences of D after %d steps, h = %g relative" % (steps, H_FD),
        "workload %s: %dx%dx%d, tau %g, u_w %g, delta width %d, k_s %.10e, C %g"
        % (wl.name, wl.nx, wl.ny, wl.nz, wl.tau, wl.u_w, wl.m, c.ks[0], c.ka[0] / c.ks[0]),
        "start: exact FP64 Couette equilibrium of the scaled wall speed, undeformed capsule"
        " in the library's FP32 frame",
        "written by: python tests/golden/make_trajectories.py c5",
        "columns: parameter (ks | C | gamma), value p, D(p(1+h)), D(p(1-h)), dD/dp",
    ])
    t0 = time.time()
    for which, p in params.items():
        dp, dm = D(which, 1 + H_FD), D(which, 1 - H_FD)
        fh.write("%s %.17e %.17e %.17e %.17e\n" % (which, p, dp, dm, (dp - dm) / (2 * H_FD * p)))
        fh.flush()
        print("c5 %s done  %.0f s" % (which, time.time() - t0), flush=True)
    _finish(fh, path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args()
    if a.what == "c5":
        sensitivities(a.threads, a.out)
    elif a.what == "c4":
        sweep_trajectories(max(1, a.threads), a.out)
    else:
        trajectory(a.what, a.threads, a.out)


if __name__ == "__main__":
    main()
