"""Writes the oracle's reference results for the full-length parity tests.

Everything here comes from the FP64 CPU oracle (oracle/) started from the
same representable inputs the GPU tests use (tests/parity_helpers.Case: the
seeded workloads, Couette populations rounded to FP32 deviations, node
positions rounded to the library's FP32 frame).  Nothing reads the HIP path.

  trajectory_c2.txt   128^3, one r = 16 capsule (5120 faces), 4-point delta:
                      Taylor deformation D every 100 steps up to 20000
  trajectory_c3.txt   256 x 128 x 128 with 200 r = 8 capsules, 2-point delta:
                      D of every capsule every 100 steps up to 10000
  sensitivities_c5_2000.txt
                      64^3, one r = 8 capsule, 3-point delta: central
                      differences (h = 1e-4 relative) of D after 2000 steps
                      with respect to k_s (C fixed), C (k_s fixed) and the
                      shear rate 2 u_w / nz (through the walls and the
                      linear Couette start)

D is (r_a - r_c)/(r_a + r_c) from the inertia tensor of the closed mesh
(Sec. III).  The runs take hours of CPU; each file is written under a
'.partial' name row by row and renamed when complete.

usage: python tests/golden/make_trajectories.py {c2,c3,c5} [--threads N]
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
    ap.add_argument("what", choices=["c2", "c3", "c5"])
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args()
    if a.what == "c5":
        sensitivities(a.threads, a.out)
    else:
        trajectory(a.what, a.threads, a.out)


if __name__ == "__main__":
    main()
