"""Benchmark: lattice-node updates per second (MLUPS) of the full coupled
IB-LB-FEM timestep on one MI355X, with the HBM roofline fraction of the
collide-stream kernel and the FP64 CPU oracle timed on the host beside it.

    python bench.py [--steps K] [--warmup W] [--workload c3] [--storage fp32]

One step = Skalak forces, spreading, collide-stream with walls, interpolation
and advection (Sec. II.C) over the whole lattice and every capsule.  The
default workload is the largest single-GPU one: the dense suspension of 200
capsules on a 256 x 128 x 128 lattice (2-point delta), FP32 populations.  W
warm-up steps and the capture of the library's step graphs come before the
timed region, which holds exactly K steps between HIP events on the
library's stream.  The same line carries, timed the same way, FP16
population storage on the same workload and the 64-run batched sweep with
FP32 and FP16 storage ("legs"), and the FP64 oracle on the host's cores
(all threads and one thread).  Inputs are synthetic (the shear-flow
workloads of paper_1004_2416_amd.workloads) and resident in HBM before
timing.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "IB-LBM step MLUPS, % HBM roofline; batched/FP16/adjoint vs plain FP32"
KERNEL_SOURCES = ("paper_1004_2416_amd/csrc/lbm_kernels.hip", "paper_1004_2416_amd/csrc/lbm_device.h",
                  "paper_1004_2416_amd/csrc/common.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "collide_stream_traffic.txt")


def bytes_per_node(storage: str) -> int:
    """Algorithmic bytes of one lattice-node update: the 19 populations read
    once and written once (FP32: 4 B, FP16: 2 B each)."""
    return 19 * 2 * (4 if storage == "fp32" else 2)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str):
    """HBM bytes per collide-stream launch from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src = kernel_source_hash()
    for line in open(TRAFFIC_FILE):
        if line.startswith("#"):
            continue
        parts = line.split()
        if len(parts) == 5 and parts[0] == workload and parts[1] == storage and parts[4] == src:
            return float(parts[2]) + float(parts[3])
    return None


def setup(workload: str, storage: str, graph: bool, variant: int = -1, box: int = -1,
          overlap: int = -1, streaming: int = -1, one_buffer: bool = False,
          fp16_mass: bool = False):
    from paper_1004_2416_amd import binding as B
    from paper_1004_2416_amd import workloads as W

    wl = W.config(workload)
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, storage=storage, one_buffer=one_buffer)
    lat.set_shear(wl.u_w, init_profile=True)
    meshes = [B.icosphere(c.level, c.r, c.center) for c in wl.capsules]
    lat.add_capsules(meshes, [c.ks for c in wl.capsules], [c.ka for c in wl.capsules], wl.m)
    lat.set_option(B.OPT_GRAPH, int(graph))
    if variant >= 0:
        lat.set_option(B.OPT_LBM_VARIANT, int(variant))
    if box >= 0:
        lat.set_option(B.OPT_STENCIL_BOX, int(box))
    if overlap >= 0:
        lat.set_option(B.OPT_OVERLAP, int(overlap))
    if streaming >= 0:
        lat.set_option(B.OPT_STREAMING, int(streaming))
    if fp16_mass:
        lat.set_option(B.OPT_FP16_MASS, 1)
    return wl, lat


def prime(stepper, warmup: int):
    """Warm-up steps, then the steps that make the library capture and
    instantiate its 16-step graphs for both parities of the step count (a
    graph is captured on the host the first time it is needed), so that the
    timed region holds steady-state steps only."""
    stepper.step(warmup)
    stepper.step(16)
    stepper.step(1)
    stepper.step(16)


def timed(stream, stepper, steps: int) -> float:
    """Milliseconds of `steps` steps between HIP events on the library's
    stream, device synchronised before and after."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    stepper.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(wl, seconds: float, nthreads: int):
    """The FP64 oracle: whole coupled steps of the same workload from the same
    initial state, after one untimed step (first touch of its arrays), until
    `seconds` have passed."""
    import numpy as np
    from oracle import oracle as O

    xs, ts, ks, ka = [], [], [], []
    off = 0
    for c in wl.capsules:
        x, t = O.icosphere(c.level, c.r, c.center)
        xs.append(x)
        ts.append(t + off)
        off += len(x)
        ks += [c.ks] * len(t)
        ka += [c.ka] * len(t)
    x = np.concatenate(xs)
    f = np.empty((19, wl.nz, wl.ny, wl.nx))
    for z in range(wl.nz):
        ux = wl.u_w * (2 * z + 1 - wl.nz) / wl.nz
        f[:, z] = O.equilibrium(1.0, [ux, 0.0, 0.0])[:, None, None]
    sim = O.Simulation(f, x, x, np.concatenate(ts), ks, ka, wl.tau, wl.u_w, wl.m,
                       nthreads=nthreads)
    sim.run(1)
    steps, t0 = 0, time.perf_counter()
    while True:
        sim.run(1)
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    threads = nthreads if nthreads > 0 else O.max_threads()
    return {"value": round(wl.n_nodes_lattice * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"{steps} full FP64 coupled steps of {wl.name} in {dt:.1f} s "
                      f"on {threads} thread(s)"}


def cpu_baseline(wl, seconds: float):
    """The oracle on all host threads (the reported value) and on one thread,
    each on a bounded sample of the workload's steps."""
    allt = cpu_leg(wl, seconds, 0)
    one = cpu_leg(wl, seconds, 1)
    allt["single_thread"] = {"value": one["value"], "unit": one["unit"], "cores": 1,
                             "sample": one["sample"]}
    allt["cpu_model"] = cpu_model()
    return allt


def copy_calibration(mib: int):
    """A plain device-to-device copy of known size, for scaling the
    rocprofv3 FETCH_SIZE / WRITE_SIZE counters; also times it (the
    achievable streaming bandwidth next to the 8 TB/s vendor figure)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "launches": 6,
                      "copy_ms": round(ms, 4), "copy_GBps": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}))


def single_leg(args, workload: str, storage: str, roofline: bool):
    """One lattice workload in the benchmark's launch configuration: warm-up
    and graph capture, then exactly args.steps timed steps."""
    wl, lat = setup(workload, storage, not args.no_graph, args.lbm_variant,
                    args.stencil_box, args.overlap, args.streaming, args.one_buffer,
                    args.fp16_mass)
    tuned = lat.autotune(64) if args.autotune else None
    split_box = lat.split_box()
    prime(lat, args.warmup)
    ms = timed(lat.stream, lat, args.steps)
    lat.synchronize()
    mlups = wl.n_nodes_lattice * args.steps / (ms * 1e-3) / 1e6
    leg = {"workload": wl.name, "storage": storage, "value": round(mlups, 1), "unit": "MLUPS",
           "ms_per_step": round(ms / args.steps, 5),
           "step_pct_hbm_roofline": round(100 * mlups * 1e6 * bytes_per_node(storage)
                                          / (HBM_PEAK_GBS * 1e9), 2),
           "membrane_node_updates_per_s": round(wl.n_membrane_nodes * args.steps / (ms * 1e-3), 1)}
    extra = {"wl": wl, "split_box": list(split_box), "tuned": tuned}
    if roofline:
        # per-phase durations from HIP events between the kernels on the
        # library's stream, then the collide-stream kernel's own duration
        # from the start and end timestamps of its dispatches
        extra["phases"] = lat.profile(args.profile_steps)
        extra["k1_ms"] = lat.lattice_kernel_ms(args.profile_steps)
        extra["D"] = lat.observables()[:4, 4]
    lat.close()
    return leg, extra


def batch_leg(args, storage: str, with_single: bool = False):
    """The batched sweep: 64 independent single-capsule runs of uneven size,
    capillary number and delta width advanced together (one launch per kernel
    of the step for all runs)."""
    import torch
    from paper_1004_2416_amd import binding as B
    from paper_1004_2416_amd import workloads as W

    wls = W.sweep_workloads()
    lats = []
    for wl in wls:
        lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau, storage=storage)
        lat.set_shear(wl.u_w, init_profile=True)
        c = wl.capsules[0]
        lat.add_capsules([B.icosphere(c.level, c.r, c.center)], [c.ks], [c.ka], wl.m)
        if args.stencil_box >= 0:
            lat.set_option(B.OPT_STENCIL_BOX, args.stencil_box)
        lats.append(lat)
    batch = B.Batch(lats)
    stream = lats[0].stream
    n_lat = sum(w.n_nodes_lattice for w in wls)
    n_mem = sum(w.n_membrane_nodes for w in wls)
    tuned = batch.autotune(64) if args.autotune else None
    if args.persistent:
        batch.set_persistent(True)
    prime(batch, args.warmup)
    ms = timed(stream, batch, args.steps)
    mlups = n_lat * args.steps / (ms * 1e-3) / 1e6
    leg = {"workload": "batched_sweep_64runs", "storage": storage, "value": round(mlups, 1),
           "unit": "MLUPS", "ms_per_step": round(ms / args.steps, 5),
           "step_pct_hbm_roofline": round(100 * mlups * 1e6 * bytes_per_node(storage)
                                          / (HBM_PEAK_GBS * 1e9), 2),
           "membrane_node_updates_per_s": round(n_mem * args.steps / (ms * 1e-3), 1)}
    if tuned:
        leg["autotuned"] = tuned
    extra = {"wls": wls, "n_lat": n_lat, "n_mem": n_mem, "tuned": tuned}
    if with_single:
        # the same runs, each stepped on its own (its own graphs, captured
        # before the timed region) for comparison
        for lat in lats:
            prime(lat, 0)
        torch.cuda.synchronize()
        k_single = max(16, (args.steps // 10) // 16 * 16)
        import torch as _t
        e0, e1 = _t.cuda.Event(enable_timing=True), _t.cuda.Event(enable_timing=True)
        e0.record(stream)
        for lat in lats:
            lat.step(k_single)
        e1.record(stream)
        torch.cuda.synchronize()
        leg["unbatched_mlups"] = round(n_lat * k_single / (e0.elapsed_time(e1) * 1e-3) / 1e6, 1)
        leg["batched_speedup"] = round(mlups / leg["unbatched_mlups"], 3)
        extra["phases"] = batch.profile(args.profile_steps)
        extra["k1_ms"] = batch.lattice_kernel_ms(args.profile_steps)
        extra["D"] = [float(lat.observables()[0, 4]) for lat in lats[:4]]
    batch.close()
    for lat in lats:
        lat.close()
    return leg, extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="c4: the batched sweep of 64 independent runs")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--stencil-box", type=int, default=-1,
                    help="IBM_OPT_STENCIL_BOX bits (-1: library default)")
    ap.add_argument("--overlap", type=int, default=1,
                    help="IBM_OPT_OVERLAP: 1 (default) splits the lattice update where it pays, "
                         "0 off, -1 library default")
    ap.add_argument("--streaming", type=int, default=-1,
                    help="population streaming pattern: 0 two buffers, 1 AA (one buffer); "
                         "-1 the library's default")
    ap.add_argument("--fp16-mass", action="store_true",
                    help="FP16 storage: the rest population takes back the mass the node's "
                         "other values lose to rounding (IBM_OPT_FP16_MASS)")
    ap.add_argument("--one-buffer", action="store_true",
                    help="one population buffer (the AA pattern; nx a multiple of 4)")
    ap.add_argument("--sensitivity", action="store_true",
                    help="time the tangent-model gradient of D instead of the step")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its kernel forms during warm-up")
    ap.add_argument("--persistent", action="store_true",
                    help="c4: each batched step as one persistent (cooperative) launch")
    ap.add_argument("--lbm-variant", type=int, default=-1,
                    help="collide-stream launch variant (IBM_OPT_LBM_VARIANT bits; "
                         "-1: the library default)")
    ap.add_argument("--profile-steps", type=int, default=400)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="time only the chosen workload (no FP16 / batched comparison legs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU path (the lattice would split into x-slabs with a 5-population halo "
              "exchange per cut face, capsules owned by the GPU holding their centre).",
              flush=True)
        sys.exit(2)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    if args.sensitivity:
        run_sensitivity(args)
        return

    t_wall = time.perf_counter()
    if args.workload == "c4":
        head, ex = batch_leg(args, args.storage, with_single=True)
        n_nodes = ex["n_lat"]
        config = {"workload": "batched_sweep_64runs", "runs": len(ex["wls"]),
                  "lattice_nodes": ex["n_lat"], "membrane_nodes": ex["n_mem"],
                  "storage": args.storage, "run_sizes": sorted({w.nx for w in ex["wls"]}),
                  "delta_widths": sorted({w.m for w in ex["wls"]}),
                  "stencil_box": args.stencil_box, "autotuned": ex["tuned"]}
        kernel = "k_batch_collide_stream"
        traffic_key = "batched_sweep_64runs"
    else:
        head, ex = single_leg(args, args.workload, args.storage, roofline=True)
        wl = ex["wl"]
        n_nodes = wl.n_nodes_lattice
        config = {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "nz": wl.nz,
                  "capsules": len(wl.capsules), "membrane_nodes": wl.n_membrane_nodes,
                  "delta_width": wl.m, "storage": args.storage, "graph": not args.no_graph,
                  "u_w": wl.u_w, "tau": wl.tau, "lbm_variant": args.lbm_variant,
                  "stencil_box": args.stencil_box,
                  "overlap": args.overlap, "split_box": ex["split_box"],
                  "fp16_mass_correction": bool(args.fp16_mass),
                  "streaming": ("aa_one_buffer" if args.one_buffer else
                                "aa" if args.streaming == 1 else "two_buffers"),
                  "autotuned": ex["tuned"]}
        kernel = "k_collide_stream_rows"
        # the stored counters were taken on the two-buffer kernel
        aa = args.one_buffer or args.streaming == 1
        traffic_key = None if aa or args.fp16_mass else wl.name
    algo = bytes_per_node(args.storage) * n_nodes
    achieved = algo / (ex["k1_ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "membrane_node_updates_per_s": head["membrane_node_updates_per_s"],
        "step_pct_hbm_roofline": head["step_pct_hbm_roofline"],
        "phase_ms": {k: round(v, 5) for k, v in ex["phases"].items()},
        "D_final": [round(float(d), 6) for d in ex["D"]],
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(traffic_key, args.storage) if traffic_key else None,
            "kernel": kernel,
            "algorithmic_bytes_per_launch": algo,
            "kernel_us": round(ex["k1_ms"] * 1e3, 2),
            "launches_timed": args.profile_steps,
        },
    }
    for k in ("unbatched_mlups", "batched_speedup"):
        if k in head:
            out[k] = head[k]
    if not args.no_legs and args.workload == "c3" and args.storage == "fp32":
        # the comparisons the metric names, timed the same way: FP16
        # population storage on the same workload, and the batched sweep with
        # FP32 and FP16 storage (aggregate over its 64 runs)
        legs = {}
        legs["c3_fp16"], _ = single_leg(args, "c3", "fp16", roofline=False)
        legs["c4_batched_fp32"], _ = batch_leg(args, "fp32")
        legs["c4_batched_fp16"], _ = batch_leg(args, "fp16")
        out["legs"] = legs
    out["wall_s"] = round(time.perf_counter() - t_wall, 1)
    if not args.no_cpu_baseline:
        base_wl = ex["wls"][0] if args.workload == "c4" else ex["wl"]
        out["cpu_baseline"] = cpu_baseline(base_wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def run_sensitivity(args):
    """Seconds for the gradient of the Taylor deformation D(T) with respect to
    (k_s, C, gamma): by the adjoint (one forward run with checkpoints and one
    reverse sweep) and by the tangent model (one primal + tangent run per
    parameter), T = --steps, next to the FP64 oracle's six central-difference
    runs (timed on a bounded sample of oracle steps and scaled to 6 T)."""
    import numpy as np
    import torch
    from paper_1004_2416_amd import binding as B
    from paper_1004_2416_amd import workloads as W

    wl = W.config(args.workload)
    cap = wl.capsules[0]
    mesh = B.icosphere(cap.level, cap.r, cap.center)
    gamma = 2.0 * wl.u_w / wl.nz
    dirs = {"ks": ([1.0], [cap.ka / cap.ks], 0.0, False, cap.ks),
            "C": ([0.0], [cap.ks], 0.0, False, cap.ka / cap.ks),
            "gamma": ([0.0], [0.0], wl.nz / 2.0, True, gamma)}
    grads, t_total = {}, 0.0
    for which, (dks, dka, duw, prof, p) in dirs.items():
        lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
        lat.set_shear(wl.u_w, init_profile=True)
        lat.add_capsules([mesh], [cap.ks], [cap.ka], wl.m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.attach_tangent(dks, dka, duw, init_profile=prof)
        lat.step(args.steps)
        grads[which] = float(lat.tangent_observables(1e-6 * p)[0, 4])
        t_total += time.perf_counter() - t0
        D = float(lat.observables()[0, 4])
        lat.close()
    # the reverse sweep: all three at once from one adjoint run
    lat = B.Lattice(wl.nx, wl.ny, wl.nz, wl.tau)
    lat.set_shear(wl.u_w, init_profile=True)
    lat.add_capsules([mesh], [cap.ks], [cap.ka], wl.m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = lat.adjoint_gradient(args.steps, checkpoint_every=100, couette_start=True)
    t_adj = time.perf_counter() - t0
    lat.close()
    adj = {"ks": g["dks"][0] + (cap.ka / cap.ks) * g["dka"][0], "C": cap.ks * g["dka"][0],
           "gamma": 0.5 * wl.nz * g["duw"]}
    out = {"metric": "seconds per gradient of D(T) w.r.t. (k_s, C, gamma)", "value": round(t_adj, 3),
           "unit": "s", "n_gpus": 1, "steps": args.steps, "higher_is_better": False,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl.name, "method": "adjoint (one reverse sweep, checkpoints "
                      "every 100 steps); tangent-linear (one pass per parameter) beside it"},
           "D_T": D, "dD_dp_adjoint": adj, "dD_dp_tangent": grads,
           "tangent_seconds": round(t_total, 3)}
    if not args.no_cpu_baseline:
        base = cpu_baseline(wl, args.cpu_seconds)
        per_step = wl.n_nodes_lattice / (base["value"] * 1e6)
        out["cpu_baseline"] = {"value": round(6 * args.steps * per_step, 1), "unit": "s",
                               "cores": base["cores"], "kind": "oracle",
                               "sample": "six FP64 oracle runs of %d steps (central differences), "
                                         "scaled from %s" % (args.steps, base["sample"])}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
