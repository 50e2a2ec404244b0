#!/usr/bin/env python3
"""Throughput of the particle-side hot path on one MI355X.

A step is one DEM step of the whole path over the 2,000,000-parcel
polydisperse cylindrical fixed bed: contact detection over the Verlet candidates,
soft-sphere parcel/wall forces, drag and integration every step; the
neighbour rebuild (cell sort + LDS-staged candidate scan), voidage/drag
deposition and the shrinking-core reaction update with its cell and bed
reductions every 20 steps (one coupling interval, dt_CFD = 20 dt_DEM), all
replayed from a HIP graph.  Inputs are generated on the host, uploaded, and
resident in HBM before the timed region.

The generated bed starts as loose lattice layers without contacts; before
anything is timed it is settled under gravity for 20,000 DEM steps (0.1 s of
bed time, neighbour lists rebuilt every 10 steps during the settling) into a
packed bed with about five contacts per parcel, whose state then seeds the
timed run.  --save-settled / --settled keep that state in a file so that a
profiled run can skip the settling.

Prints one JSON line (metric particle-steps/s) with the roofline of the
dominant kernel (the fused DEM step) and the oracle's CPU throughput on a
bounded sample of the same bed.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def step_bytes(z_mean):
    """Algorithmic HBM bytes of one parcel-step of the fused DEM-step kernel
    (mixed precision): read x (24 B), v and w (24 B), d and m (8 B); write x,
    v, w (48 B); read and write the 16 B tangential-spring record of each of
    the z/2 contact pairs of a parcel (16 z B)."""
    return 104.0 + 16.0 * z_mean


def traffic_from_profile(kernel_src):
    """HBM bytes per launch measured by rocprofv3 counters for the current
    source of the step kernel, or None if the kernel changed since."""
    path = os.path.join(ROOT, "profiles", "k_step_cfg3_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != h:
        return None
    return rec.get("bytes_per_launch")


SETTLE_STEPS = 20_000


def settle(w, steps, log=True):
    """The bed after `steps` DEM steps under gravity (coupling every
    couple_every steps), as a new workload with the same parameters."""
    import dataclasses

    from paper_2311_03908_amd.bed import Bed

    S = w.couple_every
    ws = dataclasses.replace(w, params={**w.params, "check_every": 10})
    bed = Bed(ws, device="cuda:0")
    t0 = time.perf_counter()
    bed.run(steps // S, S)
    bed.sync()
    st = bed.stats()
    s = bed.state()
    if log:
        _log(f"[bench] settled {steps} steps in {time.perf_counter() - t0:.1f} s: "
             f"{st['mean_coordination']:.2f} contacts per parcel")
    p = dict(w.parcels)
    for k in ("x", "y", "z", "vx", "vy", "vz", "wx", "wy", "wz", "nh", "nm", "nw", "nfe"):
        p[k] = s[k].double().cpu().numpy()
    bed.close()
    return dataclasses.replace(w, parcels=p)


STATE_KEYS = ("x", "y", "z", "vx", "vy", "vz", "wx", "wy", "wz", "nh", "nm", "nw", "nfe")


def save_state(w, path):
    import numpy as np

    np.savez(path, **{k: w.parcels[k] for k in STATE_KEYS})


def load_state(w, path):
    import dataclasses

    import numpy as np

    z = np.load(path)
    p = dict(w.parcels)
    for k in STATE_KEYS:
        if z[k].shape != p[k].shape:
            raise ValueError(f"{path}: state of {z[k].shape[0]} parcels, workload has {p[k].shape[0]}")
        p[k] = np.ascontiguousarray(z[k], dtype=np.float64)
    return dataclasses.replace(w, parcels=p)


def bench_batched(log=True):
    """64 beds of uneven size and temperature (the batched workload): one
    context holding all beds, 1,000 steps replayed from one HIP graph, against
    the plain loop running each bed in a context of its own, both autotuned."""
    import torch

    from paper_2311_03908_amd import workloads as W
    from paper_2311_03908_amd.bed import Bed

    w = W.cfg5()
    S = w.couple_every
    n_int = 1000 // S

    def timed(wk):
        bed = Bed(wk, device="cuda:0")
        bed.autotune()
        bed.run(2, S)
        bed.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bed.run(n_int, S)
        bed.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bed.close()
        return dt

    t_batch = timed(w)
    t_loop = 0.0
    for b in range(len(w.beds)):
        t_loop += timed(W.split_bed(w, b))
    if log:
        _log(f"[bench] batched: {len(w.beds)} beds, {w.n} parcels: one context {t_batch:.3f} s, "
             f"per-bed loop {t_loop:.3f} s")
    return {"beds": len(w.beds), "parcels": w.n, "steps": n_int * S, "batched_s": t_batch, "per_bed_loop_s": t_loop,
            "speedup": t_loop / t_batch, "particle_steps_per_s": w.n * n_int * S / t_batch}


def bench_adjoint(log=True):
    """Kinetic gradient of the 500,000-parcel bed over 20,000 reaction
    substeps (dt_react 1e-4 s, one DEM step per 10 substeps, checkpoints every
    500, FP32 state, FP64 adjoint accumulation): one dem_grad call against the
    12 plain forward runs of central finite differences (h = 1e-4 relative)
    in the same precision on the same GPU.  The gradient is checked against
    central differences of FP64-state forward runs (FP32 round-off would
    swamp differences of that step), each component relative to the largest
    component of its kind (ln k0 or E_a)."""
    import numpy as np

    from paper_2311_03908_amd import workloads as W
    from paper_2311_03908_amd.bed import Bed

    w = W.cfg4()
    spec = W.grad_spec_cfg4()
    args = (spec["n_substeps"], spec["dt_react"], spec["dyn_every"], spec["ckpt_every"])
    th = np.array(W.THETA_HEMATITE_FIT)
    bed = Bed(w, device="cuda:0")
    bed.grad(200, spec["dt_react"], spec["dyn_every"], spec["ckpt_every"], th, state_fp32=True)  # allocate
    t0 = time.perf_counter()
    J, g = bed.grad(*args, th, state_fp32=True)
    t_grad = time.perf_counter() - t0

    def central(fp32):
        fd = np.zeros(6)
        for q in range(6):
            h = 1e-4 * abs(th[q])
            Jq = []
            for sgn in (1.0, -1.0):
                tq = th.copy()
                tq[q] += sgn * h
                Jq.append(bed.grad(*args, tq, state_fp32=fp32, with_grad=False)[0])
            fd[q] = (Jq[0] - Jq[1]) / (2 * h)
        return fd

    t0 = time.perf_counter()
    central(True)
    t_fd = time.perf_counter() - t0
    fd64 = central(False)
    bed.close()
    sk = np.max(np.abs(fd64[0::2]))
    se = np.max(np.abs(fd64[1::2]))
    scale = np.array([sk, se, sk, se, sk, se])
    err = float(np.max(np.abs(g - fd64) / scale))
    if log:
        _log(f"[bench] adjoint: J={J:.6f} grad {t_grad:.2f} s, 12 forwards {t_fd:.2f} s, "
             f"max deviation from FP64 central differences {err:.2e}")
    return {"parcels": w.n, "substeps": spec["n_substeps"], "J": J, "grad": g.tolist(), "fd_grad_f64": fd64.tolist(),
            "grad_s": t_grad, "fd_12_forwards_s": t_fd, "speedup": t_fd / t_grad, "max_dev_from_fd": err,
            "state": "f32", "accumulation": "f64"}


def bench_sweep(log=True):
    """Kinetic sweep over Bed I / Bed II shaped beds (seven beds, 1.5 M
    parcels, one context): 500 DEM steps replayed from the graph (coupling
    every 20), then a 600 s fast-forward of the reaction in 1 s updates with
    the bed frozen, recording each bed's reduction degree every second."""
    import numpy as np
    import torch

    from paper_2311_03908_amd import workloads as W
    from paper_2311_03908_amd.bed import Bed

    w = W.sweep()
    S = w.couple_every
    bed = Bed(w, device="cuda:0")
    bed.autotune()
    bed.run(5, S)
    bed.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bed.run(25, S)
    bed.sync()
    torch.cuda.synchronize()
    t_dem = time.perf_counter() - t0
    curves = []
    t0 = time.perf_counter()
    for _ in range(600):
        curves.append(bed.react(1.0, keys=(), fov=False)["bed_fov"])
    torch.cuda.synchronize()
    t_react = time.perf_counter() - t0
    bed.close()
    c = np.array(curves)
    t90 = [float(np.argmax(c[:, b] >= 0.9) + 1) if np.any(c[:, b] >= 0.9) else None for b in range(c.shape[1])]
    labels = [f"Bed {k} {T:.0f} K k0=({np.exp(th[0]):.4g},{np.exp(th[2]):.4g},{np.exp(th[4]):.4g})"
              for k, T, _, th in W.SWEEP_BEDS]
    if log:
        _log(f"[bench] sweep: {len(w.beds)} beds, {w.n} parcels: 500 DEM steps {t_dem:.3f} s, "
             f"600 reaction updates {t_react:.3f} s; f_ov at 60 s {np.round(c[59], 3).tolist()}")
    return {"beds": labels, "parcels": w.n, "dem_particle_steps_per_s": w.n * 25 * S / t_dem,
            "react_parcel_updates_per_s": w.n * 600 / t_react, "fov_60s": c[59].tolist(),
            "fov_300s": c[299].tolist(), "fov_600s": c[599].tolist(), "t90_s": t90}


def bench_fluidized(w, S, steps=2000, warm=2000, log=True):
    """The settled 2M-parcel bed under its described gas: 0.3 m/s upflow with
    a +-10 % seeded perturbation per cell, 90 % H2 and N2 at 1073 K
    (workloads.fluidized).  The frozen upflow exceeds the terminal velocity
    of the finer real particles, so the bed expands and the neighbour lists
    are rebuilt on the device as the parcels move.  warm steps from the
    settled state, then steps timed (graph replay with all sources), with
    the number of rebuilds in the timed steps."""
    import torch

    from paper_2311_03908_amd import workloads as W
    from paper_2311_03908_amd.bed import Bed

    wf = W.fluidized(w)
    bed = Bed(wf, device="cuda:0")
    bed.autotune()
    bed.run(warm // S, S, sources=True)
    bed.sync()
    torch.cuda.synchronize()
    st0 = bed.stats()
    t0 = time.perf_counter()
    bed.run(steps // S, S, sources=True)
    bed.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = bed.stats()
    bed.close()
    rb = st["rebuilds"] - st0["rebuilds"]
    if log:
        _log(f"[bench] fluidized: {steps} steps in {dt:.3f} s, {rb} rebuilds, {st['mean_coordination']:.2f} contacts "
             f"per parcel")
    return {"workload": "the settled 2M-parcel bed at 0.3 m/s (+-10 %) upflow of 90 % H2 + N2, 1073 K",
            "warm_steps": warm, "steps": steps, "particle_steps_per_s": w.n * steps / dt, "ms_per_step": 1e3 * dt / steps,
            "rebuilds": rb, "checks": steps // st["check_period"], "mean_coordination": st["mean_coordination"]}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, S):
    """The oracle as it stands, built -O3 -march=native for this host, on the
    full bed: one DEM step plus one coupling (deposit with drag sums, reaction
    with cell sources) amortised over S steps, first on one thread, then on
    every thread OpenMP is given (OMP_NUM_THREADS, else all cores).  The two
    runs start from the same state and must give bit-identical results."""
    import tempfile

    import numpy as np

    from oracle import oracle as O

    path = os.path.join(tempfile.mkdtemp(prefix="ora_native_"), "libora_native.so")
    O.build_native(path)
    O.use_library(path)
    all_threads = O.host_threads()

    def one(threads):
        O.set_threads(threads)
        ora = O.Oracle(w)
        t0 = time.perf_counter()
        ora.step(1)
        t1 = time.perf_counter()
        c = ora.couple()
        r = ora.react(S * w.params["dt"])
        t2 = time.perf_counter()
        st = ora.state()
        res = [st[k] for k in ("x", "y", "z", "vx", "vy", "vz", "nh")] + [c["sumK"], r["sumEQ"], r["fov"]]
        del ora
        return t1 - t0, t2 - t1, res

    _log("[bench] cpu baseline: oracle, one thread")
    s1, c1, r1 = one(1)
    _log(f"[bench] cpu (1 thread): step {s1:.2f} s, coupling {c1:.2f} s")
    _log(f"[bench] cpu baseline: oracle, {all_threads} threads")
    sn, cn, rn = one(all_threads)
    _log(f"[bench] cpu ({all_threads} threads): step {sn:.2f} s, coupling {cn:.2f} s")
    same = all(np.array_equal(a, b) for a, b in zip(r1, rn))
    rate1 = w.n / (s1 + c1 / S)
    raten = w.n / (sn + cn / S)
    return {"value": raten, "unit": "particle-steps/s", "cores": all_threads, "kind": "oracle",
            "sample": f"full {w.n}-parcel bed: 1 DEM step + 1 coupling (deposit with drag sums, reaction with cell "
                      f"sources) amortised over {S} steps; oracle built -O3 -march=native -ffp-contract=off",
            "single_thread_value": rate1, "nproc": os.cpu_count(),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"), "cpu_model": _cpu_model(),
            "identical_to_single_thread": bool(same)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=120)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=None, help="parcel count (default: the 2M-parcel bed)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of 512 MiB three times (for counter scaling)")
    ap.add_argument("--settle-steps", type=int, default=SETTLE_STEPS)
    ap.add_argument("--save-settled", default=None, help="settle the bed, save its state (.npz) and exit")
    ap.add_argument("--settled", default=None, help="start from a state saved by --save-settled")
    ap.add_argument("--launch", default=None, metavar="B,X,G",
                    help="fixed launch shapes (step block, XCD chunk, build grid) instead of autotuning")
    ap.add_argument("--build", default=None, metavar="T,L,W",
                    help="with --launch: neighbour-build threads per block, LDS tile and item width")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (64-bed), adjoint (500k-parcel gradient) and kinetic-sweep legs")
    ap.add_argument("--skin", type=float, default=None, help="neighbour-list skin (m) of the timed run")
    ap.add_argument("--check-every", type=int, default=None, help="steps between neighbour-list checks")
    ap.add_argument("--only", choices=["batched", "adjoint", "sweep", "fluidized"], default=None,
                    help="run only one speedup leg and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2311_03908_amd import workloads as W
    from paper_2311_03908_amd.bed import Bed

    if args.only and args.only != "fluidized":
        leg = {"batched": bench_batched, "adjoint": bench_adjoint, "sweep": bench_sweep}[args.only]
        print(json.dumps(leg()), flush=True)
        return
    if args.copy_calibration:
        src = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log("[bench] copy calibration: 3 x 512 MiB read + 512 MiB write")
        del src, dst
    _log("[bench] generating workload")
    w = W.cfg3() if args.n is None else W.cfg3(n=args.n)
    if args.settled:
        w = load_state(w, args.settled)
        _log(f"[bench] state from {args.settled}")
    elif args.settle_steps > 0:
        w = settle(w, args.settle_steps)
    if args.save_settled:
        save_state(w, args.save_settled)
        _log(f"[bench] saved settled state to {args.save_settled}")
        return
    if args.skin is not None:
        w.params["skin"] = args.skin
    if args.check_every is not None:
        w.params["check_every"] = args.check_every
    S = w.couple_every
    if args.only == "fluidized":
        print(json.dumps(bench_fluidized(w, S)), flush=True)
        return
    # whole coupling intervals: the timed steps are the requested count rounded
    # down to a multiple of the coupling interval (at least one interval), the
    # warm-up rounded up
    n_int = max(1, args.steps // S)
    steps = n_int * S
    warm_int = max(1, -(-args.warmup // S))
    warm = warm_int * S
    _log(f"[bench] n={w.n} steps={steps} warmup={warm}")
    bed = Bed(w, device="cuda:0")
    if args.launch:
        bed.set_launch(*[int(v) for v in args.launch.split(",")])
        if args.build:
            bed.set_build(*[int(v) for v in args.build.split(",")])
    else:
        bed.autotune()
    bed.run(warm_int, S, sources=True)
    bed.sync()
    torch.cuda.synchronize()
    st0 = bed.stats()
    _log("[bench] timed region")
    t0 = time.perf_counter()
    bed.run(n_int, S, sources=True)
    bed.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = bed.stats()
    elapsed = t1 - t0
    rate = w.n * steps / elapsed
    z = st["mean_coordination"]
    rebuilds = st["rebuilds"] - st0["rebuilds"]
    # the step kernel's duration: one more interval after the timed region,
    # launched eagerly on the same stream with HIP events around each step
    # kernel (events recorded inside replayed graphs report no time)
    bed.profile(True)
    bed.step(S)
    bed.couple()
    bed.react(S * w.params["dt"], fov=False)
    k_ms = bed.stats()["step_kernel_ms"]
    k_launches = bed.stats()["step_kernel_launches"]
    bed.profile(False)
    bpu = step_bytes(z)
    achieved = w.n * bpu / (k_ms * 1e-3) / 1e9 if k_ms > 0 else None
    traffic = traffic_from_profile(os.path.join(ROOT, "paper_2311_03908_amd", "csrc", "k_step.hip"))
    _log(f"[bench] {rate:.4e} particle-steps/s, step kernel {k_ms * 1e3:.1f} us, z={z:.3f}, rebuilds {rebuilds}")
    out = {
        "metric": "particle-steps/s",
        "value": rate,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "polydisperse cylindrical fixed bed: 2,000,000 parcels, lognormal d_p (median "
                               "100 um, sigma 0.3), k=5, 2 ore types, 100x600 mm cylinder, 64x64x384 gas grid, "
                               "H2 at 1073 K, dt=5e-6 s, coupling every 20 steps, settled under gravity",
                   "parcels": w.n, "couple_every": S, "graph": n_int >= 2, "sources": "all (eps, drag sums, "
                   "species sources) every coupling", "rebuilds_timed": rebuilds,
                   "settle_steps": 0 if args.settled else args.settle_steps, "skin": w.params["skin"],
                   "check_every": w.params["check_every"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                     "kernel": "k_step (fused contact + drag + integrate)", "bytes_per_parcel_step": bpu,
                     "kernel_ms": k_ms, "launches_timed": k_launches, "z_mean": z,
                     "launch": {"step_block": st["step_block"], "step_xcd_chunk": st["step_xcd"],
                                "build_grid": st["build_grid"], "check_period": st["check_period"]}},
    }
    bed.close()
    if not args.no_extras:
        out["fluidized"] = bench_fluidized(w, S)
        out["batched"] = bench_batched()
        out["adjoint"] = bench_adjoint()
        out["sweep"] = bench_sweep()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, S)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
