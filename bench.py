#!/usr/bin/env python3
"""Throughput of the fused D2Q9-MRT + D2Q5 step on one MI355X.

Workload: the 8192 x 8192 annulus of the throughput problem (R* = 2,
Ra = 1e6, Da = 1e-3, Pr = 1, seeded Gaussian random porosity field, Ergun
Forchheimer coefficient), cold start, residual and wall-Nusselt check every
100 steps.  One bench step = one time step of the whole lattice (all of the
fused update, plus the check every 100 steps).  Inputs are resident in HBM
before the timed region starts.

Prints one JSON line: MLUPS (million node updates per second, one node = both
lattices), the HBM roofline of the step kernel (algorithmic bytes per launch
over its average duration from HIP events on the library's stream) and the
FP64 CPU oracle timed on a bounded sample of the same problem (all host
threads and one).  Also on the line: the same job with its host hand-overs
(create, field read-back), the FP16 and BF16 storage variants, the
1024-instance batched sweep, and the time to steady state of 64 held-out
128^2 problems from a cold start, from the learned warm start and from the
conduction-profile start.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (fused D2Q9+D2Q5) & % HBM roofline; time-to-steady warm vs cold start"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic_8192.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1409_5929_amd", "csrc", f)
                  for f in ("lbm_axi.hip", "lbm_axi_s16.hip", "lbm_axi_kernels.h", "lbm_axi_dev.h",
                            "lbm_axi_desc.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str):
    """HBM bytes per step-kernel launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(storage)
    if not e or t.get("source_sha") != kernel_source_sha():
        return None
    return e["bytes_per_launch"]


def device_copy_gbs(torch, stream, nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Bandwidth of a plain device-to-device copy on the same stream (bytes
    read plus bytes written per second): what streaming code reaches here."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    with torch.cuda.stream(stream):
        dst.copy_(src)
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dst.copy_(src)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2 * nbytes / (best * 1e-3) / 1e9


def storage_variant(Lattice, cfg, phi, storage, steps, warmup, check, stream):
    """The same 8192^2 problem with 16-bit population storage (FP32 arithmetic):
    MLUPS and the step kernel's algorithmic bandwidth (64 B per node)."""
    import torch

    n = cfg["nr"]
    lat = Lattice(cfg, phi=phi, storage=storage, check_interval=check, stream=stream.cuda_stream)
    lat.step(warmup)
    lat.set_timing(True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    kern_ms, launches = lat.kernel_time()
    lat.set_timing(False)
    pat = pattern_ceiling(lat)
    lat.close()
    bpn = 26 * 2 + 2 * 4 + 4
    achieved = (n - 2) ** 2 * bpn / (kern_ms / launches * 1e-3) / 1e9
    return {"storage": storage, "steps": steps, "warmup": warmup,
            "mlups": round(n * n * steps / (total_ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(total_ms / steps, 5), "avg_launch_ms": round(kern_ms / launches, 5),
            "bytes_per_node": bpn, "achieved_gbs": round(achieved, 1),
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            # against the 56 + 2 bytes per node of 16-bit populations and a 16-bit
            # porosity, which this layout exceeds (FP32 g_0 and porosity planes)
            "frac_at_58_bytes": round(achieved * 58 / bpn / HBM_PEAK_GBS, 4),
            "pattern_ceiling_gbs": pat, "frac_of_pattern": round(achieved / pat["pair"], 4)}


def pattern_ceiling(lat, reps: int = 20) -> dict:
    """The step's own access pattern without arithmetic on the same handle
    (lbm_axi_pattern_bandwidth): even and odd parity, their pair (harmonic mean:
    a step pair moves the same bytes in each), a plain read+write stream, and
    that stream at 2, 4, 8 and 16 bytes per lane (lbm_axi_lane_bandwidth)."""
    r = lat.pattern_bandwidth(reps=reps)
    pair = 2.0 / (1.0 / r["even_gbs"] + 1.0 / r["odd_gbs"])
    lanes = lat.lane_bandwidth(reps=max(reps // 2, 1))  # in-place stream, bytes per lane
    return {"even": round(r["even_gbs"], 1), "odd": round(r["odd_gbs"], 1), "pair": round(pair, 1),
            "stream_rw": round(r["stream_gbs"], 1), "reps": reps,
            "lane_stream_gbs": {f"{w}B": round(v, 1) for w, v in lanes.items()}}


def sweep_batch(Lattice, n_inst, steps, stream):
    """The batched parameter sweep: n_inst annuli of uneven grids and
    parameters in one handle, FP16 storage, launch shape from the autotuner,
    step graphs; aggregate MLUPS over a fixed number of steps."""
    import numpy as np
    import torch

    import lbm_inputs as li

    cfgs = li.sweep(n_inst=n_inst, seed=1409)
    nodes = int(sum(c["nr"] * c["nz"] for c in cfgs))
    fluid = int(sum((c["nr"] - 2) * (c["nz"] - 2) for c in cfgs))
    t0 = time.perf_counter()
    lat = Lattice(cfgs, storage="fp16", check_interval=1000, tol=1e-8, max_steps=2_000_000,
                  stream=stream.cuda_stream)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    tune = lat.autotune(trial_steps=10)
    lat.step(2 - lat.info()["t"] % 2)  # graphs start at even levels
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = lat.residual()["status"]
    lat.close()
    bpn = 26 * 2 + 2 * 4
    return {"instances": n_inst, "nodes": nodes, "storage": "fp16", "steps": steps,
            "mlups": round(nodes * steps / (ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(ms / steps, 5),
            "achieved_gbs": round(fluid * bpn / (ms / steps * 1e-3) / 1e9, 1),
            "bytes_per_node": bpn,
            "autotune": {"kz": tune["kz"], "blocks_per_cu": tune["blocks_per_cu"],
                         "step_ms": round(tune["ms"], 5)},
            "create_s": round(t_create, 2),
            "status_counts": {k: int(np.sum(st == v)) for k, v in
                              (("running", 0), ("converged", 1), ("diverged", 2), ("stalled", 3))}}


def sweep_to_steady(n_inst, cap, chunk=10_000, floor=3e-7, subset=(0, 1), start="conduction"):
    """The batched sweep run toward res <= 1e-8 with autotuned launches, step
    graphs and finished instances dropped from the launch after every chunk,
    up to `cap` steps.  It starts in FP16 storage, whose rounding noise keeps
    the residual near 1e-7 at a check interval of 1000, and converts the
    whole batch to FP32 in place (precision handoff) once half of the running
    instances are within 3x of that floor.  subset = (i, n) runs instances
    i, i + n, ... of the sweep in one handle (a whole sweep in n calls);
    start = "conduction" starts every instance at rest with its radial
    conduction profile of T, "cold" at rest at T_init.  Counts of converged /
    stalled / diverged instances, steps of the converged ones, node updates
    per second, and every instance's index, final state and own step count."""
    import numpy as np
    import torch

    import lbm_inputs as li
    from paper_1409_5929_amd import Lattice
    from paper_1409_5929_amd import warmstart as ws

    every = li.sweep(n_inst=n_inst, seed=1409)
    index = list(range(subset[0], n_inst, subset[1]))
    cfgs = [every[i] for i in index]
    n_run = len(cfgs)
    init = [ws.conduction_start(c) for c in cfgs] if start == "conduction" else None
    sizes = np.array([c["nr"] * c["nz"] for c in cfgs], dtype=np.float64)
    lat = Lattice(cfgs, init=init, storage="fp16", check_interval=1000, tol=1e-8, max_steps=cap)
    lat.autotune(trial_steps=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = lat.info()["t"]
    updates = 0.0
    running = n_run
    t_handoff = None
    while t < cap + 1000 and running > 0:
        r = lat.residual()
        alive = sizes[r["status"] == 0].sum()
        if t_handoff is None and t > 0:
            res_run = r["res"][r["status"] == 0]
            if res_run.size and np.mean(res_run < floor) >= 0.5:
                lat.set_storage("fp32")
                lat.autotune(trial_steps=10)  # FP32 prefers other launch shapes; 150 real steps
                t += 15 * 10
                t_handoff = t
                log(f"sweep to steady: FP16 -> FP32 at t={t}")
        lat.step(chunk)
        t += chunk
        updates += alive * chunk  # upper bound within the chunk: instances that stop mid-chunk
        running = lat.compact()
        log(f"sweep to steady: t={t}, {running} of {n_run} running, {time.perf_counter() - t0:.0f} s")
    lat.sync()
    wall = time.perf_counter() - t0
    r = lat.residual()
    steps = np.array([lat.info(i)["t"] for i in range(n_run)])
    lat.close()
    st = r["status"]
    conv = st == 1
    return {"instances": n_run, "of": n_inst, "subset": list(subset), "start": start, "cap": cap,
            "wall_s": round(wall, 1),
            "converged": int(conv.sum()), "stalled": int((st == 3).sum()), "diverged": int((st == 2).sum()),
            "running": int((st == 0).sum()), "handoff_step": t_handoff,
            "steps_converged_median": float(np.median(steps[conv])) if conv.any() else None,
            "node_updates_per_s_upper": round(updates / wall / 1e6, 1),
            "index": index, "status": [int(v) for v in st], "steps": [int(v) for v in steps],
            "res": [float(v) for v in r["res"]]}


def time_to_steady(n_problems, cap):
    """Time to steady state of 128^2 annuli of the sweep distribution
    (held-out problems of the warm-start network's training run): cold start,
    the network's predicted start and the non-learned conduction-profile
    start (fluid at rest, T = ln(r_o / r) / ln R*), each run to the stopping
    rule of the warm-start runs (res <= 1e-8 and an extrapolated remaining
    change <= 1e-4).  Steps and Nu are compared over the problems that
    converge from all three starts; wall times of those problems alone are
    taken in separate batches (the warm one includes the prediction)."""
    import numpy as np
    import torch

    from paper_1409_5929_amd import warmstart as ws
    from paper_1409_5929_amd.no import WarmStartNet

    cfgs = ws.held_out(n_problems)
    net = WarmStartNet(ws.WIDTHS, ws.GRID, ws.GRID, 32, ws.load_weights(ws.WEIGHTS))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = ws.predict(net, cfgs)
    t_pred = time.perf_counter() - t0
    net.close()
    cond_init = [ws.conduction_start(c) for c in cfgs]
    cold = ws.solve(cfgs, max_steps=cap, fields=False)
    warm = ws.solve(cfgs, init=list(pred), max_steps=cap, fields=False)
    cond = ws.solve(cfgs, init=cond_init, max_steps=cap, fields=False)
    ok = (cold["status"] == 1) & (warm["status"] == 1) & (cond["status"] == 1)
    out = dict(problems=n_problems, grid=ws.GRID, tol=ws.TOL, tail_tol=ws.TAIL_TOL, max_steps=cap,
               train_problems=ws.weights_meta()["train_problems"],
               converged_cold=int((cold["status"] == 1).sum()), converged_warm=int((warm["status"] == 1).sum()),
               converged_conduction=int((cond["status"] == 1).sum()), predict_s=round(t_pred, 3),
               warm_vs_cold=ws.compare(cold, warm, ok), conduction_vs_cold=ws.compare(cold, cond, ok),
               warm_vs_conduction=ws.compare(cond, warm, ok))
    sel = [i for i in range(n_problems) if ok[i]]
    if sel:
        sub = [cfgs[i] for i in sel]
        c_sub = ws.solve(sub, max_steps=cap, fields=False)
        w_sub = ws.solve(sub, init=[pred[i] for i in sel], max_steps=cap, fields=False)
        d_sub = ws.solve(sub, init=[cond_init[i] for i in sel], max_steps=cap, fields=False)
        out.update(wall_cold_s=round(c_sub["wall"], 3), wall_warm_s=round(w_sub["wall"] + t_pred, 3),
                   wall_conduction_s=round(d_sub["wall"], 3))
    return out


def check_summary(res, info, interval):
    """The last residual / Nusselt check of the main run: its step, residual and
    Nu_i, or a note when no check fell in the run (a check compares two check
    steps, the first at level 0, so the first one runs at level `interval`)."""
    t_check = int(info["t_check"])
    if t_check < 0 or not math.isfinite(float(res["res"][0])):
        return {"t_check": None, "residual": None, "nu_i": None,
                "note": f"no check in this run (checks at multiples of {interval} steps from "
                        f"level {interval} on; run ended at level {int(info['t'])})"}
    return {"t_check": t_check, "residual": float(res["res"][0]), "nu_i": float(res["nu_i"][0])}

def oracle_rate(cfg: dict, phi, seconds: float):
    """Steps of the FP64 oracle on (cfg, phi) until `seconds` of work are done:
    (steps, seconds, threads used)."""
    import oracle

    oracle.build(force=False)
    o = oracle.Oracle(cfg, phi_field=phi)
    o.step(1)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds and n >= 2:
            break
    o.close()
    return n, dt, oracle.threads()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, phi, seconds: float):
    """The FP64 oracle on a 1024 x 1024 corner of the same problem (inner
    wall, bottom wall), stepped until `seconds` of work are done, with all the
    host threads OpenMP is given; then the same window on one thread, in a
    child process (the oracle's thread count is fixed once it is loaded)."""
    import tempfile

    import numpy as np

    w = 1024
    c = dict(cfg)
    c.update(nr=w, nz=w, side_rmax="wall", therm_rmax="adiabatic")
    win = np.ascontiguousarray(phi[:w, :w])
    n, dt, threads = oracle_rate(c, win, seconds)
    out = dict(value=w * w * n / dt / 1e6, unit="MLUPS", cores=threads, kind="oracle",
               sample=f"{w}x{w} corner window of the {cfg['nr']}x{cfg['nz']} problem "
                      f"(same physics and porosity field), {n} steps in {dt:.1f} s, FP64",
               cpu_model=cpu_model(), host_cpus=os.cpu_count())
    one_s = max(2.0, seconds / 3)
    with tempfile.TemporaryDirectory() as d:
        np.save(os.path.join(d, "phi.npy"), win)
        with open(os.path.join(d, "cfg.json"), "w") as f:
            json.dump(c, f)
        code = ("import json, os, sys, numpy as np, bench\n"
                "d = sys.argv[1]\n"
                "c = json.load(open(os.path.join(d, 'cfg.json')))\n"
                "n, dt, t = bench.oracle_rate(c, np.load(os.path.join(d, 'phi.npy')), float(sys.argv[2]))\n"
                "print(json.dumps([n, dt, t]))\n")
        env = dict(os.environ, OMP_NUM_THREADS="1")
        try:
            r = subprocess.run([sys.executable, "-c", code, d, str(one_s)],
                               cwd=os.path.dirname(os.path.abspath(__file__)), env=env,
                               capture_output=True, text=True, timeout=300)
        except subprocess.TimeoutExpired:
            r = subprocess.CompletedProcess([], 1, "", "timed out after 300 s")
    if r.returncode == 0:
        n1, dt1, t1 = json.loads(r.stdout.strip().splitlines()[-1])
        out["single_thread"] = dict(value=w * w * n1 / dt1 / 1e6, threads=t1,
                                    sample=f"same window, {n1} steps in {dt1:.1f} s")
    else:
        out["single_thread"] = None
        log(f"single-thread oracle run failed: {r.stderr.strip()[-300:]}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--check-interval", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP16/BF16 storage runs and the batched sweep")
    ap.add_argument("--sweep-instances", type=int, default=1024)
    ap.add_argument("--sweep-steps", type=int, default=1000)
    ap.add_argument("--steady-problems", type=int, default=64)
    ap.add_argument("--steady-max-steps", type=int, default=600_000)
    ap.add_argument("--sweep-to-steady", type=int, default=0, metavar="CAP",
                    help="only run the 1024-instance sweep toward res <= 1e-8 for up to CAP steps")
    ap.add_argument("--sweep-subset", default="0/1", metavar="I/N",
                    help="with --sweep-to-steady: run instances I, I+N, ... only")
    ap.add_argument("--sweep-start", default="conduction", choices=["conduction", "cold"],
                    help="with --sweep-to-steady: start of every instance")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only run the batched sweep (the --sweep-instances / --sweep-steps line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 2 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(one large problem would be cut into z-slabs with a halo exchange per step; "
              "batches would be split by instance); rerun with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lbm_inputs as li
    from paper_1409_5929_amd import Lattice

    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    if args.sweep_only:
        stream = torch.cuda.Stream()
        print(json.dumps({"sweep": sweep_batch(Lattice, args.sweep_instances, args.sweep_steps, stream)}),
              flush=True)
        return
    if args.sweep_to_steady > 0:
        i, n = (int(v) for v in args.sweep_subset.split("/"))
        if not 0 <= i < n:
            sys.exit("--sweep-subset I/N needs 0 <= I < N")
        print(json.dumps({"sweep_to_steady": sweep_to_steady(args.sweep_instances, args.sweep_to_steady,
                                                             subset=(i, n), start=args.sweep_start)}),
              flush=True)
        return
    n = args.size
    log(f"porosity field {n}x{n} (seed 1409)")
    cfg, _ = li.variable_porosity_annulus(n=n)
    phi = li.porosity_grf(n, n, seed=1409)
    log("create lattice")
    stream = torch.cuda.Stream()  # the library launches on this stream; events are recorded on it
    phi32 = phi.astype(np.float32)
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    lat = Lattice(cfg, phi=phi32, storage=args.storage,
                  check_interval=args.check_interval, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t_create
    log(f"warmup {args.warmup} steps")
    lat.step(args.warmup)
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log(f"timed {args.steps} steps")
    lat.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    kern_ms, launches = lat.kernel_time()
    lat.set_timing(False)
    res = lat.residual()
    info = lat.info()
    log("pattern ceiling probe")
    pattern = pattern_ceiling(lat)
    t_read = time.perf_counter()
    host_fields = lat.fields()  # u_z, u_r, p, T and node classes into host memory
    t_read = time.perf_counter() - t_read
    del host_fields
    lat.close()
    copy_gbs = device_copy_gbs(torch, stream)
    variants = sweep = steady = None
    if not args.no_variants and args.storage == "fp32":
        variants = []
        for st in ("fp16", "bf16"):
            # at least 100 warm-up and 200 timed steps, whatever the main leg's counts
            log(f"storage variant {st}")
            variants.append(storage_variant(Lattice, cfg, phi.astype(np.float32), st,
                                            max(args.steps // 2, 200), max(args.warmup, 100),
                                            args.check_interval, stream))
        log(f"batched sweep: {args.sweep_instances} instances")
        sweep = sweep_batch(Lattice, args.sweep_instances, args.sweep_steps, stream)
        log(f"time to steady: {args.steady_problems} problems, cold vs warm start")
        steady = time_to_steady(args.steady_problems, args.steady_max_steps)

    fluid = (n - 2) * (n - 2)
    # 14 populations read + 14 written, porosity read; g_0 stays FP32 in 16-bit storage
    bytes_node = 116 if args.storage == "fp32" else 26 * 2 + 2 * 4 + 4
    # launches that also write u_z, u_r, T for the check (one per check interval)
    t0 = args.warmup
    macro_launches = sum(1 for t in range(t0, t0 + args.steps)
                         if args.check_interval > 0 and t % args.check_interval == 0)
    alg_bytes = launches * fluid * bytes_node + macro_launches * 12 * n * n
    avg_ms = kern_ms / max(launches, 1)
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.storage)
    mlups = n * n * args.steps / (total_ms * 1e-3) / 1e6
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"annulus {n}x{n} (R*=2, Ra=1e6, Da=1e-3, Pr=1, seeded porosity field "
                        f"mean 0.6 sd 0.15 sigma 8 clipped [0.3,0.95], Ergun F_phi), cold start, "
                        f"check every {args.check_interval} steps",
            "nr": n, "nz": n, "storage": args.storage, "check_interval": args.check_interval,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_step (fused collide-stream, even and odd AA variants)",
            "bytes_per_node": bytes_node,
            "avg_launch_ms": round(avg_ms, 5),
            "launches": launches,
            "copy_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
            # the step's exact access pattern with no arithmetic, on the same handle
            "pattern_ceiling_gbs": pattern,
            "frac_of_pattern": round(achieved / pattern["pair"], 4),
        },
        # the same job with its host hand-overs: create (allocation, porosity
        # upload, start state) before and the field read-back after the steps
        "with_host_io": {
            "create_s": round(t_create, 3),
            "readback_s": round(t_read, 3),
            "mlups": round(n * n * args.steps / (t_create + total_ms * 1e-3 + t_read) / 1e6, 1),
        },
        "storage_variants": variants,
        "sweep": sweep,
        "time_to_steady": steady,
        "check": check_summary(res, info, args.check_interval),
        "t": int(info["t"]),
    }
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle, ~{args.cpu_seconds:.0f} s)")
        out["cpu_baseline"] = cpu_baseline(cfg, phi, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
