"""Benchmark of the coupled cascaded LB time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision fp64|fp32|fp16|bf16] [--no-cpu-baseline] [--extra]
                    [--batched] [--served] [--variants] [--stability]

One step = one fused stream-collide pass of both schemes (f and gbar) over
every node of the synthetic workload, inputs resident in HBM.  Prints ONE JSON
line: MLUPS (node updates per second / 1e6, f and gbar advanced one step each),
the roofline of the fused kernel (algorithmic bytes 36 * s per node / average
kernel duration from HIP events on the library's stream, against 8 TB/s) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1909_04166_amd import lb, workloads as W  # noqa: E402

METRIC = "MLUPS (f+g per node-step) & % HBM roofline; p50/p99 solve latency batched vs plain"

# HBM bytes per launch of the step kernel on the 8192^2 grid from two rocprofv3
# counter passes (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0 KiB, the factors read on the
# library's copy kernel; see profiles/lb_fused_pmc_tiled8192.md), with the workgroup
# schedule the autotuner chose in those runs (workgroup width, rows, grid, prefetch).
# They hold only for that schedule and for the code with this fingerprint (the
# step kernels, their instantiations and launchers, the work-list builder and the
# compiler flags); otherwise the roofline's traffic is null.
KERNEL_SOURCES = ["paper_1909_04166_amd/csrc/lb_device.hpp", "paper_1909_04166_amd/csrc/lb_kernels.hip",
                  "paper_1909_04166_amd/csrc/lb_sched.hpp"]
TRAFFIC = {
    "fingerprint": "c2a26308ecb6b848",
    "workload": "tiled8192",
    "fp64": {"read": 9737072640, "write": 9663729152, "tile": [516, 512, 256, 1]},
    "fp32": {"read": 4885437440, "write": 4831841792, "tile": [516, 512, 256, 1]},
    "fp16": {"read": 3045382144, "write": 2415920128, "tile": [452, 304, 512, 1]},
}


def _code_only(text: str, hash_comments: bool) -> str:
    """Source text without comments and blank space, so that rewording a comment
    does not invalidate the recorded counters ('//' and '/* */' in the C++ files,
    '#' in build.py; none of these files has such sequences inside a string)."""
    import re
    if hash_comments:
        text = re.sub(r"#[^\n]*", "", text)
    else:
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(" ".join(line.split()) for line in text.splitlines() if line.strip())


def kernel_fingerprint() -> str:
    """Hash of the code that builds the step kernel (comments excluded) and of
    the compiler flags."""
    import hashlib
    from paper_1909_04166_amd import build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read(), f.endswith(".py")).encode())
    h.update(" ".join(build.FLAGS).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, precision: str, tile) -> dict | None:
    """Counter-measured bytes per launch, or None when they do not apply (other
    workload, other schedule, or other kernel code)."""
    rec = TRAFFIC.get(precision)
    if (rec is None or workload != TRAFFIC["workload"] or list(tile) != rec.get("tile")
            or kernel_fingerprint() != TRAFFIC["fingerprint"]):
        return None
    return rec


HBM_PEAK_GBS = 8000.0
STORE = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def make_workload(name: str):
    """Returns (case, phi0, description)."""
    if name.startswith("tiled"):
        # 128^2 stationary droplet (R = 25, ratio 1000, sigma 0.01, W 5, M 0.02) tiled
        side = int(name[len("tiled"):] or 8192)
        t = side // 128
        case, phi0 = W.droplet(128, 25.0, W=5.0)
        case, phi0 = W.tiled(case, phi0, t, t)
        desc = (f"tiled stationary droplets {side}x{side} periodic ({t}x{t} tiles of 128^2, R=25, "
                f"rho ratio 1000, sigma 0.01, W 5, M 0.02)")
        return case, phi0, desc
    if name == "rt256":
        case, phi0 = W.config("rt256")
        return case, phi0, "Rayleigh-Taylor single mode 256x1024, walls in y, At 0.5, Re 3000"
    if name == "droplet128":
        case, phi0 = W.config("droplet128")
        return case, phi0, "stationary droplet 128x128 periodic, ratio 1000, W 4, M 0.02"
    if name == "droplet128_W5":
        case, phi0 = W.droplet(128, 25.0, W=5.0)
        return case, phi0, "stationary droplet 128x128 periodic, ratio 1000, W 5, M 0.02"
    if name == "thermo512":
        case, phi0 = W.config("thermo512")
        return case, phi0, "thermocapillary drop 512x256, walls in y, ratio 10"
    raise SystemExit(f"unknown workload {name}")


def time_lattice(case, phi0, precision, steps, warmup, tile=(0, 0), vel=None, keep_tile=0, sched=None):
    """Times `steps` steps after `warmup`; keep_tile > 0 also returns the fields
    (phi, p, ux, uy) of the first keep_tile x keep_tile block after the run and
    whether the last such block equals it bit for bit (read after the timed
    region)."""
    import torch
    L = lb.Lattice(case, phi0, precision, tile=tile)
    if sched is not None:  # pinned (width, mode, rows or multiplier, prefetch): no autotuning
        L.set_schedule(*sched)
    if vel is not None:
        L.set_velocity(*vel)
    L.step(warmup)
    torch.cuda.synchronize()
    lb.lb_timing_enable(L.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc = L.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_kernel, n = lb.lb_timing_read(L.h)
    lb.lb_timing_enable(L.h, False)
    d = L.diagnostics()
    tile_used = L.tile
    first = same = None
    if keep_tile:
        k = keep_tile
        fl = L.fields()
        first = tuple(np.array(f[:k, :k]) for f in fl)
        same = all(np.array_equal(f[:k, :k], f[-k:, -k:]) for f in fl)
        del fl
    L.close()
    del L
    torch.cuda.empty_cache()
    return dict(wall_s=t1 - t0, ms_kernel=ms_kernel, rc=rc, diag=d, tile=tile_used, first_tile=first,
                tiles_identical=same)




def bench_batched(precision: str, steps: int, n: int = 256, seed: int = 20190909, warmup: int = 160,
                  sched=None):
    """Uneven batch: n independent droplet / Rayleigh-Taylor lattices, sides in
    [64, 512], density ratio log-uniform in [3, 1000], W 5;
    one persistent launch per step.  The warm-up (autotuning, then 160 steps)
    passes the batch's graph gate (the work list unchanged for 128 steps), so the
    timed steps replay captured graphs.  MLUPS count every lattice; MLUPS_stable
    only those that end stable (no NaN/Inf, max |u| below 0.3), with their count."""
    import torch
    inst = W.batch_instances(n, seed)
    nodes = sum(c["nx"] * c["ny"] for _, c, _ in inst)
    B = lb.Batch(n, nodes + 64 * n, precision)
    for _, c, p in inst:
        B.add(c, p)
    if sched is not None:  # pinned (width, mode, rows or multiplier, prefetch): no autotuning
        B.set_schedule(*sched)
    B.step(warmup)  # autotune + warm-up
    torch.cuda.synchronize()
    g0, e0 = B.launch_counts()
    lb.lb_batch_timing_enable(B.b, True)
    t0 = time.perf_counter()
    B.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, _ = lb.lb_batch_timing_read(B.b)
    g1, e1 = B.launch_counts()
    bad = []
    for s in range(n):
        d = B.diagnostics(s)
        if d["nan_flag"] != 0.0 or not d["max_u"] < 0.3:
            bad.append(s)
    stable_nodes = nodes - sum(inst[s][1]["nx"] * inst[s][1]["ny"] for s in bad)
    sched = list(lb.lb_batch_get_schedule(B.b))
    B.close()
    return {"MLUPS": round(nodes * steps / wall / 1e6, 1),
            "MLUPS_stable": round(stable_nodes * steps / wall / 1e6, 1),
            "nodes": nodes, "instances": n, "unstable_instances": len(bad),
            "unstable_kinds": sorted({inst[s][0] for s in bad}),
            "steps": steps, "warmup": warmup, "graph_steps_timed": g1 - g0, "eager_steps_timed": e1 - e0,
            "kernel_ms": round(ms, 4), "schedule": sched,
            "kernel_GBs": round(36 * STORE[precision] * nodes / (ms * 1e-3) / 1e9, 1),
            "frac": round(36 * STORE[precision] * nodes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_served(precision: str, n_req: int, rate: float, budget_gb: float = 24.0, seed: int = 5):
    """Poisson arrivals of elliptic-drop solves (sides log-uniform in [64, 1024],
    500-20000 steps, aspect 1.1-1.5, ratio 1000, W 5), continuous batching."""
    from paper_1909_04166_amd import serve
    trace = W.serve_arrivals(n_req, seed, rate)
    reqs = served_requests(n_req, rate, seed)
    per_node = 2 * 18 * STORE[precision] + 32
    cap = int(budget_gb * 1e9 / per_node)
    S = serve.Server(slots=512, node_capacity=cap, precision=precision, tick=128)
    stats = S.run(reqs)
    offered = sum(r.nodes * r.steps for r in reqs) / max(a["t"] for a in trace) / 1e9
    S.close()
    stats.update({"requests_offered": n_req, "rate_per_s": rate, "offered_GLUPS": round(offered, 1),
                  "hbm_budget_GB": budget_gb, "unstable": stats["failed"]})
    for k in ("MLUPS", "p50_s", "p99_s", "wall_s"):
        if stats.get(k) is not None:
            stats[k] = round(stats[k], 3)
    return stats


def served_requests(n_req: int, rate: float, seed: int = 5):
    """The served stream's requests (elliptic drops, W 5), fields built on demand."""
    from paper_1909_04166_amd import serve
    trace = W.serve_arrivals(n_req, seed, rate)
    reqs = []
    for i, a in enumerate(trace):
        case, _ = W.ellipse(8, a["aspect"])
        case.update(nx=a["side"], ny=a["side"], W=5.0)
        reqs.append(serve.Request(rid=i, case=case, phi0=None, steps=a["steps"], arrival=a["t"],
                                  make=(lambda s=a["side"], r=a["aspect"]: W.ellipse(s, r, W=5.0)[1])))
    return reqs


def bench_plain_fifo(n_req: int, rate: float):
    """The plain form of the served stream: requests solved one at a time in FP64,
    first come first served, each on its own lattice (no batching)."""
    import torch
    reqs = served_requests(n_req, rate)
    t0 = time.perf_counter()
    lat, updates = [], 0
    for r in reqs:
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        side = r.case["nx"]  # fixed tile (no per-shape autotuning in the plain form)
        tile = (64 if side < 256 else (128 if side < 1024 else 256), 32)
        L = lb.Lattice(r.case, r.make(), "fp64", tile=tile)
        L.step(r.steps)
        L.diagnostics()  # synchronizes
        L.close()
        done = time.perf_counter() - t0
        lat.append(done - r.arrival)
        updates += r.nodes * r.steps
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    return {"requests": n_req, "rate_per_s": rate, "MLUPS": round(updates / wall / 1e6, 1),
            "p50_s": round(float(np.percentile(lat, 50)), 3), "p99_s": round(float(np.percentile(lat, 99)), 3),
            "wall_s": round(wall, 2)}


def bench_batched_same(n_req: int, rate: float, precision: str = "fp16"):
    """The same requests as bench_plain_fifo through the continuous-batching server."""
    from paper_1909_04166_amd import serve
    reqs = served_requests(n_req, rate)
    per_node = 2 * 18 * STORE[precision] + 32
    S = serve.Server(slots=512, node_capacity=int(24e9 / per_node), precision=precision, tick=128)
    st = S.run(reqs)
    S.close()
    return {"requests": n_req, "rate_per_s": rate, "MLUPS": round(st["MLUPS"], 1),
            "p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3), "wall_s": round(st["wall_s"], 2)}


def bench_configs():
    """The paper's configurations that fit the MALL (accuracy runs; launch and
    latency bound): MLUPS in FP64 and FP32, with whether the run stayed stable.
    The droplet runs at W 5: at the specified W 4 the ratio-1000 droplet
    diverges near step 450 (in the oracle as well)."""
    out = {}
    for name, steps in (("droplet128_W5", 1000), ("rt256", 2000)):
        c, p, _ = make_workload(name)
        for prec in ("fp64", "fp32"):
            rr = time_lattice(c, p, prec, steps, 50)
            out[f"{name}_{prec}"] = {"MLUPS": round(c["nx"] * c["ny"] * steps / rr["wall_s"] / 1e6, 1),
                                     "steps": steps,
                                     "stable": bool(rr["rc"] == 0 and rr["diag"]["nan_flag"] == 0.0
                                                    and rr["diag"]["max_u"] < 0.3)}
    return out


def bench_served_compact(n_req: int = 40, rate: float = 50.0):
    """The served stream's first n_req arrivals (Poisson 50 req/s, elliptic drops
    of sides 64-1024, 500-20000 steps, ratio 1000, W 5) two ways: continuous
    batching in FP32 compute with fp16 storage, and the plain form (FP64, one
    lattice at a time, first come first served).  p50 / p99 of completion minus
    arrival and delivered MLUPS of each."""
    bat = bench_batched_same(n_req, rate, "fp16")
    plain = bench_plain_fifo(n_req, rate)
    return {"requests": n_req, "rate_per_s": rate, "batched_fp16": bat, "plain_fp64_fifo": plain,
            "p50_plain_over_batched": round(plain["p50_s"] / max(bat["p50_s"], 1e-9), 1),
            "MLUPS_batched_over_plain": round(bat["MLUPS"] / max(plain["MLUPS"], 1e-9), 2)}


def bench_variants(side: int, steps: int, warmup: int):
    """Throughput of the option kernels on the roofline grid (the tiled droplets):
    the SRT pair (same bytes as the cascaded step, 36 s per node) and the phase
    field alone under an imposed vortex-array velocity (9 + 9 values of f and two
    compute-type velocity values per node)."""
    case, phi0 = W.droplet(128, 25.0, W=5.0)
    case, phi0 = W.tiled(case, phi0, side // 128, side // 128)
    N = case["nx"] * case["ny"]
    out = {}
    for prec in ("fp64", "fp32", "fp16"):
        rr = time_lattice(dict(case, collision="srt"), phi0, prec, steps, warmup)
        gbs = 36 * STORE[prec] * N / (rr["ms_kernel"] * 1e-3) / 1e9
        out[f"srt_{prec}"] = {"MLUPS": round(N * steps / rr["wall_s"] / 1e6, 1), "kernel_GBs": round(gbs, 1),
                              "frac": round(gbs / HBM_PEAK_GBS, 4), "tile": list(rr["tile"])}
    y, x = np.mgrid[0:side, 0:side].astype(np.float64)
    vel = (0.05 * np.sin(2 * np.pi * (y + 0.5) / 128) * np.cos(2 * np.pi * (x + 0.5) / 128),
           -0.05 * np.cos(2 * np.pi * (y + 0.5) / 128) * np.sin(2 * np.pi * (x + 0.5) / 128))
    del x, y
    for coll in ("cascaded", "srt"):
        for prec in ("fp64", "fp32", "fp16"):
            rr = time_lattice(dict(case, flow="imposed", collision=coll), phi0, prec, steps, warmup, vel=vel)
            per_node = 18 * STORE[prec] + 2 * (8 if prec == "fp64" else 4)
            gbs = per_node * N / (rr["ms_kernel"] * 1e-3) / 1e9
            out[f"ace_only_{coll}_{prec}"] = {"MLUPS": round(N * steps / rr["wall_s"] / 1e6, 1),
                                              "kernel_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                              "alg_bytes_per_node": per_node, "tile": list(rr["tile"])}
    out["workload"] = (f"{side}x{side} tiled 128^2 droplets (R=25, ratio 1000, W 5); ACE-only rows "
                       "under an imposed 128-periodic vortex array, |u| <= 0.05")
    return out


def bench_stability(steps: int = 20000):
    """Sec. 7: smallest viscosity (nu_A = nu_B) with a stable run of the
    oscillating elliptic cylinder (200^2, a = 25, b = 15, kappa~ = 0.01) for the
    cascaded pair (moment changes solved as stated, and their printed closed
    forms) and the SRT pair at density ratios 500-900.  Stable: no NaN/Inf and
    max |u| < 0.1 after `steps` steps.  nu ladder 0.1 * 0.6^k, k = 0..19.  Each
    model runs as one batch of 80 lattices."""
    ratios = (500, 600, 800, 900)
    nus = [0.1 * 0.6 ** k for k in range(20)]
    stable = {}
    t0 = time.perf_counter()
    models = ("cascaded", "printed", "srt")
    for coll in models:
        B = lb.Batch(len(ratios) * len(nus), 40000 * len(ratios) * len(nus) + 1000, "fp64")
        slots = {}
        for r in ratios:
            for nu in nus:
                c, p = W.elliptic_cylinder(r, nu, collision=coll)
                slots[B.add(c, p)] = (r, nu)
        B.step(steps)
        for sl, (r, nu) in slots.items():
            d = B.diagnostics(sl)
            stable[(coll, r, nu)] = bool(d["nan_flag"] == 0 and d["max_u"] < 0.1)
        B.close()
    out = {"steps": steps, "nu_ladder": [float(f"{v:.3e}") for v in nus], "wall_s": None}
    for r in ratios:
        row = {}
        for coll in models:
            ok = [nu for nu in nus if stable[(coll, r, nu)]]
            row[f"{coll}_nu_min"] = float(f"{min(ok):.3e}") if ok else None
            row[f"{coll}_unstable"] = [float(f"{nu:.3e}") for nu in nus if not stable[(coll, r, nu)]]
        for c in ("cascaded", "printed"):
            if row[f"{c}_nu_min"] and row["srt_nu_min"]:
                row[f"srt_over_{c}"] = round(row["srt_nu_min"] / row[f"{c}_nu_min"], 1)
        out[f"ratio_{r}"] = row
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    return out


def _tile_error(gpu, orc, case):
    """phi max-abs; p and u max-abs relative to the larger of the oracle field's
    maximum and its physical scale (Laplace pressure sigma / R, capillary
    velocity sigma / mu_A)."""
    sig, R = case["sigma0"], 25.0
    ps = max(float(np.abs(orc[1]).max()), sig / R)
    us = max(float(np.abs(orc[2]).max()), float(np.abs(orc[3]).max()), sig / (case["rho_A"] * case["nu_A"]))
    return {"phi_maxabs": float(np.abs(gpu[0] - orc[0]).max()),
            "p_rel": float(np.abs(gpu[1] - orc[1]).max() / ps),
            "u_rel": float(max(np.abs(gpu[2] - orc[2]).max(), np.abs(gpu[3] - orc[3]).max()) / us)}


def cpu_baseline(target_s: float = 15.0, ref_steps: int = 0, gpu_tile=None):
    """The FP64 oracle as it stands, on the host cores.

    All cores (OpenMP over rows): an 8 x 8 block of the workload's tiles (the
    1024^2 periodic lattice of 128^2 droplets, about 0.5 GB of oracle state,
    beyond the host caches), first ref_steps steps, then more steps up to about
    target_s seconds; MLUPS over both timed segments.  Because the timed grid is
    periodic in its tiles, its first 128^2 tile after ref_steps steps is the
    oracle's answer for every tile of the GPU run after the same number of steps:
    when gpu_tile (phi, p, ux, uy of the GPU's first tile) is given, its error
    against that answer is returned too (computed outside every timed region).
    One core: the 128^2 tile for a shorter sample."""
    import ctypes
    import oracle
    case, phi0 = W.droplet(128, 25.0, W=5.0)
    n_nodes = case["nx"] * case["ny"]
    gomp = ctypes.CDLL("libgomp.so.1")

    def timed(threads, budget_s):
        gomp.omp_set_num_threads(int(threads))
        o = oracle.Oracle(case, phi0)
        o.step(10)  # thread start-up
        t0 = time.perf_counter()
        o.step(40)
        dt = time.perf_counter() - t0
        steps = int(max(50, min(500000, budget_s / max(dt / 40, 1e-9))))
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        return steps, dt

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    gomp.omp_set_num_threads(cores)
    bcase, bphi = W.tiled(case, phi0, 8, 8)
    nb = bcase["nx"] * bcase["ny"]
    o = oracle.Oracle(bcase, bphi)
    del bphi
    t0 = time.perf_counter()
    o.step(max(ref_steps, 1))
    dt1 = time.perf_counter() - t0
    err = None
    if gpu_tile is not None and ref_steps > 0:
        ref = tuple(f[:128, :128] for f in o.fields())
        err = _tile_error(gpu_tile, ref, case)
    per_step = dt1 / max(ref_steps, 1)
    more = int(max(0, min(100000, (target_s - dt1) / max(per_step, 1e-9))))
    t0 = time.perf_counter()
    o.step(more)
    dt2 = time.perf_counter() - t0
    big_steps, big_dt = max(ref_steps, 1) + more, dt1 + dt2
    del o
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    steps1, dt1s = timed(1, target_s / 3)
    # config 2 (Rayleigh-Taylor 256 x 1024), all cores, a short sample
    gomp.omp_set_num_threads(int(cores))
    rc, rp = W.config("rt256")
    o = oracle.Oracle(rc, rp)
    o.step(5)
    t0 = time.perf_counter()
    o.step(40)
    rt_dt = time.perf_counter() - t0
    out = {"value": nb * big_steps / big_dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"FP64 oracle, 1024x1024 block (8x8 tiles) of the workload's 128^2 droplets "
                     f"(R=25, ratio 1000, W 5), {big_steps} steps in {big_dt:.1f} s, OpenMP over rows "
                     f"on {cores} threads",
           "single_thread_MLUPS": round(n_nodes * steps1 / dt1s / 1e6, 2),
           "single_thread_sample": f"128x128 tile, {steps1} steps in {dt1s:.1f} s, 1 thread",
           "rt256x1024_MLUPS": round(rc["nx"] * rc["ny"] * 40 / rt_dt / 1e6, 2),
           "host": f"{model}, {os.cpu_count()} logical CPUs visible"}
    return out, err


def progress(msg: str) -> None:
    """One line per finished stage on stderr (the JSON line goes to stdout)."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="tiled8192")
    ap.add_argument("--precision", default="fp64", choices=list(STORE))
    ap.add_argument("--tile", default="0,0")
    ap.add_argument("--schedule", default="", metavar="TX,MODE,PARAM,PF",
                    help="pin the headline lattice's schedule (lb_set_schedule) instead of autotuning")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (and with it the oracle error of the headline run)")
    ap.add_argument("--no-configs", action="store_true", help="skip the paper's small configurations")
    ap.add_argument("--batched-only", action="store_true",
                    help="only time the 256-lattice batch in --precision (--schedule pins its schedule)")
    ap.add_argument("--no-batched", action="store_true", help="skip the default 256-lattice batch line")
    ap.add_argument("--no-served", action="store_true", help="skip the default served-stream comparison")
    ap.add_argument("--extra", action="store_true", help="also time the other precisions and workloads")
    ap.add_argument("--batched", action="store_true", help="also time the uneven batch (256 lattices)")
    ap.add_argument("--served", action="store_true", help="also run the served Poisson stream")
    ap.add_argument("--variants", action="store_true",
                    help="also time the SRT pair and the phase-field-only kernels on the roofline grid")
    ap.add_argument("--stability", action="store_true",
                    help="also run the nu_min stability sweep of the cascaded and SRT pairs")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="MIB",
                    help="only run the library's device copy kernel over MIB MiB (bandwidth and "
                         "counter reference) and print its GB/s")
    ap.add_argument("--copy-variants", default="0",
                    help="with --copy-ref: comma-separated lb_bandwidth_probe variants (0 = lb_copy_kernel)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    lb.lib()
    tile = tuple(int(v) for v in args.tile.split(","))
    if args.copy_ref:
        n = args.copy_ref << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        variants = [int(v) for v in args.copy_variants.split(",")]
        # bytes each variant moves: copies read and write n, the read probe reads
        # n (and writes 16 MiB), the write probe writes n, the row-pattern probes
        # read and write whole rows of 18 x 8064 two-byte values
        rows_bytes = n // (18 * 8064 * 2) * (18 * 8064 * 2)
        moved = {5: n + (16 << 20), 6: n, 7: 2 * rows_bytes, 8: 2 * rows_bytes}
        out = {"bytes": n, "variants": {}}
        for v in variants:
            run = (lambda: lb.lb_copy_kernel(b.data_ptr(), a.data_ptr(), n, stream)) if v == 0 else \
                  (lambda v=v: lb.lb_bandwidth_probe(b.data_ptr(), a.data_ptr(), n, v, stream))
            for _ in range(3):
                run()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            reps = 20
            for _ in range(reps):
                run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            out["variants"][v] = {"ms": round(ms, 4), "GBs": round(moved.get(v, 2 * n) / (ms * 1e-3) / 1e9, 1)}
        print(json.dumps(out), flush=True)
        return

    if args.batched_only:
        bsched = tuple(int(v) for v in args.schedule.split(",")) if args.schedule else None
        print(json.dumps({"batched": bench_batched(args.precision, args.steps, warmup=args.warmup, sched=bsched)}),
              flush=True)
        return

    case, phi0, desc = make_workload(args.workload)
    N = case["nx"] * case["ny"]
    print(f"[bench] {desc}: N={N} precision={args.precision} steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)
    tiled = args.workload.startswith("tiled")
    sched = tuple(int(v) for v in args.schedule.split(",")) if args.schedule else None
    r = time_lattice(case, phi0, args.precision, args.steps, args.warmup, tile, keep_tile=128 if tiled else 0,
                     sched=sched)
    del phi0
    mlups = N * args.steps / r["wall_s"] / 1e6
    progress(f"headline step timed: {mlups:.1f} MLUPS")
    s = STORE[args.precision]
    bytes_per_launch = 36 * s * N
    achieved = bytes_per_launch / (r["ms_kernel"] * 1e-3) / 1e9 if r["ms_kernel"] > 0 else None
    traffic = measured_traffic(args.workload, args.precision, r["tile"])
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall_s"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f32 compute, f16 storage",
                  "bf16": "f32 compute, bf16 storage"}[args.precision],
        "data": "synthetic",
        "config": {"workload": desc, "nx": case["nx"], "ny": case["ny"], "precision": args.precision,
                   "tile": list(r["tile"]), "kernel": "lb_fused (single-pass stream-collide, f and gbar)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": (traffic["read"] + traffic["write"]) if traffic else None,
                     "traffic_read": traffic["read"] if traffic else None,
                     "traffic_write": traffic["write"] if traffic else None,
                     "kernel_ms": round(r["ms_kernel"], 5),
                     "alg_bytes_per_launch": bytes_per_launch},
        "stable": r["rc"] == 0 and r["diag"]["nan_flag"] == 0.0,
    }
    if not args.no_configs:
        out["paper_configs"] = bench_configs()
        progress("paper configurations timed")
    if not args.no_batched:
        out["batched"] = {"fp16": bench_batched("fp16", max(args.steps, 320))}
        progress("batch timed")
        out["batched"]["fp16"]["vs_plain_fp64"] = round(out["batched"]["fp16"]["MLUPS"] / out["value"], 3)
        out["batched"]["workload"] = ("256 uneven lattices (droplet or Rayleigh-Taylor by seed 20190909, sides "
                                      "64-512, ratio log-uniform 3-1000, W 5, M 0.02), one persistent launch "
                                      "per step")
    if not args.no_served:
        out["served"] = bench_served_compact()
        progress("served stream run")
    if args.extra:
        extra = {}
        for prec in ("fp32", "fp16", "bf16"):
            rr = time_lattice(case, W.tiled(*W.droplet(128, 25.0, W=5.0), case["nx"] // 128,
                                            case["ny"] // 128)[1] if args.workload.startswith("tiled")
                              else make_workload(args.workload)[1], prec, args.steps, args.warmup)
            extra[prec] = {"MLUPS": round(N * args.steps / rr["wall_s"] / 1e6, 1),
                           "kernel_GBs": round(36 * STORE[prec] * N / (rr["ms_kernel"] * 1e-3) / 1e9, 1),
                           "tile": list(rr["tile"])}
            progress(f"extra {prec} timed")
        if args.workload == "tiled8192":  # the smaller roofline grid of the same tiling
            c4, p4, _ = make_workload("tiled4096")
            n4 = c4["nx"] * c4["ny"]
            for prec in ("fp64", "fp32", "fp16"):
                rr = time_lattice(c4, p4, prec, args.steps, args.warmup)
                extra[f"tiled4096_{prec}"] = {
                    "MLUPS": round(n4 * args.steps / rr["wall_s"] / 1e6, 1),
                    "kernel_GBs": round(36 * STORE[prec] * n4 / (rr["ms_kernel"] * 1e-3) / 1e9, 1),
                    "tile": list(rr["tile"])}
                progress(f"extra 4096^2 {prec} timed")
        out["extra"] = extra
    if args.batched:
        full = {}
        for p in ("fp16", "bf16", "fp32"):
            full[p] = bench_batched(p, 5000)
            progress(f"5000-step batch {p} timed")
        for p, rb in full.items():
            rb["vs_plain_fp64"] = round(rb["MLUPS"] / out["value"], 3)
        out.setdefault("batched", {})["5000_steps"] = full
    if args.served:
        sat = bench_served("fp16", 500, 50.0)
        progress("saturated served stream run")
        cap_glups = max(sat["MLUPS"] / 1e3, 1e-3)
        # a second stream at 70 % of the measured capacity, so latency is not pure queue growth
        mean_work = 1.93e9
        low = bench_served("fp16", 200, 0.7 * cap_glups * 1e9 / mean_work)
        progress("served stream at 0.7 load run")
        # plain form of the same stream: 60 requests of the 0.7-load trace, FP64,
        # one lattice at a time, beside the same 60 through the batching server
        rate7 = 0.7 * cap_glups * 1e9 / mean_work
        out["served_full"] = {"saturated": sat, "load_0.7": low,
                         "vs_plain_fp64": round(sat["MLUPS"] / out["value"], 3),
                         "latency_batched_vs_plain": {"batched_fp16": bench_batched_same(60, rate7),
                                                      "plain_fp64_fifo": bench_plain_fifo(60, rate7)}}
    if args.variants:
        side = case["nx"] if args.workload.startswith("tiled") else 8192
        out["variants"] = bench_variants(side, args.steps, args.warmup)
        progress("variants timed")
    if args.stability:
        out["stability"] = bench_stability()
        progress("stability sweep run")
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline starts")
        out["cpu_baseline"], err = cpu_baseline(ref_steps=args.warmup + args.steps if tiled else 0,
                                                gpu_tile=r["first_tile"])
        if err is not None:
            err.update(steps=args.warmup + args.steps, tiles_identical=r["tiles_identical"],
                       reference="FP64 oracle, the cpu_baseline run's first 128^2 tile")
            out["oracle_error"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
