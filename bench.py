"""Throughput bench of the pressure-Poisson projection hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Prints ONE JSON line.  A step is one pass of the whole hot path over one batch
of synthetic input already resident in HBM; the timed region holds exactly K
steps bracketed by device synchronisation.  The dominant kernel's duration is
measured with HIP events recorded by the library on the launch stream during
the timed region; its roofline figure uses the algorithmic bytes of one launch
(each array the kernel must read or write, once).  The CPU baseline is the FP64
oracle (test infrastructure) timed on a bounded sample on the host cores.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# The headline metric; the line's value is its projection-step figure (the
# workload in config), the Poisson FP64 / FP32+refine and fwd+adjoint figures
# are under "also".
METRIC = "Mpts/s per Poisson solve and per fwd+adjoint step, FP64 vs FP32+refine, % HBM"

# Model bytes per grid point of the metric's legs (every array each pass must
# read or write once, at its storage precision; the forward + adjoint steps are
# the sum over the kernels they launch).  The mixed solve with one refinement:
# r2c 8+4, z/y/z^-1 24, the first solve's output stored as FP32 4+4, residual
# transform 4+8+4, z/y/z^-1 24, accumulation 4+4+8 = 100 (112 if the first
# solve's output were stored in FP64).
MODEL_BYTES_PER_POINT = {
    "poisson_fp64": 80,
    "poisson_mixed_refine1": 100,
    "step_fp64": 200,
    "fwd_adjoint_step_fp64": 568,
    "fwd_adjoint_step_mixed": 416,
}

# Source files that define each kernel class (the HBM-traffic counters under
# profiles/ are keyed to a hash of these files and the compile flags, so a
# kernel changed since its counters were taken reports no traffic).
KERNEL_SOURCES = {
    "rk2_fused": ["cf_common.h", "cf_step_kernels.h", "cf_rk_fused.h", "cf_step_launch.hip"],
    "correct": ["cf_common.h", "cf_step_kernels.h", "cf_rk_fused.h", "cf_step_launch.hip"],
    "r2c_x": ["cf_common.h", "cf_fft.h", "cf_fft_kernels.h", "cf_fft_launch.hip"],
    "c2r_x": ["cf_common.h", "cf_fft.h", "cf_fft_kernels.h", "cf_fft_launch.hip"],
    "fft_z_fwd": ["cf_common.h", "cf_fft.h", "cf_fft_kernels.h", "cf_fft_launch.hip"],
    "fft_z_inv": ["cf_common.h", "cf_fft.h", "cf_fft_kernels.h", "cf_fft_launch.hip"],
    "ysolve": ["cf_common.h", "cf_pdd.h", "cf_ysolve_kernels.h", "cf_ysolve_launch.hip"],
    # whole paths: every kernel source they launch and the plan that sequences them
    "step_fp64": ["cf_common.h", "cf_fft.h", "cf_fft_kernels.h", "cf_fft_launch.hip", "cf_pdd.h",
                  "cf_ysolve_kernels.h", "cf_ysolve_launch.hip", "cf_step_kernels.h", "cf_rk_fused.h",
                  "cf_step_launch.hip", "cf_plan.hip"],
    "poisson_mixed": ["cf_common.h", "cf_fft.h", "cf_fft_kernels.h", "cf_fft_launch.hip", "cf_pdd.h",
                      "cf_ysolve_kernels.h", "cf_ysolve_launch.hip", "cf_plan.hip"],
}


def kernel_source_hash(kernel: str) -> str | None:
    """sha256 of a kernel class's source files and the flags they are built
    with (include paths left out)."""
    import hashlib

    from paper_2104_08863_amd import build as B
    files = KERNEL_SOURCES.get(kernel)
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        h.update(f.encode())
        h.update(open(os.path.join(B.CSRC, f), "rb").read())
        flags = [a for a in B.HIP_FLAGS + B.EXTRA_FLAGS.get(f, []) if not a.startswith("/")]
        h.update(" ".join(flags).encode())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` (or per step / solve of a whole path) on
    `workload` from the counter summaries in profiles/ (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, KiB, scaled by the factors a plain copy kernel gives), or None
    when no summary was taken on the current source."""
    import glob
    want = kernel_source_hash(kernel)
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt")):
        rec = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        if rec.get("kernel") == kernel and rec.get("workload") == workload and rec.get("source_sha256") == want:
            return (float(rec["fetch_kib"]) * float(rec["fetch_factor"])
                    + float(rec["write_kib"]) * float(rec["write_factor"])) * 1024
    return None


def _pmc_load(base, name):
    import collections
    import csv
    import re
    rows = list(csv.DictReader(open(f"{base}/{name}/run_counter_collection.csv")))
    agg = collections.defaultdict(list)
    for r in rows:
        k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
        agg[(k, r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def summarize_pmc(base):
    """Markdown table of rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch,
    averaged over dispatches) from the passes copy_fetch/, copy_write/ (the
    --calibrate-copy run: one elementwise kernel reading and writing 1 GiB) and
    fetch/, write/ (the bench run) under `base`, each scaled by the factor the
    calibration kernel gives for the same counter."""
    cf, cw = _pmc_load(base, "copy_fetch"), _pmc_load(base, "copy_write")
    copy = [k for (k, c) in cf if "CUDAFunctor" in k][0]
    kib = 1024 * 1024
    f_fac, w_fac = kib / cf[(copy, "FETCH_SIZE")], kib / cw[(copy, "WRITE_SIZE")]
    fe, wr = _pmc_load(base, "fetch"), _pmc_load(base, "write")
    out = [f"calibration (elementwise kernel reading and writing 1 GiB): FETCH_SIZE "
           f"{cf[(copy, 'FETCH_SIZE')]:.0f} KiB -> factor {f_fac:.3f}; WRITE_SIZE "
           f"{cw[(copy, 'WRITE_SIZE')]:.0f} KiB -> factor {w_fac:.3f}", "",
           "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read GB (scaled) | write GB (scaled) |",
           "|---|---:|---:|---:|---:|"]
    names = sorted({k for (k, c) in fe if k.startswith("cf::")}, key=lambda k: -fe[(k, "FETCH_SIZE")])
    for k in names:
        f, w = fe[(k, "FETCH_SIZE")], wr.get((k, "WRITE_SIZE"), float("nan"))
        out.append(f"| `{k}` | {f:.0f} | {w:.0f} | {f * f_fac * 1024 / 1e9:.3f} | {w * w_fac * 1024 / 1e9:.3f} |")
    return "\n".join(out)


def pmc_record(base, name, workload, units, exclude=()):
    """Traffic record (the key: value form measured_traffic reads) of a whole
    path: FETCH_SIZE and WRITE_SIZE summed over every dispatch of a cf:: kernel
    in the passes fetch/ and write/ under `base`, divided by the number of
    steps or solves (`units`) the profiled run made; kernels whose name
    contains a string in `exclude` (input generation) are left out.  Scaling
    factors from the copy_fetch/ and copy_write/ calibration passes."""
    import csv
    import re
    cf, cw = _pmc_load(base, "copy_fetch"), _pmc_load(base, "copy_write")
    copy = [k for (k, c) in cf if "CUDAFunctor" in k][0]
    kib = 1024 * 1024

    def total(pas, counter):
        t = 0.0
        for r in csv.DictReader(open(f"{base}/{pas}/run_counter_collection.csv")):
            k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
            if r["Counter_Name"] == counter and k.startswith("cf::") and not any(e in k for e in exclude):
                t += float(r["Counter_Value"])
        return t / units
    return "\n".join([f"kernel: {name}", f"workload: {workload}", f"source_sha256: {kernel_source_hash(name)}",
                      f"fetch_kib: {total('fetch', 'FETCH_SIZE'):.0f}", f"write_kib: {total('write', 'WRITE_SIZE'):.0f}",
                      f"fetch_factor: {kib / cf[(copy, 'FETCH_SIZE')]:.3f}",
                      f"write_factor: {kib / cw[(copy, 'WRITE_SIZE')]:.3f}"])


def summarize_counters(base, kernel):
    """Mean per dispatch of every counter in the rocprofv3 --pmc passes under
    `base` (each subdirectory holding a run_counter_collection.csv) for the
    kernels whose name contains `kernel`, as a markdown table."""
    import collections
    import csv
    import glob
    import re
    agg = collections.defaultdict(list)
    for path in sorted(glob.glob(os.path.join(base, "*", "run_counter_collection.csv"))):
        for r in csv.DictReader(open(path)):
            k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
            if kernel in k:
                agg[(k, r["Counter_Name"])].append(float(r["Counter_Value"]))
    out = ["| kernel | counter | dispatches | mean per dispatch |", "|---|---|---:|---:|"]
    for (k, c), v in sorted(agg.items()):
        out.append(f"| `{k}` | {c} | {len(v)} | {sum(v) / len(v):.4g} |")
    return "\n".join(out)


def summarize_trace(path):
    """Markdown table of a rocprofv3 --stats kernel_stats.csv."""
    import csv
    import re
    out = ["| kernel | calls | avg us | min us | max us | % |", "|---|---:|---:|---:|---:|---:|"]
    for r in csv.DictReader(open(path)):
        n = re.sub(r"\(.*", "", r["Name"]).replace("void ", "")
        out.append(f"| `{n}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def summarize_trace_last(path, n):
    """Markdown table of the mean duration of each kernel's last n dispatches
    in a rocprofv3 run_kernel_trace.csv (the timed launches of a run whose
    first dispatches are warm-up)."""
    import collections
    import csv
    import re
    runs = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
        runs[k].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    out = [f"| kernel | launches | avg us (last {n}) |", "|---|---:|---:|"]
    rows = []
    for k, v in runs.items():
        if not k.startswith("cf::"):
            continue
        v.sort()
        last = v[-n:]
        rows.append((sum(e - b for b, e in last) / len(last) / 1e3, k, len(v)))
    for us, k, c in sorted(rows, reverse=True):
        out.append(f"| `{k}` | {c} | {us:.1f} |")
    return "\n".join(out)


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 20) -> float:
    """Device-to-device bandwidth of a plain elementwise kernel (torch.add,
    reading and writing nbytes each), the practical ceiling the kernels' GB/s
    can be held against next to the 8 TB/s peak."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.add(a, 1.0, out=b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.add(a, 1.0, out=b)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2 * nbytes / t / 1e9, 1)


def kernel_bytes(name: str, nx: int, ny: int, nz: int, esize_spec: int, esize_phys: int = 8,
                 fused_div: bool = False) -> float:
    """Algorithmic bytes of one launch of a kernel class: every array the
    kernel must read or write, once (no halo re-reads counted)."""
    nkx = nx // 2 + 1
    phys = nx * ny * nz * esize_phys
    spec = ny * nkx * nz * 2 * esize_spec
    return {
        "r2c_x": (3 * phys if fused_div else phys) + spec,
        "fft_z_fwd": 2 * spec,
        "ysolve": 2 * spec,
        "fft_z_inv": 2 * spec,
        "c2r_x": spec + nx * ny * nz * 8,
        "divergence": 4 * phys,
        "special_lines": 0.0,
        "rk_stage1": 6 * phys,
        "rk_stage2": 9 * phys,
        "rk2_fused": 6 * phys,
        "correct": 6 * phys + nx * ny * nz * 8,
    }[name]


def _host_info():
    """Host cores and CPU model name (from /proc/cpuinfo)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _oracle_rate(call, npts, min_calls=1, max_calls=3, seconds=5.0, warm=True):
    """Mpts/s of a CPU oracle call: one warm-up call (if warm), then calls
    until `seconds` have passed or max_calls were made (at least min_calls)."""
    if warm:
        call()
    t0 = time.perf_counter()
    n = 0
    while True:
        call()
        n += 1
        if n >= max_calls or (n >= min_calls and time.perf_counter() - t0 > seconds):
            break
    dt = (time.perf_counter() - t0) / n
    return round(npts / dt / 1e6, 2), n


def cpu_baseline(wl, poisson_only: bool):
    """The oracle (plain torch CPU, FP64, all host threads) on the workload's
    own input: one projection step (or Poisson solve) of the full grid, the same
    seeded arrays the GPU line times (about 20-30 s on 16 host threads).  Also:
    one thread on a bounded sample of the same recipe (the workload's x-z planes
    with ny reduced to 16, its own tanh grid; mean of two calls), the 64^3
    Poisson solve and the 256x128x256 step (whole grids, all threads), the
    Poisson solve on 192 z-planes of the 2048x512x1536 grid, and the host's
    core count and CPU model."""
    import torch

    import oracle as O
    from paper_2104_08863_amd import synth
    threads = torch.get_num_threads()
    yf = wl.y_faces()
    box = O.Box(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, yf)
    if poisson_only:
        f = torch.tensor(synth.uniform_rhs(wl.nx, wl.ny, wl.nz, seed=0))
        call = lambda: O.poisson(f, box)  # noqa: E731
        what = "Poisson solve (torch CPU FFT + Thomas)"
    else:
        u, v, w = (torch.tensor(q) for q in synth.perturbed_poiseuille(wl.nx, wl.ny, wl.nz, yf, seed=0))
        call = lambda: O.projection_step(u, v, w, box, wl.dt, wl.nu, wl.fx)  # noqa: E731
        what = "projection step (RK2 + torch CPU FFT/Thomas Poisson + correction)"
    value, n = _oracle_rate(call, wl.npts, max_calls=1, warm=False)
    out = {"value": value, "unit": "Mpts/s", "cores": threads, "kind": "oracle",
           "sample": f"FP64 oracle {what} on the whole {wl.nx}x{wl.ny}x{wl.nz} input of the GPU line "
                     f"(same seeded arrays), one call, {threads} threads"}
    del call
    if not poisson_only:
        del u, v, w
    # one thread on a bounded sample of the same recipe
    ny_s = 16
    ys = synth.tanh_faces(ny_s, wl.gamma)
    bs = O.Box(wl.nx, ny_s, wl.nz, wl.lx, wl.lz, ys)
    if poisson_only:
        fs = torch.tensor(synth.uniform_rhs(wl.nx, ny_s, wl.nz, seed=0))
        cs = lambda: O.poisson(fs, bs)  # noqa: E731
    else:
        us, vs, ws = (torch.tensor(q) for q in synth.perturbed_poiseuille(wl.nx, ny_s, wl.nz, ys, seed=0))
        cs = lambda: O.projection_step(us, vs, ws, bs, wl.dt, wl.nu, wl.fx)  # noqa: E731
    try:
        torch.set_num_threads(1)
        v1, n1 = _oracle_rate(cs, wl.nx * ny_s * wl.nz, min_calls=2, max_calls=2, warm=False)
    finally:
        torch.set_num_threads(threads)
    out["single_thread"] = {"value": v1, "cores": 1, "calls": n1,
                            "sample": f"{wl.nx}x{ny_s}x{wl.nz} (the workload's x-z planes, ny reduced to {ny_s})"}
    # whole small grids with all threads
    w1 = synth.WORKLOADS["poisson64"]
    b1 = O.Box(w1.nx, w1.ny, w1.nz, w1.lx, w1.lz, w1.y_faces())
    f1 = torch.tensor(synth.uniform_rhs(w1.nx, w1.ny, w1.nz, seed=0))
    out["poisson_fp64_64x64x64"], _ = _oracle_rate(lambda: O.poisson(f1, b1), w1.nx * w1.ny * w1.nz)
    w4 = synth.WORKLOADS["rollout256"]
    y4 = w4.y_faces()
    b4 = O.Box(w4.nx, w4.ny, w4.nz, w4.lx, w4.lz, y4)
    u4, v4, w4f = (torch.tensor(q) for q in synth.perturbed_poiseuille(w4.nx, w4.ny, w4.nz, y4, seed=0))
    out["step_fp64_256x128x256"], _ = _oracle_rate(
        lambda: O.projection_step(u4, v4, w4f, b4, w4.dt, w4.nu, w4.fx), w4.nx * w4.ny * w4.nz, max_calls=1)
    del u4, v4, w4f
    # the 2048x512x1536 mixed workload's x-y planes with nz reduced to 192: the
    # FP64 oracle Poisson solve (the oracle has no mixed precision; the whole
    # grid would take minutes), all threads
    w3 = synth.WORKLOADS["mixed1000"]
    nz3 = 192
    b3 = O.Box(w3.nx, w3.ny, nz3, w3.lx, w3.lz * nz3 / w3.nz, w3.y_faces())
    f3 = torch.tensor(synth.uniform_rhs(w3.nx, w3.ny, nz3, seed=0))
    r3, n3 = _oracle_rate(lambda: O.poisson(f3, b3), w3.nx * w3.ny * nz3, max_calls=1, warm=False)
    out["poisson_fp64_2048x512x192"] = {"value": r3, "calls": n3,
                                       "sample": f"{w3.nx}x{w3.ny}x{nz3}: the {w3.nx}x{w3.ny}x{w3.nz} "
                                                 f"workload's x-y planes (its tanh grid), nz reduced to {nz3}"}
    del f3
    out["host"] = _host_info()
    out["host"]["torch_threads"] = threads
    return out


def _progress(what):
    """One line on stderr per finished figure (the JSON result goes to stdout)."""
    print(f"bench: {what} done", file=sys.stderr, flush=True)


def _leg(name, grid, t, **extra):
    """Mpts/s and the HBM fraction of one timed figure of the metric, against
    its model bytes per point."""
    npts = grid[0] * grid[1] * grid[2]
    d = {"grid": list(grid), "ms": round(t * 1e3, 4), "Mpts_s": round(npts / t / 1e6, 1)}
    bpp = MODEL_BYTES_PER_POINT.get(name)
    if bpp is not None:
        gbs = bpp * npts / t / 1e9
        d.update({"model_bytes_per_pt": bpp, "model_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
    d.update(extra)
    return d


def _time(fn, steps, warmup=2):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_loop_figures(wl, steps):
    """The time loop (cf_run_steps) on the step grid, on the 256x128x256 rollout
    grid and on a 64^3 grid (launch-bound: ~20 us of kernels per step), eager
    and replayed from the plan's cached HIP graphs, with plane statistics after
    every step (dt 1e-3, nu 1/550 on the small grids) and without statistics;
    and the statistics kernel alone."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    res = {}
    small = synth.Workload("loop64", 64, 64, 64, 2 * np.pi, np.pi, 2.0, nu=1.0 / 550.0, dt=1e-3, fx=3.0 / 550.0)
    for w_ in (wl, synth.WORKLOADS["rollout256"], small):
        yf = w_.y_faces()
        pl = Plan(w_.nx, w_.ny, w_.nz, w_.lx, w_.lz, yf, precision="fp64", step=True)
        st = [torch.tensor(q, device=dev) for q in synth.perturbed_poiseuille(w_.nx, w_.ny, w_.nz, yf, seed=0)]
        work = tuple(torch.empty_like(t) for t in st)
        acc = torch.zeros(w_.ny, 6, dtype=torch.float64, device=dev)
        n = 10 if w_.npts > 1e7 else 50
        fig = {"grid": [w_.nx, w_.ny, w_.nz], "steps_per_call": n}
        for every, tag in ((1, ""), (0, "nostats_")):
            for mode in ("eager", "graph"):
                t = _time(lambda: pl.run_steps(*st, n, w_.dt, w_.nu, w_.fx, work=work, stats_every=every,
                                               stats=acc if every else None, use_graph=(mode == "graph")),
                          max(2, steps // 3), warmup=1)
                fig[f"{tag}{mode}_ms_per_step"] = round(t * 1e3 / n, 4)
                fig[f"{tag}{mode}_Mpts_s"] = round(w_.nx * w_.ny * w_.nz * n / t / 1e6, 1)
        tst = _time(lambda: pl.plane_stats(*st), steps)
        fig["plane_stats_us"] = round(tst * 1e6, 1)
        fig["plane_stats_GBps"] = round(3 * 8 * w_.nx * w_.ny * w_.nz / tst / 1e9, 1)
        res[f"time_loop_fp64_{w_.nx}x{w_.ny}x{w_.nz}"] = fig
        del pl, st, work, acc
        torch.cuda.empty_cache()
    return res


def rollout_figure(steps):
    """The differentiable-rollout workload: 8 FP64 projection steps on
    256x128x256 through the autograd Function (checkpoints every 2 steps), loss
    0.5 sum(u^2 + v^2 + w^2), backward to the initial field; ms per step of
    forward + adjoint."""
    import torch

    from paper_2104_08863_amd import autograd as AG
    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    w_ = synth.WORKLOADS["rollout256"]
    yf = w_.y_faces()
    pl = Plan(w_.nx, w_.ny, w_.nz, w_.lx, w_.lz, yf, precision="fp64", adjoint=True)
    init = [torch.tensor(q, device=dev) for q in synth.perturbed_poiseuille(w_.nx, w_.ny, w_.nz, yf, seed=0)]

    def run():
        xs = [t.clone().requires_grad_(True) for t in init]
        a, b, c = AG.rollout(pl, *xs, 8, w_.dt, w_.nu, w_.fx, checkpoint_every=2)
        (0.5 * ((a * a).sum() + (b * b).sum() + (c * c).sum())).backward()
    t = _time(run, max(2, steps // 2), warmup=1)
    del pl, init
    torch.cuda.empty_cache()
    return {"rollout_fwd_adjoint_fp64_256x128x256": {
        "grid": [w_.nx, w_.ny, w_.nz], "steps": 8, "checkpoint_every": 2,
        "ms_per_step": round(t * 1e3 / 8, 4), "ms_per_rollout": round(t * 1e3, 3)}}


def profile_fwd_adjoint(steps: int):
    """FP64 forward + adjoint steps on the step grid (the fwd_adjoint_step_fp64
    figure's inputs), one warm-up step, for a kernel-trace profile."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    wl = synth.WORKLOADS["step550"]
    yf = wl.y_faces()
    pa = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, yf, precision="fp64", adjoint=True)
    u, v, w = (torch.tensor(q, device=dev) for q in synth.perturbed_poiseuille(wl.nx, wl.ny, wl.nz, yf, seed=0))
    o = tuple(torch.empty_like(u) for _ in range(3))
    g1 = tuple(torch.tensor(q, device=dev) for q in synth.random_directions(wl.nx, wl.ny, wl.nz, seed=1))
    go = tuple(torch.empty_like(u) for _ in range(3))
    for k in range(steps + 1):
        pa.projection_step(u, v, w, wl.dt, wl.nu, wl.fx, out=o)
        pa.projection_step_adjoint(u, v, w, *g1, wl.dt, wl.nu, wl.fx, out=go)
        torch.cuda.synchronize()
        print(f"fwd+adjoint step {k} done", flush=True)


def profile_poisson_mixed(calls: int):
    """Mixed-precision Poisson solves (one refinement pass) on the 2048x512x1536
    grid, the poisson_mixed_refine1_2048x512x1536 figure's input, one warm-up
    call, for a kernel-trace or counter profile."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    big = synth.WORKLOADS["mixed1000"]
    pm = Plan(big.nx, big.ny, big.nz, big.lx, big.lz, big.y_faces(), precision="mixed", refine_passes=1)
    vel = synth.powerlaw_velocity_device(big.nx, big.ny, big.nz, seed=0, device=dev)
    fb = pm.divergence(*vel)
    del vel
    torch.cuda.empty_cache()
    pb = torch.empty_like(fb)
    for k in range(calls + 1):
        pm.poisson_solve(fb, out=pb)
        torch.cuda.synchronize()
        print(f"mixed Poisson solve {k} done", flush=True)


def fwd_adjoint_mixed(steps: int = 2, warmup: int = 1):
    """Mixed-precision forward + adjoint step on the 2048x768x2048 grid (FP32
    state; the gradient overwrites the incoming adjoint field): perturbed
    Poiseuille state and an N(0, 0.1^2) adjoint field from a seeded torch CUDA
    generator."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    c5 = synth.WORKLOADS["adj2000"]
    n5 = c5.nx * c5.ny * c5.nz
    y5 = c5.y_faces()
    yc = torch.tensor(0.5 * (y5[1:] + y5[:-1]), dtype=torch.float32, device=dev)
    shp = (c5.ny, c5.nz, c5.nx)

    def gauss():
        return torch.randn(shp, dtype=torch.float32, device=dev, generator=gen) * 0.1
    u = gauss() + (1.5 * (1 - yc * yc))[:, None, None]
    v = gauss()
    v[-1] = 0
    w = gauss()
    o = tuple(torch.empty_like(u) for _ in range(3))
    g = (gauss(), gauss(), gauss())
    pm = Plan(c5.nx, c5.ny, c5.nz, c5.lx, c5.lz, y5, precision="mixed", adjoint=True)

    def fwd_adj5():
        pm.projection_step(u, v, w, c5.dt, c5.nu, c5.fx, out=o)
        pm.projection_step_adjoint(u, v, w, *g, c5.dt, c5.nu, c5.fx, out=g)
    t = _time(fwd_adj5, steps, warmup=warmup)
    finite = bool(torch.isfinite(g[0]).all() and torch.isfinite(o[0]).all())
    res = {"fwd_adjoint_step_mixed_2048x768x2048": _leg(
        "fwd_adjoint_step_mixed", (c5.nx, c5.ny, c5.nz), t, finite=finite,
        plan_workspace_GB=round(pm.info()["workspace_bytes"] / 1e9, 1),
        input="perturbed Poiseuille (seeded torch CUDA generator), FP32 state")}
    del pm, u, v, w, o, g
    torch.cuda.empty_cache()
    return res


def secondary(wl, steps):
    """The other figures of the headline metric, each timed on resident inputs:
    FP64 vs mixed (FP32 + one FP64 refinement) Poisson solves on the step grid
    and on the 2048x512x1536 grid, and the FP64 forward + adjoint step."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    res = {}
    # the 64^3 FP64 Poisson solve (launch-bound: ~20 MB of model traffic)
    w1 = synth.WORKLOADS["poisson64"]
    p1 = Plan(w1.nx, w1.ny, w1.nz, w1.lx, w1.lz, w1.y_faces(), precision="fp64")
    f1 = torch.tensor(synth.uniform_rhs(w1.nx, w1.ny, w1.nz, seed=0), device=dev)
    o1 = torch.empty_like(f1)
    t = _time(lambda: p1.poisson_solve(f1, out=o1), 200, warmup=20)
    res["poisson_fp64_64x64x64"] = _leg("poisson_fp64", (w1.nx, w1.ny, w1.nz), t)
    _progress("poisson 64^3")
    del p1, f1, o1
    npts = wl.nx * wl.ny * wl.nz
    yf = wl.y_faces()
    f = torch.tensor(synth.uniform_rhs(wl.nx, wl.ny, wl.nz, seed=0), device=dev)
    p64 = torch.empty_like(f)
    pl = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, yf, precision="fp64")
    t = _time(lambda: pl.poisson_solve(f, out=p64), steps)
    res["poisson_fp64"] = _leg("poisson_fp64", (wl.nx, wl.ny, wl.nz), t)
    del pl
    pm = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, yf, precision="mixed", refine_passes=1)
    pmx = torch.empty_like(f)
    t = _time(lambda: pm.poisson_solve(f, out=pmx), steps)
    err = float(torch.linalg.vector_norm(pmx - p64) / torch.linalg.vector_norm(p64))
    res["poisson_mixed_refine1"] = _leg("poisson_mixed_refine1", (wl.nx, wl.ny, wl.nz), t, rel_l2_vs_fp64_gpu=err)
    _progress("poisson fp64 / mixed on the step grid")
    del pm, pmx, p64, f
    torch.cuda.empty_cache()
    # uniform y faces: tridiagonal (PDD) path vs the y-transform path
    yu = np.linspace(-1.0, 1.0, wl.ny + 1)
    fu = torch.tensor(synth.uniform_rhs(wl.nx, wl.ny, wl.nz, seed=0), device=dev)
    pu = {}
    for solver in ("pdd", "dct"):
        plu = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, yu, precision="fp64", y_solver=solver)
        out_u = torch.empty_like(fu)
        t = _time(lambda: plu.poisson_solve(fu, out=out_u), steps)
        pu[solver] = out_u
        res[f"poisson_fp64_uniform_y_{solver}"] = {"grid": [wl.nx, wl.ny, wl.nz], "ms": round(t * 1e3, 4),
                                                   "Mpts_s": round(npts / t / 1e6, 1)}
        del plu
    res["poisson_fp64_uniform_y_dct"]["rel_l2_vs_pdd"] = float(
        torch.linalg.vector_norm(pu["dct"] - pu["pdd"]) / torch.linalg.vector_norm(pu["pdd"]))
    del pu, fu
    torch.cuda.empty_cache()
    # forward + adjoint step, FP64
    pa = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, yf, precision="fp64", adjoint=True)
    u, v, w = (torch.tensor(q, device=dev) for q in synth.perturbed_poiseuille(wl.nx, wl.ny, wl.nz, yf, seed=0))
    o = tuple(torch.empty_like(u) for _ in range(3))
    g1 = tuple(torch.tensor(q, device=dev) for q in synth.random_directions(wl.nx, wl.ny, wl.nz, seed=1))
    go = tuple(torch.empty_like(u) for _ in range(3))

    def fwd_adj():
        pa.projection_step(u, v, w, wl.dt, wl.nu, wl.fx, out=o)
        pa.projection_step_adjoint(u, v, w, *g1, wl.dt, wl.nu, wl.fx, out=go)
    t = _time(fwd_adj, steps)
    res["fwd_adjoint_step_fp64"] = _leg("fwd_adjoint_step_fp64", (wl.nx, wl.ny, wl.nz), t)
    _progress("fwd+adjoint fp64")
    del pa, u, v, w, o, g1, go
    torch.cuda.empty_cache()
    res.update(time_loop_figures(wl, steps))
    _progress("time loop")
    res.update(rollout_figure(steps))
    _progress("rollout")
    # mixed-precision Poisson solve on the Re_tau=1000-shaped grid
    big = synth.WORKLOADS["mixed1000"]
    pm = Plan(big.nx, big.ny, big.nz, big.lx, big.lz, big.y_faces(), precision="mixed", refine_passes=1)
    vel = synth.powerlaw_velocity_device(big.nx, big.ny, big.nz, seed=0, device=dev)
    fb = pm.divergence(*vel)
    del vel
    torch.cuda.empty_cache()
    pb = torch.empty_like(fb)
    t = _time(lambda: pm.poisson_solve(fb, out=pb), max(2, steps // 2), warmup=1)
    ctr = measured_traffic("poisson_mixed", "mixed1000")
    res["poisson_mixed_refine1_2048x512x1536"] = _leg(
        "poisson_mixed_refine1", (big.nx, big.ny, big.nz), t,
        input="f = D u of the k^-5/3 power-law field (seed 0, generated on the device)",
        counter_bytes=ctr, counter_GBps=round(ctr / t / 1e9, 1) if ctr else None,
        counter_hbm_frac=round(ctr / t / 1e9 / HBM_PEAK_GBS, 4) if ctr else None)
    # the same right-hand side solved in FP64 (the metric's FP64 vs FP32+refine)
    p64 = Plan(big.nx, big.ny, big.nz, big.lx, big.lz, big.y_faces(), precision="fp64")
    t = _time(lambda: p64.poisson_solve(fb, out=pb), max(2, steps // 2), warmup=1)
    res["poisson_fp64_2048x512x1536"] = _leg("poisson_fp64", (big.nx, big.ny, big.nz), t)
    del p64
    _progress("poisson mixed / fp64 on 2048x512x1536")
    del pm, pb, fb
    torch.cuda.empty_cache()
    res.update(partition_tuning_figures())
    _progress("partition tuning")
    res.update(drop_figures(steps))
    _progress("dropped vs exact y-solve")
    res.update(slab_figures(steps))
    _progress("y-slab split")
    res.update(fwd_adjoint_mixed(steps=2, warmup=1))
    _progress("fwd+adjoint mixed 2048x768x2048")
    return res


def slab_figures(steps):
    """The wall-normal solve of the step grid split into 8 y-slabs of 32 rows
    (cf_solve_spectral_slabs; on eight devices each would run one slab, here
    they run one after another): mean time of one slab's local pass and of one
    finishing pass, the interface rows one slab contributes, and the one-pass
    solve for comparison."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    wl = synth.WORKLOADS["step550"]
    pl = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces(), precision="fp64")
    g = 8
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    fh = torch.randn(pl.nkx, wl.ny, wl.nz, dtype=torch.complex128, device=dev, generator=gen)
    out = torch.empty_like(fh)
    iface = torch.empty(pl.info()["slab_iface_bytes"], dtype=torch.uint8, device=dev)
    t_one = _time(lambda: pl.solve_spectral(fh, out=out), steps)
    t_all = _time(lambda: pl.solve_spectral_slabs(fh, g, out=out, iface=iface), steps)
    pl.set_timing(True)
    pl.reset_timing()
    for _ in range(steps):
        pl.solve_spectral_slabs(fh, g, out=out, iface=iface)
    torch.cuda.synchronize()
    tm = pl.timings()
    pl.set_timing(False)
    info = pl.info()
    res = {"pdd_8_slabs_fp64_1024x256x512": {
        "slabs": g, "rows_per_slab": wl.ny // g, "partitions_per_slab": info["n_parts"] // g,
        "local_us_per_slab": round(1e3 * tm["slab_local"][0] / tm["slab_local"][1], 1),
        "finish_us_per_slab": round(1e3 * tm["slab_finish"][0] / tm["slab_finish"][1], 1),
        "iface_MB_per_slab": round(info["slab_iface_bytes"] / g / 1e6, 2),
        "all_slabs_ms": round(t_all * 1e3, 4), "one_pass_ms": round(t_one * 1e3, 4)}}
    del pl, fh, out, iface
    torch.cuda.empty_cache()
    return res


def drop_figures(steps):
    """The wall-normal solve of the step grid with the default drop tolerance
    (the dropped reduced system as an outer PDD of 4 groups of 4 partitions on
    most lines) against the same plan with drop_tol = 0 (exact reduced system on
    every line): mean y-solve kernel time of each, lines dropped."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    dev = torch.device("cuda", 0)
    wl = synth.WORKLOADS["step550"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    res = {}
    fh = None
    for tag, tol in (("dropped", -1.0), ("exact", 0.0)):
        pl = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces(), precision="fp64", drop_tol=tol)
        if fh is None:
            fh = torch.randn(pl.nkx, wl.ny, wl.nz, dtype=torch.complex128, device=dev, generator=gen)
        out = torch.empty_like(fh)
        _time(lambda: pl.solve_spectral(fh, out=out), 3)
        pl.set_timing(True)
        pl.reset_timing()
        for _ in range(steps):
            pl.solve_spectral(fh, out=out)
        torch.cuda.synchronize()
        tm = pl.timings()
        pl.set_timing(False)
        inf = pl.info()
        us = 1e3 * tm["ysolve"][0] / tm["ysolve"][1]
        res[tag] = {"ysolve_us": round(us, 1), "GBps": round(2 * 16 * pl.nkx * wl.ny * wl.nz / (us * 1e-6) / 1e9, 1),
                    "n_dropped_lines": inf["n_dropped_lines"], "k2_threshold": inf["k2_threshold"]}
        res["n_lines"] = inf["n_lines"]
        res["drop_parts"] = inf["drop_parts"]
        del pl, out
    del fh
    torch.cuda.empty_cache()
    return {"ysolve_drop_vs_exact_fp64_1024x256x512": res}


def partition_tuning_figures():
    """The partitioned solve timed by a CF_PLAN_TUNE_PARTS plan at creation for
    every admissible (partitions, lines per block) pair, on the step grid (FP64)
    and the 2048x512x1536 grid (mixed): the chosen pair, its time and the
    default pair's time."""
    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan
    res = {}
    for name, prec in (("step550", "fp64"), ("mixed1000", "mixed")):
        w_ = synth.WORKLOADS[name]
        yf = w_.y_faces()
        t0 = time.perf_counter()
        pt = Plan(w_.nx, w_.ny, w_.nz, w_.lx, w_.lz, yf, precision=prec, tune_parts=True)
        t_create = time.perf_counter() - t0
        rows = pt.partition_timings()
        inf = pt.info()
        del pt
        pd = Plan(w_.nx, w_.ny, w_.nz, w_.lx, w_.lz, yf, precision=prec)
        dflt = (pd.info()["n_parts"], pd.info()["lines_per_block"])
        del pd
        us = {(r[0], r[1]): r[2] for r in rows}
        res[f"ysolve_tuning_{prec}_{w_.nx}x{w_.ny}x{w_.nz}"] = {
            "candidates": len(rows), "plan_create_ms": round(t_create * 1e3, 1),
            "chosen": [inf["n_parts"], inf["lines_per_block"]],
            "chosen_us": round(us[(inf["n_parts"], inf["lines_per_block"])], 1),
            "default": list(dflt), "default_us": round(us[dflt], 1) if dflt in us else None,
            "slowest_us": round(max(us.values()), 1)}
        torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="step550")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--secondary-steps", type=int, default=6,
                    help="timed calls per secondary figure (Poisson FP64/mixed, fwd+adjoint); 0 skips them")
    ap.add_argument("--poisson-only", action="store_true",
                    help="time the Poisson solve alone instead of the projection step")
    ap.add_argument("--summarize-pmc", metavar="DIR", help="print the traffic table of rocprofv3 --pmc passes and exit")
    ap.add_argument("--summarize-trace", metavar="CSV", help="print a rocprofv3 kernel_stats.csv as markdown and exit")
    ap.add_argument("--pmc-record", nargs=4, metavar=("DIR", "NAME", "WORKLOAD", "UNITS"),
                    help="print the traffic record of a whole path (step_fp64, poisson_mixed) from the counter "
                         "passes under DIR, per one of the UNITS steps or solves the profiled run made, and exit")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("DIR", "KERNEL"),
                    help="print the mean per dispatch of every counter of the --pmc passes under DIR for the "
                         "kernels whose name contains KERNEL, and exit")
    ap.add_argument("--pmc-exclude", nargs="*", default=[], metavar="NAME",
                    help="with --pmc-record: kernels (name substrings) to leave out, e.g. input generation")
    ap.add_argument("--trace-last", type=int, default=0, metavar="N",
                    help="with --summarize-trace on a run_kernel_trace.csv: the mean of each kernel's last N "
                         "dispatches")
    ap.add_argument("--profile-fwd-adjoint", type=int, default=0, metavar="STEPS",
                    help="only run STEPS FP64 forward + adjoint steps on the step grid (for a profiler) and exit")
    ap.add_argument("--profile-fwd-adjoint-mixed", action="store_true",
                    help="only run two mixed-precision forward + adjoint steps on 2048x768x2048 (for a "
                         "profiler) and exit")
    ap.add_argument("--profile-poisson-mixed", type=int, default=0, metavar="CALLS",
                    help="only run CALLS mixed-precision Poisson solves on 2048x512x1536 (after one warm-up "
                         "call; for a profiler) and exit")
    ap.add_argument("--source-hash", metavar="KERNEL", help="print the source hash a traffic summary of KERNEL "
                    "must carry and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain elementwise kernel reading and writing BYTES bytes "
                         "three times (reference for hardware traffic counters) and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc))
        return
    if args.summarize_counters:
        print(summarize_counters(*args.summarize_counters))
        return
    if args.pmc_record:
        d, name, workload, units = args.pmc_record
        print(pmc_record(d, name, workload, int(units), args.pmc_exclude))
        return
    if args.summarize_trace:
        print(summarize_trace_last(args.summarize_trace, args.trace_last) if args.trace_last
              else summarize_trace(args.summarize_trace))
        return
    if args.source_hash:
        print(kernel_source_hash(args.source_hash))
        return
    if args.profile_fwd_adjoint_mixed:
        fwd_adjoint_mixed(steps=2, warmup=0)
        return
    if args.profile_poisson_mixed:
        profile_poisson_mixed(args.profile_poisson_mixed)
        return
    if args.profile_fwd_adjoint:
        profile_fwd_adjoint(args.profile_fwd_adjoint)
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1.0, out=b)   # one kernel: reads n*8 bytes, writes n*8 bytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); "
              "the exchange between devices is not part of it", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2104_08863_amd import synth
    from paper_2104_08863_amd.api import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = synth.WORKLOADS[args.workload]
    yf = wl.y_faces()
    plan = Plan(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, yf, precision="fp64", step=not args.poisson_only)
    info = plan.info()
    if args.poisson_only:
        f = torch.tensor(synth.uniform_rhs(wl.nx, wl.ny, wl.nz, seed=0), device=dev)
        p = torch.empty_like(f)

        def step():
            plan.poisson_solve(f, out=p)
    else:
        u, v, w = (torch.tensor(q, device=dev) for q in
                   synth.perturbed_poiseuille(wl.nx, wl.ny, wl.nz, yf, seed=0))
        outs = tuple(torch.empty_like(u) for _ in range(3))
        p = torch.empty_like(u)

        def step():
            plan.projection_step(u, v, w, wl.dt, wl.nu, wl.fx, out=outs, p=p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.reset_timing()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_timing(False)
    tim = plan.timings()
    ms = (t1 - t0) * 1e3 / args.steps
    npts = wl.nx * wl.ny * wl.nz
    value = npts / (ms * 1e-3) / 1e6

    fused = not args.poisson_only
    kb = lambda k: kernel_bytes(k, wl.nx, wl.ny, wl.nz, 8, fused_div=fused)  # noqa: E731
    kern = {k: v for k, v in tim.items() if v[1] > 0}
    dom = max(kern, key=lambda k: kern[k][0])
    avg_ms = kern[dom][0] / kern[dom][1]
    nbytes = kb(dom)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    per_kernel = {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1],
                      "GBps": round(kb(k) / (v[0] / v[1] * 1e-3) / 1e9, 1)}
                  for k, v in kern.items()}
    model_bytes = sum(kb(k) * v[1] for k, v in kern.items()) / args.steps
    what = "FP64 pressure-Poisson solve" if args.poisson_only else "FP64 projection step (RK2 + Poisson + correction)"
    traffic = measured_traffic(dom, wl.name) if not args.poisson_only else None
    step_traffic = measured_traffic("step_fp64", wl.name) if not args.poisson_only else None
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {what} {wl.nx}x{wl.ny}x{wl.nz}, "
                               f"tanh y-grid factor {wl.gamma}, box {wl.lx:.4f}x{wl.lz:.4f}, "
                               f"dt {wl.dt}, nu {wl.nu:.6g}",
                   "nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "precision": "fp64",
                   "pdd_parts": info["n_parts"], "drop_lines": info["n_drop_lines"],
                   "lines": info["n_lines"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes": nbytes},
        "model_GBps_whole_step": round(model_bytes / (ms * 1e-3) / 1e9, 1),
        "hbm_frac_whole_step": round(model_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        # counter-measured bytes of one step (all its kernels) over this run's step time
        "counter_GBps_whole_step": (round(step_traffic / (ms * 1e-3) / 1e9, 1) if step_traffic else None),
        "measured_copy_GBps": copy_bandwidth(),
        "kernels": per_kernel,
    }
    if not args.poisson_only and args.secondary_steps > 0:
        del u, v, w, outs, p, plan
        torch.cuda.empty_cache()
        out["also"] = secondary(wl, args.secondary_steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.poisson_only)
        _progress("cpu baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
