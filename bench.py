"""Benchmark: cold solves/s of the two-level Schur-complement ILU + FGMRES on one GPU.

One step = the whole hot path on one synthetic system: ilu_setup (interface
classification, permutation, partial ILUT of the subdomain blocks, MILU(0) of
the local Schur complements, level analysis) followed by fgmres_solve (each
iteration: the preconditioner apply -- L_B solve with W rows, the reduced
Schur system by GMRES(10) preconditioned with the local Schur factors, U_B
solve with the Z columns -- SpMV and modified Gram-Schmidt) to rtol 1e-8.
Inputs are generated once and are resident in HBM before the timed region.

Prints one JSON line.  The roofline entry is for the kernel class with the
largest summed duration (every class is timed on the last warm-up step, which
also gives the "kernels" breakdown); inside the timed region only that class
is timed, with HIP events on the stream the kernels run on
(ilu_kernel_timing), so the events of the other classes do not slow the
measured solves.  The CPU baseline times the
FP64 oracle on the host on a bounded sample (its full setup plus a few outer
iterations) and scales it to one solve with the GPU's iteration count.
`--factor-prec f32|f16` stores the triangular factors in FP32 / FP16 (solves
in FP32, everything else FP64); `--workload` picks another synthetic system.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS = ["trsv_LB_W", "trsv_UB_Z", "trsv_LS", "trsv_US", "spmv_A", "spmv_Coff", "mgs"]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_2303_08881_amd", "csrc")
# source file of each kernel class (traffic figures are void once it changes)
KERNEL_SOURCE = {"trsv_LB_W": "trsv.hip", "trsv_UB_Z": "trsv.hip", "trsv_LS": "trsv.hip", "trsv_US": "trsv.hip",
                 "spmv_A": "krylov.hip", "spmv_Coff": "krylov.hip", "mgs": "krylov.hip"}
# block-local solve instance of each class: k_trsv_lds<G, E, DIAG> (schedule index, DIAG)
TRSV_ROLE = {"trsv_LB_W": (0, "false"), "trsv_UB_Z": (1, "true"), "trsv_LS": (2, "false"), "trsv_US": (3, "true")}
COPY_BYTES = 256 << 20  # the calibration copy: 256 MiB read, 256 MiB written
WORKLOADS = {
    # name: (generator key, options, rtol, restart)
    "aniso3d_128_slab16": ("aniso3d_128_slab16",
                           dict(method=1, interior_fact=2, interface_fact=1, droptol=1e-3, lfil=20, inner_iters=10),
                           1e-8, 50),
    "aniso2d_64": ("aniso2d_64", dict(method=0, interior_fact=0), 1e-8, 30),
    "rot9_512": ("rot9_512", dict(method=0, interior_fact=0), 1e-10, 30),
}
DESCRIPTION = {
    "aniso3d_128_slab16": "3D 7-point -(u_xx + 0.1 u_yy + 0.01 u_zz), 128^3 (n=2097152, nnz=14581760), "
                          "16 z-slab subdomains; two-level additive Schur ILU: interior ILUT(1e-3, 20), "
                          "local Schur complements MILU(0), reduced system GMRES(10); FGMRES(50) to rtol 1e-8; "
                          "b = U(-1,1) seed 2",
    "aniso2d_64": "2D 5-point -(u_xx + 0.01 u_yy), 64^2, one block, ILU(0), FGMRES(30) to rtol 1e-8, b = A 1",
    "rot9_512": "2D 9-point rotated anisotropic diffusion (eps 1e-3, theta pi/6), 512^2 (n=262144), one block, "
                "ILU(0), FGMRES(30) to rtol 1e-10, b = U(-1,1) seed 3 (the mixed-precision operator at a quarter "
                "of its side)",
}


def source_hash(name: str) -> str:
    import hashlib

    with open(os.path.join(CSRC, name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_instance(cls: str, sched, prec: int = 0) -> str | None:
    """Kernel (demangled name prefix) that runs a kernel class in this workload (prec: storage precision of the
    triangular factors, 0 FP64, 1 FP32, 2 FP16)."""
    if cls in TRSV_ROLE:
        k, diag = TRSV_ROLE[cls]
        if sched is None or not sched[4 * k]:
            return None
        fast = lambda b: "true" if (sched[17] >> b) & 1 else "false"  # noqa: E731
        if cls == "trsv_LS" and sched[16]:  # L_S and U_S in one launch (fast only if both are)
            both = "true" if (sched[17] >> 2) & (sched[17] >> 3) & 1 else "false"
            return f"void silu::k_trsv_lds_pair<{sched[9]}, {sched[10]}, {prec}, {both}>"
        return f"void silu::k_trsv_lds<{sched[4 * k + 1]}, {sched[4 * k + 2]}, {diag}, {prec}, {fast(k)}>"
    return {"spmv_A": "void silu::k_spmv<0>", "spmv_Coff": "void silu::k_spmv<1>",
            "mgs": "void silu::k_mgs_step<"}.get(cls)


def measured_traffic(cls: str, sched, prec: int = 0):
    """HBM bytes per launch of a kernel class from profiles/traffic.json (counter runs of this workload), or None
    when there is none or the kernel's source changed since the counters were taken."""
    inst = kernel_instance(cls, sched, prec)
    if inst is None or not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        tj = json.load(f)
    for name, rec in tj.get("kernels", {}).items():
        if name.startswith(inst) and rec.get("source_sha") == source_hash(KERNEL_SOURCE[cls]):
            return rec["bytes_per_launch"]
    return None


def summarize_pmc(fetch_csv: str, write_csv: str, workload: str) -> None:
    """Write profiles/traffic.json from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of
    `bench.py --copy-calibration`: each counter is scaled by what it reads for the 256 MiB device copy."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        """Mean counter bytes per dispatch of each kernel, and the largest device-copy dispatch."""
        acc, copy = defaultdict(list), 0.0
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") == counter:
                    b = float(row["Counter_Value"]) * 1024.0
                    acc[row["Kernel_Name"]].append(b)
                    if "copyBuffer" in row["Kernel_Name"]:
                        copy = max(copy, b)
        return {k: sum(v) / len(v) for k, v in acc.items()}, copy

    (fetch, cfb), (write, cwb) = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    if cfb < COPY_BYTES / 4 or cwb < COPY_BYTES / 4:
        raise SystemExit("no calibration copy in the counter runs (run bench.py with --copy-calibration)")
    cf, cw = COPY_BYTES / cfb, COPY_BYTES / cwb
    out = {"workload": workload, "calibration": {"copy_bytes": COPY_BYTES, "fetch_counter_bytes": cfb,
                                                  "write_counter_bytes": cwb, "fetch_factor": cf,
                                                  "write_factor": cw},
           "kernels": {}}
    for name in fetch:
        src = "trsv.hip" if "k_trsv" in name else "krylov.hip" if ("k_spmv" in name or "k_mgs" in name) else None
        if src is None:
            continue
        fb, wb = fetch[name] * cf, write.get(name, 0.0) * cw
        out["kernels"][name] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                                "source_sha": source_hash(src)}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out["calibration"]))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_worker(workload: str, factor_prec: str, sample_iters: int) -> None:
    """One oracle process of the CPU baseline: full setup plus a bounded number of FGMRES iterations on the
    workload's system; prints its timings as one JSON line."""
    import oracle
    import synth

    key, opts, rtol, restart = WORKLOADS[workload]
    A, b, part, nparts = synth.workload(key)
    t0 = time.perf_counter()
    P = oracle.Precond(A, part if nparts > 1 else None, nparts, **opts)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    out = oracle.fgmres(A, P, b, rtol=rtol, restart=restart, maxit=sample_iters)
    t_iter = (time.perf_counter() - t0) / max(out["iterations"], 1)
    print(json.dumps({"t_setup": t_setup, "t_iter": t_iter, "iterations": out["iterations"]}), flush=True)


def _run_workers(workload, factor_prec, sample_iters, count):
    import subprocess

    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", "--workload", workload,
           "--factor-prec", factor_prec, "--cpu-sample-iters", str(sample_iters)]
    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, env=env, text=True) for _ in range(count)]
    outs = []
    for p in procs:
        so, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed with status {p.returncode}")
        outs.append(json.loads(so.strip().splitlines()[-1]))
    return outs


def cpu_baseline(workload, factor_prec, gpu_iters, sample_iters, cores):
    """The FP64 oracle, unchanged, on the host: one process alone (the one-core rate), then `cores` processes at
    once, each on the same bounded sample (its full setup plus `sample_iters` FGMRES iterations); every process's
    timings are scaled to one solve with the GPU's iteration count and the all-core rate is their sum."""
    one = _run_workers(workload, factor_prec, sample_iters, 1)[0]
    rate = lambda o: 1.0 / (o["t_setup"] + gpu_iters * o["t_iter"])  # noqa: E731
    many = _run_workers(workload, factor_prec, sample_iters, cores) if cores > 1 else [one]
    return {
        "value": sum(rate(o) for o in many),
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{cores} oracle processes at once, each: full setup + {many[0]['iterations']} FGMRES iterations "
                  f"of this workload, scaled to {gpu_iters} iterations per solve; rate = sum over processes",
        "cpu_model": cpu_model(),
        "one_core_value": rate(one),
        "oracle_setup_s": one["t_setup"],
        "oracle_s_per_iteration": one["t_iter"],
        "all_core_setup_s": float(np.median([o["t_setup"] for o in many])),
        "all_core_s_per_iteration": float(np.median([o["t_iter"] for o in many])),
    }


def chain_probe(silu, dev, levels=8192, reps=20):
    """Per-level time of the block-local triangular solve on a tridiagonal matrix (one row per level, so every
    level is one dependent step with no bandwidth to speak of): the floor of a level-scheduled chain."""
    import ctypes as C

    import torch

    import synth

    T = synth.aniso5(levels, 1.0, Ny=1)  # tridiagonal: L and U are chains of `levels` levels
    Ad = silu.DeviceCSR.from_host(T, dev)
    P = silu.setup(Ad, None, 1, method=silu.BJ, interior_fact=silu.ILU0, trsv_mode=silu.TRSV_BLOCK)
    r = torch.ones(T.n, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    lib = silu.lib()
    P.apply(r, z)
    torch.cuda.synchronize()
    lib.ilu_kernel_stats(0, None, None, None, 1)
    lib.ilu_kernel_timing(1)
    for _ in range(reps):
        P.apply(r, z)
    torch.cuda.synchronize()
    lib.ilu_kernel_timing(0)
    ms, cnt = C.c_double(), C.c_int64()
    lib.ilu_kernel_stats(0, C.byref(ms), C.byref(cnt), None, 1)
    P.close()
    return 1e3 * ms.value / max(cnt.value, 1) / levels


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="aniso3d_128_slab16", choices=sorted(WORKLOADS))
    ap.add_argument("--factor-prec", default="f64", choices=["f64", "f32", "f16"],
                    help="storage precision of the triangular factors (the solves run in FP32 for f32 and f16; "
                         "everything else stays FP64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=40)
    ap.add_argument("--cpu-cores", type=int, default=min(16, os.cpu_count() or 1),
                    help="oracle processes of the all-core CPU baseline")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device copy before the steps (scale for counter runs)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter files and exit")
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.workload, args.factor_prec, args.cpu_sample_iters)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the subdomains of this solver live on one "
              "device at their real per-GPU shape and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2303_08881_amd as silu
    import synth

    key, opts, rtol, restart = WORKLOADS[args.workload]
    prec = {"f64": 0, "f32": 1, "f16": 2}[args.factor_prec]
    opts = dict(opts, factor_prec=prec)
    A, b, part, nparts = synth.workload(key)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Ad = silu.DeviceCSR.from_host(A, dev)
    bd = torch.as_tensor(b).to(dev)
    pd = torch.as_tensor(part).to(dev) if nparts > 1 else None
    maxit = 2000

    def step():
        P = silu.setup(Ad, pd, nparts, **opts)
        out = silu.fgmres(Ad, P, bd, rtol=rtol, restart=restart, maxit=maxit)
        P.close()
        return out

    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    import ctypes as C

    lib = silu.lib()

    def kernel_stats():
        out = {}
        for k, name in enumerate(KERNELS):
            ms, cnt, by = C.c_double(), C.c_int64(), C.c_double()
            lib.ilu_kernel_stats(k, C.byref(ms), C.byref(cnt), C.byref(by), 1)
            if cnt.value:
                out[name] = dict(total_ms=ms.value, launches=cnt.value, avg_us=1e3 * ms.value / cnt.value,
                                 bytes_per_launch=by.value / cnt.value,
                                 gbs=by.value / (ms.value * 1e-3) / 1e9 if ms.value > 0 else 0.0)
        return out

    # Every kernel class is timed on the last warm-up step (the breakdown and
    # the choice of the dominant class); in the timed region only the dominant
    # class is, since each event pair adds time to the launch it brackets.
    kernel_stats()
    warm = {}
    for i in range(args.warmup):
        if i == args.warmup - 1:
            lib.ilu_kernel_timing(silu.KERNEL_ALL)
        step()
    torch.cuda.synchronize()
    lib.ilu_kernel_timing(0)
    if args.warmup:
        warm = kernel_stats()
    dom = max(warm, key=lambda k: warm[k]["total_ms"]) if warm else None
    lib.ilu_kernel_timing((1 << KERNELS.index(dom)) if dom else silu.KERNEL_ALL)
    torch.cuda.synchronize()
    lat, outs = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        outs.append(step())
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    lib.ilu_kernel_timing(0)
    live = kernel_stats()
    if dom is None and live:
        dom = max(live, key=lambda k: live[k]["total_ms"])
    kstats = warm or live
    roof = None
    if dom and dom in live:
        d = live[dom]
        P = silu.setup(Ad, pd, nparts, **opts)
        sched = [int(v) for v in P.export("schedule")]
        P.close()
        roof = {"kernel": dom, "instance": kernel_instance(dom, sched, prec), "bound": "hbm",
                "achieved": round(d["gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["gbs"] / HBM_PEAK_GBS, 5), "traffic": measured_traffic(dom, sched, prec),
                "avg_launch_us": round(d["avg_us"], 3), "bytes_per_launch": d["bytes_per_launch"],
                "launches": d["launches"]}
        if dom in TRSV_ROLE:
            # level-chain bound of the dominant solve: its levels per launch times
            # the per-level time of a one-row-per-level chain
            lev = {"trsv_LB_W": ["lev_LB"], "trsv_UB_Z": ["lev_UB"], "trsv_US": ["lev_US"],
                   "trsv_LS": ["lev_LS", "lev_US"] if sched[16] else ["lev_LS"]}[dom]
            P = silu.setup(Ad, pd, nparts, **opts)
            lv = [P.export(k) for k in lev]
            P.close()
            # block-local: each subdomain's chain runs on its own workgroup, so a
            # launch lasts as long as the longest per-subdomain chain
            nlev = sum(int(v.max()) + 1 if v.size else 0 for v in lv)
            t_level = chain_probe(silu, dev)
            roof.update(chain_levels=nlev, level_step_us=round(t_level, 5),
                        chain_bound_us=round(nlev * t_level, 3),
                        chain_frac=round(nlev * t_level / d["avg_us"], 4))

    its = [o["iterations"] for o in outs]
    lat_ms = np.array(lat) * 1e3
    result = {
        "metric": "solves/s + p50/p99 latency at rtol 1e-8; TRSV/SpMV HBM GB/s vs plain FP64",
        "value": round(args.steps / total, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # arithmetic of the path: FP64 throughout, or the triangular solves in
        # FP32 (factors stored in FP32 / FP16) beside FP64 Krylov and SpMV
        "dtype": {0: "f64", 1: "f32+f64", 2: "f32+f64 (f16 factors)"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "description": DESCRIPTION[args.workload], "n": A.n, "nnz": A.nnz,
                   "subdomains": nparts, "restart": restart, "rtol": rtol, "factor_prec": args.factor_prec},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "setup_ms": round(float(np.mean([o["setup_ms"] for o in outs])), 3),
        "solve_ms": round(float(np.mean([o["solve_ms"] for o in outs])), 3),
        # warm solves/s: a new right-hand side for factors already on the
        # device (the solve part of each step alone)
        "warm_solves_per_s": round(1e3 / float(np.mean([o["solve_ms"] for o in outs])), 4),
        "iterations": int(np.median(its)),
        "relres": max(o["relres"] for o in outs),
        "converged": all(o["converged"] for o in outs),
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kstats.items()},
        "kernels_timed_on": "last warm-up step" if warm else "timed region",
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.workload, args.factor_prec, result["iterations"],
                                              args.cpu_sample_iters, args.cpu_cores)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
