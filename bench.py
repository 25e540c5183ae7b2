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
# source files of each kernel class (traffic figures are void once one changes)
TRSV_SOURCES = ("trsv.hip", "trsv_split.hip", "trsv_lds.hpp")
KERNEL_SOURCE = {"trsv_LB_W": TRSV_SOURCES, "trsv_UB_Z": TRSV_SOURCES, "trsv_LS": TRSV_SOURCES,
                 "trsv_US": TRSV_SOURCES, "spmv_A": ("krylov.hip",), "spmv_Coff": ("krylov.hip",),
                 "mgs": ("krylov.hip",)}
# block-local solve instance of each class: k_trsv_lds<G, E, DIAG> (schedule index, DIAG)
TRSV_ROLE = {"trsv_LB_W": (0, "false"), "trsv_UB_Z": (1, "true"), "trsv_LS": (2, "false"), "trsv_US": (3, "true")}
COPY_BYTES = 256 << 20  # the calibration copy: 256 MiB read, 256 MiB written
WORKLOADS = {
    # name: (generator key, options, rtol, restart)
    "aniso3d_128_slab16": ("aniso3d_128_slab16",
                           dict(method=1, interior_fact=2, interface_fact=1, droptol=1e-3, lfil=20, inner_iters=10),
                           1e-8, 50),
    "aniso3d_128_slab16_rap": ("aniso3d_128_slab16",
                               dict(method=2, interior_fact=1, smooth_fact=0, inner_iters=10), 1e-8, 50),
    "aniso2d_64": ("aniso2d_64", dict(method=0, interior_fact=0), 1e-8, 30),
    "rot9_512": ("rot9_512", dict(method=0, interior_fact=0), 1e-10, 30),
    "rot9_2048": ("rot9_2048", dict(method=0, interior_fact=0), 1e-10, 30),
}
DESCRIPTION = {
    "aniso3d_128_slab16": "3D 7-point -(u_xx + 0.1 u_yy + 0.01 u_zz), 128^3 (n=2097152, nnz=14581760), "
                          "16 z-slab subdomains; two-level additive Schur ILU: interior ILUT(1e-3, 20), "
                          "local Schur complements MILU(0), reduced system GMRES(10); FGMRES(50) to rtol 1e-8; "
                          "b = U(-1,1) seed 2",
    "aniso3d_128_slab16_rap": "the 128^3 16-slab operator and right-hand side with the multiplicative two-level "
                              "method: MILU(0) of each block for R, P and L_S U_S, ILU(0) smoother, GMRES(10) on "
                              "the unformed R A P; FGMRES(50) to rtol 1e-8",
    "aniso2d_64": "2D 5-point -(u_xx + 0.01 u_yy), 64^2, one block, ILU(0), FGMRES(30) to rtol 1e-8, b = A 1",
    "rot9_512": "2D 9-point rotated anisotropic diffusion (eps 1e-3, theta pi/6), 512^2 (n=262144), one block, "
                "ILU(0), FGMRES(30) to rtol 1e-10, b = U(-1,1) seed 3 (the mixed-precision operator at a quarter "
                "of its side)",
    "rot9_2048": "2D 9-point rotated anisotropic diffusion (eps 1e-3, theta pi/6), 2048^2 (n=4194304, "
                 "nnz=37724164), one block, ILU(0), FGMRES(30) to rtol 1e-10, b = U(-1,1) seed 3",
}


def source_hash(names) -> str:
    """Hash of one source file, or of several in the given order."""
    import hashlib

    h = hashlib.sha256()
    for name in ((names,) if isinstance(names, str) else names):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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
        if k < 2 and len(sched) > 21 and sched[20 + k] > 1:  # L_B or U_B split over workgroups
            return f"void silu::k_trsv_lds_x<{sched[4 * k + 1]}, {sched[4 * k + 2]}, {diag}, {prec}>"
        return f"void silu::k_trsv_lds<{sched[4 * k + 1]}, {sched[4 * k + 2]}, {diag}, {prec}, {fast(k)}>"
    # the outer orthogonalisation: one k_arnoldi launch per Arnoldi step (w from the product, not a sum)
    return {"spmv_A": "void silu::k_spmv<0>", "spmv_Coff": "void silu::k_spmv<1>",
            "mgs": "void silu::k_arnoldi<"}.get(cls)


def measured_traffic(cls: str, sched, prec: int = 0):
    """HBM bytes per launch of a kernel class from profiles/traffic.json (counter runs of this workload), or None
    when there is none or the kernel's source changed since the counters were taken."""
    inst = kernel_instance(cls, sched, prec)
    if inst is None or not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        tj = json.load(f)
    for name, rec in tj.get("kernels", {}).items():
        if cls == "mgs" and ", false>" not in name:
            continue
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
        src = (TRSV_SOURCES if "k_trsv" in name
               else "krylov.hip" if ("k_spmv" in name or "k_mgs" in name or "k_arnoldi" in name)
               else "batch.hip" if "k_batch_solve" in name else None)
        if src is None:
            continue
        fb, wb = fetch[name] * cf, write.get(name, 0.0) * cw
        out["kernels"][name] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                                "source_sha": source_hash(src)}
    with open(traffic_json(workload), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


def traffic_json(workload: str) -> str:
    """Counter summary file of a workload (the default workload keeps the historical name)."""
    if workload == "aniso3d_128_slab16":
        return TRAFFIC_JSON
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def batch_traffic():
    """HBM bytes per launch of the batched kernel from its counter runs, or None (no file, or the kernel's
    source has changed since)."""
    try:
        with open(traffic_json("convdiff_batch512")) as f:
            tj = json.load(f)
    except OSError:
        return None
    for name, rec in tj.get("kernels", {}).items():
        if "k_batch_solve" in name and rec.get("source_sha") == source_hash("batch.hip"):
            return rec["bytes_per_launch"]
    return None


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


# ---------------------------------------------------------------------------
# batched systems: 512 convection-diffusion systems, ILU(0) + GMRES(20) each, one persistent launch
# ---------------------------------------------------------------------------
BATCH_COUNT, BATCH_SEED, BATCH_RESTART, BATCH_RTOL, BATCH_MAXIT = 512, 4, 20, 1e-8, 5000


def batch_algorithmic_bytes(mats, its, m):
    """Algorithmic bytes of one batched launch, counted as the measurement table does: per system the ILU(0)
    numeric factorization (12 bytes read and 8 written per entry), and per GMRES iteration one SpMV
    (12 nnz + 4(n+1) + 16n), the L and U solves (12 nnz(strict L or U) + 4(n+1) + 16n, + 8n for U's diagonal)
    and the MGS step of its Arnoldi index j (2j + 4) 8n; plus per restart cycle the true residual and the
    update x += M^-1 V c (V read once, two solves)."""
    total = 0.0
    for M, it in zip(mats, its):
        n, nnz = M.n, M.nnz
        rows = np.repeat(np.arange(n), np.diff(M.row_ptr))
        nl = int(np.count_nonzero(M.col < rows))
        nu = int(np.count_nonzero(M.col > rows))
        spmv = 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n
        trsv = 12.0 * (nl + nu) + 8.0 * (n + 1) + 32.0 * n + 8.0 * n
        total += 20.0 * nnz
        cycles = -(-int(it) // m) if it else 0
        for k in range(int(it)):
            j = k % m
            total += spmv + trsv + (2 * j + 4) * 8.0 * n
        total += cycles * (spmv + 8.0 * n + trsv + 8.0 * n * (m + 1))
    return total


def batch_cpu_worker(first: int, count: int) -> None:
    """Oracle process of the batched baseline: ILU(0) + GMRES(20) of systems first .. first+count-1."""
    import oracle
    import synth

    params = synth.convdiff_batch_params(BATCH_COUNT, BATCH_SEED)[first:first + count]
    t = 0.0
    done = 0
    for p in params:
        M = synth.convdiff5(*p)
        b = M.matvec(np.ones(M.n))
        t0 = time.perf_counter()
        P = oracle.Precond(M, None, 1, method=oracle.BJ, interior_fact=oracle.ILU0)
        oracle.gmres(M, P, b, rtol=BATCH_RTOL, restart=BATCH_RESTART, maxit=BATCH_MAXIT)
        t += time.perf_counter() - t0
        done += 1
    print(json.dumps({"systems": done, "seconds": t}), flush=True)


def copy_calibration(dev) -> None:
    """One 256 MiB device copy: the known traffic that scales the counter runs."""
    import torch

    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def bench_batch(args) -> None:
    import torch

    import paper_2303_08881_amd as silu
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        copy_calibration(dev)
    mats, bs = synth.convdiff_batch(BATCH_COUNT, BATCH_SEED)
    A, sr = synth.block_diagonal(mats)
    Ad = silu.DeviceCSR.from_host(A, dev)
    bd = torch.as_tensor(np.concatenate(bs)).to(dev)
    x = torch.zeros_like(bd)
    side = torch.cuda.Stream()
    m = BATCH_RESTART
    with torch.cuda.stream(side):
        B = silu.batch_setup(Ad, sr, restart=m)
        merge, wpc, threads, tune_ms = B.tune(Ad.val, bd, x, rtol=BATCH_RTOL, restart=m, maxit=BATCH_MAXIT)
        x.zero_()
        B.capture(Ad.val, bd, x, rtol=BATCH_RTOL, restart=m, maxit=BATCH_MAXIT)
        for _ in range(max(args.warmup, 1)):
            x.zero_()
            B.replay()
        side.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        launch_ms = []
        t_start = time.perf_counter()
        for _ in range(args.steps):
            x.zero_()
            e0.record()
            B.replay()
            e1.record()
            e1.synchronize()
            launch_ms.append(e0.elapsed_time(e1))
        side.synchronize()
        total = time.perf_counter() - t_start
    its, rel, st = B.results()
    sched = [int(v) for v in B.export("schedule")]
    nbytes = batch_algorithmic_bytes(mats, its, m)
    avg_ms = float(np.mean(launch_ms))
    gbs = nbytes / (avg_ms * 1e-3) / 1e9
    result = {
        "metric": "solves/s + p50/p99 latency at rtol 1e-8; TRSV/SpMV HBM GB/s vs plain FP64",
        "value": round(BATCH_COUNT * args.steps / total, 2),
        "unit": "systems/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "convdiff_batch512",
                   "description": "512 independent 2D 5-point upwind convection-diffusion systems, sides "
                                  "log-uniform in [32, 256], eps log-U[1e-3, 1], theta U[0, pi), Pe U[0, 50], "
                                  "seed 4; ILU(0) + GMRES(20) to rtol 1e-8 each, factorization and solve of "
                                  "all systems in one persistent launch, replayed from a HIP graph",
                   "systems": BATCH_COUNT, "n": A.n, "nnz": A.nnz, "restart": m, "rtol": BATCH_RTOL},
        "launch_ms_p50": round(float(np.percentile(launch_ms, 50)), 3),
        "launch_ms_p99": round(float(np.percentile(launch_ms, 99)), 3),
        "schedule": {"entries_per_row": sched[0], "merge": sched[1], "workgroups_per_cu": sched[2],
                     "grid": sched[3], "threads": sched[4], "tuned_ms": round(tune_ms, 3)},
        "iterations": {"min": int(its.min()), "median": int(np.median(its)), "max": int(its.max()),
                       "total": int(its.sum())},
        "all_converged": bool(np.all(st == 0)), "max_relres": float(rel.max()),
        "roofline": {"kernel": "k_batch_solve", "bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": batch_traffic(),
                     "avg_launch_us": round(avg_ms * 1e3, 1), "bytes_per_launch": nbytes},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        import subprocess

        sample = 16
        cmd = [sys.executable, os.path.abspath(__file__), "--batch-cpu-worker", "0", str(sample)]
        env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
        so = subprocess.run(cmd, stdout=subprocess.PIPE, env=env, text=True, check=True).stdout
        o = json.loads(so.strip().splitlines()[-1])
        result["cpu_baseline"] = {"value": round(o["systems"] / o["seconds"], 3), "unit": "systems/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"the first {sample} of the 512 systems (setup + GMRES(20) each), one "
                                            "process", "cpu_model": cpu_model()}
    print(json.dumps(result), flush=True)


# ---------------------------------------------------------------------------
# serving: Poisson arrivals of mixed requests, resident factors per matrix id
# ---------------------------------------------------------------------------
SERVE_REQUESTS, SERVE_SLOTS, SERVE_RESTART, SERVE_RTOL, SERVE_MAXIT = 64, 4, 50, 1e-8, 2000
SERVE_BUDGET = 96 << 30


def bench_serve(args) -> None:
    import threading

    import torch

    import paper_2303_08881_amd as silu
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    reqs = synth.request_stream(SERVE_REQUESTS, seed=5)
    mats, ddev = {}, {}
    for r in reqs:
        if r.matrix_id not in mats:
            A, part, p = synth.build_matrix(r)
            mats[r.matrix_id] = (A, p)
            ddev[r.matrix_id] = (silu.DeviceCSR.from_host(A, dev), torch.as_tensor(part).to(dev), p)
    bs = [torch.as_tensor(synth.uniform_rhs(mats[r.matrix_id][0].n, r.rhs_seed)).to(dev) for r in reqs]
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    base = dict(method=silu.SCHUR, interior_fact=silu.ILU0, interface_fact=silu.MILU0, inner_iters=3)

    def run(slots, prec, arrivals=None):
        """One pass over the stream on a fresh server; arrivals None = all queued at once (closed loop)."""
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        S = silu.Server(slots=slots, budget_bytes=SERVE_BUDGET, factor_prec=prec, **base)
        recs = []
        submitted = threading.Semaphore(0)

        def collect():
            for _ in reqs:
                submitted.acquire()  # a completion can only follow a submission
                recs.append(S.wait())

        waiter = threading.Thread(target=collect)
        t0 = time.perf_counter()
        waiter.start()
        for q, r in enumerate(reqs):
            if arrivals is not None:
                delay = t0 + arrivals[q] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            Ad, pd, p = ddev[r.matrix_id]
            S.submit(r.matrix_id, bs[q], xs[q], A=Ad, part=pd, nparts=p, rtol=SERVE_RTOL, restart=SERVE_RESTART,
                     maxit=SERVE_MAXIT, sync=False)
            submitted.release()
        waiter.join()
        st = S.stats()
        S.close()
        first = min(rec["submit_us"] for rec in recs)
        last = max(rec["done_us"] for rec in recs)
        lat = np.array([(rec["done_us"] - rec["submit_us"]) * 1e-3 for rec in recs])
        return {"solves_per_s": round(len(recs) / ((last - first) * 1e-6), 3),
                "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "all_converged": all(rec["status"] == 0 for rec in recs),
                "max_relres": max(rec["final_relres"] for rec in recs),
                "iterations_total": int(sum(rec["iterations"] for rec in recs)),
                "setup_ms_total": round(sum(rec["setup_ms"] for rec in recs), 2),
                "solve_ms_total": round(sum(rec["solve_ms"] for rec in recs), 2),
                "hits": st["hits"], "misses": st["misses"], "peak_bytes": st["peak_bytes"]}

    for _ in range(max(args.warmup, 1)):
        run(SERVE_SLOTS, silu.PREC_F32)
    t_start = time.perf_counter()
    closed = [run(SERVE_SLOTS, silu.PREC_F32) for _ in range(args.steps)]
    total = time.perf_counter() - t_start
    cap = float(np.median([c["solves_per_s"] for c in closed]))
    sweep = []
    for frac in (0.25, 0.5, 0.75, 1.0, 1.25):
        rate = frac * cap
        res = run(SERVE_SLOTS, silu.PREC_F32, synth.arrival_times(len(reqs), rate))
        sweep.append(dict(offered_per_s=round(rate, 3), **res))
    plain = run(1, silu.PREC_F64)
    serial32 = run(1, silu.PREC_F32)
    ns = sorted(a.n for a, _ in mats.values())
    result = {
        "metric": "solves/s + p50/p99 latency at rtol 1e-8; TRSV/SpMV HBM GB/s vs plain FP64",
        "value": round(cap, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "serve_mixed64",
                   "description": "64 requests (seed 5): half anisotropic 2D/3D diffusion, half power-law "
                                  "nonsymmetric, n log-U[1e3, 1e6], 70% new right-hand sides for one of the "
                                  "last 32 matrix ids; two-level ILU (ILU(0) interior, MILU(0) local Schur "
                                  "complements, 3 inner GMRES steps) with FP32 factors inside FP64 FGMRES(50) "
                                  "to rtol 1e-8; 4 slots, device-memory budget 96 GiB; one step = the whole "
                                  "stream queued at once on a fresh server",
                   "requests": len(reqs), "matrices": len(mats), "n_min": ns[0], "n_max": ns[-1],
                   "slots": SERVE_SLOTS},
        "p50_ms": closed[-1]["p50_ms"], "p99_ms": closed[-1]["p99_ms"],
        "closed_loop": closed[-1],
        "rate_sweep": sweep,
        "plain_fp64_one_slot": plain,
        "fp32_one_slot": serial32,
        "speedup_vs_plain_fp64": round(cap / plain["solves_per_s"], 3),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="aniso3d_128_slab16",
                    choices=sorted(WORKLOADS) + ["convdiff_batch512", "serve_mixed64"])
    ap.add_argument("--batch-cpu-worker", nargs=2, type=int, help=argparse.SUPPRESS)
    ap.add_argument("--factor-prec", default="f64", choices=["f64", "f32", "f16"],
                    help="storage precision of the triangular factors (the solves run in FP32 for f32 and f16; "
                         "everything else stays FP64)")
    ap.add_argument("--trsv-mode", default="auto", choices=["auto", "levels", "block"],
                    help="triangular solve execution (ilu_options_t.trsv_mode)")
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
    if args.batch_cpu_worker:
        batch_cpu_worker(*args.batch_cpu_worker)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the subdomains of this solver live on one "
              "device at their real per-GPU shape and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "convdiff_batch512":
        bench_batch(args)
        return
    if args.workload == "serve_mixed64":
        bench_serve(args)
        return

    import torch

    import paper_2303_08881_amd as silu
    import synth

    key, opts, rtol, restart = WORKLOADS[args.workload]
    prec = {"f64": 0, "f32": 1, "f16": 2}[args.factor_prec]
    opts = dict(opts, factor_prec=prec, trsv_mode={"auto": 0, "levels": 1, "block": 2}[args.trsv_mode])
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
        copy_calibration(dev)
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
                   "subdomains": nparts, "restart": restart, "rtol": rtol, "factor_prec": args.factor_prec,
                   "trsv_mode": args.trsv_mode},
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
