"""Benchmark of the explicit leapfrog wave solver on one MI355X.

One bench step = the whole forward hot path over the 8192 x 8192 point-singularity workload
(h = 1 + 5 phi_eps(r), eps = 4 dx, four seeded humps, tau = 0.5 dx / sqrt(max h)):
face/validation of the coefficient, Taylor start, 5000 leapfrog steps with the discrete
energy of every step, and a snapshot of the final field.  Inputs are resident in HBM before
the timed region.  `value` = interior grid-point updates per second (FP32 storage).

Also reported (same JSON line): the same workload in FP64, the 32-member batched family of
regularisations (512^2 .. 4096^2, 2000 steps each, one persistent launch), the adjoint /
forward time ratio of the 2048^2 FP64 receiver-misfit gradient (4000 steps, checkpoints every
64), the roofline of the dominant kernel (HIP events on the solver's stream) and the FP64 CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-extra] [--skip-cpu]
       python bench.py --profile-run [--dtype f32|f64]   (short run for rocprofv3: three 800-step
                        forward solves plus three plain copies used to calibrate the counters)
       python bench.py --profile-run --adjoint   (short run of the reverse sweep for rocprofv3)
       python bench.py --profile-run --workload bathymetry16384|family|implicit4096|line256   (other short runs)
       python bench.py --summarize-profile DIR [DIR ...] --out NAME (writes profiles/NAME.txt,
                        and NAME.json with calibrated bytes per launch, from rocprofv3 CSV files)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "grid-point updates/s + % HBM roofline (fwd, batched); adjoint/forward time ratio"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("fdw_stream.h", "fdw_step_f32c2.hip", "fdw_step_f32c4.hip", "fdw_internal.h"):
        with open(os.path.join(ROOT, "paper_2005_11931_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str, launch_nodes: int):
    """HBM traffic per launch from a committed rocprofv3 counter summary, if it was taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def forward_bench(fdw, torch, I, dtype, steps, warmup, n=8192, nsteps=5000):
    case = I.point_case(n=n, nsteps=nsteps)
    td = fdw.torch_dtype(dtype)
    s = fdw.solver_for_case(case, dtype=dtype)
    h = torch.as_tensor(case.h1, dtype=td, device="cuda")
    energy = torch.empty((1, nsteps), dtype=torch.float64, device="cuda")
    snap = torch.empty((n, n), dtype=td, device="cuda")
    del case
    updates = (n - 2) * (n - 2) * nsteps

    def one():
        s.set_coeff(h)
        s.step_into(nsteps, energy)
        s._check(fdw.lib().fdw_get_state(s.ctx, 0, fdw._ptr(snap), None, None))

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    e = energy[0].cpu().numpy()
    drift = float(abs(e - e[0]).max() / e[0])
    # dominant kernel: the streaming stencil; average launch duration from HIP events
    s.configure(fdw.FDW_CFG_TIMING, 1)
    s.kernel_time()
    s.set_coeff(h)
    s.step_into(nsteps, energy)
    ms, launches = s.kernel_time()
    K = s.config(fdw.FDW_CFG_TIME_BLOCK)
    S = s.config(fdw.FDW_CFG_SEGMENT_ROWS)
    s.configure(fdw.FDW_CFG_TIMING, 0)
    s._check(fdw.lib().fdw_get_state(s.ctx, 0, fdw._ptr(snap), None, None))
    final = snap.cpu().numpy()
    s.close()
    return dict(sec=dt, updates=updates, ups=updates / dt, drift=drift, kernel_ms=ms, launches=launches, K=K, S=S,
                n=n, nsteps=nsteps, final=final)


def gpu_state_after(fdw, I, case, dtype, k):
    """Field u^k of `case` computed on the GPU in storage `dtype` (host FP64 array)."""
    import numpy as np

    s = fdw.solver_for_case(case, dtype=dtype)
    s.step(k)
    u = s.get_state()[0].cpu().numpy().astype(np.float64)
    s.close()
    return u


def rel_err(a, ref):
    import numpy as np

    return float(np.abs(a - ref).max() / np.abs(ref).max())


def copy_bench(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second) of torch's copy of a
    1 GiB buffer: the practical ceiling a streaming kernel is compared with."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2.0 * nbytes / dt / 1e9


def small_bench(fdw, torch, I, steps, persistent=False, tiles=0):
    """The 256^2 FP64 line workload (1000 steps + energy): cache-resident and latency-bound,
    reported as microseconds per step with the launch sequence replayed from a graph (one
    launch per time block - the small-grid tile kernel by default, the streaming kernel with
    tiles = 1 - or one persistent launch with grid barriers)."""
    case = I.line_case(n=256, nsteps=1000)
    s = fdw.solver_for_case(case, dtype=fdw.FDW_F64)
    s.configure(fdw.FDW_CFG_USE_GRAPH, 1)
    s.configure(fdw.FDW_CFG_SMALL_TILES, tiles)
    if persistent:
        s.configure(fdw.FDW_CFG_BATCH_MODE, 1)
    h = torch.as_tensor(case.h1, device="cuda")
    e = torch.empty((1, case.nsteps), dtype=torch.float64, device="cuda")

    def one():
        s.reset()
        s.step_into(case.nsteps, e)

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(steps, 5)):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 5)
    K = s.config(fdw.FDW_CFG_TIME_BLOCK)
    s.close()
    del h
    return dict(us_per_step=dt / case.nsteps * 1e6, K=K)


def largest_bench(fdw, torch, I, steps, warmup=1, parity=True):
    """The largest single-GPU workload: 16384^2 FP32 bathymetry + delta ridge, 10^4 steps;
    then the FP32 adjoint on its central 4096^2 crop.  With parity: the FP32 field against the
    FP64 oracle after a bounded number of steps, and against the FP64 GPU solve over the
    whole horizon."""
    import numpy as np

    n, nsteps = 16384, 10000
    case = I.bathymetry_case(n=n, nsteps=nsteps)
    s = fdw.solver_for_case(case, dtype=fdw.FDW_F32)
    h = torch.as_tensor(case.h1, dtype=torch.float32, device="cuda")
    updates = (n - 2) * (n - 2) * nsteps
    # the temporal block depth (with lane columns and rows per item) chosen by the autotuner
    t0 = time.perf_counter()
    tuned = s.autotune()
    tune_s = time.perf_counter() - t0

    def one():
        s.set_coeff(h)
        s.step(nsteps)

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, steps)):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(1, steps)
    K = s.config(fdw.FDW_CFG_TIME_BLOCK)
    policy = s.config(fdw.FDW_CFG_STREAM_POLICY)
    # the dominant kernel's average launch (HIP events on the solver's stream) over one more
    # solve, against the algorithmic bytes of a launch (5 words per node)
    s.configure(fdw.FDW_CFG_TIMING, 1)
    s.kernel_time()
    one()
    ms, launches = s.kernel_time()
    s.configure(fdw.FDW_CFG_TIMING, 0)
    launch_ms = ms / max(launches, 1)
    kernel_gbs = 5 * 4 * n * n / (launch_ms * 1e-3) / 1e9
    par = {}
    if parity:
        u32 = s.get_state()[0].cpu().numpy()
        s.close()
        del h
        torch.cuda.empty_cache()
        u64 = gpu_state_after(fdw, I, case, fdw.FDW_F64, nsteps)
        par["fp32_vs_fp64_gpu_full"] = rel_err(u32.astype(np.float64), u64)
        del u32, u64
        torch.cuda.empty_cache()
        import oracle

        k = 100
        t0 = time.perf_counter()
        ref = oracle.forward_case(case, nsteps=k)["u_cur"]
        par["oracle_s"] = round(time.perf_counter() - t0, 2)
        par["vs_oracle_step"] = k
        par["fp32_vs_fp64_oracle"] = rel_err(gpu_state_after(fdw, I, case, fdw.FDW_F32, k), ref)
        del ref
    else:
        s.close()
        del h
    torch.cuda.empty_cache()
    crop = adjoint_crop_bench(fdw, torch, I, case, max(1, steps), warmup, parity=parity)
    return dict(ups=updates / dt, sec=dt, K=K, crop=crop, parity=par, tuned=tuned, tune_s=tune_s, policy=policy,
                launch_ms=launch_ms, kernel_gbs=kernel_gbs)


def family_bench(fdw, torch, I, steps, warmup, persistent=False, energy=False, fp64_smallest=0, tune=False):
    """The 32-member family, 2000 steps each: one launch per time block over all members
    (persistent=False) or one persistent cooperative launch per call (persistent=True), both
    replayed from a hipGraph; optionally with the per-step energy of every member, and with the
    fp64_smallest smallest-eps members stored in FP64 (the rest FP32)."""
    fam = I.family()
    dts = [fdw.FDW_F32] * (len(fam) - fp64_smallest) + [fdw.FDW_F64] * fp64_smallest
    s = fdw.family_solver(fam, dtype=dts)
    s.configure(fdw.FDW_CFG_USE_GRAPH, 1)
    if persistent:
        s.configure(fdw.FDW_CFG_BATCH_MODE, 1)
    tuned = s.autotune() if tune else None
    nsteps = fam[0].nsteps
    updates = sum((c.nx - 2) * (c.ny - 2) * c.nsteps for c in fam)
    bytes_alg = sum(c.nx * c.ny * (8 if d == fdw.FDW_F64 else 4) for c, d in zip(fam, dts)) * 5 * nsteps / \
        s.config(fdw.FDW_CFG_TIME_BLOCK)
    del fam
    e = torch.empty((s.count, nsteps), dtype=torch.float64, device="cuda") if energy else None

    def one():
        for m in range(s.count):
            s.reset(m)
        s.step_into(nsteps, e)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    K = s.config(fdw.FDW_CFG_TIME_BLOCK)
    policy = s.config(fdw.FDW_CFG_STREAM_POLICY)
    drift = None
    if energy:
        E = e.cpu().numpy()
        drift = float(max(abs(E[m] - E[m][0]).max() / E[m][0] for m in range(E.shape[0])))
    s.close()
    return dict(sec=dt, updates=updates, ups=updates / dt, members=32, K=K, alg_GBs=bytes_alg / dt / 1e9,
                energy_drift=drift, tuned=tuned, policy=policy)


def adjoint_bench(fdw, torch, I, steps, warmup):
    """2048^2 FP64 receiver-misfit gradient: observed traces under h_true, then the misfit and
    its adjoint at h = h_eps."""
    case, h_true = I.adjoint_case()
    N = case.nsteps
    rec = torch.as_tensor(case.receivers)
    s = fdw.solver_for_case(case, dtype=fdw.FDW_F64)
    s.set_coeff(torch.as_tensor(h_true, device="cuda"))
    tr = s.record_traces(rec)
    s.step(N)
    d = tr.clone()
    s.record_traces(None)
    s.set_coeff(torch.as_tensor(case.h1, device="cuda"))
    tr = s.record_traces(rec)
    s.step(N)
    J, tg = s.misfit(tr, d)
    s.record_traces(None)
    out = _time_gradient(fdw, torch, s, case, rec, tg, steps, warmup)
    s.close()
    return out


def adjoint_crop_bench(fdw, torch, I, full, steps, warmup, parity=True):
    """FP32 adjoint on the central 4096^2 crop of the 16384^2 bathymetry case, 4000 steps, 64
    receivers, with a seeded trace gradient as the adjoint source.  With parity: the FP32
    gradient against the FP64 gradient of the same crop and source, computed on the GPU."""
    import numpy as np

    case = I.bathymetry_crop_case(full)
    N = case.nsteps
    rec = torch.as_tensor(case.receivers)
    s = fdw.solver_for_case(case, dtype=fdw.FDW_F32)
    tg = torch.as_tensor(np.random.default_rng(5004).normal(size=(N + 1, rec.shape[0])), device="cuda")
    out = _time_gradient(fdw, torch, s, case, rec, tg, steps, warmup, tune=True)
    s.close()
    if parity:
        g32 = out.pop("grad")
        s64 = fdw.solver_for_case(case, dtype=fdw.FDW_F64)
        g64 = s64.adjoint(rec, tg, ckpt_every=64).cpu().numpy()
        s64.close()
        out["fp32_grad_vs_fp64_gpu"] = rel_err(g32, g64)
        out["fp32_grad_vs_fp64_gpu_l2"] = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    out.pop("grad", None)
    return out


def _time_gradient(fdw, torch, s, case, rec, tg, steps, warmup, tune=False):
    """Forward solve, adjoint with its own replay, forward solve recording traces and
    checkpoints (every 64 steps), adjoint from those checkpoints.  tune: first autotune the
    reverse sweep on a recorded forward run (not timed)."""
    N = case.nsteps
    tuned = None
    if tune:
        s.reset()
        s.record_checkpoints(64)
        s.step(N)
        tuned = s.autotune_adjoint(rec, tg, ckpt_every=64)
        s.record_checkpoints(None)
        s.reset()
    nb = fdw.lib().fdw_adjoint_workspace_bytes(s.ctx, 0, 64)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    g = torch.empty((case.ny, case.nx), dtype=torch.float64, device="cuda")
    recd = rec.to(device="cuda", dtype=torch.int32).contiguous()

    def fwd():
        s.reset()
        s.step(N)

    def adj():
        s._check(fdw.lib().fdw_adjoint(s.ctx, 0, fdw._ptr(recd), recd.shape[0], fdw._ptr(tg), 64, fdw._ptr(ws), nb,
                                       fdw._ptr(g), None))

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # checkpoints stored by the forward run itself: the adjoint then skips its replay
    ws2 = torch.empty(nb, dtype=torch.uint8, device="cuda")

    def fwd_rec():
        s.reset()
        s._check(fdw.lib().fdw_record_checkpoints(s.ctx, 0, 64, fdw._ptr(ws2), nb))
        s.step(N)

    def adj_rec():
        s._check(fdw.lib().fdw_adjoint(s.ctx, 0, fdw._ptr(recd), recd.shape[0], fdw._ptr(tg), 64, fdw._ptr(ws2), nb,
                                       fdw._ptr(g), None))

    tf = timed(fwd)
    ta = timed(adj)
    # the forward run of a gradient evaluation records the receiver traces as well
    s.record_traces(rec)
    tfr = timed(fwd_rec)
    s.record_traces(None)
    tar = timed(adj_rec)
    return dict(forward_s=tf, adjoint_s=ta, ratio=ta / tf, forward_recording_s=tfr, adjoint_recorded_s=tar,
                ratio_recorded=tar / tf, gradient_ratio=(tfr + tar) / tf, n=case.nx, nsteps=N,
                grad_max=float(g.abs().max()), grad=g.cpu().numpy(), adj_tuned=tuned)


# The paper's GPU timings (Section 4, Table 1): cyclic-reduction implicit solver, 100 steps of the
# Section 3.3 problem (dt = 0.05, T = 5) on N x N grids; serial CPU (i7-9800X) and RTX 2080 Ti
# seconds as printed.
TABLE1 = {256: (0.91, 0.88), 512: (3.73, 2.07), 1024: (15.92, 7.16), 2048: (64.8, 20.30), 4096: (280.54, 62.76)}


def table1_bench(fdw, torch, I, steps, oracle_budget_s=2.0):
    """Table 1's workload on this GPU: the implicit solver (factorized scheme, cyclic-reduction line
    solves) for the 100 steps of the table, FP64 and FP32, beside the FP64 oracle of the same scheme
    on the host cores (all 100 steps where that takes under oracle_budget_s, else the first k steps
    with the time scaled linearly to 100, stated per row) and the explicit leapfrog solver run to the
    same T = 5 at CFL 0.5."""
    import oracle

    rows = []
    for n in sorted(TABLE1):
        case = I.paper_table1_case(n)
        N = case.nsteps
        row = {"n": n, "steps": N, "paper_cpu_s": TABLE1[n][0], "paper_gpu_s": TABLE1[n][1]}
        for dt, name in ((fdw.FDW_F64, "f64"), (fdw.FDW_F32, "f32")):
            s = fdw.implicit_solver_for_case(case, sigma=0.25, dtype=dt)
            s.step(N)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(max(1, steps)):
                s.reset()
                s.step(N)
            torch.cuda.synchronize()
            row[f"gpu_{name}_s"] = (time.perf_counter() - t0) / max(1, steps)
            s.close()
        # explicit leapfrog to the same T at CFL 0.5 (FP32)
        dx = 100.0 / (n - 1)
        tau0 = 0.5 * dx / math.sqrt(float(case.h1.max()))
        Ne = int(math.ceil(5.0 / tau0))
        lf = I.Case(**{**case.__dict__, "tau": 5.0 / Ne, "nsteps": Ne})
        s = fdw.solver_for_case(lf, dtype=fdw.FDW_F32)
        s.step(Ne)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.reset()
        s.step(Ne)
        torch.cuda.synchronize()
        row["leapfrog_f32_s"] = time.perf_counter() - t0
        row["leapfrog_steps"] = Ne
        s.close()
        # the oracle of the implicit scheme (FP64, all host threads)
        t0 = time.perf_counter()
        oracle.adi_forward_case(case, nsteps=2)
        t2 = time.perf_counter() - t0
        k = N if t2 * N / 2 <= oracle_budget_s else max(2, int(oracle_budget_s / (t2 / 2)))
        t0 = time.perf_counter()
        oracle.adi_forward_case(case, nsteps=k)
        to = (time.perf_counter() - t0) * N / k
        row["oracle_s"] = to
        row["oracle_steps_run"] = k
        row["speedup_f64_vs_oracle"] = to / row["gpu_f64_s"]
        row["speedup_f64_vs_paper_gpu"] = TABLE1[n][1] / row["gpu_f64_s"]
        row["gpu_f64_updates_per_s"] = (n - 2) ** 2 * N / row["gpu_f64_s"]
        rows.append({k2: (round(v, 6) if isinstance(v, float) else v) for k2, v in row.items()})
        log(json.dumps(rows[-1]))
        torch.cuda.empty_cache()
    return rows


def cpu_baseline(I, budget_s=15.0):
    """The FP64 oracle on the host cores: first k steps of the same 8192^2 workload, k chosen
    from two calibration runs (3 and 13 steps; their difference removes the per-call set-up)
    so that the timed run takes about budget_s seconds.  Also returns the oracle's u^k, which
    the GPU states at the same step are compared with."""
    import oracle

    n = 8192
    case = I.point_case(n=n, nsteps=5000)
    oracle.forward_case(case, nsteps=2)  # warm-up (page faults, thread start)
    t0 = time.perf_counter()
    oracle.forward_case(case, nsteps=3)
    t3 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.forward_case(case, nsteps=13)
    t13 = time.perf_counter() - t0
    per_step = max((t13 - t3) / 10.0, 1e-3)
    setup = max(t3 - 3 * per_step, 0.0)
    k = max(4, int((budget_s - setup) / per_step))
    t0 = time.perf_counter()
    ref = oracle.forward_case(case, nsteps=k)
    dt = time.perf_counter() - t0
    ups = (n - 2) * (n - 2) * k / dt
    out = dict(value=ups, unit="grid-point updates/s", cores=oracle.threads(), kind="oracle",
               sample=f"FP64 oracle (OpenMP), 8192x8192 point-singularity workload, first {k} of 5000 steps "
                      f"including input copies ({dt:.1f} s wall)", host=host_info())
    return out, case, k, ref["u_cur"]


def host_info():
    """CPU model, logical CPUs usable by this process and host RAM, from /proc."""
    model, mem = "unknown", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return dict(cpu_model=model, cpus=len(os.sched_getaffinity(0)), ram_GiB=round(mem / 2**30, 1))


def oracle_single_thread_rate(I, n=2048, steps=20):
    """The FP64 oracle on one host thread (OMP_NUM_THREADS=1 in a child process), a short
    sample of a 2048^2 line workload: grid-point updates/s."""
    import subprocess

    code = ("import sys, time; sys.path.insert(0, %r); import oracle; from paper_2005_11931_amd import inputs as I; "
            "c = I.line_case(n=%d, nsteps=%d); oracle.forward_case(c, nsteps=2); t = time.perf_counter(); "
            "oracle.forward_case(c); print((%d - 2) ** 2 * %d / (time.perf_counter() - t))") % (ROOT, n, steps, n, steps)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    try:
        return float(r.stdout.strip().splitlines()[-1])
    except (ValueError, IndexError):
        return None


def profile_run(dtype_name: str, workload: str = "point8192"):
    """Short, profiler-friendly run: three 800-step forward solves of the 8192^2 workload with
    per-step energy (the configuration the bench times; workload bathymetry16384: three 400-step
    solves of the 16384^2 case in its autotuned configuration, no energy), then three state
    read-outs: each is a plain copy kernel (k_copy_out) that reads and writes exactly n*n words,
    used to calibrate the memory counters."""
    import torch

    from paper_2005_11931_amd import fdw
    from paper_2005_11931_amd import inputs as I

    dtype = fdw.FDW_F32 if dtype_name == "f32" else fdw.FDW_F64
    big = workload == "bathymetry16384"
    case = I.bathymetry_case(n=16384, nsteps=10000) if big else I.point_case(n=8192, nsteps=5000)
    s = fdw.solver_for_case(case, dtype=dtype)
    del case
    if big:
        # the autotuner's choice on this workload (bench line)
        s.configure(fdw.FDW_CFG_TIME_BLOCK, 8)
        s.configure(fdw.FDW_CFG_SEGMENT_ROWS, 48)
        s.configure(fdw.FDW_CFG_STREAM_POLICY, 3)
    for _ in range(3):  # three solves: the average is over ~150-300 launches, warm-up included
        s.reset()
        s.step(400 if big else 800, energy=not big)
    torch.cuda.synchronize()
    for _ in range(3):
        s.get_state()
    torch.cuda.synchronize()
    log("profile run done:", dtype_name, "K", s.config(fdw.FDW_CFG_TIME_BLOCK), "C",
        s.config(fdw.FDW_CFG_LANE_COLUMNS), "S", s.config(fdw.FDW_CFG_SEGMENT_ROWS))
    s.close()


def profile_run_family():
    """Short run of the 32-member family for rocprofv3: 400 steps with energies, once with one
    launch per time block, once with the persistent launch."""
    import torch

    from paper_2005_11931_amd import fdw
    from paper_2005_11931_amd import inputs as I

    fam = I.family()
    for persistent in (0, 1):
        s = fdw.family_solver(fam, dtype=fdw.FDW_F32)
        s.configure(fdw.FDW_CFG_BATCH_MODE, persistent)
        s.step(400, energy=True)
        torch.cuda.synchronize()
        s.close()
    log("family profile run done")


def profile_run_implicit():
    """Short run of the implicit solver for rocprofv3: the Table 1 workload at 4096^2, 20 steps in
    FP64 and in FP32."""
    import torch

    from paper_2005_11931_amd import fdw
    from paper_2005_11931_amd import inputs as I

    case = I.paper_table1_case(4096)
    for dt in (fdw.FDW_F64, fdw.FDW_F32):
        s = fdw.implicit_solver_for_case(case, sigma=0.25, dtype=dt)
        s.step(20)
        torch.cuda.synchronize()
        s.close()
    log("implicit profile run done")


def profile_run_small():
    """Short run of the 256^2 FP64 line workload for rocprofv3: three 1000-step solves with
    per-step energy, replayed from a hipGraph, on the small-grid tile kernel and then on the
    streaming kernel."""
    import torch

    from paper_2005_11931_amd import fdw
    from paper_2005_11931_amd import inputs as I

    case = I.line_case(n=256, nsteps=1000)
    for tiles in (2, 1):
        s = fdw.solver_for_case(case, dtype=fdw.FDW_F64)
        s.configure(fdw.FDW_CFG_USE_GRAPH, 1)
        s.configure(fdw.FDW_CFG_SMALL_TILES, tiles)
        e = torch.empty((1, case.nsteps), dtype=torch.float64, device="cuda")
        for _ in range(3):
            s.reset()
            s.step_into(case.nsteps, e)
        torch.cuda.synchronize()
        s.close()
    log("profile run done: small")


def profile_run_adjoint():
    """Short, profiler-friendly run of the reverse sweep: the 2048^2 FP64 receiver-misfit
    workload cut to 512 steps (checkpoints every 64), one forward solve recording traces and
    checkpoints, then one adjoint from them."""
    import torch

    from paper_2005_11931_amd import fdw
    from paper_2005_11931_amd import inputs as I

    case, _ = I.adjoint_case(nsteps=512)
    s = fdw.solver_for_case(case, dtype=fdw.FDW_F64)
    rec = torch.as_tensor(case.receivers)
    s.record_checkpoints(64)
    tr = s.record_traces(rec)
    s.step(case.nsteps)
    J, tg = s.misfit(tr, torch.zeros_like(tr))
    g = s.adjoint(rec, tg, ckpt_every=64)
    torch.cuda.synchronize()
    log("adjoint profile run done: K", s.config(fdw.FDW_CFG_ADJ_TIME_BLOCK), "C",
        s.config(fdw.FDW_CFG_ADJ_LANE_COLUMNS), "|g|", float(g.abs().max()))
    s.close()


def summarize_profile(dirs, name: str, command: str, dtype_name: str = "f32", factors=None, n: int = 8192):
    """Collects kernel statistics and FETCH_SIZE / WRITE_SIZE counter rows from rocprofv3 CSV
    output under `dirs` into profiles/<name>.txt.  When both counters were taken for the
    streaming kernel and for the calibration copy (k_copy_out: n*n words read and written per
    dispatch), the calibrated HBM bytes per streaming launch go to profiles/<name>.json."""
    import csv
    import glob

    lines = [f"# {name}", f"command: {command}", ""]
    summary = {}
    for d in dirs:
        for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
            rows = list(csv.DictReader(open(f)))
            lines.append(f"kernel stats ({os.path.basename(d)}):")
            lines.append("name | calls | total_ns | avg_ns | pct")
            for r in rows[:12]:
                lines.append(f"{r.get('Name', '')[:110]} | {r.get('Calls', '')} | {r.get('TotalDurationNs', '')} | "
                             f"{r.get('AverageNs', '')} | {r.get('Percentage', '')}")
            lines.append("")
        for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            for r in csv.DictReader(open(f)):
                kname = r.get("Kernel_Name", "")
                cname = r.get("Counter_Name", "")
                try:
                    val = float(r.get("Counter_Value", "nan"))
                except ValueError:
                    continue
                key = "copy" if "k_copy_out" in kname else ("k_step" if "k_step" in kname else
                                                             ("k_adjoint" if "k_adjoint<" in kname else None))
                if key is None:
                    continue
                summary.setdefault((key, cname), []).append(val)
    if summary:
        lines.append("counters (KiB per dispatch, mean over dispatches):")
        for (k, c), v in sorted(summary.items()):
            lines.append(f"{k} {c} mean {sum(v) / len(v):.1f} over {len(v)} dispatches")
    if factors and ("k_adjoint", "FETCH_SIZE") in summary and ("k_adjoint", "WRITE_SIZE") in summary:
        # reverse sweep of the 2048^2 FP64 workload; counters scaled by the copy calibration
        f_fetch, f_write = factors
        rd = sum(summary[("k_adjoint", "FETCH_SIZE")]) / len(summary[("k_adjoint", "FETCH_SIZE")]) * f_fetch * 1024
        wr = sum(summary[("k_adjoint", "WRITE_SIZE")]) / len(summary[("k_adjoint", "WRITE_SIZE")]) * f_write * 1024
        n = 2048
        lines += ["", f"reverse kernel (calibration factors fetch {f_fetch:.4f}, write {f_write:.4f} from the copy "
                      f"of the forward profile run): {rd / 1e6:.1f} MB read + {wr / 1e6:.1f} MB written per launch "
                      f"(algorithmic {6 * 8 * n * n / 1e6:.1f} MB read: u, du, lam, mu, h, g; "
                      f"{5 * 8 * n * n / 1e6:.1f} MB written)"]
    need = [("copy", "FETCH_SIZE"), ("copy", "WRITE_SIZE"), ("k_step", "FETCH_SIZE"), ("k_step", "WRITE_SIZE")]
    if all(k in summary for k in need):
        mean = {k: sum(summary[k]) / len(summary[k]) for k in need}
        es = 4 if dtype_name == "f32" else 8
        copy_kib = n * n * es / 1024.0
        f_fetch = copy_kib / mean[("copy", "FETCH_SIZE")]
        f_write = copy_kib / mean[("copy", "WRITE_SIZE")]
        read_b = mean[("k_step", "FETCH_SIZE")] * f_fetch * 1024.0
        write_b = mean[("k_step", "WRITE_SIZE")] * f_write * 1024.0
        alg = 5 * es * n * n
        lines += ["", f"calibration: copy of {n}x{n} words reads and writes {copy_kib:.0f} KiB; "
                      f"factors fetch {f_fetch:.4f}, write {f_write:.4f}",
                  f"streaming kernel: {read_b / 1e6:.1f} MB read + {write_b / 1e6:.1f} MB written per launch "
                  f"(algorithmic {alg / 1e6:.1f} MB: 3 words read, 2 written per node)"]
        js = {"kernel_source_hash": kernel_source_hash(), "bytes_per_launch": round(read_b + write_b),
              "read_bytes": round(read_b), "write_bytes": round(write_b), "algorithmic_bytes": alg,
              "fetch_factor": f_fetch, "write_factor": f_write, "command": command}
        with open(os.path.join(ROOT, "profiles", name + ".json"), "w") as fh:
            json.dump(js, fh, indent=1)
    out = os.path.join(ROOT, "profiles", name + ".txt")
    open(out, "w").write("\n".join(lines) + "\n")
    print(out)


def main():
    if "--summarize-profile" in sys.argv:
        ap = argparse.ArgumentParser()
        ap.add_argument("--summarize-profile", required=True, nargs="+")
        ap.add_argument("--out", required=True)
        ap.add_argument("--command", default="")
        ap.add_argument("--dtype", default="f32")
        ap.add_argument("--factors", nargs=2, type=float, default=None)
        ap.add_argument("--n", type=int, default=8192)
        a = ap.parse_args()
        summarize_profile(a.summarize_profile, a.out, a.command, a.dtype, a.factors, a.n)
        return
    if "--profile-run" in sys.argv:
        ap = argparse.ArgumentParser()
        ap.add_argument("--profile-run", action="store_true")
        ap.add_argument("--dtype", default="f32")
        ap.add_argument("--adjoint", action="store_true")
        ap.add_argument("--workload", default="point8192",
                        choices=["point8192", "bathymetry16384", "family", "implicit4096", "line256"])
        a = ap.parse_args()
        if a.adjoint:
            profile_run_adjoint()
        elif a.workload == "family":
            profile_run_family()
        elif a.workload == "implicit4096":
            profile_run_implicit()
        elif a.workload == "line256":
            profile_run_small()
        else:
            profile_run(a.dtype, a.workload)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--skip-extra", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2005_11931_amd import fdw
    from paper_2005_11931_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("forward fp32 8192^2 x 5000")
    f32 = forward_bench(fdw, torch, I, fdw.FDW_F32, args.steps, args.warmup)
    f32_final = f32.pop("final")
    log(json.dumps(f32))
    nodes = f32["n"] * f32["n"]
    K = f32["K"]
    copy_GBs = copy_bench(torch)
    log("device-to-device copy", round(copy_GBs, 1), "GB/s")
    per_launch_bytes = 5 * 4 * nodes  # read u, du, h; write u, du (FP32 words) per streaming launch
    avg_launch_s = f32["kernel_ms"] / 1e3 / max(f32["launches"], 1)
    achieved = per_launch_bytes / avg_launch_s / 1e9
    traffic = load_traffic("k_step_f32_point8192.json", nodes)
    roof = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": f"k_step<float,K={K},nodal>",
        "avg_launch_ms": round(avg_launch_s * 1e3, 4),
        "launches": f32["launches"],
        "bytes_per_launch": per_launch_bytes,
        "effective_vs_single_step_roofline": round(f32["ups"] / (HBM_PEAK_GBS * 1e9 / 20.0), 3),
        "d2d_copy_GBs": round(copy_GBs, 1),
    }
    if traffic:
        roof["traffic_GBs"] = round(traffic / avg_launch_s / 1e9, 1)
        roof["traffic_vs_copy"] = round(traffic / avg_launch_s / 1e9 / copy_GBs, 4)
    out = {
        "metric": METRIC,
        "value": round(f32["ups"], 1),
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["sec"] * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "8192x8192 point singularity h = 1 + 5 phi_eps(r), eps = 4 dx, 4 seeded humps, "
                        "5000 leapfrog steps at CFL 0.5 with per-step energy, FP32 storage",
            "grid": [8192, 8192],
            "nsteps": 5000,
            "time_block": K,
            "segment_rows": f32["S"],
            "energy_drift": f32["drift"],
        },
        "roofline": roof,
        "parity": {"point8192": {}},
    }
    if not args.skip_extra:
        log("forward fp64 8192^2 x 5000")
        f64 = forward_bench(fdw, torch, I, fdw.FDW_F64, max(1, args.steps - 1), args.warmup)
        f64_final = f64.pop("final")
        log(json.dumps(f64))
        # the whole 5000-step horizon: FP32 against the FP64 GPU solve (the oracle covers the
        # first k steps, see cpu_baseline)
        out["parity"]["point8192"]["fp32_vs_fp64_gpu_full"] = rel_err(f32_final.astype(np.float64), f64_final)
        del f64_final
        a64 = 5 * 8 * nodes / (f64["kernel_ms"] / 1e3 / max(f64["launches"], 1)) / 1e9
        out["fp64"] = {"value": round(f64["ups"], 1), "unit": "grid-point updates/s", "ms_per_step": round(
            f64["sec"] * 1e3, 2), "time_block": f64["K"], "kernel_GBs": round(a64, 1),
            "frac": round(a64 / HBM_PEAK_GBS, 4), "energy_drift": f64["drift"]}
        torch.cuda.empty_cache()
        log("batched family")
        fam = family_bench(fdw, torch, I, max(1, args.steps - 1), args.warmup, tune=True)
        log(json.dumps(fam))
        fame = family_bench(fdw, torch, I, max(1, args.steps - 1), args.warmup, energy=True)
        log(json.dumps(fame))
        famp = family_bench(fdw, torch, I, max(1, args.steps - 1), args.warmup, persistent=True, energy=True)
        log(json.dumps(famp))
        famx = family_bench(fdw, torch, I, max(1, args.steps - 1), args.warmup, energy=True, fp64_smallest=4)
        log(json.dumps(famx))
        out["batched"] = {"value": round(fam["ups"], 1), "unit": "grid-point updates/s", "members": 32,
                          "ms_per_step": round(fam["sec"] * 1e3, 2), "time_block": fam["K"],
                          "autotuned_time_block_segment_rows_lane_columns": fam["tuned"],
                          "autotuned_stream_policy": fam["policy"],
                          "alg_GBs": round(fam["alg_GBs"], 1), "frac": round(fam["alg_GBs"] / HBM_PEAK_GBS, 4),
                          "energy_value": round(fame["ups"], 1),
                          "energy_frac": round(fame["alg_GBs"] / HBM_PEAK_GBS, 4),
                          "persistent_energy_value": round(famp["ups"], 1),
                          "persistent_energy_frac": round(famp["alg_GBs"] / HBM_PEAK_GBS, 4),
                          "persistent_energy_ms_per_step": round(famp["sec"] * 1e3, 2),
                          "energy_drift_max": famp["energy_drift"],
                          "mixed_fp64_smallest4_energy_value": round(famx["ups"], 1),
                          "mixed_fp64_smallest4_energy_ms_per_step": round(famx["sec"] * 1e3, 2),
                          "workload": "32 regularisations, eps log-spaced 0.1 .. 2dx, delta line / Heaviside jump, "
                                      "512^2-4096^2, 2000 steps, FP32; value: one launch per time block covering "
                                      "all members, replayed from a hipGraph, autotuned; energy_value: the default "
                                      "configuration with the per-step energy of every member; persistent_energy_value: one cooperative "
                                      "launch per call (grid barrier between time blocks, energies summed in the "
                                      "launch), replayed from a hipGraph; mixed_fp64_smallest4: the four smallest-eps "
                                      "members (4096^2 .. 512^2) stored in FP64, the rest FP32, one launch sequence "
                                      "per storage type, with energies"}
        torch.cuda.empty_cache()
        log("adjoint 2048^2 fp64 x 4000")
        adj = adjoint_bench(fdw, torch, I, max(1, args.steps - 1), args.warmup)
        adj.pop("grad", None)
        log(json.dumps(adj))
        out["adjoint"] = {"ratio": round(adj["ratio"], 3), "forward_ms": round(adj["forward_s"] * 1e3, 2),
                          "adjoint_ms": round(adj["adjoint_s"] * 1e3, 2),
                          "ratio_recorded": round(adj["ratio_recorded"], 3),
                          "forward_recording_ms": round(adj["forward_recording_s"] * 1e3, 2),
                          "adjoint_recorded_ms": round(adj["adjoint_recorded_s"] * 1e3, 2),
                          "gradient_ratio": round(adj["gradient_ratio"], 3),
                          "workload": "2048x2048 FP64 receiver-misfit gradient, 4000 steps, 64 receivers, "
                                      "checkpoints every 64 steps; ratio: adjoint call with its own forward replay "
                                      "/ forward solve; ratio_recorded: adjoint call from checkpoints stored by the "
                                      "forward solve / forward solve; gradient_ratio: (forward solve recording the "
                                      "receiver traces and storing checkpoints + adjoint from them) / forward "
                                      "solve"}
    if not args.skip_extra:
        torch.cuda.empty_cache()
        log("small 256^2 fp64 line")
        sm = small_bench(fdw, torch, I, args.steps)
        sms = small_bench(fdw, torch, I, args.steps, tiles=1)
        smp = small_bench(fdw, torch, I, args.steps, persistent=True)
        out["small"] = {"us_per_step": round(sm["us_per_step"], 3), "time_block": sm["K"],
                        "streaming_kernel_us_per_step": round(sms["us_per_step"], 3),
                        "persistent_us_per_step": round(smp["us_per_step"], 3),
                        "workload": "256x256 FP64 line singularity h = 1 + 2 phi_0.05(x), 1000 steps with per-step "
                                    "energy, launch sequence replayed from a hipGraph (cache-resident)"}
        log("largest 16384^2 fp32")
        lg = largest_bench(fdw, torch, I, max(1, args.steps - 2), args.warmup)
        cr = lg["crop"]
        log(json.dumps(cr))
        out["parity"]["bathymetry16384"] = lg["parity"]
        out["largest"] = {"value": round(lg["ups"], 1), "unit": "grid-point updates/s",
                          "ms_per_step": round(lg["sec"] * 1e3, 2), "time_block": lg["K"],
                          "autotuned_time_block_segment_rows_lane_columns": lg["tuned"],
                          "autotuned_stream_policy": lg["policy"],
                          "autotune_s": round(lg["tune_s"], 2),
                          "avg_launch_ms": round(lg["launch_ms"], 4),
                          "kernel_GBs": round(lg["kernel_gbs"], 1),
                          "frac": round(lg["kernel_gbs"] / 8000.0, 4),
                          "workload": "16384x16384 FP32 smooth random bathymetry 0.2-1 + delta ridge eps = 2 dx, "
                                      "10000 steps, no energy, launch configuration (time block, rows per item, "
                                      "lane columns, stream policy) from the autotuner; frac: algorithmic bytes "
                                      "(5 words per node) per launch / average launch time / 8 TB/s",
                          "adjoint_crop": {"forward_ms": round(cr["forward_s"] * 1e3, 2),
                                           "adjoint_ms": round(cr["adjoint_s"] * 1e3, 2),
                                           "ratio": round(cr["ratio"], 3),
                                           "forward_recording_ms": round(cr["forward_recording_s"] * 1e3, 2),
                                           "adjoint_recorded_ms": round(cr["adjoint_recorded_s"] * 1e3, 2),
                                           "ratio_recorded": round(cr["ratio_recorded"], 3),
                                           "gradient_ratio": round(cr["gradient_ratio"], 3),
                                           "adj_autotuned_time_block_segment_rows_lane_columns": cr.get("adj_tuned"),
                                           "fp32_grad_vs_fp64_gpu": cr.get("fp32_grad_vs_fp64_gpu"),
                                           "fp32_grad_vs_fp64_gpu_l2": cr.get("fp32_grad_vs_fp64_gpu_l2"),
                                           "workload": "central 4096x4096 crop of the same case (zero Dirichlet "
                                                       "edge), FP32 state, FP64 gradient, 4000 steps, 64 "
                                                       "receivers on the row nearest y = 0.075, seeded trace "
                                                       "gradient, checkpoints every 64 steps"}}
        torch.cuda.empty_cache()
    if not args.skip_extra:
        log("table 1 workload: implicit solver")
        out["table1_implicit"] = {
            "rows": table1_bench(fdw, torch, I, min(3, max(1, args.steps - 1))),
            "workload": "Section 4 Table 1: Section 3.3 problem on N x N nodes of [0,100]^2, eps = 0.8, dt = 0.05, "
                        "T = 5 (100 steps); implicit factorized scheme (sigma = 1/4) with cyclic-reduction line "
                        "solves on this GPU (FP64 and FP32); paper_*_s: the paper's serial CPU and RTX 2080 Ti "
                        "times for its cyclic-reduction solver (context, other hardware and code); oracle_s: the "
                        "FP64 oracle of the same scheme on the host cores (Thomas algorithm; linear in the steps "
                        "when truncated); leapfrog_f32_s: the explicit solver to the same T at CFL 0.5"}
    if not args.skip_cpu:
        log("cpu baseline")
        cb, case, k, u_ref = cpu_baseline(I)
        rate1 = oracle_single_thread_rate(I)
        if rate1:
            cb["one_thread_value"] = round(rate1, 1)
            cb["one_thread_sample"] = "FP64 oracle on 1 thread, 2048x2048 line workload, 20 steps"
        out["cpu_baseline"] = cb
        # FP32 and FP64 GPU fields against the FP64 oracle at the oracle's step k
        u32 = gpu_state_after(fdw, I, case, fdw.FDW_F32, k)
        e32 = rel_err(u32, u_ref)
        del u32
        u64 = gpu_state_after(fdw, I, case, fdw.FDW_F64, k)
        e64 = float(np.abs(u64 - u_ref).max())
        del u64, u_ref, case
        out["parity"]["point8192"].update({"vs_oracle_step": k, "fp32_vs_fp64_oracle": e32,
                                           "fp64_vs_oracle_maxabs": e64})
        log("parity at step", k, "fp32 rel", e32, "fp64 max-abs", e64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
