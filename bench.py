#!/usr/bin/env python3
"""Benchmark of the PFC hot path on one MI355X.

Workload: 3D one-mode PFC on a 512^3 periodic grid in FP32 (dx = pi/4, r = -0.30, dt = 0.5,
psi0 = -0.30 + U(-0.1, 0.1) from SplitMix64 seed 23), the configuration the headline metric is
quoted on.  One step = x r2c (cube prologue) -> y forward -> z forward + semi-implicit update + z
inverse -> y inverse -> x c2r (1/N epilogue), five kernels through the C ABI; between the steps of
one call the x c2r and the next step's x r2c run as one fused kernel (the field in between is not
stored), so a call of K steps moves 10 K + 2 field-sized passes instead of 12 K.

Prints ONE JSON line on stdout: steps/s of the whole step (inputs resident in HBM), the roofline
of the dominant kernel (algorithmic bytes / its average duration, from HIP events on the stream
the kernels run on), the 3D r2c / c2r GB/s, and the FP64 CPU oracle timed on this host.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PFC steps/s at 512^3 FP32 + 3D r2c/c2r FFT HBM GB/s (% of peak)"
PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E
N = 512
R, DT, SEED = -0.30, 0.5, 23
PASS_NAMES = ["x_r2c_cube", "y_fwd", "z_fused_update", "y_inv", "x_c2r"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_512cube_f32.txt")
KERNEL_SOURCES = ["fft_core.hpp", "kernels.hpp", "dispatch_impl.hpp", "types.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_26818_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None when
    the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel].get("hbm_bytes_per_launch")


def bench_batched(nsteps):
    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    insts = pfc_inputs.batch_workload()
    psis = [pfc_inputs.pfc_initial_field_torch(pfc_inputs.derive_seed(4, 1000 + i), d["shape"], d["r"],
                                               torch.float32, "cuda:0") for i, d in enumerate(insts)]
    b = pfc.Batch(insts).bind(psis)
    b.state_init()
    variants, tuned_ms = b.autotune(steps=5)  # radix schedules (and item shapes) per pass and length
    b.step(nsteps)  # captures the graph for this nsteps and warms up
    b.check()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(nsteps)
    e1.record(stream)
    b.check()
    ms = e0.elapsed_time(e1)
    pts = sum(d["shape"][0] * d["shape"][1] for d in insts)
    # the same 48 runs as separate single-plan launches (3 kernels per instance per step), for reference
    plans = [pfc.Plan(d["shape"], dtype="f32", model=d["model"], r=d["r"], dt=d["dt"], q1sq=d["q1sq"], R1=d["R1"])
             for d in insts]
    states = [p.state_init(x) for p, x in zip(plans, psis)]
    ref_steps = min(nsteps, 100)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(ref_steps):
        for p, x, st in zip(plans, psis, states):
            p.step(x, st, 1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sep = e0.elapsed_time(e1) / ref_steps
    return {"workload": "48 2D runs {128^2,256^2,512^2,1024^2}x12, one-/two-mode, FP32, dt=0.25", "steps": nsteps,
            "ms": round(ms, 3), "batch_steps_per_s": round(1000.0 * nsteps / ms, 1),
            "points_per_step": pts, "alg_gbps": round(32.0 * pts * nsteps / ms / 1e6, 1),
            "grid_workgroups": b.grid, "autotuned_variants_by_size": {
                f"{d['shape'][0]}^2": v for d, v in zip(insts, variants)},
            "separate_launches_ms_per_step": round(ms_sep, 4),
            "separate_launches_steps_per_s": round(1000.0 / ms_sep, 1)}


def bench_hydro(nsteps, n=512, seed=9):
    """Hydrodynamic PFC (density + 3 velocity components) at n^3 FP32, rho0 = gamma = a0 = 1,
    r = -0.30, dt = 0.25: ms per step and algorithmic GB/s on the 480 B/point pass model (120 reads
    or writes of 4 B per point, a packed spectrum or a real field: 16 transforms, the 6 derivatives
    applied inside the last-axis inverse passes, 5 pointwise updates)."""
    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    shape = (n, n, n)
    plan = pfc.Plan(shape, dtype="f32", r=R, dt=0.25)
    psi = pfc_inputs.pfc_initial_field_torch(seed, shape, R, torch.float32, "cuda:0")
    v = torch.stack([pfc_inputs.uniform_torch(seed * 10 + j, shape, -0.05, 0.05, torch.float32, "cuda:0")
                     for j in range(3)])
    S, V = plan.hydro_state_init(psi, v)
    work = torch.empty(int(plan._lib.pfc_hydro_work_bytes(plan._h)), dtype=torch.uint8, device="cuda:0")
    plan.hydro_step(psi, S, v, V, 1, work=work)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan.hydro_step(psi, S, v, V, nsteps, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / nsteps
    finite = bool(torch.isfinite(psi).all().item()) and bool(torch.isfinite(v).all().item())
    del psi, v, S, V, work, plan
    torch.cuda.empty_cache()
    alg = 480.0 * n**3
    return {"workload": f"3D hydrodynamic PFC {n}^3 FP32 (psi + 3 velocity components), rho0=gamma=a0=1, r=-0.30, "
                        f"dt=0.25, seed {seed}", "steps": nsteps, "ms_per_step": round(ms, 3),
            "steps_per_s": round(1000.0 / ms, 2), "alg_gbps": round(alg / ms / 1e6, 1),
            "frac": round(alg / ms / 1e6 / PEAK_HBM_GBPS, 4), "fields_finite": finite}


def bench_amplitude(nsteps, shape=(256, 256, 256), lattice="bcc", seed=7):
    """Complex-amplitude form: the amplitudes of a lattice (6 bcc amplitudes on 256^3, or 3
    triangular ones on 2048^2), FP32 (dB = -0.15, Bx = 1, t = 0.3, v = 1, dt = 0.5, dx = pi/2),
    amplitudes 0.1 + U(-0.05, 0.05) (1 + i).  Algorithmic bytes per step: 14 (3D) or 10 (2D) reads or
    writes of the complex fields (nonlinearity, x forward, y forward in 3D, the fused last axis
    twice each way, y inverse in 3D, x inverse)."""
    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    shape, k = tuple(shape), pfc_inputs.lattice_vectors(lattice)
    npts = 1
    for v in shape:
        npts *= v
    obj = pfc.Apfc(shape, k, dtype="f32", dB=-0.15, Bx=1.0, t=0.3, v=1.0, dt=0.5)
    eta = pfc_inputs.amplitude_fields_torch(seed, len(k), shape, 0.1, torch.complex64, "cuda:0", 0.05)
    S = obj.state_init(eta)
    obj.step(eta, S, 2)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    obj.step(eta, S, nsteps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / nsteps
    finite = bool(torch.isfinite(torch.view_as_real(eta)).all().item())
    del eta, S, obj
    torch.cuda.empty_cache()
    alg = (14.0 if len(shape) == 3 else 10.0) * len(k) * npts * 8
    dims = "x".join(str(v) for v in shape)
    return {"workload": f"complex-amplitude PFC, {len(k)} {lattice} amplitudes on {dims}, FP32, dB=-0.15 Bx=1 "
                        f"t=0.3 v=1, dt=0.5, seed {seed}", "steps": nsteps, "ms_per_step": round(ms, 3),
            "steps_per_s": round(1000.0 / ms, 2), "alg_gbps": round(alg / ms / 1e6, 1),
            "frac": round(alg / ms / 1e6 / PEAK_HBM_GBPS, 4), "fields_finite": finite}


def step_passes_hbm(plan, nsteps):
    """Field-sized HBM passes per 3D step of a call of `nsteps` steps: 12 (x r2c, y, z twice, y, x
    c2r), or, where the plan fuses the x passes between steps, 10 per step plus 2 per call (the first
    step's x r2c and the last step's x c2r; pfc_plan_x_fused)."""
    return (10.0 * nsteps + 2.0) / nsteps if plan.x_fused else 12.0


def median_spread(vals):
    v = sorted(vals)
    return v[len(v) // 2], v[0], v[-1]


def bench_big(nsteps, n=2048, seed=3, dtype="f32", reps=1, profile_steps=3):
    """3D one-mode PFC at n^3 (r = -0.30, dt = 0.5, psi0 = -0.30 + U(-0.1, 0.1) from `seed`):
    steps/s (median of `reps` timed runs of nsteps steps, with the spread) and per-pass GB/s on the
    5-pass model (12 field-sized reads or writes per point).  n = 2048: the full single-GPU size;
    750 and 1400: the paper's 3D grids (mixed radix); 256 and 512 in FP64 and FP32."""
    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    shape = (n, n, n)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    plan = pfc.Plan(shape, dtype=dtype, r=R, dt=DT)
    psi = pfc_inputs.pfc_initial_field_torch(seed, shape, R, tdt, "cuda:0")
    state = plan.state_init(psi)
    plan.step(psi, state, 2)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(reps):
        e0.record(stream)
        plan.step(psi, state, nsteps)
        e1.record(stream)
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1) / nsteps)
    ms, ms_lo, ms_hi = median_spread(runs)
    units = step_passes_hbm(plan, nsteps)
    pass_ms = plan.step_timed(psi, state, profile_steps)
    F = plan.energy(psi, state).cpu().tolist()
    Rb = n**3 * (4 if dtype == "f32" else 8)
    alg = [2 * Rb, 2 * Rb, 4 * Rb, 2 * Rb, 2 * Rb]
    passes = [{"kernel": k, "avg_ms": round(t / profile_steps, 4), "alg_bytes": b,
               "alg_gbps": round(b / (t / profile_steps) / 1e6, 1),
               "frac": round(b / (t / profile_steps) / 1e6 / PEAK_HBM_GBPS, 4)}
              for k, t, b in zip(PASS_NAMES, pass_ms, alg)]
    del psi, state, plan
    torch.cuda.empty_cache()
    out = {"workload": f"3D one-mode PFC {n}^3 {dtype.upper()}, r=-0.30, dt=0.5, psi0 seed {seed}", "steps": nsteps,
           "ms_per_step": round(ms, 4), "steps_per_s": round(1000.0 / ms, 2),
           "hbm_passes_per_step": round(units, 4),
           "alg_gbps": round(units * Rb / ms / 1e6, 1), "frac": round(units * Rb / ms / 1e6 / PEAK_HBM_GBPS, 4),
           "passes": passes, "energy_finite": all(math.isfinite(v) for v in F)}
    if reps > 1:
        out["reps"] = reps
        out["steps_per_s_min_max"] = [round(1000.0 / ms_hi, 2), round(1000.0 / ms_lo, 2)]
    return out


def bench_fft(n, dtype, reps, seed):
    """Standalone 3D r2c and c2r on a seeded N(0, 1) field, natural half spectrum: ms per transform
    (average over `reps`) and GB/s on the 3-pass model Rb + 5 Cn (real field once, the half spectrum
    written or read once by the x pass and read and written by each of the y and z passes)."""
    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    shape = (n, n, n)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    s = 4 if dtype == "f32" else 8
    plan = pfc.Plan(shape, dtype=dtype, r=R, dt=DT)
    stream = torch.cuda.current_stream()
    x = pfc_inputs.normal_torch(seed, shape, tdt, "cuda:0")
    X = plan.fft_r2c(x)
    y = plan.fft_c2r(X)
    torch.cuda.synchronize()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_r2c = timed(lambda: plan.fft_r2c(x, X))
    t_c2r = timed(lambda: plan.fft_c2r(X, y))
    rt_err = (torch.linalg.vector_norm((y - x).double()) / torch.linalg.vector_norm(x.double())).item()
    Rb = n**3 * s
    Cn = n * n * (n // 2 + 1) * 2 * s
    fft_bytes = Rb + 5 * Cn
    del x, X, y, plan
    torch.cuda.empty_cache()
    return {"workload": f"3D r2c/c2r {n}^3 {dtype.upper()}, N(0,1) seed {seed}", "r2c_ms": round(t_r2c, 4),
            "c2r_ms": round(t_c2r, 4), "r2c_gbps": round(fft_bytes / t_r2c / 1e6, 1),
            "c2r_gbps": round(fft_bytes / t_c2r / 1e6, 1),
            "r2c_frac": round(fft_bytes / t_r2c / 1e6 / PEAK_HBM_GBPS, 4),
            "c2r_frac": round(fft_bytes / t_c2r / 1e6 / PEAK_HBM_GBPS, 4),
            "alg_bytes": fft_bytes, "roundtrip_rel_l2": rt_err}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_cpu(nsteps_all, nsteps_one):
    """The FP64 C oracle on this host, on the 512^3 headline workload: `nsteps_all` steps with its
    default thread count (OMP_NUM_THREADS, else all host threads) and `nsteps_one` steps on one
    thread."""
    import oracle
    import pfc_inputs

    shape = (N, N, N)
    p = oracle.Params(shape, r=R, dt=DT)
    psi0 = pfc_inputs.pfc_initial_field(SEED, shape, R).astype("float32").astype("float64")
    s0 = oracle.state_init(p, psi0)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.step(p, psi0, s0, nsteps_all)
    dt_all = time.perf_counter() - t0
    out = {"value": round(nsteps_all / dt_all, 4), "unit": "steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{nsteps_all} steps of the 512^3 workload by the FP64 C oracle (recursive Cooley-Tukey "
                     f"FFT, radix 2 at this size, OpenMP over lines) on {threads} threads, {dt_all:.1f} s",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if nsteps_one > 0:
        oracle.set_num_threads(1)
        t0 = time.perf_counter()
        oracle.step(p, psi0, s0, nsteps_one)
        dt_one = time.perf_counter() - t0
        oracle.set_num_threads(threads)
        out["one_thread"] = {"value": round(nsteps_one / dt_one, 4), "unit": "steps/s", "cores": 1,
                             "sample": f"{nsteps_one} step(s) of the same workload on 1 thread, {dt_one:.1f} s"}
    return out


def bench_adjoint(nsteps, every):
    """Gradient through the rollout (512^2, loss on psi(T), gradients w.r.t. psi0 and r, checkpoints
    every `every` steps): the FP32 run, timed forward + backward and forward only, and the FP64 check
    run of the same workload (psi0 and the target rounded to FP32 first, so both start alike), timed
    the same way, with the relative difference of dL/dr between the two precisions."""
    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    shape = (512, 512)

    def run(dtype):
        tdt = torch.float32 if dtype == "f32" else torch.float64
        plan_t = pfc.Plan(shape, dtype=dtype, r=-0.30, dt=0.5)
        psi0 = pfc_inputs.pfc_initial_field_torch(5, shape, -0.25, torch.float32, "cuda:0").to(tdt)
        target = psi0.clone()
        plan_t.step(target, plan_t.state_init(target), nsteps)
        plan = pfc.Plan(shape, dtype=dtype, r=-0.25, dt=0.5)
        pfc.loss_and_grad(plan, psi0, -0.25, target, 100, every)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, g, dr = pfc.loss_and_grad(plan, psi0, -0.25, target, nsteps, every)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        x = psi0.clone()
        st = plan.state_init(x)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.step(x, st, nsteps)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t1
        return t, tf, dr

    t, tf, dr = run("f32")
    t64, tf64, dr64 = run("f64")
    return {"workload": "2D 512^2 FP32, dt=0.5, loss on psi(T), grads w.r.t. psi0 and r, checkpoints every "
                        f"{every}", "steps": nsteps, "fwd_bwd_s": round(t, 4),
            "fwd_bwd_steps_per_s": round(nsteps / t, 1), "forward_only_steps_per_s": round(nsteps / tf, 1),
            "dL_dr": dr,
            "fp64_check": {"fwd_bwd_s": round(t64, 4), "fwd_bwd_steps_per_s": round(nsteps / t64, 1),
                           "forward_only_steps_per_s": round(nsteps / tf64, 1), "dL_dr": dr64,
                           "dL_dr_rel_diff_fp32": abs(dr - dr64) / abs(dr64)}}


def counters_workload(steps, n=N):
    """Workload of the counter runs: a plain 1 GiB device copy (calibration of FETCH_SIZE and
    WRITE_SIZE against known bytes), then `steps` steps of the n^3 FP32 workload (512: the headline;
    other sizes use their benchmark seeds: 750 -> 7, 1400 -> 8, 2048 -> 3)."""
    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    x = torch.empty(2**28, dtype=torch.float32, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)  # a plain streaming kernel of known bytes with a distinctive name
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()
    seed = {512: SEED, 750: 7, 1400: 8, 2048: 3}.get(n, SEED)
    shape = (n, n, n)
    plan = pfc.Plan(shape, dtype="f32", r=R, dt=DT)
    psi = pfc_inputs.pfc_initial_field_torch(seed, shape, R, torch.float32, "cuda:0")
    state = plan.state_init(psi)
    plan.step(psi, state, steps)
    torch.cuda.synchronize()


def write_traffic(fetch_dir, write_dir, out_path, command, n=N):
    """Per-dispatch HBM bytes of the step kernels from two rocprofv3 --pmc runs (FETCH_SIZE and
    WRITE_SIZE, KiB per dispatch), each scaled by the factor that makes the 1 GiB copy read and
    write exactly 1 GiB."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                rows += [r for r in csv.DictReader(fh) if r.get("Counter_Name") == counter]
        return rows

    def per_kernel(rows):
        acc = {}
        for r in rows:
            name = r["Kernel_Name"]
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
        return acc

    fetch = per_kernel(load(fetch_dir, "FETCH_SIZE"))
    write = per_kernel(load(write_dir, "WRITE_SIZE"))
    copy_bytes = 2**30

    def calibration(acc):
        # the 1 GiB streaming kernel: the neg kernel, or (older runs) the largest copy dispatch
        vals = [v for k, vs in acc.items() if "neg_kernel" in k for v in vs]
        if not vals:
            allv = [v for k, vs in acc.items() if "copy" in k.lower() for v in vs]
            top = max(allv)
            vals = [v for v in allv if v > 0.9 * top]
        return copy_bytes / (sum(vals) / len(vals))

    f_fac = calibration(fetch)
    w_fac = calibration(write)
    def targs(bare):
        # top-level template arguments of a kernel name "k<a, b<c, d>, e>(...)"
        out, depth, cur = [], 0, ""
        for ch in bare[bare.index("<") + 1:]:
            if ch == "<":
                depth += 1
            elif ch == ">":
                if depth == 0:
                    break
                depth -= 1
            if ch == "," and depth == 0:
                out.append(cur.strip())
                cur = ""
            else:
                cur += ch
        return out + [cur.strip()]

    kernels = {}
    for name, vals in fetch.items():
        bare = name.replace("void ", "").replace("pfc::", "")
        if "<" not in bare:
            continue
        a4 = (targs(bare) + [""] * 4)[3]  # CUBE of x_r2c, EPI of x_c2r, MODE of last_axis
        if bare.startswith("x_r2c_kernel<") and a4 == "true":
            short = "x_r2c_cube"
        elif bare.startswith("x_c2r_kernel<") and a4 == "0":
            short = "x_c2r"
        elif bare.startswith("x_c2r_r2c_kernel<"):
            short = "x_c2r_r2c_fused"
        elif bare.startswith("axis_c2c_kernel<"):
            short = "y_fwd_or_inv"
        elif bare.startswith("last_axis_kernel<") and a4 == "0":
            short = "z_fused_update"
        else:
            continue
        if short in kernels and kernels[short]["dispatches"] >= len(vals):
            continue  # several instantiations of one pass (state set-up, the step): keep the step's
        wv = write.get(name, [0.0])
        fb = sum(vals) / len(vals) * f_fac
        wb = sum(wv) / len(wv) * w_fac
        kernels[short] = {"fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                          "hbm_bytes_per_launch": round(fb + wb), "dispatches": len(vals), "kernel": bare[:120]}
    Rb = n**3 * 4  # algorithmic bytes per launch (FP32): x passes Rb + Cb, y 2 Cb, z 4 Cb (Cb = Rb)
    alg = {"x_r2c_cube": 2 * Rb, "y_fwd_or_inv": 2 * Rb, "z_fused_update": 4 * Rb, "x_c2r": 2 * Rb,
           "x_c2r_r2c_fused": 2 * Rb}
    for k, v in kernels.items():
        v["alg_bytes_per_launch"] = alg[k]
        v["traffic_over_alg"] = round(v["hbm_bytes_per_launch"] / alg[k], 4)
    out = {"command": command, "grid": [n, n, n], "kernel_hash": kernel_hash(), "copy_calibration_bytes": copy_bytes,
           "fetch_factor_bytes_per_unit": f_fac, "write_factor_bytes_per_unit": w_fac, "kernels": kernels}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


LEGS = ("headline", "fft", "fp64", "cube256", "big", "paper", "hydro", "amp", "batch", "adjoint", "cpu")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="timed steps of each headline repetition")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions of the headline (median reported)")
    ap.add_argument("--profile-steps", type=int, default=30, help="steps of the per-pass timed run")
    ap.add_argument("--fft-reps", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps of the CPU baseline (0: skip)")
    ap.add_argument("--cpu-steps-1t", type=int, default=1, help="oracle steps of the one-thread CPU baseline")
    ap.add_argument("--batch-steps", type=int, default=500, help="steps of the batched form (0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=2000, help="steps of the adjoint form (0: skip)")
    ap.add_argument("--big-steps", type=int, default=50, help="timed steps at 2048^3 (0: skip)")
    ap.add_argument("--hydro-steps", type=int, default=5, help="timed hydrodynamic steps at 512^3 (0: skip)")
    ap.add_argument("--amp-steps", type=int, default=20, help="timed complex-amplitude steps at 256^3 (0: skip)")
    ap.add_argument("--paper-steps", type=int, default=20,
                    help="timed steps at 750^3 and 1400^3, the paper's 3D grids (0: skip)")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs to run (default: all): " + ", ".join(LEGS))
    ap.add_argument("--counters", type=int, default=0, metavar="STEPS",
                    help="run only the workload of the rocprofv3 --pmc runs (copy calibration + STEPS steps)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc output folders into " + os.path.relpath(TRAFFIC_FILE, ROOT))
    ap.add_argument("--traffic-command", default="", help="command line recorded in the traffic summary")
    ap.add_argument("--grid", type=int, default=N, help="grid size n of the --counters / --write-traffic workload")
    args = ap.parse_args()
    if args.write_traffic:
        out = TRAFFIC_FILE if args.grid == N else os.path.join(ROOT, "profiles", f"traffic_{args.grid}cube_f32.txt")
        write_traffic(args.write_traffic[0], args.write_traffic[1], out, args.traffic_command, args.grid)
        return
    if args.counters:
        counters_workload(args.counters, args.grid)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the step would shard by "
              "slabs of the slowest axis with two all-to-all transposes per step).", file=sys.stderr)
        sys.exit(2)
    legs = set(x.strip() for x in args.legs.split(",") if x.strip())
    unknown = legs - set(LEGS)
    if unknown:
        print(f"unknown legs {sorted(unknown)}; known: {', '.join(LEGS)}", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2603_26818_amd as pfc
    import pfc_inputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    shape = (N, N, N)
    ms_per_step = steps_per_s = None
    roofline = passes = spread = F = None
    step_bytes = 12 * N**3 * 4
    step_units = 12.0
    if "headline" in legs:
        plan = pfc.Plan(shape, dtype="f32", r=R, dt=DT, device=0)
        log(f"[bench] drawing psi0 {shape} seed {SEED}")
        psi = pfc_inputs.pfc_initial_field_torch(SEED, shape, R, torch.float32, dev)
        state = plan.state_init(psi)
        log(f"[bench] warmup {args.warmup} steps")
        plan.step(psi, state, args.warmup)
        torch.cuda.synchronize()
        log(f"[bench] timed: {args.reps} repetitions of {args.steps} steps")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        runs = []
        t0 = time.perf_counter()
        for _ in range(args.reps):
            torch.cuda.synchronize()
            e0.record(stream)
            plan.step(psi, state, args.steps)
            e1.record(stream)
            torch.cuda.synchronize()
            runs.append(e0.elapsed_time(e1) / args.steps)
        wall = time.perf_counter() - t0
        ms_per_step, ms_lo, ms_hi = median_spread(runs)
        steps_per_s = 1000.0 / ms_per_step
        spread = {"reps": args.reps, "steps_per_rep": args.steps,
                  "steps_per_s_each": [round(1000.0 / m, 2) for m in runs],
                  "min": round(1000.0 / ms_hi, 2), "max": round(1000.0 / ms_lo, 2)}
        log(f"[bench] median {ms_per_step:.4f} ms/step ({steps_per_s:.1f} steps/s; "
            f"{spread['min']}..{spread['max']}), wall {wall:.3f} s")
        F = plan.energy(psi, state).cpu().tolist()
        if not all(math.isfinite(v) for v in F):
            log(f"[bench] non-finite energy {F}")
            sys.exit(1)
        # per-pass durations, HIP events on the same stream, in a separate run of profile-steps steps
        log(f"[bench] per-pass timing over {args.profile_steps} steps")
        pass_ms = plan.step_timed(psi, state, args.profile_steps)
        Rb = N**3 * 4  # real field, FP32
        Cb = N**3 // 2 * 8  # packed spectrum (same bytes as the real field)
        alg = [Rb + Cb, 2 * Cb, 4 * Cb, 2 * Cb, Cb + Rb]  # algorithmic HBM bytes per launch
        passes = []
        for name, tot, b in zip(PASS_NAMES, pass_ms, alg):
            avg = tot / args.profile_steps
            passes.append({"kernel": name, "avg_ms": round(avg, 5), "alg_bytes": b,
                           "alg_gbps": round(b / avg / 1e6, 1), "frac": round(b / avg / 1e6 / PEAK_HBM_GBPS, 4)})
        dom = max(passes, key=lambda p: p["avg_ms"])
        step_bytes = step_passes_hbm(plan, args.steps) * Rb
        step_units = step_passes_hbm(plan, args.steps)
        roofline = {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["alg_gbps"], "peak": PEAK_HBM_GBPS,
                    "unit": "GB/s", "frac": dom["frac"], "traffic": measured_traffic(dom["kernel"]),
                    "alg_bytes_per_launch": dom["alg_bytes"], "avg_ms": dom["avg_ms"]}
        del psi, state, plan
        torch.cuda.empty_cache()

    fft = None
    if "fft" in legs:
        log(f"[bench] r2c / c2r 512^3 FP32, {args.fft_reps} reps each")
        fft = bench_fft(N, "f32", args.fft_reps, 22)
        fft["256cube_f32"] = bench_fft(256, "f32", args.fft_reps, 21)
    fp64 = None
    if "fp64" in legs:
        log(f"[bench] FP64: r2c / c2r 512^3 and 256^3, steps at 512^3 and 256^3")
        fp64 = {"fft_512": bench_fft(N, "f64", args.fft_reps, 22), "fft_256": bench_fft(256, "f64", args.fft_reps, 21),
                "step_512": bench_big(max(args.steps // 6, 10), n=N, seed=SEED, dtype="f64", reps=5,
                                      profile_steps=10),
                "step_256": bench_big(max(args.steps // 2, 10), n=256, seed=2, dtype="f64", reps=5,
                                      profile_steps=10)}
        log(f"[bench] FP64 512^3 step {fp64['step_512']['steps_per_s']} steps/s ({fp64['step_512']['frac']:.3f}), "
            f"r2c {fp64['fft_512']['r2c_frac']:.3f} c2r {fp64['fft_512']['c2r_frac']:.3f}")
    cube256 = None
    if "cube256" in legs:
        log("[bench] 256^3 FP32 step (state, field and scratch fit the 256 MB memory-side cache)")
        cube256 = bench_big(args.steps, n=256, seed=2, dtype="f32", reps=5, profile_steps=30)
    big = None
    if "big" in legs and args.big_steps > 0:
        log(f"[bench] 2048^3 FP32: {args.big_steps} steps")
        big = bench_big(args.big_steps)
        log(f"[bench] 2048^3: {big['steps_per_s']} steps/s ({big['frac']:.3f} of peak)")
    paper = None
    if "paper" in legs and args.paper_steps > 0:
        paper = {}
        for n, seed in ((750, 7), (1400, 8)):
            log(f"[bench] {n}^3 FP32 (mixed radix): {args.paper_steps} steps")
            paper[str(n)] = bench_big(args.paper_steps, n=n, seed=seed)
            log(f"[bench] {n}^3: {paper[str(n)]['steps_per_s']} steps/s ({paper[str(n)]['frac']:.3f} of peak)")
    hydro = None
    if "hydro" in legs and args.hydro_steps > 0:
        log(f"[bench] hydrodynamic PFC 512^3 FP32: {args.hydro_steps} steps")
        hydro = bench_hydro(args.hydro_steps)
        log(f"[bench] hydro: {hydro['ms_per_step']} ms/step ({hydro['frac']:.3f} of peak)")
    amplitude = None
    if "amp" in legs and args.amp_steps > 0:
        log(f"[bench] complex-amplitude form, 6 bcc amplitudes on 256^3 FP32: {args.amp_steps} steps")
        amplitude = bench_amplitude(args.amp_steps)
        log(f"[bench] amplitude: {amplitude['ms_per_step']} ms/step ({amplitude['frac']:.3f} of peak)")
        log(f"[bench] complex-amplitude form, 3 triangular amplitudes on 2048^2 FP32: {args.amp_steps} steps")
        amplitude["2d_triangular_2048sq"] = bench_amplitude(args.amp_steps, (2048, 2048), "triangular", 8)
        log(f"[bench] amplitude 2D: {amplitude['2d_triangular_2048sq']['ms_per_step']} ms/step "
            f"({amplitude['2d_triangular_2048sq']['frac']:.3f} of peak)")
    batched = None
    if "batch" in legs and args.batch_steps > 0:
        log(f"[bench] batched form: 48 instances, {args.batch_steps} steps")
        batched = bench_batched(args.batch_steps)
        log(f"[bench] batched {batched['batch_steps_per_s']} batch steps/s")
    adjoint = None
    if "adjoint" in legs and args.adjoint_steps > 0:
        log(f"[bench] adjoint form: 512^2, {args.adjoint_steps} steps")
        adjoint = bench_adjoint(args.adjoint_steps, 50)
        log(f"[bench] adjoint {adjoint['fwd_bwd_steps_per_s']} steps/s forward+backward (FP64 check run "
            f"{adjoint['fp64_check']['fwd_bwd_steps_per_s']}; dL/dr FP32 vs FP64 "
            f"{adjoint['fp64_check']['dL_dr_rel_diff_fp32']:.1e})")
    cpu = None
    if "cpu" in legs and args.cpu_steps > 0:
        log(f"[bench] CPU oracle: {args.cpu_steps} FP64 steps of the same 512^3 workload, then "
            f"{args.cpu_steps_1t} on one thread")
        cpu = bench_cpu(args.cpu_steps, args.cpu_steps_1t)
        log(f"[bench] CPU oracle {cpu['value']} steps/s on {cpu['cores']} threads ({cpu['cpu_model']})")

    out = {
        "metric": METRIC, "value": round(steps_per_s, 2) if steps_per_s else None, "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5) if ms_per_step else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D one-mode PFC step, 512^3 periodic grid, FP32, dx=pi/4, r=-0.30, dt=0.5, "
                               "psi0=-0.30+U(-0.1,0.1) SplitMix64 seed 23", "grid": list(shape)},
        "timing": {"value_is": "median of the repetitions", **spread} if spread else None,
        "roofline": roofline, "cpu_baseline": cpu, "fft": fft, "passes": passes, "fp64": fp64,
        "cube256_f32": cube256, "big_2048": big, "paper_grids": paper, "hydro": hydro, "amplitude": amplitude,
        "batched": batched, "adjoint": adjoint,
        "step_hbm_passes": round(step_units, 4),
        "step_alg_gbps": round(step_bytes / ms_per_step / 1e6, 1) if ms_per_step else None,
        "step_frac": round(step_bytes / ms_per_step / 1e6 / PEAK_HBM_GBPS, 4) if ms_per_step else None,
        "energy_after": F[0] if F else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
