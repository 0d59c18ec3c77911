"""Benchmark: WENO-ZA6 interface reconstructions per second on one MI355X.

Workload (N = 1): 2D Euler, gamma = 1.4, 2048 x 2048 cells on [0,1]^2,
transmissive boundaries, seeded four-quadrant Riemann data (seed 0),
characteristic-wise WENO-ZA6 dimension by dimension, SSP-RK3 at CFL 0.5,
FP64.  One "step" is one full SSP-RK3 step (three right-hand sides, each an
x-sweep and a y-sweep over every interface plus the wave-speed reductions);
the default times the configuration's 200 steps from t = 0.

value = interface reconstructions per second = 3 * ((nx+1) ny + nx (ny+1))
        * steps / wall time, with the state resident in HBM.
Also reported: the rate sustained over 8 s of back-to-back steps (the
board then holds its power limit and runs slower than in a short burst),
the same run with FP32 reconstruction and its density error against the
FP64 run, the dominant kernel against the FP64 vector peak, and the oracle
timed on the host cores over a bounded sample of the workload.

Usage:  python bench.py [--gpus 1] [--steps 200] [--warmup 10]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FLOPs of one sweep launch, from the oracle's counting scalar
# (python -m oracle.count_flops; checked by tests/test_flop_counts.py):
# per interface, per cell for the physical flux, per cell for the flux
# difference / accumulation / RK3 stage.
FLOPS_2D = {
    "x": {"interface": 1371.0, "cell_flux": 15.0, "cell_update": 8},
    "y": {"interface": 1371.0, "cell_flux": 15.0, "cell_update": 32},
}
FLOPS_1D_IR = 1000.0 + 10.0   # 1D Euler: per interface + per-cell physical flux
# 2D Euler FLOPs per interface of the order-2r schemes, same count (the
# oracle evaluates the indicators of r != 3 as the defining integral of
# eq:SI, which is not a minimal count; see the order study).
FLOPS_2D_ORDER_IR = {2: 751.0, 3: 1371.0, 4: 3559.0, 5: 7843.0}
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 FLOP/clk
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (packed issue)
PEAK_HBM_GBS = 8000.0


def ir_per_rhs(nx, ny):
    return (nx + 1) * ny + nx * (ny + 1)


def sweep_flops(nx, ny, d):
    f = FLOPS_2D[d]
    nir = (nx + 1) * ny if d == "x" else nx * (ny + 1)
    cells = nx * ny
    return nir * f["interface"] + cells * (f["cell_flux"] + f["cell_update"])


def sweep_bytes(nx, ny, d):
    """Algorithmic HBM bytes of one sweep launch, averaged over the three RK3
    stages (FP64, m = 4, 32 B per cell and array): the x-sweep reads Q (and
    Q^n in stages 2 and 3) and writes the partial stage ca Q^n + cb (Q + dt
    L_x); the y-sweep reads Q and that partial stage and writes Q^(s+1)."""
    cells = nx * ny
    return cells * 32 * 8 // 3 if d == "x" else cells * 32 * 3


# Measured HBM traffic of the sweeps (rocprofv3 FETCH_SIZE and WRITE_SIZE,
# scaled by the same counters on a plain copy): valid only while the kernel
# sources hash to the value recorded next to the figures.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_xy_2d_euler_2048_fp64_traffic.md")
KERNEL_SOURCES = ("za_device.hpp", "za_kernels.hpp", "za_lib.hip")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_26272_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """Bytes per launch recorded for `kernel`, or None if absent or stale."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    rec = {}
    for ln in lines:
        if ":" in ln and ln.startswith("- "):
            k, v = ln[2:].split(":", 1)
            rec[k.strip()] = v.strip().strip("`")
    if rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    try:
        return float(rec["traffic " + kernel])
    except (KeyError, ValueError):
        return None


def run_gpu(P, q0_np, steps, warmup, torch, Context, settle_s=0.5, timing_pass=True):
    """Time `steps` RK3 steps of the product path (za_solve with its captured
    step graphs, no per-launch events) from q0 resident in HBM.

    Warm-up: `warmup` steps, then calls of the timed length until the GPU
    has run for at least settle_s seconds (its clocks ramp up over the first
    tens of milliseconds of load, when a sweep launch takes ~25 % longer),
    which also captures the step graph before the timed call.
    Per-kernel times come from a second run of the same steps with one HIP
    event pair around every launch on the library's stream (which runs the
    steps as direct launches)."""
    dev = torch.device("cuda:0")
    q0 = torch.from_numpy(q0_np).to(dev)
    q = q0.clone()
    ctx = Context(P)
    n_warm = 0
    t_w = time.perf_counter()
    if warmup > 0:
        ctx.solve(q, 0.0, warmup)
        n_warm += warmup
    torch.cuda.synchronize()
    # calls of the timed length: the first captures the step graph of this
    # state buffer (a one-time cost that must not land in the timed call)
    while n_warm < warmup + steps or time.perf_counter() - t_w < settle_s:
        ctx.solve(q, 0.0, steps)
        n_warm += steps
        torch.cuda.synchronize()
    warm_s = time.perf_counter() - t_w
    q.copy_(q0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ctx.solve(q, 0.0, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    avg_ms, counts = [0.0, 0.0, 0.0], [0, 0, 0]
    if timing_pass:
        q2 = q0.clone()
        ctx.set_timing(True)
        ctx.solve(q2, 0.0, steps)
        avg_ms, counts = ctx.kernel_times()
        ctx.set_timing(False)
        del q2
    ctx.close()
    return q, t1 - t0, info, avg_ms, counts, {"warmup_steps_run": n_warm, "warmup_s": warm_s}


def sustained_rate(P, q0_np, torch, Context, seconds, chunk=500):
    """RK3 steps back to back for `seconds` (za_solve calls of `chunk` steps,
    the state reset to q0 every four calls): ms per step over the calls
    that start in the second half of the window.  Under minutes of this load
    the board holds its power limit and the clocks settle below the level of
    a short burst after a brief warm-up."""
    dev = torch.device("cuda:0")
    q0 = torch.from_numpy(q0_np).to(dev)
    q = q0.clone()
    ctx = Context(P)
    ctx.solve(q, 0.0, chunk)   # captures the step graph of this buffer
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    late_steps, late_s, calls = 0, 0.0, 0
    while True:
        if calls % 4 == 0:
            q.copy_(q0)
        t0 = time.perf_counter()
        ctx.solve(q, 0.0, chunk)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        calls += 1
        if t0 - t_start >= 0.5 * seconds:
            late_steps += chunk
            late_s += t1 - t0
        if t1 - t_start >= seconds:
            break
    ctx.close()
    return {"seconds": round(time.perf_counter() - t_start, 2), "steps_timed": late_steps,
            "ms_per_step": late_s / late_steps * 1e3}


def cpu_info():
    """Host CPU: model name, logical CPUs of the machine (nproc) and of this
    process's affinity mask, and the thread-count environment."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": aff,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(P, q0_np, seconds):
    """The oracle (as it stands) on the host cores: repeated full right-hand
    sides of the workload until `seconds` have elapsed (at least one), with
    OpenMP over rows on every CPU this process may use (OMP_NUM_THREADS if
    set, which is the host's CPU share on a shared GPU machine), and one more on
    a single thread."""
    import oracle
    hw = cpu_info()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or hw["affinity_cpus"] or os.cpu_count() or 1
    oracle.set_threads(threads)
    used = oracle.get_threads()
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.rhs(P, q0_np)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    irs = n * ir_per_rhs(P.nx, P.ny) / dt
    out = {"value": irs, "unit": "IR/s", "cores": used, "kind": "oracle",
           "sample": f"{n} full right-hand side(s) of the 2D Euler {P.nx}x{P.ny} workload "
                     f"(one RK3 stage each, {ir_per_rhs(P.nx, P.ny)} IR) in {dt:.1f} s, FP64, "
                     f"OpenMP over rows on {used} threads",
           "host": hw}
    # the same oracle on one thread (one right-hand side), for reference
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.rhs(P, q0_np)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    out["single_thread"] = {"value": ir_per_rhs(P.nx, P.ny) / dt1, "unit": "IR/s", "cores": 1,
                            "sample": f"one full right-hand side in {dt1:.1f} s"}
    return out


def run_serving(lam, n_requests, budget, slots, seed=None, max_1d=65536, max_2d=1024):
    """Replay a seeded Poisson stream against the continuous-batching server.
    Latency is measured from each request's scheduled arrival time to the
    server's finish timestamp (host steady clock)."""
    import numpy as np

    from paper_2603_26272_amd import workloads as W
    from paper_2603_26272_amd.za import Server

    reqs = W.serving_stream(lam, n_requests=n_requests, seed=seed, max_1d=max_1d, max_2d=max_2d)
    ids = [None] * len(reqs)
    with Server(budget, slots) as sv:
        t0 = time.perf_counter()
        t0_ns = time.monotonic_ns()
        for i, r in enumerate(reqs):
            dt = t0 + r.arrival - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            ids[i] = sv.submit(r.problem, r.q0, r.steps)
        sv.drain()
        t1 = time.perf_counter()
        lat, irs, statuses, waits = [], 0, [], []
        fl = {0: 0.0, 1: 0.0}   # algorithmic FLOPs of FP64 (0) and FP32-reconstruction (1) requests
        first_arr = None
        last_fin = 0
        for r, rid in zip(reqs, ids):
            done, st, q, stats = sv.poll(rid, r.problem)
            statuses.append(st)
            # the server stamps with the same monotonic clock as time.monotonic_ns
            arr = t0_ns + int(r.arrival * 1e9)      # scheduled arrival
            lat.append((stats["finish_ns"] - arr) * 1e-9)
            waits.append((stats["admit_ns"] - stats["arrival_ns"]) * 1e-9)
            irs += stats["interfaces"]
            m = r.problem.m
            per_ir = FLOPS_2D["x"]["interface"] if m == 4 else FLOPS_1D_IR
            fl[int(r.problem.precision)] += stats["interfaces"] * per_ir
            first_arr = arr if first_arr is None else min(first_arr, arr)
            last_fin = max(last_fin, stats["finish_ns"])
    span = (last_fin - first_arr) * 1e-9
    lat = np.array(lat)
    return {"rate_req_s": lam, "requests": n_requests, "ok": int(sum(1 for s in statuses if s == 0)),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_admission_wait_s": float(np.mean(waits)),
            "throughput_req_s": n_requests / span, "throughput_IR_s": irs / span,
            "flop_rate_fp64_requests_TFLOP_s": fl[0] / span / 1e12,
            "flop_rate_fp32_requests_TFLOP_s": fl[1] / span / 1e12,
            "roofline_frac_fp64": fl[0] / span / (PEAK_FP64_TFLOPS * 1e12),
            "roofline_frac_fp32": fl[1] / span / (PEAK_FP32_TFLOPS * 1e12),
            # share of the vector ALU's issue capacity: non-packed FP32 issues at the FP64 rate
            "roofline_frac_valu_issue": (fl[0] + fl[1]) / span / (PEAK_FP64_TFLOPS * 1e12),
            "makespan_s": span,
            "wall_s": t1 - t0}


# ---------------------------------------------------------------------------
# studies of the other workloads (python bench.py --study NAME); each prints
# one JSON line of its own
# ---------------------------------------------------------------------------
def study_c0(torch, Context):
    """Smooth advection u_t + u_x = 0, sin(pi x), periodic [-1,1], T = 2,
    dt = 0.5 dx^2: GPU errors, observed orders, GPU and oracle time."""
    import math

    import numpy as np

    import oracle
    from paper_2603_26272_amd import workloads as W
    rows = []
    for N in (25, 50, 100, 200, 400):
        P, q0 = W.advection_sine(N)
        q = torch.from_numpy(q0).to("cuda")
        with Context(P) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = ctx.solve(q, 2.0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        x = W.centres(N, -1.0, 1.0)
        e = np.abs(q.cpu().numpy()[0, 0] - np.sin(math.pi * (x - 2.0)))
        row = {"N": N, "steps": info["steps"], "linf": float(e.max()), "l1": float(e.mean()),
               "gpu_s": t1 - t0, "gpu_IR_s": 3 * (N + 1) * info["steps"] / (t1 - t0)}
        if N <= 200:
            t0 = time.perf_counter()
            qo, *_ = oracle.solve(P, q0, 2.0)
            row["oracle_s"] = time.perf_counter() - t0
            row["max_abs_diff_vs_oracle"] = float(np.abs(qo - q.cpu().numpy()).max())
        rows.append(row)
    for a, b in zip(rows, rows[1:]):
        b["order_linf"] = math.log2(a["linf"] / b["linf"])
        b["order_l1"] = math.log2(a["l1"] / b["l1"])
    return {"study": "c0 smooth advection convergence (FP64)", "rows": rows,
            "oracle_threads": oracle.get_threads()}


def study_c1(torch, Context, seeds=(16, 256), steps=2000):
    """1D Euler N = 4096, 2000 CFL steps: one request alone (GPU context, graph
    replay), 16 and 256 seeds batched through the server (one slot each), and
    the oracle on seed 0."""
    import numpy as np

    import oracle
    from paper_2603_26272_amd import workloads as W
    from paper_2603_26272_amd.za import Server
    P, q0 = W.riemann_1d(0, 4096)
    ir_run = 3 * 4097 * steps
    q = torch.from_numpy(q0).to("cuda")
    with Context(P) as ctx:
        ctx.solve(q.clone(), 0.0, 20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.solve(q, 0.0, steps)
        torch.cuda.synchronize()
        t_alone = time.perf_counter() - t0
    gpu0 = q.cpu().numpy()
    batched = []
    probs = [W.riemann_1d(s, 4096) for s in range(max(seeds))]
    for ns in seeds:
        with Server(1 << 30, ns) as sv:
            t0 = time.perf_counter()
            ids = [sv.submit(Pk, qk, steps) for Pk, qk in probs[:ns]]
            sv.drain()
            t_batch = time.perf_counter() - t0
            served0 = sv.poll(ids[0], probs[0][0])[2]
        batched.append({"seeds": ns, "s": t_batch, "IR_s": ns * ir_run / t_batch,
                        "served_equals_alone_bitwise": bool(np.array_equal(served0, gpu0))})
    t0 = time.perf_counter()
    ref, *_ = oracle.solve(P, q0, 0.0, steps)
    t_orc = time.perf_counter() - t0
    scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
    return {"study": "c1 1D Euler N=4096, 2000 steps (FP64)",
            "alone": {"s": t_alone, "IR_s": ir_run / t_alone, "t_final": info["t"]},
            "batched": batched,
            "oracle": {"s": t_orc, "IR_s": ir_run / t_orc, "threads": 1},
            "seed0_max_rel_diff_vs_oracle": float((np.abs(gpu0 - ref) / (np.abs(ref) + scale)).max())}


def study_c3(torch, Context, n=4096, steps=200):
    """Precision: 2D quadrants at 4096^2 in FP64 and FP32 reconstruction, and
    the smooth 2D density wave at 128^2 .. 1024^2 (T = 0.05, dt = 0.5 h^2)."""
    import math

    import numpy as np

    from paper_2603_26272_amd import workloads as W
    out = {"study": "c3 FP32 reconstruction vs FP64"}
    P, q0 = W.quadrants_2d(0, n)
    res = {}
    for name, PP in (("fp64", P), ("fp32", P.fp32())):
        q = torch.from_numpy(q0).to("cuda")
        with Context(PP) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.solve(q, 0.0, steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        res[name] = (q[0].clone(), dt)
        del q
    e = (res["fp32"][0] - res["fp64"][0]).abs()
    ir = 3 * ir_per_rhs(n, n) * steps
    out["quadrants_4096"] = {"steps": steps, "fp64_IR_s": ir / res["fp64"][1], "fp32_IR_s": ir / res["fp32"][1],
                             "density_l1": float(e.mean()), "density_linf": float(e.max())}
    rows = []
    for m in (128, 256, 512, 1024):
        row = {"n": m}
        Pw, qw = W.smooth_wave_2d(m)
        exact = W.smooth_wave_2d_exact(m, 0.05)
        for name, PP in (("fp64", Pw), ("fp32", Pw.fp32())):
            q = torch.from_numpy(qw).to("cuda")
            with Context(PP) as ctx:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = ctx.solve(q, 0.05)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            err = np.abs(q[0].cpu().numpy() - exact)
            row[name] = {"linf": float(err.max()), "l1": float(err.mean()), "steps": info["steps"], "s": dt}
        rows.append(row)
    for a, b in zip(rows, rows[1:]):
        for name in ("fp64", "fp32"):
            b[name]["order_l1"] = math.log2(a[name]["l1"] / b[name]["l1"])
    out["smooth_wave"] = rows
    return out


def study_orders(torch, Context, n=2048, steps=20):
    """The fourth- to tenth-order schemes (r = 2..5) on the 2D Euler workload
    (FP64, 2048^2, 20 steps each, per-kernel HIP-event times), and the
    convergence order of the 2D Euler right-hand side on the smooth density
    wave (n = 16, 32, 64) against its exact value."""
    import math

    import numpy as np

    from paper_2603_26272_amd import workloads as W
    out = {"study": "even orders 2r = 4, 6, 8, 10 (2D Euler FP64)", "runs": [], "rhs_convergence": []}
    P, q0 = W.quadrants_2d(0, n)
    ir_step = 3 * ir_per_rhs(n, n)
    for r in (2, 3, 4, 5):
        Pr = P.with_(order=r)
        _, wall, info, avg_ms, counts, _ = run_gpu(Pr, q0, steps, 2, torch, Context)
        fl = {d: ((n + 1) * n if d == "x" else n * (n + 1)) * FLOPS_2D_ORDER_IR[r] for d in ("x", "y")}
        out["runs"].append({
            "r": r, "order": 2 * r, "steps": steps, "IR_s": ir_step * steps / wall,
            "ms_per_step": wall / steps * 1e3, "x_ms": avg_ms[0], "y_ms": avg_ms[1],
            "oracle_flop_per_ir": FLOPS_2D_ORDER_IR[r],
            "x_tflops_oracle_count": fl["x"] / (avg_ms[0] * 1e-3) / 1e12,
            "y_tflops_oracle_count": fl["y"] / (avg_ms[1] * 1e-3) / 1e12})
    for r in (2, 3, 4, 5):
        row = {"r": r, "linf": []}
        for m in (16, 32, 64):
            Pw, qw = W.smooth_wave_2d(m)
            Pw = Pw.with_(order=r)
            q = torch.from_numpy(qw).to("cuda")
            with Context(Pw) as ctx:
                L = ctx.rhs(q).cpu().numpy()
            x = W.centres(m, 0.0, 1.0)[None, :]
            y = W.centres(m, 0.0, 1.0)[:, None]
            exact = -0.8 * math.pi * np.cos(2.0 * math.pi * (x + y))   # -(rho_x + rho_y)
            row["linf"].append(float(np.abs(L[0] - exact).max()))
        row["rates"] = [math.log2(a / b) for a, b in zip(row["linf"], row["linf"][1:])]
        out["rhs_convergence"].append(row)
    return out


def study_scalar(torch, Context):
    """Scalar laws of Section 4.1 on the GPU: the multi-wave advection run
    (N = 400, T = 20) against its exact solution, Burgers (N = 80, T = 0.2)
    against the characteristic solution away from the shock, Buckley-Leverett
    (N = 200, T = 0.3) against an N = 3200 run of the same code, and the
    throughput of 2D scalar sweeps at 2048^2 (advection and Buckley-Leverett,
    20 steps)."""
    import numpy as np

    from paper_2603_26272_amd import workloads as W
    from paper_2603_26272_amd.problem import ADVECTION, BUCKLEY, PERIODIC, Problem
    out = {"study": "scalar laws (Section 4.1)"}

    def solve(P, q0, T):
        q = torch.from_numpy(np.ascontiguousarray(q0)).to("cuda")
        with Context(P) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = ctx.solve(q, T)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        return q.cpu().numpy()[0, 0], info, wall

    P, q0 = W.multiwave(400)
    q, info, wall = solve(P, q0, W.MULTIWAVE_T)
    x = W.centres(400, -1.0, 1.0)
    e = np.abs(q - W.multiwave_exact(x))
    g = (x > -0.8) & (x < -0.6)
    out["multiwave"] = {"N": 400, "T": W.MULTIWAVE_T, "steps": info["steps"], "wall_s": wall,
                        "l1": float(e.mean() * 2.0), "linf": float(e.max()), "gaussian_linf": float(e[g].max()),
                        "max": float(q.max()), "min": float(q.min())}
    P, q0 = W.burgers_sine(80)
    q, info, wall = solve(P, q0, W.BURGERS_T)
    x = W.centres(80, 0.0, 1.0)
    e = np.abs(q - W.burgers_sine_exact(x, W.BURGERS_T))
    xs = 0.5 + 0.5 * W.BURGERS_T
    far = np.abs(((x - xs) + 0.5) % 1.0 - 0.5) > 0.1
    out["burgers"] = {"N": 80, "T": W.BURGERS_T, "steps": info["steps"], "linf_away_from_shock": float(e[far].max()),
                      "linf_near_shock": float(e[~far].max())}
    P, q0 = W.buckley_step(200)
    q, info, wall = solve(P, q0, W.BUCKLEY_T)
    Pf, qf = W.buckley_step(3200)
    rf, _, _ = solve(Pf, qf, W.BUCKLEY_T)
    out["buckley"] = {"N": 200, "T": W.BUCKLEY_T, "steps": info["steps"],
                      "l1_vs_N3200": float(np.abs(q - rf.reshape(200, 16).mean(axis=1)).mean() * 2.0),
                      "max": float(q.max()), "min": float(q.min())}
    n = 2048
    x = W.centres(n, 0.0, 1.0)[None, :]
    y = W.centres(n, 0.0, 1.0)[:, None]
    base = 0.5 + 0.4 * np.sin(2 * np.pi * (x + 2 * y)) + 0.3 * (x > 0.5) * (y < 0.4)
    rows = []
    for name, system in (("advection_2d", ADVECTION), ("buckley_2d", BUCKLEY)):
        P = Problem(dim=2, system=system, nx=n, ny=n, bc_x=PERIODIC, bc_y=PERIODIC, adv_speed=(1.0, 0.5))
        _, wall, info, avg_ms, counts, _ = run_gpu(P, np.ascontiguousarray(base.reshape(1, n, n)), 20, 2, torch,
                                                Context)
        rows.append({"workload": f"{name} {n}x{n} FP64", "IR_s": 3 * ir_per_rhs(n, n) * 20 / wall,
                     "ms_per_step": wall / 20 * 1e3, "x_ms": avg_ms[0], "y_ms": avg_ms[1]})
    out["throughput_2d"] = rows
    return out


def study_pp(torch, Context, n=2048, steps=20):
    """Cost and reach of the positivity-preserving limiter: the 2D Euler
    workload (2048^2, 20 steps) with and without it (every face evaluates
    its half states; few are limited), and the near-vacuum diverging
    quadrants at 1024^2 to T = 0.05, which fail without it."""
    import numpy as np

    from paper_2603_26272_amd import workloads as W
    from paper_2603_26272_amd.za import ZA_OK
    out = {"study": "positivity-preserving limiter (2D Euler FP64)", "runs": []}
    P, q0 = W.quadrants_2d(0, n)
    ir_step = 3 * ir_per_rhs(n, n)
    for pp in (0, 1):
        _, wall, info, avg_ms, counts, _ = run_gpu(P.with_(pp_limiter=pp, cfl=0.45), q0, steps, 2, torch, Context)
        out["runs"].append({"workload": f"quadrants {n}x{n} CFL 0.45", "pp_limiter": pp, "IR_s": ir_step * steps / wall,
                            "ms_per_step": wall / steps * 1e3, "x_ms": avg_ms[0], "y_ms": avg_ms[1]})
    m = 1024
    Pv, qv = W.vacuum_quadrants_2d(m)
    for pp in (0, 1):
        q = torch.from_numpy(qv).to("cuda")
        with Context(Pv.with_(pp_limiter=pp)) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve(q, 0.05, check=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        rho = q[0]
        pr = 0.4 * (q[3] - 0.5 * (q[1] ** 2 + q[2] ** 2) / rho)
        out["runs"].append({"workload": f"vacuum quadrants {m}x{m} to T = 0.05", "pp_limiter": pp,
                            "status": res["status"], "ok": res["status"] == ZA_OK, "steps": res["steps"],
                            "t": res["t"], "wall_s": wall,
                            "rho_min": float(rho.min()) if res["status"] == ZA_OK else None,
                            "p_min": float(pr.min()) if res["status"] == ZA_OK else None})
    return out


def study_adr(torch, Context, n=256):
    """Approximate dispersion relation (Section 3.2) of CT6, WENO-ZA6 with tau
    and with tau', and the other even orders: Phi(phi) of every resolvable
    mode of an n-cell periodic grid from libza's right-hand side, at three
    amplitudes (the Z weights are scale-invariant up to epsilon)."""
    import numpy as np

    from paper_2603_26272_amd import adr
    out = {"study": f"approximate dispersion relation, N = {n}", "schemes": {}}
    for name, kw in adr.SCHEMES.items():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, Phi = adr.adr_gpu(n, **kw)
        wall = time.perf_counter() - t0
        amp = max(float(np.abs(adr.adr_gpu(n, amplitude=a, **kw)[1] - Phi).max()) for a in (1e-3, 1e3))
        k = int(np.argmax(Phi.imag))
        pick = [int(np.argmin(np.abs(phi - v))) for v in (0.25, 0.5, 0.7, 1.0, 1.5, 2.0, 2.5, 3.0, np.pi)]
        out["schemes"][name] = {"wall_s": wall, "max_im": float(Phi.imag[k]), "phi_at_max_im": float(phi[k]),
                                "max_abs_phi_error_below_0.5": float(np.abs(Phi - phi)[phi < 0.5].max()),
                                "amplitude_dependence": amp,
                                "samples": [[float(phi[i]), float(Phi[i].real), float(Phi[i].imag)] for i in pick]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sustained-s", type=float, default=8.0,
                    help="seconds of back-to-back steps for the sustained rate (0: skip)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-rates", type=str, default="10,25,50,100,200",
                    help="Poisson rates (req/s) of the serving leg")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-budget-gb", type=float, default=4.0)
    ap.add_argument("--study", choices=["c0", "c1", "c3", "orders", "scalar", "pp", "adr", "serving"], default=None,
                    help="run one workload study instead of the benchmark line")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the library runs on one MI355X "
              f"(the multi-GPU slab decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2603_26272_amd import workloads as W
    from paper_2603_26272_amd.za import Context

    torch.cuda.set_device(0)
    if args.study:
        if args.study == "c0":
            res = study_c0(torch, Context)
        elif args.study == "c1":
            res = study_c1(torch, Context)
        elif args.study == "c3":
            res = study_c3(torch, Context)
        elif args.study == "orders":
            res = study_orders(torch, Context)
        elif args.study == "scalar":
            res = study_scalar(torch, Context)
        elif args.study == "pp":
            res = study_pp(torch, Context)
        elif args.study == "adr":
            res = study_adr(torch, Context)
        else:
            rates = [float(x) for x in args.serving_rates.split(",") if x]
            res = {"study": "serving sweep", "hbm_budget_gb": args.serving_budget_gb,
                   "runs": [run_serving(lam, args.serving_requests, int(args.serving_budget_gb * (1 << 30)), 64)
                            for lam in rates]}
        print(json.dumps(res), flush=True)
        return
    P, q0 = W.quadrants_2d(args.seed, args.n)
    nx, ny = P.nx, P.ny
    ir_step = 3 * ir_per_rhs(nx, ny)

    def log(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    q64, wall, info, avg_ms, counts, warm = run_gpu(P, q0, args.steps, args.warmup, torch, Context)
    assert info["steps"] == args.steps, info
    value = ir_step * args.steps / wall
    ms_step = wall / args.steps * 1e3
    log(f"FP64 {value:.4g} IR/s, {ms_step:.4f} ms/step")

    names = ["x-sweep", "y-sweep", "wave-speed"]
    dom = 0 if avg_ms[0] >= avg_ms[1] else 1
    d = "x" if dom == 0 else "y"
    fl = sweep_flops(nx, ny, d)
    achieved = fl / (avg_ms[dom] * 1e-3) / 1e12
    kname = "k_sweep_xl" if d == "x" else "k_sweep_y"   # the 2D FP64 stage kernels
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(kname),
                "kernel": f"{kname} (2D Euler FP64)",
                "avg_launch_ms": avg_ms[dom], "launches": counts[dom],
                "timing": "HIP events around every launch on the library's stream, in a second run of the "
                          "same steps after the timed one",
                "algorithmic_flop_per_launch": fl,
                "algorithmic_bytes_per_launch": sweep_bytes(nx, ny, d)}
    kernels = {names[k]: {"avg_ms": avg_ms[k], "launches": counts[k]} for k in range(3)}
    for k, dd in ((0, "x"), (1, "y")):
        kernels[names[k]]["tflops"] = sweep_flops(nx, ny, dd) / (avg_ms[k] * 1e-3) / 1e12 if avg_ms[k] else None

    out = {
        "metric": "WENO-ZA6 interface recons/s (2D Euler, FP64 vs FP32) + served p50/p99 latency",
        "value": value,
        "unit": "IR/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded four-quadrant Riemann data)",
        "config": {"workload": f"2D Euler {nx}x{ny} four-quadrant Riemann, transmissive, "
                               f"WENO-ZA6 characteristic-wise, SSP-RK3 CFL 0.5, FP64",
                   "nx": nx, "ny": ny, "seed": args.seed, "ir_per_step": ir_step,
                   "t_final": info["t"]},
        "timed": "za_solve of the steps (captured step graphs, no per-launch events); state resident in HBM",
        "warmup_detail": warm,
        "roofline": roofline,
        "kernels": kernels,
        # scalar WENO reconstructions: 2 splits x 4 characteristic fields per IR
        "split_field_recons_per_s": 8 * value,
    }

    if args.sustained_s > 0:
        su = sustained_rate(P, q0, torch, Context, args.sustained_s)
        su["value"] = ir_step / (su["ms_per_step"] * 1e-3)
        su["note"] = ("za_solve calls run back to back; rate over the second half of the window, "
                      "with the board at its power limit")
        out["sustained"] = su
        log(f"sustained: {su['value']:.4g} IR/s, {su['ms_per_step']:.4f} ms/step")

    if not args.no_fp32:
        out["fp32"] = fp32_leg(P, q0, q64, args, torch, Context, log)

    if not args.no_serving:
        rates = [float(x) for x in args.serving_rates.split(",") if x]
        runs = []
        for lam in rates:
            runs.append(run_serving(lam, args.serving_requests, int(args.serving_budget_gb * (1 << 30)), 64))
            log(f"serving {lam:g} req/s: p50 {runs[-1]['p50_latency_s']:.3f} s, p99 {runs[-1]['p99_latency_s']:.3f} s, "
                f"{runs[-1]['throughput_IR_s']:.3g} IR/s")
        out["serving"] = {"workload": f"Poisson stream of {args.serving_requests} requests per rate: half 1D Euler N "
                                      "log-uniform [512, 65536], half 2D Euler n x n log-uniform [128, 1024]; "
                                      "Riemann or smooth data; 50-500 RK3 steps; FP64 or FP32 reconstruction "
                                      "(seed = rate)",
                          "hbm_budget_gb": args.serving_budget_gb, "max_slots": 64, "runs": runs}
        top = max(runs, key=lambda r: r["rate_req_s"])
        out["p50_latency_s"] = top["p50_latency_s"]
        out["p99_latency_s"] = top["p99_latency_s"]

    if not args.no_cpu_baseline:
        cb = cpu_baseline(P, q0, args.cpu_seconds)
        cb["gpu_over_cpu"] = value / cb["value"]
        out["cpu_baseline"] = cb
        log(f"cpu baseline {cb['value']:.3g} IR/s on {cb['cores']} threads")
    print(json.dumps(out), flush=True)


def fp32_leg(P, q0, q64, args, torch, Context, log, oracle_steps=10):
    """FP32 reconstruction on the same workload: throughput, the slower sweep
    against the FP32 vector peak, and the density error of the FP32 result
    (i) against the FP64 GPU run after the timed steps and (ii) against the
    FP64 oracle after `oracle_steps` steps, next to the FP64 GPU run's own
    distance to the oracle there (which ties (i) to the oracle)."""
    import numpy as np

    import oracle
    nx, ny = P.nx, P.ny
    ir_step = 3 * ir_per_rhs(nx, ny)
    P32 = P.fp32()
    q32, wall32, info32, avg32, cnt32, warm32 = run_gpu(P32, q0, args.steps, args.warmup, torch, Context)
    names = ["x-sweep", "y-sweep", "wave-speed"]
    r64 = q64[0].double()
    e = (q32[0].double() - r64).abs()
    res = {"value": ir_step * args.steps / wall32, "unit": "IR/s",
           "ms_per_step": wall32 / args.steps * 1e3,
           "density_err_vs_gpu_fp64": {"steps": args.steps, "l1": float(e.mean()), "linf": float(e.max())},
           "avg_launch_ms": {names[k]: avg32[k] for k in range(3)},
           "warmup_detail": warm32}
    log(f"FP32 reconstruction {res['value']:.4g} IR/s")
    dom = 0 if avg32[0] >= avg32[1] else 1
    d = "x" if dom == 0 else "y"
    fl = sweep_flops(nx, ny, d)
    ach = fl / (avg32[dom] * 1e-3) / 1e12
    res["roofline"] = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                       "frac": ach / PEAK_FP32_TFLOPS, "kernel": f"k_sweep_{d} (2D Euler FP32 reconstruction)",
                       "avg_launch_ms": avg32[dom],
                       "note": "FP32 vector peak with packed FP32 issue; the library is built without packed "
                               "FP32 instructions, whose non-packed issue rate equals the FP64 rate (78.6)",
                       "frac_of_unpacked_issue_rate": ach / PEAK_FP64_TFLOPS,
                       "algorithmic_flop_per_launch": fl,
                       "algorithmic_bytes_per_launch": sweep_bytes(nx, ny, d),
                       "hbm_GB_s_algorithmic": sweep_bytes(nx, ny, d) / (avg32[dom] * 1e-3) / 1e9}
    # against the FP64 oracle after a few steps
    n = min(oracle_steps, args.steps)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    ref, steps, t, st = oracle.solve(P, q0, 0.0, n)
    t_orc = time.perf_counter() - t0
    got = {}
    for name, PP in (("fp64", P), ("fp32", P32)):
        q = torch.from_numpy(q0).to("cuda")
        with Context(PP) as ctx:
            ctx.solve(q, 0.0, n)
        got[name] = q.cpu().numpy()
        del q
    e32 = np.abs(got["fp32"][0] - ref[0])
    e64 = np.abs(got["fp64"][0] - ref[0])
    res["density_err_vs_fp64_oracle"] = {
        "steps": n, "l1": float(e32.mean()), "linf": float(e32.max()),
        "gpu_fp64_vs_oracle": {"l1": float(e64.mean()), "linf": float(e64.max())},
        "oracle_s": t_orc, "oracle_threads": oracle.get_threads()}
    log(f"FP32 density vs oracle after {n} steps: L1 {e32.mean():.3g}, Linf {e32.max():.3g} "
        f"(FP64 GPU: Linf {e64.max():.3g})")
    return res


if __name__ == "__main__":
    main()
