"""Benchmark: phi_0..phi_4 actions of a 3D advection-diffusion-reaction Kronecker sum.

Workload: n = 256^3 (N = 16,777,216 dofs), A_mu = 0.5 * FD2 Laplacian + central
advection (beta_mu = 1, 0.5, 0.25) - I, Dirichlet, h = 1/257, tau = 1e-3,
v ~ N(0, 1) (seed 2), phi-functions on the same vector, p = 4, one scale,
tolerance 2^-53 ||v||_2, FP64 throughout.

One step is one pass of the whole path: host planning of (s, q), the device Taylor
exponentials of the small matrices and their squarings, and the phi-action call
(phiks_plan + phiks_apply + phiks_plan_destroy), all on one stream.  Inputs are
resident in HBM before the timed region.  The value is dofs/s = N * steps / time.

Also reported (same JSON line): the roofline of the dominant kernel (the FP64 MFMA
mu-mode product of the call), measured live with HIP events recorded by the library
around every mu-mode launch of the calls of sampled timed steps, and the CPU oracle
timed on this host for one full call.  Device memory comes from the library itself (no
other GPU framework is loaded).
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

METRIC = ("φ-action dofs/s and μ-mode GFLOP/s (% MFMA peak), FP64 vs FP32-MFMA; "
          "p99 lat")
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 (matrix)
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 (matrix)
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per mu-mode launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since those counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "mu_mode_gemm_adr3d_256_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in ("gemm_f64.hpp", "gemm_f64_dl.hpp", "tucker_f64.hpp", "kernel_tuning.inc"):
        h.update(open(os.path.join(ROOT, "paper_2210_07667_amd", "csrc", f), "rb").read())
    m1 = re.search(r"kernel_source_sha256: (\w+)", text)
    m2 = re.search(r"traffic_bytes_per_launch: ([0-9.eE+-]+)", text)
    if not m1 or not m2 or m1.group(1) != h.hexdigest():
        return None
    return float(m2.group(1))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, plan_info):
    """Time the oracle (as it stands) on this host.  All-core leg: its own planner plus one
    full phi_0..phi_4 call of the same workload.  One-core leg, a bounded sample: one
    Tucker operator (the three loop mode products) and the small exponentials of one
    mode on one thread, scaled to a full call (T_exec Tucker operators, d modes of
    exponentials) plus the planner's time (single-threaded Python either way)."""
    from oracle import bound, expm as oexpm, gll as ogll, phiks as ophiks, tensor
    all_threads = tensor.threads()
    t0 = time.perf_counter()
    xi = bound.kron_sum_rectangle([w.tau * a for a in w.A])
    s, q, _ = bound.plan(xi, w.p, w.n_scales, w.tol, w.task)
    t1 = time.perf_counter()
    ophiks.phi_same_vector(w.A, w.tau, w.v, w.p, w.n_scales, s, q)
    t2 = time.perf_counter()
    plan_s = t1 - t0
    # one-core sample
    t_exec = (q - 1) + s * w.p + w.n_scales
    try:
        import threadpoolctl
        limiter = threadpoolctl.threadpool_limits(1)
    except Exception:
        limiter = None
    tensor.set_threads(1)
    try:
        theta, _ = ogll.gll(q)
        B = w.tau * np.asarray(w.A[0])
        e0 = time.perf_counter()
        mats = [oexpm.expm_taylor((1.0 - th) * B / 2.0 ** s) for th in theta[:-1]]
        E = oexpm.expm_taylor(B / 2.0 ** s)
        for _ in range(s):
            E = E @ E
        e1 = time.perf_counter()
        tensor.tucker(w.v, w.n, [mats[0]] * len(w.n))
        e2 = time.perf_counter()
    finally:
        tensor.set_threads(all_threads)
        if limiter is not None:
            limiter.unregister()
    expm_1 = (e1 - e0) * len(w.n)
    tucker_1 = e2 - e1
    one_core_s = plan_s + expm_1 + t_exec * tucker_1
    try:
        nproc = len(os.sched_getaffinity(0))
    except Exception:
        nproc = os.cpu_count() or 1
    return {"value": w.N / (t2 - t0), "unit": "dofs/s", "cores": int(all_threads),
            "kind": "oracle",
            "sample": (f"one full call at 256^3 on {all_threads} threads (planner {plan_s:.1f} s + "
                       f"phi-actions {t2 - t1:.1f} s, plan s={s} q={q}); mu-mode products by "
                       "plain C loops (OpenMP over output fibres), small exponentials by a "
                       "Taylor series on NumPy matmuls"),
            "seconds": t2 - t0, "nproc": nproc, "cpu_model": _cpu_model(),
            "one_core": {"value": w.N / one_core_s, "unit": "dofs/s", "cores": 1,
                         "seconds_extrapolated": one_core_s,
                         "sample": (f"one Tucker operator {tucker_1:.1f} s and one mode's "
                                    f"{q} small exponentials {e1 - e0:.1f} s on one thread, "
                                    f"scaled by T_exec = {t_exec} and d = {len(w.n)}, plus the "
                                    f"planner {plan_s:.1f} s")}}


def combine_section(ph, reps=5):
    """Linear combinations (phiks_combine, eqs. integrandcomb / comb): the 256^3 ADR
    operator with p = 4 and five N(0, 1) vectors, and the 3D Allen-Cahn 64^3 workload
    (p = 4, two scales, tau = 1e-3 and 1e-2) with one step of the scheme of eq.
    expRK4s6 on it.  Plans built once; wall time without kernel events, then one call
    with events for the mu-mode kernel rate."""
    import workloads
    from paper_2210_07667_amd import integrators as gi

    def timed(A, tau, vs, p, ns):
        N = int(vs[0].size)
        plan = ph.phiks_plan(A, tau, p, ns, 2.0 ** -53, "lincomb")
        dv = [ph.DeviceArray.from_numpy(x) for x in vs]
        out = ph.DeviceArray(ns * N)
        ws = ph.DeviceArray(plan.workspace_size() // 8 + 1)
        ptrs = [x.ptr for x in dv]
        ph.phiks_combine(plan, ptrs, out.ptr, ws.ptr, ws.nbytes)
        ph.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ph.phiks_combine(plan, ptrs, out.ptr, ws.ptr, ws.nbytes)
        ph.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        ph.phiks_kernel_timing_read()
        ph.phiks_kernel_timing(True)
        ph.phiks_combine(plan, ptrs, out.ptr, ws.ptr, ws.nbytes)
        ph.synchronize()
        ph.phiks_kernel_timing(False)
        km, kl, kf = ph.phiks_kernel_timing_read()
        info = plan.info()
        plan.close()
        for x in dv + [out, ws]:
            x.free()
        return {"call_ms": ms, "dofs_per_s": N / (ms * 1e-3), "plan": info,
                "mu_mode_launches": kl, "mu_mode_ms": km,
                "mu_mode_tflops": (kf / (km * 1e-3)) / 1e12 if km > 0 else 0.0,
                "mu_mode_frac_fp64_peak": ((kf / (km * 1e-3)) / 1e12 / FP64_PEAK_TFLOPS) if km > 0 else 0.0}

    out = {}
    wa = workloads.config_adr_3d()
    vs = [workloads.randn_vec(wa.n, 90 + k) for k in range(5)]
    log("[bench] combination 256^3 p=4")
    out["adr3d_256^3_p4"] = timed(wa.A, wa.tau, vs, 4, 1)
    del vs
    for tau in (1e-3, 1e-2):
        w = workloads.config_allen_cahn_3d(tau=tau)
        log(f"[bench] combination allen-cahn 64^3 tau={tau}")
        r = timed(w.A, w.tau, w.vs, w.p, w.n_scales)
        # one step of the fourth-order six-stage scheme (four combinations + stage vectors)
        u0 = w.vs[0]
        g = gi.AllenCahnNonlinearity(u0.size)
        gi.exprk4s6(w.A, u0, g, tau, 1)
        ph.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            gi.exprk4s6(w.A, u0, g, tau, 1)
        ph.synchronize()
        r["exprk4s6_step_ms"] = (time.perf_counter() - t0) * 1e3 / reps
        r["exprk4s6_note"] = "one step incl. its plan builds and host-to-device copy of u_0"
        out[f"allen_cahn_64^3_p4_2scales_tau{tau:g}"] = r
    return out


def small_2d_section(ph, reps=50):
    """The 2D FD Laplacian 32x32 workload (tau = 1e-3, phi_0..phi_3, one scale): plan
    build, small exponentials and phi-action call latency, each waited for."""
    import workloads
    w = workloads.config_fd2_2d()
    v = ph.DeviceArray.from_numpy(w.v)
    out = ph.DeviceArray((w.p + 1) * w.N)
    plan_ms, call_ms = [], []
    for it in range(reps + 3):
        c0 = time.perf_counter()
        pl = ph.phiks_plan(w.A, w.tau, w.p, 1, w.tol, "same_vector", [float(np.linalg.norm(w.v))])
        ph.synchronize()
        c1 = time.perf_counter()
        ws = ph.DeviceArray(pl.workspace_size() // 8 + 1)
        ph.synchronize()
        c2 = time.perf_counter()
        ph.phiks_apply(pl, v.ptr, out.ptr, ws.ptr, ws.nbytes)
        ph.synchronize()
        c3 = time.perf_counter()
        info = pl.info()
        pl.close()
        ws.free()
        if it >= 3:
            plan_ms.append((c1 - c0) * 1e3)
            call_ms.append((c3 - c2) * 1e3)
    return {"workload": "fd2_2d_32x32_phi0-3_tau1e-3", "N": w.N, "plan": info,
            "plan_ms_p50": float(np.median(plan_ms)), "call_ms_p50": float(np.median(call_ms)),
            "call_ms_p90": float(np.percentile(call_ms, 90)),
            "dofs_per_s_call": w.N / (np.median(call_ms) * 1e-3),
            "note": "plan = host planner + device small exponentials; call = phiks_apply, "
                    "each waited for on the host"}


def batched_section(ph, reps=3, precision=0):
    """The 512-problem batched workload (d in {2, 3}, n_mu in 16..128, Chebyshev D^2,
    tau log-uniform, phi_0..phi_3): one phiks_batch_apply against the same problems
    run one by one through phiks_apply (plans built beforehand in both cases), in the
    mu-mode arithmetic `precision` (FP64 or FP32 MFMA)."""
    import workloads
    problems = workloads.config_batch()
    norms = [float(np.linalg.norm(b.v)) for b in problems]
    tp0 = time.perf_counter()
    batch = ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems], 3, 1,
                                2.0 ** -53, vnorms=norms, precision=precision)
    ph.synchronize()
    plan_s = time.perf_counter() - tp0
    dv = [ph.DeviceArray.from_numpy(b.v) for b in problems]
    outs = [ph.DeviceArray(4 * b.N) for b in problems]
    ws = ph.DeviceArray(batch.workspace_size() // 8 + 1)
    vp, op = [v.ptr for v in dv], [o.ptr for o in outs]
    # two untimed calls: the first runs eagerly, the second captures the launches into
    # a graph that the timed calls replay
    for _ in range(2):
        ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
    ph.synchronize()
    # wall time without kernel events (a timestamped dispatch idles the GPU ~9 us after
    # each of the ~230 launches), then one more call with events for the kernel rate
    t0 = time.perf_counter()
    for _ in range(reps):
        ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
    ph.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3 / reps
    ph.phiks_kernel_timing_read()
    ph.phiks_kernel_timing(True)
    ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
    ph.synchronize()
    ph.phiks_kernel_timing(False)
    k_ms, k_launch, k_flops = ph.phiks_kernel_timing_read()
    smax = max(batch.info(i)["s"] for i in range(len(problems)))
    batch.close()
    ws.free()
    # the same problems through the single-problem path, one call each
    plans = [ph.phiks_plan(b.A, b.tau, 3, 1, 2.0 ** -53, "same_vector", [nv], precision=precision)
             for b, nv in zip(problems, norms)]
    wsz = max(pl.workspace_size() for pl in plans)
    ws1 = ph.DeviceArray(wsz // 8 + 1)
    for pl, v, o in zip(plans, vp, op):
        ph.phiks_apply(pl, v, o, ws1.ptr, ws1.nbytes)
    ph.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for pl, v, o in zip(plans, vp, op):
            ph.phiks_apply(pl, v, o, ws1.ptr, ws1.nbytes)
    ph.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3 / reps
    for pl in plans:
        pl.close()
    ws1.free()
    for x in dv + outs:
        x.free()
    total = sum(b.N for b in problems)
    return {"workload": "batched_512_cheb_d2_phi0-3_tau1e-4..1e-2_" +
                        ("fp32" if precision == ph.PHIKS_FP32 else "fp64"), "problems": len(problems),
            "total_dofs": total, "apply_ms": batch_ms, "dofs_per_s": total / (batch_ms * 1e-3),
            "plan_s": plan_s, "max_s": smax, "mu_mode_launches": k_launch,
            "mu_mode_tflops": (k_flops / (k_ms * 1e-3)) / 1e12 if k_ms > 0 else 0.0,
            "mu_mode_ms": k_ms, "single_calls_ms": seq_ms,
            "speedup_vs_single_calls": seq_ms / batch_ms}


def serving_section(ph, rates=(100, 300, 600), duration=1.5, mixed=False):
    """Served requests of the serving workload (12 sessions: FD2 / ADR / Brusselator-type
    diffusion on 256^2, 1024^2, 64^3, 128^3, 192^3; p in 1..4; tau log-uniform) arriving as
    a Poisson stream at each rate; latency is submission to completion as the server
    stamps it.  mixed=True: the odd-numbered sessions' requests take FP32 mu-mode
    products (the rest FP64).  Every session's plan is built once before the timed
    streams."""
    import queue
    import threading
    import workloads
    sessions = workloads.serving_sessions()
    prec = [ph.PHIKS_FP32 if (mixed and k % 2 == 1) else ph.PHIKS_FP64 for k in range(len(sessions))]
    GiB = 1 << 30
    server = ph.Server(hbm_budget=64 * GiB, workspace_bytes=32 * GiB, max_active=32, lanes=3)
    rng = np.random.default_rng(4)
    ops = [server.register(sess.A) for sess in sessions]
    vin = [[ph.DeviceArray.from_numpy(rng.standard_normal(sess.N)) for _ in range(2)]
           for sess in sessions]
    pools = []
    for sess in sessions:
        q = queue.Queue()
        for _ in range(24):
            q.put(ph.DeviceArray((sess.p + 1) * sess.N))
        pools.append(q)
    # plans: one request per session (cache misses), not timed
    warm = []
    for si, sess in enumerate(sessions):
        buf = pools[si].get()
        warm.append((server.submit(ops[si], sess.tau, sess.p, 1, 2.0 ** -53, vin[si][0].ptr, buf.ptr,
                                   precision=prec[si]), si, buf))
    for t, si, buf in warm:
        server.wait(t)
        pools[si].put(buf)
    out = []
    for k, rate in enumerate(rates):
        arrivals = workloads.poisson_arrivals(rate, duration, 40 + k)
        picks = rng.integers(len(sessions), size=len(arrivals))
        lat = []
        waitq = queue.Queue()

        def waiter():
            while True:
                item = waitq.get()
                if item is None:
                    return
                t, si, buf = item
                lat.append(server.wait(t))
                pools[si].put(buf)

        th = threading.Thread(target=waiter)
        th.start()
        dofs = 0
        t0 = time.perf_counter()
        for j, (at, si) in enumerate(zip(arrivals, picks)):
            delay = t0 + at - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            sess = sessions[si]
            buf = pools[si].get()
            t = server.submit(ops[si], sess.tau, sess.p, 1, 2.0 ** -53, vin[si][j % 2].ptr, buf.ptr,
                              precision=prec[si])
            waitq.put((t, si, buf))
            dofs += sess.N
        waitq.put(None)
        th.join()
        wall = time.perf_counter() - t0
        la = np.asarray(lat) * 1e3
        out.append({"rate_per_s": rate, "requests": len(la), "p50_ms": float(np.percentile(la, 50)),
                    "p99_ms": float(np.percentile(la, 99)), "mean_ms": float(la.mean()),
                    "throughput_per_s": len(la) / wall, "dofs_per_s": dofs / wall})
        log(f"[bench] serving{' mixed' if mixed else ''} rate {rate}/s: p50 {out[-1]['p50_ms']:.2f} ms "
            f"p99 {out[-1]['p99_ms']:.2f} ms")
    st = server.stats()
    server.close()
    return {"workload": "serving_12_sessions_poisson" + ("_fp64_fp32_mix" if mixed else "_fp64"),
            "sessions": [s.name + ("_fp32" if p == ph.PHIKS_FP32 else "") for s, p in zip(sessions, prec)],
            "duration_s_per_rate": duration, "rates": out, "server": st,
            "engine": "3 size lanes (own streams), step-level continuous batching, slot per request"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 512-problem batched section")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the served-requests section")
    ap.add_argument("--no-combine", action="store_true",
                    help="skip the linear-combination section")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 2D 32x32 latency section")
    ap.add_argument("--counters", action="store_true",
                    help="hardware-counter run: copy N doubles device-to-device once (a plain "
                         "copy of known size, to scale byte counters), then run exactly one "
                         "step (one plan, one call) and exit, so the counted launches are "
                         "the mix of a timed step")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the phi-action path here is single-GPU "
              "(multi-GPU slab sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import paper_2210_07667_amd as ph
    import workloads

    if ph.device_count() < 1:
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    w = workloads.config_adr_3d(n=args.n)
    log(f"[bench] workload {w.name} N={w.N} tau={w.tau} p={w.p}")
    v = ph.DeviceArray.from_numpy(w.v)
    st = 0  # null stream

    if args.counters:
        tmp = ph.DeviceArray(w.N)
        ph.copy_device(tmp, v, st)
        ph.synchronize()
        tmp.free()
        log(f"[bench] calibration copy of {w.N * 8} bytes done")
        pl = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, stream=st)
        ws = ph.DeviceArray(pl.workspace_size() // 8 + 1)
        out = ph.DeviceArray(w.n_scales * (w.p + 1) * w.N)
        ph.phiks_apply(pl, v.ptr, out.ptr, ws.ptr, ws.nbytes, st)
        ph.synchronize()
        print(json.dumps({"counters": "one step: calibration copy, one plan, one call",
                          "copy_bytes": w.N * 8, "plan": pl.info()}), flush=True)
        pl.close()
        return
    plan = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, stream=st)
    info = plan.info()
    ws = ph.DeviceArray(plan.workspace_size() // 8 + 1)
    out = ph.DeviceArray(w.n_scales * (w.p + 1) * w.N)
    plan.close()
    log(f"[bench] plan {info}, workspace {ws.nbytes / 2**30:.2f} GiB")

    def step(timed=False):
        pl = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, stream=st)
        ph.phiks_kernel_timing(timed)      # events on the call's launches only
        ph.phiks_apply(pl, v.ptr, out.ptr, ws.ptr, ws.nbytes, st)
        ph.phiks_kernel_timing(False)
        pl.close()

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    ph.synchronize()

    # HIP events on every mu-mode launch of the calls of a sample of the timed steps
    # (every tenth and the last): a timestamped dispatch costs about 9 us of idle time
    # after the kernel, so events on every step would slow the steps they measure
    sampled = {i for i in range(args.steps) if i % 10 == 9 or i == args.steps - 1}
    ph.phiks_kernel_timing_read()          # clear
    ph.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i in sampled)
        log(f"[bench] step {i + 1}/{args.steps}")
    ph.synchronize()
    wall = time.perf_counter() - t0
    k_ms, k_launch, k_flops = ph.phiks_kernel_timing_read()
    ms_step = wall * 1e3 / args.steps

    # phi-action call alone with the plan built once (reported beside the step)
    pl = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, stream=st)
    ph.synchronize()
    reps = max(3, args.steps // 2)
    a0 = time.perf_counter()
    for _ in range(reps):
        ph.phiks_apply(pl, v.ptr, out.ptr, ws.ptr, ws.nbytes, st)
    ph.synchronize()
    apply_ms = (time.perf_counter() - a0) * 1e3 / reps
    # per-call distribution: 20 calls, each waited for (adds the synchronisation, tens of us)
    calls = []
    for _ in range(20):
        c0 = time.perf_counter()
        ph.phiks_apply(pl, v.ptr, out.ptr, ws.ptr, ws.nbytes, st)
        ph.synchronize()
        calls.append((time.perf_counter() - c0) * 1e3)
    pl.close()
    # plan build alone (host planner + device exponentials), each waited for
    plans = []
    for _ in range(10):
        c0 = time.perf_counter()
        plx = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, stream=st)
        ph.synchronize()
        plans.append((time.perf_counter() - c0) * 1e3)
        plx.close()
    ph.synchronize()
    # mu-mode flops of one call: T_exec Tucker operators of sum_mu 2 N n_mu each
    call_flops = info["tucker_exec"] * sum(2.0 * w.N * a.shape[0] for a in w.A)

    # the same call with the mu-mode products in FP32 MFMA or BF16x3 (everything else FP64)
    ref64 = out.to_numpy()
    N = w.N

    def mixed(precision, peak):
        plm = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, stream=st,
                            precision=precision)
        ph.phiks_apply(plm, v.ptr, out.ptr, ws.ptr, ws.nbytes, st)
        ph.synchronize()
        # wall time without kernel events, then one call with them for the kernel rate
        b0 = time.perf_counter()
        for _ in range(reps):
            ph.phiks_apply(plm, v.ptr, out.ptr, ws.ptr, ws.nbytes, st)
        ph.synchronize()
        ms = (time.perf_counter() - b0) * 1e3 / reps
        ph.phiks_kernel_timing_read()
        ph.phiks_kernel_timing(True)
        ph.phiks_apply(plm, v.ptr, out.ptr, ws.ptr, ws.nbytes, st)
        ph.synchronize()
        ph.phiks_kernel_timing(False)
        km, _, kf = ph.phiks_kernel_timing_read()
        plm.close()
        got = out.to_numpy()
        err = max(float(np.abs(got[l * N:(l + 1) * N] - ref64[l * N:(l + 1) * N]).max()
                        / np.abs(ref64[l * N:(l + 1) * N]).max()) for l in range(w.p + 1))
        ach = (kf / (km * 1e-3)) / 1e12 if km > 0 else 0.0
        return {"apply_only_ms": ms, "apply_only_dofs_per_s": N / (ms * 1e-3),
                "mu_mode_tflops": ach, "peak_tflops": peak, "frac": ach / peak,
                "max_rel_err_vs_fp64": err}

    fp32 = mixed(ph.PHIKS_FP32, FP32_PEAK_TFLOPS)
    bf16x3 = mixed(ph.PHIKS_BF16X3, BF16_PEAK_TFLOPS / 3)
    # BF16x3 keeps FP32 tensors in HBM: 2 N 4 bytes per product of 2 N n flops
    bf16x3["hbm_gbps_algorithmic"] = bf16x3["mu_mode_tflops"] * 1e3 * 4.0 / w.n[0]
    bf16x3["hbm_frac"] = bf16x3["hbm_gbps_algorithmic"] / HBM_PEAK_GBPS
    bf16x3["note"] = ("peak_tflops is the dense BF16 MFMA peak / 3 (three products per "
                      "FP32 product); mu_mode_tflops counts 2 M N K per product")

    achieved = (k_flops / (k_ms * 1e-3)) / 1e12 if k_ms > 0 else 0.0
    n_mu = w.n[0]
    line = {
        "metric": METRIC,
        "value": w.N / (ms_step * 1e-3),
        "unit": "dofs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"adr3d_{n_mu}^3_phi0-4_same_vector_tau1e-3_fp64",
                   "N": w.N, "p": w.p, "n_scales": w.n_scales, "tol": "2^-53*||v||",
                   "plan": info},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(), "traffic_unit": "bytes per launch",
                     "kernel": "gemm_f64_dl_kernel (mu-mode products of the phi-action "
                               "call; the plan's small n x n GEMMs are not timed)",
                     "launches": k_launch, "timed_steps": len(sampled),
                     "avg_launch_ms": k_ms / max(k_launch, 1),
                     "flops_per_launch": k_flops / max(k_launch, 1)},
        "apply_only_ms": apply_ms,
        "apply_only_dofs_per_s": w.N / (apply_ms * 1e-3),
        "apply_call_ms": {"p10": float(np.percentile(calls, 10)), "p50": float(np.median(calls)),
                          "p90": float(np.percentile(calls, 90)), "calls": len(calls),
                          "note": "each call waited for on the host"},
        "plan_ms": {"p50": float(np.median(plans)), "min": float(min(plans)), "calls": len(plans),
                    "note": "host planner + device small exponentials, waited for"},
        "mu_mode_gflops_per_s": achieved * 1e3,
        "mu_mode_gflops_per_s_of_call": call_flops / (apply_ms * 1e-3) / 1e9,
        "fp32_mfma": fp32,
        "bf16x3_mfma": bf16x3,
    }
    if not args.no_combine:
        line["combine"] = combine_section(ph)
    if not args.no_small:
        log("[bench] 2D 32x32 latency")
        line["small_2d"] = small_2d_section(ph)
    if not args.no_batched:
        log("[bench] batched workload (512 problems)")
        line["batched"] = batched_section(ph)
        line["batched_fp32"] = batched_section(ph, precision=ph.PHIKS_FP32)
    if not args.no_serving:
        log("[bench] serving workload")
        line["serving"] = serving_section(ph)
        line["serving_mixed"] = serving_section(ph, mixed=True)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle (one full call)")
        line["cpu_baseline"] = cpu_baseline(w, info)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
