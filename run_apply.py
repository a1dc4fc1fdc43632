"""Time one phi-action call (phiks_apply or phiks_combine) in one arithmetic.

    python run_apply.py --precision bf16x3 --n 256 --reps 5
    python run_apply.py --task lincomb --reps 3
    python run_apply.py --workload allen_cahn --task lincomb --tau 1e-2 --reps 10

Workloads: the 3D advection-diffusion-reaction operator at n^3 (tau = 1e-3, p = 4, one
scale; same vector: phi_0..phi_4 of one N(0, 1) vector; linear combination: five N(0, 1)
vectors v_0..v_4) or the 3D Allen-Cahn 64^3 combination (p = 4, two scales, its u_0 and
tau g(u_0) as inputs).  Tolerance 2^-53 ||v||.  Builds the plan once, then runs one
warm-up call, `reps` timed calls on the null stream and one more call with kernel
events, and prints one JSON line with the plan, the mean call time and the mu-mode
kernel time of the last call.  Meant for profilers (rocprofv3 --kernel-trace / --pmc):
the process launches nothing but the plan's kernels and the calls."""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default="fp64")
    ap.add_argument("--task", choices=["same_vector", "lincomb"], default="same_vector")
    ap.add_argument("--workload", choices=["adr", "allen_cahn"], default="adr")
    ap.add_argument("--n", type=int, default=256, help="n per mode of the ADR workload")
    ap.add_argument("--tau", type=float, default=1e-3)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    if args.workload == "allen_cahn" and args.task != "lincomb":
        ap.error("the Allen-Cahn workload is a linear combination (--task lincomb)")

    import paper_2210_07667_amd as ph
    import workloads

    prec = {"fp64": ph.PHIKS_FP64, "fp32": ph.PHIKS_FP32, "bf16x3": ph.PHIKS_BF16X3}[args.precision]
    if args.workload == "adr":
        w = workloads.config_adr_3d(n=args.n, tau=args.tau)
        vs = [w.v] if args.task == "same_vector" else [workloads.randn_vec(w.n, 90 + k)
                                                       for k in range(w.p + 1)]
        ns = w.n_scales
    else:
        w = workloads.config_allen_cahn_3d(tau=args.tau)
        vs, ns = w.vs, w.n_scales
    plan = ph.phiks_plan(w.A, w.tau, w.p, ns, w.tol, args.task, precision=prec)
    dv = [ph.DeviceArray.from_numpy(x) for x in vs]
    ws = ph.DeviceArray(plan.workspace_size() // 8 + 1)
    if args.task == "same_vector":
        out = ph.DeviceArray(ns * (w.p + 1) * w.N)

        def call():
            ph.phiks_apply(plan, dv[0].ptr, out.ptr, ws.ptr, ws.nbytes, 0)
    else:
        out = ph.DeviceArray(ns * w.N)
        ptrs = [x.ptr for x in dv]

        def call():
            ph.phiks_combine(plan, ptrs, out.ptr, ws.ptr, ws.nbytes, 0)
    call()
    ph.synchronize()
    print(f"[run_apply] {args.precision} {args.workload} {args.task} n={w.n} plan={plan.info()} warm",
          flush=True)
    # call time without kernel events (a timestamped dispatch idles the GPU after each
    # launch), then one call with them for the mu-mode kernel time
    t0 = time.perf_counter()
    for i in range(args.reps):
        call()
    ph.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.reps
    ph.phiks_kernel_timing_read()
    ph.phiks_kernel_timing(True)
    call()
    ph.synchronize()
    ph.phiks_kernel_timing(False)
    k_ms, k_launch, k_flops = ph.phiks_kernel_timing_read()
    print(json.dumps({"precision": args.precision, "workload": args.workload, "task": args.task,
                      "n": w.n, "tau": w.tau, "n_scales": ns, "plan": plan.info(),
                      "call_ms": ms, "mu_mode_ms_per_call": k_ms,
                      "mu_mode_launches_per_call": k_launch,
                      "mu_mode_tflops": k_flops / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0}),
          flush=True)
    plan.close()


if __name__ == "__main__":
    main()
