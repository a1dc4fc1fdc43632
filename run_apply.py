"""Time phiks_apply on the 3D advection-diffusion-reaction workload in one arithmetic.

    python run_apply.py --precision bf16x3 --n 256 --reps 5

Builds the plan once (tau = 1e-3, phi_0..phi_4 of one vector, tolerance 2^-53 ||v||),
then runs one warm-up call, `reps` timed calls of phiks_apply on the null stream and one
more call with kernel events, and prints one JSON line with the plan, the mean call time
and the mu-mode kernel time of the last call.  Meant for profilers
(rocprofv3 --kernel-trace / --pmc): the process launches nothing but the plan's
kernels and the timed calls."""
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
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()

    import paper_2210_07667_amd as ph
    import workloads

    prec = {"fp64": ph.PHIKS_FP64, "fp32": ph.PHIKS_FP32, "bf16x3": ph.PHIKS_BF16X3}[args.precision]
    w = workloads.config_adr_3d(n=args.n)
    v = ph.DeviceArray.from_numpy(w.v)
    plan = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, precision=prec)
    ws = ph.DeviceArray(plan.workspace_size() // 8 + 1)
    out = ph.DeviceArray(w.n_scales * (w.p + 1) * w.N)
    ph.phiks_apply(plan, v.ptr, out.ptr, ws.ptr, ws.nbytes, 0)
    ph.synchronize()
    print(f"[run_apply] {args.precision} n={args.n} plan={plan.info()} warm", flush=True)
    # call time without kernel events (a timestamped dispatch idles the GPU after each
    # launch), then one call with them for the mu-mode kernel time
    t0 = time.perf_counter()
    for i in range(args.reps):
        ph.phiks_apply(plan, v.ptr, out.ptr, ws.ptr, ws.nbytes, 0)
    ph.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.reps
    ph.phiks_kernel_timing_read()
    ph.phiks_kernel_timing(True)
    ph.phiks_apply(plan, v.ptr, out.ptr, ws.ptr, ws.nbytes, 0)
    ph.synchronize()
    ph.phiks_kernel_timing(False)
    k_ms, k_launch, k_flops = ph.phiks_kernel_timing_read()
    print(json.dumps({"precision": args.precision, "n": args.n, "plan": plan.info(),
                      "apply_ms": ms, "mu_mode_ms_per_call": k_ms,
                      "mu_mode_launches_per_call": k_launch,
                      "mu_mode_tflops": k_flops / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0}),
          flush=True)
    plan.close()


if __name__ == "__main__":
    main()
