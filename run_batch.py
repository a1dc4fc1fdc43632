"""Time phiks_batch_apply on the batched workload (512 uneven problems).

    python run_batch.py --count 512 --reps 3 [--precision fp32]

Plans the batch once (d in {2, 3}, n_mu in 16..128, Chebyshev second-derivative
operators, tau log-uniform in [1e-4, 1e-2], phi_0..phi_3 of one vector, tolerance
2^-53 ||v||), then runs two warm-up calls (eager, then captured into a graph), `reps` timed
calls of phiks_batch_apply on the null stream (graph replays) and one more call with kernel
events (eager), and prints one JSON line with the call
time and the mu-mode kernel time of the last call.  Meant for profilers
(rocprofv3 --kernel-trace / --pmc): the process launches nothing but the plan's
kernels and the timed calls."""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    args = ap.parse_args()

    import paper_2210_07667_amd as ph
    import workloads

    problems = workloads.config_batch(count=args.count)
    norms = [float(np.linalg.norm(b.v)) for b in problems]
    prec = ph.PHIKS_FP32 if args.precision == "fp32" else ph.PHIKS_FP64
    batch = ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems], 3, 1,
                                2.0 ** -53, vnorms=norms, precision=prec)
    dv = [ph.DeviceArray.from_numpy(b.v) for b in problems]
    outs = [ph.DeviceArray(4 * b.N) for b in problems]
    ws = ph.DeviceArray(batch.workspace_size() // 8 + 1)
    vp, op = [v.ptr for v in dv], [o.ptr for o in outs]
    for _ in range(2):   # eager, then captured into the graph the timed calls replay
        ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
    ph.synchronize()
    print(f"[run_batch] {len(problems)} problems warm", flush=True)
    # call time without kernel events (a timestamped dispatch idles the GPU after each
    # launch), then one call with them for the mu-mode kernel time
    t0 = time.perf_counter()
    for _ in range(args.reps):
        ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
    ph.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.reps
    ph.phiks_kernel_timing_read()
    ph.phiks_kernel_timing(True)
    ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
    ph.synchronize()
    ph.phiks_kernel_timing(False)
    k_ms, k_launch, k_flops = ph.phiks_kernel_timing_read()
    print(json.dumps({"problems": len(problems), "precision": args.precision,
                      "total_dofs": sum(b.N for b in problems),
                      "apply_ms": ms, "mu_mode_ms_per_call": k_ms,
                      "mu_mode_launches_per_call": k_launch,
                      "mu_mode_tflops": k_flops / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0}),
          flush=True)
    batch.close()


if __name__ == "__main__":
    main()
