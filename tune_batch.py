"""Autotuner of the batched path's tile-class rules (phiks_batch_tuning).

    python tune_batch.py [--count 512] [--reps 5] [--write]

Plans the batched workload once (512 problems: d in {2, 3}, n_mu in {16, ..., 128},
Chebyshev D^2, tau log-uniform, phi_0..phi_3, FP64), then for every combination of the
rules -- the side from which 64 x 64 tiles are used (32, 48, 64), the skinny 32 x 128 /
128 x 32 classes (off, on), 128 x 64 tiles for mode-1 plain stores, for plain stores of
modes > 1 and for the squaring epilogue (each off, on) -- runs one eager call, one that
captures the launches and `reps` graph replays, timing the replays, and checks every
output bitwise against the default rules' (any tile class gives the same bits).  Prints
one JSON line per combination and the fastest; --write records the fastest in
paper_2210_07667_amd/csrc/batch_tuning.inc, or the file --out names (rebuild the library
afterwards).
"""
import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2210_07667_amd", "csrc", "batch_tuning.inc"),
                    help="where --write records the fastest rules")
    args = ap.parse_args()
    import paper_2210_07667_amd as ph
    import workloads
    if ph.device_count() < 1:
        print("tune_batch.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    problems = workloads.config_batch(count=args.count)
    norms = [float(np.linalg.norm(b.v)) for b in problems]
    batch = ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems], 3, 1,
                                2.0 ** -53, vnorms=norms)
    dv = [ph.DeviceArray.from_numpy(b.v) for b in problems]
    outs = [ph.DeviceArray(4 * b.N) for b in problems]
    ws = ph.DeviceArray(batch.workspace_size() // 8 + 1)
    vp, op = [x.ptr for x in dv], [o.ptr for o in outs]
    start = ph.batch_tuning()
    ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
    ph.synchronize()
    ref = [o.to_numpy() for o in outs]
    results = []
    for sq_min, skinny, m1, mk, lc in itertools.product((32, 48, 64), (0, 1), (0, 1), (0, 1), (0, 1)):
        rules = {"sq_min": sq_min, "skinny": skinny, "wide_m1": m1, "wide_mk": mk, "wide_lc": lc}
        ph.batch_tuning(rules)
        for _ in range(2):                       # eager, then capture
            ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
        ph.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.reps):
            ph.phiks_batch_apply(batch, vp, op, ws.ptr, ws.nbytes)
        ph.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.reps
        same = all(np.array_equal(o.to_numpy(), r) for o, r in zip(outs, ref))
        results.append({**rules, "ms": ms, "bitwise_equal": same})
        print(json.dumps(results[-1]), flush=True)
        if not same:
            print("outputs differ from the default rules' (must not happen)", file=sys.stderr)
            sys.exit(1)
    ph.batch_tuning(start)
    best = min(results, key=lambda r: r["ms"])
    base = next(r for r in results if all(r[k] == start[k] for k in start))
    print(json.dumps({"best": best, "default": base, "gain": base["ms"] / best["ms"]}), flush=True)
    if args.write:
        path = args.out
        with open(path, "w") as f:
            f.write("// Tile-class rules of the batched path's grouped FP64 launches (BatchTuning in\n"
                    "// batch.hpp), written by tune_batch.py: the fastest of "
                    f"{len(results)} combinations on the\n"
                    f"// batched workload ({args.count} problems), {best['ms']:.2f} ms per call against "
                    f"{base['ms']:.2f} ms with the\n// rules in place before the run.\n"
                    f"constexpr BatchTuning kBatchTuningTuned{{{best['sq_min']}, {best['skinny']}, "
                    f"{best['wide_m1']}, {best['wide_mk']}, {best['wide_lc']}}};\n")
        print(f"wrote {path}", flush=True)
    batch.close()


if __name__ == "__main__":
    main()
