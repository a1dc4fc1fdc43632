"""GPU checks of the batched entry points (phiks_batch_plan / phiks_batch_apply).

The batch runs every problem's own plan and recurrence; its results must be bitwise
those of phiks_plan + phiks_apply on the problem alone (same (s, q), same GEMM views,
same per-element K order).  The single-problem path is checked against the oracle in
test_gpu_parity.py; here the smaller problems are also checked against the oracle
directly.  Bar for that FP64 comparison: 256 * 2^s * 2^-53.  Scaling and squaring
doubles a relative rounding error at each of the s levels (exp(B/2^j) squared, and
the phi recurrence of eq. simul likewise), so two correct FP64 evaluations that
round differently differ by about 2^s u after s levels; the factor 256 covers the
modes, the up to 12 quadrature nodes and the contraction lengths (n <= 128).  The
Chebyshev operators of this workload are far from normal with tau*||A|| up to 1e5,
so s reaches 14 here."""
import numpy as np
import pytest

import workloads
from oracle import phiks as ophiks

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")
TOL = 2.0 ** -53


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def single(b, p, ns, precision=0):
    plan = ph.phiks_plan(b.A, b.tau, p, ns, TOL, "same_vector", [np.linalg.norm(b.v)],
                         precision=precision)
    out = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(b.v))
    ph.synchronize()
    info = plan.info()
    plan.close()
    return out.to_numpy(), info


def run_batch(problems, p, ns, vs=None, precision=0):
    vs = vs if vs is not None else [b.v for b in problems]
    batch = ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems], p, ns, TOL,
                                vnorms=[np.linalg.norm(v) for v in vs], precision=precision)
    dv = [ph.DeviceArray.from_numpy(v) for v in vs]
    outs = ph.batch_apply_arrays(batch, dv)
    ph.synchronize()
    return batch, [o.to_numpy() for o in outs]


def ragged_problems(seed=11):
    """Odd and even sizes (16-byte loads on and off), d = 1, 2, 3."""
    rng = np.random.default_rng(seed)
    shapes = [[15], [40], [17, 33], [50, 24], [33, 15, 17], [48, 50, 21], [64, 16], [97]]
    out = []
    for k, n in enumerate(shapes):
        A = [workloads.cheb_d2_dirichlet(m) if (k + j) % 2 == 0 else workloads.adr_1d(m, 0.5, 1.0, -1.0)
             for j, m in enumerate(n)]
        tau = float(10 ** rng.uniform(-4, -2))
        out.append(workloads.BatchProblem(n=n, A=A, tau=tau, v=workloads.randn_vec(n, 100 + k)))
    return out


CASES = {
    "batched_workload_24": (lambda: workloads.config_batch(count=24, seed=5), 3, 1),
    "ragged_p2_two_scales": (ragged_problems, 2, 2),
    "exp_only": (lambda: ragged_problems(12)[:5], 0, 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_batch_bitwise_equals_single(name):
    make, p, ns = CASES[name]
    problems = make()
    print(f"[batch] {name}: {len(problems)} problems, N = {[b.N for b in problems]}", flush=True)
    batch, outs = run_batch(problems, p, ns)
    for i, b in enumerate(problems):
        ref, info = single(b, p, ns)
        assert batch.info(i) == info, (i, b.n)
        assert outs[i].shape == ref.shape
        if not np.array_equal(outs[i], ref):
            diff = np.abs(outs[i] - ref).max() / np.abs(ref).max()
            pytest.fail(f"problem {i} n={b.n} differs from the single path (rel {diff:.3e})")
    batch.close()


def test_batch_small_problems_vs_oracle():
    problems = [b for b in workloads.config_batch(count=24, seed=5) if b.N <= 40000][:6]
    assert problems
    batch, outs = run_batch(problems, 3, 1)
    for i, b in enumerate(problems):
        info = batch.info(i)
        ref = ophiks.phi_same_vector(b.A, b.tau, b.v, 3, 1, info["s"], info["q"])
        got = outs[i].reshape(1, 4, -1)
        err = max(float(np.abs(got[0, l] - ref[0, l]).max() / np.abs(ref[0, l]).max())
                  for l in range(4))
        bar = 256 * 2.0 ** info["s"] * 2.0 ** -53
        print(f"[batch vs oracle] n={b.n} tau={b.tau:.2e} plan={info} rel err {err:.2e} "
              f"(bar {bar:.1e})")
        assert err < bar


def test_batch_second_call_new_vectors():
    problems = ragged_problems(13)
    batch, _ = run_batch(problems, 2, 1)
    vs2 = [workloads.randn_vec(b.n, 500 + k) for k, b in enumerate(problems)]
    dv = [ph.DeviceArray.from_numpy(v) for v in vs2]
    outs = [o.to_numpy() for o in ph.batch_apply_arrays(batch, dv)]
    for i, b in enumerate(problems):
        c = workloads.BatchProblem(n=b.n, A=b.A, tau=b.tau, v=vs2[i])
        plan = ph.phiks_plan(c.A, c.tau, 2, 1, TOL, "same_vector", [np.linalg.norm(problems[i].v)])
        ref = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(c.v)).to_numpy()
        plan.close()
        assert np.array_equal(outs[i], ref), i


def test_batch_workspace_too_small():
    problems = ragged_problems(14)[:3]
    batch = ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems], 2, 1, TOL)
    dv = [ph.DeviceArray.from_numpy(b.v) for b in problems]
    outs = [ph.DeviceArray(3 * b.N) for b in problems]
    ws = ph.DeviceArray(max(batch.workspace_size() // 8 - 1, 1))
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_batch_apply(batch, [v.ptr for v in dv], [o.ptr for o in outs], ws.ptr, ws.nbytes)
    assert e.value.status == ph.PHIKS_EWORKSPACE


def test_full_batched_workload_sampled():
    """The 512-problem workload as the benchmark runs it; a sample of problems is
    compared bitwise with the single path."""
    problems = workloads.config_batch()
    batch, outs = run_batch(problems, 3, 1)
    rng = np.random.default_rng(0)
    sample = sorted(set(rng.choice(len(problems), size=8, replace=False).tolist()) |
                    {int(np.argmax([b.N for b in problems]))})
    for i in sample:
        ref, info = single(problems[i], 3, 1)
        assert batch.info(i) == info
        assert np.array_equal(outs[i], ref), (i, problems[i].n)
    print(f"[batch 512] sampled {sample}: bitwise equal")


def test_batch_graph_replays_match_eager():
    """phiks_batch_apply captures its launches into a HIP graph on the second call with
    one pointer set and replays it on later calls.  Every call's outputs (cleared to NaN
    before it, with an unrelated single-problem call and a synchronisation between the
    calls) must be bitwise the first, eager call's; switching to other output pointers
    runs eagerly, and the next call with the first set runs eagerly and the one after it
    captures again."""
    problems = workloads.config_batch(count=24, seed=7)
    p, ns = 3, 1
    norms = [np.linalg.norm(b.v) for b in problems]
    batch = ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems], p, ns, TOL,
                                vnorms=norms)
    dv = [ph.DeviceArray.from_numpy(b.v) for b in problems]
    outs = [ph.DeviceArray(ns * (p + 1) * b.N) for b in problems]
    outs2 = [ph.DeviceArray(ns * (p + 1) * b.N) for b in problems]
    ws = ph.DeviceArray(batch.workspace_size() // 8 + 1)
    nans = [ph.DeviceArray.from_numpy(np.full(o.n, np.nan)) for o in outs]
    ph.batch_apply_arrays(batch, dv, outs, ws)          # first sight of these pointers: eager
    ph.synchronize()
    ref = [o.to_numpy() for o in outs]
    assert all(np.isfinite(r).all() for r in ref)
    b0 = problems[0]
    plan = ph.phiks_plan(b0.A, b0.tau, p, ns, TOL, "same_vector", [norms[0]])
    # calls: 0 capture + launch, 1-2 replays, 3 eager (after the switch), 4 capture, 5 replay
    for call in range(6):
        for o, z in zip(outs, nans):
            ph.copy_device(o, z)
        print(f"[batch graph] call {call}", flush=True)
        ph.batch_apply_arrays(batch, dv, outs, ws)
        ph.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o.to_numpy(), ref[i]), (call, i, problems[i].n)
        ph.apply_arrays(plan, dv[0])                     # eager work between the calls
        ph.synchronize()
        if call == 2:
            ph.batch_apply_arrays(batch, dv, outs2, ws)  # other pointers: eager
            ph.synchronize()
            for i, o in enumerate(outs2):
                assert np.array_equal(o.to_numpy(), ref[i]), ("switch", i)
    plan.close()
    batch.close()


FP32_CASES = {
    "batched_workload_24": (lambda: workloads.config_batch(count=24, seed=5), 3, 1),
    # odd sizes (products launched alone, as their single calls are) and d = 1
    "ragged_p2_two_scales": (ragged_problems, 2, 2),
}


@pytest.mark.parametrize("name", list(FP32_CASES))
def test_fp32_batch_bitwise_equals_single_fp32_calls(name):
    """FP32-MFMA batches: every product of a problem runs, grouped with the other
    problems', in the configuration (tile, load width, kernel) its single FP32 call gives it
    (or alone when no grouped kernel has that configuration), so each problem's outputs are
    bitwise those of phiks_apply with a PHIKS_FP32 plan."""
    make, p, ns = FP32_CASES[name]
    problems = make()
    print(f"[batch fp32] {name}: {len(problems)} problems", flush=True)
    batch, outs = run_batch(problems, p, ns, precision=ph.PHIKS_FP32)
    for i, b in enumerate(problems):
        ref, info = single(b, p, ns, precision=ph.PHIKS_FP32)
        assert batch.info(i) == info
        assert np.array_equal(outs[i], ref), (name, i, b.n)
    batch.close()


def test_fp32_full_batched_workload_sampled_and_against_oracle():
    """The 512-problem workload in FP32: a sample bitwise against single FP32 calls, and
    the smallest sampled problems against the FP64 oracle within the FP32 bar of
    test_gpu_mixed.py (2e-6: the rounding of each level's FP32 products is not amplified
    by the contractive recurrence; measured <= 4.1e-7 up to s = 10)."""
    problems = workloads.config_batch()
    batch, outs = run_batch(problems, 3, 1, precision=ph.PHIKS_FP32)
    rng = np.random.default_rng(1)
    sample = sorted(set(rng.choice(len(problems), size=8, replace=False).tolist()) |
                    {int(np.argmax([b.N for b in problems]))})
    for i in sample:
        ref, info = single(problems[i], 3, 1, precision=ph.PHIKS_FP32)
        assert batch.info(i) == info
        assert np.array_equal(outs[i], ref), (i, problems[i].n)
    small = sorted(sample, key=lambda i: problems[i].N)[:3]
    for i in small:
        b = problems[i]
        info = batch.info(i)
        o = ophiks.phi_same_vector(b.A, b.tau, b.v, 3, 1, info["s"], info["q"])
        got = outs[i].reshape(1, 4, -1)
        err = max(float(np.abs(got[0, l] - o[0, l]).max() / np.abs(o[0, l]).max()) for l in range(4))
        bar = 2e-6
        print(f"[batch fp32] problem {i} n={b.n} s={info['s']}: rel err vs oracle {err:.2e} (bar {bar:.1e})")
        assert err < bar
    batch.close()
