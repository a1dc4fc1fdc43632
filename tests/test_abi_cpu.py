"""C ABI checks that need no GPU: the library loads, exports every entry point of
include/phiks.h, validates arguments, and its host planning steps (Gauss-Lobatto
rule, rectangle, remainder, (s, q) choice) agree with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads
from oracle import bound, gll

ph = pytest.importorskip("paper_2210_07667_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "phiks.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|double|const char\*)\s+(phiks_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    lib = ctypes.CDLL(ph.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(ph.SYMBOLS)


def test_status_strings():
    for code in range(ph.PHIKS_ETIMEDOUT, 1):
        assert ph.status_string(code) != "unknown status"
    assert ph.status_string(ph.PHIKS_ETIMEDOUT - 1) == "unknown status"


@pytest.mark.parametrize("q", range(2, 13))
def test_gll_matches_oracle(q):
    t1, w1 = ph.phiks_gll(q)
    t2, w2 = gll.gll(q)
    assert np.max(np.abs(np.subtract(t1, t2))) <= 2.3e-16
    assert np.max(np.abs(np.subtract(w1, w2))) <= 2.3e-16


def test_remainder_matches_exact_quadrature_error():
    """Contour integral with the recurrence-evaluated kernel (library) against the
    exact quadrature error computed in high precision (oracle)."""
    rng = np.random.default_rng(0)
    for _ in range(120):
        q = int(rng.integers(3, 13))
        mag = 10 ** rng.uniform(-2.5, 1.6)
        ang = rng.uniform(0, 2 * np.pi)
        w = complex(mag * np.cos(ang), mag * np.sin(ang))
        a = ph.phiks_remainder(q, 5, w)
        b = bound.quad_errors(q, w, 5)
        for x, y in zip(a, b):
            assert abs(x - y) <= 1e-8 * y + 1e-300, (q, w, x, y)


@pytest.mark.parametrize("kind", ["adr", "dense", "cheb"])
def test_rectangle_matches_oracle(kind):
    rng = np.random.default_rng(3)
    B = {"adr": workloads.adr_1d(40, 0.5, 1.0, -1.0),
         "dense": rng.standard_normal((33, 33)),
         "cheb": workloads.cheb_d2_dirichlet(24)}[kind]
    a = np.array(ph.phiks_rectangle(B))
    b = np.array(bound.rectangle(B))
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


CONFIGS = [
    lambda: workloads.config_fd2_2d(),
    lambda: workloads.config_allen_cahn_3d(tau=1e-3),
    lambda: workloads.config_allen_cahn_3d(tau=1e-2),
    lambda: workloads.config_adr_3d(tau=1e-3),
    lambda: workloads.config_adr_3d(tau=1e-4),
]


@pytest.mark.parametrize("make", CONFIGS)
def test_plan_matches_oracle_planner(make):
    w = make()
    got = ph.phiks_plan_params(w.A, w.tau, w.p, w.n_scales, w.tol, w.task)
    xi = bound.kron_sum_rectangle([w.tau * a for a in w.A])
    assert got == tuple(bound.plan(xi, w.p, w.n_scales, w.tol, w.task))


def test_plan_matches_oracle_on_small_sweep():
    rng = np.random.default_rng(4)
    for trial in range(6):
        d = int(rng.integers(1, 4))
        n = [int(rng.integers(2, 9)) for _ in range(d)]
        A = [workloads.adr_1d(k, 0.5, float(rng.uniform(-2, 2)), -1.0) for k in n]
        tau = float(10 ** rng.uniform(-3, -1))
        p = int(rng.integers(1, 6))
        ns = int(rng.integers(1, 4))
        task = "same_vector" if trial % 2 == 0 else "lincomb"
        vn = None
        if trial % 3 == 2:
            vn = [float(x) for x in rng.uniform(0.1, 10, 1 if task == "same_vector" else p + 1)]
        got = ph.phiks_plan_params(A, tau, p, ns, 2.0 ** -53, task, vn)
        xi = bound.kron_sum_rectangle([tau * a for a in A])
        ref = bound.plan(xi, p, ns, 2.0 ** -53, task, vn)
        assert got == tuple(ref), (trial, d, n, tau, p, ns, task)


def test_invalid_arguments_are_rejected():
    A = [workloads.fd2_dirichlet(4)]
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, -1.0, 2, 1, 1e-10)
    assert e.value.status == ph.PHIKS_EINVAL
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, float("nan"), 2, 1, 1e-10)
    assert e.value.status == ph.PHIKS_ENONFINITE
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, 1e-3, 2, 1, 0.0)
    assert e.value.status == ph.PHIKS_EINVAL
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, 1e-3, 99, 1, 1e-10)
    assert e.value.status == ph.PHIKS_EINVAL
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, 1e-3, 2, 0, 1e-10)
    assert e.value.status == ph.PHIKS_EINVAL
    bad = workloads.fd2_dirichlet(4)
    bad[1, 2] = np.inf
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params([bad], 1e-3, 2, 1, 1e-10)
    assert e.value.status == ph.PHIKS_ENONFINITE
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params([np.zeros((2000, 2000))], 1e-3, 2, 1, 1e-10)
    assert e.value.status == ph.PHIKS_EINVAL
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, 1e-3, 2, 1, 1e-10, "lincomb", [1.0, -2.0, 1.0])
    assert e.value.status == ph.PHIKS_EINVAL
    assert ph.phiks_plan_params_raw(0, None, None, 1e-3, 1, 1, 1e-10, 0, None) == ph.PHIKS_EINVAL
    # an unknown arithmetic is rejected before any device work
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan(A, 1e-3, 2, 1, 1e-10, precision=3)
    assert e.value.status == ph.PHIKS_EINVAL


def test_shapes_beyond_32_bit_views_are_rejected():
    """Within the documented limits (n_mu <= 1024, N <= 2^40) but with a mode whose
    leading extent prod(n_<mu) or trailing extent prod(n_>mu) exceeds 2^31 - 1:
    refused with EINVAL before any planning, for real and complex operators and for
    phiks_tucker."""
    n = [2, 1024, 1024, 1024, 2]                  # N / n_1 = 2^31
    A = [np.diag(-np.ones(k)) for k in n]          # finite, cheap rectangles
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, 1e-3, 0, 1, 1e-10)
    assert e.value.status == ph.PHIKS_EINVAL
    Ac = [a.astype(complex) for a in A]
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params_complex(Ac, 1e-3, 0, 1, 1e-10, "same_vector")
    assert e.value.status == ph.PHIKS_EINVAL
    # one size smaller fits: every extent is then 2 * 1024 * 1024 * 1023 < 2^31
    ok = [2, 1024, 1024, 1023, 2]
    s, q, t = ph.phiks_plan_params([np.diag(-np.ones(k)) for k in ok], 1e-3, 0, 1, 1e-10)
    assert t >= 1
    lib = ctypes.CDLL(ph.LIB_PATH)
    lib.phiks_tucker.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    nn = (ctypes.c_int64 * 5)(*n)
    Lp = (ctypes.c_void_p * 5)(*([8] * 5))          # never dereferenced: refused first
    assert lib.phiks_tucker(5, nn, Lp, 8, 8, 8, 1 << 40, None) == ph.PHIKS_EINVAL


def test_unreachable_tolerance_gives_enoplan():
    """A tolerance far below what q <= 12 can reach at any s <= 64."""
    A = [workloads.fd2_dirichlet(8)]
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(A, 1e-2, 3, 1, 1e-300)
    assert e.value.status == ph.PHIKS_ENOPLAN


def test_host_only_calls_on_null_plan():
    lib = ctypes.CDLL(ph.LIB_PATH)
    lib.phiks_plan_info.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
    assert lib.phiks_plan_info(None, None, None, None, None) == ph.PHIKS_EINVAL
    lib.phiks_workspace_size.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.phiks_workspace_size(None, None) == ph.PHIKS_EINVAL
    lib.phiks_apply.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_void_p]
    assert lib.phiks_apply(None, None, None, None, 0, None) == ph.PHIKS_EINVAL
    lib.phiks_plan_destroy.argtypes = [ctypes.c_void_p]
    lib.phiks_plan_destroy(None)


def test_batch_plan_rejects_bad_problems_before_device_work():
    problems = workloads.config_batch(count=6, seed=5)
    taus = [b.tau for b in problems]
    taus[4] = -1.0
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_batch_plan([b.A for b in problems], taus, 3, 1, 1e-10)
    assert e.value.status == ph.PHIKS_EINVAL
    assert "problem 4" in str(e.value)
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems], 3, 1, 1e-10,
                            precision=ph.PHIKS_BF16X3)     # batches run in FP64 or FP32
    assert e.value.status == ph.PHIKS_EINVAL
    with pytest.raises(ValueError):
        ph.phiks_batch_plan([b.A for b in problems], [b.tau for b in problems[:-1]], 3, 1, 1e-10)


def test_batched_workload_shapes():
    """The batched workload has the advertised mix: d in {2, 3}, sizes from the set,
    tau in [1e-4, 1e-2]."""
    problems = workloads.config_batch()
    assert len(problems) == 512
    ds = [len(b.n) for b in problems]
    assert set(ds) == {2, 3} and 200 < ds.count(3) < 312
    assert all(m in workloads.BATCH_SIZES for b in problems for m in b.n)
    assert all(1e-4 <= b.tau <= 1e-2 for b in problems)
    assert all(b.A[0].shape == (b.n[0], b.n[0]) and b.v.shape == (b.N,) for b in problems)


def test_complex_planner_reproduces_table1():
    """The library's complex planner (Bendixson rectangle of complex operators) on the
    validation operators of Section 4.1: every (s, q, T#) of Table 1, both tasks."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    for task in ("same_vector", "lincomb"):
        for d, cols in gold[task].items():
            for n, ref in cols.items():
                A, v = workloads.validation_table1(int(d), int(n))
                nv = float(np.linalg.norm(v))
                vn = [nv] if task == "same_vector" else [nv] * 6
                got = ph.phiks_plan_params_complex(A, 1.0, 5, 2, 2.0 ** -53, task, vn)
                if task == "same_vector":
                    assert got == tuple(ref), (task, d, n, got)
                else:
                    assert got[2] == ref[2], (task, d, n, got)


def test_complex_planner_matches_oracle_on_dense_operators():
    """Dense complex operators and a complex step: library planner == oracle planner."""
    rng = np.random.default_rng(3)
    for trial in range(4):
        n = [int(x) for x in rng.integers(3, 12, size=int(rng.integers(1, 4)))]
        A = [(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) for k in n]
        tau = complex(rng.uniform(0.05, 0.5), rng.uniform(-0.3, 0.3))
        got = ph.phiks_plan_params_complex(A, tau, 3, 1, 2.0 ** -53, "same_vector")
        xi = bound.kron_sum_rectangle([tau * a for a in A])
        ref = bound.plan(xi, 3, 1, 2.0 ** -53, "same_vector")
        assert got == tuple(ref), (trial, n, tau, got, ref)


def test_batch_dryrun_checks_the_512_problem_schedule():
    """The batched launch schedule of the 512-problem workload, built on synthetic device
    addresses by the library itself (phiks_batch_dryrun: every table entry inside its
    problem's buffers, tile bookkeeping, every mu-mode product once, fork plan), with the
    plans the host planner gives; also odd shapes, p = 0 and two scales."""
    probs = workloads.config_batch()
    plans = [ph.phiks_plan_params(b.A, b.tau, 3, 1, 2.0 ** -53, "same_vector",
                                  [float(np.linalg.norm(b.v))])[:2] for b in probs]
    launches, nbytes, bad, why = ph.batch_dryrun([b.n for b in probs], plans, 3, 1, 4)
    print(f"[dryrun] 512 problems: {launches} launches, {nbytes} table bytes")
    assert bad == 0, why
    assert launches > 0 and nbytes > 0
    shapes = [[7], [5, 3], [9, 10, 11], [1, 1], [130, 3, 2], [2, 3, 2, 3, 2]]
    pl = [(2, 5), (1, 3), (4, 12), (1, 4), (3, 7), (2, 9)]
    for p in (0, 1, 4):
        for ns in (1, 2):
            for fk in (0, 1, 4):
                _, _, bad, why = ph.batch_dryrun(shapes, pl, p, ns, fk)
                assert bad == 0, (p, ns, fk, why)
    with pytest.raises(ph.PhiksError):
        ph.batch_dryrun([[7]], [(0, 5)], 2, 2)       # s < n_scales - 1
    with pytest.raises(ph.PhiksError):
        ph.batch_dryrun([[7]], [(1, 2)], 2, 1)       # q below 3


def test_batch_tuning_rules_roundtrip_and_schedules_stay_consistent():
    """The batched path's tile rules (phiks_batch_tuning) can be read and replaced, bad
    values are refused, and the 512-problem schedule passes the dry-run checks under
    other rules too."""
    start = ph.batch_tuning()
    try:
        probs = workloads.config_batch(count=64, seed=9)
        plans = [ph.phiks_plan_params(b.A, b.tau, 3, 1, 2.0 ** -53)[:2] for b in probs]
        for rules in ({"sq_min": 32, "skinny": 0}, {"sq_min": 64, "wide_mk": 1, "wide_lc": 1},
                      {"sq_min": 1, "wide_m1": 0}):
            got = ph.batch_tuning(rules)
            assert all(got[k] == v for k, v in rules.items())
            _, _, bad, why = ph.batch_dryrun([b.n for b in probs], plans, 3, 1, 4)
            assert bad == 0, (rules, why)
        with pytest.raises(ph.PhiksError):
            ph.batch_tuning({"skinny": 2})
        with pytest.raises(ph.PhiksError):
            ph.batch_tuning({"sq_min": 0})
    finally:
        ph.batch_tuning(start)
    assert ph.batch_tuning() == start


DEFAULT_OPTIONS = (3, 12, 64, ph.PHIKS_RECT_BENDIXSON)


@pytest.fixture
def planner_defaults():
    """Tests that change the process-wide planner options put the defaults back."""
    assert ph.planner_options() == DEFAULT_OPTIONS
    yield
    ph.planner_options(*DEFAULT_OPTIONS)
    assert ph.planner_options() == DEFAULT_OPTIONS


@pytest.mark.parametrize("kind", ["adr", "dense", "cheb", "skew"])
def test_norm_centered_rectangle_matches_oracle(kind):
    rng = np.random.default_rng(5)
    B = {"adr": workloads.adr_1d(40, 0.5, 1.0, -1.0),
         "dense": rng.standard_normal((33, 33)),
         "cheb": workloads.cheb_d2_dirichlet(24),
         "skew": np.triu(rng.standard_normal((9, 9)), 1) - np.triu(rng.standard_normal((9, 9)), 1).T}[kind]
    a = np.array(ph.phiks_range_rectangle(B, ph.PHIKS_RECT_NORM_CENTERED))
    b = np.array(bound.rectangle(B, "norm_centered"))
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())
    assert np.allclose(ph.phiks_range_rectangle(B, ph.PHIKS_RECT_BENDIXSON), ph.phiks_rectangle(B))
    with pytest.raises(ph.PhiksError):
        ph.phiks_range_rectangle(B, 7)


def test_planner_options_change_the_plan_as_the_oracle_does(planner_defaults):
    """q range, s limit and rectangle kind: library planner == oracle planner under the
    same options, for real and complex problems."""
    rng = np.random.default_rng(6)
    settings = [(3, 12, 64, "norm_centered"), (5, 9, 64, "bendixson"), (4, 7, 40, "norm_centered")]
    for qmin, qmax, smax, kind in settings:
        rect = ph.PHIKS_RECT_NORM_CENTERED if kind == "norm_centered" else ph.PHIKS_RECT_BENDIXSON
        ph.planner_options(qmin, qmax, smax, rect)
        assert ph.planner_options() == (qmin, qmax, smax, rect)
        for make in (CONFIGS[0], CONFIGS[3]):
            w = make()
            got = ph.phiks_plan_params(w.A, w.tau, w.p, w.n_scales, w.tol, w.task)
            xi = bound.kron_sum_rectangle([w.tau * a for a in w.A], kind)
            ref = bound.plan(xi, w.p, w.n_scales, w.tol, w.task, q_min=qmin, q_max=qmax, s_max=smax)
            assert got == tuple(ref), (qmin, qmax, smax, kind, got, ref)
        n = [5, 7]
        A = [rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)) for k in n]
        tau = complex(0.3, 0.1)
        got = ph.phiks_plan_params_complex(A, tau, 3, 1, 2.0 ** -53, "lincomb")
        xi = bound.kron_sum_rectangle([tau * a for a in A], kind)
        ref = bound.plan(xi, 3, 1, 2.0 ** -53, "lincomb", q_min=qmin, q_max=qmax, s_max=smax)
        assert got == tuple(ref), (qmin, qmax, smax, kind, got, ref)


def test_planner_options_limits_and_errors(planner_defaults):
    w = workloads.config_adr_3d(tau=1e-3)
    s, q, _ = ph.phiks_plan_params(w.A, w.tau, w.p, w.n_scales, w.tol, w.task)
    ph.planner_options(s_max=s - 3)          # the search stops before the chosen s: no plan
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_params(w.A, w.tau, w.p, w.n_scales, w.tol, w.task)
    assert e.value.status == ph.PHIKS_ENOPLAN
    assert f"s <= {s - 3}" in str(e.value)
    for bad in [(2, 12, 64, 0), (6, 5, 64, 0), (3, 13, 64, 0), (3, 12, 65, 0), (3, 12, -1, 0),
                (3, 12, 64, 2)]:
        with pytest.raises(ph.PhiksError) as e:
            ph.planner_options(*bad)
        assert e.value.status == ph.PHIKS_EINVAL
    assert ph.planner_options() == (3, 12, s - 3, ph.PHIKS_RECT_BENDIXSON)   # unchanged


def _options_in_subprocess(env_extra, code):
    import subprocess
    import sys
    env = dict(os.environ, **env_extra)
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, text=True,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=120)


def test_planner_options_from_the_environment():
    code = ("import paper_2210_07667_amd as ph\n"
            "print(ph.planner_options())\n")
    r = _options_in_subprocess({"PHIKS_QMIN": "5", "PHIKS_SMAX": "30",
                                "PHIKS_PLAN_RECT": "normcentered"}, code)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "(5, 12, 30, 1)"
    # an invalid setting keeps the defaults, fails every plan until replaced
    code = ("import paper_2210_07667_amd as ph, workloads\n"
            "w = workloads.config_fd2_2d()\n"
            "for call in (lambda: ph.planner_options(),\n"
            "             lambda: ph.phiks_plan_params(w.A, w.tau, w.p, w.n_scales, w.tol, w.task)):\n"
            "    try:\n"
            "        call()\n"
            "        print('accepted')\n"
            "    except ph.PhiksError as e:\n"
            "        print('refused', e.status)\n"
            "print(ph.planner_options(3, 12, 64, 0))\n"
            "print(ph.phiks_plan_params(w.A, w.tau, w.p, w.n_scales, w.tol, w.task))\n")
    for bad in ({"PHIKS_QMAX": "20"}, {"PHIKS_QMIN": "four"}, {"PHIKS_PLAN_RECT": "circle"}):
        r = _options_in_subprocess(bad, code)
        assert r.returncode == 0, r.stderr
        lines = r.stdout.strip().splitlines()
        assert lines[0] == lines[1] == f"refused {ph.PHIKS_EINVAL}", (bad, lines)
        assert lines[2] == "(3, 12, 64, 0)", (bad, lines)
        ref = ph.phiks_plan_params(*(lambda w: (w.A, w.tau, w.p, w.n_scales, w.tol, w.task))(
            workloads.config_fd2_2d()))
        assert lines[3] == str(tuple(ref)), (bad, lines)
