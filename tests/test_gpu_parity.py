"""GPU parity: libphiks (HIP, gfx950) against the FP64 CPU oracle.

All calls go through the C ABI (ctypes binding).  Parity is measured with the same
plan (s, q): the library's planner and the oracle's planner are checked to choose
the same (s, q) on the CPU, and here the oracle is run with the plan the library
reports.  Bar: relative infinity-norm difference <= 1e-12 (FP64 path); the error
of one mu-mode product is ~ n eps, and the squaring recurrence multiplies it by at
most ~2^s (s <= 8 here), so 1e-12 leaves a margin above rounding.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import bound, phiks as ophiks, tensor

pytestmark = pytest.mark.gpu

ph = pytest.importorskip("paper_2210_07667_amd")
TOL = 1e-12


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def relerr(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def to_dev(x):
    return ph.DeviceArray.from_numpy(x)


# ----------------------------------------------------------- Tucker operator
TUCKER_SHAPES = [[1], [7], [33], [300], [5, 3], [64, 64], [17, 130], [129, 65], [3, 4, 5],
                 [40, 33, 20], [64, 64, 64], [2, 3, 2, 3], [9, 10, 11, 8], [256, 3, 2],
                 [2, 257, 3], [5, 5, 5, 5, 5]]


@pytest.mark.parametrize("n", TUCKER_SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_tucker_vs_oracle(n):
    print(f"[tucker] n={n}", flush=True)
    rng = np.random.default_rng(sum(n))
    Ls = [rng.standard_normal((k, k)) / math.sqrt(k) for k in n]
    v = rng.standard_normal(int(np.prod(n)))
    out = ph.tucker_arrays(n, [to_dev(L) for L in Ls], to_dev(v))
    ph.synchronize()
    ref = tensor.tucker(v, n, Ls)
    assert relerr(out.to_numpy(), ref) < 1e-13


# ------------------------------------------------------------- phi actions
def run_apply(A, tau, v, p, ns, tol=2.0 ** -53):
    plan = ph.phiks_plan(A, tau, p, ns, tol, "same_vector")
    out = ph.apply_arrays(plan, to_dev(v))
    ph.synchronize()
    info = plan.info()
    plan.close()
    N = int(np.prod([a.shape[0] for a in A]))
    return out.to_numpy().reshape(ns, p + 1, N), info


def run_combine(A, tau, vs, p, ns, tol=2.0 ** -53):
    plan = ph.phiks_plan(A, tau, p, ns, tol, "lincomb")
    out = ph.combine_arrays(plan, [None if x is None else to_dev(x) for x in vs])
    ph.synchronize()
    info = plan.info()
    plan.close()
    N = int(np.prod([a.shape[0] for a in A]))
    return out.to_numpy().reshape(ns, N), info


SV_CASES = [
    ("adr", [6], 0.5, 3, 1),
    ("adr", [5, 4, 3], 2e-2, 4, 2),
    ("adr", [33, 17], 5e-3, 5, 3),
    ("adr", [3, 3, 2, 2], 0.05, 2, 1),
    ("adr", [40, 30, 20], 1e-3, 4, 2),
    ("fd2", [65, 70], 2e-3, 4, 1),
    ("cheb", [24, 20], 1e-3, 3, 1),
    # d = 6 as in the validation of Section 4.1 (real part of its operators)
    ("val", [8, 8, 8, 8, 8, 8], 1.0, 4, 1),
    ("val", [11, 10, 9, 8, 9, 10], 1.0, 3, 2),
    # direct-to-LDS kernel with ragged tiles: every mode has K a multiple of 8 and
    # 128 x 64 or 64 x 128 tiles that overhang both M and N (200 = 128 + 72, 88 = 64 + 24)
    ("adr", [200, 88, 136], 1e-3, 4, 1),
]


def ops(kind, n):
    if kind == "val":
        return [workloads.fd2_dirichlet(k) / 100.0 for k in n]
    if kind == "fd2":
        return [workloads.fd2_dirichlet(k) for k in n]
    if kind == "cheb":
        return [workloads.cheb_d2_dirichlet(k) for k in n]
    betas = [1.0, 0.5, 0.25, 0.125]
    return [workloads.adr_1d(k, 0.5, betas[i], -1.0) for i, k in enumerate(n)]


@pytest.mark.parametrize("kind,n,tau,p,ns", SV_CASES)
def test_apply_vs_oracle(kind, n, tau, p, ns):
    print(f"[apply] {kind} n={n} tau={tau} p={p} ns={ns}", flush=True)
    A = ops(kind, n)
    v = workloads.randn_vec(n, 21)
    got, info = run_apply(A, tau, v, p, ns)
    ref = ophiks.phi_same_vector(A, tau, v, p, ns, info["s"], info["q"])
    for j in range(ns):
        for ell in range(p + 1):
            assert relerr(got[j, ell], ref[j, ell]) < TOL, (j, ell, info)


def test_apply_fd2_32x32_workload():
    """2D FD Laplacian 32x32, tau = 1e-3, phi_0..phi_3, tolerance 2^-53 ||v||."""
    w = workloads.config_fd2_2d()
    got, info = run_apply(w.A, w.tau, w.v, w.p, w.n_scales, w.tol)
    ref = ophiks.phi_same_vector(w.A, w.tau, w.v, w.p, w.n_scales, info["s"], info["q"])
    for ell in range(w.p + 1):
        assert relerr(got[0, ell], ref[0, ell]) < TOL


def test_apply_under_other_planner_options():
    """Planner options (norm-centred rectangle, q in 5..8): the library plans as the
    oracle planner does under the same options, and the action matches the oracle at
    that plan."""
    n, tau, p = [24, 20, 16], 1e-3, 3
    A = ops("cheb", n)
    v = workloads.randn_vec(n, 23)
    tol = 2.0 ** -53 * float(np.linalg.norm(v))
    old = ph.planner_options(5, 8, 64, ph.PHIKS_RECT_NORM_CENTERED)
    try:
        print(f"[apply options] n={n} tau={tau} p={p}", flush=True)
        got, info = run_apply(A, tau, v, p, 1, tol)
    finally:
        ph.planner_options(*old)
    xi = bound.kron_sum_rectangle([tau * a for a in A], "norm_centered")
    s, q, _ = bound.plan(xi, p, 1, tol, "same_vector", q_min=5, q_max=8)
    assert (info["s"], info["q"]) == (s, q)
    ref = ophiks.phi_same_vector(A, tau, v, p, 1, s, q)
    for ell in range(p + 1):
        assert relerr(got[0, ell], ref[0, ell]) < TOL, (ell, info)


def test_apply_exponential_only():
    A = ops("adr", [20, 9, 7])
    v = workloads.randn_vec([20, 9, 7], 22)
    got, info = run_apply(A, 0.02, v, 0, 3)
    ref = ophiks.phi_same_vector(A, 0.02, v, 0, 3, info["s"], info["q"])
    assert info["s"] == 2 and info["q"] == 0
    for j in range(3):
        assert relerr(got[j, 0], ref[j, 0]) < TOL


LC_CASES = [
    ([6], 0.3, 3, 1),
    ([5, 4, 3], 2e-2, 4, 3),
    ([31, 18], 5e-3, 2, 2),
    ([12, 11, 10], 1e-2, 5, 2),
    # p-batched node Tuckers on the direct-to-LDS kernel, ragged 128 x 64 tiles
    ([96, 72, 104], 5e-3, 3, 1),
]


@pytest.mark.parametrize("n,tau,p,ns", LC_CASES)
def test_combine_vs_oracle(n, tau, p, ns):
    print(f"[combine] n={n} tau={tau} p={p} ns={ns}", flush=True)
    A = ops("adr", n)
    rng = np.random.default_rng(23)
    N = int(np.prod(n))
    vs = [rng.standard_normal(N) for _ in range(p + 1)]
    got, info = run_combine(A, tau, vs, p, ns)
    ref = ophiks.phi_lincomb(A, tau, vs, p, ns, info["s"], info["q"])
    for j in range(ns):
        assert relerr(got[j], ref[j]) < TOL, (j, info)


def test_combine_inputs_at_uneven_addresses():
    """Small combinations run the node Tuckers of all inputs in one launch per mode; mode 1
    reads the inputs through one stride when they lie equally far apart, else one launch
    per input.  Both layouts (the inputs placed in one buffer at offsets 0, N, 2N, or 0,
    N + 2, 2N + 10 doubles) must give the same bits, and the oracle's values."""
    n, tau, p, ns = [24, 20, 16], 2e-2, 3, 2
    A = ops("adr", n)
    N = int(np.prod(n))
    rng = np.random.default_rng(36)
    vs = [rng.standard_normal(N) for _ in range(p + 1)]
    plan = ph.phiks_plan(A, tau, p, ns, 2.0 ** -53, "lincomb")
    ws = ph.DeviceArray(plan.workspace_size() // 8 + 1)
    dv = [to_dev(x) for x in vs]
    big = ph.DeviceArray(p * N + 16)
    out = ph.DeviceArray(ns * N)
    results = []
    for offs in ([0, N, 2 * N], [0, N + 2, 2 * N + 10]):
        assert offs[-1] + N <= p * N + 16
        for k, o in enumerate(offs):
            ph.memcpy_dtod(big.ptr + 8 * o, dv[k + 1].ptr, 8 * N)
        ptrs = [dv[0].ptr] + [big.ptr + 8 * o for o in offs]
        ph.phiks_combine(plan, ptrs, out.ptr, ws.ptr, ws.nbytes)
        ph.synchronize()
        results.append(out.to_numpy().reshape(ns, N))
    info = plan.info()
    plan.close()
    for x in dv + [big, out, ws]:
        x.free()
    assert np.array_equal(results[0], results[1])
    ref = ophiks.phi_lincomb(A, tau, vs, p, ns, info["s"], info["q"])
    for j in range(ns):
        assert relerr(results[1][j], ref[j]) < TOL, (j, info)


def test_combine_six_modes():
    """Linear combination with d = 6 (the validation dimension of Section 4.1)."""
    n = [9, 8, 10, 8, 9, 8]
    A = ops("val", n)
    vs = [workloads.randn_vec(n, 60 + k) for k in range(4)]
    print(f"[combine] val n={n}", flush=True)
    got, info = run_combine(A, 1.0, vs, 3, 2)
    ref = ophiks.phi_lincomb(A, 1.0, vs, 3, 2, info["s"], info["q"])
    for j in range(2):
        assert relerr(got[j], ref[j]) < TOL, (j, info)


def test_combine_with_missing_vectors():
    A = ops("adr", [9, 8, 7])
    rng = np.random.default_rng(24)
    vs = [None, rng.standard_normal(504), None, rng.standard_normal(504)]
    got, info = run_combine(A, 0.03, vs, 3, 2)
    ref = ophiks.phi_lincomb(A, 0.03, vs, 3, 2, info["s"], info["q"])
    for j in range(2):
        assert relerr(got[j], ref[j]) < TOL


def test_combine_allen_cahn_64_workload():
    """3D Allen-Cahn 64^3 combination exp(tau K)u0 + sum_l phi_l(tau K) tau g(u0), p = 4,
    two scales, tau = 1e-3 and 1e-2."""
    for tau in (1e-3, 1e-2):
        w = workloads.config_allen_cahn_3d(tau=tau)
        print(f"[combine] allen-cahn 64^3 tau={tau}", flush=True)
        got, info = run_combine(w.A, w.tau, w.vs, w.p, w.n_scales, w.tol)
        ref = ophiks.phi_lincomb(w.A, w.tau, w.vs, w.p, w.n_scales, info["s"], info["q"])
        for j in range(w.n_scales):
            assert relerr(got[j], ref[j]) < TOL, (tau, j, info)


def test_plan_matches_library_planner_and_counts():
    w = workloads.config_adr_3d(n=64)
    s, q, t = ph.phiks_plan_params(w.A, w.tau, w.p, w.n_scales, w.tol, w.task)
    plan = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task)
    info = plan.info()
    plan.close()
    assert (info["s"], info["q"], info["tucker_paper"]) == (s, q, t)
    assert info["tucker_exec"] == (q - 1) + s * w.p + w.n_scales


def test_workspace_too_small_is_rejected():
    A = ops("adr", [8, 8])
    plan = ph.phiks_plan(A, 1e-2, 2, 1, 1e-12)
    v = to_dev(np.ones(64))
    out = ph.DeviceArray(3 * 64)
    ws = ph.DeviceArray(8)
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_apply(plan, v.ptr, out.ptr, ws.ptr, 64)
    assert e.value.status == ph.PHIKS_EWORKSPACE
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_combine(plan, [v.ptr] * 3, out.ptr, ws.ptr, 1 << 20)
    assert e.value.status == ph.PHIKS_EINVAL    # plan made for the same-vector task
    plan.close()


# ------------------------------------------------------- full-size 256^3 case
def test_adr_256_full_size_against_oracle():
    """3D ADR 256^3, phi_0..phi_4 on one vector, tau = 1e-3, tolerance 2^-53 ||v||:
    the whole output against the oracle run with the same (s, q), plus the
    recurrence phi_l = tau K phi_{l+1} + I/l! as an independent property."""
    w = workloads.config_adr_3d()
    print("[apply] adr 256^3 full size", flush=True)
    got, info = run_apply(w.A, w.tau, w.v, w.p, w.n_scales, w.tol)
    print(f"[apply] plan {info}; running oracle", flush=True)
    ref = ophiks.phi_same_vector(w.A, w.tau, w.v, w.p, w.n_scales, info["s"], info["q"])
    for ell in range(w.p + 1):
        assert relerr(got[0, ell], ref[0, ell]) < TOL, ell
    B = [w.tau * a for a in w.A]
    for ell in range(w.p):
        lhs = got[0, ell]
        rhs = tensor.kron_sum_apply(B, got[0, ell + 1]) + w.v / math.factorial(ell)
        assert relerr(lhs, rhs) < 1e-9, ell


def test_adr_256_combination_full_size_against_oracle():
    """phiks_combine on the 3D ADR 256^3 operator, p = 4, five N(0, 1) inputs (the timed
    combination workload): the whole output against the oracle at the same (s, q), and the
    linearity property sum_l phi_l(tau K) v_l = sum of the l-th outputs of same-vector calls
    (a different path through the library: node sums per vector, not per node input)."""
    w = workloads.config_adr_3d()
    p = w.p
    vs = [workloads.randn_vec(w.n, 90 + k) for k in range(p + 1)]
    print("[combine] adr 256^3 full size", flush=True)
    got, info = run_combine(w.A, w.tau, vs, p, 1)
    print(f"[combine] plan {info}; same-vector calls", flush=True)
    lin = np.zeros(w.N)
    for ell in range(p + 1):
        out, _ = run_apply(w.A, w.tau, vs[ell], p, 1)
        lin += out[0, ell]
    print(f"[combine] against the same-vector calls: {relerr(got[0], lin):.2e}", flush=True)
    assert relerr(got[0], lin) < 1e-11
    print("[combine] running oracle", flush=True)
    ref = ophiks.phi_lincomb(w.A, w.tau, vs, p, 1, info["s"], info["q"])
    print(f"[combine] against the oracle: {relerr(got[0], ref[0]):.2e}", flush=True)
    assert relerr(got[0], ref[0]) < TOL, info


@pytest.mark.parametrize("n", [[2, 3, 2, 2, 2, 3, 2, 2], [6, 5, 4, 3, 4, 5, 3, 4]],
                         ids=["d8_tiny", "d8_small"])
def test_largest_d_and_p(n):
    """d = PHIKS_MAX_D = 8 modes and p = PHIKS_MAX_P = 8, three scales, both tasks,
    against the oracle at the library's plan."""
    print(f"[max d,p] n={n}", flush=True)
    betas = [1.0, -0.5, 0.25, 0.75, -1.0, 0.5, -0.25, 0.125]
    A = [workloads.adr_1d(k, 0.5, betas[i], -1.0) for i, k in enumerate(n)]
    tau, p, ns = 0.05, 8, 3
    v = workloads.randn_vec(n, 13)
    got, info = run_apply(A, tau, v, p, ns)
    ref = ophiks.phi_same_vector(A, tau, v, p, ns, info["s"], info["q"])
    for j in range(ns):
        for ell in range(p + 1):
            assert relerr(got[j, ell], ref[j, ell]) < TOL, (j, ell, info)
    rng = np.random.default_rng(14)
    vs = [rng.standard_normal(int(np.prod(n))) for _ in range(p + 1)]
    got, info = run_combine(A, tau, vs, p, ns)
    ref = ophiks.phi_lincomb(A, tau, vs, p, ns, info["s"], info["q"])
    for j in range(ns):
        assert relerr(got[j], ref[j]) < TOL, (j, info)


# ------------------------------------------------------ degenerate problems
from oracle import brute  # noqa: E402  (closed forms of the scalar phi-functions)


def test_zero_operator_and_zero_vector():
    """K = 0: phi_l(0) v = v / l! (the quadrature is exact for these polynomial integrands
    and every exponential is the identity); v = 0: every output exactly zero."""
    n, p, ns = [5, 4, 3], 4, 2
    A = [np.zeros((k, k)) for k in n]
    v = workloads.randn_vec(n, 31)
    got, info = run_apply(A, 1e-2, v, p, ns)
    print(f"[zero K] plan {info}", flush=True)
    for j in range(ns):
        for ell in range(p + 1):
            assert relerr(got[j, ell], v / math.factorial(ell)) < 1e-14, (j, ell)
    B = ops("adr", n)
    got, info = run_apply(B, 2e-2, np.zeros(int(np.prod(n))), p, ns)
    assert not np.any(got), info


def test_scalar_problem_closed_form():
    """d = 1, n = 1: phi_l(tau a) v by its closed form (60-digit evaluation)."""
    for a, tau in [(-3.7, 0.5), (2.0, 0.25), (-150.0, 1e-2)]:
        v = np.array([1.3])
        got, info = run_apply([np.array([[a]])], tau, v, 4, 2)
        for j in range(2):
            z = tau * a * 2.0 ** -j
            for ell in range(5):
                ref = brute.phi_scalar(ell, z).real * 1.3
                assert abs(got[j, ell, 0] - ref) <= 1e-12 * abs(ref), (a, tau, j, ell, info)


def test_diagonal_operators_closed_form():
    """Diagonal A_mu: K is diagonal, so phi_l(tau K) v acts elementwise with the scalar
    closed form at tau (lambda_1 + lambda_2 + lambda_3), including sizes 1 and 128."""
    rng = np.random.default_rng(32)
    n = [7, 1, 128]
    lams = [-rng.uniform(0.0, 300.0, k) for k in n]
    A = [np.diag(l) for l in lams]
    tau, p = 1e-2, 3
    v = workloads.randn_vec(n, 33)
    got, info = run_apply(A, tau, v, p, 1)
    # vec order: index i_1 fastest
    K = (lams[2][:, None, None] + lams[1][None, :, None] + lams[0][None, None, :]).ravel()
    for ell in range(p + 1):
        ref = np.array([brute.phi_scalar(ell, tau * k).real for k in K]) * v
        assert relerr(got[0, ell], ref) < 1e-12, (ell, info)


def test_exponential_of_a_wide_spectrum_operator():
    """exp(tau A) v with p = 0 (so s = 0: the exponential at c = 1) for Chebyshev D^2 (n = 48,
    tau = 0.046): the mean eigenvalue of tau A lies ~740 below the top of its Hermitian part,
    so exp(tau A - (tr/n) I) would exceed the double range although exp(tau A) v is of
    order 1; the shift is capped to keep every intermediate finite.  Bar: the exponential
    takes t ~ log2(||tau A||_1 / 2) = 13 squarings here, each doubling a relative rounding
    error, so two correct FP64 evaluations differ by about 2^t u; 256 2^t u as for the
    batched Chebyshev problems (with t for s)."""
    A = [workloads.cheb_d2_dirichlet(48)]
    tau = 0.046445297112915125
    B = tau * A[0]
    spread = np.linalg.eigvalsh((B + B.T) / 2).max() - np.trace(B) / 48
    assert spread > 709.0                  # the case the cap is for
    t = int(np.ceil(np.log2(np.abs(B).sum(axis=0).max() / 2.0)))
    bar = 256.0 * 2.0 ** t * 2.0 ** -53
    v = workloads.randn_vec([48], 37)
    got, info = run_apply(A, tau, v, 0, 1)
    assert info["s"] == 0, info
    assert np.all(np.isfinite(got))
    ref = ophiks.phi_same_vector(A, tau, v, 0, 1, info["s"], info["q"])
    assert relerr(got[0, 0], ref[0, 0]) < bar
    # and as one mode of a three-mode problem next to advection-diffusion and a dense mode
    rng = np.random.default_rng(38)
    A3 = [workloads.adr_1d(16, 0.5, 1.0, -1.0), workloads.cheb_d2_dirichlet(48),
          rng.standard_normal((12, 12))]
    v3 = workloads.randn_vec([16, 48, 12], 39)
    got, info = run_apply(A3, tau, v3, 0, 1)
    assert np.all(np.isfinite(got))
    ref = ophiks.phi_same_vector(A3, tau, v3, 0, 1, info["s"], info["q"])
    assert relerr(got[0, 0], ref[0, 0]) < bar


def test_size_one_modes_vs_oracle():
    """Modes of size 1 between larger ones (a 1 x 1 A_mu shifts K by its entry)."""
    n = [1, 9, 1, 6]
    A = [np.array([[-0.8]]), workloads.adr_1d(9, 0.5, 1.0, -1.0), np.array([[0.3]]),
         workloads.adr_1d(6, 0.5, -0.5, -1.0)]
    v = workloads.randn_vec(n, 34)
    got, info = run_apply(A, 5e-2, v, 3, 2)
    ref = ophiks.phi_same_vector(A, 5e-2, v, 3, 2, info["s"], info["q"])
    for j in range(2):
        for ell in range(4):
            assert relerr(got[j, ell], ref[j, ell]) < TOL, (j, ell, info)


# ------------------------------------------------------------ two streams
def test_plans_and_calls_pipelined_over_two_streams():
    """Step i's plan built on one stream while step i - 1's call runs on another (the call
    ordered after its plan, the release after the call): every output bitwise equal to the
    same plan and call on the null stream."""
    n = [40, 33, 20]
    A = ops("adr", n)
    v = workloads.randn_vec(n, 35)
    taus = [2e-3, 5e-3, 1e-2, 3e-3]
    p, ns = 3, 2
    ref = [run_apply(A, t, v, p, ns)[0] for t in taus]
    N = int(np.prod(n))
    dv = to_dev(v)
    outs = [ph.DeviceArray(ns * (p + 1) * N) for _ in taus]
    s_plan, s_call = ph.stream_create(), ph.stream_create()
    try:
        mk = lambda t: ph.phiks_plan(A, t, p, ns, 2.0 ** -53, "same_vector", stream=s_plan)
        nxt = mk(taus[0])
        for i in range(len(taus)):
            pl = nxt
            ws = ph.DeviceArray(pl.workspace_size() // 8 + 1)
            ph.stream_order(s_plan, s_call)
            ph.phiks_apply(pl, dv.ptr, outs[i].ptr, ws.ptr, ws.nbytes, s_call)
            if i + 1 < len(taus):
                nxt = mk(taus[i + 1])
            ph.stream_order(s_call, s_plan)
            pl.close()
            ph.stream_synchronize(s_call)
            ws.free()
        ph.stream_synchronize(s_plan)
        for i in range(len(taus)):
            got = outs[i].to_numpy().reshape(ns, p + 1, N)
            assert np.array_equal(got, ref[i]), i
    finally:
        ph.synchronize()
        ph.stream_destroy(s_plan)
        ph.stream_destroy(s_call)
