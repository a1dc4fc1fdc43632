"""Pins of the oracle's phi-actions and planner.

* Brute force: the augmented-matrix exponential of Section 2 (AMH Theorem 2.1) on
  assembled K, including the 32 x 32 FD Laplacian problem itself.
* The recurrence phi_l(X) = X phi_{l+1}(X) + I/l!.
* Scalar and diagonal closed forms, K = 0, and multi-scale consistency.
* Table 1 of Section 4.1 for the planner.
"""
import json
import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import workloads
from oracle import bound, brute, phiks, tensor

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _plan(A, tau, p, shat, task, tol=2.0 ** -53):
    xi = bound.kron_sum_rectangle([tau * a for a in A])
    s, q, _ = bound.plan(xi, p, shat, tol, task)
    return s, q


CASES = [
    ("adr_543", [5, 4, 3], 2e-2),
    ("adr_6", [6], 0.5),
    ("adr_3322", [3, 3, 2, 2], 0.05),
    ("fd2_77", [7, 7], 1e-2),
]


def _ops(name, n):
    if name.startswith("fd2"):
        return [workloads.fd2_dirichlet(k) for k in n]
    betas = [1.0, 0.5, 0.25, 0.125]
    return [workloads.adr_1d(k, 0.5, betas[i], -1.0) for i, k in enumerate(n)]


@pytest.mark.parametrize("name,n,tau", CASES)
def test_same_vector_vs_augmented(name, n, tau):
    A = _ops(name, n)
    v = workloads.randn_vec(n, 11)
    p, shat = 4, 2
    s, q = _plan(A, tau, p, shat, "same_vector")
    out = phiks.phi_same_vector(A, tau, v, p, shat, s, q)
    for j in range(shat):
        ref = brute.phi_actions_dense(A, tau, v, p, c=2.0 ** -j)
        for ell in range(p + 1):
            assert relerr(out[j, ell], ref[ell]) < 1e-12, (j, ell)


@pytest.mark.parametrize("name,n,tau", CASES)
def test_lincomb_vs_augmented(name, n, tau):
    A = _ops(name, n)
    rng = np.random.default_rng(12)
    p, shat = 4, 3
    N = int(np.prod(n))
    vs = [rng.standard_normal(N) for _ in range(p + 1)]
    s, q = _plan(A, tau, p, shat, "lincomb")
    out = phiks.phi_lincomb(A, tau, vs, p, shat, s, q)
    for j in range(shat):
        assert relerr(out[j], brute.augmented(A, tau, vs, c=2.0 ** -j)) < 1e-12


def test_lincomb_without_exp_term_and_sparse_vectors():
    A = _ops("adr_543", [5, 4, 3])
    rng = np.random.default_rng(13)
    vs = [None, rng.standard_normal(60), None, rng.standard_normal(60)]
    s, q = _plan(A, 3e-2, 3, 1, "lincomb")
    out = phiks.phi_lincomb(A, 3e-2, vs, 3, 1, s, q)
    assert relerr(out[0], brute.augmented(A, 3e-2, vs)) < 1e-12


def test_fd2_32x32_problem_vs_augmented():
    """The 2D 32x32 FD Laplacian workload (tau = 1e-3, phi_0..phi_3) against the
    exponential of the 1027 x 1027 augmented matrix."""
    w = workloads.config_fd2_2d()
    s, q = _plan(w.A, w.tau, w.p, w.n_scales, "same_vector")
    out = phiks.phi_same_vector(w.A, w.tau, w.v, w.p, w.n_scales, s, q)
    ref = brute.phi_actions_dense(w.A, w.tau, w.v, w.p)
    for ell in range(w.p + 1):
        assert relerr(out[0, ell], ref[ell]) < 1e-12


def test_recurrence_residual():
    """phi_l(X) v = X phi_{l+1}(X) v + v/l!  with X = tau K applied by mu-mode products."""
    A = _ops("adr_543", [5, 4, 3])
    tau = 0.04
    v = workloads.randn_vec([5, 4, 3], 14)
    s, q = _plan(A, tau, 5, 1, "same_vector")
    out = phiks.phi_same_vector(A, tau, v, 5, 1, s, q)[0]
    B = [tau * a for a in A]
    for ell in range(0, 5):
        lhs = out[ell]
        rhs = tensor.kron_sum_apply(B, out[ell + 1]) + v / math.factorial(ell)
        assert relerr(lhs, rhs) < 1e-12


@pytest.mark.parametrize("z", [-3.0, 0.7, -40.0, 1e-3])
def test_scalar_closed_form(z):
    """d = 1, n = 1: phi_l(z) v from (e^z - sum_{k<l} z^k/k!)/z^l."""
    A = [np.array([[z]])]
    v = np.array([1.7])
    s, q = _plan(A, 1.0, 5, 1, "same_vector")
    out = phiks.phi_same_vector(A, 1.0, v, 5, 1, s, q)[0]
    for ell in range(6):
        ref = brute.phi_scalar(ell, z) * 1.7
        assert abs(out[ell][0] - ref) <= 1e-13 * abs(ref)


def test_diagonal_operators_closed_form():
    d1, d2 = np.array([-5.0, -1.0, 0.5]), np.array([-2.0, 0.25])
    A = [np.diag(d1), np.diag(d2)]
    v = workloads.randn_vec([3, 2], 15)
    s, q = _plan(A, 1.0, 3, 1, "same_vector")
    out = phiks.phi_same_vector(A, 1.0, v, 3, 1, s, q)[0]
    lam = np.add.outer(d2, d1).reshape(-1)      # eigenvalue of K at vec index
    for ell in range(4):
        ref = np.array([brute.phi_scalar(ell, z) for z in lam]).real * v
        assert relerr(out[ell], ref) < 1e-13


def test_zero_operator_gives_v_over_factorial():
    A = [np.zeros((3, 3)), np.zeros((2, 2))]
    v = workloads.randn_vec([3, 2], 16)
    out = phiks.phi_same_vector(A, 1.0, v, 4, 1, 0, 3)[0]
    for ell in range(5):
        assert relerr(out[ell], v / math.factorial(ell)) < 1e-15


def test_scales_agree_with_fresh_calls():
    """Output at scale j equals a fresh computation with tau / 2^j (eq. scaldiffphi)."""
    A = _ops("adr_543", [5, 4, 3])
    tau = 0.08
    v = workloads.randn_vec([5, 4, 3], 17)
    s, q = _plan(A, tau, 3, 3, "same_vector")
    multi = phiks.phi_same_vector(A, tau, v, 3, 3, s, q)
    for j in range(1, 3):
        s2, q2 = _plan(A, tau / 2 ** j, 3, 1, "same_vector")
        one = phiks.phi_same_vector(A, tau / 2 ** j, v, 3, 1, s2, q2)[0]
        assert relerr(multi[j], one) < 1e-12


def test_squaring_block_identity_p2():
    """Section 3.2: exp(2^-j [[K, v2, v1], [0, 0, 1], [0, 0, 0]]) has blocks
    Phi_j(K) v_2 and Phi_j(K) v_{1,2}; one squaring step maps level j to j-1."""
    rng = np.random.default_rng(18)
    A = [rng.standard_normal((3, 3)) * 0.5, rng.standard_normal((2, 2)) * 0.5]
    K = tensor.kron_sum_dense(A)
    v1, v2 = rng.standard_normal(6), rng.standard_normal(6)
    import scipy.linalg
    def blocks(j):
        M = np.zeros((8, 8))
        M[:6, :6] = K
        M[:6, 6], M[:6, 7], M[6, 7] = v2, v1, 1.0
        E = scipy.linalg.expm(M / 2.0 ** j)
        return E[:6, :6], E[:6, 6], E[:6, 7]
    for j in (1, 2, 3):
        Ej, q1, q2 = blocks(j)           # Q_1 = Phi_j v_2, Q_2 = Phi_j v_{1,2}
        _, r1, r2 = blocks(j - 1)
        assert relerr(Ej @ q1 + q1, r1) < 1e-13
        assert relerr(Ej @ q2 + q1 / 2.0 ** j + q2, r2) < 1e-13


# --------------------------------------------------------- planner vs Table 1
def _table1_case(args):
    task, d, n = args
    A, v = workloads.validation_table1(d, n)
    xi = bound.kron_sum_rectangle(A)
    nv = float(np.linalg.norm(v))
    vn = [nv] if task == "same_vector" else [nv] * 6
    return bound.plan(xi, 5, 2, 2.0 ** -53, task, vn)


def test_planner_reproduces_table1():
    """Same vector: (s, q, T#) of every column of Table 1.  Linear combination: T# of
    every column (the paper's s within a run of equal T# is not reproduced: its
    choice there depends on rounding in its own bound evaluation)."""
    gold = json.load(open(os.path.join(GOLD, "table1.json")))
    jobs = [(task, int(d), int(n)) for task in ("same_vector", "lincomb")
            for d in gold[task] for n in gold[task][d]]
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        got = list(ex.map(_table1_case, jobs))
    for (task, d, n), (s, q, T) in zip(jobs, got):
        ref = gold[task][str(d)][str(n)]
        if task == "same_vector":
            assert (s, q, T) == tuple(ref), (task, d, n)
        else:
            assert T == ref[2], (task, d, n)


def test_largest_d_and_p_vs_augmented():
    """The largest shapes the interface admits in d and p (d = 8 modes, p = 8, three
    scales), both tasks, against the augmented-matrix exponential (N + p = 584)."""
    n = [2, 3, 2, 2, 2, 3, 2, 2]
    betas = [1.0, -0.5, 0.25, 0.75, -1.0, 0.5, -0.25, 0.125]
    A = [workloads.adr_1d(k, 0.5, betas[i], -1.0) for i, k in enumerate(n)]
    tau, p, shat = 0.05, 8, 3
    v = workloads.randn_vec(n, 13)
    s, q = _plan(A, tau, p, shat, "same_vector")
    out = phiks.phi_same_vector(A, tau, v, p, shat, s, q)
    for j in range(shat):
        ref = brute.phi_actions_dense(A, tau, v, p, c=2.0 ** -j)
        for ell in range(p + 1):
            assert relerr(out[j, ell], ref[ell]) < 1e-12, (j, ell)
    rng = np.random.default_rng(14)
    vs = [rng.standard_normal(int(np.prod(n))) for _ in range(p + 1)]
    s, q = _plan(A, tau, p, shat, "lincomb")
    out = phiks.phi_lincomb(A, tau, vs, p, shat, s, q)
    for j in range(shat):
        assert relerr(out[j], brute.augmented(A, tau, vs, c=2.0 ** -j)) < 1e-12, j
