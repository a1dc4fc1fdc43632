"""Pins of the oracle's building blocks against closed forms and library routines.

Each test compares the oracle with something other than itself: textbook values of
the Gauss-Lobatto rule, Kronecker products (Lemma 1, Section 2), scipy's expm,
mpmath quadrature, and exact polynomial integrals.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg

from oracle import bound, expm, gll, tensor


# ---------------------------------------------------------------- GLL (Section 3.3)
def test_gll_q3_q4_q5_closed_forms():
    t, w = gll.gll(3)
    assert np.allclose(t, [0, 0.5, 1], atol=1e-16)
    assert np.allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-16)
    t, w = gll.gll(4)
    r5 = math.sqrt(5.0)
    assert np.allclose(t, [0, (5 - r5) / 10, (5 + r5) / 10, 1], atol=1e-16)
    assert np.allclose(w, [1 / 12, 5 / 12, 5 / 12, 1 / 12], atol=1e-16)
    t, w = gll.gll(5)                       # [-1,1]: 0, +-sqrt(3/7), +-1; 32/45, 49/90, 1/10
    x = math.sqrt(3.0 / 7.0)
    assert np.allclose(t, [0, (1 - x) / 2, 0.5, (1 + x) / 2, 1], atol=1e-16)
    assert np.allclose(w, [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20], atol=1e-16)


@pytest.mark.parametrize("q", range(3, 13))
def test_gll_exact_to_degree_2q_minus_3(q):
    theta, w = gll.gll_mp(q)
    with mp.workdps(50):
        for deg in range(0, 2 * q - 2):
            quad = mp.fsum(wi * ti ** deg for wi, ti in zip(w, theta))
            assert abs(quad - mp.mpf(1) / (deg + 1)) < mp.mpf(10) ** -40
        deg = 2 * q - 2                     # first degree that is not exact
        quad = mp.fsum(wi * ti ** deg for wi, ti in zip(w, theta))
        assert abs(quad - mp.mpf(1) / (deg + 1)) > mp.mpf(10) ** -20
    t = [float(x) for x in theta]
    assert t[0] == 0.0 and abs(t[-1] - 1) < 1e-30 and all(np.diff(t) > 0)


# ---------------------------------------------- mu-mode / Tucker (Section 2, Lemma 1)
@pytest.mark.parametrize("n", [[3], [4, 3], [2, 3, 4], [3, 1, 2, 2]])
def test_tucker_matches_kronecker_product(n):
    rng = np.random.default_rng(1)
    L = [rng.standard_normal((k, k)) for k in n]
    v = rng.standard_normal(int(np.prod(n)))
    M = np.ones((1, 1))
    for Lm in L:                            # L_d x ... x L_1
        M = np.kron(Lm, M)
    assert np.allclose(tensor.tucker(v, n, L), M @ v, rtol=1e-13, atol=1e-13)


def test_mode_product_loops_vs_contraction():
    rng = np.random.default_rng(2)
    n = [3, 4, 2]
    v = rng.standard_normal(24)
    for mu in (1, 2, 3):
        L = rng.standard_normal((n[mu - 1], n[mu - 1]))
        a = tensor.mode_product(tensor.as_tensor(v, n), L, mu).reshape(-1)
        b = tensor.mode_product_loops(v, n, L, mu)
        assert np.allclose(a, b, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n", [[1], [17], [5, 1, 3], [33, 7], [6, 5, 4, 3], [64, 3, 40]])
def test_mode_product_loops_vs_library_contraction(n):
    """The C loops against numpy.tensordot on every mode, real and complex."""
    rng = np.random.default_rng(sum(n))
    v = rng.standard_normal(int(np.prod(n)))
    vc = v + 1j * rng.standard_normal(v.size)
    for mu in range(1, len(n) + 1):
        L = rng.standard_normal((n[mu - 1], n[mu - 1]))
        Lc = L + 1j * rng.standard_normal(L.shape)
        for vv, LL in ((v, L), (vc, L), (v, Lc), (vc, Lc)):
            V = tensor.as_tensor(vv, n)
            a = tensor.mode_product(V, LL, mu)
            b = tensor.mode_product_tensordot(V, LL, mu)
            assert a.shape == V.shape
            assert np.abs(a - b).max() <= 1e-14 * max(np.abs(b).max(), 1.0), (n, mu)


def test_mode_product_loops_exact_on_integers():
    """Small integer entries make every product and partial sum exact in FP64, so the
    loops must equal integer arithmetic bit for bit (index or transpose mistakes show
    as wrong integers)."""
    rng = np.random.default_rng(11)
    n = [5, 3, 4, 2]
    v = rng.integers(-9, 10, int(np.prod(n)))
    for mu in range(1, len(n) + 1):
        L = rng.integers(-9, 10, (n[mu - 1], n[mu - 1]))
        got = tensor.mode_product(tensor.as_tensor(v.astype(float), n), L.astype(float), mu)
        ref = np.zeros(v.size, dtype=np.int64)
        nlo = int(np.prod(n[: mu - 1])) if mu > 1 else 1
        nmu, nhi = n[mu - 1], int(np.prod(n[mu:])) if mu < len(n) else 1
        for b in range(nhi):
            for i in range(nmu):
                for a in range(nlo):
                    ref[a + nlo * (i + nmu * b)] = sum(
                        int(L[i, j]) * int(v[a + nlo * (j + nmu * b)]) for j in range(nmu))
        assert np.array_equal(got.reshape(-1), ref.astype(float)), mu


def test_d2_matrix_form():
    """exp(K) v = vec(exp(A_1) V exp(A_2)^T) for d = 2 (Section 1)."""
    rng = np.random.default_rng(3)
    A1, A2 = rng.standard_normal((4, 4)), rng.standard_normal((3, 3))
    v = rng.standard_normal(12)
    V = v.reshape(3, 4).T                   # column j holds entries j*n1 .. (j+1)*n1-1
    ref = (scipy.linalg.expm(A1) @ V @ scipy.linalg.expm(A2).T).T.reshape(-1)
    got = tensor.tucker(v, [4, 3], [scipy.linalg.expm(A1), scipy.linalg.expm(A2)])
    assert np.allclose(got, ref, rtol=1e-13)
    K = tensor.kron_sum_dense([A1, A2])
    assert np.allclose(scipy.linalg.expm(K) @ v, ref, rtol=1e-12)


def test_kron_sum_apply_matches_dense():
    rng = np.random.default_rng(4)
    A = [rng.standard_normal((k, k)) for k in (3, 2, 4)]
    v = rng.standard_normal(24)
    assert np.allclose(tensor.kron_sum_apply(A, v), tensor.kron_sum_dense(A) @ v)


# ------------------------------------------------------------------- small expm
@pytest.mark.parametrize("seed,scale", [(0, 0.1), (1, 1.0), (2, 7.0), (3, 40.0)])
def test_expm_taylor_vs_scipy(seed, scale):
    rng = np.random.default_rng(seed)
    X = scale * rng.standard_normal((12, 12)) / 4
    ref = scipy.linalg.expm(X)
    got = expm.expm_taylor(X)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12


def test_expm_closed_forms():
    d = np.array([-3.0, 0.5, 2.0, -40.0])
    assert np.allclose(expm.expm_taylor(np.diag(d)), np.diag(np.exp(d)), rtol=1e-14)
    N = np.diag([1.0, 2.0, 3.0], k=1)       # nilpotent: exp = I + N + N^2/2 + N^3/6
    ref = np.eye(4) + N + N @ N / 2 + N @ N @ N / 6
    assert np.allclose(expm.expm_taylor(N), ref, rtol=1e-15, atol=1e-15)
    th = 2.5                                # rotation generator
    R = expm.expm_taylor(np.array([[0.0, -th], [th, 0.0]]))
    assert np.allclose(R, [[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]],
                       atol=1e-15)


def test_expm_with_mpmath_high_precision():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((6, 6)) * 1.5
    with mp.workdps(40):
        ref = mp.expm(mp.matrix(X.tolist()))
        ref = np.array(ref.tolist(), dtype=float)
    assert np.abs(expm.expm_taylor(X) - ref).max() / np.abs(ref).max() < 5e-14


# ------------------------------------------------------- remainder (Section 3.3)
@pytest.mark.parametrize("q,ell,w", [(3, 1, -2.0 + 0.5j), (5, 2, 1.5 - 1j),
                                     (7, 3, -6.0 + 3j), (12, 5, -20 - 4j), (9, 4, 0.3j)])
def test_quad_error_vs_mpmath_quad(q, ell, w):
    theta, wts = gll.gll_mp(q, 60)
    with mp.workdps(60):
        wz = mp.mpc(w.real, w.imag)
        f = lambda t: t ** (ell - 1) / mp.factorial(ell - 1) * mp.exp((1 - t) * wz)
        exact = mp.quad(f, [0, 0.5, 1])
        qs = mp.fsum(wi * f(ti) for wi, ti in zip(wts, theta))
        ref = abs(exact - qs)
    got = bound.quad_errors(q, w, ell)[ell - 1]
    assert abs(got - float(ref)) <= 1e-10 * float(ref)


def test_quad_error_vanishes_for_polynomials_up_to_degree():
    """e^((1-theta) w) -> as w -> 0 the error behaves like |w|^(2q-2-(l-1)) (first
    non-exact power of the Taylor expansion of the integrand)."""
    q, ell = 4, 2
    e1 = bound.quad_errors(q, 1e-2 + 0j, ell)[ell - 1]
    e2 = bound.quad_errors(q, 5e-3 + 0j, ell)[ell - 1]
    order = math.log(e1 / e2) / math.log(2)
    assert abs(order - (2 * q - 2 - (ell - 1))) < 0.05


def test_rectangle_is_tight():
    """Each side of the rectangle is attained by a Rayleigh quotient: the extreme
    eigenvectors of the Hermitian part H = (B + B*)/2 give Re = its edges, those of
    (B - B*)/(2i) give Im = its edges.  For a normal matrix the rectangle is the
    bounding box of the eigenvalues."""
    rng = np.random.default_rng(8)
    B = rng.standard_normal((9, 9)) + 0.4j * rng.standard_normal((9, 9))
    a, b, c, d = bound.rectangle(B)
    H = (B + B.conj().T) / 2
    S = (B - B.conj().T) / 2j
    for M, lo, hi, part in ((H, a, b, np.real), (S, c, d, np.imag)):
        ev, U = np.linalg.eigh(M)
        for x, edge in ((U[:, 0], lo), (U[:, -1], hi)):
            r = (x.conj() @ B @ x) / (x.conj() @ x)
            assert abs(part(r) - edge) <= 1e-12 * max(1.0, abs(edge))
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)))
    lam = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    Nrm = Q @ np.diag(lam) @ Q.conj().T
    box = bound.rectangle(Nrm)
    ref = (lam.real.min(), lam.real.max(), lam.imag.min(), lam.imag.max())
    assert np.allclose(box, ref, atol=1e-12)


def test_rectangle_contains_numerical_range():
    rng = np.random.default_rng(7)
    B = rng.standard_normal((8, 8)) + 0.3j * rng.standard_normal((8, 8))
    a, b, c, d = bound.rectangle(B)
    for _ in range(200):                    # Rayleigh quotients lie in W(B)
        x = rng.standard_normal(8) + 1j * rng.standard_normal(8)
        r = (x.conj() @ B @ x) / (x.conj() @ x)
        assert a - 1e-12 <= r.real <= b + 1e-12 and c - 1e-12 <= r.imag <= d + 1e-12
    ev = np.linalg.eigvals(B)
    assert np.all(ev.real >= a - 1e-12) and np.all(ev.real <= b + 1e-12)


def test_norm_centered_rectangle_closed_forms():
    """Centre tr(B)/n, half-widths ||H - Re(sigma) I||_2 and ||S - Im(sigma) I||_2
    (S = (B - B^H)/(2i)), worked by hand:
    * diag(1, 2, 6): sigma = 3, H - 3I = diag(-2, -1, 3) -> [0, 6] x i[0, 0];
    * diag(0, 0, 3i): sigma = i, H = 0, S = diag(0, 0, 3), S - I = diag(-1, -1, 2)
      -> [0, 0] x i[-1, 3] (the Bendixson box is [0, 0] x i[0, 3]);
    * [[0, 1], [-1, 0]]: sigma = 0, H = 0, S = [[0, -i], [i, 0]] with eigenvalues +-1
      -> [0, 0] x i[-1, 1]."""
    cases = [
        (np.diag([1.0, 2.0, 6.0]), (0.0, 6.0, 0.0, 0.0)),
        (np.diag([0.0, 0.0, 3.0j]), (0.0, 0.0, -1.0, 3.0)),
        (np.array([[0.0, 1.0], [-1.0, 0.0]]), (0.0, 0.0, -1.0, 1.0)),
    ]
    for B, ref in cases:
        assert np.allclose(bound.rectangle(B, "norm_centered"), ref, atol=1e-14), B
    assert np.allclose(bound.rectangle(np.diag([0.0, 0.0, 3.0j])), (0.0, 0.0, 0.0, 3.0),
                       atol=1e-14)


def test_norm_centered_rectangle_contains_bendixson_and_shifts():
    """The norm-centred box contains the Bendixson box (so W(B)), is centred at the mean
    eigenvalue tr(B)/n, and moves with B + c I by c."""
    rng = np.random.default_rng(11)
    for trial in range(6):
        n = 3 + trial
        B = rng.standard_normal((n, n)) + (0.5j * rng.standard_normal((n, n)) if trial % 2 else 0)
        a, b, c, d = bound.rectangle(B)
        A_, B_, C_, D_ = bound.rectangle(B, "norm_centered")
        assert A_ <= a + 1e-12 and B_ >= b - 1e-12 and C_ <= c + 1e-12 and D_ >= d - 1e-12
        mean = np.linalg.eigvals(B).mean()
        assert abs((A_ + B_) / 2 - mean.real) < 1e-12 and abs((C_ + D_) / 2 - mean.imag) < 1e-12
        for _ in range(50):
            x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
            r = (x.conj() @ B @ x) / (x.conj() @ x)
            assert A_ - 1e-12 <= r.real <= B_ + 1e-12 and C_ - 1e-12 <= r.imag <= D_ + 1e-12
        shift = 0.7 - 1.3j
        moved = bound.rectangle(B + shift * np.eye(n), "norm_centered")
        expect = (A_ + shift.real, B_ + shift.real, C_ + shift.imag, D_ + shift.imag)
        assert np.allclose(moved, expect, atol=1e-12)
    try:
        bound.rectangle(np.eye(2), "ellipse")
    except ValueError:
        pass
    else:
        raise AssertionError("unknown kinds are refused")
