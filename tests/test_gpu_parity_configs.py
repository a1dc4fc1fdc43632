"""GPU parity at the shapes the serving and integrator workloads use, beyond the small
cases of test_gpu_parity.py: 2D grids at the largest mode size (n_mu = 1024, where the
small exponentials dominate the cost and the plans reach s >= 10), a 3D 192^3
request, the Neumann Brusselator-type diffusion operators, one step of the
fourth-order six-stage exponential Runge-Kutta scheme on the 3D Allen-Cahn 64^3
workload, and the small exponentials themselves against the oracle's expm.

Every comparison runs the oracle with the library's (s, q).  Bar for the phi-actions
(relative infinity norm per output): fp64_bar below, 1e-12 except where the squaring
recurrence of a large plan amplifies rounding beyond it; the measured differences are
printed.  Bar for the small exponentials: see exp_bar."""
import math

import numpy as np
import pytest

import workloads
from oracle import expm as oexpm, gll as ogll, integrators as oi, phiks as ophiks

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")
TOL = 1e-12
U = 2.0 ** -53


def fp64_bar(n_max, s):
    """1e-12, or 8 sqrt(n) 2^s u when that is larger.  Both sides form exp(2^-j tau K) by
    squaring exp(tau K / 2^s) s - j times (Section 3.1), and the recurrence of eq.
    simul carries the level-s values through the same s steps.  A relative error e of
    the level-s quantities grows to ~2^s e at level 0 along the slowly decaying modes
    (each squaring doubles it), and one product at size n rounds to ~sqrt(n) u with
    random-sign errors.  So two correct FP64 computations that round differently
    differ by ~sqrt(n) 2^s u; the factor 8 covers the few products per level.  At
    n = 1024, s = 11 that is 5.8e-11; for s <= 8, n <= 256 the 1e-12 bar applies."""
    return max(TOL, 8.0 * math.sqrt(n_max) * 2.0 ** s * U)


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def relerr(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def session(name, p=None):
    """The first serving session with this name (and phi order p, if given): operators,
    tau and p of the serving workload, seed 4."""
    for s in workloads.serving_sessions():
        if s.name == name and (p is None or s.p == p):
            return s
    raise KeyError(name)


def apply_vs_oracle(A, tau, p, ns, v, label):
    print(f"[{label}] tau={tau:.6g} p={p} ns={ns}", flush=True)
    plan = ph.phiks_plan(A, tau, p, ns, 2.0 ** -53, "same_vector")
    out = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(v))
    ph.synchronize()
    info = plan.info()
    plan.close()
    got = out.to_numpy().reshape(ns, p + 1, -1)
    print(f"[{label}] plan {info}; running the oracle", flush=True)
    ref = ophiks.phi_same_vector(A, tau, v, p, ns, info["s"], info["q"])
    errs = [[relerr(got[j, l], ref[j, l]) for l in range(p + 1)] for j in range(ns)]
    bar = fp64_bar(max(a.shape[0] for a in A), info["s"])
    print(f"[{label}] rel errors {np.array(errs).tolist()} (bar {bar:.2e})")
    return info, errs, bar


def test_adr_1024x1024_serving_request():
    """2D ADR 1024^2 (n_mu = PHIKS_MAX_N), phi_0..phi_3, tau of the serving session:
    plan s = 11, q = 11 (44 Tucker operators, two of the serving scales' levels)."""
    ses = session("adr_1024x1024")
    v = workloads.randn_vec(ses.n, 81)
    info, errs, bar = apply_vs_oracle(ses.A, ses.tau, ses.p, 2, v, "adr 1024^2")
    assert info["s"] >= 10
    assert max(max(e) for e in errs) < bar


def test_brusselator_1024x1024_neumann_request():
    """2D Brusselator-type diffusion, Neumann FD2 by ghost reflection (rows 0 and n-1
    (-2, 2)/h^2, nonsymmetric), shift -(b+1) split over the directions; p = 1, s = 12."""
    ses = session("bruss_1024x1024", p=1)
    v = workloads.randn_vec(ses.n, 82)
    info, errs, bar = apply_vs_oracle(ses.A, ses.tau, ses.p, 1, v, "bruss 1024^2")
    assert info["s"] >= 10
    assert max(max(e) for e in errs) < bar


def test_brusselator_192_cubed_request():
    """3D 192^3 serving shape (7.1 M values), Neumann Brusselator-type operator."""
    ses = session("bruss_192x192x192")
    v = workloads.randn_vec(ses.n, 83)
    info, errs, bar = apply_vs_oracle(ses.A, ses.tau, ses.p, 1, v, "bruss 192^3")
    assert bar == TOL
    assert max(max(e) for e in errs) < bar


@pytest.mark.parametrize("tau", [1e-3, 1e-2])
def test_exprk4s6_step_allen_cahn_64(tau):
    """One step of the scheme of eq. expRK4s6 (four phiks_combine calls, stages 3/4 and
    5/6 as the two scales of one combination) on the 3D Allen-Cahn 64^3 workload
    (K = 0.01 FD2 Laplacian, g(u) = u - u^3, u_0 ~ U(-0.9, 0.9) seed 1), GPU driver
    against the oracle driver."""
    from paper_2210_07667_amd import integrators as gi
    w = workloads.config_allen_cahn_3d(tau=tau)
    u0 = w.vs[0]
    print(f"[expRK4s6 allen-cahn 64^3] tau={tau}", flush=True)
    u = gi.exprk4s6(w.A, u0, gi.AllenCahnNonlinearity(u0.size), tau, 1).to_numpy()
    ref = oi.exprk4s6(w.A, u0, lambda t, x: x - x ** 3, tau, 1)
    err = relerr(u, ref)
    print(f"[expRK4s6 allen-cahn 64^3] tau={tau} rel error vs oracle {err:.3e}")
    assert err < TOL


# ------------------------------------------------------------ small exponentials
def exp_bar(n, squarings):
    """Bar for one small exponential against the oracle's, both scaling and squaring
    (degree-24 Taylor on the device, the series to full precision in the oracle): as for
    fp64_bar, each of the t squarings behind a matrix doubles a relative error along
    its slowly decaying modes, and each product at size n rounds to ~sqrt(n) u, so two
    correct computations differ by ~sqrt(n) 2^t u; bar 8 sqrt(n) 2^t u."""
    return 8.0 * math.sqrt(n) * 2.0 ** squarings * U


EXP_CASES = [
    # Chebyshev D^2 of size 128, tau = 1e-2: ||tau A||_1 ~ 1e5, s = 15 (the batched
    # workload's stiffest operators)
    ("cheb 128", lambda: [workloads.cheb_d2_dirichlet(128)] * 2, 1e-2, 3),
    # FD2 Laplacian of size 1024 (n_mu = PHIKS_MAX_N), tau = 1e-3: s = 10
    ("fd2 1024", lambda: [workloads.fd2_dirichlet(1024)] * 2, 1e-3, 3),
    # nonsymmetric ADR operator of size 1024 at the serving session's tau (s = 11)
    ("adr 1024", lambda: session("adr_1024x1024").A, session("adr_1024x1024").tau, 3),
]


@pytest.mark.parametrize("case", range(len(EXP_CASES)), ids=[c[0] for c in EXP_CASES])
def test_small_exponentials_vs_oracle(case):
    """The plan's node matrices exp((1 - theta_i) tau A / 2^s) and levels exp(tau A / 2^j)
    (device degree-24 Taylor + squaring) against the oracle's scaled Taylor series.
    The oracle's levels are squarings of its exp(tau A / 2^s), as the method's are.
    Error: max |G - R| / max |R| per matrix."""
    label, mk, tau, p = EXP_CASES[case]
    A = mk()
    print(f"[expm {label}] tau={tau}", flush=True)
    plan = ph.phiks_plan(A, tau, p, 1, 2.0 ** -53, "same_vector")
    info = plan.info()
    s, q = info["s"], info["q"]
    theta, _ = ogll.gll(q)
    worst = 0.0
    for mu in range(len(A)):
        if mu > 0 and A[mu] is A[0]:
            continue
        B = tau * np.asarray(A[mu])
        n = B.shape[0]
        nrm = float(np.abs(B).sum(axis=0).max())
        for i in sorted({0, (q - 1) // 2, q - 2}):
            R = oexpm.expm_taylor((1.0 - theta[i]) * B / 2.0 ** s)
            G = plan.matrix(mu, ph.PHIKS_MATRIX_NODE, i)
            t = max(0, math.ceil(math.log2(max((1.0 - theta[i]) * nrm / 2.0 ** s, 1e-300) / 0.5)))
            e = relerr(G, R)
            print(f"[expm {label}] mode {mu + 1} node {i}: rel err {e:.3e} (bar {exp_bar(n, t):.1e})")
            worst = max(worst, e / exp_bar(n, t))
        R = oexpm.expm_taylor(B / 2.0 ** s)
        t0 = max(0, math.ceil(math.log2(max(nrm / 2.0 ** s, 1e-300) / 0.5)))
        for j in range(s, -1, -1):
            G = plan.matrix(mu, ph.PHIKS_MATRIX_LEVEL, j)
            sq = t0 + (s - j)
            e = relerr(G, R)
            if j in (s, s // 2, 0):
                print(f"[expm {label}] mode {mu + 1} level {j}: rel err {e:.3e} (bar {exp_bar(n, sq):.1e})")
            worst = max(worst, e / exp_bar(n, sq))
            R = R @ R
    plan.close()
    print(f"[expm {label}] worst error / bar = {worst:.3f}")
    assert worst < 1.0
