"""Exponential integrators on the oracle's phi-actions (test infrastructure only).

exp_euler: the exponential Euler scheme in its linear-combination form (eq. expEullc),
    u_{n+1} = exp(tau K) u_n + phi_1(tau K) (tau g(t_n, u_n)).
etd2rk: the second-order exponential Runge-Kutta scheme in its linear-combination form
    (eq. ETD2RKlc),
    u_{n2}  = exp(tau K) u_n + phi_1(tau K) (tau g_n),
    u_{n+1} = exp(tau K) u_n + phi_1(tau K) (tau g_n) + phi_2(tau K) (tau (g(t_{n+1}, u_{n2}) - g_n)).
Every step is one or two calls of phi_lincomb (Section 3.2); the plan (s, q) of each
call shape is chosen once per step size with the tolerance read relative (vector
norms taken as 1), since the operator and tau do not change between steps.
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np

from . import bound
from .phiks import phi_lincomb, phi_same_vector


def _plan(A: Sequence[np.ndarray], tau: float, p: int, tol: float):
    xi = bound.kron_sum_rectangle([tau * np.asarray(a) for a in A])
    s, q, _ = bound.plan(xi, p, 1, tol, "lincomb")
    return s, q


def exp_euler(A, u0: np.ndarray, g: Callable[[float, np.ndarray], np.ndarray], T: float,
              steps: int, tol: float = 2.0 ** -53) -> np.ndarray:
    tau = T / steps
    s, q = _plan(A, tau, 1, tol)
    u = np.asarray(u0, dtype=np.float64).copy()
    for n in range(steps):
        t = n * tau
        u = phi_lincomb(A, tau, [u, tau * g(t, u)], 1, 1, s, q)[0]
    return u


def etd2rk(A, u0: np.ndarray, g: Callable[[float, np.ndarray], np.ndarray], T: float,
           steps: int, tol: float = 2.0 ** -53) -> np.ndarray:
    tau = T / steps
    s1, q1 = _plan(A, tau, 1, tol)
    s2, q2 = _plan(A, tau, 2, tol)
    u = np.asarray(u0, dtype=np.float64).copy()
    for n in range(steps):
        t = n * tau
        gn = g(t, u)
        u2 = phi_lincomb(A, tau, [u, tau * gn], 1, 1, s1, q1)[0]
        u = phi_lincomb(A, tau, [u, tau * gn, tau * (g(t + tau, u2) - gn)], 2, 1, s2, q2)[0]
    return u


def adr_nonlinearity(prob):
    """g(t, u) = 1/(1 + u^2) + Psi(t) of the ADR problem of Section 4.2."""
    def g(t, u):
        et = math.exp(t)
        return 1.0 / (1.0 + u * u) + et * prob.w - 1.0 / (1.0 + (et * prob.u0) ** 2)
    return g


def exprk3s3(A, u0: np.ndarray, g: Callable[[float, np.ndarray], np.ndarray], T: float,
             steps: int, tol: float = 2.0 ** -53) -> np.ndarray:
    """Third-order exponential Runge-Kutta scheme with the reduced tableau of eq.
    expRK3s3: c_3 = 2 c_2 = 1/2, gamma = (3c_3 - 2) c_3 / ((2 - 3c_2) c_2) = -4/5.
      U_2     = e^(c_2 tau K) u_n + c_2 tau phi_1(c_2 tau K) g_n
      U_3     = e^(c_3 tau K) u_n + c_3 tau phi_1(c_3 tau K) g_n
                + tau (gamma c_2 phi_2(c_2 tau K) + c_3^2/c_2 phi_2(c_3 tau K)) D_2
      u_{n+1} = e^(tau K) u_n + tau phi_1(tau K) g_n
                + tau phi_2(tau K) (gamma D_2 + D_3) / (gamma c_2 + c_3),
    D_j = g(t_n + c_j tau, U_j) - g_n.  A call of phi_lincomb with step h returns
    e^(hK) v_0 + sum_l phi_l(hK) v_l, so every argument v_l carries its own h^l."""
    c2, c3 = 0.25, 0.5
    gam = (3 * c3 - 2) * c3 / ((2 - 3 * c2) * c2)
    tau = T / steps
    plans = {}

    def lc(h, vs, p):
        if (h, p) not in plans:
            plans[(h, p)] = _plan(A, h, p, tol)
        s, q = plans[(h, p)]
        return phi_lincomb(A, h, vs, p, 1, s, q)[0]

    u = np.asarray(u0, dtype=np.float64).copy()
    for n in range(steps):
        t = n * tau
        gn = g(t, u)
        U2 = lc(c2 * tau, [u, c2 * tau * gn], 1)
        D2 = g(t + c2 * tau, U2) - gn
        # phi_2 at two times: the c_3 part joins stage 3's combination, the c_2 part
        # is a second combination without exponential term
        U3 = lc(c3 * tau, [u, c3 * tau * gn, tau * (c3 ** 2 / c2) * D2], 2)
        U3 = U3 + lc(c2 * tau, [None, None, tau * gam * c2 * D2], 2)
        D3 = g(t + c3 * tau, U3) - gn
        u = lc(tau, [u, tau * gn, tau * (gam * D2 + D3) / (gam * c2 + c3)], 2)
    return u


def exprk4s6(A, u0: np.ndarray, g: Callable[[float, np.ndarray], np.ndarray], T: float,
             steps: int, tol: float = 2.0 ** -53) -> np.ndarray:
    return exprk4s6_blocks([A], u0, g, T, steps, tol)


def exprk4s6_blocks(blocks, u0: np.ndarray, g: Callable[[float, np.ndarray], np.ndarray],
                    T: float, steps: int, tol: float = 2.0 ** -53) -> np.ndarray:
    """Fourth-order six-stage exponential Runge-Kutta scheme with the reduced tableau of
    eq. expRK4s6, c = (c_2, c_3, c_4, c_5, c_6) = (1/3, 1/3, 2/3, 1/2, 1): stages 3
    and 4 come from one two-scale linear combination with step c_4 tau (c_3 = c_4/2 is
    its half-step output, eq. scallincomb), stages 5 and 6 from one with step tau.
      U_i     = e^(c_i tau K) u_n + c_i tau phi_1(c_i tau K) g_n + tau sum_j a_ij D_j
      u_{n+1} = e^(tau K) u_n + tau phi_1(tau K) g_n + tau (b_5 D_5 + b_6 D_6),
    with a_32 = c_3^2/c_2 phi_{2,3}, a_42 = c_4^2/c_2 phi_{2,4} and a_{5,3}, a_{5,4},
    a_{6,3}, a_{6,4}, b_5, b_6 as in the tableau.  K may be block diagonal (blocks[b]:
    the A_mu of block b, u the concatenated state; exprk4s6 is the one-block case)."""
    c2, c3, c4, c5, c6 = 1 / 3, 1 / 3, 2 / 3, 0.5, 1.0
    tau = T / steps
    plans = {}

    def lc(h, vs, p, ns):
        return _lc_blocks(blocks, plans, h, vs, p, ns, tol)

    u = np.asarray(u0, dtype=np.float64).copy()
    for n in range(steps):
        t = n * tau
        gn = g(t, u)
        U2 = lc(c2 * tau, [u, c2 * tau * gn], 1, 1)[0]
        D2 = g(t + c2 * tau, U2) - gn
        # step h = c_4 tau: output 0 is stage 4, output 1 (h/2 = c_3 tau) stage 3
        h = c4 * tau
        o = lc(h, [u, h * gn, tau * (c4 ** 2 / c2) * D2], 2, 2)
        U4, U3 = o[0], o[1]
        D3 = g(t + c3 * tau, U3) - gn
        D4 = g(t + c4 * tau, U4) - gn
        # step h = c_6 tau = tau: output 0 is stage 6, output 1 (c_5 = 1/2) stage 5
        v2 = tau * (c4 * c6 ** 2 / (c3 * (c4 - c3)) * D3 + c3 * c6 ** 2 / (c4 * (c3 - c4)) * D4)
        v3 = tau * (2 * c6 ** 3 / (c3 * (c3 - c4)) * D3 + 2 * c6 ** 3 / (c4 * (c4 - c3)) * D4)
        o = lc(tau, [u, tau * gn, v2, v3], 3, 2)
        U6, U5 = o[0], o[1]
        D5 = g(t + c5 * tau, U5) - gn
        D6 = g(t + c6 * tau, U6) - gn
        w2 = tau * (c6 / (c5 * (c6 - c5)) * D5 + c5 / (c6 * (c5 - c6)) * D6)
        w3 = tau * (2 / (c5 * (c5 - c6)) * D5 + 2 / (c6 * (c6 - c5)) * D6)
        u = lc(tau, [u, tau * gn, w2, w3], 3, 1)[0]
    return u


# ----------------------------------------------- block-diagonal operators (two species)
def _blocks_split(blocks, w):
    """Views of the concatenated state w per block (block b: prod of its n_mu values)."""
    out, off = [], 0
    for A in blocks:
        N = int(np.prod([a.shape[0] for a in A]))
        out.append(w[off:off + N])
        off += N
    return out


def _lc_blocks(blocks, plans, h, vs, p, ns, tol):
    """phi_lincomb on every diagonal block of K = diag(K_1, K_2, ...) (Section 4.4: the
    actions of a block-diagonal operator are those of its blocks); vs are concatenated
    vectors or None.  Returns an (ns, N) array."""
    parts = [_blocks_split(blocks, v) if v is not None else [None] * len(blocks) for v in vs]
    res = []
    for b, A in enumerate(blocks):
        key = ("lc", b, h, p, ns)
        if key not in plans:
            xi = bound.kron_sum_rectangle([h * np.asarray(a) for a in A])
            s, q, _ = bound.plan(xi, p, ns, tol, "lincomb")
            plans[key] = (s, q)
        s, q = plans[key]
        res.append(phi_lincomb(A, h, [parts[k][b] for k in range(p + 1)], p, ns, s, q))
    return np.concatenate(res, axis=1)


def _sv_blocks(blocks, plans, h, v, p, ns, tol):
    """phi_same_vector on every diagonal block; returns an (ns, p + 1, N) array."""
    res = []
    for b, (A, x) in enumerate(zip(blocks, _blocks_split(blocks, v))):
        key = ("sv", b, h, p, ns)
        if key not in plans:
            xi = bound.kron_sum_rectangle([h * np.asarray(a) for a in A])
            s, q, _ = bound.plan(xi, p, ns, tol, "same_vector")
            plans[key] = (s, q)
        s, q = plans[key]
        res.append(phi_same_vector(A, h, x, p, ns, s, q))
    return np.concatenate(res, axis=2)


def exprk4s5(blocks, w0: np.ndarray, g: Callable[[float, np.ndarray], np.ndarray], T: float,
             steps: int, tol: float = 2.0 ** -53, smart: bool = False) -> np.ndarray:
    """Fourth-order five-stage exponential Runge-Kutta scheme of the reduced tableau of
    eq. expRK4s5 (c = (1/2, 1/2, 1, 1/2)), for w' = K w + g(t, w) with K block diagonal:
    blocks[b] is the list of A_mu of block b's Kronecker sum, w the concatenated state.
    With D_j = g(t_n + c_j tau, U_j) - g_n and phi_{k,j} = phi_k(c_j tau K):
      U_2 = e^(tau K/2) u_n + tau/2 phi_1(tau K/2) g_n
      U_3 = U_2 + tau phi_{2,3} D_2
      U_4 = e^(tau K) u_n + tau phi_1(tau K) g_n + tau phi_{2,4} (D_2 + D_3)
      U_5 = U_2 + tau (a_52 (D_2 + D_3) + a_54 D_4),  a_54 = phi_{2,5}/4 - a_52,
            a_52 = phi_{2,5}/2 - phi_{3,4} + phi_{2,4}/4 - phi_{3,5}/2
      u_{n+1} = e^(tau K) u_n + tau phi_1(tau K) g_n
                + tau ((-phi_2 + 4 phi_3) D_4 + (4 phi_2 - 8 phi_3) D_5).
    smart=False takes the stages one by one as linear combinations (stage 5 mixes the
    scales tau/2 and tau, so it is two combinations); smart=True assembles them from the
    five lines of eq. expRK4s5_smart: two-scale outputs (j = 0, 1) of phi_1 on the
    first line (taken here as the combination e^(c tau K) u_n + c tau phi_1(c tau K) g_n,
    which equals u_n + c tau phi_1(c tau K) f_n), of phi_2 on D_2 and on D_3 (same
    vector), the two-scale combination phi_2/4^j D_4 + phi_3/8^j 4 (D_2 + D_3 - D_4),
    and phi_2 (4 D_5 - D_4) + phi_3 (4 D_4 - 8 D_5)."""
    tau = T / steps
    plans = {}
    w = np.asarray(w0, dtype=np.float64).copy()
    h2 = 0.5 * tau
    for n in range(steps):
        t = n * tau
        gn = g(t, w)
        if not smart:
            U2 = _lc_blocks(blocks, plans, h2, [w, h2 * gn], 1, 1, tol)[0]
            D2 = g(t + h2, U2) - gn
            U3 = _lc_blocks(blocks, plans, h2, [w, h2 * gn, tau * D2], 2, 1, tol)[0]
            D3 = g(t + h2, U3) - gn
            U4 = _lc_blocks(blocks, plans, tau, [w, tau * gn, tau * (D2 + D3)], 2, 1, tol)[0]
            D4 = g(t + tau, U4) - gn
            D = D2 + D3 - D4
            U5 = _lc_blocks(blocks, plans, h2, [w, h2 * gn, tau * (0.5 * D + 0.25 * D4),
                                                -0.5 * tau * D], 3, 1, tol)[0]
            U5 = U5 + _lc_blocks(blocks, plans, tau, [None, None, 0.25 * tau * D, -tau * D],
                                 3, 1, tol)[0]
            D5 = g(t + h2, U5) - gn
            w = _lc_blocks(blocks, plans, tau, [w, tau * gn, tau * (4 * D5 - D4),
                                                tau * (4 * D4 - 8 * D5)], 3, 1, tol)[0]
            continue
        E = _lc_blocks(blocks, plans, tau, [w, tau * gn], 1, 2, tol)      # scales 1, 1/2
        D2 = g(t + h2, E[1]) - gn
        P2 = _sv_blocks(blocks, plans, tau, D2, 2, 2, tol)                  # phi_l(tau K/2^j) D_2
        D3 = g(t + h2, E[1] + tau * P2[1, 2]) - gn
        P3 = _sv_blocks(blocks, plans, tau, D3, 2, 2, tol)
        D4 = g(t + tau, E[0] + tau * (P2[0, 2] + P3[0, 2])) - gn
        L4 = _lc_blocks(blocks, plans, tau, [None, None, D4, 4.0 * (D2 + D3 - D4)], 3, 2, tol)
        U5 = E[1] + tau * (0.5 * (P2[1, 2] + P3[1, 2]) + 0.25 * (P2[0, 2] + P3[0, 2])
                           - L4[1] - 0.25 * L4[0])
        D5 = g(t + h2, U5) - gn
        L5 = _lc_blocks(blocks, plans, tau, [None, None, 4.0 * D5 - D4, 4.0 * D4 - 8.0 * D5],
                        3, 1, tol)
        w = E[0] + tau * L5[0]
    return w


def brusselator_nonlinearity(a: float, b: float, N: int):
    """g(w) = (a + u^2 v, b u - u^2 v) for w = (u, v), each of N values (the reaction
    terms of the Brusselator system of Section 4.4)."""
    def g(t, w):
        u, v = w[:N], w[N:]
        uuv = u * u * v
        return np.concatenate([a + uuv, b * u - uuv])
    return g
