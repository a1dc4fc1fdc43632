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
from .phiks import phi_lincomb


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
