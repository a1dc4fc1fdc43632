"""Gauss-Lobatto-Legendre rule on [0, 1] (oracle).

Section 3.3 of the paper selects the Gauss-Lobatto-Legendre formula with q points,
q in [3, 12]; its nodes include both endpoints (theta_1 = 0, theta_q = 1).  The
interior nodes are the zeros of P'_{q-1}(2t - 1) (P_k the Legendre polynomial) and
the weights on [-1, 1] are 2 / (q (q-1) P_{q-1}(x_i)^2); on [0, 1] they are halved.
Computed here in mpmath by Newton's method from Chebyshev-Lobatto starting points.
"""
from __future__ import annotations

from functools import lru_cache
from typing import List, Tuple

import mpmath as mp


def _legendre(n: int, x):
    """P_n(x) and P_{n-1}(x) by the three-term recurrence."""
    p_prev, p = mp.mpf(1), x
    if n == 0:
        return mp.mpf(1), mp.mpf(0)
    for k in range(2, n + 1):
        p_prev, p = p, ((2 * k - 1) * x * p - (k - 1) * p_prev) / k
    return p, p_prev


@lru_cache(maxsize=None)
def gll_mp(q: int, dps: int = 60) -> Tuple[tuple, tuple]:
    """(theta, w) as mpmath numbers, theta ascending on [0, 1]."""
    if q < 2:
        raise ValueError("Gauss-Lobatto needs q >= 2")
    with mp.workdps(dps + 10):
        n = q - 1
        interior = []
        for k in range(1, n):
            x = -mp.cos(mp.pi * k / n)
            for _ in range(200):
                P, Pm1 = _legendre(n, x)
                dP = n * (x * P - Pm1) / (x * x - 1)
                # Legendre equation: (1 - x^2) P'' = 2 x P' - n (n + 1) P
                d2P = (2 * x * dP - n * (n + 1) * P) / (1 - x * x)
                step = dP / d2P
                x -= step
                if abs(step) < mp.mpf(10) ** (-(dps + 5)):
                    break
            interior.append(x)
        xs = [mp.mpf(-1)] + interior + [mp.mpf(1)]
        ws = [2 / (n * (n + 1) * _legendre(n, x)[0] ** 2) for x in xs]
        theta = tuple((x + 1) / 2 for x in xs)
        w = tuple(wi / 2 for wi in ws)
    return theta, w


def gll(q: int) -> Tuple[List[float], List[float]]:
    """(theta, w) rounded to float64, theta_1 = 0 and theta_q = 1 exactly."""
    theta, w = gll_mp(q)
    t = [float(x) for x in theta]
    t[0], t[-1] = 0.0, 1.0
    return t, [float(x) for x in w]
