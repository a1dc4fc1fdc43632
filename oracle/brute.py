"""Exact references used only to pin the oracle (tiny sizes).

* ``augmented``: Section 2 restates Theorem 2.1 of Al-Mohy and Higham: the first N
  rows of exp(c [[tau K, v_p ... v_1], [0, J]]) [v_0; 0; ...; 0; 1], with J the p x p
  matrix with ones on the superdiagonal, equal
  exp(c tau K) v_0 + sum_l c^l phi_l(c tau K) v_l.  K is assembled densely and the
  exponential is scipy's (a library routine independent of the oracle's own expm).
* ``phi_scalar``: the closed form phi_l(z) = (e^z - sum_{k<l} z^k/k!)/z^l, and
  phi_l(0) = 1/l!, of the integral definition (formula (phifunctions)).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import mpmath as mp
import numpy as np
import scipy.linalg

from .tensor import kron_sum_dense


def augmented(A: Sequence[np.ndarray], tau: float, vs: Sequence[Optional[np.ndarray]],
              c: float = 1.0) -> np.ndarray:
    K = kron_sum_dense(A)
    N = K.shape[0]
    p = len(vs) - 1
    present = [x for x in vs if x is not None]
    dt = np.result_type(K, *present) if present else K.dtype
    M = np.zeros((N + p, N + p), dtype=dt)
    M[:N, :N] = tau * K
    for col in range(p):                     # columns v_p, v_{p-1}, ..., v_1
        vec = vs[p - col]
        if vec is not None:
            M[:N, N + col] = vec
    for k in range(p - 1):
        M[N + k, N + k + 1] = 1.0
    rhs = np.zeros(N + p, dtype=dt)
    if vs[0] is not None:
        rhs[:N] = vs[0]
    if p > 0:
        rhs[-1] = 1.0
    return (scipy.linalg.expm(c * M) @ rhs)[:N]


def phi_actions_dense(A: Sequence[np.ndarray], tau: float, v: np.ndarray, p: int,
                      c: float = 1.0) -> np.ndarray:
    """phi_l(c tau K) v for l = 0..p, each from its own augmented exponential."""
    N = len(v)
    out = np.zeros((p + 1, N), dtype=np.result_type(v, *A))
    out[0] = augmented(A, tau, [v], c)
    for ell in range(1, p + 1):
        vs = [None] * (ell + 1)
        vs[ell] = v
        out[ell] = augmented(A, tau, vs, c) / c ** ell
    return out


def phi_scalar(ell: int, z: complex) -> complex:
    """Closed form evaluated in 60-digit arithmetic (it cancels badly near z = 0)."""
    if z == 0:
        return 1.0 / math.factorial(ell)
    with mp.workdps(60):
        zz = mp.mpc(complex(z).real, complex(z).imag)
        head = mp.fsum(zz ** k / mp.factorial(k) for k in range(ell))
        val = (mp.exp(zz) - head) / zz ** ell
    return complex(val)
