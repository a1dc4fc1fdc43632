"""The phiks algorithm, written step by step in FP64 (oracle).

Both tasks of Section 3 of the paper, for K = A_d (+) ... (+) A_1 and B_mu = tau A_mu:

* ``same_vector``: exp(2^-j tau K) v and phi_l(2^-j tau K) v, l = 1..p, for the
  scales j = 0..n_scales-1.  Quadrature (eq. integrandsimul) at the scaled operator
  K/2^s, then the squaring recurrence (eq. simul) for j = s..1, l = p..1.
* ``lincomb``: exp(c_j tau K) v_0 + sum_l c_j^l phi_l(c_j tau K) v_l with c_j = 2^-j
  (eq. scallincomb).  Quadrature of the auxiliary combinations (eq. integrandcomb),
  then the squaring recurrence (eq. comb).

Every exponential of the large operator is a Tucker operator (eq. Tuckerprod,
eq. tucker) with small exponentials exp((1 - theta_i) B_mu / 2^s); those at coarser
levels come from squaring, exp(B_mu/2^(j-1)) = exp(B_mu/2^j)^2 (Section 3.1).
The quadrature rule is Gauss-Lobatto-Legendre; the node theta_q = 1 needs no
Tucker operator (its exponential is the identity), as Section 3.3 notes.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np

from .expm import expm_taylor
from .gll import gll
from .tensor import tucker


def _node_matrices(Bs, theta_i: float, s: int):
    return [expm_taylor((1.0 - theta_i) * B / 2.0 ** s) for B in Bs]


def phi_same_vector(A: Sequence[np.ndarray], tau: float, v: np.ndarray, p: int,
                    n_scales: int, s: int, q: int, with_exp: bool = True) -> np.ndarray:
    """Return out[j, l] = phi_l(2^-j tau K) v for j < n_scales, l = 0..p (l = 0: exp).

    Steps (Section 3.1): P_l = sum_i w_i theta_i^(l-1)/(l-1)! Tucker_i(v)
    (eq. integrandsimul), then for j = s..1 and l = p..1
    P_l <- 2^-l (Tucker(P_l; E_j) + sum_{k<=l} P_k/(l-k)!) with E_j = exp(B/2^j)
    (eq. simul), the right-hand side taking the values before the step.
    """
    n = [a.shape[0] for a in A]
    N = int(np.prod(n))
    Bs = [tau * np.asarray(a) for a in A]
    dt = np.result_type(v, *Bs)
    out = np.zeros((n_scales, p + 1, N), dtype=dt)
    if s < n_scales - 1:
        raise ValueError("need s >= n_scales - 1")
    E = [expm_taylor(B / 2.0 ** s) for B in Bs]           # exp(B_mu / 2^s)
    P = [np.zeros(N, dtype=dt) for _ in range(p)]
    if p > 0:
        theta, w = gll(q)
        for th, wi in zip(theta, w):
            X = v if th == 1.0 else tucker(v, n, _node_matrices(Bs, th, s))
            for ell in range(1, p + 1):
                P[ell - 1] = P[ell - 1] + (wi * th ** (ell - 1) / math.factorial(ell - 1)) * X

    def emit(level):
        if level < n_scales:
            if with_exp:
                out[level, 0] = tucker(v, n, E)
            for ell in range(1, p + 1):
                out[level, ell] = P[ell - 1]

    emit(s)
    for j in range(s, 0, -1):
        old = [x.copy() for x in P]
        for ell in range(p, 0, -1):
            acc = tucker(old[ell - 1], n, E)
            for k in range(1, ell + 1):
                acc = acc + old[k - 1] / math.factorial(ell - k)
            P[ell - 1] = acc / 2.0 ** ell
        E = [e @ e for e in E]                              # exp(B/2^(j-1))
        emit(j - 1)
    return out


def phi_lincomb(A: Sequence[np.ndarray], tau: float, vs: Sequence[Optional[np.ndarray]],
                p: int, n_scales: int, s: int, q: int) -> np.ndarray:
    """Return out[j] = exp(c_j tau K) v_0 + sum_{l=1}^p c_j^l phi_l(c_j tau K) v_l,
    c_j = 2^-j, j < n_scales.  vs = [v_0, ..., v_p]; None entries are zero vectors.

    Q_l denotes Phi(K) v_{p-l+1..p} = sum_{m=1}^{l} phi_m(K/2^j) v_{p-l+m} / 2^(m j)
    (Section 3.2).  Quadrature (eq. integrandcomb) with the node inputs
    U_il = sum_{k=1}^{l} theta_i^(l-k)/(l-k)! v_{p+1-k} / 2^((l-k+1) s); squaring
    (eq. comb) Q_l <- Tucker(Q_l; E_j) + sum_{k<=l} Q_k / ((l-k)! 2^((l-k) j)),
    l = p..1, on the values before the step.  Q_p at level j is the requested
    combination without the exponential term.
    """
    n = [a.shape[0] for a in A]
    N = int(np.prod(n))
    Bs = [tau * np.asarray(a) for a in A]
    present = [x for x in vs if x is not None]
    dt = np.result_type(*(present + Bs)) if present else np.float64
    vv = [np.zeros(N, dtype=dt) if x is None else np.asarray(x, dtype=dt) for x in vs]
    if s < n_scales - 1:
        raise ValueError("need s >= n_scales - 1")
    out = np.zeros((n_scales, N), dtype=dt)
    E = [expm_taylor(B / 2.0 ** s) for B in Bs]
    Q = [np.zeros(N, dtype=dt) for _ in range(p)]
    if p > 0:
        theta, w = gll(q)
        for th, wi in zip(theta, w):
            Ls = None if th == 1.0 else _node_matrices(Bs, th, s)
            for ell in range(1, p + 1):
                U = np.zeros(N, dtype=dt)
                for k in range(1, ell + 1):
                    U = U + (th ** (ell - k) / math.factorial(ell - k)
                             / 2.0 ** ((ell - k + 1) * s)) * vv[p + 1 - k]
                X = U if Ls is None else tucker(U, n, Ls)
                Q[ell - 1] = Q[ell - 1] + wi * X

    def emit(level):
        if level < n_scales:
            acc = Q[p - 1].copy() if p > 0 else np.zeros(N, dtype=dt)
            if vs[0] is not None:
                acc = acc + tucker(vv[0], n, E)
            out[level] = acc

    emit(s)
    for j in range(s, 0, -1):
        old = [x.copy() for x in Q]
        for ell in range(p, 0, -1):
            acc = tucker(old[ell - 1], n, E)
            for k in range(1, ell + 1):
                acc = acc + old[k - 1] / (math.factorial(ell - k) * 2.0 ** ((ell - k) * j))
            Q[ell - 1] = acc
        E = [e @ e for e in E]
        emit(j - 1)
    return out
