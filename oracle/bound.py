"""Choice of the scaling s and of the number q of quadrature points (oracle).

Follows Section 3.3 of the paper:

* The remainder of the q-point rule for the integrand f_l(theta, X) =
  theta^(l-1)/(l-1)! exp((1-theta) X) is bounded in 2-norm by (1 + sqrt 2) times
  the supremum, over a convex set Omega containing the numerical range W(K), of the
  modulus of the *scalar* remainder (estimate (CPestimate), using that W(K) is a
  (1 + sqrt 2)-spectral set).  The paper evaluates that scalar remainder as a contour
  integral of the kernel k_q over an ellipse; mathematically the contour integral
  equals the scalar quadrature error itself,
        R_q(f_l(., w)) = phi_l(w) - sum_i w_i theta_i^(l-1)/(l-1)! e^((1-theta_i) w),
  which is what the oracle computes, directly from that definition, in mpmath with
  as many digits as the cancellation needs.
* Omega is the rectangle Xi = Xi_1 + ... + Xi_d, Xi_mu covering W(B_mu) (B_mu = tau
  A_mu); W(K) is the Minkowski sum of the W(A_mu).  Reading used by default: Xi_mu is
  the Bendixson rectangle [lambda_min(H), lambda_max(H)] x i[lambda_min(S),
  lambda_max(S)] with H = (B + B^H)/2 and S = (B - B^H)/(2i); the alternative reading
  (``rectangle(..., "norm_centered")``) centres the box at tr(B)/n with the 2-norms of
  the shifted H and S as half-widths.
* By the maximum modulus principle the supremum is taken on the boundary of Xi,
  discretised by ``M_SIDE`` equispaced points per side (corners included).
* Same vector (formula (Tpsv)): starting from s = 0 (here from s = n_scales - 1 so
  that all requested scales exist) take the smallest q in [3, 12] with
  b_{q,l}(s) ||v|| <= delta 2^(l s) for l = 1..p; linear combination (formula
  (Tlcp)): sum_{k=1}^{l} b_{q,l-k+1}(s) ||v_{p+1-k}|| / 2^((l-k+1) s) <= delta for
  l = 1..p.  s is increased until the Tucker count T#(s+1) exceeds T#(s); an s
  with no feasible q counts as T# = infinity, and equal counts do not stop the
  search (strictly larger only).
"""
from __future__ import annotations

import functools
import math
from typing import List, Optional, Sequence, Tuple

import mpmath as mp
import numpy as np

from .gll import gll_mp

Q_MIN, Q_MAX = 3, 12
S_MAX = 64
M_SIDE = 16                       # boundary points per side of the rectangle
CP_CONST = 1.0 + math.sqrt(2.0)   # Crouzeix-Palencia constant


RECT_KINDS = ("bendixson", "norm_centered")


def rectangle(B: np.ndarray, kind: str = "bendixson") -> Tuple[float, float, float, float]:
    """A rectangle (re_lo, re_hi, im_lo, im_hi) containing W(B).

    Section 3.3 builds it from the Hermitian part H = (B + B^H)/2 and the skew-Hermitian
    part, written here as the Hermitian S = (B - B^H)/(2i), without fixing how; two
    readings:
    * ``bendixson``: [lambda_min(H), lambda_max(H)] x i[lambda_min(S), lambda_max(S)];
    * ``norm_centered``: centred at sigma = tr(B)/n (the shift of the remark in Section
      3.1), half-widths ||H - Re(sigma) I||_2 and ||S - Im(sigma) I||_2.
    """
    B = np.asarray(B)
    Bh = B.conj().T
    H = (B + Bh) / 2.0
    S = (B - Bh) / 2.0j
    if kind == "bendixson":
        eh = np.linalg.eigvalsh(H)
        es = np.linalg.eigvalsh(S)
        return float(eh[0]), float(eh[-1]), float(es[0]), float(es[-1])
    if kind == "norm_centered":
        n = B.shape[0]
        sigma = complex(np.trace(B)) / n
        eye = np.eye(n)
        hr = float(np.linalg.norm(H - sigma.real * eye, 2))
        hi = float(np.linalg.norm(S - sigma.imag * eye, 2))
        return sigma.real - hr, sigma.real + hr, sigma.imag - hi, sigma.imag + hi
    raise ValueError(f"unknown rectangle kind {kind!r}")


def kron_sum_rectangle(Bs: Sequence[np.ndarray],
                       kind: str = "bendixson") -> Tuple[float, float, float, float]:
    """Xi = Xi_1 + ... + Xi_d (sum of the rectangles of the B_mu)."""
    r = [0.0, 0.0, 0.0, 0.0]
    for B in Bs:
        x = rectangle(B, kind)
        for k in range(4):
            r[k] += x[k]
    return tuple(r)


def boundary_points(xi, m_side: int = M_SIDE) -> List[complex]:
    """M_SIDE points on each side of the rectangle, counter-clockwise from re_lo + i im_lo."""
    a, b, c, d = xi
    corners = [complex(a, c), complex(b, c), complex(b, d), complex(a, d)]
    pts = []
    for k in range(4):
        z0, z1 = corners[k], corners[(k + 1) % 4]
        for m in range(m_side):
            pts.append(z0 + (z1 - z0) * (m / m_side))
    return pts


def phi_mp(ell: int, w):
    """phi_l(w) = int_0^1 theta^(l-1)/(l-1)! e^((1-theta)w) dtheta (formula (phifunctions)),
    l >= 1: power series sum_k w^k/(k+l)! for |w| <= 1, closed form otherwise."""
    if abs(w) <= 1:
        tot, term, k = mp.mpc(0), 1 / mp.factorial(ell), 0
        eps = mp.mpf(10) ** (-mp.mp.dps - 5)
        while True:
            tot += term
            k += 1
            term = term * w / (k + ell)
            if abs(term) < eps:
                break
        return tot
    head = mp.fsum(w ** k / mp.factorial(k) for k in range(ell))
    return (mp.exp(w) - head) / w ** ell


def quad_errors(q: int, w: complex, p: int) -> List[float]:
    """|R_q(f_l(., w))| for l = 1..p: exact quadrature error of the q-point
    Gauss-Lobatto rule for theta -> theta^(l-1)/(l-1)! exp((1-theta) w)."""
    theta, wts = gll_mp(q, 130)
    dps = 40
    while True:
        with mp.workdps(dps):
            wz = mp.mpc(w.real, w.imag)
            ex = [mp.exp((1 - th) * wz) for th in theta]
            out, resolved = [], True
            for ell in range(1, p + 1):
                f = mp.factorial(ell - 1)
                terms = [wi * th ** (ell - 1) * e / f for wi, th, e in zip(wts, theta, ex)]
                ph = phi_mp(ell, wz)
                err = ph - mp.fsum(terms)
                mag = max(abs(ph), mp.fsum(abs(t) for t in terms))
                floor = mag * mp.mpf(10) ** (-(dps - 12))
                if abs(err) < floor:
                    if dps < 120:
                        resolved = False
                        break
                    out.append(float(floor))      # below resolution: a safe upper bound
                else:
                    out.append(float(abs(err)))
        if resolved:
            return out
        dps *= 2


def bounds_at(xi, s: int, q: int, p: int) -> List[float]:
    """b_{q,l}(s) = (1 + sqrt 2) max_{w on boundary of Xi/2^s} |R_q(f_l(., w))|, l = 1..p.
    A pure function of its arguments, so its values are kept (a plan made again for the
    same rectangle, as time integrators do every step size, does not recompute them)."""
    return list(_bounds_at(tuple(float(x) for x in xi), int(s), int(q), int(p)))


@functools.lru_cache(maxsize=4096)
def _bounds_at(xi, s: int, q: int, p: int):
    sc = 2.0 ** (-s)
    best = [0.0] * p
    for w in boundary_points(xi):
        e = quad_errors(q, w * sc, p)
        for k in range(p):
            best[k] = max(best[k], e[k])
    return tuple(CP_CONST * b for b in best)


def tucker_count(task: str, s: int, q: int, p: int, n_scales: int) -> int:
    """Formula (Tpsv) for the same vector, formula (Tlcp) for a linear combination."""
    if task == "same_vector":
        return q + s * p + n_scales
    return q * p + s * p + n_scales


def feasible(task: str, b: List[float], s: int, p: int, tol: float,
             vnorms: Optional[Sequence[float]]) -> bool:
    if task == "same_vector":
        nv = 1.0 if vnorms is None else float(vnorms[0])
        return all(b[ell - 1] * nv <= tol * 2.0 ** (ell * s) for ell in range(1, p + 1))
    nv = [1.0] * (p + 1) if vnorms is None else [float(x) for x in vnorms]
    for ell in range(1, p + 1):
        tot = 0.0
        for k in range(1, ell + 1):
            tot += b[ell - k] * nv[p + 1 - k] / 2.0 ** ((ell - k + 1) * s)
        if tot > tol:
            return False
    return True


def plan(xi, p: int, n_scales: int, tol: float, task: str = "same_vector",
         vnorms: Optional[Sequence[float]] = None, q_min: int = Q_MIN,
         q_max: int = Q_MAX, s_max: int = S_MAX) -> Tuple[int, int, int]:
    """Return (s, q, T#) chosen as in Section 3.3.  p = 0 needs no quadrature."""
    s0 = max(0, n_scales - 1)
    if p == 0:
        return s0, 0, n_scales
    prev = None                     # (s, q, T)
    for s in range(s0, s_max + 1):
        q_found = None
        for q in range(q_min, q_max + 1):
            if feasible(task, bounds_at(xi, s, q, p), s, p, tol, vnorms):
                q_found = q
                break
        T = math.inf if q_found is None else tucker_count(task, s, q_found, p, n_scales)
        if prev is not None and T > prev[2]:
            return prev
        prev = (s, q_found, T)
    if prev is None or prev[1] is None:
        raise RuntimeError("no (s, q) satisfies the tolerance")
    return prev
