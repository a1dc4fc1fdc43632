"""Exponential integrators on the library's phi-actions (all vector work on the GPU).

exp_euler follows the exponential Euler scheme in its linear-combination form
(eq. expEullc), etd2rk the second-order exponential Runge-Kutta scheme in its
linear-combination form (eq. ETD2RKlc).  Every step is one or two phiks_combine calls
(plans built once per step size, tolerance read relative: vector norms taken as 1)
plus phiks_vector_op for the stage vectors.  The nonlinearity is a callable
g(t, u_ptr, out_ptr) that writes g(t, u) into out on the device, e.g. ADRNonlinearity.
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np

from . import (PHIKS_VOP_AXPBY, PHIKS_VOP_BRUSS_U, PHIKS_VOP_BRUSS_V, PHIKS_VOP_CUBIC,
               PHIKS_VOP_RATIONAL, DeviceArray, memcpy_dtod, phiks_apply, phiks_combine,
               phiks_plan, vector_op)


class ADRNonlinearity:
    """g(t, u) = 1/(1 + u^2) + Psi(t) of the advection-diffusion-reaction problem of
    Section 4.2, Psi(t) = e^t w - 1/(1 + (e^t u_0)^2), evaluated on the device."""

    def __init__(self, u0: np.ndarray, w: np.ndarray, stream: int = 0):
        self.N = int(u0.size)
        self.u0 = DeviceArray.from_numpy(u0)
        self.w = DeviceArray.from_numpy(w)
        self.tmp = DeviceArray(self.N)
        self.stream = stream

    def __call__(self, t: float, u_ptr: int, out_ptr: int) -> None:
        et = math.exp(t)
        N, st, tmp = self.N, self.stream, self.tmp.ptr
        vector_op(PHIKS_VOP_RATIONAL, N, 1.0, u_ptr, 1.0, None, tmp, st)          # 1/(1+u^2)
        vector_op(PHIKS_VOP_RATIONAL, N, -1.0, self.u0.ptr, et, tmp, tmp, st)     # -1/(1+(e^t u0)^2)
        vector_op(PHIKS_VOP_AXPBY, N, 1.0, tmp, et, self.w.ptr, out_ptr, st)      # + e^t w


class AllenCahnNonlinearity:
    """g(u) = u - u^3 (the Allen-Cahn reaction kept outside K)."""

    def __init__(self, N: int, stream: int = 0):
        self.N, self.stream = N, stream

    def __call__(self, t: float, u_ptr: int, out_ptr: int) -> None:
        vector_op(PHIKS_VOP_CUBIC, self.N, 1.0, u_ptr, 0.0, None, out_ptr, self.stream)


def _start(u0, N):
    if isinstance(u0, DeviceArray):
        u = DeviceArray(N)
        vector_op(PHIKS_VOP_AXPBY, N, 1.0, u0.ptr, 0.0, None, u.ptr)
        return u
    return DeviceArray.from_numpy(np.asarray(u0, dtype=np.float64))


def exp_euler(A: Sequence[np.ndarray], u0, g: Callable[[float, int, int], None], T: float,
              steps: int, tol: float = 2.0 ** -53, stream: int = 0) -> DeviceArray:
    """u_{n+1} = exp(tau K) u_n + phi_1(tau K) (tau g(t_n, u_n)), tau = T / steps."""
    tau = T / steps
    N = int(np.prod([a.shape[0] for a in A]))
    plan = phiks_plan(A, tau, 1, 1, tol, "lincomb", stream=stream)
    ws = DeviceArray(plan.workspace_size() // 8 + 1)
    u, un, gb = _start(u0, N), DeviceArray(N), DeviceArray(N)
    for n in range(steps):
        g(n * tau, u.ptr, gb.ptr)
        vector_op(PHIKS_VOP_AXPBY, N, tau, gb.ptr, 0.0, None, gb.ptr, stream)
        phiks_combine(plan, [u.ptr, gb.ptr], un.ptr, ws.ptr, ws.nbytes, stream)
        u, un = un, u
    plan.close()
    return u


def etd2rk(A: Sequence[np.ndarray], u0, g: Callable[[float, int, int], None], T: float,
           steps: int, tol: float = 2.0 ** -53, stream: int = 0) -> DeviceArray:
    """u_n2    = exp(tau K) u_n + phi_1(tau K) (tau g_n)
    u_{n+1} = exp(tau K) u_n + phi_1(tau K) (tau g_n) + phi_2(tau K) (tau (g(t_n + tau, u_n2) - g_n))."""
    tau = T / steps
    N = int(np.prod([a.shape[0] for a in A]))
    p1 = phiks_plan(A, tau, 1, 1, tol, "lincomb", stream=stream)
    p2 = phiks_plan(A, tau, 2, 1, tol, "lincomb", stream=stream)
    ws = DeviceArray(max(p1.workspace_size(), p2.workspace_size()) // 8 + 1)
    u, un, u2 = _start(u0, N), DeviceArray(N), DeviceArray(N)
    gn, g2, v1, v2 = (DeviceArray(N) for _ in range(4))
    for n in range(steps):
        t = n * tau
        g(t, u.ptr, gn.ptr)
        vector_op(PHIKS_VOP_AXPBY, N, tau, gn.ptr, 0.0, None, v1.ptr, stream)
        phiks_combine(p1, [u.ptr, v1.ptr], u2.ptr, ws.ptr, ws.nbytes, stream)
        g(t + tau, u2.ptr, g2.ptr)
        vector_op(PHIKS_VOP_AXPBY, N, tau, g2.ptr, -tau, gn.ptr, v2.ptr, stream)
        phiks_combine(p2, [u.ptr, v1.ptr, v2.ptr], un.ptr, ws.ptr, ws.nbytes, stream)
        u, un = un, u
    p1.close()
    p2.close()
    return u


def _pair(buf: DeviceArray, N: int):
    """Pointers to the two outputs of a two-scale combination (scale 1, scale 1/2)."""
    return buf.ptr, buf.ptr + 8 * N


def exprk3s3(A: Sequence[np.ndarray], u0, g: Callable[[float, int, int], None], T: float,
             steps: int, tol: float = 2.0 ** -53, stream: int = 0) -> DeviceArray:
    """Third-order scheme of eq. expRK3s3 (c_3 = 2 c_2 = 1/2, gamma = -4/5):
      U_2     = e^(c_2 tau K) u_n + c_2 tau phi_1(c_2 tau K) g_n
      U_3     = e^(c_3 tau K) u_n + c_3 tau phi_1(c_3 tau K) g_n
                + tau (gamma c_2 phi_2(c_2 tau K) + c_3^2/c_2 phi_2(c_3 tau K)) D_2
      u_{n+1} = e^(tau K) u_n + tau phi_1(tau K) g_n + tau phi_2(tau K) (gamma D_2 + D_3) / (gamma c_2 + c_3)
    with D_j = g(t_n + c_j tau, U_j) - g_n."""
    c2, c3 = 0.25, 0.5
    gam = (3 * c3 - 2) * c3 / ((2 - 3 * c2) * c2)
    tau = T / steps
    N = int(np.prod([a.shape[0] for a in A]))
    P2 = phiks_plan(A, c2 * tau, 1, 1, tol, "lincomb", stream=stream)
    P3 = phiks_plan(A, c3 * tau, 2, 1, tol, "lincomb", stream=stream)
    P3b = phiks_plan(A, c2 * tau, 2, 1, tol, "lincomb", stream=stream)
    Pf = phiks_plan(A, tau, 2, 1, tol, "lincomb", stream=stream)
    plans = (P2, P3, P3b, Pf)
    ws = DeviceArray(max(p.workspace_size() for p in plans) // 8 + 1)
    u, un = _start(u0, N), DeviceArray(N)
    gn, U2, U3, D2, D3, v1, v2, tmp = (DeviceArray(N) for _ in range(8))
    AX = PHIKS_VOP_AXPBY
    for n in range(steps):
        t = n * tau
        g(t, u.ptr, gn.ptr)
        vector_op(AX, N, c2 * tau, gn.ptr, 0.0, None, v1.ptr, stream)
        phiks_combine(P2, [u.ptr, v1.ptr], U2.ptr, ws.ptr, ws.nbytes, stream)
        g(t + c2 * tau, U2.ptr, D2.ptr)
        vector_op(AX, N, 1.0, D2.ptr, -1.0, gn.ptr, D2.ptr, stream)
        vector_op(AX, N, c3 * tau, gn.ptr, 0.0, None, v1.ptr, stream)
        vector_op(AX, N, tau * c3 * c3 / c2, D2.ptr, 0.0, None, v2.ptr, stream)
        phiks_combine(P3, [u.ptr, v1.ptr, v2.ptr], U3.ptr, ws.ptr, ws.nbytes, stream)
        vector_op(AX, N, tau * gam * c2, D2.ptr, 0.0, None, v2.ptr, stream)
        phiks_combine(P3b, [None, None, v2.ptr], tmp.ptr, ws.ptr, ws.nbytes, stream)
        vector_op(AX, N, 1.0, U3.ptr, 1.0, tmp.ptr, U3.ptr, stream)
        g(t + c3 * tau, U3.ptr, D3.ptr)
        vector_op(AX, N, 1.0, D3.ptr, -1.0, gn.ptr, D3.ptr, stream)
        vector_op(AX, N, tau, gn.ptr, 0.0, None, v1.ptr, stream)
        den = gam * c2 + c3
        vector_op(AX, N, tau * gam / den, D2.ptr, tau / den, D3.ptr, v2.ptr, stream)
        phiks_combine(Pf, [u.ptr, v1.ptr, v2.ptr], un.ptr, ws.ptr, ws.nbytes, stream)
        u, un = un, u
    for p in plans:
        p.close()
    return u


def exprk4s6(A: Sequence[np.ndarray], u0, g: Callable[[float, int, int], None], T: float,
             steps: int, tol: float = 2.0 ** -53, stream: int = 0) -> DeviceArray:
    """Fourth-order six-stage scheme of eq. expRK4s6 with c = (1/3, 1/3, 2/3, 1/2, 1):
    four combinations per step -- stage 2; stages 4 and 3 as the two scales of one
    combination with step c_4 tau (c_3 = c_4/2); stages 6 and 5 likewise with step tau;
    the update (coefficients as in the tableau)."""
    c2, c3, c4, c5, c6 = 1 / 3, 1 / 3, 2 / 3, 0.5, 1.0
    tau = T / steps
    N = int(np.prod([a.shape[0] for a in A]))
    P2 = phiks_plan(A, c2 * tau, 1, 1, tol, "lincomb", stream=stream)
    P34 = phiks_plan(A, c4 * tau, 2, 2, tol, "lincomb", stream=stream)
    P56 = phiks_plan(A, tau, 3, 2, tol, "lincomb", stream=stream)
    Pf = phiks_plan(A, tau, 3, 1, tol, "lincomb", stream=stream)
    plans = (P2, P34, P56, Pf)
    ws = DeviceArray(max(p.workspace_size() for p in plans) // 8 + 1)
    u, un = _start(u0, N), DeviceArray(N)
    gn, U2, D2, D3, D4, D5, D6, v1, v2, v3 = (DeviceArray(N) for _ in range(10))
    O34, O56 = DeviceArray(2 * N), DeviceArray(2 * N)
    AX = PHIKS_VOP_AXPBY
    a53 = (c4 * c6 ** 2 / (c3 * (c4 - c3)), c3 * c6 ** 2 / (c4 * (c3 - c4)))
    a63 = (2 * c6 ** 3 / (c3 * (c3 - c4)), 2 * c6 ** 3 / (c4 * (c4 - c3)))
    b2 = (c6 / (c5 * (c6 - c5)), c5 / (c6 * (c5 - c6)))
    b3 = (2 / (c5 * (c5 - c6)), 2 / (c6 * (c6 - c5)))

    def diff(tt, U_ptr, D):
        g(tt, U_ptr, D.ptr)
        vector_op(AX, N, 1.0, D.ptr, -1.0, gn.ptr, D.ptr, stream)

    for n in range(steps):
        t = n * tau
        g(t, u.ptr, gn.ptr)
        vector_op(AX, N, c2 * tau, gn.ptr, 0.0, None, v1.ptr, stream)
        phiks_combine(P2, [u.ptr, v1.ptr], U2.ptr, ws.ptr, ws.nbytes, stream)
        diff(t + c2 * tau, U2.ptr, D2)
        vector_op(AX, N, c4 * tau, gn.ptr, 0.0, None, v1.ptr, stream)
        vector_op(AX, N, tau * c4 * c4 / c2, D2.ptr, 0.0, None, v2.ptr, stream)
        phiks_combine(P34, [u.ptr, v1.ptr, v2.ptr], O34.ptr, ws.ptr, ws.nbytes, stream)
        U4, U3 = _pair(O34, N)
        diff(t + c3 * tau, U3, D3)
        diff(t + c4 * tau, U4, D4)
        vector_op(AX, N, tau, gn.ptr, 0.0, None, v1.ptr, stream)
        vector_op(AX, N, tau * a53[0], D3.ptr, tau * a53[1], D4.ptr, v2.ptr, stream)
        vector_op(AX, N, tau * a63[0], D3.ptr, tau * a63[1], D4.ptr, v3.ptr, stream)
        phiks_combine(P56, [u.ptr, v1.ptr, v2.ptr, v3.ptr], O56.ptr, ws.ptr, ws.nbytes, stream)
        U6, U5 = _pair(O56, N)
        diff(t + c5 * tau, U5, D5)
        diff(t + c6 * tau, U6, D6)
        vector_op(AX, N, tau * b2[0], D5.ptr, tau * b2[1], D6.ptr, v2.ptr, stream)
        vector_op(AX, N, tau * b3[0], D5.ptr, tau * b3[1], D6.ptr, v3.ptr, stream)
        phiks_combine(Pf, [u.ptr, v1.ptr, v2.ptr, v3.ptr], un.ptr, ws.ptr, ws.nbytes, stream)
        u, un = un, u
    for p in plans:
        p.close()
    return u


class BrusselatorNonlinearity:
    """g(w) = (a + u^2 v, b u - u^2 v) for w = (u, v), N values each (the reaction terms of
    the Brusselator system of Section 4.4), on the device; out must not alias w."""

    def __init__(self, a: float, b: float, N: int, stream: int = 0):
        self.a, self.b, self.N, self.stream = a, b, N, stream

    def __call__(self, t: float, w_ptr: int, out_ptr: int) -> None:
        N, st = self.N, self.stream
        vector_op(PHIKS_VOP_BRUSS_U, N, self.a, w_ptr, 0.0, w_ptr + 8 * N, out_ptr, st)
        vector_op(PHIKS_VOP_BRUSS_V, N, self.b, w_ptr, 0.0, w_ptr + 8 * N, out_ptr + 8 * N, st)


class _Blocks:
    """The diagonal blocks of K = diag(K_1, K_2, ...): plans per (task, step, p, scales) and
    the phi-action calls of each block on its slice of concatenated device vectors."""

    def __init__(self, blocks, tol, stream):
        self.blocks = [list(A) for A in blocks]
        self.sizes = [int(np.prod([a.shape[0] for a in A])) for A in self.blocks]
        self.offs = [int(sum(self.sizes[:b])) for b in range(len(self.sizes))]
        self.N = int(sum(self.sizes))
        self.tol, self.stream = tol, stream
        self.plans = {}
        self.ws = None
        self.tmp = None

    def prepare(self, keys):
        """Build every plan up front (one workspace for all of them)."""
        for task, h, p, ns in keys:
            for b, A in enumerate(self.blocks):
                self.plans[(task, b, h, p, ns)] = phiks_plan(A, h, p, ns, self.tol, task,
                                                             stream=self.stream)
        self.ws = DeviceArray(max(pl.workspace_size() for pl in self.plans.values()) // 8 + 1)
        width = max(ns * (p + 1 if task == "same_vector" else 1) for task, _, p, ns in keys)
        self.tmp = DeviceArray(width * max(self.sizes))

    def close(self):
        for pl in self.plans.values():
            pl.close()

    def lc(self, h, vptrs, p, ns, outs):
        """outs[j] <- scale j of e^(c_j h K) v_0 + sum_l c_j^l phi_l(c_j h K) v_l (full length)."""
        for b in range(len(self.blocks)):
            off, Nb = 8 * self.offs[b], self.sizes[b]
            pv = [None if x is None else x + off for x in vptrs]
            pl = self.plans[("lincomb", b, h, p, ns)]
            if ns == 1:
                phiks_combine(pl, pv, outs[0] + off, self.ws.ptr, self.ws.nbytes, self.stream)
                continue
            phiks_combine(pl, pv, self.tmp.ptr, self.ws.ptr, self.ws.nbytes, self.stream)
            for j in range(ns):
                memcpy_dtod(outs[j] + off, self.tmp.ptr + 8 * j * Nb, 8 * Nb, self.stream)

    def sv(self, h, v_ptr, p, ns, ell, outs):
        """outs[j] <- phi_ell(h K / 2^j) v (full length), from one same-vector call per block."""
        for b in range(len(self.blocks)):
            off, Nb = 8 * self.offs[b], self.sizes[b]
            pl = self.plans[("same_vector", b, h, p, ns)]
            phiks_apply(pl, v_ptr + off, self.tmp.ptr, self.ws.ptr, self.ws.nbytes, self.stream)
            for j in range(ns):
                memcpy_dtod(outs[j] + off, self.tmp.ptr + 8 * (j * (p + 1) + ell) * Nb, 8 * Nb,
                            self.stream)


def exprk4s5(blocks, w0, g: Callable[[float, int, int], None], T: float, steps: int,
             tol: float = 2.0 ** -53, stream: int = 0, smart: bool = True) -> DeviceArray:
    """Fourth-order five-stage scheme of eq. expRK4s5 (c = (1/2, 1/2, 1, 1/2)) for
    w' = K w + g(t, w) with K block diagonal (blocks[b]: the A_mu of block b; w the
    concatenated state), with phi_{k,j} = phi_k(c_j tau K), D_j = g(t_n + c_j tau, U_j) - g_n:
      U_2 = e^(tau K/2) u_n + tau/2 phi_1(tau K/2) g_n,  U_3 = U_2 + tau phi_{2,3} D_2,
      U_4 = e^(tau K) u_n + tau phi_1(tau K) g_n + tau phi_{2,4} (D_2 + D_3),
      U_5 = U_2 + tau (a_52 (D_2 + D_3 - D_4) + phi_{2,5} D_4 / 4),
      a_52 = phi_{2,5}/2 - phi_{3,4} + phi_{2,4}/4 - phi_{3,5}/2,
      u_{n+1} = e^(tau K) u_n + tau phi_1(tau K) g_n + tau (phi_2 (4 D_5 - D_4) + phi_3 (4 D_4 - 8 D_5)).
    smart=True evaluates the five lines of eq. expRK4s5_smart, two calls per line (one per
    block): the two-scale combination for the phi_1 line, same-vector phi_2 at two scales
    of D_2 and of D_3, the two-scale combination phi_2/4^j D_4 + phi_3/8^j 4 (D_2 + D_3 -
    D_4), and phi_2 (4 D_5 - D_4) + phi_3 (4 D_4 - 8 D_5); smart=False takes the stages one
    by one as combinations (stage 5 in two, since it mixes the steps tau/2 and tau)."""
    tau = T / steps
    h2 = 0.5 * tau
    B = _Blocks(blocks, tol, stream)
    if smart:
        B.prepare([("lincomb", tau, 1, 2), ("same_vector", tau, 2, 2), ("lincomb", tau, 3, 2),
                   ("lincomb", tau, 3, 1)])
    else:
        B.prepare([("lincomb", h2, 1, 1), ("lincomb", h2, 2, 1), ("lincomb", tau, 2, 1),
                   ("lincomb", h2, 3, 1), ("lincomb", tau, 3, 1)])
    N = B.N
    u = _start(w0, N)
    un = DeviceArray(N)
    (gn, U, D2, D3, D4, D5, E0, E1, P20, P21, Q20, Q21, L40, L41, x1, x2, x3,
     tmp) = (DeviceArray(N) for _ in range(18))
    AX = PHIKS_VOP_AXPBY

    def diff(tt, U_ptr, D):
        g(tt, U_ptr, D.ptr)
        vector_op(AX, N, 1.0, D.ptr, -1.0, gn.ptr, D.ptr, stream)

    for n in range(steps):
        t = n * tau
        g(t, u.ptr, gn.ptr)
        if smart:
            vector_op(AX, N, tau, gn.ptr, 0.0, None, x1.ptr, stream)
            B.lc(tau, [u.ptr, x1.ptr], 1, 2, [E0.ptr, E1.ptr])          # scales 1, 1/2
            diff(t + h2, E1.ptr, D2)
            B.sv(tau, D2.ptr, 2, 2, 2, [P20.ptr, P21.ptr])              # phi_2(tau K/2^j) D_2
            vector_op(AX, N, 1.0, E1.ptr, tau, P21.ptr, U.ptr, stream)
            diff(t + h2, U.ptr, D3)
            B.sv(tau, D3.ptr, 2, 2, 2, [Q20.ptr, Q21.ptr])
            vector_op(AX, N, 1.0, P20.ptr, 1.0, Q20.ptr, tmp.ptr, stream)
            vector_op(AX, N, 1.0, E0.ptr, tau, tmp.ptr, U.ptr, stream)
            diff(t + tau, U.ptr, D4)
            vector_op(AX, N, 4.0, D2.ptr, 4.0, D3.ptr, x3.ptr, stream)
            vector_op(AX, N, 1.0, x3.ptr, -4.0, D4.ptr, x3.ptr, stream)
            B.lc(tau, [None, None, D4.ptr, x3.ptr], 3, 2, [L40.ptr, L41.ptr])
            # U_5 = E_1 + tau (1/2 (P2_1 + Q2_1) + 1/4 (P2_0 + Q2_0) - L4_1 - 1/4 L4_0)
            vector_op(AX, N, 0.5, P21.ptr, 0.5, Q21.ptr, x1.ptr, stream)
            vector_op(AX, N, 1.0, x1.ptr, 0.25, tmp.ptr, x1.ptr, stream)
            vector_op(AX, N, 1.0, x1.ptr, -1.0, L41.ptr, x1.ptr, stream)
            vector_op(AX, N, 1.0, x1.ptr, -0.25, L40.ptr, x1.ptr, stream)
            vector_op(AX, N, 1.0, E1.ptr, tau, x1.ptr, U.ptr, stream)
            diff(t + h2, U.ptr, D5)
            vector_op(AX, N, 4.0, D5.ptr, -1.0, D4.ptr, x2.ptr, stream)
            vector_op(AX, N, 4.0, D4.ptr, -8.0, D5.ptr, x3.ptr, stream)
            B.lc(tau, [None, None, x2.ptr, x3.ptr], 3, 1, [tmp.ptr])
            vector_op(AX, N, 1.0, E0.ptr, tau, tmp.ptr, un.ptr, stream)
        else:
            vector_op(AX, N, h2, gn.ptr, 0.0, None, x1.ptr, stream)
            B.lc(h2, [u.ptr, x1.ptr], 1, 1, [U.ptr])
            diff(t + h2, U.ptr, D2)
            vector_op(AX, N, tau, D2.ptr, 0.0, None, x2.ptr, stream)
            B.lc(h2, [u.ptr, x1.ptr, x2.ptr], 2, 1, [U.ptr])
            diff(t + h2, U.ptr, D3)
            vector_op(AX, N, tau, gn.ptr, 0.0, None, E0.ptr, stream)          # tau g_n
            vector_op(AX, N, tau, D2.ptr, tau, D3.ptr, x2.ptr, stream)
            B.lc(tau, [u.ptr, E0.ptr, x2.ptr], 2, 1, [U.ptr])
            diff(t + tau, U.ptr, D4)
            vector_op(AX, N, 1.0, D2.ptr, 1.0, D3.ptr, tmp.ptr, stream)
            vector_op(AX, N, 1.0, tmp.ptr, -1.0, D4.ptr, tmp.ptr, stream)      # D = D2 + D3 - D4
            vector_op(AX, N, 0.5 * tau, tmp.ptr, 0.25 * tau, D4.ptr, x2.ptr, stream)
            vector_op(AX, N, -0.5 * tau, tmp.ptr, 0.0, None, x3.ptr, stream)
            B.lc(h2, [u.ptr, x1.ptr, x2.ptr, x3.ptr], 3, 1, [U.ptr])
            vector_op(AX, N, 0.25 * tau, tmp.ptr, 0.0, None, x2.ptr, stream)
            vector_op(AX, N, -tau, tmp.ptr, 0.0, None, x3.ptr, stream)
            B.lc(tau, [None, None, x2.ptr, x3.ptr], 3, 1, [E1.ptr])
            vector_op(AX, N, 1.0, U.ptr, 1.0, E1.ptr, U.ptr, stream)
            diff(t + h2, U.ptr, D5)
            vector_op(AX, N, 4.0 * tau, D5.ptr, -tau, D4.ptr, x2.ptr, stream)
            vector_op(AX, N, 4.0 * tau, D4.ptr, -8.0 * tau, D5.ptr, x3.ptr, stream)
            B.lc(tau, [u.ptr, E0.ptr, x2.ptr, x3.ptr], 3, 1, [un.ptr])
        u, un = un, u
    B.close()
    return u
