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

from . import (PHIKS_VOP_AXPBY, PHIKS_VOP_CUBIC, PHIKS_VOP_RATIONAL, DeviceArray, phiks_combine,
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
