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
