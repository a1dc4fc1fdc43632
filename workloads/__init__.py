"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module builds *inputs only*: the small matrices A_mu of a Kronecker sum
K = A_d (+) ... (+) A_1 and the vectors the phi-functions act on.  It holds none of
the method's arithmetic (no quadrature, no exponentials, no mu-mode products), so
that the oracle and the GPU path can both draw the same data without sharing code.

Layout convention (Lemma 1 of the paper, Section 2): a vector v of length
N = n_1 * ... * n_d is vec(V) of the order-d tensor V, stacked by columns, i.e. the
index i_1 runs fastest.  As a NumPy array that is the C-ordered shape
(n_d, ..., n_1).  Matrices are dense float64 (or complex128), row-major, A[i, j]
being the coefficient of u_j in row i.

The operators follow the discretisations the paper uses (Section 1 and Section 4):
second-order finite differences with homogeneous Dirichlet boundary conditions on a
uniform grid of [0, 1] with h = 1/(n+1), central differences for advection, and
(for batched workloads) Chebyshev spectral second-derivative matrices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "fd2_dirichlet", "central_adv_dirichlet", "adr_1d", "cheb_d2_dirichlet",
    "randn_vec", "uniform_vec", "Workload", "config_fd2_2d", "config_allen_cahn_3d",
    "config_adr_3d", "validation_table1", "BatchProblem", "config_batch",
    "fd2_neumann", "Session", "serving_sessions", "poisson_arrivals", "ADRProblem",
    "adr_integration_problem", "BrusselatorProblem", "brusselator_problem",
]


def fd2_dirichlet(n: int, length: float = 1.0) -> np.ndarray:
    """tridiag(1, -2, 1)/h^2 on n interior points of [0, length], h = length/(n+1)."""
    h = length / (n + 1)
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx, idx] = -2.0
    A[idx[:-1], idx[:-1] + 1] = 1.0
    A[idx[1:], idx[1:] - 1] = 1.0
    return A / (h * h)


def central_adv_dirichlet(n: int, beta: float, length: float = 1.0) -> np.ndarray:
    """beta * (u_{i+1} - u_{i-1}) / (2h), homogeneous Dirichlet, h = length/(n+1)."""
    h = length / (n + 1)
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx[:-1], idx[:-1] + 1] = 1.0
    A[idx[1:], idx[1:] - 1] = -1.0
    return (beta / (2.0 * h)) * A


def adr_1d(n: int, eps: float, beta: float, react: float) -> np.ndarray:
    """eps * FD2 + central advection with speed beta + react * I (one direction)."""
    return eps * fd2_dirichlet(n) + central_adv_dirichlet(n, beta) + react * np.eye(n)


def cheb_d2_dirichlet(n: int) -> np.ndarray:
    """Chebyshev second-derivative matrix on the n interior Chebyshev-Lobatto points
    of [-1, 1] (Dirichlet: first and last rows/columns of the (n+2)-point matrix removed).
    Dense, nonsymmetric; spectral radius grows like n^4."""
    m = n + 1
    x = np.cos(np.pi * np.arange(m + 1) / m)
    c = np.ones(m + 1)
    c[0] = c[-1] = 2.0
    c *= (-1.0) ** np.arange(m + 1)
    X = np.tile(x, (m + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1.0 / c) / (dX + np.eye(m + 1))
    D -= np.diag(D.sum(axis=1))
    D2 = D @ D
    return np.ascontiguousarray(D2[1:-1, 1:-1])


def randn_vec(n: Sequence[int], seed: int) -> np.ndarray:
    """v ~ N(0, 1) in vec order (i_1 fastest), float64."""
    N = int(np.prod(n))
    return np.random.default_rng(seed).standard_normal(N)


def uniform_vec(n: Sequence[int], seed: int, lo: float, hi: float) -> np.ndarray:
    N = int(np.prod(n))
    return np.random.default_rng(seed).uniform(lo, hi, N)


def grid_1d(n: int) -> np.ndarray:
    """Interior grid points of [0, 1] with h = 1/(n+1)."""
    return np.arange(1, n + 1) / (n + 1)


@dataclass
class Workload:
    """One phi-action problem: operators, step, vectors and requested outputs."""
    name: str
    n: List[int]                       # n[0] = n_1 (fastest index)
    A: List[np.ndarray]                # A[mu-1] = A_mu
    tau: float
    p: int                             # highest phi index
    n_scales: int                      # number of time scales requested
    task: str                          # "same_vector" or "lincomb"
    tol: float                         # relative tolerance (norms taken as 1)
    v: Optional[np.ndarray] = None     # same-vector input
    vs: Optional[List[Optional[np.ndarray]]] = None   # lincomb inputs v_0..v_p
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def d(self) -> int:
        return len(self.n)


def config_fd2_2d(n: int = 32, tau: float = 1e-3, seed: int = 0, p: int = 3) -> Workload:
    """2D FD Laplacian, Dirichlet, n x n, phi_0..phi_p on one N(0,1) vector."""
    A = fd2_dirichlet(n)
    return Workload(name=f"fd2_2d_{n}x{n}", n=[n, n], A=[A, A.copy()], tau=tau, p=p,
                    n_scales=1, task="same_vector", tol=2.0 ** -53,
                    v=randn_vec([n, n], seed))


def config_allen_cahn_3d(n: int = 64, tau: float = 1e-3, seed: int = 1,
                         eps: float = 0.01, p: int = 4) -> Workload:
    """3D Allen-Cahn u' = eps*Lap(u) + u - u^3 with FD Dirichlet Laplacian.  The linear
    part K is eps*Lap (the +u term is kept in g); one linear combination
    exp(tau K) v_0 + sum_l phi_l(tau K) v_l with v_0 = u_0, v_l = tau*g(u_0)."""
    A = eps * fd2_dirichlet(n)
    u0 = uniform_vec([n, n, n], seed, -0.9, 0.9)
    g = u0 - u0 ** 3
    vs = [u0] + [tau * g for _ in range(p)]
    return Workload(name=f"allen_cahn_3d_{n}^3", n=[n, n, n], A=[A, A.copy(), A.copy()],
                    tau=tau, p=p, n_scales=2, task="lincomb", tol=2.0 ** -53, vs=vs,
                    meta={"eps": eps})


def config_adr_3d(n: int = 256, tau: float = 1e-3, seed: int = 2, p: int = 4,
                  betas=(1.0, 0.5, 0.25), eps: float = 0.5, react: float = -1.0) -> Workload:
    """3D advection-diffusion-reaction: A_mu = eps*FD2 + beta_mu*central_adv + react*I."""
    A = [adr_1d(n, eps, b, react) for b in betas]
    return Workload(name=f"adr_3d_{n}^3", n=[n, n, n], A=A, tau=tau, p=p, n_scales=1,
                    task="same_vector", tol=2.0 ** -53, v=randn_vec([n, n, n], seed),
                    meta={"betas": list(betas), "eps": eps, "react": react})


def validation_table1(d: int, n: int):
    """The code-validation operators of Section 4.1: A_mu = FD2 of (1+i)/100 * Lap on
    [0,1]^d (Dirichlet) and v = samples of 4096(1+i) prod_mu x_mu(1-x_mu).
    Returns (A list of complex matrices, v complex vector in vec order)."""
    A = (1.0 + 1.0j) / 100.0 * fd2_dirichlet(n)
    x = grid_1d(n)
    f = x * (1.0 - x)
    v = np.array([1.0 + 0.0j])
    for _ in range(d):
        v = np.kron(f, v)          # i_1 fastest: new (slower) index on the left
    v = 4096.0 * (1.0 + 1.0j) * v
    return [A.copy() for _ in range(d)], v


@dataclass
class BatchProblem:
    """One problem of a batch: phi_0..phi_p of tau K on v, K = A_d (+) ... (+) A_1."""
    n: List[int]
    A: List[np.ndarray]
    tau: float
    v: np.ndarray

    @property
    def N(self) -> int:
        return int(np.prod(self.n))


BATCH_SIZES = (16, 24, 32, 48, 64, 96, 128)


def config_batch(count: int = 512, seed: int = 3, sizes: Sequence[int] = BATCH_SIZES,
                 tau_range=(1e-4, 1e-2)) -> List[BatchProblem]:
    """Many uneven problems: d in {2, 3} with equal probability, each n_mu drawn
    uniformly from `sizes`, A_mu the Dirichlet Chebyshev second-derivative matrix of
    size n_mu, tau log-uniform in tau_range, v ~ N(0, 1).  Shared settings of such a
    batch: p = 3, one scale, tolerance 2^-53 ||v||_2."""
    rng = np.random.default_rng(seed)
    cache = {}
    out = []
    for _ in range(count):
        d = int(rng.integers(2, 4))
        n = [int(x) for x in rng.choice(np.asarray(sizes), size=d)]
        tau = float(np.exp(rng.uniform(np.log(tau_range[0]), np.log(tau_range[1]))))
        for m in n:
            if m not in cache:
                cache[m] = cheb_d2_dirichlet(m)
        vseed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(BatchProblem(n=n, A=[cache[m].copy() for m in n], tau=tau,
                                v=randn_vec(n, vseed)))
    return out


def fd2_neumann(n: int, length: float = 1.0) -> np.ndarray:
    """Second difference on n grid points of [0, length] including both ends
    (h = length/(n-1)), homogeneous Neumann conditions by ghost reflection
    (u_{-1} = u_1, u_n = u_{n-2}): rows 0 and n-1 read (-2, 2)/h^2."""
    h = length / (n - 1)
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx, idx] = -2.0
    A[idx[:-1], idx[:-1] + 1] = 1.0
    A[idx[1:], idx[1:] - 1] = 1.0
    A[0, 1] = 2.0
    A[n - 1, n - 2] = 2.0
    return A / (h * h)


@dataclass
class Session:
    """A stream of requests sharing one operator, step and phi order (a time stepper
    calling the same phi-functions every step): phi_0..phi_p of tau K, one scale."""
    name: str
    n: List[int]
    A: List[np.ndarray]
    tau: float
    p: int

    @property
    def N(self) -> int:
        return int(np.prod(self.n))


SERVING_SHAPES = ([256, 256], [1024, 1024], [64, 64, 64], [128, 128, 128], [192, 192, 192])


def serving_sessions(count: int = 12, seed: int = 4, shapes=SERVING_SHAPES) -> List[Session]:
    """Sessions of the serving workload: shape drawn from `shapes`; operator one of
    the FD2 Laplacian (Dirichlet), advection-diffusion-reaction (eps = 0.5, beta =
    (1, 0.5, 0.25) per direction, reaction -1 split over the directions as in the ADR
    workload) or the diffusion part of a Brusselator-type system (d = 0.02 times the
    Neumann Laplacian with the shift -(b+1) = -4 split evenly over the directions);
    p in 1..4; tau log-uniform in [1e-4, 1e-2]."""
    rng = np.random.default_rng(seed)
    kinds = ("fd2", "adr", "bruss")
    out = []
    for k in range(count):
        n = list(shapes[int(rng.integers(len(shapes)))])
        kind = kinds[int(rng.integers(len(kinds)))]
        d = len(n)
        if kind == "fd2":
            A = [fd2_dirichlet(m) for m in n]
        elif kind == "adr":
            betas = (1.0, 0.5, 0.25)
            A = [adr_1d(m, 0.5, betas[j], -1.0) for j, m in enumerate(n)]
        else:
            A = [0.02 * fd2_neumann(m) - (4.0 / d) * np.eye(m) for m in n]
        tau = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        p = int(rng.integers(1, 5))
        out.append(Session(name=f"{kind}_{'x'.join(map(str, n))}", n=n, A=A, tau=tau, p=p))
    return out


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return np.asarray(out)
        out.append(t)


@dataclass
class ADRProblem:
    """The evolutionary advection-diffusion-reaction problem of Section 4.2:
    u_t = eps Lap u + alpha (d_1 + d_2 + d_3) u + 1/(1 + u^2) + Psi(t, x) on [0,1]^3,
    homogeneous Dirichlet, u_0 = 64 prod x_j (1 - x_j), Psi chosen so that the exact
    solution is e^t u_0.  Semi-discretised with n interior points per direction
    (second-order centred differences, exact for this u_0), K = A_3 (+) A_2 (+) A_1 with
    A_mu = eps FD2 + alpha central_adv.  Then Psi(t) = e^t w - 1/(1 + e^(2t) u_0^2) with
    w = u_0 - eps Lap u_0 - alpha sum_j d_j u_0 (analytic, at the grid points)."""
    n: int
    eps: float
    alpha: float
    A: List[np.ndarray]
    u0: np.ndarray
    w: np.ndarray

    def exact(self, t: float) -> np.ndarray:
        return math.exp(t) * self.u0


def adr_integration_problem(n: int = 20, eps: float = 0.5, alpha: float = 10.0) -> ADRProblem:
    x = grid_1d(n)
    f = x * (1.0 - x)            # f_j(x) = x (1 - x)
    df = 1.0 - 2.0 * x           # f'
    d2f = -2.0 * np.ones_like(x)  # f''

    def tens(a, b, c):           # vec order: x_1 fastest
        return np.kron(c, np.kron(b, a))

    u0 = 64.0 * tens(f, f, f)
    lap = 64.0 * (tens(d2f, f, f) + tens(f, d2f, f) + tens(f, f, d2f))
    grad = 64.0 * (tens(df, f, f) + tens(f, df, f) + tens(f, f, df))
    w = u0 - eps * lap - alpha * grad
    Amu = eps * fd2_dirichlet(n) + central_adv_dirichlet(n, alpha)
    return ADRProblem(n=n, eps=eps, alpha=alpha, A=[Amu.copy() for _ in range(3)], u0=u0, w=w)



@dataclass
class BrusselatorProblem:
    """The two-species Brusselator system of Section 4.4 on [0, 1]^d with homogeneous
    Neumann conditions: u' = d_1 Lap u - (b + 1) u + a + u^2 v, v' = d_2 Lap v + b u - u^2 v,
    u_0 = 64^2 prod x_j^2 (1 - x_j)^2 (the paper's d = 3 form, 4^(2d) in general),
    v_0 = c.  Semi-discretised on n grid points per direction including both ends with
    the Neumann second difference of fd2_neumann (reading: the paper's fourth-order
    closure is not stated).  K is block diagonal: blocks[0] the A_mu of K_1 = d_1 Lap -
    (b + 1) (the shift split evenly over the directions), blocks[1] those of
    K_2 = d_2 Lap.  The state w = (u, v) is concatenated in vec order."""
    n: int
    d: int
    a: float
    b: float
    blocks: List[List[np.ndarray]]
    w0: np.ndarray

    @property
    def N(self) -> int:
        return self.n ** self.d


def brusselator_problem(n: int = 10, d: int = 3, a: float = 1.0, b: float = 3.0,
                        c: float = 1.0, d1: float = 0.02, d2: float = 0.02) -> BrusselatorProblem:
    x = np.arange(n) / (n - 1)
    f = (4.0 * x * (1.0 - x)) ** 2      # per direction: 4^2 x^2 (1 - x)^2
    u0 = np.array([1.0])
    for _ in range(d):
        u0 = np.kron(f, u0)              # i_1 fastest
    L = fd2_neumann(n)
    K1 = [d1 * L - ((b + 1.0) / d) * np.eye(n) for _ in range(d)]
    K2 = [d2 * L for _ in range(d)]
    w0 = np.concatenate([u0, c * np.ones(n ** d)])
    return BrusselatorProblem(n=n, d=d, a=a, b=b, blocks=[K1, K2], w0=w0)
