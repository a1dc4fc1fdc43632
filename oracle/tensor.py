"""mu-mode product and Tucker operator (oracle), Section 2 of the paper.

vec(V) stacks by columns (Lemma 1): the first index i_1 runs fastest.  A vector of
length N = n_1...n_d is therefore viewed as the C-ordered NumPy array of shape
(n_d, ..., n_1); mode mu is axis d - mu of that array.

The mu-mode product V x_mu L has entries
    w_{i_1..i_d} = sum_j v_{i_1..i_{mu-1} j i_{mu+1}..i_d} L[i_mu, j],
computed here by explicit loops over the output entries and j (``loops.c``, plain
C compiled with gcc on first use; OpenMP over the outer loops).  Complex operands
are split into real and imaginary parts, each part a real loop product.
``mode_product_tensordot`` (one library contraction) and ``mode_product_loops``
(pure Python, tiny sizes) are independent forms used only to pin the loops.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "loops.c")
_LIB = os.path.join(_HERE, "liboracle_loops.so")
_loops = None


def build_loops(force: bool = False) -> str:
    """Compile loops.c into liboracle_loops.so next to it (gcc -O2 -fopenmp) when the
    library is missing, older than its source, or `force` is set."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=_HERE)
    os.close(fd)
    try:
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp],
                       check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        os.replace(tmp, _LIB)
    finally:
        if os.path.exists(tmp):
            os.unlink(tmp)
    return _LIB


def _lib():
    global _loops
    if _loops is None:
        lib = ctypes.CDLL(build_loops())
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_mode_product.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                            dp, dp, dp, dp]
        lib.oracle_mode_product.restype = None
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _loops = lib
    return _loops


def threads() -> int:
    """OpenMP threads the loop products run on."""
    return int(_lib().oracle_threads())


def set_threads(n: int) -> None:
    """Run the loop products on n OpenMP threads from now on."""
    _lib().oracle_set_threads(int(n))


def _real_loops(v: np.ndarray, nlo: int, nmu: int, nhi: int, L: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
    L = np.ascontiguousarray(L, dtype=np.float64)
    Lt = np.ascontiguousarray(L.T)
    w = np.empty_like(v)
    dp = ctypes.POINTER(ctypes.c_double)
    _lib().oracle_mode_product(nlo, nmu, nhi, L.ctypes.data_as(dp), Lt.ctypes.data_as(dp),
                               v.ctypes.data_as(dp), w.ctypes.data_as(dp))
    return w


def as_tensor(v: np.ndarray, n: Sequence[int]) -> np.ndarray:
    return np.asarray(v).reshape(tuple(reversed(list(n))))


def mode_product(V: np.ndarray, L: np.ndarray, mu: int) -> np.ndarray:
    """V x_mu L for V of shape (n_d, ..., n_1) and 1-based mode mu, by loops."""
    shape = V.shape
    n = list(reversed(shape))                     # n[0] = n_1
    nlo = int(np.prod(n[: mu - 1])) if mu > 1 else 1
    nmu = n[mu - 1]
    nhi = int(np.prod(n[mu:])) if mu < len(n) else 1
    L = np.asarray(L)
    assert L.shape == (nmu, nmu)
    if np.iscomplexobj(V) or np.iscomplexobj(L):
        Vr, Vi = np.real(V).reshape(-1), np.imag(V).reshape(-1)
        Lr, Li = np.real(L), np.imag(L)
        re = _real_loops(Vr, nlo, nmu, nhi, Lr) - _real_loops(Vi, nlo, nmu, nhi, Li)
        im = _real_loops(Vi, nlo, nmu, nhi, Lr) + _real_loops(Vr, nlo, nmu, nhi, Li)
        return (re + 1j * im).reshape(shape)
    return _real_loops(V, nlo, nmu, nhi, L).reshape(shape)


def mode_product_tensordot(V: np.ndarray, L: np.ndarray, mu: int) -> np.ndarray:
    """The same product as one library contraction (pins only)."""
    ax = V.ndim - mu
    W = np.tensordot(L, V, axes=([1], [ax]))      # new axis 0 is i_mu
    return np.ascontiguousarray(np.moveaxis(W, 0, ax))


def tucker(v: np.ndarray, n: Sequence[int], Ls: Sequence[np.ndarray]) -> np.ndarray:
    """vec(V x_1 L_1 x_2 ... x_d L_d) for v = vec(V); Ls[mu-1] = L_mu."""
    V = as_tensor(v, n)
    for mu, L in enumerate(Ls, start=1):
        V = mode_product(V, L, mu)
    return V.reshape(-1)


def mode_product_loops(v: np.ndarray, n: Sequence[int], L: np.ndarray, mu: int) -> np.ndarray:
    """Same as mode_product, written as explicit loops over the mu-fibres (tiny sizes only)."""
    n = list(n)
    nlo = int(np.prod(n[: mu - 1])) if mu > 1 else 1
    nmu = n[mu - 1]
    nhi = int(np.prod(n[mu:])) if mu < len(n) else 1
    out = np.zeros(len(v), dtype=np.result_type(v, L))
    for b in range(nhi):
        for a in range(nlo):
            for i in range(nmu):
                acc = 0.0
                for j in range(nmu):
                    acc += L[i, j] * v[a + nlo * (j + nmu * b)]
                out[a + nlo * (i + nmu * b)] = acc
    return out


def kron_sum_dense(A: Sequence[np.ndarray]) -> np.ndarray:
    """K = A_d (+) ... (+) A_1 = sum_mu I x .. x A_mu x .. x I assembled densely (pins only)."""
    n = [a.shape[0] for a in A]
    N = int(np.prod(n))
    dt = np.result_type(*A)
    K = np.zeros((N, N), dtype=dt)
    for mu in range(len(A)):
        M = np.ones((1, 1), dtype=dt)
        for nu in range(len(A)):             # build I_d x ... x I_1 from the slow end
            factor = A[nu] if nu == mu else np.eye(n[nu])
            M = np.kron(factor, M)
        K = K + M
    return K


def kron_sum_apply(A: Sequence[np.ndarray], v: np.ndarray) -> np.ndarray:
    """K v without forming K: sum over mu of V x_mu A_mu."""
    n = [a.shape[0] for a in A]
    V = as_tensor(v, n)
    out = np.zeros_like(V, dtype=np.result_type(V, *A))
    for mu, a in enumerate(A, start=1):
        out = out + mode_product(V, a, mu)
    return out.reshape(-1)
