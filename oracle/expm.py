"""Small-matrix exponential for the oracle: scaled Taylor series plus squaring.

The paper evaluates the exponentials of the small matrices with a double-precision
Pade scaling-and-squaring code (Section 4, first paragraph).  The oracle instead
writes out the definition exp(X) = sum_k X^k / k!: X is scaled by 2^-t so that
||X / 2^t||_1 <= 1/2, the series is summed until the next term cannot change the
result in double precision, and the result is squared t times.  It is slower than
Pade but is the plain definition, and it shares no code with the GPU path.
"""
from __future__ import annotations

import math

import numpy as np


def expm_taylor(X: np.ndarray) -> np.ndarray:
    X = np.asarray(X)
    n = X.shape[0]
    if n == 0:
        return X.copy()
    nrm = float(np.abs(X).sum(axis=0).max())
    t = 0
    if nrm > 0.5:
        t = int(math.ceil(math.log2(nrm / 0.5)))
    Y = X / (2.0 ** t)
    ynrm = nrm / (2.0 ** t)
    S = np.eye(n, dtype=Y.dtype)
    term = np.eye(n, dtype=Y.dtype)
    # ||Y||_1 <= 1/2: the tail after degree k is below 2 * 0.5^(k+1)/(k+1)!
    for k in range(1, 60):
        term = term @ Y / k
        S = S + term
        if ynrm ** (k + 1) / math.factorial(k + 1) * 2.0 < 2.0 ** -64:
            break
    for _ in range(t):
        S = S @ S
    return S
