"""Oracle: triangle quadrature for face samples (test infrastructure only).

The paper integrates each face overlap with "2D Gauss quadrature" on
fan sub-triangles (Sec. 4.1, face samples) without naming the rule.  The hot
path samples whole slave triangles with a fixed n x n rule (n*n samples per
triangle).  Reading taken: the Stroud conical-product rule, which has n*n
points, strictly positive weights (a negative mortar weight would flip the
sign of a barrier term) and is exact for polynomials of total degree 2n-1.

Construction (Duffy map of the unit square onto the reference triangle):
  xi  = u_i,             u_i: Gauss-Jacobi(alpha=1, beta=0) nodes on [0,1],
  eta = v_j (1 - u_i),   v_j: Gauss-Legendre nodes on [0,1],
  w   = W_i W_j,         sum w = 1/2 (the reference-triangle area).
Slave barycentrics of the sample are beta^s = (1 - xi - eta, xi, eta).

The Gauss nodes come from scipy / numpy library routines (a library
primitive standing in for one step of the definition).
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi


def stroud_rule(n: int) -> np.ndarray:
    """Return an (n*n, 3) float64 array of (xi, eta, w) for q = i*n + j."""
    if n < 1:
        raise ValueError("rule order must be >= 1")
    # Gauss-Jacobi on [-1,1] with weight (1-x)^1 (1+x)^0, mapped to [0,1]:
    # u = (1+x)/2, (1-u) du = (1-x)/2 dx/2  =>  W = w/4.
    xj, wj = roots_jacobi(n, 1.0, 0.0)
    u = (1.0 + xj) / 2.0
    wu = wj / 4.0
    # Gauss-Legendre on [-1,1] mapped to [0,1]: v = (1+x)/2, W = w/2.
    xl, wl = np.polynomial.legendre.leggauss(n)
    v = (1.0 + xl) / 2.0
    wv = wl / 2.0
    out = np.empty((n * n, 3))
    for i in range(n):
        for j in range(n):
            q = i * n + j
            out[q, 0] = u[i]
            out[q, 1] = v[j] * (1.0 - u[i])
            out[q, 2] = wu[i] * wv[j]
    return out
