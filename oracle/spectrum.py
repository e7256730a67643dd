"""Spectral interval of the 1D pencil (A_Y, M_Y) (oracle; test infrastructure only).

Alg. 2 (Sec. 5) needs intervals [a, b] containing sigma(A, D) = sigma(A_Y^x, M^x)
and [c, d] containing sigma(B, C) = sigma(-A_Y^y, M^y); the paper computes the
generalised eigenvalues with a banded eigensolver (Crawford).  Here:

* lower end, closed form (a reading; the paper only cites the eigensolver):
  Dirichlet  a = pi^2 / l^2 + omega^2 / 2 (l the interval length): a Galerkin
             eigenvalue is never below the continuous one it approximates;
  Neumann    a = omega^2 / 2 exactly (constants lie in the space, K 1 = 0);
* upper end: the largest generalised eigenvalue from a library eigensolver
  (dense LAPACK for small N, sparse shift-invert Lanczos otherwise);
* the rigorous bounds of Lemma "Spectrum" (Sec. 5.2):
  sigma(L^{-T} M L^{-1}) in [2h^2/(24p^4 + omega^2 h^2), C], whose reciprocals
  bound sigma(A_Y, M).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .basis import DIRICHLET, Operators1D


def lower_end(ops: Operators1D, omega2: float) -> float:
    B = ops.basis
    if B.bc == DIRICHLET:
        ell = B.x[-1] - B.x[0]
        return math.pi ** 2 / ell ** 2 + omega2 / 2.0
    return omega2 / 2.0


def extreme_eigenvalues(ops: Operators1D, omega2: float):
    """(lambda_min, lambda_max) of A_Y v = lambda M v from a library eigensolver."""
    A = ops.A(omega2)
    M = ops.M
    N = A.shape[0]
    if N <= 1500:
        w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
        return float(w[0]), float(w[-1])
    lmax = spla.eigsh(A.tocsc(), k=1, M=M.tocsc(), which="LA", return_eigenvectors=False,
                      tol=1e-12)[0]
    lmin = spla.eigsh(A.tocsc(), k=1, M=M.tocsc(), sigma=0.0, which="LM",
                      return_eigenvectors=False, tol=1e-12)[0]
    return float(lmin), float(lmax)


def interval(ops: Operators1D, omega2: float):
    """[a, b] with the closed-form lower end and the computed largest eigenvalue."""
    return lower_end(ops, omega2), extreme_eigenvalues(ops, omega2)[1]


def lemma_bounds(ops: Operators1D, omega2: float):
    """Bounds on sigma(A_Y, M) implied by Lemma "Spectrum" (Sec. 5.2):
    lambda(A_Y, M) = 1 / lambda(L^{-T} M L^{-1}) lies in [1/C, (24p^4 + omega^2 h^2)/(2h^2)],
    h the smallest element, C = min(l^2/pi^2, max(1, 2/omega^2)) (Dirichlet) or
    max(1, 2/omega^2) (Neumann; omega != 0)."""
    B = ops.basis
    h = float(np.min(B.delta))
    p = B.p
    upper = (24.0 * p ** 4 + omega2 * h * h) / (2.0 * h * h)
    big = max(1.0, 2.0 / omega2) if omega2 > 0 else math.inf
    if B.bc == DIRICHLET:
        ell = B.x[-1] - B.x[0]
        C = min(ell ** 2 / math.pi ** 2, big)
    else:
        C = big
    return 1.0 / C, upper
