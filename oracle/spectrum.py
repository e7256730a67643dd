"""Spectral interval of the 1D pencil (A_Y, M_Y) (oracle; test infrastructure only).

Alg. 2 (Sec. 5) needs intervals [a, b] containing sigma(A, D) = sigma(A_Y^x, M^x)
and [c, d] containing sigma(B, C) = sigma(-A_Y^y, M^y); the paper computes the
generalised eigenvalues with a banded eigensolver (Crawford).  Here:

* lower end (a reading; the paper only cites the eigensolver): the smallest
  eigenvalue k^2 of -u'' = lambda u on the interval (length l) with the same end
  conditions, plus omega^2 / 2: a Galerkin eigenvalue is never below the continuous
  one it approximates (Rayleigh-Ritz).  With u = sin(k x + phi_l), an end condition
  alpha u + du/dn = 0 fixes the phase by tan(phi) = k / alpha (Dirichlet: phi = 0,
  Neumann: phi = pi/2), and the other end closes it: k l + phi_l + phi_r = pi.  Both
  phases grow with k, so the smallest root is found by bisection on (0, pi / l];
  Dirichlet at both ends gives pi^2 / l^2, Neumann at both 0, one of each (pi/(2l))^2;
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


def _phase(kind: str, alpha: float, k: float) -> float:
    if kind == DIRICHLET:
        return 0.0
    return math.atan2(k, alpha)  # Neumann: alpha = 0 gives pi/2


def continuous_lowest(B) -> float:
    """Smallest eigenvalue of -u'' = lambda u on [x_0, x_n] with B's end conditions."""
    ell = B.x[-1] - B.x[0]
    (kl, kr), (al, ar) = B.ends, B.alpha
    def f(k):
        return k * ell + _phase(kl, al, k) + _phase(kr, ar, k) - math.pi
    if f(0.0) >= 0.0:          # Neumann at both ends: constants
        return 0.0
    lo, hi = 0.0, math.pi / ell
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return lo * lo


def lower_end(ops: Operators1D, omega2: float, kap: float = 1.0, sig=None) -> float:
    """Lower end of sigma(kap K + sig M, M) (sig defaults to omega^2 / 2)."""
    sig = omega2 / 2.0 if sig is None else sig
    return kap * continuous_lowest(ops.basis) + sig


def extreme_eigenvalues(ops: Operators1D, omega2: float, kap: float = 1.0, sig=None):
    """(lambda_min, lambda_max) of (kap K + sig M) v = lambda M v from a library eigensolver
    (sig defaults to omega^2 / 2, i.e. A_Y)."""
    A = ops.A(omega2) if (kap == 1.0 and sig is None) else (kap * ops.K + (omega2 / 2.0 if sig is None else sig) * ops.M).tocsr()
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


def interval(ops: Operators1D, omega2: float, kap: float = 1.0, sig=None):
    """[a, b] with the continuous lower end and the computed largest eigenvalue."""
    return lower_end(ops, omega2, kap, sig), extreme_eigenvalues(ops, omega2, kap, sig)[1]


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
    if B.ends == (DIRICHLET, DIRICHLET):
        ell = B.x[-1] - B.x[0]
        C = min(ell ** 2 / math.pi ** 2, big)
    else:
        C = big
    return 1.0 / C, upper
