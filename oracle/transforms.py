"""Transforms between grid values and coefficients, and the Burgers IMEX step
(oracle; test infrastructure only).  Sec. 6 ("Transforms and time-evolution").

* Grid: on each element the m = p + 1 Chebyshev points of the first kind,
  x_k = sin(pi (m - 2k + 1) / (2m)), k = 1..m, mapped affinely to the element
  (a reading: the paper's "p points" for degrees 0..p is read as p + 1 points, so
  that the transform is square and invertible; the points run from right to left
  as the formula gives them).  Values are stored element-major: index e m + k - 1.
* F_p: values at those points -> Legendre coefficients of degrees 0..p (the
  interpolant), stored degree-major (k n + e) like every Legendre array here.
  The paper composes a DCT with a fast Chebyshev-Legendre transform; this oracle
  solves the interpolation system with the Legendre Vandermonde matrix (library
  routine), which defines the same map.  F_p^{-1} evaluates the series.
  In 2D: F F_p^x ... applied to rows and columns, V -> F_x V F_y^T.
* R and D: Q-basis coefficients -> Legendre coefficients of the function and of its
  x-derivative (the connection and derivative relations of Sec. 2.2, from
  oracle/basis.py).
* Burgers (u_t + u u_x = eps Laplace u, zero Dirichlet), one step of the splitting
  of Sec. 6: implicit Euler for the linear part, u_{k+1/2} = (I - dt eps Laplace)^{-1}
  u_k, solved as the screened problem omega^2 = 1 / (dt eps) with right-hand side
  omega^2 u_k; then explicit Euler for the nonlinear part at the grid points,
  u_{k+1} = u_{k+1/2} - dt u_{k+1/2} d/dx u_{k+1/2} (a reading: the paper prints a
  plus sign, the PDE as written needs the minus), transformed back to Legendre
  coefficients.
"""
from __future__ import annotations

import numpy as np

from .basis import Basis1D, connection_full, derivative_full, restriction
from . import adi as _adi


def chebyshev_points(m: int) -> np.ndarray:
    """x_k = sin(pi (m - 2k + 1) / (2m)), k = 1..m (first kind, descending)."""
    k = np.arange(1, m + 1)
    return np.sin(np.pi * (m - 2 * k + 1) / (2.0 * m))


def grid(B: Basis1D) -> np.ndarray:
    """Physical grid points, element-major (element e owns indices e m .. e m + m - 1)."""
    t = chebyshev_points(B.p + 1)
    return np.concatenate([B.x[e] + (t + 1.0) * B.delta[e] / 2.0 for e in range(B.n)])


def _vandermonde(p: int) -> np.ndarray:
    """V[k, j] = P_j(t_k) at the m = p + 1 reference points."""
    return np.polynomial.legendre.legvander(chebyshev_points(p + 1), p)


def values_to_legendre_1d(B: Basis1D, v: np.ndarray) -> np.ndarray:
    """F_p on every element: element-major values (n m, ...) -> degree-major coefficients."""
    m = B.p + 1
    V = _vandermonde(B.p)
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros((B.Nleg,) + v.shape[1:])
    for e in range(B.n):
        c = np.linalg.solve(V, v[e * m:(e + 1) * m])
        for k in range(m):
            out[k * B.n + e] = c[k]
    return out


def legendre_to_values_1d(B: Basis1D, c: np.ndarray) -> np.ndarray:
    """F_p^{-1}: degree-major coefficients -> element-major values."""
    m = B.p + 1
    V = _vandermonde(B.p)
    c = np.asarray(c, dtype=np.float64)
    out = np.zeros((B.n * m,) + c.shape[1:])
    for e in range(B.n):
        ce = np.stack([c[k * B.n + e] for k in range(m)])
        out[e * m:(e + 1) * m] = V @ ce
    return out


def values_to_legendre(Bx: Basis1D, By: Basis1D, V: np.ndarray) -> np.ndarray:
    """2D: F_x V F_y^T."""
    return values_to_legendre_1d(By, values_to_legendre_1d(Bx, V).T).T


def legendre_to_values(Bx: Basis1D, By: Basis1D, F: np.ndarray) -> np.ndarray:
    """2D: F_x^{-1} F F_y^{-T}."""
    return legendre_to_values_1d(By, legendre_to_values_1d(Bx, F).T).T


def q_to_legendre(Bx: Basis1D, By: Basis1D, U: np.ndarray, deriv_x: bool = False) -> np.ndarray:
    """Legendre coefficients of u (R_x U R_y^T) or of d/dx u (D_x U R_y^T), U in the
    restricted hat+bubble bases."""
    Rx = (connection_full(Bx) @ restriction(Bx)).tocsr()
    Dx = (derivative_full(Bx) @ restriction(Bx)).tocsr()
    Ry = (connection_full(By) @ restriction(By)).tocsr()
    L = (Dx if deriv_x else Rx) @ U
    return np.asarray((Ry @ np.asarray(L).T).T)


def burgers_step(opx, opy, eps: float, dt: float, F: np.ndarray, tol: float = 1e-12,
                 solve: str = "fdm") -> np.ndarray:
    """One IMEX step: Legendre coefficients of u_k -> those of u_{k+1} (see module doc).
    solve: "fdm" (exact discrete solve) or "adi" (Alg. 2 at tol)."""
    Bx, By = opx.basis, opy.basis
    w2 = 1.0 / (dt * eps)
    G = w2 * _adi.load(opx, opy, F)
    if solve == "adi":
        U = _adi.ADIPlan(opx, opy, w2, tol).solve(G)
    elif solve == "dense":
        U = _adi.solve_dense(opx, opy, w2, G)
    else:
        U = _adi.solve_fdm(opx, opy, w2, G, refine=2)
    V = legendre_to_values(Bx, By, q_to_legendre(Bx, By, U))
    Vx = legendre_to_values(Bx, By, q_to_legendre(Bx, By, U, deriv_x=True))
    return values_to_legendre(Bx, By, V - dt * Vx * V)
