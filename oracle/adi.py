"""Generalised ADI and exact reference solves (oracle; test infrastructure only).

The 2D discretisation (Sec. 3.2, eq. 2d:poisson; restated in Sec. 5 as
eq. adi:poisson) is the generalised Sylvester equation

    A_Y^x U M^y + M^x U A_Y^y = G,   A_Y = K + (omega^2/2) M,   G = T_x F T_y^T,

(rows of U index the x-basis, columns the y-basis).  Alg. 2 solves
A U C - D U B = F; this equation is that form with

    A = A_Y^x,  D = M^x,  C = M^y,  B = -A_Y^y,

so sigma(A, D) in [a, b] (positive) and sigma(B, C) in [-b_y, -a_y].  Alg. 2 asks
for reverse Cholesky factors of B - p_j C, which is negative definite; the
factor is taken of its negation A_Y^y + p_j M^y (a reading).  The final step
W_J C^{-1} needs a factorisation of C = M^y, which the precomputation list
does not name; it is factorised as well (a reading).

Error metric (a reading of the unspecified norm in the ADI lemma): the
Frobenius norm of V (U - U_J) L^T with D = V^T V, C = L^T L, i.e.
sqrt(tr(E M^y E^T M^x)), relative to the same norm of U: the relative L^2
error of the function.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import Operators1D
from .cholesky import factor_arrowhead
from . import shifts as _shifts
from . import spectrum as _spectrum


def load(opx: Operators1D, opy: Operators1D, F: np.ndarray) -> np.ndarray:
    """G = R_x^T M_P^x F M_P^y R_y = T_x F T_y^T (Sec. 3.2)."""
    return np.asarray(opx.T @ (opy.T @ np.asarray(F).T).T)


def axis_operators(opx: Operators1D, opy: Operators1D, omega2: float, coef=None):
    """(A_x, A_y): A_Y of both axes, or with coef = (kx, sx, ky, sy) the general pair
    A_x = kx K_x + sx M_x, A_y = ky K_y + sy M_y, i.e. Alg. 2's A U C - D U B = F with
    A = A_x, D = M_x, C = M_y, B = -A_y (anisotropic or unequally screened problems)."""
    if coef is None:
        return opx.A(omega2), opy.A(omega2)
    kx, sx, ky, sy = coef
    return (kx * opx.K + sx * opx.M).tocsr(), (ky * opy.K + sy * opy.M).tocsr()


def apply_operator(opx: Operators1D, opy: Operators1D, omega2: float, U: np.ndarray, coef=None) -> np.ndarray:
    """A_Y^x U M^y + M^x U A_Y^y (or A_x U M^y + M^x U A_y with coef)."""
    Ax, Ay = axis_operators(opx, opy, omega2, coef)
    UMy = (opy.M @ U.T).T
    UAy = (Ay @ U.T).T
    return np.asarray(Ax @ UMy + opx.M @ UAy)


def rel_l2_error(U: np.ndarray, Uref: np.ndarray, opx: Operators1D, opy: Operators1D) -> float:
    """sqrt(tr(E M^y E^T M^x)) / sqrt(tr(Uref M^y Uref^T M^x)), E = U - Uref."""
    def sq(X):
        XMy = (opy.M @ X.T).T
        return float(np.sum((opx.M @ X) * XMy))
    return (max(sq(U - Uref), 0.0) / sq(Uref)) ** 0.5


# --------------------------------------------------------------------------
# Exact references.
# --------------------------------------------------------------------------

def solve_dense(opx: Operators1D, opy: Operators1D, omega2: float, G: np.ndarray, coef=None) -> np.ndarray:
    """Dense Kronecker solve (A_Y^x (x) M^y + M^x (x) A_Y^y) vec_r(U) = vec_r(G) (small N)."""
    Ax, Ay = (A.toarray() for A in axis_operators(opx, opy, omega2, coef))
    Mx, My = opx.M.toarray(), opy.M.toarray()
    Op = np.kron(Ax, My) + np.kron(Mx, Ay)
    u = np.linalg.solve(Op, np.asarray(G).reshape(-1))
    return u.reshape(G.shape)


def solve_fdm(opx: Operators1D, opy: Operators1D, omega2: float, G: np.ndarray,
              refine: int = 1, coef=None) -> np.ndarray:
    """Fast diagonalisation (Lynch et al. 1964, cited in Sec. 1): A_Y V = M V Lambda
    per dimension (library eigensolver), U = V_x [(V_x^T G V_y) / (lx_i + ly_j)] V_y^T,
    followed by ``refine`` FP64 residual-correction steps."""
    Ax, Ay = axis_operators(opx, opy, omega2, coef)
    lx, Vx = sla.eigh(Ax.toarray(), opx.M.toarray())
    ly, Vy = sla.eigh(Ay.toarray(), opy.M.toarray())
    den = lx[:, None] + ly[None, :]

    def inv(R):
        return Vx @ ((Vx.T @ R @ Vy) / den) @ Vy.T
    U = inv(G)
    for _ in range(refine):
        U = U + inv(G - apply_operator(opx, opy, omega2, U, coef))
    return U


# --------------------------------------------------------------------------
# Alg. 2 (generalised ADI), with the factorisations of Alg. 1.
# --------------------------------------------------------------------------

class ADIPlan:
    """Precomputation of Alg. 2 for A = A_Y^x, D = M^x, C = M^y, B = -A_Y^y."""

    def __init__(self, opx: Operators1D, opy: Operators1D, omega2: float, eps: float,
                 interval=None, J=None, coef=None):
        self.opx, self.opy, self.omega2, self.eps = opx, opy, omega2, eps
        kx, sx, ky, sy = coef if coef is not None else (1.0, omega2 / 2.0, 1.0, omega2 / 2.0)
        if interval is None:
            ax, bx = _spectrum.interval(opx, omega2, kx, sx)
            ay, by = _spectrum.interval(opy, omega2, ky, sy)
            interval = (ax, bx, -by, -ay)
        self.interval = tuple(float(v) for v in interval)
        a, b, c, d = self.interval
        self.J, self.p, self.q = _shifts.adi_shifts(a, b, c, d, eps, J=J)
        Ax, Ay = axis_operators(opx, opy, omega2, coef)
        # reverse Cholesky of A - q_j D and of -(B - p_j C) = A_Y^y + p_j M^y
        self.fx = [factor_arrowhead(Ax - qj * opx.M, opx.basis) for qj in self.q]
        self.fy = [factor_arrowhead(Ay + pj * opy.M, opy.basis) for pj in self.p]
        self.fmass = factor_arrowhead(opy.M, opy.basis)
        self.Ax, self.Ay = Ax, Ay

    def solve(self, G: np.ndarray, return_history: bool = False):
        """Solve loop of Alg. 2 with F = G."""
        Mx, My = self.opx.M, self.opy.M
        W = np.zeros_like(G, dtype=np.float64)
        hist = []
        for j in range(self.J):
            pj, qj = self.p[j], self.q[j]
            # W_{j-1/2} = (G - (A - p_j D) W_{j-1}) (B - p_j C)^{-1},
            # (B - p_j C)^{-1} = -(A_Y^y + p_j M^y)^{-1} (symmetric): a row solve
            R1 = G - (self.Ax @ W - pj * (Mx @ W))
            Wh = -self.fy[j].solve(R1.T).T
            # W_j = (A - q_j D)^{-1} (G - W_{j-1/2} (B - q_j C)),  B - q_j C = -(A_Y^y + q_j M^y)
            R2 = G + ((self.Ay @ Wh.T).T + qj * (My @ Wh.T).T)
            W = self.fx[j].solve(R2)
            if return_history:
                hist.append((Wh.copy(), W.copy()))
        U = self.fmass.solve(W.T).T          # W_J C^{-1}
        return (U, hist) if return_history else U


def solve_adi(opx, opy, omega2, G, eps, interval=None, coef=None):
    return ADIPlan(opx, opy, omega2, eps, interval=interval, coef=coef).solve(G)
