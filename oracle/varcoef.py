"""Variable-coefficient operator and ADI-preconditioned (flexible) CG (oracle;
test infrastructure only).

Sec. 7 of the paper solves a problem with a non-constant coefficient by a CG
iteration whose preconditioner is the constant-coefficient operator inverted
by ADI (Alg. 2) to a loose tolerance (1e-4).  Here the coefficient multiplies
the gradient (divergence form):

    -div(a grad u) = f  on a rectangle, zero Dirichlet or zero Neumann,

    a_h(u, v) = sum_e sum_(i,j) w_i w_j a(x_i, y_j) grad u . grad v   (Galerkin
    form evaluated with a tensor Gauss-Legendre rule of q = p + 2 points per
    element and dimension; exact when a is a polynomial of degree <= 3 in each
    variable, since the rule integrates degree 2q - 1 = 2p + 3 exactly).

In matrix form, with E_v, E_d the values and x-derivatives of the hat+bubble
basis at the Gauss points, W = w_x w_y^T (weights including the Jacobians):

    Y = E_d^x^T [W . A . (E_d^x U E_v^y^T)] E_v^y + E_v^x^T [W . A . (E_v^x U E_d^y^T)] E_d^y.

With a = 1 this is K (x) M + M (x) K (Sec. 3.2 with omega = 0), which the
tests check.

Sec. 7's own example adds a potential instead: (-Delta + c) u = f with
c = -10 log r on (-1, 1)^2, zero Dirichlet, on the tensor mesh graded towards the
origin with breakpoints -1, -10^-1, ..., -10^-m, 0, 10^-m, ..., 10^-1, 1 per axis,
solved by CG preconditioned with the ADI inverse of the weak Laplacian
(K (x) M + M (x) K) at tolerance 1e-4, to a relative residual of 1e-8 (Table 1 of
the paper lists the iteration counts).  The potential term is integrated with
the same Gauss rule (a reading: the paper evaluates it through its Chebyshev
transforms); c has a logarithmic singularity at a mesh vertex, never at a
Gauss point.

Krylov methods (plain definitions):
* ``pcg``: preconditioned conjugate gradients (Hestenes-Stiefel form);
* ``fcg``: flexible CG with truncation m (Notay 2000): each new direction is
  the preconditioned residual A-orthogonalised against the last m directions,
  alpha_k = d_k^T r_k / d_k^T A d_k.  For a fixed symmetric positive definite
  preconditioner and m >= 1 it produces the PCG iterates.
Both stop when ||b - A x||_2 / ||b||_2 <= tol, the residual taken from the
recurrence, and report the true residual at the end.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.special as ss

from .basis import Basis1D, Operators1D


def quadrature_order(p: int) -> int:
    """Gauss points per element and dimension: q = p + 2."""
    return p + 2


@dataclasses.dataclass(frozen=True)
class GaussGrid1D:
    x: np.ndarray      # physical points, element-major (element e owns x[e q:(e+1) q])
    w: np.ndarray      # weights including the Jacobian delta_e / 2
    t: np.ndarray      # reference points on [-1, 1], length q
    wt: np.ndarray     # reference weights, length q
    q: int


def gauss_grid(B: Basis1D) -> GaussGrid1D:
    q = quadrature_order(B.p)
    t, wt = np.polynomial.legendre.leggauss(q)
    xs, ws = [], []
    for e in range(B.n):
        xs.append(B.x[e] + (t + 1.0) * B.delta[e] / 2.0)
        ws.append(wt * B.delta[e] / 2.0)
    return GaussGrid1D(x=np.concatenate(xs), w=np.concatenate(ws), t=t, wt=wt, q=q)


def local_functions(p: int, t: np.ndarray):
    """Values and reference derivatives of the element-local functions
    [left hat, right hat, W_0, ..., W_{p-2}] at the points t (Sec. 2.1:
    W_k = (P_k - P_{k+2}) / (2k + 3), W_k' = -P_{k+1})."""
    t = np.asarray(t, dtype=np.float64)
    V = np.zeros((t.size, p + 1))
    D = np.zeros((t.size, p + 1))
    V[:, 0], D[:, 0] = (1.0 - t) / 2.0, -0.5
    V[:, 1], D[:, 1] = (1.0 + t) / 2.0, 0.5
    for k in range(p - 1):
        V[:, 2 + k] = (ss.eval_legendre(k, t) - ss.eval_legendre(k + 2, t)) / (2 * k + 3)
        D[:, 2 + k] = -ss.eval_legendre(k + 1, t)
    return V, D


def local_to_global(B: Basis1D) -> np.ndarray:
    """G[e, l] = global index of local function l of element e, or -1 when the
    function is not in the basis (a boundary hat under Dirichlet conditions)."""
    hat_pos = {v: i for i, v in enumerate(B.hat_vertices())}
    G = np.full((B.n, B.p + 1), -1, dtype=np.int64)
    for e in range(B.n):
        G[e, 0] = hat_pos.get(e, -1)
        G[e, 1] = hat_pos.get(e + 1, -1)
        for m in range(B.p - 1):
            G[e, 2 + m] = B.bubble_index(m, e)
    return G


def eval_matrices(B: Basis1D):
    """Sparse E_v (values) and E_d (d/dx) of the global basis at the Gauss
    points of ``gauss_grid(B)``: shape (n q, N)."""
    g = gauss_grid(B)
    V, D = local_functions(B.p, g.t)
    G = local_to_global(B)
    rows, cols, vv, dd = [], [], [], []
    for e in range(B.n):
        for l in range(B.p + 1):
            if G[e, l] < 0:
                continue
            rows.append(e * g.q + np.arange(g.q))
            cols.append(np.full(g.q, G[e, l]))
            vv.append(V[:, l])
            dd.append(D[:, l] * 2.0 / B.delta[e])
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    shape = (B.n * g.q, B.N)
    Ev = sp.csr_matrix((np.concatenate(vv), (rows, cols)), shape=shape)
    Ed = sp.csr_matrix((np.concatenate(dd), (rows, cols)), shape=shape)
    return Ev, Ed


@dataclasses.dataclass
class VarCoefOperator:
    """The operator U -> Y of the module docstring for one coefficient field
    a (sampled on the tensor Gauss grid, shape (n_x q_x, n_y q_y)), plus, when c
    is given (same grid), the potential term of Sec. 7's problem
    (-Delta + c) u = f:

        sum_e sum_(i,j) w_i w_j c(x_i, y_j) u v  =  E_v^x^T [W . C . (E_v^x U E_v^y^T)] E_v^y."""

    bx: Basis1D
    by: Basis1D
    a: np.ndarray
    c: Optional[np.ndarray] = None

    def __post_init__(self):
        self.gx, self.gy = gauss_grid(self.bx), gauss_grid(self.by)
        self.Evx, self.Edx = eval_matrices(self.bx)
        self.Evy, self.Edy = eval_matrices(self.by)
        assert self.a.shape == (self.gx.x.size, self.gy.x.size)
        W = np.outer(self.gx.w, self.gy.w)
        self.Wa = W * self.a
        self.Wc = None
        if self.c is not None:
            assert self.c.shape == self.a.shape
            self.Wc = W * self.c

    def apply(self, U: np.ndarray) -> np.ndarray:
        ux = (self.Evy @ (self.Edx @ U).T).T             # d/dx u at the points: E_d^x U E_v^y^T
        uy = (self.Edy @ (self.Evx @ U).T).T             # d/dy u: E_v^x U E_d^y^T
        Qx = self.Wa * ux
        Qy = self.Wa * uy
        Y = np.asarray(self.Edx.T @ (self.Evy.T @ Qx.T).T + self.Evx.T @ (self.Edy.T @ Qy.T).T)
        if self.Wc is not None:
            u = (self.Evy @ (self.Evx @ U).T).T          # u at the points: E_v^x U E_v^y^T
            Y = Y + np.asarray(self.Evx.T @ (self.Evy.T @ (self.Wc * u).T).T)
        return Y

    def dense(self) -> np.ndarray:
        """The N_x N_y square matrix acting on row-major vec(U) (small sizes)."""
        Nx, Ny = self.bx.N, self.by.N
        A = np.zeros((Nx * Ny, Nx * Ny))
        E = np.zeros((Nx, Ny))
        for k in range(Nx * Ny):
            E.flat[k] = 1.0
            A[:, k] = self.apply(E).reshape(-1)
            E.flat[k] = 0.0
        return A


@dataclasses.dataclass
class KrylovResult:
    x: np.ndarray
    iters: int
    converged: bool
    res_history: List[float]     # recurrence residual norms relative to ||b||, one per iterate
    true_rel_res: float
    iterates: Optional[List[np.ndarray]] = None


def _dot(a, b):
    return float(np.sum(a * b))


def _true_rel_res(apply, b, x, bn):
    if bn == 0.0:
        return 0.0
    r = b - apply(x)
    return float(np.sqrt(_dot(r, r)) / bn)


def pcg(apply: Callable, precond: Callable, b: np.ndarray, tol: float, maxit: int,
        keep_iterates: bool = False) -> KrylovResult:
    """Preconditioned CG from x_0 = 0."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.sqrt(_dot(b, b))
    hist = [1.0]
    its = [x.copy()] if keep_iterates else None
    z = precond(r)
    d = z.copy()
    rz = _dot(r, z)
    k = 0
    converged = bn == 0.0
    while not converged and k < maxit:
        q = apply(d)
        alpha = rz / _dot(d, q)
        x = x + alpha * d
        r = r - alpha * q
        k += 1
        hist.append(np.sqrt(_dot(r, r)) / bn)
        if keep_iterates:
            its.append(x.copy())
        if hist[-1] <= tol:
            converged = True
            break
        z = precond(r)
        rz_new = _dot(r, z)
        d = z + (rz_new / rz) * d
        rz = rz_new
    return KrylovResult(x, k, converged, hist, _true_rel_res(apply, b, x, bn), its)


def fcg(apply: Callable, precond: Callable, b: np.ndarray, tol: float, maxit: int, m: int = 1,
        keep_iterates: bool = False) -> KrylovResult:
    """Flexible CG with truncation m (m = 0 keeps no previous direction, i.e.
    preconditioned steepest descent)."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.sqrt(_dot(b, b))
    hist = [1.0]
    its = [x.copy()] if keep_iterates else None
    dirs: List[tuple] = []   # (d_i, q_i = A d_i, d_i^T q_i)
    k = 0
    converged = bn == 0.0
    while not converged and k < maxit:
        z = precond(r)
        d = z.copy()
        for (di, qi, dqi) in dirs:
            d = d - (_dot(z, qi) / dqi) * di
        q = apply(d)
        dq = _dot(d, q)
        alpha = _dot(d, r) / dq
        x = x + alpha * d
        r = r - alpha * q
        k += 1
        hist.append(np.sqrt(_dot(r, r)) / bn)
        if keep_iterates:
            its.append(x.copy())
        if m > 0:
            dirs.append((d, q, dq))
            dirs = dirs[-m:]
        if hist[-1] <= tol:
            converged = True
    return KrylovResult(x, k, converged, hist, _true_rel_res(apply, b, x, bn), its)
