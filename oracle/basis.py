"""1D hat+bubble basis and its operators (oracle; test infrastructure only).

Follows Sec. 2 of the paper ("Integrated Legendre functions") and App. A
("Recurrences"):

* bubbles W_k(x) = (1 - x^2) P^{(1,1)}_k(x) / (2(k+1)) = (P_k - P_{k+2})/(2k+3)
  (Sec. 2.1 definition; App. A eq. app:1), mapped to each element by the
  affine map a_j (Sec. 2.2);
* the block quasi-matrix C^x = [hats | W_0 block | W_1 block | ...] grouped by
  degree (Sec. 2.2, "degree-major" order), and the piecewise Legendre basis
  P^x = [P_0 block | P_1 block | ...] (Sec. 2.2);
* connection C = P R (Sec. 2.2.1, blocks R_00, R_10, R_kj of App. A),
  derivative d/dx C = P D (Sec. 2.2.2, blocks D_00, D_kk of App. A) and the
  direct-sum Legendre mass M_P (Sec. 2.2.1);
* mass M = R^T M_P R, weak Laplacian K = D^T M_P D and load T = R^T M_P
  (Sec. 2.2.1-2.2.2, Sec. 3.1);
* Dirichlet restriction: drop the first and last hat (Sec. 2.3, P_D);
  Neumann keeps the full basis C (Sec. 3.3, Sec. 5 "Y = C");
* general boundary conditions (Sec. 3.3): each end is Dirichlet (its hat
  dropped), Neumann (its hat kept) or Robin alpha u + du/dn = 0 (its hat kept
  and alpha <v, u> at that end added to the weak Laplacian; Neumann is alpha = 0).
  Mixed conditions choose the kind per end.

Index conventions (0-based, n elements, degree p):
  hats      Dirichlet: vertices 1..n-1 -> 0..n-2;  Neumann: vertices 0..n -> 0..n
  bubble    (m, e), m = 0..p-2, e = 0..n-1 -> n_h + m*n + e
  Legendre  (k, e), k = 0..p,   e = 0..n-1 -> k*n + e
so N = n_h + n(p-1) (= np-1 Dirichlet, np+1 Neumann; Sec. 3.1 gives N = pn-1)
and Nleg = (p+1)n.

Reading of a garbled passage: the App. A block R_kj (k = j +- 1) is read as
R_{j-1,j} = I/(2j+1), R_{j+1,j} = -I/(2j+1), which is what W_{j-1} =
(P_{j-1} - P_{j+1})/(2j+1) requires.

Two independent assemblies are given: ``assemble`` builds the matrices from
the paper's factorised relations (R, D, M_P), and ``assemble_quadrature``
integrates basis functions evaluated from the Jacobi definition with Gauss
quadrature. The tests pin them against each other.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.special as ss

DIRICHLET = "dirichlet"
NEUMANN = "neumann"
ROBIN = "robin"


@dataclasses.dataclass(frozen=True)
class Basis1D:
    """A 1D mesh x_0 < ... < x_n with degree p and boundary conditions: bc is one kind for
    both ends, or a pair (left, right) of kinds; alpha the Robin coefficients of the ends."""

    x: np.ndarray  # breakpoints, length n+1
    p: int
    bc: object
    alpha: tuple = (0.0, 0.0)

    @property
    def ends(self) -> tuple:
        return (self.bc, self.bc) if isinstance(self.bc, str) else tuple(self.bc)

    @property
    def n(self) -> int:
        return len(self.x) - 1

    @property
    def delta(self) -> np.ndarray:
        return np.diff(self.x)

    @property
    def nh(self) -> int:
        left, right = self.ends
        return self.n - 1 + (left != DIRICHLET) + (right != DIRICHLET)

    @property
    def N(self) -> int:
        return self.nh + self.n * (self.p - 1)

    @property
    def Nleg(self) -> int:
        return (self.p + 1) * self.n

    def hat_vertices(self) -> np.ndarray:
        """Vertex number of each retained hat, in index order."""
        left, right = self.ends
        return np.arange(0 if left != DIRICHLET else 1, self.n + 1 if right != DIRICHLET else self.n)

    def bubble_index(self, m, e):
        return self.nh + np.asarray(m) * self.n + np.asarray(e)

    def leg_index(self, k, e):
        return np.asarray(k) * self.n + np.asarray(e)


def make_basis(n: int, p: int, a: float = 0.0, b: float = 1.0, bc=DIRICHLET,
               breaks=None, alpha=(0.0, 0.0)) -> Basis1D:
    ends = (bc, bc) if isinstance(bc, str) else tuple(bc)
    if len(ends) != 2 or any(k not in (DIRICHLET, NEUMANN, ROBIN) for k in ends) or min(alpha) < 0:
        raise ValueError(bc)
    if isinstance(bc, str) and bc == ROBIN:
        raise ValueError("give Robin conditions per end")
    if p < 1 or n < 1:
        raise ValueError("need n >= 1 and p >= 1")
    if breaks is None:
        x = np.linspace(a, b, n + 1)
    else:
        x = np.asarray(breaks, dtype=np.float64)
        if len(x) != n + 1 or np.any(np.diff(x) <= 0):
            raise ValueError("breaks must be n+1 increasing points")
    alpha = tuple(float(alpha[i]) if ends[i] == ROBIN else 0.0 for i in range(2))
    return Basis1D(x=x, p=p, bc=bc if isinstance(bc, str) else ends, alpha=alpha)


# --------------------------------------------------------------------------
# Factorised assembly: the relations C = P R, C' = P D, <P^T, P> = M_P.
# --------------------------------------------------------------------------

def _full_hat_columns(B: Basis1D):
    """Column index of every vertex hat in the full basis C (n+1 hats)."""
    return np.arange(B.n + 1)


def connection_full(B: Basis1D) -> sp.csr_matrix:
    """R_C: coefficients of C^x (all n+1 hats, W_0..W_{p-2}) in P^x up to degree p.

    Blocks R_00 and R_10 (App. A): in element e the left-vertex hat is
    (P_0 - P_1)/2 and the right-vertex hat (P_0 + P_1)/2.  Blocks R_kj (App. A,
    from eq. app:1): W_m = (P_m - P_{m+2})/(2m+3).
    """
    n, p = B.n, B.p
    ncols = (n + 1) + n * (p - 1)
    rows, cols, vals = [], [], []
    for e in range(n):
        # left vertex e, right vertex e+1
        rows += [0 * n + e, 1 * n + e, 0 * n + e, 1 * n + e]
        cols += [e, e, e + 1, e + 1]
        vals += [0.5, -0.5, 0.5, 0.5]
    for m in range(p - 1):
        for e in range(n):
            c = (n + 1) + m * n + e
            rows += [m * n + e, (m + 2) * n + e]
            cols += [c, c]
            vals += [1.0 / (2 * m + 3), -1.0 / (2 * m + 3)]
    return sp.csr_matrix((vals, (rows, cols)), shape=(B.Nleg, ncols))


def derivative_full(B: Basis1D) -> sp.csr_matrix:
    """D: d/dx C^x = P^x D (Sec. 2.2.2; blocks D_00, D_kk of App. A).

    Hats have slope -1/delta_e (left vertex) and +1/delta_e (right vertex) on
    element e; W_m'(t) = -P_{m+1}(t) (eq. deriv) and dt/dx = 2/delta_e.
    """
    n, p = B.n, B.p
    d = B.delta
    ncols = (n + 1) + n * (p - 1)
    rows, cols, vals = [], [], []
    for e in range(n):
        rows += [e, e]
        cols += [e, e + 1]
        vals += [-1.0 / d[e], 1.0 / d[e]]
    for m in range(p - 1):
        for e in range(n):
            rows.append((m + 1) * n + e)
            cols.append((n + 1) + m * n + e)
            vals.append(-2.0 / d[e])
    return sp.csr_matrix((vals, (rows, cols)), shape=(B.Nleg, ncols))


def legendre_mass(B: Basis1D) -> sp.dia_matrix:
    """M_P = (delta_1/2 M_P) (+) ... (+) (delta_n/2 M_P), M_P = diag(2/(2k+1)) (Sec. 2.1-2.2.1)."""
    n, p = B.n, B.p
    diag = np.empty(B.Nleg)
    for k in range(p + 1):
        diag[k * n:(k + 1) * n] = (B.delta / 2.0) * (2.0 / (2 * k + 1))
    return sp.diags(diag)


def restriction(B: Basis1D) -> sp.csr_matrix:
    """P_D (Sec. 2.3): keeps every column of C except the hats of Dirichlet ends."""
    n, p = B.n, B.p
    ncols_full = (n + 1) + n * (p - 1)
    keep = list(B.hat_vertices()) + list(range(n + 1, ncols_full))
    return sp.csr_matrix((np.ones(len(keep)), (keep, np.arange(len(keep)))),
                         shape=(ncols_full, len(keep)))


@dataclasses.dataclass
class Operators1D:
    basis: Basis1D
    K: sp.csr_matrix  # weak Laplacian  -Delta_Y = D^T M_P D (restricted)
    M: sp.csr_matrix  # mass            M_Y = R^T M_P R (restricted)
    T: sp.csr_matrix  # load            R_Y^T M_P  (N x Nleg)

    def A(self, omega2: float) -> sp.csr_matrix:
        """A_Y = -Delta_Y + (omega^2/2) M_Y (eq. 2d:poisson, ADI section)."""
        return (self.K + (omega2 / 2.0) * self.M).tocsr()


def assemble(B: Basis1D) -> Operators1D:
    """K, M and T from the paper's factorised relations (Sec. 2.2, Sec. 3.1)."""
    R = connection_full(B)
    D = derivative_full(B)
    MP = legendre_mass(B)
    PD = restriction(B)
    RY = (R @ PD).tocsr()
    DY = (D @ PD).tocsr()
    K = (DY.T @ MP @ DY + robin_term(B)).tocsr()
    M = (RY.T @ MP @ RY).tocsr()
    T = (RY.T @ MP).tocsr()
    for A in (K, M, T):
        A.eliminate_zeros()
    return Operators1D(basis=B, K=K, M=M, T=T)


def robin_term(B: Basis1D) -> sp.csr_matrix:
    """alpha_l v(a) u(a) + alpha_r v(b) u(b) (Sec. 3.3's boundary term): the basis functions
    evaluated at the two ends (eval_matrix), weighted by the Robin coefficients."""
    out = sp.csr_matrix((B.N, B.N))
    for side, xe in ((0, B.x[0]), (1, B.x[-1])):
        if B.alpha[side] != 0.0:
            e = eval_matrix(B, np.array([xe]))
            out = out + B.alpha[side] * sp.csr_matrix(e.T @ e)
    return out


# --------------------------------------------------------------------------
# Independent assembly by Gauss quadrature of explicitly evaluated functions.
# --------------------------------------------------------------------------

def _bubble_poly(k: int) -> np.poly1d:
    """W_k(t) = (1 - t^2) P^{(1,1)}_k(t) / (2(k+1)) (Sec. 2.1 definition)."""
    jac = ss.jacobi(k, 1.0, 1.0)
    return np.poly1d([-1.0, 0.0, 1.0]) * np.poly1d(jac.coeffs) / (2.0 * (k + 1))


def assemble_quadrature(B: Basis1D, extra_points: int = 4) -> Operators1D:
    """Dense K, M, T by Gauss-Legendre quadrature on each element.

    Every basis function is evaluated from its definition (hats as linear
    functions, bubbles from the Jacobi form); nothing from ``assemble`` is used.
    Exact for the polynomial degrees involved.  Intended for small p (the
    monomial form of the Jacobi polynomial is ill-conditioned for large p).
    """
    n, p = B.n, B.p
    t, w = np.polynomial.legendre.leggauss(p + 2 + extra_points)
    N, Nleg = B.N, B.Nleg
    K = np.zeros((N, N))
    M = np.zeros((N, N))
    T = np.zeros((N, Nleg))
    polys = [_bubble_poly(m) for m in range(p - 1)]
    dpolys = [q.deriv() for q in polys]
    hat_pos = {v: i for i, v in enumerate(B.hat_vertices())}
    for e in range(n):
        de = B.delta[e]
        jac = de / 2.0
        # local functions: (global index, values at t, d/dx values at t)
        loc = []
        for v, val, dval in ((e, (1 - t) / 2, -np.ones_like(t) / de),
                             (e + 1, (1 + t) / 2, np.ones_like(t) / de)):
            if v in hat_pos:
                loc.append((hat_pos[v], val, dval))
        for m in range(p - 1):
            loc.append((int(B.bubble_index(m, e)), polys[m](t), dpolys[m](t) * 2.0 / de))
        for (i, vi, di) in loc:
            for (j, vj, dj) in loc:
                M[i, j] += jac * np.sum(w * vi * vj)
                K[i, j] += jac * np.sum(w * di * dj)
            for k in range(p + 1):
                T[i, int(B.leg_index(k, e))] += jac * np.sum(w * vi * ss.eval_legendre(k, t))
    # Robin ends: only the end vertex's hat is nonzero there, with value 1
    for side, v in ((0, 0), (1, n)):
        if B.alpha[side] != 0.0 and v in hat_pos:
            K[hat_pos[v], hat_pos[v]] += B.alpha[side]
    return Operators1D(basis=B, K=sp.csr_matrix(K), M=sp.csr_matrix(M), T=sp.csr_matrix(T))


# --------------------------------------------------------------------------
# Evaluation helpers (used to check solutions against known functions).
# --------------------------------------------------------------------------

def eval_matrix(B: Basis1D, xs: np.ndarray) -> np.ndarray:
    """V[i, j] = value of basis function j at point xs[i] (dense)."""
    xs = np.asarray(xs, dtype=np.float64)
    V = np.zeros((len(xs), B.N))
    e_of = np.clip(np.searchsorted(B.x, xs, side="right") - 1, 0, B.n - 1)
    hat_pos = {v: i for i, v in enumerate(B.hat_vertices())}
    polys = [_bubble_poly(m) for m in range(B.p - 1)] if B.p <= 20 else None
    for r, (xv, e) in enumerate(zip(xs, e_of)):
        t = (2 * xv - B.x[e] - B.x[e + 1]) / (B.x[e + 1] - B.x[e])
        if e in hat_pos:
            V[r, hat_pos[e]] += (1 - t) / 2
        if e + 1 in hat_pos:
            V[r, hat_pos[e + 1]] += (1 + t) / 2
        for m in range(B.p - 1):
            if polys is not None:
                val = polys[m](t)
            else:
                val = (ss.eval_legendre(m, t) - ss.eval_legendre(m + 2, t)) / (2 * m + 3)
            V[r, int(B.bubble_index(m, e))] = val
    return V


def legendre_coefficients(B: Basis1D, f, extra_points: int = 8) -> np.ndarray:
    """Piecewise Legendre coefficients (degrees 0..p) of f by Gauss quadrature.

    f_{k,e} = <P_{k,e}, f> / <P_{k,e}, P_{k,e}> with <P_{k,e},P_{k,e}> = delta_e/(2k+1)
    (Sec. 2.2.1: coefficients are (M_P)^{-1} <P^T, f>).
    """
    t, w = np.polynomial.legendre.leggauss(B.p + 1 + extra_points)
    c = np.zeros(B.Nleg)
    for e in range(B.n):
        xe = B.x[e] + (t + 1) * B.delta[e] / 2
        fv = f(xe)
        for k in range(B.p + 1):
            c[int(B.leg_index(k, e))] = (2 * k + 1) / 2.0 * np.sum(w * fv * ss.eval_legendre(k, t))
    return c
