"""Reverse Cholesky of B^3-arrowhead matrices and the O(N) solve (oracle).

Follows Sec. 4 of the paper: the theorem that A = L^T L (L lower triangular,
"reverse" Cholesky: starting bottom-right) has no fill, Alg. 1 ("Reverse
Cholesky for B^3-Arrowhead Matrices") and the corollary giving the block
inverse of L.

Matrix partition (degree-major order, see ``basis``):
    S = [[A0, B], [B^T, D]]   A0 = hat block (n_h x n_h),
                               D  = bubble block = D_1 (+) ... (+) D_n (interlaced),
    D_e = the (p-1) x (p-1) bubble block of element e (degrees 0..p-2).

Alg. 1, read with two corrections to garbled lines: the Schur complement is
A~0 = A0 - sum_k M_k M_k^T (the proof of the theorem has the minus; the
algorithm's listing drops "A0 -"), and the matrices written L~_{k,j} in the
construction of M_k are the blocks of L~^{-1}, as in the proof.

Steps here:
 1. for every element: D_e = L_e^T L_e (reverse Cholesky; done as
    flip -> numpy Cholesky -> flip, a library step);
 2. M = B L~^{-1}, i.e. the coupling block of L is C = L~^{-T} B^T;
 3. A~0 = A0 - C^T C;
 4. A~0 = L0^T L0 (reverse Cholesky);
 5. L = [[L0, 0], [C, L~]].
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import Basis1D


def reverse_cholesky_dense(A: np.ndarray) -> np.ndarray:
    """Lower-triangular L with A = L^T L, via the exchange matrix J:
    J A J = G G^T (standard Cholesky), so A = (J G J)(J G^T J) and L = J G^T J."""
    A = np.asarray(A, dtype=np.float64)
    G = np.linalg.cholesky(A[::-1, ::-1])
    return np.ascontiguousarray(G.T[::-1, ::-1])


@dataclasses.dataclass
class ArrowheadFactor:
    basis: Basis1D
    Le: np.ndarray      # (n, p-1, p-1) per-element lower-triangular bubble factors
    C: np.ndarray       # (N_b, n_h) coupling block of L (degree-major bubble rows)
    L0: np.ndarray      # (n_h, n_h) lower-triangular hat factor

    def to_dense(self) -> np.ndarray:
        B = self.basis
        N, nh, n = B.N, B.nh, B.n
        L = np.zeros((N, N))
        L[:nh, :nh] = self.L0
        L[nh:, :nh] = self.C
        for e in range(n):
            idx = B.bubble_index(np.arange(B.p - 1), e)
            L[np.ix_(idx, idx)] = self.Le[e]
        return L

    # -- the solve of the corollary: S^{-1} b = L^{-1} L^{-T} b ------------
    def solve(self, b: np.ndarray) -> np.ndarray:
        """x = S^{-1} b for b of shape (N,) or (N, k)."""
        B = self.basis
        nh, n, p = B.nh, B.n, B.p
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        if vec:
            b = b[:, None]
        bh, bb = b[:nh], b[nh:]
        # bubbles in per-element order: bb[m*n + e] -> (e, m)
        bb_e = bb.reshape(p - 1, n, -1).transpose(1, 0, 2)
        # L^T y = b : L~^T y_b = b_b, then L0^T y_h = b_h - C^T y_b
        yb_e = np.empty_like(bb_e)
        for e in range(n):
            yb_e[e] = sla.solve_triangular(self.Le[e], bb_e[e], trans="T", lower=True)
        yb = yb_e.transpose(1, 0, 2).reshape(n * (p - 1), -1)
        if nh:
            yh = sla.solve_triangular(self.L0, bh - self.C.T @ yb, trans="T", lower=True)
            # L x = y : L0 x_h = y_h, then L~ x_b = y_b - C x_h
            xh = sla.solve_triangular(self.L0, yh, lower=True)
            rb = yb - self.C @ xh
        else:
            xh = bh[:0]
            rb = yb
        rb_e = rb.reshape(p - 1, n, -1).transpose(1, 0, 2)
        xb_e = np.empty_like(rb_e)
        for e in range(n):
            xb_e[e] = sla.solve_triangular(self.Le[e], rb_e[e], lower=True)
        xb = xb_e.transpose(1, 0, 2).reshape(n * (p - 1), -1)
        x = np.vstack([xh, xb])
        return x[:, 0] if vec else x


def factor_arrowhead(S, basis: Basis1D) -> ArrowheadFactor:
    """Alg. 1 on an SPD B^3-arrowhead matrix S in degree-major order."""
    B = basis
    nh, n, p = B.nh, B.n, B.p
    S = S.toarray() if sp.issparse(S) else np.asarray(S, dtype=np.float64)
    A0 = S[:nh, :nh]
    Bblk = S[:nh, nh:]                 # n_h x N_b
    Le = np.zeros((n, p - 1, p - 1))
    for e in range(n):                 # step 1: element bubble blocks
        idx = B.bubble_index(np.arange(p - 1), e) - nh
        De = S[nh + idx][:, nh + idx]
        Le[e] = reverse_cholesky_dense(De)
    # step 2: C = L~^{-T} B^T, element by element
    C = np.zeros((n * (p - 1), nh))
    for e in range(n):
        idx = B.bubble_index(np.arange(p - 1), e) - nh
        C[idx] = sla.solve_triangular(Le[e], Bblk[:, idx].T, trans="T", lower=True)
    # steps 3-4: Schur complement of the hats and its reverse Cholesky
    At0 = A0 - C.T @ C
    L0 = reverse_cholesky_dense(At0) if nh else np.zeros((0, 0))
    return ArrowheadFactor(basis=B, Le=Le, C=C, L0=L0)


def predicted_pattern(basis: Basis1D) -> np.ndarray:
    """Boolean mask of entries of L allowed to be nonzero (Sec. 4 theorem,
    made concrete for this basis): hat block lower bidiagonal; bubble (e,m)
    rows couple to hats only for m in {0, 1} and only to the vertices of e;
    bubble block lower triangular within an element at degree offsets 0, 2."""
    B = basis
    N, nh, n, p = B.N, B.nh, B.n, B.p
    P = np.zeros((N, N), dtype=bool)
    for i in range(nh):
        P[i, i] = True
        if i > 0:
            P[i, i - 1] = True
    hat_pos = {v: i for i, v in enumerate(B.hat_vertices())}
    for e in range(n):
        for m in range(p - 1):
            r = int(B.bubble_index(m, e))
            P[r, r] = True
            if m >= 2:
                P[r, int(B.bubble_index(m - 2, e))] = True
            if m <= 1:
                for v in (e, e + 1):
                    if v in hat_pos:
                        P[r, hat_pos[v]] = True
    return P
