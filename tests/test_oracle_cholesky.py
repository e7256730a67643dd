"""Pins for the oracle's reverse Cholesky (Sec. 4 theorem, Alg. 1, corollary)."""
import numpy as np
import pytest

from oracle import basis, cholesky


CASES = [(basis.DIRICHLET, 4, 8, None, 0.0), (basis.NEUMANN, 3, 7, [0, 0.2, 0.9, 1.3], 2.0),
         (basis.DIRICHLET, 1, 5, None, 3.0), (basis.NEUMANN, 2, 2, None, 1.0),
         (basis.DIRICHLET, 5, 3, [0, .1, .2, .5, .7, 1.0], 1e4), (basis.NEUMANN, 6, 12, None, 1e-3)]


def build(bc, n, p, breaks, shift):
    a, b = (breaks[0], breaks[-1]) if breaks else (0.0, 1.0)
    B = basis.make_basis(n, p, a, b, bc, breaks=breaks)
    ops = basis.assemble(B)
    return B, (ops.K + shift * ops.M).toarray()


@pytest.mark.parametrize("bc,n,p,breaks,shift", CASES)
def test_reconstruction_and_flip_cholesky(bc, n, p, breaks, shift):
    B, S = build(bc, n, p, breaks, shift)
    L = cholesky.factor_arrowhead(S, B).to_dense()
    assert np.allclose(np.triu(L, 1), 0.0)
    assert np.all(np.diag(L) > 0)
    assert np.abs(L.T @ L - S).max() <= 1e-14 * np.abs(S).max()
    # uniqueness of Cholesky with positive diagonal: equals the dense flip-Cholesky
    Lf = cholesky.reverse_cholesky_dense(S)
    assert np.abs(L - Lf).max() <= 1e-12 * np.abs(Lf).max()


@pytest.mark.parametrize("bc,n,p,breaks,shift", CASES)
def test_no_fill(bc, n, p, breaks, shift):
    """Theorem (Sec. 4): the reverse Cholesky factor keeps the arrowhead pattern.
    Checked on the dense library factor, which knows nothing of the structure."""
    B, S = build(bc, n, p, breaks, shift)
    Lf = cholesky.reverse_cholesky_dense(S)
    mask = cholesky.predicted_pattern(B)
    assert np.abs(Lf[~mask]).max(initial=0.0) <= 1e-13 * np.abs(Lf).max()


@pytest.mark.parametrize("bc,n,p,breaks,shift", CASES)
def test_solve(bc, n, p, breaks, shift):
    B, S = build(bc, n, p, breaks, shift)
    f = cholesky.factor_arrowhead(S, B)
    rhs = np.random.default_rng(1).standard_normal((B.N, 3))
    x = f.solve(rhs)
    assert np.abs(S @ x - rhs).max() <= 1e-12 * np.abs(rhs).max() * max(1.0, np.abs(S).max())
    assert np.allclose(x, np.linalg.solve(S, rhs), rtol=1e-10, atol=1e-12)


def test_schur_complement_is_tridiagonal():
    B, S = build(basis.NEUMANN, 6, 9, None, 0.7)
    f = cholesky.factor_arrowhead(S, B)
    At0 = f.L0.T @ f.L0
    assert np.abs(np.triu(At0, 2)).max() <= 1e-13 * np.abs(At0).max()


def test_mass_matrix_factor():
    """The mass matrix alone (no stiffness) is also an SPD arrowhead."""
    B = basis.make_basis(4, 9, 0.0, 1.0, basis.DIRICHLET)
    M = basis.assemble(B).M.toarray()
    L = cholesky.factor_arrowhead(M, B).to_dense()
    assert np.abs(L.T @ L - M).max() <= 1e-15
