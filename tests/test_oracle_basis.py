"""Pins for the oracle's 1D operators (Sec. 2, Sec. 3.1, App. A)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "appendix_a_entries.json")))


def ref_element(p, bc=basis.NEUMANN):
    return basis.make_basis(1, p, -1.0, 1.0, bc)


def test_printed_values_reference_element():
    """Entries the paper prints (Sec. 2.1, App. A) on one element [-1, 1]."""
    B = ref_element(6)
    R = basis.connection_full(B).toarray()
    D = basis.derivative_full(B).toarray()
    MP = basis.legendre_mass(B).toarray()
    # M_P = diag(2, 2/3, 2/5, ...)
    assert np.allclose(np.diag(MP)[:3], GOLD["legendre_mass_diag_first3"]["values"], rtol=0, atol=1e-15)
    # L_W: bubble columns of R (full basis: 2 hats, then W_0..W_4)
    assert np.allclose(R[:4, 2:5], GOLD["lowering_LW_block"]["values"], rtol=0, atol=1e-15)
    # R_00, R_10: hat columns on P_0 and P_1
    assert np.allclose(R[0, :2], GOLD["R00_row"]["values"])
    assert np.allclose(R[1, :2], GOLD["R10_row"]["values"])
    # D_00 and D_kk with delta = 2
    assert np.allclose(D[0, :2] * 2.0, GOLD["D00_row_times_delta"]["values"])
    for m in range(5):
        assert D[m + 1, 2 + m] * 2.0 == pytest.approx(GOLD["Dkk_times_delta"]["value"])
    # -Delta_W = diag(2/(2k+3)) (Sec. 2.1)
    ops = basis.assemble(B)
    K = ops.K.toarray()
    assert np.allclose(np.diag(K)[2:5], GOLD["bubble_stiffness_diag_first3"]["values"], atol=1e-15)


@pytest.mark.parametrize("bc", [basis.DIRICHLET, basis.NEUMANN])
@pytest.mark.parametrize("n,p,breaks", [(1, 2, None), (3, 7, [0.0, 0.2, 0.9, 1.3]), (4, 10, None),
                                        (2, 3, [-1.0, 0.1, 2.0])])
def test_factorised_assembly_matches_quadrature(bc, n, p, breaks):
    a, b = (breaks[0], breaks[-1]) if breaks else (0.0, 1.0)
    B = basis.make_basis(n, p, a, b, bc, breaks=breaks)
    o1 = basis.assemble(B)
    o2 = basis.assemble_quadrature(B)
    for name in "KMT":
        A1 = getattr(o1, name).toarray()
        A2 = getattr(o2, name).toarray()
        assert np.abs(A1 - A2).max() <= 1e-13 * max(1.0, np.abs(A1).max()), name


def test_neumann_constants_and_partition_of_unity():
    B = basis.make_basis(5, 6, 0.0, 2.0, basis.NEUMANN, breaks=[0, 0.3, 0.5, 1.1, 1.7, 2.0])
    ops = basis.assemble(B)
    ones = np.zeros(B.N)
    ones[:B.nh] = 1.0                      # sum of all hats = 1
    assert np.abs(ops.K @ ones).max() < 1e-13
    e0 = np.zeros(B.Nleg)
    e0[:B.n] = 1.0                         # f = 1: P_0 coefficient 1 on every element
    assert np.allclose(ops.M @ ones, ops.T @ e0, atol=1e-15)


def test_linear_elements_match_textbook_eigenvalues():
    """p = 1 (hats only): generalised eigenvalues of (K, M) on [0, 1], Dirichlet,
    uniform h, are (6/h^2)(1 - cos k pi h)/(2 + cos k pi h)."""
    n = 9
    B = basis.make_basis(n, 1, 0.0, 1.0, basis.DIRICHLET)
    ops = basis.assemble(B)
    lam = sla.eigh(ops.K.toarray(), ops.M.toarray(), eigvals_only=True)
    h = 1.0 / n
    k = np.arange(1, n)
    ref = 6.0 / h ** 2 * (1 - np.cos(k * math.pi * h)) / (2 + np.cos(k * math.pi * h))
    assert np.allclose(lam, np.sort(ref), rtol=1e-12)


def test_b3_arrowhead_structure():
    """Sec. 2.2-2.3: K is block diagonal with a tridiagonal hat block and diagonal
    bubble blocks; M couples hats only to W_0 and W_1, and bubbles only at
    degree offsets 0 and +-2 within an element."""
    B = basis.make_basis(4, 7, 0.0, 1.0, basis.DIRICHLET)
    ops = basis.assemble(B)
    K, M = ops.K.toarray(), ops.M.toarray()
    nh, n = B.nh, B.n
    assert np.count_nonzero(K[:nh, nh:]) == 0
    Kb = K[nh:, nh:]
    assert np.count_nonzero(Kb - np.diag(np.diag(Kb))) == 0
    assert np.count_nonzero(np.triu(K[:nh, :nh], 2)) == 0
    assert np.count_nonzero(M[:nh, nh + 2 * n:]) == 0
    Mb = M[nh:, nh:]
    r, c = np.nonzero(Mb)
    assert set(np.unique(np.abs(r - c))) <= {0, 2 * n}


def test_load_of_legendre_polynomial():
    """T maps coefficients of f to <basis_i, f>; check against integrals of an
    explicit polynomial evaluated at Gauss points."""
    B = basis.make_basis(3, 5, 0.0, 1.0, basis.NEUMANN, breaks=[0, 0.25, 0.6, 1.0])
    ops = basis.assemble(B)
    f = lambda x: 1 + x - 3 * x ** 3 + x ** 5
    coef = basis.legendre_coefficients(B, f)
    g = ops.T @ coef
    t, w = np.polynomial.legendre.leggauss(12)
    ref = np.zeros(B.N)
    for e in range(B.n):
        xs = B.x[e] + (t + 1) * B.delta[e] / 2
        V = basis.eval_matrix(B, xs)
        ref += (B.delta[e] / 2) * (V.T @ (w * f(xs)))
    assert np.allclose(g, ref, atol=1e-14)
