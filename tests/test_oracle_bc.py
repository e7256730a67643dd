"""Pins of the oracle's general boundary conditions (Sec. 3.3: Robin alpha u + du/dn = g,
mixed kinds per end) and of Alg. 2 with general axis operators (A U C - D U B = F with
A = kx K + sx M, D = M_x, C = M_y, B = -(ky K + sy M)).

* the continuous lowest eigenvalue used as the spectral lower end: the closed forms
  pi^2/l^2 (Dirichlet), 0 (Neumann), (pi/(2l))^2 (one of each), and k tan(k l / 2) = alpha for
  a symmetric Robin pair; the Galerkin lowest eigenvalue lies above it and converges to it;
* a 1D Robin problem with a manufactured solution, inhomogeneous data on both ends, solved
  with the assembled operators (a wrong sign or end of the boundary term fails it);
* both assemblies (factorised relations, quadrature) agree with Robin and mixed ends;
* 2D: the oracle's ADI against the dense Kronecker solve for mixed/Robin ends and for
  anisotropic, unequally screened axis operators.
"""
import math

import numpy as np
import pytest
import scipy.optimize as so

from oracle import adi as oadi
from oracle import basis as obasis
from oracle import spectrum as ospec


def test_lowest_eigenvalue_closed_forms():
    for ell in (1.0, 2.5):
        B = lambda bc, alpha=(0.0, 0.0): obasis.make_basis(3, 4, 0.0, ell, bc, alpha=alpha)
        assert ospec.continuous_lowest(B("dirichlet")) == pytest.approx(math.pi ** 2 / ell ** 2, rel=1e-13)
        assert ospec.continuous_lowest(B("neumann")) == 0.0
        for mixed in (("dirichlet", "neumann"), ("neumann", "dirichlet")):
            assert ospec.continuous_lowest(B(mixed)) == pytest.approx((math.pi / (2 * ell)) ** 2, rel=1e-13)
        for alpha in (0.3, 4.0, 50.0):
            # symmetric Robin pair: u = cos(k (x - l/2)), so k tan(k l / 2) = alpha
            k = so.brentq(lambda k: k * math.tan(k * ell / 2) - alpha, 1e-12, math.pi / ell - 1e-12)
            lam = ospec.continuous_lowest(B(("robin", "robin"), (alpha, alpha)))
            assert lam == pytest.approx(k * k, rel=1e-12)
        # Robin tends to Neumann as alpha -> 0 and to Dirichlet as alpha -> infinity
        assert ospec.continuous_lowest(B(("robin", "dirichlet"), (1e-9, 0))) == pytest.approx(
            (math.pi / (2 * ell)) ** 2, rel=1e-6)
        assert ospec.continuous_lowest(B(("robin", "dirichlet"), (1e9, 0))) == pytest.approx(
            math.pi ** 2 / ell ** 2, rel=1e-6)


@pytest.mark.parametrize("bc,alpha", [(("dirichlet", "neumann"), (0, 0)), (("robin", "robin"), (2.0, 0.5)),
                                      (("neumann", "robin"), (0, 7.0)), (("robin", "dirichlet"), (3.0, 0))])
def test_galerkin_lowest_eigenvalue_above_and_converging(bc, alpha):
    lam = ospec.continuous_lowest(obasis.make_basis(1, 1, 0.0, 1.5, bc, alpha=alpha))
    for p, tol in ((4, 1e-2), (12, 1e-10)):
        o = obasis.assemble(obasis.make_basis(3, p, 0.0, 1.5, bc, alpha=alpha))
        lmin, lmax = ospec.extreme_eigenvalues(o, 0.0)
        # above the continuous eigenvalue, up to the eigensolver's rounding (about eps lambda_max)
        assert lmin >= lam - 1e-14 * lmax
        assert lmin - lam <= tol * max(lam, 1.0)


def test_robin_manufactured_1d():
    """-u'' + c u = f on [0.2, 1.7], alpha_l u - u' = g_l at the left end, alpha_r u + u' = g_r at
    the right, u = exp(x) cos(2x): weak form (K + c M) U = T f + g_l Q(a) + g_r Q(b)."""
    a, b, c = 0.2, 1.7, 3.0
    al, ar = 1.5, 0.25
    u = lambda x: np.exp(x) * np.cos(2 * x)
    du = lambda x: np.exp(x) * (np.cos(2 * x) - 2 * np.sin(2 * x))
    d2u = lambda x: np.exp(x) * (-3 * np.cos(2 * x) - 4 * np.sin(2 * x))
    f = lambda x: -d2u(x) + c * u(x)
    gl, gr = al * u(a) - du(a), ar * u(b) + du(b)
    B = obasis.make_basis(4, 18, a, b, ("robin", "robin"), alpha=(al, ar))
    o = obasis.assemble(B)
    rhs = o.T @ obasis.legendre_coefficients(B, f)
    rhs = rhs + gl * obasis.eval_matrix(B, [a])[0] + gr * obasis.eval_matrix(B, [b])[0]
    U = np.linalg.solve((o.K + c * o.M).toarray(), rhs)
    xs = np.linspace(a, b, 37)
    assert np.abs(obasis.eval_matrix(B, xs) @ U - u(xs)).max() < 1e-11
    # the same data with the boundary term's sign flipped misses by far
    Kbad = o.K - 2 * obasis.robin_term(B)
    Ubad = np.linalg.solve((Kbad + c * o.M).toarray(), rhs)
    assert np.abs(obasis.eval_matrix(B, xs) @ Ubad - u(xs)).max() > 1e-3


@pytest.mark.parametrize("bc,alpha", [(("dirichlet", "neumann"), (0, 0)), (("neumann", "dirichlet"), (0, 0)),
                                      (("robin", "robin"), (2.0, 0.5)), (("robin", "dirichlet"), (4.0, 0))])
def test_assemblies_agree_with_general_ends(bc, alpha):
    B = obasis.make_basis(3, 6, 0.0, 1.0, bc, breaks=[0.0, 0.3, 0.45, 1.0], alpha=alpha)
    o1, o2 = obasis.assemble(B), obasis.assemble_quadrature(B)
    assert np.abs((o1.K - o2.K).toarray()).max() < 1e-12
    assert np.abs((o1.M - o2.M).toarray()).max() < 1e-14
    assert B.nh == len(B.hat_vertices()) == 2 + sum(k != "dirichlet" for k in B.ends)


@pytest.mark.parametrize("bcx,ax,bcy,ay,coef", [
    (("dirichlet", "neumann"), (0, 0), ("neumann", "dirichlet"), (0, 0), None),
    (("robin", "robin"), (2.0, 0.5), "dirichlet", (0, 0), None),
    ("dirichlet", (0, 0), "dirichlet", (0, 0), (3.0, 0.0, 0.25, 5.0)),
    (("robin", "neumann"), (1.0, 0), "neumann", (0, 0), (1.0, 2.0, 0.5, 0.1)),
])
def test_adi_general_matches_kronecker(bcx, ax, bcy, ay, coef):
    ox = obasis.assemble(obasis.make_basis(3, 6, 0.0, 1.0, bcx, alpha=ax))
    oy = obasis.assemble(obasis.make_basis(2, 7, -1.0, 1.0, bcy, alpha=ay))
    omega2 = 0.0 if coef is not None else 1.0
    G = np.random.default_rng(7).standard_normal((ox.basis.N, oy.basis.N))
    ref = oadi.solve_dense(ox, oy, omega2, G, coef=coef)
    for eps in (1e-6, 1e-12):
        U = oadi.solve_adi(ox, oy, omega2, G, eps, coef=coef)
        assert oadi.rel_l2_error(U, ref, ox, oy) <= eps * (1 + 1e-3) + 1e-13
    # the operator the ADI inverts is the one the dense solve inverts
    assert np.abs(oadi.apply_operator(ox, oy, omega2, ref, coef=coef) - G).max() < 1e-9
