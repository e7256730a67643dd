"""Pins of the transform and Burgers oracle (oracle/transforms.py), Sec. 6.

* the grid formula sin(pi (m - 2k + 1) / (2m)) equals cos((2k - 1) pi / (2m)), the
  roots of the Chebyshev polynomial T_m (library routine);
* a piecewise polynomial of degree <= p is transformed exactly: its Legendre
  coefficients, known in closed form, are recovered from its grid values, and the
  inverse transform reproduces the values; F F^{-1} = I on random coefficients;
* R U R^T and D U R^T against direct evaluation of the basis functions and of
  their derivatives (finite differences of the basis evaluation);
* the Burgers step: with dt -> 0 the step is the identity to first order; for
  u = 0 it stays 0; and on a tiny grid it equals a brute-force step built from the
  dense Kronecker solve and pointwise evaluation of the hat+bubble expansion.
"""
import numpy as np
import pytest

import workloads
from oracle import adi as oadi
from oracle import basis as obasis
from oracle import transforms as otr


def test_grid_points_are_chebyshev_roots():
    for m in (1, 2, 5, 9, 65):
        x = otr.chebyshev_points(m)
        k = np.arange(1, m + 1)
        assert np.allclose(x, np.cos((2 * k - 1) * np.pi / (2 * m)), atol=1e-15)
        c = np.zeros(m + 1)
        c[m] = 1.0
        assert np.abs(np.polynomial.chebyshev.chebval(x, c)).max() < 1e-13


def test_closed_form_coefficients():
    """t^3 = 3/5 P_1(t) + 2/5 P_3(t) on the reference element; on [2, 5] the local
    coordinate t = (2x - 7) / 3 carries it over."""
    B = obasis.make_basis(1, 4, 2.0, 5.0, "dirichlet")
    xs = otr.grid(B)
    c = otr.values_to_legendre_1d(B, ((2 * xs - 7) / 3) ** 3)
    assert np.allclose(c, [0.0, 0.6, 0.0, 0.4, 0.0], atol=1e-14)
    # constants and the grid on each element of a non-uniform mesh
    B = obasis.make_basis(3, 2, 0.0, 1.0, "dirichlet", breaks=[0.0, 0.1, 0.5, 1.0])
    xs = otr.grid(B)
    assert np.all((xs[:3] > 0.0) & (xs[:3] < 0.1)) and np.all((xs[3:6] > 0.1) & (xs[3:6] < 0.5))
    assert np.allclose(otr.values_to_legendre_1d(B, np.ones(9)), [1, 1, 1, 0, 0, 0, 0, 0, 0], atol=1e-14)


@pytest.mark.parametrize("n,p", [(1, 1), (3, 4), (4, 9)])
def test_polynomials_transform_exactly(n, p):
    """A global polynomial of degree p is its own interpolant: the transform of its grid values
    equals its L2 projection computed by Gauss quadrature (a different route), and the inverse
    transform of random piecewise Legendre series equals their direct evaluation."""
    B = obasis.make_basis(n, p, -1.0, 2.0, "dirichlet", breaks=np.linspace(-1.0, 2.0, n + 1) ** 3 / 4)
    rng = np.random.default_rng(n + p)
    poly = np.polynomial.Polynomial(rng.standard_normal(p + 1))
    xs = otr.grid(B)
    assert np.allclose(otr.values_to_legendre_1d(B, poly(xs)), obasis.legendre_coefficients(B, poly),
                       atol=1e-10)
    c = rng.standard_normal(B.Nleg)
    v = np.zeros(xs.size)
    t = np.cos((2 * np.arange(1, p + 2) - 1) * np.pi / (2 * (p + 1)))
    for e in range(n):
        v[e * (p + 1):(e + 1) * (p + 1)] = np.polynomial.legendre.legval(t, c[e::n])
    assert np.allclose(otr.legendre_to_values_1d(B, c), v, atol=1e-12)
    assert np.allclose(otr.values_to_legendre_1d(B, v), c, atol=1e-11)


def test_2d_round_trip():
    Bx = obasis.make_basis(3, 5, 0.0, 1.0, "dirichlet")
    By = obasis.make_basis(2, 7, 0.0, 1.0, "neumann")
    F = np.random.default_rng(1).standard_normal((Bx.Nleg, By.Nleg))
    V = otr.legendre_to_values(Bx, By, F)
    assert np.allclose(otr.values_to_legendre(Bx, By, V), F, atol=1e-11)


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_connection_and_derivative_against_evaluation(bc):
    Bx = obasis.make_basis(3, 6, 0.0, 1.0, bc, breaks=[0.0, 0.2, 0.7, 1.0])
    By = obasis.make_basis(2, 4, -1.0, 1.0, bc)
    U = np.random.default_rng(2).standard_normal((Bx.N, By.N))
    xs, ys = otr.grid(Bx), otr.grid(By)
    Ex, Ey = obasis.eval_matrix(Bx, xs), obasis.eval_matrix(By, ys)
    # grid points are interior to their elements, so the elementwise evaluation is unambiguous
    vals = Ex @ U @ Ey.T
    assert np.allclose(otr.legendre_to_values(Bx, By, otr.q_to_legendre(Bx, By, U)), vals, atol=1e-11)
    h = 1e-6
    dEx = (obasis.eval_matrix(Bx, xs + h) - obasis.eval_matrix(Bx, xs - h)) / (2 * h)
    dvals = dEx @ U @ Ey.T
    got = otr.legendre_to_values(Bx, By, otr.q_to_legendre(Bx, By, U, deriv_x=True))
    assert np.abs(got - dvals).max() <= 1e-6 * np.abs(dvals).max()


def test_burgers_step_limits():
    Bx = obasis.make_basis(2, 4, 0.0, 1.0, "dirichlet")
    o = obasis.assemble(Bx)
    assert np.abs(otr.burgers_step(o, o, 0.1, 1e-3, np.zeros((Bx.Nleg, Bx.Nleg)))).max() == 0.0
    # a smooth u_k vanishing on the boundary: one tiny step changes it by O(dt)
    f = lambda x: np.sin(np.pi * x)
    F = np.outer(obasis.legendre_coefficients(Bx, f), obasis.legendre_coefficients(Bx, f))
    d1 = np.abs(otr.burgers_step(o, o, 0.1, 1e-4, F) - F).max()
    d2 = np.abs(otr.burgers_step(o, o, 0.1, 2e-4, F) - F).max()
    assert d1 < 1e-2 and 1.5 < d2 / d1 < 2.5


def test_burgers_step_against_brute_force():
    """Tiny grid: the implicit half-step by the dense Kronecker solve of
    (M (x) M + dt eps (K (x) M + M (x) K)) vec U = vec(load(u_k)), the explicit half-step by
    evaluating the hat+bubble expansion and its x-derivative at the grid (eval_matrix,
    finite differences), and interpolation back by the Legendre Vandermonde system."""
    eps, dt = 0.1, 1e-2
    B = obasis.make_basis(2, 3, 0.0, 1.0, "dirichlet")
    o = obasis.assemble(B)
    F = np.random.default_rng(3).standard_normal((B.Nleg, B.Nleg)) * 0.3
    M, K = o.M.toarray(), o.K.toarray()
    A = np.kron(M, M) + dt * eps * (np.kron(K, M) + np.kron(M, K))
    U = np.linalg.solve(A, oadi.load(o, o, F).reshape(-1)).reshape(B.N, B.N)
    xs = otr.grid(B)
    E = obasis.eval_matrix(B, xs)
    h = 1e-6
    dE = (obasis.eval_matrix(B, xs + h) - obasis.eval_matrix(B, xs - h)) / (2 * h)
    V = E @ U @ E.T
    Vx = dE @ U @ E.T
    W = V - dt * Vx * V
    # interpolate back: per element the Legendre Vandermonde system at the reference points
    Vand = np.polynomial.legendre.legvander(otr.chebyshev_points(B.p + 1), B.p)
    m, n = B.p + 1, B.n
    ref = np.zeros((B.Nleg, B.Nleg))
    for ex in range(n):
        for ey in range(n):
            blk = np.linalg.solve(Vand, np.linalg.solve(Vand, W[ex * m:(ex + 1) * m, ey * m:(ey + 1) * m]).T).T
            for kx in range(m):
                for ky in range(m):
                    ref[kx * n + ex, ky * n + ey] = blk[kx, ky]
    got = otr.burgers_step(o, o, eps, dt, F, solve="dense")
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()


def test_burgers_step_follows_characteristics():
    """With a vanishing viscosity the step approximates the inviscid Burgers flow
    u_t + u u_x = 0, whose solution for a short time is u(x, y, t) = u0(x - t u, y)
    (characteristics; fixed-point iteration).  Explicit Euler is first-order accurate,
    so the step lands within O(dt^2) of it, while the opposite sign of the convection
    term would miss by O(dt)."""
    eps, dt = 1e-6, 1e-3
    B = obasis.make_basis(4, 12, 0.0, 1.0, "dirichlet")
    o = obasis.assemble(B)
    f = lambda x: np.sin(np.pi * x)
    cx = obasis.legendre_coefficients(B, f)
    F = np.outer(cx, cx)
    got = otr.legendre_to_values(B, B, otr.burgers_step(o, o, eps, dt, F))
    xs = otr.grid(B)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    u = f(X) * f(Y)
    for _ in range(50):
        u = f(X - dt * u) * f(Y)
    step = np.abs(u - f(X) * f(Y)).max()
    assert step > 1e-3
    assert np.abs(got - u).max() < 2e-2 * step
