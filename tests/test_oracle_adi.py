"""Pins for the oracle's ADI (Sec. 5, Alg. 2 and its error lemma) and references."""
import math

import numpy as np
import pytest

import workloads
from oracle import adi, basis, spectrum


def ops_pair(nx, px, ny, py, bc, xr=(0.0, 1.0), yr=(0.0, 1.0)):
    Bx = basis.make_basis(nx, px, xr[0], xr[1], bc)
    By = basis.make_basis(ny, py, yr[0], yr[1], bc)
    return basis.assemble(Bx), basis.assemble(By)


CASES = [(4, 8, 4, 8, "dirichlet", 0.0), (3, 6, 3, 6, "neumann", 1.0), (2, 9, 2, 9, "dirichlet", 10.0),
         (4, 8, 3, 10, "dirichlet", 0.0), (2, 12, 5, 6, "neumann", 0.3), (3, 7, 6, 5, "dirichlet", 50.0)]


@pytest.mark.parametrize("nx,px,ny,py,bc,w2", CASES)
@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-10, 1e-12])
def test_adi_meets_lemma_bound_against_dense_kronecker(nx, px, ny, py, bc, w2, eps):
    ox, oy = ops_pair(nx, px, ny, py, bc, yr=(0.0, 2.0))
    F = workloads.legendre_rhs(nx, px, ny, py, seed=7)
    G = adi.load(ox, oy, F)
    Uref = adi.solve_dense(ox, oy, w2, G)
    plan = adi.ADIPlan(ox, oy, w2, eps)
    U = plan.solve(G)
    err = adi.rel_l2_error(U, Uref, ox, oy)
    assert err <= eps * (1 + 1e-6) + 1e-14


def test_fdm_with_refinement_matches_dense():
    ox, oy = ops_pair(3, 8, 4, 6, "neumann")
    G = adi.load(ox, oy, workloads.legendre_rhs(3, 8, 4, 6, seed=2))
    assert adi.rel_l2_error(adi.solve_fdm(ox, oy, 0.5, G), adi.solve_dense(ox, oy, 0.5, G), ox, oy) < 1e-13


def test_small_config_error():
    cfg = workloads.CFG_SMALL
    ox, oy = ops_pair(cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.bc)
    G = adi.load(ox, oy, workloads.legendre_rhs(cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.seed))
    plan = adi.ADIPlan(ox, oy, cfg.omega2, cfg.tol)
    err = adi.rel_l2_error(plan.solve(G), adi.solve_dense(ox, oy, cfg.omega2, G), ox, oy)
    assert err <= cfg.tol


def test_manufactured_sine():
    """u = sin(pi x) sin(pi y) on [-1,1] x [0,2], omega^2 = 10, f = (2 pi^2 + omega^2) u."""
    w2 = 10.0
    ox, oy = ops_pair(4, 14, 4, 14, "dirichlet", xr=(-1.0, 1.0), yr=(0.0, 2.0))
    fx, fy, scale = workloads.manufactured_sin(w2)
    F = scale * np.outer(basis.legendre_coefficients(ox.basis, fx),
                         basis.legendre_coefficients(oy.basis, fy))
    G = adi.load(ox, oy, F)
    U = adi.ADIPlan(ox, oy, w2, 1e-13).solve(G)
    xs = np.linspace(-1, 1, 23)
    ys = np.linspace(0, 2, 19)
    vals = basis.eval_matrix(ox.basis, xs) @ U @ basis.eval_matrix(oy.basis, ys).T
    exact = np.outer(np.sin(math.pi * xs), np.sin(math.pi * ys))
    assert np.abs(vals - exact).max() < 1e-11


def test_polynomial_solution_is_exact():
    """u = x(1-x) y(1-y) is in the discrete space for p >= 2, and f = 2x(1-x) + 2y(1-y)
    is a polynomial, so the Galerkin solution equals u (to rounding)."""
    ox, oy = ops_pair(3, 4, 2, 5, "dirichlet")
    q = lambda x: x * (1 - x)
    one = lambda x: np.ones_like(x)
    cq_x, c1_x = basis.legendre_coefficients(ox.basis, q), basis.legendre_coefficients(ox.basis, one)
    cq_y, c1_y = basis.legendre_coefficients(oy.basis, q), basis.legendre_coefficients(oy.basis, one)
    F = 2 * np.outer(c1_x, cq_y) + 2 * np.outer(cq_x, c1_y)
    G = adi.load(ox, oy, F)
    U = adi.ADIPlan(ox, oy, 0.0, 1e-14).solve(G)
    xs, ys = np.linspace(0, 1, 17), np.linspace(0, 1, 13)
    vals = basis.eval_matrix(ox.basis, xs) @ U @ basis.eval_matrix(oy.basis, ys).T
    assert np.abs(vals - np.outer(q(xs), q(ys))).max() < 1e-13


def test_round_trip_random_U():
    ox, oy = ops_pair(3, 7, 4, 5, "neumann")
    U0 = np.random.default_rng(3).standard_normal((ox.basis.N, oy.basis.N))
    G = adi.apply_operator(ox, oy, 2.0, U0)
    U = adi.ADIPlan(ox, oy, 2.0, 1e-12).solve(G)
    assert adi.rel_l2_error(U, U0, ox, oy) <= 1e-12


def test_half_steps_satisfy_their_equations():
    """Each half step of Alg. 2 solves its shifted equation (checked by the residual)."""
    ox, oy = ops_pair(3, 6, 4, 5, "dirichlet")
    G = adi.load(ox, oy, workloads.legendre_rhs(3, 6, 4, 5, 9))
    plan = adi.ADIPlan(ox, oy, 1.0, 1e-6)
    _, hist = plan.solve(G, return_history=True)
    Ax, Ay, Mx, My = plan.Ax.toarray(), plan.Ay.toarray(), ox.M.toarray(), oy.M.toarray()
    Wprev = np.zeros_like(G)
    for j, (Wh, W) in enumerate(hist):
        p, q = plan.p[j], plan.q[j]
        # W_{j-1/2} (B - p C) = G - (A - p D) W_{j-1},  B = -A_y, C = M_y, D = M_x
        r1 = Wh @ (-Ay - p * My) - (G - (Ax - p * Mx) @ Wprev)
        r2 = (Ax - q * Mx) @ W - (G - Wh @ (-Ay - q * My))
        scale = np.abs(G).max() + np.abs(Wh).max() * np.abs(Ay).max()
        assert np.abs(r1).max() < 1e-11 * scale
        assert np.abs(r2).max() < 1e-11 * scale
        Wprev = W


def test_interval_contains_spectrum_and_inside_lemma():
    for bc, w2 in (("dirichlet", 0.0), ("neumann", 1.0), ("dirichlet", 10.0)):
        B = basis.make_basis(6, 9, 0.0, 1.0, bc)
        ops = basis.assemble(B)
        lo = spectrum.lower_end(ops, w2)
        lmin, lmax = spectrum.extreme_eigenvalues(ops, w2)
        assert lo <= lmin * (1 + 1e-10)
        if bc == "neumann":
            assert lmin == pytest.approx(w2 / 2, rel=1e-8)
        Lo, Hi = spectrum.lemma_bounds(ops, w2)
        assert Lo <= lmin * (1 + 1e-9) and lmax <= Hi  # dense eigh is ~1e-11 accurate at the low end
