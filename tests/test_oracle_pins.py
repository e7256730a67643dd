"""Independent pins for oracle functions that every GPU parity verdict relies on.

* ``adi.rel_l2_error``, the error metric of the ADI lemma (Sec. 5.1; the norm of
  V E L^T with M^x = V^T V, M^y = L^T L), against the L2 norm of the function
  difference computed by tensor Gauss quadrature of the basis functions evaluated
  pointwise (no assembled matrix involved);
* ``shifts.iteration_count`` (Alg. 2) from both sides: J shifts reach the
  tolerance and a family of J - 1 shifts does not, measured on the rational
  function itself (the Zolotarev ratio of the shift family on a fine grid);
* ``spectrum.lemma_bounds`` (Sec. 5.2 lemma "Spectrum") against the textbook
  eigenvalues of linear elements, for which both ends of the lemma are sharp as
  h -> 0: the lower end pi^2/l^2 is the continuous Dirichlet eigenvalue and the
  upper end 12/h^2 + omega^2/2 is the limit of the highest discrete mode.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import adi, basis, shifts, spectrum


def _gauss_l2_sq(Bx, By, X):
    """integral of u_h^2 over the rectangle for u_h(x, y) = sum X[i, j] phi_i(x) psi_j(y),
    by a tensor Gauss rule with p + 2 points per element (exact for the degree-2p
    polynomial integrand on each element)."""
    def rule(B):
        t, w = np.polynomial.legendre.leggauss(B.p + 2)
        pts, wts = [], []
        for e in range(B.n):
            pts.append(B.x[e] + (t + 1.0) * B.delta[e] / 2.0)
            wts.append(w * B.delta[e] / 2.0)
        return np.concatenate(pts), np.concatenate(wts)
    xs, wx = rule(Bx)
    ys, wy = rule(By)
    vals = basis.eval_matrix(Bx, xs) @ X @ basis.eval_matrix(By, ys).T
    return float(wx @ (vals ** 2) @ wy)


NONSQUARE = [((3, 5, 0.0, 1.0, None), (5, 4, 0.0, 2.0, None), "dirichlet"),
             ((4, 6, -1.0, 1.0, None), (2, 9, 0.0, 0.5, None), "neumann"),
             ((4, 4, 0.0, 1.0, [0.0, 0.1, 0.35, 0.7, 1.0]), (3, 7, 0.0, 3.0, [0.0, 2.0, 2.5, 3.0]), "dirichlet"),
             ((2, 12, 0.0, 1.0, [0.0, 0.01, 1.0]), (6, 2, -2.0, 1.0, None), "neumann")]


@pytest.mark.parametrize("mx,my,bc", NONSQUARE)
def test_rel_l2_error_against_pointwise_quadrature(mx, my, bc):
    Bx = basis.make_basis(mx[0], mx[1], mx[2], mx[3], bc, breaks=mx[4])
    By = basis.make_basis(my[0], my[1], my[2], my[3], bc, breaks=my[4])
    ox, oy = basis.assemble(Bx), basis.assemble(By)
    rng = np.random.default_rng(17)
    Uref = rng.standard_normal((Bx.N, By.N))
    U = Uref + 1e-3 * rng.standard_normal((Bx.N, By.N))
    ref = math.sqrt(_gauss_l2_sq(Bx, By, U - Uref) / _gauss_l2_sq(Bx, By, Uref))
    assert adi.rel_l2_error(U, Uref, ox, oy) == pytest.approx(ref, rel=1e-10)
    # transposing the roles of the axes gives a different value on these grids, so a
    # swap of M^x and M^y inside the metric would not pass the line above
    assert Bx.N != By.N


# intervals of the configurations (large gamma, where the Zolotarev bound is tight)
WIDE = [(9.8696, 5.031e4, -5.031e4, -9.8696), (0.5, 3.056e10, -3.056e10, -0.5),
        (7.4674, 1.3077e8, -1.3077e8, -7.4674), (9.87, 5.0e4, -2.6e3, -2.47),
        (0.005, 2.093e9, -1.8e9, -509.87)]


@pytest.mark.parametrize("iv", WIDE)
@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-10, 1e-12])
def test_iteration_count_is_the_least_sufficient(iv, eps):
    """J is the least count whose bound 4 exp(-pi^2 J / log 16 gamma) is <= eps, and a
    family of J - 1 shifts, built the same way, misses eps on its own rational function."""
    J = shifts.iteration_count(*iv, eps)
    assert shifts.zolotarev_bound(*iv, J) <= eps < shifts.zolotarev_bound(*iv, J - 1)
    _, p, q = shifts.adi_shifts(*iv, eps)
    assert shifts.zolotarev_ratio(p, q, *iv) <= eps
    _, p1, q1 = shifts.adi_shifts(*iv, eps, J=J - 1)
    assert shifts.zolotarev_ratio(p1, q1, *iv) > eps


@pytest.mark.parametrize("n", [16, 64, 256])
@pytest.mark.parametrize("w2", [0.0, 4.0])
def test_lemma_bounds_sharp_for_linear_elements(n, w2):
    """p = 1 on [0, 2], Dirichlet: the extreme generalised eigenvalues of (A_Y, M) approach
    the lemma's ends, within O(h^2) (the factor the textbook eigenvalues
    (6/h^2)(1 - cos k pi h)/(2 + cos k pi h) + omega^2/2 give)."""
    ell = 2.0
    B = basis.make_basis(n, 1, 0.0, ell, basis.DIRICHLET)
    ops = basis.assemble(B)
    lam = sla.eigh(ops.A(w2).toarray(), ops.M.toarray(), eigvals_only=True)
    lo, hi = spectrum.lemma_bounds(ops, w2)
    h = ell / n
    assert lo <= lam[0] and lam[-1] <= hi
    # lower end: 1/C = max(pi^2/l^2, min(1, w2/2)) against pi^2/l^2 + w2/2
    assert lo == pytest.approx(max(math.pi ** 2 / ell ** 2, min(1.0, w2 / 2.0)), rel=1e-15)
    if w2 == 0.0:
        assert lam[0] / lo <= 1.0 + (math.pi * h) ** 2 / 6.0
    # upper end: 12/h^2 + w2/2, reached by the alternating mode as h -> 0
    assert hi == pytest.approx(12.0 / h ** 2 + w2 / 2.0, rel=1e-14)
    assert lam[-1] / hi >= 1.0 - 2.0 * (math.pi / n) ** 2
