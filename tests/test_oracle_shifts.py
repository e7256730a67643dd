"""Pins for the oracle's elliptic functions, J and the Zolotarev shifts (Sec. 5, Alg. 2)."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import shifts

KPS = [0.9, 0.5, 0.21, 0.2, 0.05, 2e-4, 1e-6, 5.7e-8, 1.6e-11, 2.4e-12]


@pytest.mark.parametrize("kp", KPS)
def test_K_against_mpmath(kp):
    mp.mp.dps = 40
    ref = mp.ellipk(1 - mp.mpf(kp) ** 2)
    assert shifts.ellipk_from_kp(kp) == pytest.approx(float(ref), rel=1e-14)


@pytest.mark.parametrize("kp", KPS)
def test_dn_against_mpmath(kp):
    mp.mp.dps = 50
    m = 1 - mp.mpf(kp) ** 2
    K = shifts.ellipk_from_kp(kp)
    for t in [0.0, 1e-3, 0.05, 0.25, 0.5, 0.7, 0.95, 0.999, 1.0]:
        u = t * K
        ref = float(mp.ellipfun("dn", mp.mpf(u), m=m))
        assert shifts.jacobi_dn(u, kp) == pytest.approx(ref, rel=2e-13), (kp, t)


@pytest.mark.parametrize("kp", KPS)
def test_dn_special_values(kp):
    K = shifts.ellipk_from_kp(kp)
    assert shifts.jacobi_dn(0.0, kp) == pytest.approx(1.0, rel=1e-14)
    assert shifts.jacobi_dn(K, kp) == pytest.approx(kp, rel=1e-13)
    assert shifts.jacobi_dn(K / 2, kp) == pytest.approx(math.sqrt(kp), rel=1e-13)


INTERVALS = [(9.8696, 5.031e4, -5.031e4, -9.8696), (0.5, 3.056e10, -3.056e10, -0.5),
             (7.4674, 1.3077e8, -1.3077e8, -7.4674), (9.87, 5.0e4, -2.6e3, -2.47),
             (0.005, 2.093e9, -1.8e9, -509.87), (1.0, 3.0, -2.0, -0.5)]


@pytest.mark.parametrize("iv", INTERVALS)
@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-10, 1e-12])
def test_shifts_in_intervals_and_meet_bound(iv, eps):
    a, b, c, d = iv
    J, p, q = shifts.adi_shifts(a, b, c, d, eps)
    assert all(a * (1 - 1e-14) <= x <= b * (1 + 1e-14) for x in p)
    assert all(c * (1 + 1e-14) <= x <= d * (1 - 1e-14) for x in q)
    assert min(p) > 0 > max(q)
    rho = shifts.zolotarev_ratio(p, q, a, b, c, d)
    assert rho <= shifts.zolotarev_bound(a, b, c, d, J) * (1 + 1e-4)
    assert shifts.zolotarev_bound(a, b, c, d, J) <= eps * (1 + 1e-12)


def test_mobius_fourth_point():
    a, b, c, d = 9.87, 5.0e4, -2.6e3, -2.47
    gamma = abs(c - a) * abs(d - b) / (abs(c - b) * abs(d - a))
    alpha = -1 + 2 * gamma + 2 * math.sqrt(gamma * gamma - gamma)
    T = shifts.mobius(a, b, c, d, alpha)
    assert T(-alpha) == pytest.approx(a, rel=1e-14)
    assert T(-1.0) == pytest.approx(b, rel=1e-14)
    assert T(alpha) == pytest.approx(d, rel=1e-13)


def test_symmetric_formula_equals_general_mobius():
    a, b = 9.8696, 5.031e4
    J, p, q = shifts.adi_shifts(a, b, -b, -a, 1e-10)
    gamma = (a + b) ** 2 / (4 * a * b)
    alpha = -1 + 2 * gamma + 2 * math.sqrt(gamma * gamma - gamma)
    assert alpha == pytest.approx(b / a, rel=1e-10)
    T = shifts.mobius(a, b, -b, -a, alpha)
    K = shifts.ellipk_from_kp(1 / alpha)
    for j in range(1, J + 1):
        dn = shifts.jacobi_dn((2 * j - 1) * K / (2 * J), 1 / alpha)
        assert p[j - 1] == pytest.approx(T(-alpha * dn), rel=1e-9)
        assert q[j - 1] == pytest.approx(T(alpha * dn), rel=1e-9)


def test_iteration_count_formula():
    """J = ceil(log(16 gamma) log(4/eps)/pi^2) (Alg. 2); gamma = 1/4 * (a+b)^2/(ab) symmetric."""
    a, b = 1.0, 1e6
    gamma = (a + b) ** 2 / (4 * a * b)
    for eps in (1e-4, 1e-8, 1e-12):
        J = shifts.iteration_count(a, b, -b, -a, eps)
        assert J == math.ceil(math.log(16 * gamma) * math.log(4 / eps) / math.pi ** 2)
    # J grows like log N log(1/eps): doubling log(b/a) roughly doubles J (Sec. 5.2 lemma)
    J1 = shifts.iteration_count(1.0, 1e4, -1e4, -1.0, 1e-10)
    J2 = shifts.iteration_count(1.0, 1e8, -1e8, -1.0, 1e-10)
    assert 1.7 < J2 / J1 < 2.1


def test_high_precision_shifts():
    """Shifts from mpmath at 50 digits agree with the double-precision ones."""
    mp.mp.dps = 50
    a, b = mp.mpf("0.5"), mp.mpf("3.056e10")
    J, p, _ = shifts.adi_shifts(float(a), float(b), -float(b), -float(a), 1e-10)
    alpha = b / a
    m = 1 - 1 / alpha ** 2
    K = mp.ellipk(m)
    for j in range(1, J + 1):
        dn = mp.ellipfun("dn", (2 * j - 1) * K / (2 * J), m=m)
        assert p[j - 1] == pytest.approx(float(a / dn), rel=1e-12)
