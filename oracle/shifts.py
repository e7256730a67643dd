"""Iteration count and Zolotarev ADI shifts (oracle; test infrastructure only).

Alg. 2 of the paper (Sec. 5, precomputation) takes, for sigma(A, D) in [a, b]
and sigma(B, C) in [c, d],

    gamma = |c-a||d-b| / (|c-b||d-a|),   J = ceil(log(16 gamma) log(4/eps) / pi^2),

and shifts p_j > 0 > q_j from the explicit formula it cites (Fortunato and
Townsend 2020, eq. (2.4)), which the paper does not print.  The reading used
here (that construction restated):

    alpha = -1 + 2 gamma + 2 sqrt(gamma^2 - gamma),   complementary modulus k' = 1/alpha,
    u_j   = (2j - 1) K(k) / (2J),                       j = 1..J,
    p_j   = T(-alpha dn(u_j, k)),   q_j = T(alpha dn(u_j, k)),

with T the Mobius map sending -alpha, -1, 1, alpha to a, b, c, d.  Shifts are
ordered by increasing u_j (the paper states no order).

Elliptic functions, from first principles:
  K(k)  = pi / (2 AGM(1, k'))                  (Gauss's arithmetic-geometric mean)
  dn    : for k' <= 0.2 the hyperbolic-secant lattice sum
          dn(u, k) = (pi / (2K')) sum_m sech(pi (u - 2mK) / (2K')),  K' = K(k'),
          which converges geometrically with ratio exp(-pi K / K'); for larger
          k' the descending AGM (Landen) recursion for the amplitude, with the
          reflection dn(u) = k' / dn(K - u) for u > K/2.
k' is used directly (never 1 - k^2), since it reaches ~1e-12 at these sizes.
"""
from __future__ import annotations

import math


def agm(a: float, b: float) -> float:
    for _ in range(200):
        an, bn = 0.5 * (a + b), math.sqrt(a * b)
        if abs(an - bn) <= 4e-16 * an:
            return 0.5 * (an + bn)
        a, b = an, bn
    return 0.5 * (a + b)


def ellipk_from_kp(kp: float) -> float:
    """Complete elliptic integral K(k) as a function of k' = sqrt(1-k^2)."""
    return math.pi / (2.0 * agm(1.0, kp))


def _k_from_kp(kp: float) -> float:
    return math.sqrt((1.0 - kp) * (1.0 + kp))


def _dn_sech_sum(u: float, kp: float, K: float) -> float:
    Kp = ellipk_from_kp(_k_from_kp(kp))
    c = math.pi / (2.0 * Kp)
    s = 0.0
    for m in range(-8, 9):
        x = c * (u - 2.0 * m * K)
        if abs(x) < 700.0:
            s += 1.0 / math.cosh(x)
    return c * s


def _dn_landen(u: float, kp: float) -> float:
    a, b, c = 1.0, kp, _k_from_kp(kp)
    seq = []
    while abs(c) > 1e-17 * a and len(seq) < 60:
        seq.append((a, c))
        a, b, c = 0.5 * (a + b), math.sqrt(a * b), 0.5 * (a - b)
    seq.append((a, c))
    nsteps = len(seq) - 1
    phi = (2.0 ** nsteps) * a * u
    phis = [phi]
    for i in range(nsteps, 0, -1):
        ai, ci = seq[i]
        phi = 0.5 * (phi + math.asin(ci / ai * math.sin(phi)))
        phis.append(phi)
    phi0, phi1 = phis[-1], phis[-2] if len(phis) > 1 else phis[-1]
    return math.cos(phi0) / math.cos(phi1 - phi0)


def jacobi_dn(u: float, kp: float) -> float:
    """dn(u, k) for 0 <= u <= K(k), with the modulus given by k' = sqrt(1-k^2)."""
    K = ellipk_from_kp(kp)
    if kp <= 0.2:
        return _dn_sech_sum(u, kp, K)
    if u > 0.5 * K:
        return kp / _dn_landen(K - u, kp)
    return _dn_landen(u, kp)


def iteration_count(a: float, b: float, c: float, d: float, eps: float) -> int:
    gamma = abs(c - a) * abs(d - b) / (abs(c - b) * abs(d - a))
    return int(math.ceil(math.log(16.0 * gamma) * math.log(4.0 / eps) / math.pi ** 2))


def mobius(a: float, b: float, c: float, d: float, alpha: float):
    """T with T(-alpha)=a, T(-1)=b, T(1)=c (and T(alpha)=d by the choice of alpha),
    as the composition of the cross-ratio map phi(z) = cr(z; -alpha, -1, 1)
    with the inverse of psi(w) = cr(w; a, b, c)."""
    def T(z: float) -> float:
        phi = -2.0 * (z + alpha) / ((z - 1.0) * (alpha - 1.0))
        return (a * (b - c) - phi * c * (b - a)) / ((b - c) - phi * (b - a))
    return T


def adi_shifts(a: float, b: float, c: float, d: float, eps: float, J: int | None = None):
    """(J, p, q): shift lists for sigma(A, D) in [a, b], sigma(B, C) in [c, d]."""
    if not (a < b and c < d and (d < a or b < c)):
        raise ValueError("intervals must be nonempty and disjoint")
    gamma = abs(c - a) * abs(d - b) / (abs(c - b) * abs(d - a))
    if J is None:
        J = iteration_count(a, b, c, d, eps)
    alpha = -1.0 + 2.0 * gamma + 2.0 * math.sqrt(gamma * gamma - gamma)
    kp = 1.0 / alpha
    K = ellipk_from_kp(kp)
    symmetric = (c == -b and d == -a)
    T = mobius(a, b, c, d, alpha)
    ps, qs = [], []
    for j in range(1, J + 1):
        dn = jacobi_dn((2 * j - 1) * K / (2 * J), kp)
        if symmetric:
            # T(z) = -b/z when [c, d] = [-b, -a] (then alpha = b/a)
            ps.append(a / dn)
            qs.append(-a / dn)
        else:
            ps.append(T(-alpha * dn))
            qs.append(T(alpha * dn))
    return J, ps, qs


def zolotarev_ratio(ps, qs, a, b, c, d, npts: int = 4000) -> float:
    """max_{[a,b]} |r| / min_{[c,d]} |r| for r(z) = prod (z - p_j)/(z - q_j),
    on log-spaced grids (both intervals have one sign)."""
    import numpy as np

    def logr(z):
        z = np.asarray(z)[:, None]
        return np.sum(np.log(np.abs(z - np.asarray(ps)[None, :]))
                      - np.log(np.abs(z - np.asarray(qs)[None, :])), axis=1)

    def grid(lo, hi):
        s = 1.0 if lo > 0 else -1.0
        lo_, hi_ = sorted((abs(lo), abs(hi)))
        g = np.geomspace(lo_, hi_, npts)
        return s * g
    lab = logr(grid(a, b))
    lcd = logr(grid(c, d))
    return float(np.exp(np.max(lab) - np.min(lcd)))


def zolotarev_bound(a, b, c, d, J) -> float:
    """4 exp(-pi^2 J / log(16 gamma)), the bound behind the choice of J."""
    gamma = abs(c - a) * abs(d - b) / (abs(c - b) * abs(d - a))
    return 4.0 * math.exp(-math.pi ** 2 * J / math.log(16.0 * gamma))
