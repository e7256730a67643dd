"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds no arithmetic of the method: only problem descriptions and random
draws.  Inputs are shaped like the paper's experiments (screened Poisson on a
rectangle, uniform or given breakpoints, random Legendre right-hand sides;
Sec. 4 and Sec. 5 experiments use "random samples" for f).

Right-hand side recipe: the piecewise tensor-Legendre coefficients of f are

    F[(kx, ex), (ky, ey)] = Z * (1 + kx)^-2 * (1 + ky)^-2,   Z ~ N(0, 1) i.i.d.,

indexed degree-major (row kx*nx + ex, column ky*ny + ey), drawn with
numpy.random.default_rng(seed).standard_normal in row-major order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Problem:
    """One screened-Poisson problem on [ax, bx] x [ay, by]."""

    name: str
    nx: int
    px: int
    ny: int
    py: int
    omega2: float
    bc: str            # "dirichlet" or "neumann" (both axes)
    tol: float
    seed: int
    ax: float = 0.0
    bx: float = 1.0
    ay: float = 0.0
    by: float = 1.0

    def dims(self):
        def N(n, p):
            return n * p - 1 if self.bc == "dirichlet" else n * p + 1
        return N(self.nx, self.px), N(self.ny, self.py)

    def leg_dims(self):
        return (self.px + 1) * self.nx, (self.py + 1) * self.ny


def legendre_rhs(nx: int, px: int, ny: int, py: int, seed: int) -> np.ndarray:
    """F of shape ((px+1) nx, (py+1) ny), FP64, per the module recipe."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal(((px + 1) * nx, (py + 1) * ny))
    kx = np.arange((px + 1) * nx) // nx
    ky = np.arange((py + 1) * ny) // ny
    return Z * (1.0 + kx)[:, None] ** -2 * (1.0 + ky)[None, :] ** -2


def q_degrees(n: int, p: int, bc: str) -> np.ndarray:
    """Polynomial degree of each coefficient in the degree-major hat+bubble order:
    hats have degree 1, the bubble block W_m (m = 0..p-2) degree m + 2."""
    nh = n - 1 if bc == "dirichlet" else n + 1
    return np.concatenate([np.ones(nh, dtype=np.int64), 2 + np.arange(n * (p - 1)) // n])


def decaying_coefficients(nx: int, px: int, ny: int, py: int, bc: str, seed: int) -> np.ndarray:
    """A random coefficient array U in the hat+bubble basis with entries
    Z (1+kx)^-2 (1+ky)^-2, k the degree of the basis function (round-trip tests)."""
    rng = np.random.default_rng(seed)
    kx, ky = q_degrees(nx, px, bc), q_degrees(ny, py, bc)
    Z = rng.standard_normal((kx.size, ky.size))
    return Z * (1.0 + kx)[:, None] ** -2 * (1.0 + ky)[None, :] ** -2


def highfreq_coefficients(nx: int, px: int, ny: int, py: int, bc: str, seed: int) -> np.ndarray:
    """A random coefficient array concentrated on the highest degrees: N(0,1) entries where
    either degree is at least p - 3, hats with alternating signs along each axis, and zero
    elsewhere (round-trip tests of the error bound on rough solutions)."""
    rng = np.random.default_rng(seed)
    kx, ky = q_degrees(nx, px, bc), q_degrees(ny, py, bc)
    Z = rng.standard_normal((kx.size, ky.size))
    top = (kx[:, None] >= px - 3) | (ky[None, :] >= py - 3)
    sx = np.where(kx == 1, (-1.0) ** np.arange(kx.size), 0.0)
    sy = np.where(ky == 1, (-1.0) ** np.arange(ky.size), 0.0)
    return np.where(top, Z, 0.0) + np.outer(sx, sy)


# The problem families (uniform meshes, both axes share the BC):
CFG_SMALL = Problem("poisson_n4_p8_dirichlet", 4, 8, 4, 8, 0.0, "dirichlet", 1e-12, 0)
CFG_FP64_1K = Problem("screened_n32_p32_dirichlet_w2_10", 32, 32, 32, 32, 10.0, "dirichlet",
                      1e-12, 1, ax=-1.0, bx=1.0, ay=0.0, by=2.0)
CFG_MIXED_4K_D = Problem("poisson_n64_p64_dirichlet", 64, 64, 64, 64, 0.0, "dirichlet", 1e-10, 2)
CFG_MIXED_4K_N = Problem("screened_n64_p64_neumann_w2_1", 64, 64, 64, 64, 1.0, "neumann", 1e-10, 2)
CFG_VARCOEF_1K = Problem("varcoef_n32_p32_dirichlet", 32, 32, 32, 32, 0.0, "dirichlet", 1e-10, 4)

PROBLEMS = {p.name: p for p in (CFG_SMALL, CFG_FP64_1K, CFG_MIXED_4K_D, CFG_MIXED_4K_N,
                                CFG_VARCOEF_1K)}


@dataclasses.dataclass(frozen=True)
class BatchInstance:
    nx: int
    px: int
    ny: int
    py: int
    omega2: float
    bc: str
    seed: int


def draw_batch(count: int = 512, seed: int = 3, nmax_dofs: int = 2049):
    """Independent instances: per axis n in {4,8,16,32,64}, p in {8,16,32,64,128},
    redrawn until n p + 1 <= nmax_dofs; omega^2 log-uniform in [1e-2, 1e3];
    BC Dirichlet or Neumann with equal probability, the same on both axes."""
    rng = np.random.default_rng(seed)
    ns = np.array([4, 8, 16, 32, 64])
    ps = np.array([8, 16, 32, 64, 128])
    out = []
    for i in range(count):
        def axis():
            while True:
                n, p = int(rng.choice(ns)), int(rng.choice(ps))
                if n * p + 1 <= nmax_dofs:
                    return n, p
        nx, px = axis()
        ny, py = axis()
        omega2 = float(10.0 ** rng.uniform(-2.0, 3.0))
        bc = "dirichlet" if rng.random() < 0.5 else "neumann"
        out.append(BatchInstance(nx, px, ny, py, omega2, bc, seed * 100003 + i))
    return out


def manufactured_sin(omega2: float):
    """u = sin(pi x) sin(pi y), f = (2 pi^2 + omega^2) u, as separable factors."""
    def fx(x):
        return np.sin(math.pi * x)
    return fx, fx, 2.0 * math.pi ** 2 + omega2


# ---------------------------------------------------------------------------
# Variable coefficients a(x, y) for -div(a grad u) = f, sampled at given points
# (the tensor grid of quadrature points of the discretisation).
# ---------------------------------------------------------------------------

def _se_factor(x: np.ndarray, ell: float, jitter: float) -> np.ndarray:
    """A square root S (S S^T = C) of the squared-exponential covariance
    C_ij = exp(-(x_i - x_j)^2 / (2 ell^2)) + jitter delta_ij, by a symmetric
    eigendecomposition (negative rounding-level eigenvalues clipped)."""
    d = x[:, None] - x[None, :]
    C = np.exp(-0.5 * (d / ell) ** 2) + jitter * np.eye(x.size)
    lam, V = np.linalg.eigh(C)
    return V * np.sqrt(np.clip(lam, 0.0, None))[None, :]


def grf_coefficient(xs: np.ndarray, ys: np.ndarray, seed: int, ell: float = 0.2,
                    jitter: float = 1e-10) -> np.ndarray:
    """a = 1 + exp(g)/2 on the tensor grid xs x ys, g a centred Gaussian field
    with separable squared-exponential covariance (length scale ell, variance 1),
    sampled as g = S_x Z S_y^T with Z ~ N(0, 1) i.i.d. (default_rng(seed))."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((xs.size, ys.size))
    g = _se_factor(np.asarray(xs, float), ell, jitter) @ Z @ _se_factor(np.asarray(ys, float), ell, jitter).T
    return 1.0 + 0.5 * np.exp(g)


def singular_coefficient(xs: np.ndarray, ys: np.ndarray, x0: float) -> np.ndarray:
    """a = |x - x0|^(1/2) + 1/10 on the tensor grid xs x ys."""
    return np.repeat((np.sqrt(np.abs(np.asarray(xs, float) - x0)) + 0.1)[:, None], len(ys), axis=1)


def singular_x0(seed: int) -> float:
    """x0 ~ U(0, 1) for the singular coefficient family."""
    return float(np.random.default_rng(seed).uniform(0.0, 1.0))


# ---------------------------------------------------------------------------
# Sec. 7's singular problem (-Delta - 10 log r) u = 1 on (-1, 1)^2, zero Dirichlet,
# on a tensor mesh graded towards the origin.
# ---------------------------------------------------------------------------

def graded_breakpoints(m: int) -> np.ndarray:
    """-1, -10^-1, ..., -10^-m, 0, 10^-m, ..., 10^-1, 1: 2 (m + 1) cells on (-1, 1)."""
    pos = 10.0 ** -np.arange(m, 0, -1)          # 10^-m, ..., 10^-1
    return np.concatenate([[-1.0], -pos[::-1], [0.0], pos, [1.0]])


def log_potential(xs: np.ndarray, ys: np.ndarray, scale: float = 10.0) -> np.ndarray:
    """c(x, y) = -scale log sqrt(x^2 + y^2) on the tensor grid xs x ys."""
    return -scale * 0.5 * np.log(np.asarray(xs, float)[:, None] ** 2 + np.asarray(ys, float)[None, :] ** 2)


def constant_rhs(n: int, p: int, value: float = 1.0) -> np.ndarray:
    """The piecewise Legendre coefficients of a constant f (degree 0 on every element), as a
    1D vector of length (p + 1) n in degree-major order; F = outer(fx, fy) in 2D."""
    f = np.zeros((p + 1) * n)
    f[:n] = value
    return f


# ---------------------------------------------------------------------------
# Burgers' equation (Sec. 6): a discontinuous initial condition.
# ---------------------------------------------------------------------------

def burgers_initial(nx: int, px: int, ny: int, py: int, blocks: int = 3, seed: int = 0) -> np.ndarray:
    """Piecewise Legendre coefficients ((px+1) nx x (py+1) ny, degree-major) of a piecewise
    constant u0: blocks x blocks equal tiles of the element mesh (nx and ny divisible by
    blocks), each with a constant drawn U(-1, 1) (default_rng(seed), row-major over tiles).
    Only the degree-0 coefficients are nonzero."""
    if nx % blocks or ny % blocks:
        raise ValueError("the tiles must be unions of elements")
    vals = np.random.default_rng(seed).uniform(-1.0, 1.0, (blocks, blocks))
    F = np.zeros(((px + 1) * nx, (py + 1) * ny))
    F[:nx, :ny] = np.repeat(np.repeat(vals, nx // blocks, axis=0), ny // blocks, axis=1)
    return F
