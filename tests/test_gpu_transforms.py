"""GPU parity of the grid transforms and of the Burgers step (Sec. 6) against the oracle.

Tolerances come from the rounding of the dot products each pass computes: an entry of
T_x V T_y^T computed in FP64 (by either side) is within about (m_x + m_y) eps of the
entry, relative to the same product formed with absolute values, |T_x| |V| |T_y|^T
(eps = 2^-53; the test allows a factor 4).  The Burgers step also carries the
ADI tolerance of its solve through the evaluation and the derivative.
"""
import numpy as np
import pytest

import workloads
from oracle import basis as obasis
from oracle import transforms as otr
from tests.gpu_helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

EPS = 2.0 ** -53

# (n_x, p_x, n_y, p_y, bc, x breakpoints): chunk sizes 8, 16 and 33 (one, two and four
# chunks of outputs), ragged column tiles, non-uniform elements
CASES = [
    (3, 5, 4, 7, "dirichlet", None),
    (2, 12, 5, 20, "neumann", [0.0, 0.3, 1.0]),
    (9, 40, 5, 64, "dirichlet", list(np.cumsum([0.0, 0.05, 0.1, 0.2, 0.1, 0.05, 0.2, 0.1, 0.1, 0.1]))),
    (2, 128, 3, 100, "neumann", None),
]


@pytest.fixture(scope="module")
def hp():
    from paper_2402_11299_amd import hpadi
    hpadi.lib()
    return hpadi


def setup(hp, case):
    nx, px, ny, py, bc, brx = case
    ax, bx = (brx[0], brx[-1]) if brx else (0.0, 1.0)
    Bx = obasis.make_basis(nx, px, ax, bx, bc, brx)
    By = obasis.make_basis(ny, py, -1.0, 1.0, bc)
    x = hp.Op1D(nx, px, ax, bx, bc, brx)
    y = hp.Op1D(ny, py, -1.0, 1.0, bc)
    return Bx, By, x, y


def dense_1d(B, fn):
    """The 1D map fn as a dense matrix (applied to the identity)."""
    return fn(np.eye(B.Nleg))


def check(got, ref, bound, what):
    err = np.abs(got - ref)
    ratio = (err / np.maximum(bound, 1e-300)).max()
    print(f"  {what}: max err {err.max():.2e}, max err / rounding bound {ratio:.3f}", flush=True)
    assert np.all(err <= bound), what


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}_{c[2]}x{c[3]}_{c[4]}")
def test_transforms_match_oracle(hp, case):
    import torch
    print(f"transforms {case[:5]}", flush=True)
    Bx, By, x, y = setup(hp, case)
    t = hp.Transform(x, y)
    rng = np.random.default_rng(11)
    V = rng.standard_normal((Bx.Nleg, By.Nleg))
    F = rng.standard_normal((Bx.Nleg, By.Nleg)) / (1.0 + np.arange(Bx.Nleg) // Bx.n)[:, None]
    Tx = dense_1d(Bx, lambda I: otr.values_to_legendre_1d(Bx, I))
    Ty = dense_1d(By, lambda I: otr.values_to_legendre_1d(By, I))
    Ix = dense_1d(Bx, lambda I: otr.legendre_to_values_1d(Bx, I))
    Iy = dense_1d(By, lambda I: otr.legendre_to_values_1d(By, I))
    mx, my = Bx.p + 1, By.p + 1
    gamma = 4 * (mx + my + 4) * EPS

    Fg = t.values_to_legendre(torch.from_numpy(V).cuda()).cpu().numpy()
    check(Fg, otr.values_to_legendre(Bx, By, V), gamma * (np.abs(Tx) @ np.abs(V) @ np.abs(Ty).T), "F_p")
    Vg = t.legendre_to_values(torch.from_numpy(F).cuda()).cpu().numpy()
    check(Vg, otr.legendre_to_values(Bx, By, F), gamma * (np.abs(Ix) @ np.abs(F) @ np.abs(Iy).T), "F_p^-1")
    # the round trip is the identity up to the rounding of both transforms
    back = t.values_to_legendre(torch.from_numpy(Vg).cuda()).cpu().numpy()
    assert np.abs(back - F).max() <= 1e-12 * np.abs(F).max() * (mx + my)
    t.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}_{c[2]}x{c[3]}_{c[4]}")
@pytest.mark.parametrize("deriv", [0, 1])
def test_q_to_values_match_oracle(hp, case, deriv):
    import torch
    print(f"q_to_values {case[:5]} deriv={deriv}", flush=True)
    Bx, By, x, y = setup(hp, case)
    t = hp.Transform(x, y)
    U = np.random.default_rng(12).standard_normal((Bx.N, By.N))
    Vg = t.q_to_values(torch.from_numpy(U).cuda(), deriv_x=bool(deriv)).cpu().numpy()
    ref = otr.legendre_to_values(Bx, By, otr.q_to_legendre(Bx, By, U, deriv_x=bool(deriv)))
    # the oracle converts to Legendre coefficients and then evaluates, so its rounding is bounded
    # through the absolute values of both factors (the library applies their product)
    Ix = otr.legendre_to_values_1d(Bx, np.eye(Bx.Nleg))
    Iy = otr.legendre_to_values_1d(By, np.eye(By.Nleg))
    Ex = np.abs(Ix) @ np.abs(_q_matrix(Bx, bool(deriv)))
    Ey = np.abs(Iy) @ np.abs(_q_matrix(By, False))
    gamma = 4 * (Bx.p + By.p + 6) * EPS
    check(Vg, ref, gamma * (np.abs(Ex) @ np.abs(U) @ np.abs(Ey).T), "values of du/dx" if deriv else "values of u")
    t.close()


def _q_matrix(B, deriv):
    """Legendre coefficients of the basis functions (or their derivatives), Nleg x N."""
    R = (obasis.connection_full(B) @ obasis.restriction(B)).toarray()
    D = (obasis.derivative_full(B) @ obasis.restriction(B)).toarray()
    return D if deriv else R


@pytest.mark.parametrize("bc,n,p,breaks,steps,prec", [
    ("dirichlet", 3, 8, None, 1, "fp64"),
    ("dirichlet", 9, 12, None, 3, "fp64"),
    ("neumann", 4, 20, [-1.0, -0.2, 0.0, 0.5, 1.0], 2, "fp64"),
    ("dirichlet", 6, 16, None, 2, "mixed"),
])
def test_burgers_steps_match_oracle(hp, bc, n, p, breaks, steps, prec):
    """Steps of the IMEX scheme from the discontinuous initial condition (eps = 0.1, as in
    Sec. 6) against the oracle's steps with the exact discrete solve (fast diagonalisation).
    The GPU solve meets tol = 1e-12 in the ADI lemma's norm; the step's evaluation and
    derivative amplify that by at most about 2 p^2 / delta_min dt max|u| relative, which
    the 1e-9 allowance covers for these sizes."""
    import torch
    print(f"burgers {bc} n={n} p={p} steps={steps} {prec}", flush=True)
    eps, dt, tol = 0.1, 1e-3, 1e-12
    a, b = (breaks[0], breaks[-1]) if breaks else (-1.0, 1.0)
    B = obasis.make_basis(n, p, a, b, bc, breaks)
    o = obasis.assemble(B)
    op = hp.Op1D(n, p, a, b, bc, breaks)
    F0 = workloads.burgers_initial(n, p, n, p, blocks=n if n % 3 else 3, seed=5)
    ref = F0.copy()
    for _ in range(steps):
        ref = otr.burgers_step(o, o, eps, dt, ref)
    bu = hp.Burgers(op, op, eps, dt, tol, prec)
    Fg = torch.from_numpy(F0).cuda()
    st = bu.step(Fg, steps)
    got = Fg.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  J={st.J} rounds={st.rounds} rel max err {err:.2e}", flush=True)
    assert st.status == hp.HPADI_OK
    assert err <= 1e-9
    bu.close()


def test_full_size_transforms_sampled(hp):
    """n = p = 64 on both axes (N = 4095, 4160 grid points per axis), in the launch
    configuration of the benchmark: sampled element blocks of F_p, F_p^{-1} and of the
    Q -> values map against the oracle on one element (the reference-element transform
    does not depend on the element), and the full round trip."""
    import torch
    n = p = 64
    m = p + 1
    print("full-size transforms n=p=64", flush=True)
    x = hp.Op1D(n, p, 0.0, 1.0, "dirichlet")
    t = hp.Transform(x, x)
    rng = np.random.default_rng(13)
    V = torch.from_numpy(rng.standard_normal((n * m, n * m))).cuda()
    F = t.values_to_legendre(V)
    B1 = obasis.make_basis(1, p, 0.0, 1.0, "neumann")
    Vh, Fh = V.cpu().numpy(), F.cpu().numpy()
    T1 = otr.values_to_legendre_1d(B1, np.eye(m))
    for ex, ey in [(0, 0), (63, 63), (17, 40), (40, 17), (5, 62)]:
        blk = Vh[ex * m:(ex + 1) * m, ey * m:(ey + 1) * m]
        ref = otr.values_to_legendre(B1, B1, blk)
        got = Fh[ex::n, ey::n]
        bound = 4 * (2 * m + 4) * EPS * (np.abs(T1) @ np.abs(blk) @ np.abs(T1).T)
        assert np.all(np.abs(got - ref) <= bound), (ex, ey)
    back = t.legendre_to_values(F)
    assert (back - V).abs().max().item() <= 1e-12 * V.abs().max().item() * 2 * m
    # Q -> values of u and du/dx on sampled blocks: gather the local coefficients
    U = rng.standard_normal((n * p - 1, n * p - 1))
    Ud = torch.from_numpy(U).cuda()
    Bx = obasis.make_basis(n, p, 0.0, 1.0, "dirichlet")
    for deriv in (False, True):
        Vq = t.q_to_values(Ud, deriv_x=deriv).cpu().numpy()
        for ex, ey in [(0, 0), (63, 30), (31, 63)]:
            Bex = obasis.make_basis(1, p, Bx.x[ex], Bx.x[ex + 1], "neumann")
            Bey = obasis.make_basis(1, p, Bx.x[ey], Bx.x[ey + 1], "neumann")
            loc = _local(U, ex, ey, n, p)
            ref = otr.legendre_to_values(Bex, Bey, otr.q_to_legendre(Bex, Bey, loc, deriv_x=deriv))
            got = Vq[ex * m:(ex + 1) * m, ey * m:(ey + 1) * m]
            scale = np.abs(ref).max()
            assert np.abs(got - ref).max() <= 1e-12 * scale * (1 + 2 * p * deriv), (deriv, ex, ey)
    t.close()


def _local(U, ex, ey, n, p):
    """Local hat+bubble coefficients [left hat, right hat, W_0 .. W_{p-2}] of element pair
    (ex, ey) of a Dirichlet array (absent boundary hats are zero)."""
    def idx(e):
        out = []
        for v in (e, e + 1):
            out.append(v - 1 if 1 <= v <= n - 1 else -1)
        out += [n - 1 + j * n + e for j in range(p - 1)]
        return out
    ix, iy = idx(ex), idx(ey)
    L = np.zeros((p + 1, p + 1))
    for a, i in enumerate(ix):
        for b, j in enumerate(iy):
            if i >= 0 and j >= 0:
                L[a, b] = U[i, j]
    return L
