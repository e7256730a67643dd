"""GPU parity of the variable-coefficient operator and the ADI-preconditioned
Krylov solvers (Sec. 7) against the FP64 oracle (oracle/varcoef.py).

Tolerances: the operator is FP64 with a different summation order, 1e-12
relative; the solvers are judged by the oracle's own FP64 true residual of the
GPU result, which must meet the requested 1e-10, and by the iteration count of
the oracle's PCG/FCG with its own ADI preconditioner of the same tolerance
(equal up to one iteration: the two preconditioners agree to rounding).
"""
import numpy as np
import pytest

import workloads
from oracle import adi as oadi
from oracle import basis as obasis
from oracle import varcoef as ovc
from tests.gpu_helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]


@pytest.fixture(scope="module")
def hp():
    from paper_2402_11299_amd import hpadi
    hpadi.lib()
    return hpadi


def _setup(hp, nx, px, ny, py, bc, coef, seed, breaks_x=None):
    import torch
    Bx = obasis.make_basis(nx, px, 0.0, 1.0, bc) if breaks_x is None else obasis.Basis1D(np.asarray(breaks_x), px, bc)
    By = obasis.make_basis(ny, py, 0.0, 1.0, bc)
    gx, gy = ovc.gauss_grid(Bx), ovc.gauss_grid(By)
    if coef == "grf":
        a = workloads.grf_coefficient(gx.x, gy.x, seed=seed)
    elif coef == "singular":
        a = workloads.singular_coefficient(gx.x, gy.x, workloads.singular_x0(seed))
    elif coef == "one":
        a = np.ones((gx.x.size, gy.x.size))
    else:
        a = np.outer(1.0 + gx.x + 0.5 * gx.x ** 3, 2.0 - gy.x ** 2)
    x = hp.Op1D(nx, px, 0.0, 1.0, bc, breaks=breaks_x)
    y = hp.Op1D(ny, py, 0.0, 1.0, bc)
    vc = hp.VarCoef(x, y, torch.from_numpy(a).cuda())
    return Bx, By, a, x, y, vc


@pytest.mark.parametrize("nx,px,ny,py,bc,coef", [
    (3, 5, 4, 6, "dirichlet", "grf"), (2, 8, 3, 4, "neumann", "cubic"), (5, 3, 5, 3, "dirichlet", "singular"),
    (4, 16, 4, 16, "dirichlet", "grf"), (1, 2, 2, 3, "neumann", "grf"), (8, 32, 6, 33, "dirichlet", "grf")])
def test_operator_matches_oracle(hp, nx, px, ny, py, bc, coef):
    import torch
    print(f"varcoef apply {nx},{px},{ny},{py},{bc},{coef}", flush=True)
    Bx, By, a, x, y, vc = _setup(hp, nx, px, ny, py, bc, coef, seed=9)
    op = ovc.VarCoefOperator(Bx, By, a)
    U = np.random.default_rng(4).standard_normal((Bx.N, By.N))
    Y = vc.apply(torch.from_numpy(U).cuda()).cpu().numpy()
    Yref = op.apply(U)
    assert np.abs(Y - Yref).max() <= 1e-12 * np.abs(Yref).max()
    vc.close()


def test_operator_nonuniform_mesh(hp):
    import torch
    br = [0.0, 0.05, 0.2, 0.5, 1.0]
    Bx, By, a, x, y, vc = _setup(hp, 4, 6, 3, 5, "dirichlet", "grf", seed=2, breaks_x=br)
    op = ovc.VarCoefOperator(Bx, By, a)
    U = np.random.default_rng(5).standard_normal((Bx.N, By.N))
    Y = vc.apply(torch.from_numpy(U).cuda()).cpu().numpy()
    assert np.abs(Y - op.apply(U)).max() <= 1e-12 * np.abs(op.apply(U)).max()


def test_grid_matches_oracle(hp):
    x = hp.Op1D(3, 7, -1.0, 2.0, "neumann")
    xs, ws = hp.VarCoef.grid(x)
    g = ovc.gauss_grid(obasis.make_basis(3, 7, -1.0, 2.0, "neumann"))
    assert np.abs(xs - g.x).max() <= 1e-14 and np.abs(ws - g.w).max() <= 1e-14


@pytest.mark.parametrize("truncation", [0, 1, 2])
@pytest.mark.parametrize("coef", ["grf", "singular"])
def test_krylov_small_matches_oracle(hp, truncation, coef):
    import torch
    print(f"krylov small m={truncation} {coef}", flush=True)
    Bx, By, a, x, y, vc = _setup(hp, 4, 8, 4, 8, "dirichlet", coef, seed=3)
    ox, oy = obasis.assemble(Bx), obasis.assemble(By)
    op = ovc.VarCoefOperator(Bx, By, a)
    b = oadi.load(ox, oy, workloads.legendre_rhs(4, 8, 4, 8, seed=4))
    pre = hp.Plan(x, y, 0.0, 1e-4, "fp64")
    opre = oadi.ADIPlan(ox, oy, 0.0, 1e-4, interval=tuple(pre.interval))
    X, st, hist = vc.solve(torch.from_numpy(b).cuda(), pre, tol=1e-10, maxit=200, truncation=truncation,
                           hist_len=200)
    Xh = X.cpu().numpy()
    r = b - op.apply(Xh)
    true_rel = np.linalg.norm(r) / np.linalg.norm(b)
    if truncation == 0:
        ref = ovc.pcg(op.apply, lambda R: opre.solve(R), b, 1e-10, 200)
    else:
        ref = ovc.fcg(op.apply, lambda R: opre.solve(R), b, 1e-10, 200, m=truncation)
    print(f"  gpu iters={st.iters} true={true_rel:.2e} (lib {st.true_rel_res:.2e}); oracle iters={ref.iters}", flush=True)
    assert st.status == hp.HPADI_OK
    assert true_rel <= 1e-10 * (1 + 1e-6) and abs(st.true_rel_res - true_rel) <= 1e-3 * true_rel + 1e-15
    assert abs(st.iters - ref.iters) <= 1
    n = min(len(hist), len(ref.res_history), 5)
    assert np.allclose(hist[:n], ref.res_history[:n], rtol=1e-6)
    pre.close()
    vc.close()


def test_unit_coefficient_matches_plan_operator(hp):
    import torch
    Bx, By, a, x, y, vc = _setup(hp, 4, 10, 3, 9, "neumann", "one", seed=0)
    U = torch.from_numpy(np.random.default_rng(8).standard_normal((Bx.N, By.N))).cuda()
    plan = hp.Plan(x, y, 1.0, 1e-6, "fp64")  # A_Y = K + M/2; K (x) M + M (x) K = plan operator - M (x) M
    Y1 = vc.apply(U).cpu().numpy()
    Y2 = plan.apply(U).cpu().numpy()
    ox, oy = obasis.assemble(Bx), obasis.assemble(By)
    MM = (ox.M @ (oy.M @ U.cpu().numpy().T).T)
    assert np.abs(Y1 - (Y2 - MM)).max() <= 1e-12 * np.abs(Y1).max()
    plan.close()


@pytest.mark.parametrize("coef", ["grf", "singular"])
def test_full_size_fcg_reaches_tolerance(hp, coef):
    """n = p = 32 (N = 1023), the problem size of the learned-correction workload."""
    import torch
    cfg = workloads.CFG_VARCOEF_1K
    print(f"full-size fcg {coef}", flush=True)
    Bx, By, a, x, y, vc = _setup(hp, cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.bc, coef, seed=cfg.seed)
    ox, oy = obasis.assemble(Bx), obasis.assemble(By)
    op = ovc.VarCoefOperator(Bx, By, a)
    b = oadi.load(ox, oy, workloads.legendre_rhs(cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.seed))
    pre = hp.Plan(x, y, 0.0, 1e-4, "fp64")
    X, st, _ = vc.solve(torch.from_numpy(b).cuda(), pre, tol=cfg.tol, maxit=300, truncation=1)
    r = b - op.apply(X.cpu().numpy())
    true_rel = np.linalg.norm(r) / np.linalg.norm(b)
    print(f"  iters={st.iters} true={true_rel:.2e} t={st.t_ms:.1f} ms", flush=True)
    assert st.status == hp.HPADI_OK and true_rel <= cfg.tol * (1 + 1e-3)
    pre.close()
    vc.close()
