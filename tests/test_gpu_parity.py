"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances:
* factorisation, load, operator apply: FP64 rounding, 1e-12 relative;
* FP64 ADI with the same interval and shifts as the oracle's Alg. 2: the two
  runs differ only in rounding order, 1e-10 relative in the error norm;
* ADI against an exact solve: the tolerance of the ADI lemma (Sec. 5.1),
  tol * (1 + 1e-3) (the interval margin makes the GPU run at least as accurate);
* mixed precision: the requested tolerance (1e-10) against the exact solve.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import adi as oadi
from oracle import basis as obasis
from oracle import cholesky as ochol
from tests.gpu_helpers import ROUNDING_ALLOWANCE, factor_len, gpu_available, structured_to_dense

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]


@pytest.fixture(scope="module")
def hp():
    from paper_2402_11299_amd import hpadi
    hpadi.lib()
    return hpadi


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    return _t


def oracle_ops(n, p, bc, lo=0.0, hi=1.0):
    return obasis.assemble(obasis.make_basis(n, p, lo, hi, bc))


def oracle_interval(ox, oy, w2):
    from oracle import spectrum
    ax, bx = spectrum.interval(ox, w2)
    ay, by = spectrum.interval(oy, w2)
    return (ax, bx * 1.001, -by * 1.001, -ay)


FACTOR_CASES = [(4, 8, "dirichlet", 0.0), (3, 7, "neumann", 2.0), (1, 5, "dirichlet", 1.0),
                (1, 2, "neumann", 1.0), (5, 3, "dirichlet", 10.0), (6, 12, "neumann", 0.1),
                (2, 33, "dirichlet", 0.0), (3, 64, "neumann", 1.0)]


@pytest.mark.parametrize("n,p,bc,w2", FACTOR_CASES)
def test_factor_matches_oracle(hp, torch, n, p, bc, w2):
    print(f"factor case n={n} p={p} bc={bc} w2={w2}", flush=True)
    x = hp.Op1D(n, p, 0.0, 1.0, bc)
    ox = oracle_ops(n, p, bc)
    iv = oracle_interval(ox, ox, w2)
    plan = hp.Plan(x, x, w2, 1e-8, "fp64", interval=iv)
    Ay = ox.A(w2).toarray()
    My = ox.M.toarray()
    for j in list(range(min(plan.J, 4))) + [plan.J - 1, -1]:
        buf = hp.hpadi_plan_export_factor(plan.handle, j, 1, factor_len(n, p, bc))
        L = structured_to_dense(buf, n, p, bc)
        S = My if j == -1 else Ay + plan.p[j] * My
        Lref = ochol.reverse_cholesky_dense(S)
        assert np.abs(L - Lref).max() <= 1e-12 * np.abs(Lref).max(), j
        assert np.abs(L.T @ L - S).max() <= 1e-13 * np.abs(S).max(), j
    plan.close()


@pytest.mark.parametrize("nx,px,ny,py,bc", [(4, 8, 4, 8, "dirichlet"), (3, 7, 5, 6, "neumann"),
                                            (1, 2, 2, 3, "neumann"), (32, 32, 32, 32, "dirichlet"),
                                            (16, 32, 12, 24, "neumann")])
def test_load_and_apply_match_oracle(hp, torch, nx, px, ny, py, bc):
    print(f"load/apply case {nx},{px},{ny},{py},{bc}", flush=True)
    x, y = hp.Op1D(nx, px, 0, 1, bc), hp.Op1D(ny, py, 0, 2, bc)
    ox, oy = oracle_ops(nx, px, bc), oracle_ops(ny, py, bc, 0.0, 2.0)
    w2 = 3.0
    plan = hp.Plan(x, y, w2, 1e-6, "fp64", interval=oracle_interval(ox, oy, w2))
    F = workloads.legendre_rhs(nx, px, ny, py, seed=11)
    G = plan.load(torch.from_numpy(F).cuda()).cpu().numpy()
    Gref = oadi.load(ox, oy, F)
    assert np.abs(G - Gref).max() <= 1e-14 * max(1.0, np.abs(Gref).max())
    U0 = np.random.default_rng(5).standard_normal((ox.basis.N, oy.basis.N))
    Y = plan.apply(torch.from_numpy(U0).cuda()).cpu().numpy()
    Yref = oadi.apply_operator(ox, oy, w2, U0)
    assert np.abs(Y - Yref).max() <= 1e-12 * np.abs(Yref).max()
    plan.close()


ADI_CASES = [(4, 8, 4, 8, "dirichlet", 0.0, 1e-12), (3, 6, 3, 6, "neumann", 1.0, 1e-12),
             (2, 9, 2, 9, "dirichlet", 10.0, 1e-10), (4, 8, 3, 10, "dirichlet", 0.0, 1e-10),
             (2, 12, 5, 6, "neumann", 0.3, 1e-12), (1, 2, 3, 3, "neumann", 2.0, 1e-8),
             (7, 5, 3, 17, "dirichlet", 50.0, 1e-12), (5, 4, 5, 4, "neumann", 1e3, 1e-12),
             (8, 64, 4, 64, "dirichlet", 1.0, 1e-10)]


@pytest.mark.parametrize("nx,px,ny,py,bc,w2,tol", ADI_CASES)
def test_fp64_adi_matches_oracle_alg2(hp, torch, nx, px, ny, py, bc, w2, tol):
    print(f"adi case {nx},{px},{ny},{py},{bc},{w2},{tol}", flush=True)
    x, y = hp.Op1D(nx, px, 0, 1, bc), hp.Op1D(ny, py, 0, 2, bc)
    ox, oy = oracle_ops(nx, px, bc), oracle_ops(ny, py, bc, 0.0, 2.0)
    iv = oracle_interval(ox, oy, w2)
    plan = hp.Plan(x, y, w2, tol, "fp64", interval=iv)
    oplan = oadi.ADIPlan(ox, oy, w2, tol, interval=iv)
    assert plan.J == oplan.J
    assert np.allclose(plan.p, oplan.p, rtol=1e-12) and np.allclose(plan.q, oplan.q, rtol=1e-12)
    F = workloads.legendre_rhs(nx, px, ny, py, seed=3)
    G = oadi.load(ox, oy, F)
    U, st = plan.solve(torch.from_numpy(G).cuda())
    U = U.cpu().numpy()
    Uo = oplan.solve(G)
    assert oadi.rel_l2_error(U, Uo, ox, oy) <= 1e-10
    # element by element: the same shifts in FP64; the GPU works in mass-balanced
    # coordinates, the oracle on U, so the roundings differ by up to the mass matrices'
    # condition number times the unit roundoff
    ediff = np.abs(U - Uo).max() / np.abs(Uo).max()
    cond = max(np.linalg.cond(ox.M.toarray()), np.linalg.cond(oy.M.toarray()))
    print(f"  J={plan.J} elementwise max rel diff vs oracle Alg. 2: {ediff:.2e} (cond M {cond:.1e})", flush=True)
    assert ediff <= max(1e-11, 4 * 2.2e-16 * cond)
    # exact solve: dense Kronecker on small grids, fast diagonalisation with refinement else
    small = ox.basis.N * oy.basis.N <= 4096
    Uref = oadi.solve_dense(ox, oy, w2, G) if small else oadi.solve_fdm(ox, oy, w2, G, refine=2)
    assert oadi.rel_l2_error(U, Uref, ox, oy) <= tol * (1 + 1e-3) + 1e-13
    plan.close()


@pytest.mark.parametrize("nx,px,ny,py,bc,w2", [(8, 16, 8, 16, "dirichlet", 0.0), (6, 20, 7, 18, "neumann", 1.0),
                                                (4, 33, 4, 33, "neumann", 0.5)])
def test_mixed_precision_reaches_tolerance(hp, torch, nx, px, ny, py, bc, w2):
    print(f"mixed case {nx},{px},{ny},{py},{bc},{w2}", flush=True)
    x, y = hp.Op1D(nx, px, 0, 1, bc), hp.Op1D(ny, py, 0, 1, bc)
    ox, oy = oracle_ops(nx, px, bc), oracle_ops(ny, py, bc)
    plan = hp.Plan(x, y, w2, 1e-10, "mixed")
    G = oadi.load(ox, oy, workloads.legendre_rhs(nx, px, ny, py, seed=2))
    U, st = plan.solve(torch.from_numpy(G).cuda())
    Uref = oadi.solve_fdm(ox, oy, w2, G, refine=2)
    err = oadi.rel_l2_error(U.cpu().numpy(), Uref, ox, oy)
    print("mixed rounds", st.rounds, "est", st.est_rel_err, "err", err, "phase ms", list(st.t_ms), flush=True)
    assert st.est_rel_err <= 1e-10 and err <= st.est_rel_err + ROUNDING_ALLOWANCE
    assert st.rounds >= 2
    # phase times: FP32 rounds, FP64 rounds and residuals all ran
    assert st.t_ms[0] > 0 and st.t_ms[1] > 0 and st.t_ms[2] > 0
    plan.close()


@pytest.mark.parametrize("draw", ["decaying", "flat", "highfreq"])
@pytest.mark.parametrize("nx,px,bc,w2", [(8, 16, "dirichlet", 0.0), (6, 20, "neumann", 1.0),
                                         (16, 32, "dirichlet", 3.0)])
def test_mixed_error_bound_is_sound(hp, torch, nx, px, bc, w2, draw):
    """The stopping bound of the mixed solve (the ADI lemma, Sec. 5.1, with the correction
    and the iterate measured in the lemma's norm) is at least the true relative error
    against a known exact solution (round trip U0 -> G0 = A U0 -> U), for smooth, flat
    and high-degree solutions; and the solve meets its tolerance."""
    print(f"bound case {nx},{px},{bc},{w2},{draw}", flush=True)
    x = hp.Op1D(nx, px, 0, 1, bc)
    ox = oracle_ops(nx, px, bc)
    gen = {"decaying": workloads.decaying_coefficients, "highfreq": workloads.highfreq_coefficients,
           "flat": lambda a, b, c, d, e, seed: np.random.default_rng(seed).standard_normal((ox.basis.N, ox.basis.N))}
    U0 = gen[draw](nx, px, nx, px, bc, seed=21)
    G0 = oadi.apply_operator(ox, ox, w2, U0)
    for tol in (1e-10, 1e-8):
        plan = hp.Plan(x, x, w2, tol, "mixed")
        U, st = plan.solve(torch.from_numpy(G0).cuda())
        err = oadi.rel_l2_error(U.cpu().numpy(), U0, ox, ox)
        print(f"  tol {tol}: rounds={st.rounds} est={st.est_rel_err:.3e} err={err:.3e}", flush=True)
        assert st.status == hp.HPADI_OK
        assert st.est_rel_err <= tol and err <= st.est_rel_err + ROUNDING_ALLOWANCE
        plan.close()


@pytest.mark.parametrize("lw,clw,rlw", [(8, 0, 0), (0, 8, 0), (0, 0, 8), (4, 0, 0)])
@pytest.mark.parametrize("nx,px,ny,py", [(8, 128, 4, 32), (8, 64, 4, 64)])
def test_mixed_workgroup_widths_long_chains(hp, torch, lw, clw, rlw, nx, px, ny, py):
    """p = 128 or 64 (64- or 32-step chains, whose recurrences read lane copies of their
    coefficients) on few elements, every workgroup width per direction: the last workgroup
    of a pass holds lines that do not exist, whose lanes must not disturb the others (a
    regression: lane copies of coefficients left stale by such lanes gave NaN at 8 lines
    per workgroup)."""
    w2, bc = 10.0, "neumann"
    print(f"widths {lw},{clw},{rlw} at {nx},{px} x {ny},{py}", flush=True)
    x, y = hp.Op1D(nx, px, 0, 1, bc), hp.Op1D(ny, py, 0, 1, bc)
    ox, oy = oracle_ops(nx, px, bc), oracle_ops(ny, py, bc)
    U0 = workloads.decaying_coefficients(nx, px, ny, py, bc, seed=52)
    G0 = oadi.apply_operator(ox, oy, w2, U0)
    o = hp.hpadi_options()
    o.lines_per_block, o.col_lines_per_block, o.row_lines_per_block = lw, clw, rlw
    plan = hp.Plan(x, y, w2, 1e-10, "mixed", options=o)
    U, st = plan.solve(torch.from_numpy(G0).cuda())
    err = oadi.rel_l2_error(U.cpu().numpy(), U0, ox, oy)
    print(f"  rounds={st.rounds} est={st.est_rel_err:.2e} err={err:.2e}", flush=True)
    assert st.status == hp.HPADI_OK and err <= 1e-10
    plan.close()


@pytest.mark.parametrize("refine_tol", [0.0, 1e-8])
def test_mixed_shift_families(hp, torch, refine_tol):
    """A mixed plan builds one shift family for its FP32 round (inner_tol, default 3e-7) and
    one for its first FP64 refinement round (default tol / inner_tol); both counts are
    those of the Zolotarev formula for the plan's interval, and the solve meets the
    tolerance.  A third round would take a looser ladder family, never more shifts."""
    nx, px, bc, w2, tol = 8, 16, "dirichlet", 0.0, 1e-10
    x, y = hp.Op1D(nx, px, 0, 1, bc), hp.Op1D(nx, px, 0, 1, bc)
    ox = oracle_ops(nx, px, bc)
    opts = hp.hpadi_options()
    opts.refine_tol = refine_tol
    plan = hp.Plan(x, y, w2, tol, "mixed", options=opts)
    G = oadi.load(ox, ox, workloads.legendre_rhs(nx, px, nx, px, seed=4))
    U, st = plan.solve(torch.from_numpy(G).cuda())
    eps1 = refine_tol if refine_tol > 0 else tol / 3e-7
    assert st.J == hp.hpadi_shifts(plan.interval, 3e-7)[0] == plan.J
    assert st.J_refine == hp.hpadi_shifts(plan.interval, eps1)[0]
    assert st.J + st.J_refine <= st.iters <= st.J + (st.rounds - 1) * st.J_refine
    Uref = oadi.solve_fdm(ox, ox, w2, G, refine=2)
    err = oadi.rel_l2_error(U.cpu().numpy(), Uref, ox, ox)
    print("families", st.J, st.J_refine, "rounds", st.rounds, "err", err, flush=True)
    assert err <= tol
    plan.close()


def test_fp64_1k_config_against_fdm(hp, torch):
    """Screened Poisson, omega^2 = 10 on [-1,1] x [0,2], n = p = 32 (N = 1023), tol 1e-12."""
    cfg = workloads.CFG_FP64_1K
    print("cfg", cfg.name, flush=True)
    x = hp.Op1D(cfg.nx, cfg.px, cfg.ax, cfg.bx, cfg.bc)
    y = hp.Op1D(cfg.ny, cfg.py, cfg.ay, cfg.by, cfg.bc)
    ox = oracle_ops(cfg.nx, cfg.px, cfg.bc, cfg.ax, cfg.bx)
    oy = oracle_ops(cfg.ny, cfg.py, cfg.bc, cfg.ay, cfg.by)
    plan = hp.Plan(x, y, cfg.omega2, cfg.tol, "fp64")
    F = workloads.legendre_rhs(cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.seed)
    G = torch.from_numpy(F).cuda()
    Gd = plan.load(G)
    U, st = plan.solve(Gd)
    Uref = oadi.solve_fdm(ox, oy, cfg.omega2, oadi.load(ox, oy, F), refine=2)
    err = oadi.rel_l2_error(U.cpu().numpy(), Uref, ox, oy)
    print("J", plan.J, "err", err, flush=True)
    assert err <= cfg.tol * (1 + 1e-3)
    plan.close()


def test_manufactured_sine_fp64(hp, torch):
    """u = sin(pi x) sin(pi y) on [-1,1] x [0,2], omega^2 = 10 (the 1K configuration's domain)."""
    w2 = 10.0
    n, p = 8, 24
    x, y = hp.Op1D(n, p, -1, 1, "dirichlet"), hp.Op1D(n, p, 0, 2, "dirichlet")
    Bx = obasis.make_basis(n, p, -1, 1, "dirichlet")
    By = obasis.make_basis(n, p, 0, 2, "dirichlet")
    fx, fy, scale = workloads.manufactured_sin(w2)
    F = scale * np.outer(obasis.legendre_coefficients(Bx, fx), obasis.legendre_coefficients(By, fy))
    plan = hp.Plan(x, y, w2, 1e-13, "fp64")
    U, _ = plan.solve(plan.load(torch.from_numpy(F).cuda()))
    xs, ys = np.linspace(-1, 1, 29), np.linspace(0, 2, 31)
    vals = obasis.eval_matrix(Bx, xs) @ U.cpu().numpy() @ obasis.eval_matrix(By, ys).T
    assert np.abs(vals - np.outer(np.sin(math.pi * xs), np.sin(math.pi * ys))).max() < 1e-11
    plan.close()


def test_plan_errors(hp):
    xn = hp.Op1D(4, 6, 0, 1, "neumann")
    with pytest.raises(hp.HpadiError) as ei:
        hp.Plan(xn, xn, 0.0, 1e-8)
    assert ei.value.status == hp.HPADI_ESINGULAR
    xd = hp.Op1D(4, 6, 0, 1, "dirichlet")
    with pytest.raises(hp.HpadiError) as ei:
        hp.Plan(xd, xd, 0.0, 1e-8, interval=(1.0, 10.0, 2.0, 20.0))
    assert ei.value.status == hp.HPADI_EINTERVAL
    # an interval whose shifts make K + (w/2 - q) M indefinite: q_j > lambda_min
    with pytest.raises(hp.HpadiError) as ei:
        hp.Plan(xd, xd, 0.0, 1e-8, interval=(-5e4, -20.0, -1e6, -9e5))
    assert ei.value.status in (hp.HPADI_ENOTSPD, hp.HPADI_EINTERVAL)
