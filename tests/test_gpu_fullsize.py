"""GPU parity at the full benchmark size, n = p = 64 (N = 4095 Dirichlet, 4097
Neumann), in the launch configuration bench.py times.

The exact discrete solution is known by construction (round trip): U0 is drawn,
G0 = A_Y^x U0 M^y + M^x U0 A_Y^y is formed by the FP64 oracle, the GPU solves
G0, and the relative L2 function error against U0 (the norm of the ADI lemma,
Sec. 5.1) must meet the requested tolerance 1e-10.  Three draws: coefficients
decaying like (1+k)^-2 in the degree (the shape of a solution for the
benchmark's right-hand sides), flat N(0,1) coefficients (every mode equally
excited) and coefficients on the highest degrees only (the hardest case for the
refinement).  For mixed solves the stopping bound must also cover the true error.
"""
import numpy as np
import pytest

import workloads
from oracle import adi as oadi
from oracle import basis as obasis
from tests.gpu_helpers import ROUNDING_ALLOWANCE, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

CASES = [(workloads.CFG_MIXED_4K_D, "mixed"), (workloads.CFG_MIXED_4K_N, "mixed"),
         (workloads.CFG_MIXED_4K_D, "fp64"), (workloads.CFG_MIXED_4K_N, "fp64")]


@pytest.fixture(scope="module")
def hp():
    from paper_2402_11299_amd import hpadi
    hpadi.lib()
    return hpadi


@pytest.mark.parametrize("cfg,prec", CASES, ids=lambda v: getattr(v, "name", v))
@pytest.mark.parametrize("draw", ["decaying", "flat", "highfreq"])
def test_full_size_round_trip(hp, cfg, prec, draw):
    import torch
    print(f"full-size round trip {cfg.name} {prec} {draw}", flush=True)
    ox = obasis.assemble(obasis.make_basis(cfg.nx, cfg.px, cfg.ax, cfg.bx, cfg.bc))
    oy = obasis.assemble(obasis.make_basis(cfg.ny, cfg.py, cfg.ay, cfg.by, cfg.bc))
    if draw == "decaying":
        U0 = workloads.decaying_coefficients(cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.bc, seed=cfg.seed + 100)
    elif draw == "highfreq":
        U0 = workloads.highfreq_coefficients(cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.bc, seed=cfg.seed + 400)
    else:
        U0 = np.random.default_rng(cfg.seed + 200).standard_normal((ox.basis.N, oy.basis.N))
    G0 = oadi.apply_operator(ox, oy, cfg.omega2, U0)
    x = hp.Op1D(cfg.nx, cfg.px, cfg.ax, cfg.bx, cfg.bc)
    y = hp.Op1D(cfg.ny, cfg.py, cfg.ay, cfg.by, cfg.bc)
    plan = hp.Plan(x, y, cfg.omega2, cfg.tol, prec)
    U, st = plan.solve(torch.from_numpy(G0).cuda())
    err = oadi.rel_l2_error(U.cpu().numpy(), U0, ox, oy)
    print(f"  rounds={st.rounds} J={st.J} est={st.est_rel_err:.2e} err={err:.2e}", flush=True)
    assert st.status == hp.HPADI_OK
    assert err <= cfg.tol
    if prec == "mixed":
        # the stopping bound (ADI lemma in its own norm) is sound
        assert st.est_rel_err <= cfg.tol and err <= st.est_rel_err + ROUNDING_ALLOWANCE
    plan.close()


@pytest.mark.parametrize("lw,clw", [(1, 0), (8, 1), (1, 8), (4, 0)])
def test_full_size_workgroup_widths(hp, lw, clw):
    """The same round trip with one line per workgroup (column passes placed panel by
    panel on one XCD) and the other widths of the half-sweeps."""
    import torch
    cfg = workloads.CFG_MIXED_4K_D
    print(f"full-size round trip lines_per_block={lw} col={clw}", flush=True)
    ox = obasis.assemble(obasis.make_basis(cfg.nx, cfg.px, cfg.ax, cfg.bx, cfg.bc))
    oy = obasis.assemble(obasis.make_basis(cfg.ny, cfg.py, cfg.ay, cfg.by, cfg.bc))
    U0 = workloads.decaying_coefficients(cfg.nx, cfg.px, cfg.ny, cfg.py, cfg.bc, seed=cfg.seed + 300)
    G0 = oadi.apply_operator(ox, oy, cfg.omega2, U0)
    x = hp.Op1D(cfg.nx, cfg.px, cfg.ax, cfg.bx, cfg.bc)
    y = hp.Op1D(cfg.ny, cfg.py, cfg.ay, cfg.by, cfg.bc)
    o = hp.hpadi_options()
    o.lines_per_block = lw
    o.col_lines_per_block = clw
    for prec in ("mixed", "fp64"):
        plan = hp.Plan(x, y, cfg.omega2, cfg.tol, prec, options=o)
        U, st = plan.solve(torch.from_numpy(G0).cuda())
        err = oadi.rel_l2_error(U.cpu().numpy(), U0, ox, oy)
        print(f"  {prec}: rounds={st.rounds} err={err:.2e}", flush=True)
        assert st.status == hp.HPADI_OK and err <= cfg.tol
        plan.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_nonuniform_mesh(hp, prec):
    """n = p = 64 on a mesh with jittered breakpoints (element widths within +-30% of uniform):
    the general half-sweep kernels (the uniform-mesh kernels need equal widths), at full size,
    round trip against the exact solution."""
    import torch
    rng = np.random.default_rng(31)
    n = p = 64
    w = 1.0 + 0.3 * rng.uniform(-1.0, 1.0, n)
    br = np.concatenate([[0.0], np.cumsum(w / w.sum())])
    br[-1] = 1.0
    print(f"full-size non-uniform mesh {prec}", flush=True)
    ox = obasis.assemble(obasis.make_basis(n, p, 0.0, 1.0, "dirichlet", breaks=br))
    U0 = workloads.decaying_coefficients(n, p, n, p, "dirichlet", seed=32)
    G0 = oadi.apply_operator(ox, ox, 0.0, U0)
    x = hp.Op1D(n, p, 0.0, 1.0, "dirichlet", breaks=list(br))
    plan = hp.Plan(x, x, 0.0, 1e-10, prec)
    U, st = plan.solve(torch.from_numpy(G0).cuda())
    err = oadi.rel_l2_error(U.cpu().numpy(), U0, ox, ox)
    print(f"  rounds={st.rounds} J={st.J} est={st.est_rel_err:.2e} err={err:.2e}", flush=True)
    assert st.status == hp.HPADI_OK and err <= 1e-10
    plan.close()
