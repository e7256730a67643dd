"""Failure handling, forced from the host (every kernel still runs to its end):

* a non-finite right-hand side: the mixed solve ends ENOCONV (no hang, no
  fault); the bound it reports is not finite;
* an unreachable tolerance (1e-20, below FP64 rounding): ENOCONV after the round
  limit, with an answer as accurate as FP64 allows;
* data beyond the FP32 range (|G| ~ 1e40): the FP32 round overflows, the solve
  starts again with FP64 rounds only and meets the tolerance;
* a learned correction with garbage weights: the corrected FCG is given up and
  plain ADI-PCG (Sec. 7) finishes the solve to the tolerance on the FP64 true
  residual.
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


def _round_trip(n, p, bc, w2, scale=1.0):
    o = obasis.assemble(obasis.make_basis(n, p, 0.0, 1.0, bc))
    U0 = scale * workloads.decaying_coefficients(n, p, n, p, bc, seed=31)
    return o, U0, oadi.apply_operator(o, o, w2, U0)


def test_nonfinite_rhs_ends_enoconv(hp):
    import torch
    print("failure: NaN in G", flush=True)
    o, U0, G0 = _round_trip(8, 16, "dirichlet", 1.0)
    G0[3, 5] = np.nan
    x = hp.Op1D(8, 16, 0.0, 1.0, "dirichlet")
    plan = hp.Plan(x, x, 1.0, 1e-10, "mixed")
    U = torch.empty((x.N, x.N), dtype=torch.float64, device="cuda")
    st = hp.hpadi_solve(plan.handle, torch.from_numpy(G0).cuda(), U, raise_on_noconv=False)
    print(f"  status {st.status} rounds {st.rounds} est {st.est_rel_err}", flush=True)
    assert st.status == hp.HPADI_ENOCONV and not np.isfinite(st.est_rel_err)
    plan.close()


def test_unreachable_tolerance_ends_enoconv(hp):
    import torch
    print("failure: tol 1e-20", flush=True)
    o, U0, G0 = _round_trip(8, 16, "neumann", 2.0)
    x = hp.Op1D(8, 16, 0.0, 1.0, "neumann")
    plan = hp.Plan(x, x, 2.0, 1e-20, "mixed")
    U = torch.empty((x.N, x.N), dtype=torch.float64, device="cuda")
    st = hp.hpadi_solve(plan.handle, torch.from_numpy(G0).cuda(), U, raise_on_noconv=False)
    err = oadi.rel_l2_error(U.cpu().numpy(), U0, o, o)
    print(f"  status {st.status} rounds {st.rounds} est {st.est_rel_err:.2e} err {err:.2e}", flush=True)
    assert st.status == hp.HPADI_ENOCONV and st.rounds == 8
    assert err <= 1e-12


@pytest.mark.parametrize("scale", [1e40, 1e-150])
def test_beyond_fp32_range(hp, scale):
    """Entries of G far outside FP32's range (overflow at 1e40, underflow to zero at
    1e-150): the mixed solve must still meet 1e-10 (FP64 rounds only, after the FP32
    round is seen to fail)."""
    import torch
    print(f"failure: |G| scaled by {scale:g}", flush=True)
    o, U0, G0 = _round_trip(8, 16, "dirichlet", 0.0, scale=scale)
    x = hp.Op1D(8, 16, 0.0, 1.0, "dirichlet")
    plan = hp.Plan(x, x, 0.0, 1e-10, "mixed")
    U, st = plan.solve(torch.from_numpy(G0).cuda())
    # the error of the rescaled arrays (squares of 1e-150 underflow in the error norm)
    err = oadi.rel_l2_error(U.cpu().numpy() / scale, U0 / scale, o, o)
    print(f"  status {st.status} rounds {st.rounds} fp32 rounds {st.fp32_rounds} est {st.est_rel_err:.2e} "
          f"err {err:.2e}", flush=True)
    assert st.status == hp.HPADI_OK and err <= 1e-10
    plan.close()


@pytest.mark.parametrize("damping", [0.0, 0.5])
def test_garbage_network_falls_back_to_pcg(hp, damping):
    import torch
    print(f"failure: garbage network weights, damping {damping}", flush=True)
    n = p = 8
    x = hp.Op1D(n, p, 0.0, 1.0, "dirichlet")
    xs, _ = hp.VarCoef.grid(x)
    a = workloads.grf_coefficient(xs, xs, seed=41)
    vc = hp.VarCoef(x, x, torch.from_numpy(a).cuda())
    pre = hp.Plan(x, x, 0.0, 1e-4, "fp64")
    b = pre.load(torch.from_numpy(workloads.legendre_rhs(n, p, n, p, seed=42)).cuda())
    rng = np.random.default_rng(43)
    net = hp.Net(params=(1e6 * rng.standard_normal(hp.lib().hpadi_net_num_params())).astype(np.float32))
    net.set_damping(damping)
    xl, st, _ = vc.solve(b, pre, tol=1e-10, maxit=200, truncation=1, net=net)
    B = obasis.make_basis(n, p, 0.0, 1.0, "dirichlet")
    op = ovc.VarCoefOperator(B, B, a)
    bh = b.cpu().numpy()
    tr = np.linalg.norm(bh - op.apply(xl.cpu().numpy())) / np.linalg.norm(bh)
    print(f"  status {st.status} iters {st.iters} fallback {st.fallback_iters} true res {tr:.2e}", flush=True)
    assert st.status == hp.HPADI_OK and tr <= 1e-10 * (1 + 1e-3)
    if damping > 0.0:
        # z + omega c takes the garbage in: the corrected run is given up
        assert st.fallback_iters > 0
    # damping 0: the energy-optimal combination of z and the correction never does worse
    # than z in the energy norm, so the garbage does not derail the run (tolerance met above)
    net.close()
    pre.close()
    vc.close()
