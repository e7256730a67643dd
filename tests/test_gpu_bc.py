"""GPU parity of the general boundary conditions (Sec. 3.3: Dirichlet, Neumann or Robin per
end) and of Alg. 2 with general axis operators A = kx K_x + sx M_x, B = -(ky K_y + sy M_y),
D = M_x, C = M_y, against the oracle.

* FP64 ADI element by element against the oracle's Alg. 2 with the same interval and shifts
  (tolerance from the mass matrices' conditioning, as for the plain problem), and against the
  dense Kronecker solve within the ADI tolerance;
* the operator application (hpadi_apply) against the oracle's;
* mixed precision against the exact solution (round trip), including n = p = 64 with Robin
  ends and anisotropic coefficients (the uniform-mesh kernels, 65 hats).
"""
import numpy as np
import pytest

import workloads
from oracle import adi as oadi
from oracle import basis as obasis
from oracle import spectrum as ospec
from tests.gpu_helpers import ROUNDING_ALLOWANCE, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

# (n_x, p_x, bc_x, alpha_x, n_y, p_y, bc_y, alpha_y, coef or None (then omega^2 = w2), w2)
CASES = [
    (5, 9, ("dirichlet", "neumann"), (0, 0), 4, 12, ("neumann", "dirichlet"), (0, 0), None, 0.0),
    (6, 10, ("robin", "robin"), (2.0, 0.5), 5, 8, "dirichlet", (0, 0), None, 0.0),
    (4, 16, "dirichlet", (0, 0), 6, 9, "dirichlet", (0, 0), (3.0, 0.0, 0.25, 5.0), 0.0),
    (8, 8, ("robin", "neumann"), (1.0, 0), 4, 16, "neumann", (0, 0), (1.0, 2.0, 0.5, 0.1), 0.0),
    (4, 12, ("neumann", "robin"), (0, 4.0), 4, 12, ("neumann", "robin"), (0, 4.0), None, 1.0),
]


@pytest.fixture(scope="module")
def hp():
    from paper_2402_11299_amd import hpadi
    hpadi.lib()
    return hpadi


def setup(hp, case):
    nx, px, bcx, ax, ny, py, bcy, ay, coef, w2 = case
    x = hp.Op1D(nx, px, 0.0, 1.0, bcx, alpha=ax)
    y = hp.Op1D(ny, py, -1.0, 1.0, bcy, alpha=ay)
    ox = obasis.assemble(obasis.make_basis(nx, px, 0.0, 1.0, bcx, alpha=ax))
    oy = obasis.assemble(obasis.make_basis(ny, py, -1.0, 1.0, bcy, alpha=ay))
    return x, y, ox, oy, coef, w2


def oracle_interval(ox, oy, coef, w2):
    kx, sx, ky, sy = coef if coef is not None else (1.0, w2 / 2, 1.0, w2 / 2)
    ax, bx = ospec.interval(ox, w2, kx, sx)
    ay, by = ospec.interval(oy, w2, ky, sy)
    return (ax, bx * 1.01, -by * 1.01, -ay)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[2]}-{c[6]}-{c[8]}".replace(" ", ""))
def test_fp64_adi_general_matches_oracle(hp, case):
    import torch
    print(f"general ADI {case}", flush=True)
    x, y, ox, oy, coef, w2 = setup(hp, case)
    tol = 1e-12
    iv = oracle_interval(ox, oy, coef, w2)
    plan = hp.Plan(x, y, w2, tol, "fp64", interval=iv, coef=coef)
    oplan = oadi.ADIPlan(ox, oy, w2, tol, interval=iv, coef=coef)
    assert plan.J == oplan.J
    assert np.allclose(plan.p, oplan.p, rtol=1e-12) and np.allclose(plan.q, oplan.q, rtol=1e-12)
    F = workloads.legendre_rhs(x.n, x.p, y.n, y.p, seed=5)
    G = oadi.load(ox, oy, F)
    U, st = plan.solve(torch.from_numpy(G).cuda())
    U = U.cpu().numpy()
    Uo = oplan.solve(G)
    ediff = np.abs(U - Uo).max() / np.abs(Uo).max()
    cond = max(np.linalg.cond(ox.M.toarray()), np.linalg.cond(oy.M.toarray()))
    print(f"  J={plan.J} elementwise max rel diff {ediff:.2e} (cond M {cond:.1e})", flush=True)
    assert ediff <= max(1e-11, 4 * 2.2e-16 * cond)
    Uref = oadi.solve_dense(ox, oy, w2, G, coef=coef)
    assert oadi.rel_l2_error(U, Uref, ox, oy) <= tol * (1 + 1e-3) + 1e-13
    # the operator itself
    Y = plan.apply(torch.from_numpy(Uref).cuda()).cpu().numpy()
    Yref = oadi.apply_operator(ox, oy, w2, Uref, coef=coef)
    assert np.abs(Y - Yref).max() <= 1e-12 * np.abs(Yref).max()
    plan.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[2]}-{c[6]}-{c[8]}".replace(" ", ""))
def test_mixed_general_round_trip(hp, case):
    """Interval computed by the library (continuous lower end for the ends), mixed precision,
    against the exact solution of a round trip G0 = A U0 (oracle)."""
    import torch
    print(f"general mixed {case}", flush=True)
    x, y, ox, oy, coef, w2 = setup(hp, case)
    U0 = np.random.default_rng(9).standard_normal((ox.basis.N, oy.basis.N))
    G0 = oadi.apply_operator(ox, oy, w2, U0, coef=coef)
    plan = hp.Plan(x, y, w2, 1e-10, "mixed", coef=coef)
    U, st = plan.solve(torch.from_numpy(G0).cuda())
    err = oadi.rel_l2_error(U.cpu().numpy(), U0, ox, oy)
    print(f"  rounds={st.rounds} est={st.est_rel_err:.2e} err={err:.2e}", flush=True)
    assert st.status == hp.HPADI_OK and err <= 1e-10
    assert err <= st.est_rel_err + ROUNDING_ALLOWANCE
    plan.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_robin_anisotropic(hp, prec):
    """n = p = 64 on both axes with Robin conditions at both x ends (65 hats) and Dirichlet in
    y, anisotropic coefficients: the uniform-mesh kernels with kappa != 1 and the Robin term."""
    import torch
    print(f"full-size Robin/anisotropic {prec}", flush=True)
    n = p = 64
    coef = (2.0, 0.0, 0.5, 3.0)
    x = hp.Op1D(n, p, 0.0, 1.0, ("robin", "robin"), alpha=(1.5, 0.25))
    y = hp.Op1D(n, p, 0.0, 1.0, "dirichlet")
    ox = obasis.assemble(obasis.make_basis(n, p, 0.0, 1.0, ("robin", "robin"), alpha=(1.5, 0.25)))
    oy = obasis.assemble(obasis.make_basis(n, p, 0.0, 1.0, "dirichlet"))
    kx = workloads.q_degrees(n, p, "neumann")
    ky = workloads.q_degrees(n, p, "dirichlet")
    U0 = np.random.default_rng(21).standard_normal((kx.size, ky.size)) * (1.0 + kx)[:, None] ** -2 * \
        (1.0 + ky)[None, :] ** -2
    G0 = oadi.apply_operator(ox, oy, 0.0, U0, coef=coef)
    plan = hp.Plan(x, y, 0.0, 1e-10, prec, coef=coef)
    U, st = plan.solve(torch.from_numpy(G0).cuda())
    err = oadi.rel_l2_error(U.cpu().numpy(), U0, ox, oy)
    print(f"  rounds={st.rounds} J={st.J} est={st.est_rel_err:.2e} err={err:.2e}", flush=True)
    assert st.status == hp.HPADI_OK and err <= 1e-10
    plan.close()
