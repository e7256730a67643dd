"""GPU parity of the batched solve (one graph replaying independent mixed
solves) against the same instances solved one by one, and against the FP64
oracle for small instances.

Every instance must meet the requested relative error 1e-10 in the norm of the
ADI lemma; two correct answers differ by at most twice that.  A second replay
of the graph must reproduce the first bit for bit (no atomics touch U).
"""
import numpy as np
import pytest

import workloads
from oracle import adi as oadi
from oracle import basis as obasis
from tests.gpu_helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

# (nx, px, ny, py, omega2, bc): the general path (n = 4), the longest chains
# (p = 128), unequal axes, both boundary conditions
INSTANCES = [(4, 8, 4, 16, 1.0, "neumann"), (4, 128, 8, 8, 0.5, "dirichlet"), (8, 128, 4, 32, 10.0, "neumann"),
             (16, 16, 32, 8, 0.01, "dirichlet"), (32, 32, 8, 64, 100.0, "neumann"), (8, 64, 8, 64, 0.0, "dirichlet"),
             (64, 8, 16, 32, 3.0, "dirichlet"), (4, 32, 64, 16, 1e3, "neumann")]


@pytest.fixture(scope="module")
def hp():
    from paper_2402_11299_amd import hpadi
    hpadi.lib()
    return hpadi


def test_batch_matches_single_solves(hp):
    import torch
    probs, Gs, Us, singles, oracles = [], [], [], [], []
    for k, (nx, px, ny, py, w2, bc) in enumerate(INSTANCES):
        print(f"batch instance {k}: {nx},{px},{ny},{py},{w2},{bc}", flush=True)
        x, y = hp.Op1D(nx, px, 0.0, 1.0, bc), hp.Op1D(ny, py, 0.0, 1.0, bc)
        G = torch.from_numpy(workloads.decaying_coefficients(nx, px, ny, py, bc, seed=50 + k)).cuda()
        pl = hp.Plan(x, y, w2, 1e-10, "mixed")
        Us1, _ = pl.solve(G)
        singles.append(Us1.cpu().numpy())
        pl.close()
        probs.append((x, y, w2))
        Gs.append(G)
        Us.append(torch.empty_like(G))
        oracles.append((obasis.assemble(obasis.make_basis(nx, px, 0.0, 1.0, bc)),
                        obasis.assemble(obasis.make_basis(ny, py, 0.0, 1.0, bc)), G.cpu().numpy(), w2))
    batch = hp.Batch(probs, 1e-10, Gs, Us, autotune=True)
    st, extra = batch.solve()
    first = [u.cpu().numpy().copy() for u in Us]
    print(f"  extra FP64 rounds: {extra}; tuned lines per block: {[batch.info(i)[0] for i in range(len(probs))]}",
          flush=True)
    for k, (ox, oy, G, w2) in enumerate(oracles):
        assert st[k].status == hp.HPADI_OK and st[k].est_rel_err <= 1e-10
        d = oadi.rel_l2_error(first[k], singles[k], ox, oy)
        print(f"  instance {k}: |U_batch - U_single| = {d:.2e}, est {st[k].est_rel_err:.2e}", flush=True)
        assert d <= 2e-10
        if ox.basis.N * oy.basis.N <= 40000:
            Uref = oadi.solve_fdm(ox, oy, w2, G, refine=2)
            e = oadi.rel_l2_error(first[k], Uref, ox, oy)
            print(f"    vs oracle: {e:.2e}", flush=True)
            assert e <= 1e-10
    st2, _ = batch.solve()
    for k in range(len(probs)):
        assert np.array_equal(Us[k].cpu().numpy(), first[k])
    batch.close()
