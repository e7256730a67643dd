"""The allocation-free load (hpadi_load_noalloc) against hpadi_load, through the C ABI.

Both compute G = T_x F T_y^T (Sec. 3.2) with the same per-entry gathers, so the
results must agree bit for bit; the allocation-free one works in column blocks
through the library's fixed scratch array.  Two calls in a row share that array:
the first one large enough to need several column blocks with a ragged last block,
the second one smaller.
"""
import ctypes

import numpy as np
import pytest

from gpu_helpers import gpu_available

pytestmark = pytest.mark.gpu


def _load_both(hp, torch, nx, px, ny, py, bc, seed):
    import workloads
    x = hp.Op1D(nx, px, 0.0, 1.0, bc)
    y = hp.Op1D(ny, py, 0.0, 1.0, bc)
    plan = hp.Plan(x, y, 1.0, 1e-6, "fp64")
    F = torch.from_numpy(workloads.legendre_rhs(nx, px, ny, py, seed)).cuda()
    G_ref = torch.full((x.N, y.N), np.nan, dtype=torch.float64, device="cuda")
    G_na = torch.full((x.N, y.N), np.nan, dtype=torch.float64, device="cuda")
    L = hp.lib()
    rc = L.hpadi_load(plan.handle, ctypes.c_void_p(F.data_ptr()), F.stride(0), ctypes.c_void_p(G_ref.data_ptr()),
                      G_ref.stride(0))
    assert rc == 0, hp.lib().hpadi_strerror(rc)
    rc = L.hpadi_load_noalloc(plan.handle, ctypes.c_void_p(F.data_ptr()), F.stride(0),
                              ctypes.c_void_p(G_na.data_ptr()), G_na.stride(0))
    assert rc == 0, hp.lib().hpadi_strerror(rc)
    torch.cuda.synchronize()
    out = G_ref.cpu().numpy(), G_na.cpu().numpy(), x, y, F.cpu().numpy()
    plan.close()
    return out


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_noalloc_load_matches_load_two_calls():
    import torch
    from oracle import adi as oadi
    from oracle import basis as obasis
    from paper_2402_11299_amd import hpadi as hp
    hp.lib()
    # 1) N_x = 4095 (Nleg_x = 4160, blocks of 448 columns), N_y = 1023: three blocks, the
    #    last one 127 columns wide
    print("noalloc load: n=p=64 x n=16,p=64 dirichlet", flush=True)
    Gr, Gn, _, _, _ = _load_both(hp, torch, 64, 64, 16, 64, "dirichlet", 11)
    assert np.isfinite(Gr).all()
    assert np.array_equal(Gr, Gn)
    # 2) a smaller problem on the same scratch (one block), checked against the oracle too
    print("noalloc load: n=4,p=8 x n=8,p=16 neumann", flush=True)
    Gr, Gn, x, y, F = _load_both(hp, torch, 4, 8, 8, 16, "neumann", 12)
    assert np.array_equal(Gr, Gn)
    ox = obasis.assemble(obasis.make_basis(4, 8, 0.0, 1.0, "neumann"))
    oy = obasis.assemble(obasis.make_basis(8, 16, 0.0, 1.0, "neumann"))
    Go = oadi.load(ox, oy, F)
    assert np.abs(Gn - Go).max() <= 1e-14 * max(1.0, np.abs(Go).max())
