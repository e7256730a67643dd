"""GPU parity of the learned-correction network (BF16 matrix-core kernels,
FP32 accumulation) against the FP64 oracle (oracle/net.py), and its use inside
the flexible CG of the variable-coefficient problem.

Tolerances: BF16 activations and weights carry 8 significant bits (relative
rounding 2^-9 ~ 2e-3 per value); the forward output is compared with an FP64
forward that rounds the same quantities to BF16 (1e-2 relative, the residual
differences come from FP32 vs FP64 accumulation and GELU near rounding ties) and
with the unrounded FP64 forward (5e-2); gradients with the unrounded FP64
gradient, 5e-2 relative per layer (the BF16 gradient images of the backward pass).
"""
import numpy as np
import pytest

import workloads
from oracle import adi as oadi
from oracle import basis as obasis
from oracle import net as onet
from oracle import varcoef as ovc
from tests.gpu_helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]


@pytest.fixture(scope="module")
def hp():
    from paper_2402_11299_amd import hpadi
    hpadi.lib()
    return hpadi


def flat_params(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for (W, b) in params]).astype(np.float32)


def unflat(vec):
    out, off = [], 0
    for l in range(len(onet.CHANNELS) - 1):
        cin, cout = onet.CHANNELS[l], onet.CHANNELS[l + 1]
        W = vec[off:off + 9 * cin * cout].reshape(3, 3, cin, cout).astype(np.float64)
        off += 9 * cin * cout
        b = vec[off:off + cout].astype(np.float64)
        off += cout
        out.append((W, b))
    return out


def bf16(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params, x):
    """The oracle forward with the BF16 roundings of the GPU kernels: hidden
    activations and the weights of the two 32 -> 32 layers."""
    h = x
    for l, (W, b) in enumerate(params):
        Wl = bf16(W) if l in (1, 2) else W
        pre = onet.conv3x3(h, Wl, b)
        h = bf16(onet.gelu(pre)) if l < len(params) - 1 else pre
    return h[..., 0]


def random_batch(rng, B, H, W):
    x = rng.standard_normal((B, H, W, 3))
    zn = rng.standard_normal((B, H, W))
    t = zn + 0.3 * rng.standard_normal((B, H, W))
    w = rng.uniform(0.2, 1.0, (B, H, W))
    return x, zn, t, w


@pytest.mark.parametrize("B,H,W", [(2, 20, 37), (1, 5, 64), (3, 33, 16)])
def test_forward_matches_oracle(hp, B, H, W):
    import torch
    print(f"net forward {B}x{H}x{W}", flush=True)
    params = onet.init_params(3)
    params[-1] = (params[-1][0] * 10.0, params[-1][1] + 0.1)  # a correction of order one
    rng = np.random.default_rng(1)
    x = rng.standard_normal((B, H, W, 3))
    net = hp.Net(flat_params(params))
    out = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    ref_b = forward_bf16(params, x)
    ref, _ = onet.forward(params, x)
    ref = ref[..., 0]
    e_b = np.linalg.norm(out - ref_b) / np.linalg.norm(ref_b)
    e = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print(f"  rel err vs bf16-rounded oracle {e_b:.2e}, vs fp64 oracle {e:.2e}", flush=True)
    assert e_b <= 1e-2 and e <= 5e-2
    net.close()


def test_gradient_matches_oracle(hp):
    import torch
    params = onet.init_params(5)
    params[-1] = (params[-1][0] * 10.0, params[-1][1])
    rng = np.random.default_rng(2)
    x, zn, t, w = random_batch(rng, 2, 16, 32)
    L_ref, g_ref = onet.grad(params, x, zn, t, w)
    net = hp.Net(flat_params(params))
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    L, g = net.loss_grad(f32(x), f32(zn), f32(t), f32(w))
    print(f"  loss gpu {L:.6f} oracle {L_ref:.6f}", flush=True)
    assert abs(L - L_ref) <= 1e-2 * L_ref
    gl = unflat(g)
    for l in range(len(params)):
        for k, name in ((0, "W"), (1, "b")):
            a, r = gl[l][k], g_ref[l][k]
            err = np.linalg.norm(a - r) / np.linalg.norm(r)
            print(f"  layer {l} {name}: rel err {err:.2e}", flush=True)
            assert err <= 5e-2, (l, name, err)
    net.close()


def test_training_reduces_loss(hp):
    """Fit a fixed smooth map of the inputs (t = zn + 0.5 x_1 - 0.25 x_2 smoothed) from random images."""
    import torch
    rng = np.random.default_rng(3)
    n, c = 64, 32
    x = rng.standard_normal((n, c, c, 3)).astype(np.float32)
    zn = x[..., 0].copy()
    t = zn + 0.5 * x[..., 1] - 0.25 * x[..., 2]
    w = np.ones((n, c, c), dtype=np.float32)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    net = hp.Net(seed=7)
    hist = net.train(f32(x), f32(zn), f32(t), f32(w), batch=8, steps=300, lr=3e-3, seed=1)
    print(f"  loss {hist[0]:.4f} -> {hist[-20:].mean():.4f}", flush=True)
    assert np.isfinite(hist).all()
    assert hist[-20:].mean() < 0.2 * hist[:5].mean()
    net.close()


def _varcoef_problem(hp, cfg, seed):
    import torch
    x = hp.Op1D(cfg.nx, cfg.px, 0.0, 1.0, cfg.bc)
    y = hp.Op1D(cfg.ny, cfg.py, 0.0, 1.0, cfg.bc)
    xs, _ = hp.VarCoef.grid(x)
    ys, _ = hp.VarCoef.grid(y)
    a = workloads.grf_coefficient(xs, ys, seed=seed)
    vc = hp.VarCoef(x, y, torch.from_numpy(a).cuda())
    return x, y, vc, a


def test_learned_fcg_small(hp):
    """Pairs from plain ADI-PCG iterates on a small problem, a short training, and the
    corrected FCG: it must still reach the tolerance on the FP64 true residual (the
    energy-optimal combination never does worse than the plain preconditioned residual
    in the energy norm; a corrected run that fails falls back to plain ADI-PCG)."""
    import torch
    cfg = workloads.Problem("varcoef_n8_p8", 8, 8, 8, 8, 0.0, "dirichlet", 1e-10, 11)
    x, y, vc, a = _varcoef_problem(hp, cfg, seed=11)
    pre = hp.Plan(x, y, 0.0, 1e-4, "fp64")
    b = pre.load(torch.from_numpy(workloads.legendre_rhs(8, 8, 8, 8, seed=12)).cuda())
    xstar, st0, _ = vc.solve(b, pre, tol=1e-13, maxit=300, truncation=0)
    X, ZN, T, W = vc.pairs(pre, b, xstar, crop=32, crops_per_iter=4, cap=400, tol=1e-10, seed=5)
    assert X.shape[0] > 20
    net = hp.Net(seed=3)
    hist = net.train(X.contiguous(), ZN.contiguous(), T.contiguous(), W.contiguous(), batch=8, steps=200, lr=2e-3)
    assert np.isfinite(hist).all()
    xl, st, _ = vc.solve(b, pre, tol=1e-10, maxit=300, truncation=1, net=net)
    xp, stp, _ = vc.solve(b, pre, tol=1e-10, maxit=300, truncation=1)
    Bx = obasis.make_basis(8, 8, 0.0, 1.0, "dirichlet")
    op = ovc.VarCoefOperator(Bx, Bx, a)
    bh = b.cpu().numpy()
    tr = np.linalg.norm(bh - op.apply(xl.cpu().numpy())) / np.linalg.norm(bh)
    print(f"  loss {hist[0]:.3f} -> {hist[-10:].mean():.3f}; learned FCG {st.iters} it "
          f"({st.corrections} corrections), plain {stp.iters} it; true res {tr:.2e}", flush=True)
    assert st.status == hp.HPADI_OK and tr <= 1e-10 * (1 + 1e-3)
    # the correction is combined energy-optimally with the plain preconditioned residual:
    # it may fail to help, but it must not cost more than a few iterations
    assert st.iters <= stp.iters + 3
    # damped addition z + c/2 (scale kept on the device): still reaches the tolerance
    net.set_damping(0.5)
    xd, std, _ = vc.solve(b, pre, tol=1e-10, maxit=300, truncation=1, net=net)
    trd = np.linalg.norm(bh - op.apply(xd.cpu().numpy())) / np.linalg.norm(bh)
    print(f"  damped: {std.iters} it ({std.corrections} corrections); true res {trd:.2e}", flush=True)
    assert std.status == hp.HPADI_OK and trd <= 1e-10 * (1 + 1e-3) and std.corrections == std.iters
    with pytest.raises(hp.HpadiError):
        net.set_damping(-1.0)
    # correction at every second iteration only (iterations 0, 2, 4, ...)
    net.set_period(2)
    xe, ste, _ = vc.solve(b, pre, tol=1e-10, maxit=300, truncation=1, net=net)
    tre = np.linalg.norm(bh - op.apply(xe.cpu().numpy())) / np.linalg.norm(bh)
    assert ste.status == hp.HPADI_OK and tre <= 1e-10 * (1 + 1e-3) and ste.corrections == (ste.iters + 1) // 2
    with pytest.raises(hp.HpadiError):
        net.set_period(0)
    net.close()
    pre.close()
    vc.close()
