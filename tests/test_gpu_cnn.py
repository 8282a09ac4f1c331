"""CNN reconstructor kernels (through the C ABI) against the FP64 oracle.

Both sides use the same bf16-rounded weights and inputs.  The GPU stores
hidden activations in bf16 (the operands of the next products), carries
upstream gradients as bf16 hi/lo pairs (~16 bits) and accumulates in FP32.
Two gates per tensor (relative L2):
  * against the exact FP64 oracle: <= 2e-2.  Each stored activation is
    rounded by up to 2^-9; the first-layer weight gradient sums many terms
    of both signs, which amplifies that relative error by ~10x;
  * against the oracle with the same bf16 activation rounding
    (act_round=bf16_round): <= 1e-4 on the small net, where only FP32
    accumulation and the hi/lo gradient split remain (measured ~5e-6); on
    the full net <= 1e-2: a pre-activation accumulated in FP32 (GPU) or FP64
    (oracle) occasionally falls on the other side of a bf16 rounding
    boundary (a quantisation decision the two summation orders cannot take
    identically), and the first-layer weight gradient's cancellation
    amplifies those flips (measured 4.8e-3 there, <= 2e-4 on the outputs).
Adam and input preparation are FP32 elementwise: 1e-5.
"""
import numpy as np
import pytest

from oracle import cnn as ocnn
from tests.gpu_common import torch_cuda, rel_l2, say

pytestmark = pytest.mark.gpu

SMALL = dict(n_sub=9, c1=3, c2=5, c3=4, hidden=37, n_out=11)
FULL = dict(n_sub=40, c1=32, c2=64, c3=64, hidden=2048, n_out=600)


def bf16_round(a):
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _setup(cfg, B, seed):
    from paper_1607_07624_amd.cnn import CNN, he_init
    torch = torch_cuda()
    net = CNN(batch_max=max(B, 4), **cfg)
    p = he_init(net.shapes, seed)
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so their gradients and the ReLU masks are exercised
    off = 0
    for k in ocnn.PARAM_ORDER:
        n = int(np.prod(net.shapes[k]))
        if k.startswith("b") or k.startswith("fb"):
            p[off:off + n] = rng.normal(0, 0.05, n)
        off += n
    net.set_params(torch.from_numpy(p))
    x = rng.normal(0, 1.0, (B, cfg["n_sub"], cfg["n_sub"], 4)).astype(np.float32)
    tgt = rng.normal(0, 1.0, (B, cfg["n_out"])).astype(np.float32)
    # oracle sees the bf16-rounded weights (biases stay FP32 on both sides) and input
    pb = p.copy()
    off = 0
    for k in ocnn.PARAM_ORDER:
        n = int(np.prod(net.shapes[k]))
        if not (k.startswith("b") or k.startswith("fb")):
            pb[off:off + n] = bf16_round(p[off:off + n])
        off += n
    po = ocnn.unflatten_params(pb.astype(np.float64), net.shapes)
    return net, torch, p, po, x, bf16_round(x), tgt


TOL_Q = {"small": 1e-4, "full": 1e-2}


@pytest.mark.parametrize("cfg,B", [(SMALL, 5), (FULL, 16)], ids=["small", "full"])
def test_forward_matches_oracle(cfg, B):
    net, torch, p, po, x, xb, tgt = _setup(cfg, B, 3)
    out = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = ocnn.forward(po, xb.astype(np.float64))
    refq, _ = ocnn.forward(po, xb.astype(np.float64), act_round=ocnn.bf16_round)
    e, eq = rel_l2(out, ref), rel_l2(out, refq)
    say(f"[gpu] cnn forward {cfg['n_sub']}x{cfg['n_out']} B={B}: rel err {e:.3e} (exact), {eq:.3e} (bf16 act)")
    assert e <= 2e-2
    assert eq <= TOL_Q["small" if cfg is SMALL else "full"]


@pytest.mark.parametrize("cfg,B,weighted", [(SMALL, 5, False), (FULL, 16, False), (SMALL, 6, True)],
                         ids=["small", "full", "small-weighted"])
def test_gradients_match_oracle(cfg, B, weighted):
    net, torch, p, po, x, xb, tgt = _setup(cfg, B, 5)
    w = np.random.default_rng(6).uniform(0.2, 3.0, B).astype(np.float32) if weighted else None
    g, loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(),
                            None if w is None else torch.from_numpy(w).cuda())
    g = g.cpu().numpy()
    lo, go, _ = ocnn.loss_and_grads(po, xb.astype(np.float64), tgt.astype(np.float64), weights=w)
    lq, gq, _ = ocnn.loss_and_grads(po, xb.astype(np.float64), tgt.astype(np.float64),
                                    act_round=ocnn.bf16_round, weights=w)
    assert abs(float(loss.cpu()) - lo) <= 2e-2 * lo
    tq = TOL_Q["small" if cfg is SMALL else "full"]
    assert abs(float(loss.cpu()) - lq) <= tq * lq
    off = 0
    for k in ocnn.PARAM_ORDER:
        n = int(np.prod(net.shapes[k]))
        e = rel_l2(g[off:off + n], go[k].ravel())
        eq = rel_l2(g[off:off + n], gq[k].ravel())
        say(f"[gpu] cnn grad {k}: rel err {e:.3e} (exact FP64), {eq:.3e} (bf16 activations)")
        assert e <= 2e-2, k
        assert eq <= tq, k
        off += n
    g2, _ = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(),
                          None if w is None else torch.from_numpy(w).cuda())
    assert np.array_equal(g, g2.cpu().numpy())          # deterministic


def test_adam_step_matches_formula():
    net, torch, p, po, x, xb, tgt = _setup(SMALL, 4, 7)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    g, _ = net.gradients(xd, td)
    g = g.cpu().numpy().astype(np.float64)
    net.train_step(xd, td, 1e-3)
    w1 = net.get_params().cpu().numpy().astype(np.float64)
    ref, m, v = ocnn.adam_step(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    assert np.abs(w1 - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def test_training_reduces_loss_on_device():
    net, torch, p, po, x, xb, tgt = _setup(SMALL, 8, 9)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    loss = torch.empty(1, device="cuda")
    net.train_step(xd, td, 3e-3, loss=loss)
    l0 = float(loss.cpu())
    for _ in range(200):
        net.train_step(xd, td, 3e-3, loss=loss)
    assert float(loss.cpu()) < 0.3 * l0


def test_prepare_matches_oracle():
    from paper_1607_07624_amd.cnn import prepare
    torch = torch_cuda()
    rng = np.random.default_rng(11)
    S, B = 12, 3
    pup = rng.uniform(0.2, 2.0, (B, 4, S, S)).astype(np.float32)
    ref = rng.uniform(0.2, 2.0, (4, S, S)).astype(np.float32)
    valid = np.sort(rng.choice(S * S, 60, replace=False)).astype(np.int32)
    x = prepare(torch.from_numpy(pup).cuda(), torch.from_numpy(ref).cuda(), torch.from_numpy(valid).cuda())
    exp = ocnn.network_input(pup, ref, valid)
    assert np.abs(x.cpu().numpy() - exp).max() <= 1e-5 * np.abs(exp).max()
