"""CNN reconstructor kernels (through the C ABI) against the FP64 oracle.

Both sides use the same bf16-rounded weights and inputs; the oracle is
exact FP64 from there on.  The GPU carries every hidden activation and every
upstream gradient as a bf16 pair hi + lo (the value to ~2^-17 relative),
multiplies on the bf16 matrix cores and accumulates in FP32.  Gates per
tensor, relative L2 and per element (max |error| / max |reference|):
  * forward outputs: <= 1e-4 (pair rounding ~7.6e-6 per operand and FP32
    accumulation over up to 2048 terms, ~1e-5 expected);
  * parameter gradients: <= 1e-4 (the same per-operand errors, amplified by
    the cancellation in the sums over the batch and the positions: a bias
    or first-layer weight gradient is a small sum of many terms of both
    signs; measured <= 1.1e-5);
  * the loss: <= 1e-4 relative.
The forward runs at 1, 3, 8, 16 and 21 frames, which crosses every
batch-size form of the matrix-vector kernel (1, 4, 8, 16 rows), its limit
on the rows of the convolutions (at most 512, reached at 16 frames by the
last convolution only) and the tiled MFMA product at every layer (21
frames), also with alpha and beta (the loop's accumulate form).  Forward
and gradients also run at 256 frames, the timed training batch: the
products' split-K forms, the implicit patches of the second and third
convolutions and the two-stream backward as the training step uses them.
The full network's convolutions run as one block per frame; a network
with 64 first-layer channels (outside that kernel) checks the tiled
forward products.
Adam and input preparation are FP32 elementwise: 1e-5.
"""
import numpy as np
import pytest

from oracle import cnn as ocnn
from tests.gpu_common import torch_cuda, rel_l2, rel_max, say

pytestmark = pytest.mark.gpu

SMALL = dict(n_sub=9, c1=3, c2=5, c3=4, hidden=37, n_out=11)
FULL = dict(n_sub=40, c1=32, c2=64, c3=64, hidden=2048, n_out=600)
# 64 first-layer channels: outside the one-block-per-frame convolution kernel,
# so the forward pass takes the tiled products (implicit patches of the second
# and third convolutions from 16 frames on)
WIDE = dict(n_sub=40, c1=64, c2=64, c3=64, hidden=256, n_out=100)
FWD_TOL = 1e-4
GRAD_TOL = 1e-4
# A ReLU input within ~1e-5 of its layer's spread from zero can land on
# either side between FP64 and the kernels' FP32 sums (operands good to
# ~2^-17, sums of up to 2048 terms), and a flipped mask changes every
# gradient below it by that element's full upstream value: the 256-frame
# inputs of the gradient test had one conv3 input at 5e-7 of its spread
# and gave 1e-4 errors in the four convolution tensors (1e-6 in the fully
# connected ones, above the flip).  Large batches are therefore drawn with
# every ReLU input at least 1e-4 spreads away from zero.
RELU_MARGIN = 1e-4


def bf16_round(a):
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _relu_inputs(po, xb):
    """The FP64 inputs of the four ReLUs, each [B, -1]."""
    B = xb.shape[0]
    z1 = ocnn.conv_forward(xb, po["w1"], po["b1"])
    z2 = ocnn.conv_forward(np.maximum(z1, 0.0), po["w2"], po["b2"])
    z3 = ocnn.conv_forward(np.maximum(z2, 0.0), po["w3"], po["b3"])
    zh = np.maximum(z3, 0.0).reshape(B, -1) @ po["fw1"].T + po["fb1"]
    return [z.reshape(B, -1) for z in (z1, z2, z3, zh)]


def _setup(cfg, B, seed, relu_margin=None):
    """Network and inputs; with relu_margin, every frame whose ReLU inputs
    (FP64, bf16-rounded weights and input) come within relu_margin times
    their layer's spread of zero is drawn again (seeded), so that no ReLU
    decision lies inside the band where FP64 and the kernels' FP32 sums can
    take it differently."""
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
    if relu_margin is not None:
        sd = [z.std() for z in _relu_inputs(po, bf16_round(x).astype(np.float64))]
        redraw = np.random.default_rng(seed + 2)
        bad = np.arange(B)
        for _ in range(200):
            zs = _relu_inputs(po, bf16_round(x[bad]).astype(np.float64))
            near = np.zeros(len(bad), bool)
            for z, s in zip(zs, sd):
                near |= (np.abs(z) < relu_margin * s).any(axis=1)
            bad = bad[near]
            if len(bad) == 0:
                break
            x[bad] = redraw.normal(0, 1.0, (len(bad),) + x.shape[1:]).astype(np.float32)
        assert len(bad) == 0, "could not draw frames clear of the ReLU band"
    return net, torch, p, po, x, bf16_round(x), tgt


FWD_CASES = [(SMALL, 5), (FULL, 1), (FULL, 3), (FULL, 8), (FULL, 16), (FULL, 21), (FULL, 256), (WIDE, 2), (WIDE, 32)]


@pytest.mark.parametrize("cfg,B", FWD_CASES, ids=["small-5", "full-1", "full-3", "full-8", "full-16", "full-21",
                                                  "full-256", "wide-2", "wide-32"])
def test_forward_matches_oracle(cfg, B):
    net, torch, p, po, x, xb, tgt = _setup(cfg, B, 3)
    out = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = ocnn.forward(po, xb.astype(np.float64))
    e, em = rel_l2(out, ref), rel_max(out, ref)
    say(f"[gpu] cnn forward {cfg['n_sub']}x{cfg['n_out']} B={B}: rel err {e:.3e} (max {em:.3e})")
    assert e <= FWD_TOL and em <= FWD_TOL
    # accumulate form: out = alpha net(x) + beta out
    acc0 = np.random.default_rng(B).normal(0, 1.0, out.shape).astype(np.float32)
    acc = torch.from_numpy(acc0).cuda()
    net.forward_acc(torch.from_numpy(x).cuda(), acc, 0.4, 0.75)
    refa = 0.4 * ref + 0.75 * acc0.astype(np.float64)
    ea = rel_max(acc.cpu().numpy(), refa)
    say(f"[gpu]   accumulate form (alpha 0.4, beta 0.75): max err {ea:.3e}")
    assert ea <= FWD_TOL
    net.close()


@pytest.mark.parametrize("cfg,B,weighted", [(SMALL, 5, False), (FULL, 16, False), (SMALL, 6, True),
                                            (FULL, 3, True), (FULL, 256, False), (FULL, 256, True), (WIDE, 32, False)],
                         ids=["small", "full", "small-weighted", "full-3-weighted", "full-256", "full-256-weighted",
                              "wide-32"])
def test_gradients_match_oracle(cfg, B, weighted):
    many = B >= 64 or cfg is WIDE                       # enough ReLU inputs for one near zero
    net, torch, p, po, x, xb, tgt = _setup(cfg, B, 5, relu_margin=RELU_MARGIN if many else None)
    w = np.random.default_rng(6).uniform(0.2, 3.0, B).astype(np.float32) if weighted else None
    g, loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(),
                            None if w is None else torch.from_numpy(w).cuda())
    g = g.cpu().numpy()
    lo, go, _ = ocnn.loss_and_grads(po, xb.astype(np.float64), tgt.astype(np.float64), weights=w)
    say(f"[gpu] cnn loss B={B}: {float(loss.cpu()):.6e} (oracle {lo:.6e})")
    assert abs(float(loss.cpu()) - lo) <= FWD_TOL * lo
    off = 0
    for k in ocnn.PARAM_ORDER:
        n = int(np.prod(net.shapes[k]))
        e, em = rel_l2(g[off:off + n], go[k].ravel()), rel_max(g[off:off + n], go[k].ravel())
        say(f"[gpu] cnn grad {k}: rel err {e:.3e} (max {em:.3e}) against exact FP64")
        assert e <= GRAD_TOL and em <= GRAD_TOL, k
        off += n
    g2, _ = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(),
                          None if w is None else torch.from_numpy(w).cuda())
    assert np.array_equal(g, g2.cpu().numpy())          # deterministic
    net.close()


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


def test_checkpoint_round_trip(tmp_path):
    """Training resumed from a checkpoint (parameters, Adam moments, step)
    follows the uninterrupted run bit for bit; without the optimiser state
    (parameters only) it does not."""
    from paper_1607_07624_amd.cnn import CNN
    net, torch, p, po, x, xb, tgt = _setup(SMALL, 8, 13)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    for _ in range(5):
        net.train_step(xd, td, 3e-3)
    path = str(tmp_path / "cnn_ckpt.npz")
    net.save(path)
    w_ckpt = net.get_params().cpu().numpy()
    for _ in range(7):
        net.train_step(xd, td, 3e-3)
    a = net.get_params().cpu().numpy()
    net2 = CNN(batch_max=8, **SMALL)
    net2.load(path)
    assert np.array_equal(net2.get_params().cpu().numpy(), w_ckpt)
    for _ in range(7):
        net2.train_step(xd, td, 3e-3)
    b = net2.get_params().cpu().numpy()
    say(f"[gpu] cnn checkpoint: resumed run equal {np.array_equal(a, b)}")
    assert np.array_equal(a, b)
    net3 = CNN(batch_max=8, **SMALL)
    net3.set_params(w_ckpt)                                  # parameters only: fresh Adam state
    for _ in range(7):
        net3.train_step(xd, td, 3e-3)
    assert not np.array_equal(net3.get_params().cpu().numpy(), a)
    bad = CNN(batch_max=8, **dict(SMALL, hidden=38))
    with pytest.raises(ValueError):
        bad.load(path)
    for n_ in (net, net2, net3, bad):
        n_.close()


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


def test_gradients_under_graph_capture():
    """pwfs_cnn_gradients captured in a HIP graph (its backward forks a second
    stream from the captured one and joins it back): replays with new inputs
    copied into the captured buffers give the eager call's loss and gradients
    bit for bit, with eager work between the replays."""
    net, torch, p, po, x, xb, tgt = _setup(FULL, 16, 21)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    g_buf = torch.empty(net.n_params, device="cuda")
    l_buf = torch.empty(1, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        net.gradients(xd, td, grads=g_buf, loss=l_buf)              # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        net.gradients(xd, td, grads=g_buf, loss=l_buf)
    rng = np.random.default_rng(22)
    for rep in range(3):
        x2 = torch.from_numpy(rng.normal(0, 1.0, x.shape).astype(np.float32)).cuda()
        t2 = torch.from_numpy(rng.normal(0, 1.0, tgt.shape).astype(np.float32)).cuda()
        ge, le = net.gradients(x2, t2)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()              # eager work between replays
        xd.copy_(x2)
        td.copy_(t2)
        graph.replay()
        torch.cuda.synchronize()
        same = torch.equal(g_buf, ge) and torch.equal(l_buf.reshape(()), le.reshape(()))
        say(f"[gpu] cnn gradients graph replay {rep}: equal to eager {same} ({float(junk):.1f})")
        assert same
    net.close()
