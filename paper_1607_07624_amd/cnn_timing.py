"""Throughput of the learned reconstructor's kernels on seeded random data
(no sensor in the loop): one training step (forward, backward, Adam) at a
training batch, and the forward pass at loop batch sizes.

Rates are frames per second and the algorithmic bf16 flop rate: 2 M N K per
product of the network (forward: the three convolutions as im2col products
and the two fully connected layers; a training step adds the weight- and
data-gradient products of every layer except the first layer's data
gradient), counted once, i.e. without the repeated products of the split
(hi/lo) operands.  Run as

    python -m paper_1607_07624_amd.cnn_timing [--batch 256] [--steps 50]

which prints one JSON line.
"""
from __future__ import annotations

import argparse
import json


def layer_products(n_sub=40, c1=32, c2=64, c3=64, hidden=2048, n_out=600):
    """(M per frame, N, K) of the five forward products (M: output rows per frame)."""
    s1 = (n_sub + 1) // 2
    s2 = (s1 + 1) // 2
    s3 = (s2 + 1) // 2
    return [(s1 * s1, c1, 4 * 9), (s2 * s2, c2, c1 * 9), (s3 * s3, c3, c2 * 9),
            (1, hidden, s3 * s3 * c3), (1, n_out, hidden)]


def flops_per_frame(train: bool, **shape) -> float:
    fwd = [2.0 * m * n * k for (m, n, k) in layer_products(**shape)]
    if not train:
        return sum(fwd)
    return sum(fwd) + 2.0 * sum(fwd) - fwd[0]     # weight gradients of all layers, data gradients but the first's


def measure(batch: int = 256, steps: int = 50, fwd_batches=(1, 16), fwd_calls: int = 400, seed: int = 0) -> dict:
    import numpy as np
    import torch
    from .cnn import CNN, he_init

    dev = torch.device("cuda", torch.cuda.current_device())
    bmax = max(batch, *fwd_batches)
    net = CNN(batch_max=bmax)
    net.set_params(he_init(net.shapes, seed))
    rng = np.random.default_rng(seed + 1)
    x = torch.from_numpy(rng.normal(0, 1e-2, (bmax, 40, 40, 4)).astype(np.float32)).to(dev)
    y = torch.from_numpy(rng.normal(0, 1.0, (bmax, 600)).astype(np.float32)).to(dev)
    loss = torch.empty(1, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    xb, yb = x[:batch].contiguous(), y[:batch].contiguous()
    for _ in range(5):
        net.train_step(xb, yb, 1e-4, loss=loss)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        net.train_step(xb, yb, 1e-4, loss=loss)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    fl = flops_per_frame(True) * batch
    out["train"] = {"batch": batch, "ms_per_step": round(ms, 4), "frames_per_s": round(batch / (ms * 1e-3), 1),
                    "tflops": round(fl / (ms * 1e-3) / 1e12, 2), "flop_per_step": fl}
    for B in fwd_batches:
        xf = x[:B].contiguous()
        o = torch.empty((B, 600), device=dev)
        for _ in range(10):
            net.forward(xf, o)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(fwd_calls):
            net.forward(xf, o)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / fwd_calls
        fl = flops_per_frame(False) * B
        out[f"forward_b{B}"] = {"us_per_call": round(ms * 1e3, 2), "frames_per_s": round(B / (ms * 1e-3), 1),
                                "tflops": round(fl / (ms * 1e-3) / 1e12, 3)}
    net.close()
    out["peak_bf16_tflops"] = 2500.0
    out["flop_convention"] = "2 M N K per product of the network, each counted once"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--fwd-calls", type=int, default=400)
    args = ap.parse_args()
    print(json.dumps(measure(args.batch, args.steps, fwd_calls=args.fwd_calls)), flush=True)


if __name__ == "__main__":
    main()
