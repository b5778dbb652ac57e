"""Training pipeline of the value network (learned leaf evaluator).

Every step runs in the library's kernels: training pairs come from
``dvc_init_states`` (mixed 2/3/4-player mid-game states, half of them after
the mover's draw) and ``dvc_valuenet_labels`` (perspective seat drawn from
Philox, label = that seat's win rate over random playouts); training is
``dvc_valuenet_train_step`` (forward, backward and Adam on the matrix cores).
Python only sequences the calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import torch

from . import (dvc_init_states, dvc_valuenet_epoch_order, dvc_valuenet_init,
               dvc_valuenet_labels, dvc_valuenet_train_step, dvc_valuenet_train_workspace_bytes,
               deal_params)

# mid-game positions of 2-4 players, half of them after the mover's draw
TRAIN_DEAL = dict(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                  revealed_max=8, phase_mix=1)
DATA_TREE_ID = 0xDA7A


@dataclass
class TrainConfig:
    n_data: int = 1 << 23
    playouts: int = 256
    batch: int = 8192
    epochs: int = 20
    lr: float = 1e-3
    data_seed: int = 4
    init_seed: int = 44


def make_data(n: int, playouts: int, seed: int, index_base: int = 0, chunk: int = 1 << 20,
              device="cuda"):
    """(states int32 [n,4], persp uint8 [n], labels float32 [n]) on the device."""
    states = torch.empty((n, 4), dtype=torch.int32, device=device)
    persp = torch.empty(n, dtype=torch.uint8, device=device)
    labels = torch.empty(n, dtype=torch.float32, device=device)
    params = deal_params(**TRAIN_DEAL)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        dvc_init_states(hi - lo, params, seed, index_base=index_base + lo, out=states[lo:hi])
        p, y = dvc_valuenet_labels(states[lo:hi], playouts, seed, tree_id=DATA_TREE_ID,
                                   index_base=index_base + lo)
        persp[lo:hi] = p
        labels[lo:hi] = y
    return states, persp, labels


def epoch_permutation(seed: int, epoch: int, n: int):
    """Batch order of an epoch: row i -> (a*i + b) mod n with a odd, a bijection
    when n is a power of two; a and b are Philox words (dvc_valuenet_epoch_order)."""
    return dvc_valuenet_epoch_order(seed, epoch, n)


def train(cfg: TrainConfig, data=None, net=None, log_every: int = 0, log=None):
    """Train a fresh (or given) network; returns (net, history of (step, loss),
    timing) with timing = {"steps", "wall_s", "gpu_s"}: host seconds of the loop
    and GPU seconds between HIP events recorded around it on the current
    stream.  Every `log_every` steps the batch loss is recorded (and passed to
    `log`)."""
    if data is None:
        data = make_data(cfg.n_data, cfg.playouts, cfg.data_seed)
    states, persp, labels = data
    n = states.shape[0]
    assert n & (n - 1) == 0, "the epoch permutation needs a power-of-two data set"
    if net is None:
        net = dvc_valuenet_init(cfg.init_seed)
    ws = torch.empty(dvc_valuenet_train_workspace_bytes(cfg.batch), dtype=torch.uint8,
                     device=states.device)
    loss = torch.zeros(1, dtype=torch.float32, device=states.device)
    steps_per_epoch = n // cfg.batch
    hist = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    step = 0
    for epoch in range(cfg.epochs):
        a, b = epoch_permutation(cfg.data_seed, epoch, n)
        for k in range(steps_per_epoch):
            step += 1
            want = log_every and (step % log_every == 0 or step == 1)
            dvc_valuenet_train_step(net, states, persp, labels, step=step, lr=cfg.lr,
                                    batch=cfg.batch, perm_a=a, perm_b=b, row_base=k * cfg.batch,
                                    ws=ws, loss_out=loss if want else None)
            if want:
                hist.append((step, float(loss.item())))
                if log is not None:
                    log(f"step {step} loss {hist[-1][1]:.5f}")
    e1.record()
    torch.cuda.synchronize()
    return net, hist, {"steps": step, "wall_s": time.perf_counter() - t0,
                       "gpu_s": e0.elapsed_time(e1) / 1e3}


def main(argv=None):
    """Train on freshly generated pairs and print the time per step (for profiling)."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description="value-network training on generated pairs")
    ap.add_argument("--pairs-log2", type=int, default=23)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8192)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    cfg = TrainConfig(n_data=1 << args.pairs_log2, epochs=args.epochs, batch=args.batch)
    t0 = time.perf_counter()
    data = make_data(cfg.n_data, cfg.playouts, cfg.data_seed)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    _, hist, tm = train(cfg, data=data, log_every=1024, log=lambda m: print(m, flush=True))
    print(json.dumps({"pairs": cfg.n_data, "data_s": t_data, "steps": tm["steps"],
                      "step_ms": tm["gpu_s"] / tm["steps"] * 1e3,
                      "loss_last": hist[-1][1] if hist else None}), flush=True)


if __name__ == "__main__":
    main()
