"""Value-network search against pure-playout search on one GPU.

For a batch of fresh 2-4 player deals (root draw), the same trees are
searched three times with the library's tree-search kernel:
  * playouts: every leaf gets `ppl` random playouts (two seeds, so that the
    self-agreement of two playout searches bounds what any cheaper
    evaluator can be expected to reach);
  * value mode: every leaf is scored by the trained network, except leaves
    whose value for the root player lies within `band` of 1/2, which get
    `ppl` playouts instead.
Reported: root-move agreement of the value search with the playout search,
the self-agreement ceiling, GPU time per decision of both (HIP events around
one launch each), the share of leaves that fell back to playouts, and the
network's mean squared error against many-playout estimates on held-out
positions next to the noise floor of those estimates.
"""
from __future__ import annotations

import time

import torch

from . import (deal_params, dvc_init_states, dvc_mcts_workspace_bytes, dvc_valuenet_infer,
               dvc_valuenet_labels, mcts_params, mcts_search, mcts_tree_stats)
from .valuenet import TRAIN_DEAL, TrainConfig, make_data, train

ROOT_DEAL = dict(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), fresh=1, root_draw=1)


def timed_search(roots, mp, seed, ws):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    best, _ = mcts_search(roots, mp, seed, workspace=ws, want_children=False)
    e1.record()
    torch.cuda.synchronize()
    return best, e0.elapsed_time(e1) / 1e3


def value_mse(net, n=4096, playouts=4096, seed=99, index_base=1 << 28):
    """MSE of the network against `playouts`-playout win rates on held-out positions."""
    states = dvc_init_states(n, deal_params(**TRAIN_DEAL), seed, index_base=index_base)
    persp, labels = dvc_valuenet_labels(states, playouts, seed, tree_id=0xE7A1,
                                        index_base=index_base)
    v = dvc_valuenet_infer(net, states, persp)
    mse = float(((v - labels) ** 2).mean().item())
    floor = float((labels * (1 - labels)).mean().item() / playouts)
    return mse, floor


def compare(n_trees=1024, iterations=4096, ppl=64, band=0.05, train_cfg: TrainConfig = None,
            net=None, seed=5, log=print):
    t0 = time.perf_counter()
    train_info = {}
    if net is None:
        cfg = train_cfg or TrainConfig()
        data = make_data(cfg.n_data, cfg.playouts, cfg.data_seed)
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        net, hist, t_train = train(cfg, data=data, log_every=1024)
        train_info = {"pairs": cfg.n_data, "label_playouts": cfg.playouts, "batch": cfg.batch,
                      "epochs": cfg.epochs, "data_s": t_data, "train_s": t_train,
                      "loss_first": hist[0][1] if hist else None,
                      "loss_last": hist[-1][1] if hist else None}
        log(f"trained: {train_info}")
        del data
    mse, floor = value_mse(net)
    roots = dvc_init_states(n_trees, deal_params(**ROOT_DEAL), seed)
    mp_roll = mcts_params(iterations=iterations, playouts_per_leaf=ppl, max_depth=4)
    mp_val = mcts_params(iterations=iterations, playouts_per_leaf=1, max_depth=4, leaf_eval=1,
                         fallback_band=band, fallback_playouts=ppl, valuenet=net)
    ws = torch.empty(max(dvc_mcts_workspace_bytes(n_trees, mp_roll),
                         dvc_mcts_workspace_bytes(n_trees, mp_val)), dtype=torch.uint8,
                     device=roots.device)
    best_roll, t_roll = timed_search(roots, mp_roll, seed, ws)
    best_roll2, _ = timed_search(roots, mp_roll, seed + 1000, ws)
    best_val, t_val = timed_search(roots, mp_val, seed, ws)
    stats = mcts_tree_stats(ws, n_trees, mp_val)
    net_leaves = int(stats["net_leaves"].sum())
    played = int(stats["played_leaves"].sum())
    out = {
        "trees": n_trees, "iterations": iterations, "playouts_per_leaf": ppl, "band": band,
        "root_move_agreement": float((best_val == best_roll).float().mean().item()),
        "rollout_self_agreement": float((best_roll2 == best_roll).float().mean().item()),
        "gpu_s_per_decision_rollout": t_roll / n_trees,
        "gpu_s_per_decision_value": t_val / n_trees,
        "speedup": t_roll / t_val,
        "fallback_rate": played / max(1, played + net_leaves),
        "value_mse_vs_4096_playouts": mse, "mse_noise_floor": floor,
        "training": train_info,
    }
    return out, net
