"""Search experiments on one GPU.

compare(): value-network search against pure-playout search.  For a batch of fresh 2-4 player deals (root draw), the same trees are
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

root_parallel_vs_single(): K independent trees per root amalgamated at the
root (the paper's decomposition) against one tree with K times the
iterations.
"""
from __future__ import annotations

import time

import torch

from . import (deal_params, dvc_init_states, dvc_mcts_workspace_bytes, dvc_valuenet_infer,
               dvc_valuenet_labels, mcts_params, mcts_search, mcts_search_root_parallel,
               mcts_tree_stats)
from .valuenet import TRAIN_DEAL, TrainConfig, make_data, train

# forward 2*(160*256 + 256*256 + 256), backward: data gradient through layer 2
# (2*256*256) and the weight gradients of layers 2 and 1 (2*256*256, 2*256*160)
FLOP_PER_ROW_TRAIN = 2 * (160 * 256 + 256 * 256 + 256) + 2 * 256 * 256 * 2 + 2 * 256 * 160

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
        log(f"training pairs ready: {cfg.n_data} in {t_data:.2f} s")
        net, hist, t_train = train(cfg, data=data, log_every=1024, log=log)
        steps = cfg.epochs * (cfg.n_data // cfg.batch)
        train_info = {"pairs": cfg.n_data, "label_playouts": cfg.playouts, "batch": cfg.batch,
                      "epochs": cfg.epochs, "data_s": t_data, "train_s": t_train,
                      "steps": steps, "step_ms": t_train / steps * 1e3,
                      "train_tflops": steps * cfg.batch * FLOP_PER_ROW_TRAIN / t_train / 1e12,
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


def _timed(fn):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1) / 1e3


def root_parallel_vs_single(n_roots=256, trees_per_root=32, iterations=1024, ppl=32, seed=6):
    """The paper's decomposition (independent trees amalgamated at the root,
    Sec. III-B) against one tree with the same total number of iterations.
    Reported: decisions/s of both, and how often their decisions agree next to
    how often two root-parallel searches with different seeds agree."""
    roots = dvc_init_states(n_roots, deal_params(**ROOT_DEAL), seed)
    K = trees_per_root
    mp = mcts_params(iterations=iterations, playouts_per_leaf=ppl, max_depth=4)
    mp_one = mcts_params(iterations=iterations * K, playouts_per_leaf=ppl, max_depth=4)
    ws = torch.empty(max(dvc_mcts_workspace_bytes(n_roots * K, mp),
                         dvc_mcts_workspace_bytes(n_roots, mp_one)), dtype=torch.uint8,
                     device=roots.device)
    mcts_search_root_parallel(roots, K, mp, seed, workspace=ws, want_children=False)
    (b_rp, _), t_rp = _timed(lambda: mcts_search_root_parallel(roots, K, mp, seed, workspace=ws,
                                                               want_children=False))
    (b_rp2, _), _ = _timed(lambda: mcts_search_root_parallel(roots, K, mp, seed + 1000,
                                                             workspace=ws, want_children=False))
    (b_one, _), t_one = _timed(lambda: mcts_search(roots, mp_one, seed, workspace=ws,
                                                   want_children=False))
    return {
        "roots": n_roots, "trees_per_root": K, "iterations_per_tree": iterations,
        "playouts_per_leaf": ppl,
        "root_parallel_decisions_per_s": n_roots / t_rp,
        "single_tree_decisions_per_s": n_roots / t_one,
        "speedup": t_one / t_rp,
        "agreement_root_parallel_vs_single": float((b_rp == b_one).float().mean().item()),
        "agreement_root_parallel_two_seeds": float((b_rp == b_rp2).float().mean().item()),
    }


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--what", choices=["value", "root-parallel", "all"], default="all")
    ap.add_argument("--trees", type=int, default=1024)
    ap.add_argument("--iterations", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--pairs-log2", type=int, default=23)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.what in ("value", "all"):
        cfg = TrainConfig(n_data=1 << args.pairs_log2, epochs=args.epochs)
        out, _ = compare(n_trees=args.trees, iterations=args.iterations, train_cfg=cfg,
                         log=lambda m: print(m, flush=True))
        print(json.dumps({"value_vs_rollout": out}), flush=True)
    if args.what in ("root-parallel", "all"):
        print(json.dumps({"root_parallel_vs_single": root_parallel_vs_single()}), flush=True)


if __name__ == "__main__":
    main()
