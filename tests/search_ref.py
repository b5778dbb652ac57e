"""The simplified tree search restated as a plain loop (tests only).

Independent of the oracle's search code: the moves come from
``rules_ref`` (written from the rules), the per-iteration world from the
oracle's sampler (``determinize``, a pinned input here) and leaf playouts
from the oracle's rollout (pinned by exact enumeration).  What this loop
fixes is the search itself (Sec. II-B, Sec. III-A):

* iteration i samples a world, then descends from the root.  A finished game
  is a leaf; at the depth threshold the node is a leaf; otherwise the lowest
  candidate guess without a child is added and its child is the leaf; else
  the candidate child with the largest UCT score, first created on ties:
  q = W/n, e = LN[N_parent]/n, u = c sqrt(e), score = q + u, each step
  rounded to float32, LN[k] = float32(log k);
* the leaf's value per seat: the winner takes every playout of a finished
  game; otherwise `ppl` random playouts with leaf id i (playout mode), or
  the network's value of each seat (value mode), played out instead when the
  searching player's value is within `band` of 1/2;
* every node on the path gains the leaf's weight in N; every node below the
  root gains in W the value of the seat that chose its guess -- the player to
  move at its parent, not the searching player.

Passes (``leaves_per_pass`` B): B descents, each adding its N at once, then
the B leaves' values in iteration order.  Pipelined passes (``pipeline``):
a pass's values go in only after the next pass's descents, the last pass's
at the end.
"""
from __future__ import annotations

import math

import numpy as np

import positions as POS
import rules_ref as R


def search(orc, root, iters, ppl, max_depth, seed, tree, c_uct=None, value=None, band=0.05,
           fallback_playouts=64, leaves_per_pass=1, pipeline=0):
    """Returns the tree as a list of nodes {parent, key, chooser, n, w} in
    creation order (node 0 is the root) and the decision.  value: None for
    playout leaves, else a function (position dict, seat) -> value."""
    c = np.float32(math.sqrt(2.0)) if c_uct is None else np.float32(c_uct)
    weight = fallback_playouts if value is not None else ppl
    key = [seed & 0xFFFFFFFF, seed >> 32]
    nodes = [{"parent": -1, "key": -1, "chooser": -1, "n": 0, "w": np.float32(0), "kids": []}]
    M = POS.unpack(root)["mover"]

    def credit(path, vals):
        for k in path[1:]:
            nodes[k]["w"] = np.float32(nodes[k]["w"] + vals[nodes[k]["chooser"]])

    pending = []          # (path, values) of a pipelined pass not yet credited
    passed = []           # this pass's (iteration, path, position, over, winner)
    for i in range(iters):
        world, _ = orc.determinize(root, seed, tree, i)
        pos = POS.unpack(world)
        x, depth, path = 0, 0, [0]
        over, winner = False, -1
        while not over and not (max_depth > 0 and depth >= max_depth):
            cands = R.candidates(pos)
            words = orc.philox([depth, R.CHANCE_DOMAIN, i, tree], key)
            have = {nodes[k]["key"] for k in nodes[x]["kids"]}
            untried = sorted(cands - have)
            if untried:
                a = untried[0]
                nodes.append({"parent": x, "key": a, "chooser": pos["mover"], "n": 0,
                              "w": np.float32(0), "kids": []})
                nodes[x]["kids"].append(len(nodes) - 1)
                path.append(len(nodes) - 1)
                pos, over, winner = R.play(pos, a, words)
                break
            lp = np.float32(math.log(nodes[x]["n"]))
            best, best_s = None, None
            for k in nodes[x]["kids"]:
                if nodes[k]["key"] not in cands:
                    continue
                n = np.float32(nodes[k]["n"])
                s = nodes[k]["w"] / n + c * np.sqrt(lp / n)
                if best is None or s > best_s:
                    best, best_s = k, s
            pos, over, winner = R.play(pos, nodes[best]["key"], words)
            x = best
            path.append(x)
            depth += 1
        for k in path:
            nodes[k]["n"] += weight
        passed.append((i, path, pos, over, winner))
        if len(passed) < leaves_per_pass and i + 1 < iters:
            continue
        # the pass is complete: a pipelined search credits the previous pass now
        for pth, vals in pending:
            credit(pth, vals)
        pending = []
        for it, pth, lpos, lover, lwin in passed:
            vals = [np.float32(0)] * 4
            if lover:
                vals[lwin] = np.float32(weight)
            else:
                playout = value is None
                if value is not None:
                    v = [np.float32(value(lpos, q)) for q in range(lpos["P"])]
                    if abs(v[M] - np.float32(0.5)) < np.float32(band):
                        playout = True
                    else:
                        vals = [np.float32(weight) * v[q] for q in range(lpos["P"])] + \
                               [np.float32(0)] * (4 - lpos["P"])
                if playout:
                    _, _, wins = orc.rollout(POS.pack(lpos), weight, seed, tree_id=tree,
                                             leaf_id_base=it, want_winner=False, want_length=False)
                    vals = [np.float32(w) for w in wins[0]]
            if pipeline:
                pending.append((pth, vals))
            else:
                credit(pth, vals)
        passed = []
    for pth, vals in pending:
        credit(pth, vals)
    root_kids = nodes[0]["kids"]
    best = max(root_kids, key=lambda k: (nodes[k]["n"], -root_kids.index(k)))
    return nodes, nodes[best]["key"]
