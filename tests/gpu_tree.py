"""Read the searched trees the GPU search leaves in its workspace.

Test helper: it decodes the tree storage described in include/dvc.h's
workspace notes (a 16-word header per tree, then per node a record followed
by its first block of 64 child entries {key | chooser << 16, N, W, node id},
overflow blocks chained through a next-block table) into the same fields as
the oracle's tree dump, so that whole trees can be compared node by node.
"""
from __future__ import annotations

import numpy as np

HEADER_WORDS = 16
BLOCK_ENTRIES = 64
BLOCK_WORDS = 4 * BLOCK_ENTRIES
NO_BLOCK = 0xFFFFFFFF


def shape(iterations: int, continue_choice: int = 0, vanilla: int = 0) -> dict:
    node_words = 80 if continue_choice else 40
    nodes_cap = (2 * iterations if vanilla else iterations) + 1
    return {"node_words": node_words, "node_stride": node_words + BLOCK_WORDS,
            "nodes_cap": nodes_cap, "ovf_cap": nodes_cap // BLOCK_ENTRIES + 2}


def decode(words: np.ndarray, iterations: int, continue_choice: int = 0) -> np.ndarray:
    """One tree's workspace words (uint32) -> array with fields parent, key,
    chooser, n, w (node 0 = root: parent -1, n = root visits), creation order."""
    sh = shape(iterations, continue_choice)
    W = words.astype(np.uint32, copy=False)
    n_nodes = int(W[0])
    ovf_base = HEADER_WORDS + sh["nodes_cap"] * sh["node_stride"]
    bnext = ovf_base + sh["ovf_cap"] * BLOCK_WORDS
    out = np.zeros(n_nodes, np.dtype([("parent", np.int64), ("key", np.int64),
                                      ("chooser", np.int64), ("n", np.uint32),
                                      ("w", np.float32)]))
    out["parent"][0] = -1
    out["key"][0] = -1
    out["n"][0] = W[2]
    seen = np.zeros(n_nodes, bool)
    seen[0] = True
    for nd in range(n_nodes):
        rec = HEADER_WORDS + nd * sh["node_stride"]
        nc = int(W[rec + 2])
        blk = nd
        for ci in range(nc):
            if ci and ci % BLOCK_ENTRIES == 0:
                blk = int(W[bnext + blk])
                assert blk != NO_BLOCK
            if blk < sh["nodes_cap"]:
                off = HEADER_WORDS + blk * sh["node_stride"] + sh["node_words"]
            else:
                off = ovf_base + (blk - sh["nodes_cap"]) * BLOCK_WORDS
            e = off + (ci % BLOCK_ENTRIES) * 4
            c = int(W[e + 3])
            assert 0 < c < n_nodes and not seen[c], (nd, ci, c)
            seen[c] = True
            out["parent"][c] = nd
            out["key"][c] = int(W[e]) & 0xFFFF
            out["chooser"][c] = int(W[e]) >> 16
            out["n"][c] = W[e + 1]
            out["w"][c] = W[e + 2:e + 3].view(np.float32)[0]
    assert seen.all()
    return out


def trees(workspace, n_trees: int, tree_bytes: int, iterations: int,
          continue_choice: int = 0) -> list:
    """Decode every tree of a workspace tensor (uint8, tree_bytes per tree)."""
    raw = workspace[:n_trees * tree_bytes].cpu().numpy().view(np.uint32)
    per = tree_bytes // 4
    return [decode(raw[t * per:(t + 1) * per], iterations, continue_choice)
            for t in range(n_trees)]


def assert_same_tree(got: np.ndarray, ref: np.ndarray):
    """GPU tree vs the oracle's dump: same nodes in creation order, same
    parent, key, chooser, N and W (bit pattern) for every non-root node, same
    root visit count."""
    assert len(got) == len(ref), (len(got), len(ref))
    assert int(got["n"][0]) == int(ref["n"][0])
    g, r = got[1:], ref[1:]
    assert np.array_equal(g["parent"], r["parent"].astype(np.int64))
    assert np.array_equal(g["key"], r["key"].astype(np.int64))
    assert np.array_equal(g["chooser"], r["chooser"].astype(np.int64))
    assert np.array_equal(g["n"], r["n"].astype(np.uint32))
    bad = np.flatnonzero(g["w"].view(np.uint32) != r["w"].astype(np.float32).view(np.uint32))
    assert bad.size == 0, (bad[:5] + 1, g["w"][bad[:5]], r["w"][bad[:5]])
