"""GPU parity of whole searched trees, below the root's children.

Bar: bit-exact.  The GPU search leaves its trees in the workspace; they are
decoded (``gpu_tree``) and compared node by node with the oracle's tree dump:
creation order, parent, guess key, chooser, N and W.  A node's W is the wins
(or network values) of the player who chose its guess, so the nodes below the
root's children check credit to other players than the searching one
(Sec. II-B: the results weight the nodes on the path).

* playout leaves: mixed 2/3/4-player roots, depth thresholds 3 and 4 and none,
  with the continue choice, one and four leaves per pass; roots with more
  than 128 legal guesses (three blocks of root children); a four-player root
  whose third opponent holds 17 tiles (guesses of pairs 64-71);
* value leaves (the learned evaluator with its playout fallback) with the
  integer network of ``exact_net``, whose outputs 0, 1/2 and 1 are exact in
  any summation order, so the search's own rules are compared without
  rounding: band 0 (every leaf scored by the network) and band 0.05 (leaves
  whose root-player value is 1/2 fall back to 64 playouts), deep trees
  (several times as many iterations as the root has guesses), one to four
  leaves per pass (four leaves' perspective rows fill one matrix tile).
"""
import numpy as np
import pytest

import exact_net
import gpu_tree
import positions as POS

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dvc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_10720_amd as D
    D.lib()
    return D


def _roots(orc, n, seed, **kw):
    args = dict(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=12,
                revealed_max=5, root_draw=1)
    args.update(kw)
    return orc.init_states(n, orc.deal_params(**args), seed=seed)


def _search_and_compare(orc, dvc, roots, mo, md, seed, tree_base=0):
    """Run the GPU batch once, then every tree against the oracle's dump."""
    n = len(roots)
    per_tree = dvc.dvc_mcts_workspace_bytes(1, md)
    ws = torch.zeros(per_tree * n, dtype=torch.uint8, device="cuda")
    best, _ = dvc.mcts_search(torch.from_numpy(np.ascontiguousarray(roots).view(np.int32)).cuda(),
                              md, seed, tree_base, workspace=ws, want_children=False)
    torch.cuda.synchronize()
    assert dvc.dvc_check() == 0
    got = gpu_tree.trees(ws, n, per_tree, md.iterations, md.continue_choice)
    stats = dvc.mcts_tree_stats(ws, n, md)
    deep = 0
    for t in range(n):
        ref_best, ref = orc.mcts_tree(roots[t], mo, seed, tree_base + t)
        print(f"tree {t}: {len(ref)} nodes", flush=True)
        gpu_tree.assert_same_tree(got[t], ref)
        assert int(best[t].item()) == ref_best
        deep += int(np.sum(ref["depth"] >= 2))
    return stats, deep


@pytest.mark.parametrize("dmax,cont,lpp", [(3, 0, 1), (4, 0, 4), (0, 0, 1), (0, 1, 2)])
def test_playout_trees_node_by_node(orc, dvc, dmax, cont, lpp):
    roots = _roots(orc, 8, 401 + dmax + 10 * cont)
    kw = dict(iterations=300, playouts_per_leaf=8, max_depth=dmax, continue_choice=cont,
              leaves_per_pass=lpp)
    _, deep = _search_and_compare(orc, dvc, roots, orc.mcts_params(**kw), dvc.mcts_params(**kw), 13)
    assert deep > 200


# roots of the batched workload (2048 mixed mid-game roots, seed 3) with more
# than 128 legal guesses: the root's children fill three child blocks
WIDE_ROOTS = [392, 910, 1214, 1269, 1571, 1827, 1863, 1899]


@pytest.mark.parametrize("lpp,pipe", [(1, 0), (2, 1)])
def test_wide_roots_node_by_node(orc, dvc, lpp, pipe):
    roots = _roots(orc, 2048, 3, pile_max=16, revealed_max=8)[WIDE_ROOTS]
    assert min(int(orc.legal_actions(r).sum()) for r in roots) > 128
    kw = dict(iterations=400, playouts_per_leaf=8, max_depth=4, leaves_per_pass=lpp, pipeline=pipe)
    _, deep = _search_and_compare(orc, dvc, roots, orc.mcts_params(**kw), dvc.mcts_params(**kw), 3)
    assert deep > 200


def _long_row_root():
    """Four players, the mover's third opponent holding 17 tiles (its slot 16
    hidden: guesses of pairs 64-71), after the mover's draw, empty pool."""
    owner = [3] * 17 + [0, 1, 2, 0, 1, 2, 0]
    hidden = {3, 5, 8, 11, 14, 16, 17, 20, 21, 22}
    return POS.pack({"P": 4, "owner": owner, "revealed": set(range(24)) - hidden, "mover": 0,
                     "phase": 1, "drawn": 20})


@pytest.mark.parametrize("lpp,pipe", [(1, 0), (2, 1)])
def test_long_row_root_node_by_node(orc, dvc, lpp, pipe):
    root = _long_row_root()
    legal = np.nonzero(orc.legal_actions(root))[0]
    assert any(a // 12 >= 64 for a in legal)
    roots = np.stack([root, root])
    kw = dict(iterations=300, playouts_per_leaf=8, max_depth=4, leaves_per_pass=lpp, pipeline=pipe)
    _, deep = _search_and_compare(orc, dvc, roots, orc.mcts_params(**kw), dvc.mcts_params(**kw), 5)
    assert deep > 200


def _value_kw(net, band, iters, dmax, lpp):
    return dict(iterations=iters, playouts_per_leaf=1, max_depth=dmax, leaf_eval=1,
                fallback_band=band, fallback_playouts=64, valuenet=net, leaves_per_pass=lpp)


@pytest.mark.parametrize("band,dmax,lpp", [(0.0, 4, 1), (0.05, 4, 1), (0.0, 0, 2), (0.05, 3, 2),
                                           (0.05, 4, 3), (0.0, 4, 4)])
def test_value_mode_trees_node_by_node(orc, dvc, band, dmax, lpp):
    p = exact_net.params()
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(p).cuda())
    roots = _roots(orc, 8, 411 + int(band * 100) + dmax)
    legal = max(int(orc.legal_actions(r).sum()) for r in roots)
    iters = 4 * legal
    mo = orc.mcts_params(**_value_kw(p, band, iters, dmax, lpp))
    md = dvc.mcts_params(**_value_kw(net, band, iters, dmax, lpp))
    stats, deep = _search_and_compare(orc, dvc, roots, mo, md, 17)
    assert deep > 100
    played = int(stats["played_leaves"].sum())
    scored = int(stats["net_leaves"].sum())
    if band == 0.0:
        assert played == 0 and scored > 0
    else:
        # value 1/2 for the root player (equal hidden counts) falls back
        assert played > 0 and scored > 0, (played, scored)


def test_value_mode_mixed_batch_against_single_trees(orc, dvc):
    """Value-mode trees are packed four to a workgroup: a tree's result does not
    depend on its neighbours (a batch of 10 vs each tree alone)."""
    p = exact_net.params()
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(p).cuda())
    roots = _roots(orc, 10, 431, pile_max=16, revealed_max=8)
    md = dvc.mcts_params(**_value_kw(net, 0.05, 160, 4, 1))
    st = torch.from_numpy(roots.view(np.int32)).cuda()
    best, kids = dvc.mcts_search(st, md, 19, 50)
    for t in (0, 3, 9):
        b1, k1 = dvc.mcts_search(st[t:t + 1], md, 19, 50 + t)
        assert int(b1[0].item()) == int(best[t].item())
        assert torch.equal(k1[0], kids[t])
    assert dvc.dvc_check() == 0
