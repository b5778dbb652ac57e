"""GPU parity of the un-simplified tree variants (through the C ABI).

Bar: bit-exact against the CPU oracle -- chosen action and every root
statistic (action, visit count, win-sum bits) -- for each simplification of
Sec. III-A switched off alone and together: the continue/stop choice after a
right guess, no depth threshold, and worlds as the root's children
(vanilla, root statistics summed per action over the worlds).  Also: value
mode with band 1 equals the playout search under the variants, root-parallel
search with the continue choice, and the parameter errors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from test_gpu_mcts import dev_states, assert_same, merged_view, assert_same_merged  # noqa: E402

MODES = {
    "continue": dict(continue_choice=1, max_depth=4),
    "continue_unlimited": dict(continue_choice=1, max_depth=0),
    "unlimited": dict(max_depth=0),
    "vanilla": dict(vanilla=1, max_depth=4),
    "vanilla_continue_unlimited": dict(vanilla=1, continue_choice=1, max_depth=0),
}


@pytest.fixture(scope="module")
def dvc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_10720_amd as D
    D.lib()
    return D


def run_both(orc, dvc, roots, iters, ppl, seed, tree_base=0, **mode):
    mo = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, **mode)
    md = dvc.mcts_params(iterations=iters, playouts_per_leaf=ppl, **mode)
    print(f"roots {len(roots)} iters {iters} ppl {ppl} seed {seed} mode {mode}", flush=True)
    best_ref, kids_ref = orc.mcts_search(roots, mo, seed, tree_base)
    best, kids = dvc.mcts_search(dev_states(roots), md, seed, tree_base)
    torch.cuda.synchronize()
    assert dvc.dvc_check() == 0
    act, n, w = dvc.children_view(kids)
    return best_ref, kids_ref, best.cpu().numpy(), act.numpy(), n.numpy(), w.numpy()


@pytest.mark.parametrize("mode", sorted(MODES))
def test_fresh_two_player_deal(orc, dvc, mode):
    """The single-tree workload: one fresh two-player deal, 2000 x 16."""
    roots = orc.init_states(1, orc.deal_params(p_min=2, p_max=2, fresh=1, root_draw=1), seed=1)
    assert_same(*run_both(orc, dvc, roots, 2000, 16, seed=1, **MODES[mode]))


@pytest.mark.parametrize("mode", sorted(MODES))
def test_mixed_mid_game_roots(orc, dvc, mode):
    """2/3/4-player mid-game roots, 400 iterations x 8 playouts, ragged tree ids."""
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(12, dp, seed=17)
    assert_same(*run_both(orc, dvc, roots, 400, 8, seed=4, tree_base=33, **MODES[mode]))


@pytest.mark.parametrize("mode", ["continue_unlimited", "vanilla_continue_unlimited"])
def test_endgames_reach_the_end_of_the_game(orc, dvc, mode):
    """Small endgames (1-3 hidden tiles per player, pool 0-2) whose trees run
    to decided states; ragged playout counts."""
    import positions as POS
    rng = np.random.default_rng(3)
    roots = []
    while len(roots) < 10:
        pos = POS.tiny_endgame(rng, 2 + len(roots) % 3, hidden_per_seat=(1, 3), pool=(0, 2),
                               phase1=True)
        r = POS.pack(pos)
        if orc.validate(r) == 0 and pos["phase"] == 1:
            roots.append(r)
    roots = np.stack(roots)
    for iters, ppl in [(1, 1), (37, 3), (300, 65)]:
        assert_same(*run_both(orc, dvc, roots, iters, ppl, seed=iters, **MODES[mode]))


def test_batched_workload_trees_0_to_63_with_continue_choice(orc, dvc):
    """The batched workload (1024 iterations x 32 playouts), continue choice on."""
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(64, dp, seed=3)
    assert_same(*run_both(orc, dvc, roots, 1024, 32, seed=3, continue_choice=1, max_depth=0))


def test_vanilla_batched_trees_0_to_15(orc, dvc):
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(16, dp, seed=3)
    assert_same(*run_both(orc, dvc, roots, 1024, 32, seed=3, vanilla=1, max_depth=4))


@pytest.mark.parametrize("mode", ["continue_unlimited", "vanilla"])
def test_value_mode_band_one_equals_playouts(orc, dvc, mode):
    """band 1: every leaf is played out with fallback_playouts, so value mode
    equals the playout search under the same variant."""
    params = orc.vn_init(44)
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(params).cuda())
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8, root_draw=1)
    roots = orc.init_states(9, dp, seed=27)
    mo = orc.mcts_params(iterations=150, playouts_per_leaf=64, **MODES[mode])
    best_ref, kids_ref = orc.mcts_search(roots, mo, 7)
    md = dvc.mcts_params(iterations=150, playouts_per_leaf=5, leaf_eval=1, fallback_band=1.0,
                         fallback_playouts=64, valuenet=net, **MODES[mode])
    best, kids = dvc.mcts_search(dev_states(roots), md, 7)
    torch.cuda.synchronize()
    assert dvc.dvc_check() == 0
    act, n, w = dvc.children_view(kids)
    assert_same(best_ref, kids_ref, best.cpu().numpy(), act.numpy(), n.numpy(), w.numpy())


def test_root_parallel_with_continue_choice(orc, dvc):
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(5, dp, seed=61)
    kw = dict(iterations=200, playouts_per_leaf=8, continue_choice=1, max_depth=0)
    best_ref, m_ref = orc.mcts_search_merged(roots, 4, orc.mcts_params(**kw), 6, 100)
    best, kids = dvc.mcts_search_root_parallel(dev_states(roots), 4, dvc.mcts_params(**kw), 6, 100)
    torch.cuda.synchronize()
    assert dvc.dvc_check() == 0
    assert_same_merged(best_ref, m_ref, best, kids, dvc)


def test_vanilla_root_parallel_is_rejected(dvc):
    st = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(dvc.DvcError):
        dvc.mcts_search_root_parallel(st, 2, dvc.mcts_params(iterations=10, vanilla=1), 1)


def test_workspace_grows_with_the_variants(dvc):
    base = dvc.dvc_mcts_workspace_bytes(3, dvc.mcts_params(iterations=100))
    cont = dvc.dvc_mcts_workspace_bytes(3, dvc.mcts_params(iterations=100, continue_choice=1))
    van = dvc.dvc_mcts_workspace_bytes(3, dvc.mcts_params(iterations=100, vanilla=1))
    assert base < cont and base < van and base % 16 == 0 and cont % 16 == 0 and van % 16 == 0


# ---------------------------------------------------------------------------
# leaf batching: B leaves per pass evaluated together
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B,ppl", [(2, 32), (3, 21), (4, 16), (16, 5), (5, 64), (16, 1)])
def test_leaf_batching_matches_oracle(orc, dvc, B, ppl):
    """Playouts of a pass packed into the tree's 64 lanes, including leaves
    split across two chunks of 64 (ppl 21, 5) and ragged last passes."""
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(10, dp, seed=40 + B)
    assert_same(*run_both(orc, dvc, roots, 301, ppl, seed=5, tree_base=3, max_depth=4,
                          leaves_per_pass=B))


def test_leaf_batching_single_tree_workload(orc, dvc):
    """The single-tree workload (fresh two-player deal, 2000 x 16) with four
    leaves per pass: 64 playouts per pass."""
    roots = orc.init_states(1, orc.deal_params(p_min=2, p_max=2, fresh=1, root_draw=1), seed=1)
    assert_same(*run_both(orc, dvc, roots, 2000, 16, seed=1, max_depth=4, leaves_per_pass=4))


def test_leaf_batching_batched_workload_trees_0_to_63(orc, dvc):
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(64, dp, seed=3)
    assert_same(*run_both(orc, dvc, roots, 1024, 32, seed=3, max_depth=4, leaves_per_pass=2))


@pytest.mark.parametrize("mode", ["continue_unlimited", "vanilla_continue_unlimited"])
def test_leaf_batching_with_variants(orc, dvc, mode):
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(8, dp, seed=47)
    assert_same(*run_both(orc, dvc, roots, 257, 8, seed=6, leaves_per_pass=4, **MODES[mode]))


def test_leaf_batching_value_mode_band_one_equals_playouts(orc, dvc):
    """Value mode, two leaves per matrix tile, band 1: every leaf is played
    out, so the search equals the batched playout search."""
    params = orc.vn_init(44)
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(params).cuda())
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8, root_draw=1)
    roots = orc.init_states(9, dp, seed=29)
    mo = orc.mcts_params(iterations=151, playouts_per_leaf=64, max_depth=4, leaves_per_pass=2)
    best_ref, kids_ref = orc.mcts_search(roots, mo, 7)
    md = dvc.mcts_params(iterations=151, playouts_per_leaf=5, leaf_eval=1, fallback_band=1.0,
                         fallback_playouts=64, valuenet=net, max_depth=4, leaves_per_pass=2)
    best, kids = dvc.mcts_search(dev_states(roots), md, 7)
    torch.cuda.synchronize()
    assert dvc.dvc_check() == 0
    act, n, w = dvc.children_view(kids)
    assert_same(best_ref, kids_ref, best.cpu().numpy(), act.numpy(), n.numpy(), w.numpy())


def test_leaf_batching_value_mode_root_values_vs_oracle(orc, dvc):
    """Band 0, two leaves per tile: with as many iterations as root guesses
    every root child is expanded once and its W is 64 * v(chooser) of its
    leaf; the second row group of the tile is compared as well as the first."""
    params = orc.vn_init(44)
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(params).cuda())
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=12, revealed_max=6, root_draw=1)
    roots = orc.init_states(4, dp, seed=31)
    for t in range(4):
        k = int(orc.legal_actions(roots[t]).sum())
        kw = dict(iterations=k, playouts_per_leaf=1, max_depth=4, leaf_eval=1, fallback_band=0.0,
                  fallback_playouts=64, leaves_per_pass=2)
        _, kids_ref = orc.mcts_search(roots[t:t + 1], orc.mcts_params(valuenet=params, **kw), 7, t)
        _, kids = dvc.mcts_search(dev_states(roots[t:t + 1]), dvc.mcts_params(valuenet=net, **kw), 7, t)
        torch.cuda.synchronize()
        act, n, w = dvc.children_view(kids)
        kr = kids_ref[0]
        assert np.array_equal(act.numpy()[0], kr["action"].astype(np.int64))
        assert np.array_equal(n.numpy()[0], kr["n"].astype(np.int64))
        tol = 64 * (2.0 ** -7 * np.abs(kr["w"] / 64) + 1e-3)
        assert np.all(np.abs(w.numpy()[0] - kr["w"]) <= tol + 1e-6)


def test_leaf_batching_root_parallel(orc, dvc):
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8, root_draw=1)
    roots = orc.init_states(4, dp, seed=63)
    kw = dict(iterations=130, playouts_per_leaf=16, max_depth=4, leaves_per_pass=4)
    best_ref, m_ref = orc.mcts_search_merged(roots, 3, orc.mcts_params(**kw), 6, 100)
    best, kids = dvc.mcts_search_root_parallel(dev_states(roots), 3, dvc.mcts_params(**kw), 6, 100)
    torch.cuda.synchronize()
    assert dvc.dvc_check() == 0
    assert_same_merged(best_ref, m_ref, best, kids, dvc)


def test_leaf_batching_argument_errors(dvc):
    st = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
    for bad in (dict(leaves_per_pass=0), dict(leaves_per_pass=17),
                dict(leaves_per_pass=5, leaf_eval=1, valuenet=st)):
        with pytest.raises(dvc.DvcError):
            dvc.mcts_search(st, dvc.mcts_params(**bad), 1)
