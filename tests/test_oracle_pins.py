"""Pins of the oracle's tree moves, credit rule and value leaf (CPU only).

Each check compares the oracle with a reference written in the tests from
the paper's rules, sharing no code with it:
* the candidate guesses at a state (``rules_ref.candidates``) against
  ``oracle_legal_actions`` on thousands of generated states;
* one guess played inside the tree (``rules_ref.play``: reveal on a right
  guess; on a wrong one the drawn tile, or an own tile by word 0 when none was
  drawn; elimination; the next player's draw by word 1) against
  ``oracle_apply_action``, over right and wrong guesses, with and without a
  drawn tile, and endgames;
* whole searched trees (every node's parent, guess, chooser, N and W) against
  the plain loop of ``search_ref`` with depth thresholds 2 and 3, where nodes
  below the root's children are credited with their own chooser's wins;
* value mode with the network of ``exact_net`` (outputs exactly 0, 1/2, 1,
  stated in closed form), band 0 and band 0.05, against the same loop.
``test_oracle_mutations.py`` plants a mistake in each of these parts of the
oracle and checks that one of these checks fails.
"""
import numpy as np
import pytest

import exact_net
import positions as POS
import rules_ref as R
import search_ref


def _states(orc, n, seed, phase_mix=1, **kw):
    args = dict(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8, phase_mix=phase_mix)
    args.update(kw)
    return orc.init_states(n, orc.deal_params(**args), seed)


def _endgames(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        P = int(rng.integers(2, 5))
        d = POS.tiny_endgame(rng, P, hidden_per_seat=(1, 3), pool=(0, 3), phase1=True)
        out.append(POS.pack(d))
    return np.array(out, np.uint32)


def _undecided(orc, S):
    keep = [s for s in S if len(R.seats_in(POS.unpack(s))) >= 2
            and R.hidden(POS.unpack(s), POS.unpack(s)["mover"])]
    return np.array(keep, np.uint32)


def _is_right(pos, a):
    r, slot, value = R.decode_action(a)
    t = R.row(pos, (pos["mover"] + r) % pos["P"])[slot]
    return 2 * value + (t & 1) == t


def check_candidates(orc, n=1500):
    S = np.concatenate([_states(orc, n, 301), _endgames(300, 302)])
    S = _undecided(orc, S)
    assert len(S) > n
    for s in S:
        ref = R.candidates(POS.unpack(s))
        got = set(np.flatnonzero(orc.legal_actions(s)).tolist())
        assert got == ref, (s.tolist(), sorted(got ^ ref)[:8])


def check_in_tree_step(orc, n=500):
    rng = np.random.default_rng(303)
    S = np.concatenate([_states(orc, n, 304, root_draw=1, phase_mix=0),
                        _states(orc, n // 2, 305, pile_min=0, pile_max=0, root_draw=1,
                                phase_mix=0),
                        _endgames(n, 306)])
    S = _undecided(orc, S)
    kinds = {"right": 0, "wrong_drawn": 0, "wrong_own": 0, "over": 0}
    for k, s in enumerate(S):
        pos = POS.unpack(s)
        cands = sorted(R.candidates(pos))
        if not cands:
            continue
        right = [a for a in cands if _is_right(pos, a)]
        picks = [int(rng.choice(cands))]
        if right:
            picks.append(int(rng.choice(right)))
        for a in picks:
            it, depth, tree, seed = int(rng.integers(0, 5000)), int(rng.integers(0, 4)), k, 91
            words = orc.philox([depth, R.CHANCE_DOMAIN, it, tree], [seed, 0])
            ref, over, win = R.play(pos, a, words)
            got, g_over, g_win = orc.apply_action(s, a, seed, tree, it, depth)
            assert g_over == over and g_win == win, (s.tolist(), a)
            assert np.array_equal(got, POS.pack(ref)), (s.tolist(), a)
            is_right = a in right
            kinds["right" if is_right else
                  "wrong_drawn" if pos["drawn"] is not None else "wrong_own"] += 1
            kinds["over"] += over
    assert min(kinds.values()) >= 20, kinds


def _compare_tree(orc, root, mp, seed, tree, ref_nodes, ref_best):
    best, got = orc.mcts_tree(root, mp, seed, tree)
    assert len(got) == len(ref_nodes)
    for x, r in enumerate(ref_nodes):
        g = got[x]
        assert (int(g["parent"]), int(g["key"]), int(g["chooser"]), int(g["n"])) == \
            (r["parent"], r["key"], r["chooser"], r["n"]), x
        assert np.float32(g["w"]).view(np.uint32) == np.float32(r["w"]).view(np.uint32), x
    assert best == ref_best
    return got


def check_search_trees(orc):
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=12,
                         revealed_max=5, root_draw=1)
    roots = orc.init_states(6, dp, seed=307)
    deep = 0
    for t, root in enumerate(roots):
        dmax = 2 + t % 2
        iters, ppl, seed = 150 + 50 * (t % 3), 4, 17
        mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=dmax)
        nodes, best = search_ref.search(orc, root, iters, ppl, dmax, seed, t)
        got = _compare_tree(orc, root, mp, seed, t, nodes, best)
        # credit below the root's children goes to other players than the root's
        M = POS.unpack(root)["mover"]
        deep += int(np.sum((got["depth"] >= 2) & (got["chooser"] != M)))
    assert deep > 100


def check_value_trees(orc):
    p = exact_net.params()
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=12,
                         revealed_max=5, root_draw=1)
    roots = orc.init_states(6, dp, seed=308)
    for t, root in enumerate(roots):
        band = 0.0 if t % 2 == 0 else 0.05
        dmax, iters, seed = 3, 160, 23
        mp = orc.mcts_params(iterations=iters, playouts_per_leaf=1, max_depth=dmax, leaf_eval=1,
                             fallback_band=band, fallback_playouts=64, valuenet=p)
        nodes, best = search_ref.search(orc, root, iters, 1, dmax, seed, t,
                                        value=exact_net.closed_form, band=band,
                                        fallback_playouts=64)
        _compare_tree(orc, root, mp, seed, t, nodes, best)


def check_pass_trees(orc):
    """Passes of B leaves, pipelined (a pass's wins credited after the next
    pass's descents), playout and value leaves, against the loop of
    ``search_ref`` with the same pass rule; on these roots the pipelined trees
    differ from the plain passes' trees, so crediting a pass at once fails."""
    p = exact_net.params()
    dp = orc.deal_params(p_min=2, p_max=3, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=6,
                         revealed_max=5, root_draw=1)
    roots = orc.init_states(6, dp, seed=311)
    differ = 0
    for t, root in enumerate(roots):
        B = (1, 2, 4)[t % 3]
        if t >= 3:   # value leaves with the integer network
            band = 0.05 if t % 2 else 0.0
            kw = dict(value=exact_net.closed_form, band=band, fallback_playouts=64)
            mk = lambda pipe: orc.mcts_params(iterations=300, playouts_per_leaf=1, max_depth=3,
                                              leaf_eval=1, fallback_band=band,
                                              fallback_playouts=64, valuenet=p,
                                              leaves_per_pass=B, pipeline=pipe)
            iters, ppl = 300, 1
        else:
            kw = {}
            mk = lambda pipe: orc.mcts_params(iterations=400, playouts_per_leaf=4, max_depth=3,
                                              leaves_per_pass=B, pipeline=pipe)
            iters, ppl = 400, 4
        nodes, best = search_ref.search(orc, root, iters, ppl, 3, 29, t, leaves_per_pass=B,
                                        pipeline=1, **kw)
        _compare_tree(orc, root, mk(1), 29, t, nodes, best)
        plain, _ = search_ref.search(orc, root, iters, ppl, 3, 29, t, leaves_per_pass=B, **kw)
        differ += [(n["key"], n["n"], n["w"]) for n in plain] != \
            [(n["key"], n["n"], n["w"]) for n in nodes]
    assert differ >= 4, differ


def test_pipelined_and_batched_passes(orc):
    check_pass_trees(orc)


def test_candidate_guesses(orc):
    check_candidates(orc)


def test_in_tree_step(orc):
    check_in_tree_step(orc)


def test_search_trees_with_depth(orc):
    check_search_trees(orc)


def test_value_mode_trees(orc):
    check_value_trees(orc)


def test_exact_network_closed_form(orc):
    """The oracle's network (exact and bf16 mirror) on the integer network
    gives the closed form of ``exact_net`` in float32 on 3000 states."""
    p = exact_net.params()
    S = _states(orc, 3000, 309)
    q = np.array([i % POS.unpack(s)["P"] for i, s in enumerate(S)], np.int32)
    ref = np.array([exact_net.closed_form(POS.unpack(s), int(qq)) for s, qq in zip(S, q)],
                   np.float32)
    for mirror in (False, True):
        v = orc.vn_forward(p, S, q, bf16_mirror=mirror).astype(np.float32)
        assert np.array_equal(v, ref)
    assert set(np.unique(ref)) == {0.0, 0.5, 1.0}


@pytest.mark.parametrize("P", [2, 3, 4])
def test_chooser_is_the_player_to_move(orc, P):
    """The root's children are the searching player's guesses, and a guess
    inside the tree ends the turn, so the level below belongs to another
    player (on the oracle's tree dump)."""
    dp = orc.deal_params(p_min=P, p_max=P, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=8,
                         revealed_max=3, root_draw=1)
    root = orc.init_states(1, dp, seed=310 + P)[0]
    mp = orc.mcts_params(iterations=120, playouts_per_leaf=2, max_depth=3)
    _, got = orc.mcts_tree(root, mp, 5, 0)
    M = POS.unpack(root)["mover"]
    assert np.all(got["chooser"][got["depth"] == 1] == M)
    lvl2 = got[got["depth"] == 2]
    assert len(lvl2) > 0 and np.all(lvl2["chooser"] != M)
