"""Pins of the oracle's un-simplified tree variants (CPU only).

The paper's simplified search (Sec. III-A) drops three things, and each can
be switched back on:

* continue choice (simplification 2 off): after a right guess the same player
  chooses between stopping (key 864) and guessing again (key 865 + action).
  Pinned by a separate UCB1 loop at depth threshold 1 that re-derives the
  leaf rule (the random policy's continue coin) from the game rules, and by
  structural invariants of whole trees: who chooses each node, which keys
  follow which, visit-count identities;
* no depth threshold (simplification 3 off, max_depth 0): a threshold beyond
  the longest possible game changes nothing, a small one bounds the tree;
* vanilla (simplification 1 off): the root's children are the sampled worlds.
  With a single possible world the search equals the simplified one; the
  world nodes are exactly the worlds the sampler draws, visited once per
  iteration that draws them; the paper's 12*11*10*9 count of plausible sets
  for four same-coloured tiles is 4! times the number of ascending rows the
  sampler can produce, and the sampler reaches all of them.
"""
import math

import numpy as np
import pytest

import positions as POS
from test_oracle_mcts import _sampler_law, C_UCT

STOP = 864


def _mid_roots(orc, n, seed, P):
    dp = orc.deal_params(p_min=P, p_max=P, fresh=0, pile_min=0, pile_max=12 if P > 2 else 16,
                         revealed_max=4, root_draw=1)
    return orc.init_states(n, dp, seed)


def _rows(pos):
    return [sorted(t for t in range(24) if pos["owner"][t] == q) for q in range(pos["P"])]


def _world_key(world_packed, M):
    """2 bits per tile: the holder's seat relative to M when an opponent holds
    the tile hidden, else 0."""
    w = POS.unpack(world_packed)
    key = 0
    for t in range(24):
        o = w["owner"][t]
        if o >= 0 and o != M and t not in w["revealed"]:
            key |= ((o - M) % w["P"]) << (2 * t)
    return key


# ---------------------------------------------------------------------------
# continue choice
# ---------------------------------------------------------------------------
def _leaf_after_guess(orc, world, action, seed, tree, it):
    """Leaf of a depth-one iteration with the continue choice on, from the
    rules: a wrong guess (or a right one that ends the game) is played as in
    the simplified tree; after a right guess the random policy's coin (word 3
    of the chance block, below 2^31 = go on) keeps the mover guessing with the
    drawn tile still hidden, else the turn passes as in the simplified tree."""
    pos = POS.unpack(world)
    M, P = pos["mover"], pos["P"]
    r, slot, v = action // 288 + 1, (action // 12) % 24, action % 12
    q = (M + r) % P
    t = _rows(pos)[q][slot]
    passed, term, win = orc.apply_action(world, action, seed, tree, it, 0)
    if term or 2 * v + (t & 1) != t:
        return passed, term, win
    w = orc.philox([0, 0xC0000000, it, tree], [seed & 0xFFFFFFFF, seed >> 32])
    if int(w[3]) >= 1 << 31:
        return passed, False, -1
    pos["revealed"] = set(pos["revealed"]) | {t}
    return POS.pack(pos), False, -1


def _ucb1_continue_reference(orc, root, iters, ppl, seed, tree):
    legal = np.flatnonzero(orc.legal_actions(root))
    mover = orc.unpack(root)["mover"]
    arms, N, W = [], {}, {}
    n_root = 0
    for i in range(iters):
        untried = [a for a in legal if a not in N]
        if untried:
            a = int(untried[0])
            arms.append(a)
            N[a], W[a] = 0, np.float32(0)
        else:
            lp = np.float32(math.log(n_root))
            best, best_s = None, None
            for a in arms:
                n = np.float32(N[a])
                s = W[a] / n + C_UCT * np.sqrt(lp / n)
                if best is None or s > best_s:
                    best, best_s = a, s
            a = best
        world, _ = orc.determinize(root, seed, tree, i)
        leaf, term, win = _leaf_after_guess(orc, world, a, seed, tree, i)
        if term:
            wins = np.zeros(4, np.uint32)
            wins[win] = ppl
        else:
            _, _, w4 = orc.rollout(leaf, ppl, seed, tree_id=tree, leaf_id_base=i,
                                   want_winner=False, want_length=False)
            wins = w4[0]
        N[a] += ppl
        W[a] = np.float32(W[a] + np.float32(wins[mover]))
        n_root += ppl
    best = max(arms, key=lambda a: (N[a], -arms.index(a)))
    return arms, N, W, best


@pytest.mark.parametrize("case", range(3))
def test_continue_choice_depth_one_is_ucb1(orc, case):
    roots = orc.init_states(3, orc.deal_params(p_min=2, p_max=3, fresh=0, pile_min=0,
                                               pile_max=8, revealed_max=6, root_draw=1), 80)
    root = roots[case]
    iters, ppl, seed, tree = 250, 4, 91, case
    mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=1, continue_choice=1)
    best, kids = orc.mcts_search(root, mp, seed, tree_id_base=tree)
    arms, N, W, ref_best = _ucb1_continue_reference(orc, root, iters, ppl, seed, tree)
    k = kids[0][kids[0]["action"] != 0xFFFF]
    assert [int(a) for a in k["action"]] == arms
    assert [int(n) for n in k["n"]] == [N[a] for a in arms]
    assert [float(w) for w in k["w"]] == [float(W[a]) for a in arms]
    assert best[0] == ref_best
    # the leaf rule matters: the simplified search differs on these roots
    _, kids_s = orc.mcts_search(root, orc.mcts_params(iterations=iters, playouts_per_leaf=ppl,
                                                      max_depth=1), seed, tree_id_base=tree)
    assert not np.array_equal(kids_s[0]["w"], kids[0]["w"])


def _check_tree(t, iters, ppl, cont):
    """Identities every searched tree satisfies."""
    par, key, ch = t["parent"], t["key"], t["chooser"]
    assert par[0] == -1 and t["n"][0] == iters * ppl
    kids_n = np.zeros(len(t), np.int64)
    np.add.at(kids_n, par[1:], t["n"][1:].astype(np.int64))
    # N(X) = sum of the children's N + ppl per iteration whose leaf is X
    spare = t["n"].astype(np.int64) - kids_n
    assert np.all(spare >= 0) and np.all(spare % ppl == 0)
    assert np.all(t["w"][1:] <= t["n"][1:]) and np.all(t["w"] == np.round(t["w"]))
    for x in range(1, len(t)):
        p, k = par[x], key[x]
        if k < 0:
            continue                     # world node
        if p == 0 or key[p] < 0:
            assert k < STOP, "the root's moves are plain guesses"
            continue
        if k >= STOP:
            assert cont, "stop / continued guesses only with the continue choice"
            assert key[p] != STOP, "a stop is followed by the next player's guesses"
            assert ch[x] == ch[p], "the player who guessed right chooses again"
        else:
            assert ch[x] != ch[p], "after a wrong guess or a stop the turn has passed"
    # each key at most once among a node's children
    pairs = set()
    for x in range(1, len(t)):
        assert (par[x], key[x]) not in pairs or key[x] < 0
        pairs.add((par[x], key[x]))


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("cont", [0, 1])
def test_tree_structure(orc, P, cont):
    roots = _mid_roots(orc, 3, 70 + P, P)
    iters, ppl = 500, 4
    for i, root in enumerate(roots):
        mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=0,
                             continue_choice=cont)
        best, t = orc.mcts_tree(root, mp, 4, tree_id=i)
        _check_tree(t, iters, ppl, cont)
        if cont:
            assert np.any(t["key"] == STOP) and np.any(t["key"] > STOP)
        # the dump's root children are the search's root children
        _, kids = orc.mcts_search(root, mp, 4, i)
        k = kids[0][kids[0]["action"] != 0xFFFF]
        rc = t[t["parent"] == 0]
        assert np.array_equal(rc["key"], k["action"].astype(np.int32))
        assert np.array_equal(rc["n"], k["n"]) and np.array_equal(rc["w"], k["w"])
        assert best == int(k["action"][np.flatnonzero(k["n"] == k["n"].max())[0]])


def test_continue_choice_expands_stop_first(orc):
    """Below a right guess the lowest untried key is the stop (864), then the
    further guesses 865 + a in action order."""
    roots = _mid_roots(orc, 2, 75, 2)
    mp = orc.mcts_params(iterations=800, playouts_per_leaf=2, max_depth=0, continue_choice=1)
    _, t = orc.mcts_tree(roots[0], mp, 6)
    for x in np.flatnonzero(np.isin(np.arange(len(t)), t["parent"][t["key"] >= STOP])):
        ks = t["key"][t["parent"] == x]
        hi = ks[ks >= STOP]
        assert hi[0] == STOP and np.all(np.diff(hi) > 0)


# ---------------------------------------------------------------------------
# depth threshold
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cont", [0, 1])
def test_threshold_beyond_the_longest_game_changes_nothing(orc, cont):
    rng = np.random.default_rng(12)
    for case in range(4):
        pos = POS.tiny_endgame(rng, 2 + case % 2, hidden_per_seat=(1, 3), pool=(0, 2),
                               phase1=True)
        root = POS.pack(pos)
        if orc.validate(root) or pos["phase"] == 0:
            continue
        # every guess reveals a tile (pool tiles are drawn first), the winner
        # keeps one hidden, and a stop only follows a right guess
        unrevealed = 24 - len(pos["revealed"])
        longest = (unrevealed - 1) * (2 if cont else 1)
        out = []
        for d in (longest, 0, 64):
            mp = orc.mcts_params(iterations=300, playouts_per_leaf=4, max_depth=d,
                                 continue_choice=cont)
            out.append(orc.mcts_search(root, mp, 3, case))
        for best, kids in out[1:]:
            assert best[0] == out[0][0][0] and np.array_equal(kids, out[0][1])


@pytest.mark.parametrize("d", [1, 2, 3])
def test_threshold_bounds_the_tree(orc, d):
    rng = np.random.default_rng(5)
    pos = POS.tiny_endgame(rng, 2, hidden_per_seat=(3, 3), pool=(2, 2), phase1=True)
    root = POS.pack(pos)
    assert orc.validate(root) == 0
    mp = orc.mcts_params(iterations=600, playouts_per_leaf=2, max_depth=d, continue_choice=1)
    _, t = orc.mcts_tree(root, mp, 2)
    assert t["depth"].max() == d
    mp0 = orc.mcts_params(iterations=600, playouts_per_leaf=2, max_depth=0, continue_choice=1)
    _, t0 = orc.mcts_tree(root, mp0, 2)
    assert t0["depth"].max() > 3


# ---------------------------------------------------------------------------
# vanilla: worlds as nodes
# ---------------------------------------------------------------------------
def _single_world_root():
    """Two players; each hidden opponent slot has exactly one consistent
    value (black 4 below the revealed 6 with 0 and 2 in the mover's row;
    white 13 between the revealed 11 and 15), so only one world exists."""
    owner = [-1] * 24
    for t in (4, 6, 11, 13, 15, 20):
        owner[t] = 1
    for t in (0, 2, 8, 17, 21):
        owner[t] = 0
    pos = {"P": 2, "owner": owner, "revealed": {6, 11, 15, 20, 21}, "mover": 0, "phase": 1,
           "drawn": 17}
    return pos, POS.pack(pos)


def test_vanilla_single_world_is_the_simplified_search(orc):
    pos, root = _single_world_root()
    for cont in (0, 1):
        kw = dict(iterations=400, playouts_per_leaf=4, max_depth=0, continue_choice=cont)
        best_s, kids_s = orc.mcts_search(root, orc.mcts_params(**kw), 5, 2)
        best_v, kids_v = orc.mcts_search(root, orc.mcts_params(vanilla=1, **kw), 5, 2)
        live = kids_s[0][kids_s[0]["action"] != 0xFFFF]
        # one world: its guesses are the simplified root's, indexed by action id
        assert np.array_equal(np.flatnonzero(kids_v[0]["action"] != 0xFFFF),
                              np.sort(live["action"].astype(np.int64)))
        v = kids_v[0][live["action"].astype(np.int64)]
        assert np.array_equal(v["n"], live["n"]) and np.array_equal(v["w"], live["w"])
        assert best_v[0] == best_s[0]
        _, t = orc.mcts_tree(root, orc.mcts_params(vanilla=1, **kw), 5, 2)
        worlds = t[(t["key"] < 0) & (t["parent"] == 0)]
        assert len(worlds) == 1
        assert int(worlds["world"][0]) == (1 << 8) | (1 << 26)
        assert worlds["n"][0] == 400 * 4


@pytest.mark.parametrize("P", [2, 3])
def test_vanilla_world_nodes_are_the_sampled_worlds(orc, P):
    """The root's children are the distinct sampled worlds in order of first
    appearance, each visited ppl times per iteration that drew it; a guess's
    root statistics are its sums over the worlds."""
    root = _mid_roots(orc, 1, 90 + P, P)[0]
    iters, ppl, seed, tree = 300, 2, 7, 3
    M = orc.unpack(root)["mover"]
    mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=4, vanilla=1)
    best, t = orc.mcts_tree(root, mp, seed, tree)
    order, count = [], {}
    for i in range(iters):
        k = _world_key(orc.determinize(root, seed, tree, i)[0], M)
        if k not in count:
            order.append(k)
            count[k] = 0
        count[k] += 1
    worlds = t[t["parent"] == 0]
    assert np.all(worlds["key"] == -1)
    assert [int(k) for k in worlds["world"]] == order
    assert [int(n) for n in worlds["n"]] == [ppl * count[k] for k in order]
    _check_tree(t, iters, ppl, 0)
    # aggregation and decision
    _, kids = orc.mcts_search(root, mp, seed, tree)
    wid = set(np.flatnonzero(t["parent"] == 0).tolist())
    n = np.zeros(864, np.int64)
    w = np.zeros(864, np.float64)
    for x in range(len(t)):
        if t["parent"][x] in wid:
            n[t["key"][x]] += int(t["n"][x])
            w[t["key"][x]] += float(t["w"][x])
    assert np.array_equal(kids[0]["n"].astype(np.int64), n)
    assert np.array_equal(kids[0]["w"].astype(np.float64), w)
    assert best == int(np.flatnonzero(n == n.max())[0]) == int(kids[0]["action"][best])


def test_vanilla_plausible_sets_of_four_same_coloured_tiles(orc):
    """The paper's 11,880 plausible sets for four hidden tiles of one colour
    (12*11*10*9 ordered choices) are 4! orderings of each ascending row, so
    there are C(12, 4) = 495 worlds; the sampler reaches every one of them
    and the vanilla root only ever holds such worlds."""
    owner = [-1] * 24
    opp = [2, 8, 14, 20]                   # four black tiles, none revealed
    mine = [1, 5, 9, 13, 17]               # white tiles only
    for t in opp:
        owner[t] = 1
    for t in mine:
        owner[t] = 0
    pos = {"P": 2, "owner": owner, "revealed": set(), "mover": 0, "phase": 1, "drawn": 17}
    law = _sampler_law(pos)
    assert 12 * 11 * 10 * 9 == 11880 == 24 * len(law)
    assert set(law) == {tuple(c) for c in __import__("itertools").combinations(range(0, 24, 2), 4)}
    root = POS.pack(pos)
    mp = orc.mcts_params(iterations=600, playouts_per_leaf=1, max_depth=2, vanilla=1)
    _, t = orc.mcts_tree(root, mp, 3)
    worlds = t[t["parent"] == 0]
    keys = {int(k) for k in worlds["world"]}
    as_sets = {tuple(x for x in range(24) if (k >> (2 * x)) & 3) for k in keys}
    assert as_sets <= set(law)
    assert len(worlds) > 150               # dilution: most iterations open a new world


# ---------------------------------------------------------------------------
# leaf batching: B descents per pass, visits at once, wins after the pass
# ---------------------------------------------------------------------------
def _ucb1_batched_reference(orc, root, iters, ppl, seed, tree, B):
    """UCB1 over the root's guesses where arms are pulled in passes of B:
    within a pass every pull counts its visits at once (the later pulls of the
    pass see them, with no wins), the pass's leaves are then played out and
    their wins added in pull order."""
    legal = np.flatnonzero(orc.legal_actions(root))
    mover = orc.unpack(root)["mover"]
    arms, N, W = [], {}, {}
    n_root = 0
    for i0 in range(0, iters, B):
        pulls = []
        for i in range(i0, min(iters, i0 + B)):
            untried = [a for a in legal if a not in N]
            if untried:
                a = int(untried[0])
                arms.append(a)
                N[a], W[a] = 0, np.float32(0)
            else:
                lp = np.float32(math.log(n_root))
                best, best_s = None, None
                for c in arms:
                    n = np.float32(N[c])
                    s = W[c] / n + C_UCT * np.sqrt(lp / n)
                    if best is None or s > best_s:
                        best, best_s = c, s
                a = best
            N[a] += ppl
            n_root += ppl
            pulls.append((i, a))
        for i, a in pulls:
            world, _ = orc.determinize(root, seed, tree, i)
            leaf, term, win = orc.apply_action(world, a, seed, tree, i, 0)
            if term:
                wins = np.zeros(4, np.uint32)
                wins[win] = ppl
            else:
                _, _, w4 = orc.rollout(leaf, ppl, seed, tree_id=tree, leaf_id_base=i,
                                       want_winner=False, want_length=False)
                wins = w4[0]
            W[a] = np.float32(W[a] + np.float32(wins[mover]))
    best = max(arms, key=lambda a: (N[a], -arms.index(a)))
    return arms, N, W, best


@pytest.mark.parametrize("B", [2, 3, 4])
def test_leaf_batching_depth_one_is_batched_ucb1(orc, B):
    roots = orc.init_states(2, orc.deal_params(p_min=2, p_max=3, fresh=0, pile_min=0,
                                               pile_max=8, revealed_max=6, root_draw=1), 83)
    for case, root in enumerate(roots):
        iters, ppl, seed, tree = 203, 4, 92, case
        mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=1,
                             leaves_per_pass=B)
        best, kids = orc.mcts_search(root, mp, seed, tree_id_base=tree)
        arms, N, W, ref_best = _ucb1_batched_reference(orc, root, iters, ppl, seed, tree, B)
        k = kids[0][kids[0]["action"] != 0xFFFF]
        assert [int(a) for a in k["action"]] == arms
        assert [int(n) for n in k["n"]] == [N[a] for a in arms]
        assert [float(w) for w in k["w"]] == [float(W[a]) for a in arms]
        assert best[0] == ref_best
    # batching changes the search once selection starts
    kw = dict(iterations=600, playouts_per_leaf=4, max_depth=1)
    _, k1 = orc.mcts_search(roots[1], orc.mcts_params(**kw), 92, tree_id_base=1)
    _, kb = orc.mcts_search(roots[1], orc.mcts_params(leaves_per_pass=B, **kw), 92, tree_id_base=1)
    assert not (np.array_equal(k1[0]["n"], kb[0]["n"]) and np.array_equal(k1[0]["w"], kb[0]["w"]))


@pytest.mark.parametrize("cont,vanilla", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_leaf_batching_tree_identities(orc, cont, vanilla):
    """Whole trees with B = 4 (and a ragged last pass): every visit is counted
    once, the identities of a searched tree hold, and a pass's descents
    spread over different children."""
    for P in (2, 3):
        root = _mid_roots(orc, 1, 95 + P, P)[0]
        iters, ppl = 401, 4
        mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=0,
                             continue_choice=cont, vanilla=vanilla, leaves_per_pass=4)
        _, t = orc.mcts_tree(root, mp, 8)
        _check_tree(t, iters, ppl, cont)


def test_leaf_batching_first_pass_is_the_expansion_sweep(orc):
    """While the root still has untried guesses every descent expands the
    next one, whatever the batch: the first B iterations give the same root as
    B sequential iterations."""
    root = orc.init_states(1, orc.deal_params(p_min=3, p_max=3, fresh=1, root_draw=1), 99)[0]
    n_legal = int(orc.legal_actions(root).sum())
    B = 16
    assert n_legal >= B
    a = orc.mcts_search(root, orc.mcts_params(iterations=B, playouts_per_leaf=8,
                                              leaves_per_pass=B), 3, 4)
    b = orc.mcts_search(root, orc.mcts_params(iterations=B, playouts_per_leaf=8), 3, 4)
    assert a[0][0] == b[0][0] and np.array_equal(a[1], b[1])
