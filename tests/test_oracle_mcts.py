"""Pins of the oracle's tree search (CPU only).

* depth threshold 1 reduces the search to UCB1 (Auer, Cesa-Bianchi, Fischer
  2002) over the root moves, each pull being "sample a world, play the move,
  run the playouts"; a separate loop written here from the textbook rule
  must reproduce the oracle's visit counts, win sums and decision exactly;
* visit-count identities of the full search;
* a root whose only legal guess wins at once is chosen and scores W = N;
* the determinization sampler: every sampled world is consistent with what
  the searching player sees; with two players no attempt fails; the one-slot
  sampler is uniform over the consistent values.  Beyond that its
  distribution is parity unpinned (it is a heuristic sampler, not uniform
  over consistent worlds).
"""
import math

import numpy as np
import pytest

import positions as POS

C_UCT = np.float32(math.sqrt(2.0))


def _roots(orc, n, seed, p_min=2, p_max=2, fresh=1, **kw):
    dp = orc.deal_params(p_min=p_min, p_max=p_max, fresh=fresh, root_draw=1, **kw)
    return orc.init_states(n, dp, seed)


def _ucb1_reference(orc, root, iters, ppl, seed, tree):
    """Textbook UCB1 over the root's legal guesses; one arm pull per iteration."""
    legal = np.flatnonzero(orc.legal_actions(root))
    mover = orc.unpack(root)["mover"]
    arms = []          # arms in the order they were first pulled
    N, W = {}, {}
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
        leaf, term, win = orc.apply_action(world, a, seed, tree, i, 0)
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


@pytest.mark.parametrize("case", range(4))
def test_depth_one_is_ucb1(orc, case):
    roots = _roots(orc, 4, seed=40 + case, p_min=2, p_max=3)
    root = roots[case]
    iters, ppl, seed, tree = 300, 4, 77, case
    mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=1)
    best, kids = orc.mcts_search(root, mp, seed, tree_id_base=tree)
    arms, N, W, ref_best = _ucb1_reference(orc, root, iters, ppl, seed, tree)
    k = kids[0][kids[0]["action"] != 0xFFFF]
    assert [int(a) for a in k["action"]] == arms
    assert [int(n) for n in k["n"]] == [N[a] for a in arms]
    assert [float(w) for w in k["w"]] == [float(W[a]) for a in arms]
    assert best[0] == ref_best


@pytest.mark.parametrize("P", [2, 3, 4])
def test_visit_count_identities(orc, P):
    roots = _roots(orc, 3, seed=50 + P, p_min=P, p_max=P, fresh=0, pile_min=2, pile_max=12,
                   revealed_max=3)
    iters, ppl = 400, 8
    mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=4)
    best, kids = orc.mcts_search(roots, mp, 5)
    for t in range(3):
        k = kids[t][kids[t]["action"] != 0xFFFF]
        legal = orc.legal_actions(roots[t])
        # every iteration passes through exactly one root child
        assert int(k["n"].sum()) == iters * ppl
        assert np.all(k["n"] % ppl == 0) and np.all(k["n"] >= ppl)
        assert np.all(k["w"] <= k["n"]) and np.all(k["w"] >= 0)
        assert np.all(k["w"] == np.round(k["w"]))
        # children are distinct legal root actions, created lowest id first
        acts = [int(a) for a in k["action"]]
        assert len(set(acts)) == len(acts)
        assert all(legal[a] for a in acts)
        first_sweep = sorted(np.flatnonzero(legal).tolist())
        assert acts[:len(first_sweep)] == first_sweep
        # the decision is the most visited child, earliest on ties
        nmax = k["n"].max()
        assert best[t] == acts[int(np.flatnonzero(k["n"] == nmax)[0])]


def test_forced_win_root(orc):
    # opponent keeps one hidden tile with a single consistent value: the only
    # legal guess ends the game, every iteration wins
    pos = POS.two_player_last_tiles(1)
    root = POS.pack(pos)
    legal = np.flatnonzero(orc.legal_actions(root))
    assert len(legal) == 1
    mp = orc.mcts_params(iterations=50, playouts_per_leaf=16, max_depth=4)
    best, kids = orc.mcts_search(root, mp, 3)
    k = kids[0][kids[0]["action"] != 0xFFFF]
    assert best[0] == legal[0]
    assert len(k) == 1 and k["n"][0] == 50 * 16 and k["w"][0] == 50 * 16


def _consistent(orc, root, world):
    r, w = orc.unpack(root), orc.unpack(world)
    M = r["mover"]
    assert w["P"] == r["P"] and w["mover"] == M and w["phase"] == r["phase"]
    assert w["drawn"] == r["drawn"]
    assert w["rows"][M] == r["rows"][M] and w["rev"][M] == r["rev"][M]
    for q in range(r["P"]):
        assert len(w["rows"][q]) == len(r["rows"][q])
        assert w["rev"][q] == r["rev"][q]
        for j, t in enumerate(r["rows"][q]):
            tw = w["rows"][q][j]
            assert tw % 2 == t % 2, "colour of a slot changed"
            if r["rev"][q][j]:
                assert tw == t, "revealed tile changed"
    assert orc.validate(world) == 0


@pytest.mark.parametrize("P", [2, 3, 4])
def test_determinization_consistent(orc, P):
    dp = orc.deal_params(p_min=P, p_max=P, pile_min=0, pile_max=12, revealed_max=6, root_draw=1)
    roots = orc.init_states(150, dp, seed=60 + P)
    attempts = []
    for t, root in enumerate(roots):
        for i in range(6):
            world, a = orc.determinize(root, 9, t, i)
            _consistent(orc, root, world)
            attempts.append(a)
    if P == 2:
        assert max(attempts) == 0, "one opponent: the sampler cannot fail"


def test_determinization_one_slot_uniform(orc):
    # the last-tile duel: the single hidden opponent slot has k consistent
    # values; the sampler must pick each with probability 1/k
    from scipy import stats
    k = 6
    root = POS.pack(POS.two_player_last_tiles(k))
    counts = {}
    for i in range(6000):
        world, a = orc.determinize(root, 4, 0, i)
        t = orc.unpack(world)["rows"][1][-1]
        counts[t] = counts.get(t, 0) + 1
    assert len(counts) == k
    assert stats.chisquare(list(counts.values())).pvalue > 1e-4


def test_determinization_fallback_is_smallest_world(orc):
    # many opponents with long hidden runs and no pool make the sampler fail
    # sometimes; the fallback world must still be consistent
    dp = orc.deal_params(p_min=4, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=0,
                         revealed_max=0, root_draw=1)
    roots = orc.init_states(300, dp, seed=70)
    used = 0
    for t, root in enumerate(roots):
        for i in range(20):
            world, a = orc.determinize(root, 1, t, i)
            _consistent(orc, root, world)
            if a == 64:
                used += 1
    print("fallback used", used, "of", 300 * 20)


def test_ln_table_matches_libm(orc):
    for k in [1, 2, 3, 10, 1000, 32000, 262143, 262144]:
        assert orc.ln_entry(k) == np.float32(math.log(k))


# ---------------------------------------------------------------------------
# root-parallel search: K trees per root amalgamated into one root (Sec. III-B)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("K", [1, 3])
def test_merged_search_sums_independent_trees(orc, K):
    """The amalgamated root is the per-action sum of K independent trees whose
    tree ids are base + r*K + k; the decision is its most visited action,
    lowest action id on ties; every merged visit count adds up to K*iters*ppl."""
    roots = _roots(orc, 3, seed=41, p_min=2, p_max=4, fresh=0, hand=(0, 0, 4, 4, 3),
                   pile_min=0, pile_max=12, revealed_max=4)
    iters, ppl, base = 60, 4, 10
    mp = orc.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=3)
    best, merged = orc.mcts_search_merged(roots, K, mp, seed=8, tree_id_base=base)
    for r in range(3):
        n = np.zeros(864, np.int64)
        w = np.zeros(864, np.float64)
        for k in range(K):
            _, kids = orc.mcts_search(roots[r:r + 1], mp, 8, base + r * K + k)
            for c in kids[0]:
                if c["action"] == 0xFFFF:
                    break
                n[c["action"]] += int(c["n"])
                w[c["action"]] += float(c["w"])
        m = merged[r]
        assert np.array_equal(m["n"].astype(np.int64), n)
        # rollout-mode win sums are integers, so float sums are exact
        assert np.array_equal(m["w"].astype(np.float64), w)
        created = n > 0
        assert np.array_equal(m["action"] != 0xFFFF, created)
        assert np.array_equal(np.flatnonzero(created), m["action"][created].astype(np.int64))
        assert n.sum() == K * iters * ppl
        assert best[r] == int(np.flatnonzero(n == n.max())[0])


def test_merged_search_one_tree_matches_single_search(orc):
    roots = _roots(orc, 4, seed=43)
    mp = orc.mcts_params(iterations=200, playouts_per_leaf=8, max_depth=4)
    best_m, merged = orc.mcts_search_merged(roots, 1, mp, seed=2, tree_id_base=5)
    best_s, kids = orc.mcts_search(roots, mp, 2, 5)
    for r in range(4):
        live = kids[r][kids[r]["action"] != 0xFFFF]
        m = merged[r][live["action"].astype(np.int64)]
        assert np.array_equal(m["n"], live["n"]) and np.array_equal(m["w"], live["w"])
        top = live["n"].max()
        if np.sum(live["n"] == top) == 1:
            assert best_m[r] == best_s[r]


def _sampler_law(pos):
    """Exact law of the world sampler for one opponent, enumerated from its
    stated procedure: per run of hidden opponent slots between revealed tiles
    (lo, hi), in row order, the bounds right to left (largest available tile
    of the slot's colour below the next bound), then values left to right,
    uniform over the available tiles of the slot's colour in (previous value,
    bound]; available = neither in the mover's row nor revealed nor taken."""
    from fractions import Fraction
    m = pos["mover"]
    opp = 1 - m
    rev = set(pos["revealed"])
    avail0 = {t for t in range(24) if pos["owner"][t] != m and t not in rev}
    row = sorted(t for t in range(24) if pos["owner"][t] == opp)
    segs, cur, lo = [], [], -1
    for t in row:
        if t in rev:
            if cur:
                segs.append((lo, t, cur))
            cur, lo = [], t
        else:
            cur.append(t)
    if cur:
        segs.append((lo, 24, cur))
    law = {}

    def rec(si, avail, chosen, p):
        if si == len(segs):
            law[tuple(sorted(chosen))] = law.get(tuple(sorted(chosen)), 0) + p
            return
        lo, hi, slots = segs[si]
        bounds, b = [], hi
        for t in reversed(slots):
            c = [u for u in avail if u % 2 == t % 2 and u < b]
            b = max(c)
            bounds.append(b)
        bounds.reverse()
        assert bounds[0] > lo

        def fill(j, avail, prev, chosen, p):
            if j == len(slots):
                rec(si + 1, avail, chosen, p)
                return
            c = sorted(u for u in avail if u % 2 == slots[j] % 2 and prev < u <= bounds[j])
            for u in c:
                fill(j + 1, avail - {u}, u, chosen + [u], p / len(c))

        fill(0, avail, lo, chosen, p)

    rec(0, avail0, [], Fraction(1))
    return law


def test_determinization_matches_its_exact_law(orc):
    """Two runs of hidden opponent slots (one and two slots) in a two-player
    position: the frequencies of the sampled worlds over 30,000 iterations match
    the sampler's exact law, enumerated from its procedure (chi-square)."""
    from scipy import stats
    owner = [-1] * 24
    opp_row = [2, 7, 10, 15, 20]
    mover_row = [0, 5, 12, 13, 19, 22]
    for t in opp_row:
        owner[t] = 1
    for t in mover_row:
        owner[t] = 0
    pos = {"P": 2, "owner": owner, "revealed": {7, 20, 5}, "mover": 0, "phase": 1,
           "drawn": 22}
    root = POS.pack(pos)
    law = _sampler_law(pos)
    assert abs(sum(law.values()) - 1) == 0 and len(law) > 10
    counts = {}
    n = 30000
    for i in range(n):
        world, a = orc.determinize(root, 9, 3, i)
        assert a == 0
        w = POS.unpack(world)
        hidden = tuple(sorted(t for t in range(24) if w["owner"][t] == 1 and t not in w["revealed"]))
        counts[hidden] = counts.get(hidden, 0) + 1
    assert set(counts) <= set(law)
    keys = sorted(law)
    f_obs = [counts.get(k, 0) for k in keys]
    f_exp = [float(law[k]) * n for k in keys]
    assert stats.chisquare(f_obs, f_exp).pvalue > 1e-4
