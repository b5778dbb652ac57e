"""Pins of the oracle's game rules and state generator (CPU only).

* codec: the oracle's unpacker agrees with an independent packer;
* invariants after every guess of many playouts (tile conservation, rows in
  ascending order, one new reveal per guess, reveals never undone, the drawn
  tile stays hidden until a wrong guess), exactly one winner, termination
  within 23 - R0 guesses, game length = tiles revealed;
* closed form: a last-tile duel won with probability exactly 1/k;
* exact enumeration (tests/bruteforce.py, written separately) of tiny
  endgames vs the oracle's Monte Carlo at 5 sigma;
* generator: validity, hand sizes, reveal counts, mover, draws, uniformity.
"""
import math

import numpy as np
import pytest

import bruteforce as BF  # noqa: E402
import positions as POS


def _check_rows(d, pos0_revealed_count, k):
    seen = []
    for q in range(d["P"]):
        row = d["rows"][q]
        assert row == sorted(row) and len(set(row)) == len(row), "row not ascending"
        seen += row
    seen += d["pile"]
    assert sorted(seen) == list(range(24)), "tile conservation"
    assert d["pile"] == sorted(d["pile"])
    nrev = sum(sum(r) for r in d["rev"])
    assert nrev == pos0_revealed_count + k, "exactly one reveal per guess"
    if d["drawn"] >= 0:
        m = d["mover"]
        assert d["drawn"] in d["rows"][m]
    return nrev


@pytest.mark.parametrize("P", [2, 3, 4])
def test_invariants_after_every_guess(orc, P):
    dp = orc.deal_params(p_min=P, p_max=P, pile_min=0, pile_max=16, revealed_max=8,
                         phase_mix=1)
    states = orc.init_states(200, dp, seed=11 + P)
    for i, s in enumerate(states):
        d0 = orc.unpack(s)
        r0 = sum(sum(r) for r in d0["rev"])
        for p in range(8):
            winner, length, trace = orc.playout(s, 99, p, i, 0, trace=True)
            assert len(trace) == length
            assert 1 <= length <= 23 - r0, "termination bound"
            prev_rev = {(q, t) for q in range(P) for j, t in enumerate(d0["rows"][q]) if d0["rev"][q][j]}
            prev_pile = set(d0["pile"])
            for k, d in enumerate(trace):
                _check_rows(d, r0, k + 1)
                rev = {(q, t) for q in range(P) for j, t in enumerate(d["rows"][q]) if d["rev"][q][j]}
                assert prev_rev <= rev, "a revealed tile was hidden again"
                assert set(d["pile"]) <= prev_pile, "pile grew"
                prev_rev, prev_pile = rev, set(d["pile"])
            last = trace[-1]
            alive = [q for q in range(P) if not all(last["rev"][q])]
            assert alive == [winner], "exactly one player left and it is the winner"


def test_drawn_tile_hidden_until_wrong_guess(orc):
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=4, pile_max=16, revealed_max=3)
    states = orc.init_states(100, dp, seed=5)
    def revealed(d):
        return {t for q in range(d["P"]) for j, t in enumerate(d["rows"][q]) if d["rev"][q][j]}

    for i, s in enumerate(states):
        _, _, trace = orc.playout(s, 3, 0, i, 0, trace=True)
        prev = revealed(orc.unpack(s))
        for d in trace:
            now = revealed(d)
            if d["drawn"] >= 0 and d["drawn"] in now:
                # only the guess that just failed may reveal the drawn tile
                assert now - prev == {d["drawn"]}
            prev = now


def test_codec_matches_independent_packer(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        P = int(rng.integers(2, 5))
        pos = POS.tiny_endgame(rng, P, hidden_per_seat=(1, 3), pool=(0, 6), phase1=bool(rng.integers(0, 2)))
        w = POS.pack(pos)
        d = orc.unpack(w)
        for q in range(P):
            assert d["rows"][q] == sorted(t for t in range(24) if pos["owner"][t] == q)
            assert d["rev"][q] == [int(t in pos["revealed"]) for t in d["rows"][q]]
        assert d["pile"] == [t for t in range(24) if pos["owner"][t] == -1]
        assert d["mover"] == pos["mover"] and d["phase"] == pos["phase"]
        assert d["drawn"] == (-1 if pos["drawn"] is None else pos["drawn"])
        assert np.array_equal(orc.pack(d), w)


def test_validate_rejects_malformed(orc):
    rng = np.random.default_rng(4)
    pos = POS.tiny_endgame(rng, 3, phase1=True)
    good = POS.pack(pos)
    assert orc.validate(good) == 0
    bad = good.copy(); bad[2] |= 1 << 30                      # stray high bit
    assert orc.validate(bad) != 0
    bad = good.copy(); bad[0] = int(bad[0]) & ~(3 << 26) & 0xFFFFFFFF   # one player
    assert orc.validate(bad) != 0
    # a pool tile marked revealed
    pool = [t for t in range(24) if pos["owner"][t] == -1]
    if pool:
        bad = good.copy(); bad[3] |= 1 << pool[0]
        assert orc.validate(bad) != 0
    # mover without hidden tiles
    p2 = dict(pos)
    m = pos["mover"]
    p2["revealed"] = set(pos["revealed"]) | {t for t in range(24) if pos["owner"][t] == m}
    p2["drawn"] = None
    assert orc.validate(POS.pack(p2)) != 0
    # tile owned by a seat >= P
    p3 = dict(pos); o = list(pos["owner"]); o[o.index(0)] = 3; p3["owner"] = o
    assert orc.validate(POS.pack(p3)) != 0


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 12])
def test_closed_form_last_tile_duel(orc, k):
    pos = POS.two_player_last_tiles(k)
    law = BF.outcome_law(pos)
    assert BF.win_probs(law, 2)[0] == BF.Fraction(1, k)
    n = 200_000
    winner, length, wins = orc.rollout(POS.pack(pos), n, seed=17, leaf_id_base=k)
    p_hat = wins[0, 0] / n
    sigma = math.sqrt((1 / k) * (1 - 1 / k) / n) + 1e-12
    assert abs(p_hat - 1 / k) <= 5 * sigma + 1e-9
    assert np.all(length == 1)


def _compare_law(orc, pos, n, seed, leaf):
    law = BF.outcome_law(pos)
    P = pos["P"]
    winner, length, wins = orc.rollout(POS.pack(pos), n, seed=seed, leaf_id_base=leaf)
    exact = BF.win_probs(law, P)
    for q in range(P):
        p = float(exact[q])
        sig = math.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(wins[0, q] / n - p) <= 5 * sig + 1e-9, (q, wins[0] / n, [float(x) for x in exact])
    # every (winner, length) cell
    for (w, L), pr in law.items():
        p = float(pr)
        obs = np.count_nonzero((winner == w) & (length == L)) / n
        sig = math.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(obs - p) <= 5 * sig + 1e-9, ((w, L), obs, p)
    # nothing outside the support
    support = set(law.keys())
    pairs = set(zip(winner.tolist(), length.tolist()))
    assert pairs <= support
    mean = float(BF.mean_length(law))
    assert abs(length.mean() - mean) <= 5 * length.std() / math.sqrt(n) + 1e-9


@pytest.mark.parametrize("case", range(10))
def test_exact_enumeration_two_players(orc, case):
    rng = np.random.default_rng(100 + case)
    pos = POS.tiny_endgame(rng, 2, hidden_per_seat=(1, 3), pool=(0, 2), phase1=bool(case % 2))
    _compare_law(orc, pos, 100_000, seed=1000 + case, leaf=case)


@pytest.mark.parametrize("case", range(6))
def test_exact_enumeration_three_players(orc, case):
    rng = np.random.default_rng(200 + case)
    pos = POS.tiny_endgame(rng, 3, hidden_per_seat=(1, 2), pool=(0, 1), phase1=bool(case % 2))
    _compare_law(orc, pos, 100_000, seed=2000 + case, leaf=case)


def test_exact_enumeration_four_players(orc):
    rng = np.random.default_rng(300)
    pos = POS.tiny_endgame(rng, 4, hidden_per_seat=(1, 1), pool=(0, 1))
    _compare_law(orc, pos, 100_000, seed=3000, leaf=0)


def test_terminal_leaf_has_zero_length(orc):
    rng = np.random.default_rng(9)
    pos = POS.tiny_endgame(rng, 2, hidden_per_seat=(1, 1), pool=(0, 0))
    # reveal the non-mover's last hidden tile: the mover is the only one left
    o = 1 - pos["mover"]
    pos["revealed"] = set(pos["revealed"]) | {t for t in range(24) if pos["owner"][t] == o}
    w, L, _ = orc.rollout(POS.pack(pos), 10, seed=1)
    assert np.all(w == pos["mover"]) and np.all(L == 0)


# ---------------------------------------------------------------------------
# generator
# ---------------------------------------------------------------------------
def test_generator_structure(orc):
    dp = orc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                         revealed_max=8)
    S = orc.init_states(3000, dp, seed=2)
    Ps = []
    for s in S:
        assert orc.validate(s) == 0
        d = orc.unpack(s)
        P = d["P"]
        Ps.append(P)
        h0 = {2: 4, 3: 4, 4: 3}[P]
        pile = len(d["pile"])
        assert 0 <= pile <= min(16, 24 - P * h0)
        drawn = 24 - P * h0 - pile
        for q in range(P):
            assert len(d["rows"][q]) == h0 + drawn // P + (1 if q < drawn % P else 0)
            assert sum(d["rev"][q]) <= min(8, len(d["rows"][q]) - 1)
        assert d["mover"] == drawn % P and d["phase"] == 0 and d["drawn"] == -1
    counts = np.bincount(Ps, minlength=5)[2:]
    assert counts.min() > 850


def test_generator_uniformity(orc):
    # c[1]-style states: pile size uniform on 0..16, owner of each tile
    # uniform given the pile size (chi-square, generous thresholds)
    from scipy import stats
    dp = orc.deal_params(p_min=2, p_max=2, pile_min=0, pile_max=16, revealed_max=8)
    S = orc.init_states(17_000, dp, seed=21)
    piles = np.array([len(orc.unpack(s)["pile"]) for s in S[:4000]])
    obs = np.bincount(piles, minlength=17)
    assert stats.chisquare(obs).pvalue > 1e-4
    # with a fresh deal every tile lands in the pool with probability 16/24
    dp2 = orc.deal_params(p_min=2, p_max=2, fresh=1)
    F = orc.init_states(6000, dp2, seed=22)
    in_pool = np.zeros(24)
    seat0 = np.zeros(24)
    for s in F:
        w = [int(x) for x in s]
        owner = [(((w[0] >> t) & 1) | (((w[1] >> t) & 1) << 1)) for t in range(24)]
        for t in range(24):
            in_pool[t] += owner[t] == 0
            seat0[t] += owner[t] == 1
    p = 16 / 24
    z = (in_pool - 6000 * p) / math.sqrt(6000 * p * (1 - p))
    assert np.abs(z).max() < 5
    p0 = 4 / 24
    z0 = (seat0 - 6000 * p0) / math.sqrt(6000 * p0 * (1 - p0))
    assert np.abs(z0).max() < 5


def test_generator_root_draw_and_fresh(orc):
    dp = orc.deal_params(p_min=2, p_max=4, fresh=1, root_draw=1)
    S = orc.init_states(500, dp, seed=5)
    for s in S:
        d = orc.unpack(s)
        P = d["P"]
        h0 = {2: 4, 3: 4, 4: 3}[P]
        assert sum(map(sum, d["rev"])) == 0
        assert d["phase"] == 1 and d["mover"] == 0
        assert d["drawn"] in d["rows"][0] and len(d["rows"][0]) == h0 + 1
        assert len(d["pile"]) == 24 - P * h0 - 1


def test_generator_index_base_is_an_offset(orc):
    dp = orc.deal_params(p_min=2, p_max=4, phase_mix=1)
    a = orc.init_states(64, dp, seed=8)
    b = orc.init_states(32, dp, seed=8, index_base=32)
    assert np.array_equal(a[32:], b)
