"""Exact outcome distribution of the random-policy Da Vinci Code playout.

Written independently of the oracle: it walks every chance branch of a
position with exact rational probabilities (fractions.Fraction) and returns
the joint law of (winner, number of guesses).  Usable on tiny endgames only
(a handful of hidden tiles), where the branching stays small.

The random policy (Sec. II-A rules, Sec. II-B "decisions at random"):
  * turn start: the mover draws a uniformly random pool tile (if any);
  * the guess targets a uniformly random hidden tile among all other
    players' hidden tiles, pooled;
  * the guessed value is uniform over the tile ids of the target's colour
    that lie strictly between the nearest revealed tiles around the target
    in its row and are neither in the mover's row nor revealed;
  * right guess: the target is revealed; the mover goes on guessing with
    probability 1/2, else the turn ends;
  * wrong guess: the drawn tile is revealed, or, if nothing was drawn, a
    uniformly random hidden tile of the mover's row; the turn ends;
  * a player with no hidden tile is out; turns pass to the next player in
    seat order that is still in; the last player in wins.

Positions are plain dicts: {"P", "owner": list of 24 (-1 = pool),
"revealed": set of tile ids, "mover", "phase" (1 = has drawn), "drawn"}.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache


def _key(pos: dict):
    return (pos["P"], tuple(pos["owner"]), frozenset(pos["revealed"]), pos["mover"],
            pos["phase"], pos["drawn"])


def _hidden(owner, revealed, seat):
    return [t for t in range(24) if owner[t] == seat and t not in revealed]


def _alive(P, owner, revealed):
    return [q for q in range(P) if _hidden(owner, revealed, q)]


def _add(acc, dist, w):
    for k, v in dist.items():
        acc[k] = acc.get(k, 0) + w * v


@lru_cache(maxsize=None)
def _solve(P, owner, revealed, mover, phase, drawn):
    """Law of (winner, guesses still to come) from this position."""
    alive = _alive(P, owner, revealed)
    if len(alive) == 1:
        return {(alive[0], 0): Fraction(1)}
    if phase == 0:
        pool = [t for t in range(24) if owner[t] == -1]
        if not pool:
            return _solve(P, owner, revealed, mover, 1, None)
        acc = {}
        for d in pool:
            o2 = list(owner)
            o2[d] = mover
            _add(acc, _solve(P, tuple(o2), revealed, mover, 1, d), Fraction(1, len(pool)))
        return acc
    targets = [t for t in range(24) if owner[t] not in (-1, mover) and t not in revealed]
    acc = {}
    for t in targets:
        o = owner[t]
        row = sorted(x for x in range(24) if owner[x] == o)
        lo = max([x for x in row if x < t and x in revealed], default=-1)
        hi = min([x for x in row if x > t and x in revealed], default=24)
        cands = [x for x in range(lo + 1, hi) if x % 2 == t % 2 and owner[x] != mover
                 and x not in revealed]
        w_t = Fraction(1, len(targets))
        for v in cands:
            w = w_t * Fraction(1, len(cands))
            if v == t:
                rev2 = revealed | {t}
                if len(_alive(P, owner, rev2)) == 1:
                    sub = {(mover, 0): Fraction(1)}
                else:
                    sub = {}
                    _add(sub, _solve(P, owner, rev2, mover, 1, drawn), Fraction(1, 2))
                    nxt = _next(P, owner, rev2, mover)
                    _add(sub, _solve(P, owner, rev2, nxt, 0, None), Fraction(1, 2))
            else:
                if drawn is not None:
                    options = [drawn]
                else:
                    options = _hidden(owner, revealed, mover)
                sub = {}
                for r in options:
                    rev2 = revealed | {r}
                    al = _alive(P, owner, rev2)
                    if len(al) == 1:
                        res = {(al[0], 0): Fraction(1)}
                    else:
                        res = _solve(P, owner, rev2, _next(P, owner, rev2, mover), 0, None)
                    _add(sub, res, Fraction(1, len(options)))
            shifted = {(k[0], k[1] + 1): p for k, p in sub.items()}
            _add(acc, shifted, w)
    return acc


def _next(P, owner, revealed, m):
    for k in range(1, P + 1):
        q = (m + k) % P
        if _hidden(owner, revealed, q):
            return q
    raise AssertionError("no player left")


def outcome_law(pos: dict) -> dict:
    """{(winner, length): Fraction} for one playout from ``pos``."""
    return _solve(pos["P"], tuple(pos["owner"]), frozenset(pos["revealed"]), pos["mover"],
                  pos["phase"], pos["drawn"])


def win_probs(law: dict, P: int):
    out = [Fraction(0)] * P
    for (w, _), p in law.items():
        out[w] += p
    return out


def mean_length(law: dict) -> Fraction:
    return sum(p * k[1] for k, p in law.items())
