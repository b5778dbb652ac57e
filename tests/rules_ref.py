"""The tree's moves restated from the game rules, independently of the oracle.

Written from the rules (Sec. II-A) and the simplified tree (Sec. III-A), on
the plain position dicts of ``positions.py`` (owner per tile, revealed set,
mover, phase, drawn tile), with no code from the oracle:

* a guess names a seat to the mover's left at distance r (1..P-1), a slot
  of that seat's row (ascending, 0 = lowest) and a value; the colour is the
  slot's, which everybody sees.  It is a candidate when the seat still has a
  hidden tile, the slot is hidden, and the guessed tile lies strictly
  between the revealed tiles nearest to the slot in that row, is not in the
  mover's own row and is not revealed anywhere (the mover cannot hold or see
  it, so it might be the slot's tile);
* inside the tree a guess ends the turn: a right guess reveals the target;
  a wrong one reveals the tile the mover drew this turn, or, when it drew
  none (empty pool), one of its own hidden tiles picked by word 0 of the
  chance block; a player without hidden tiles is out and the last one left
  wins; otherwise the next seat still in draws a pool tile picked by word 1
  (when the pool is not empty) and is to move, having drawn.

Random words come from the Philox block (depth, 0xC0000000, iteration,
tree) of the search's seed; a pick among k from word w is floor(w k / 2^32).
"""
from __future__ import annotations

import copy

CHANCE_DOMAIN = 0xC0000000


def row(pos: dict, seat: int) -> list:
    return sorted(t for t in range(24) if pos["owner"][t] == seat)


def hidden(pos: dict, seat: int) -> list:
    return [t for t in row(pos, seat) if t not in pos["revealed"]]


def seats_in(pos: dict) -> list:
    return [s for s in range(pos["P"]) if hidden(pos, s)]


def pick(w: int, k: int) -> int:
    return (int(w) * k) >> 32


def action_id(r: int, slot: int, value: int) -> int:
    return ((r - 1) * 24 + slot) * 12 + value


def decode_action(a: int):
    return a // 288 + 1, (a // 12) % 24, a % 12


def candidates(pos: dict) -> set:
    """Every candidate guess of the mover, as action ids."""
    m, P = pos["mover"], pos["P"]
    mine = set(row(pos, m))
    out = set()
    for r in range(1, P):
        seat = (m + r) % P
        if not hidden(pos, seat):
            continue
        tiles = row(pos, seat)
        for slot, t in enumerate(tiles):
            if t in pos["revealed"]:
                continue
            below = [x for x in tiles[:slot] if x in pos["revealed"]]
            above = [x for x in tiles[slot + 1:] if x in pos["revealed"]]
            lo = below[-1] if below else -1
            hi = above[0] if above else 24
            for value in range(12):
                g = 2 * value + (t & 1)
                if lo < g < hi and g not in mine and g not in pos["revealed"]:
                    out.add(action_id(r, slot, value))
    return out


def next_in(pos: dict, m: int) -> int:
    P = pos["P"]
    for k in range(1, P + 1):
        s = (m + k) % P
        if hidden(pos, s):
            return s
    raise AssertionError("nobody left")


def play(pos: dict, a: int, words) -> tuple:
    """Play guess `a` in the tree with chance words `words` (4 ints).
    Returns (new position, game over, winner or -1)."""
    out = copy.deepcopy(pos)
    out["revealed"] = set(pos["revealed"])
    m, P = pos["mover"], pos["P"]
    r, slot, value = decode_action(a)
    seat = (m + r) % P
    t = row(pos, seat)[slot]
    if 2 * value + (t & 1) == t:
        out["revealed"].add(t)
    elif pos["drawn"] is not None:
        out["revealed"].add(pos["drawn"])
    else:
        own = hidden(pos, m)
        out["revealed"].add(own[pick(words[0], len(own))])
    left = seats_in(out)
    if len(left) == 1:
        out["phase"], out["drawn"] = 1, None
        return out, True, left[0]
    nm = next_in(out, m)
    out["mover"], out["phase"], out["drawn"] = nm, 1, None
    pool = [x for x in range(24) if out["owner"][x] == -1]
    if pool:
        d = pool[pick(words[1], len(pool))]
        out["owner"][d] = nm
        out["drawn"] = d
    return out, False, -1
