"""Seeded synthetic positions for tests, in the packed 16-byte format.

Input generation only: nothing here implements the rules of a playout or the
search.  Positions are described as plain dicts
  {"P", "owner": 24 ints (-1 pool, else seat), "revealed": set, "mover",
   "phase", "drawn"}
and packed independently of the oracle and of the HIP library.
"""
from __future__ import annotations

import numpy as np


def pack(pos: dict) -> np.ndarray:
    w = [0, 0, 0, 0]
    for t, o in enumerate(pos["owner"]):
        code = 0 if o < 0 else o + 1
        for k in range(3):
            if (code >> k) & 1:
                w[k] |= 1 << t
    for t in pos["revealed"]:
        w[3] |= 1 << t
    w[0] |= (pos["mover"] & 3) << 24
    w[0] |= ((pos["P"] - 1) & 3) << 26
    w[0] |= (pos["phase"] & 1) << 28
    if pos["drawn"] is not None:
        w[0] |= 1 << 29
        w[1] |= (pos["drawn"] & 31) << 24
    return np.array(w, dtype=np.uint32)


def unpack(w) -> dict:
    w = [int(x) for x in w]
    owner = []
    for t in range(24):
        code = ((w[0] >> t) & 1) | (((w[1] >> t) & 1) << 1) | (((w[2] >> t) & 1) << 2)
        owner.append(code - 1)
    return {"P": ((w[0] >> 26) & 3) + 1, "owner": owner,
            "revealed": {t for t in range(24) if (w[3] >> t) & 1},
            "mover": (w[0] >> 24) & 3, "phase": (w[0] >> 28) & 1,
            "drawn": ((w[1] >> 24) & 31) if (w[0] >> 29) & 1 else None}


def tiny_endgame(rng: np.random.Generator, P: int, hidden_per_seat=(1, 2), pool=(0, 2),
                 phase1=False) -> dict:
    """A position where almost every tile is revealed: each player keeps 1-2
    hidden tiles and the pool holds 0-2 tiles, so exact enumeration is cheap."""
    while True:
        perm = rng.permutation(24)
        npool = int(rng.integers(pool[0], pool[1] + 1))
        owner = [-1] * 24
        rest = perm[npool:]
        # deal the rest round-robin-ish with random sizes >= 2
        sizes = [2] * P
        for _ in range(len(rest) - 2 * P):
            sizes[int(rng.integers(0, P))] += 1
        pos = 0
        rows = []
        for q in range(P):
            row = sorted(int(x) for x in rest[pos:pos + sizes[q]])
            pos += sizes[q]
            rows.append(row)
            for t in row:
                owner[t] = q
        revealed = set()
        for q in range(P):
            h = int(rng.integers(hidden_per_seat[0], hidden_per_seat[1] + 1))
            h = min(h, len(rows[q]))
            hid = set(int(x) for x in rng.choice(rows[q], size=h, replace=False))
            revealed |= set(rows[q]) - hid
        mover = int(rng.integers(0, P))
        d = {"P": P, "owner": owner, "revealed": revealed, "mover": mover, "phase": 0,
             "drawn": None}
        if phase1:
            hid_m = [t for t in rows[mover] if t not in revealed]
            d["phase"] = 1
            if npool == 0 and len(hid_m) >= 2:
                d["drawn"] = None
            elif len(hid_m) >= 2:
                d["drawn"] = int(rng.choice(hid_m))
            else:
                continue
        return d


def two_player_last_tiles(k: int) -> dict:
    """Two players, each with exactly one hidden tile; the mover has already
    passed its draw without drawing (phase 1, nothing drawn) and the
    opponent's hidden tile (black 11, id 22) has exactly k consistent values
    for the mover: itself and k-1 black pool tiles just below it.  A right
    guess ends the game for the mover, a wrong one reveals the mover's last
    hidden tile, so the mover wins with probability exactly 1/k."""
    assert 1 <= k <= 12
    owner = [-1] * 24
    revealed = set()
    target = 22
    decoys = [target - 2 * j for j in range(1, k)]
    low_blacks = [t for t in range(0, target, 2) if t not in decoys]
    owner[target] = 1
    for t in low_blacks:                 # opponent row: low blacks revealed, 22 hidden
        owner[t] = 1
        revealed.add(t)
    for t in range(1, 24, 2):            # mover row: all whites, only id 1 hidden
        owner[t] = 0
        if t != 1:
            revealed.add(t)
    # decoys stay in the pool (owner -1)
    return {"P": 2, "owner": owner, "revealed": revealed, "mover": 0, "phase": 1,
            "drawn": None}
