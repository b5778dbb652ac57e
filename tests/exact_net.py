"""A value network whose every output is exact in any summation order.

Test input, not a trained evaluator.  With 0/1 features, weights of +-1 and
+-256 and zero biases, every pre-activation is a small integer, so the
float32 sums of the matrix cores and the double sums of the oracle agree
exactly whatever their order, every bfloat16 rounding is the identity, and
the sigmoid sees z in {-256 k, 0, +256 k}: its result is exactly 0, 1/2 or 1
in float and in double.  A value-mode search that uses this network must
therefore match the oracle bit for bit at any depth and fallback band; what
is left to compare is the search's own rule (which seat's value a node
receives, when a leaf falls back to playouts), not rounding.

The network computes, for perspective seat q of a P-player state,
    v_q = step(hidden(q) - hidden((q + 1) mod P))
with hidden(s) the number of hidden tiles in seat s's row and step(x) = 1,
1/2, 0 for x > 0, = 0, < 0.  ``closed_form`` states that rule directly.

Features (the interface's encoding): index 6 t + k for tile t, k = 0..3 the
tile's owner relative to q as a one-hot, k = 4 revealed, k = 5 in the pool;
148..159 padding.  Flat parameter order: W1 [256][160] (row = output), b1,
W2 [256][256], b2, w3 [256], b3.
"""
from __future__ import annotations

import numpy as np

NPARAM = 107265
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 40960, 41216, 106752, 107008, 107264
Z_SCALE = 256.0


def params() -> np.ndarray:
    p = np.zeros(NPARAM, np.float32)
    W1 = p[OFF_W1:OFF_B1].reshape(256, 160)
    for t in range(24):
        # unit t: tile t is held hidden by the perspective seat
        W1[t, 6 * t + 0] = 1.0
        W1[t, 6 * t + 4] = -1.0
        # unit 24 + t: tile t is held hidden by the next seat
        W1[24 + t, 6 * t + 1] = 1.0
        W1[24 + t, 6 * t + 4] = -1.0
    W2 = p[OFF_W2:OFF_B2].reshape(256, 256)
    W2[0, 0:24] = 1.0
    W2[0, 24:48] = -1.0
    W2[1, 0:24] = -1.0
    W2[1, 24:48] = 1.0
    w3 = p[OFF_W3:OFF_B3]
    w3[0] = Z_SCALE
    w3[1] = -Z_SCALE
    return p


def closed_form(pos: dict, q: int) -> float:
    """v_q of a position dict (tests/positions.py format)."""
    P = pos["P"]

    def hidden(s):
        return sum(1 for t in range(24) if pos["owner"][t] == s and t not in pos["revealed"])

    d = hidden(q) - hidden((q + 1) % P)
    return 1.0 if d > 0 else 0.0 if d < 0 else 0.5
