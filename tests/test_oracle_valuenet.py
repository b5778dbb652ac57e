"""Pins of the value-network oracle (CPU only).

* bfloat16 rounding equals torch's float32 -> bfloat16 conversion (a library
  routine, round to nearest even) on random and tie-breaking values;
* the encoder: one owner bit per owned tile, pool tiles flagged, revealed
  tiles owned, exactly one mover bit, zero padding, rotation with the
  perspective seat;
* exact-mode gradients of the mean squared error against central finite
  differences in double precision;
* one exact-mode forward pass against a plain numpy forward on the same
  encoded features (a second route through the same definition: matrix
  products from the library instead of the oracle's loops);
* the bf16-mirror gradient stays close to the exact one;
* Adam's first step moves every weight by lr * sign(g) (closed form);
* initialization bounds.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_bf16_matches_torch(orc):
    rng = np.random.default_rng(0)
    vals = list(rng.standard_normal(2000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 2000))
    # exact ties between two bf16 values, both parities of the kept bit
    for base in [1.0, 1.5, -3.25, 1e-3]:
        b = np.array([base], np.float32).view(np.uint32)[0]
        vals.append(np.array([b | 0x8000], np.uint32).view(np.float32)[0])
        vals.append(np.array([(b | 0x10000) | 0x8000], np.uint32).view(np.float32)[0])
    for v in vals:
        ref = float(torch.tensor(float(v), dtype=torch.float32).to(torch.bfloat16).float())
        assert orc.bf16(float(v)) == ref, v


def test_encoder_structure(orc):
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8, phase_mix=1)
    S = orc.init_states(300, dp, seed=3)
    for s in S:
        d = orc.unpack(s)
        P = d["P"]
        feats = [orc.vn_encode(s, q) for q in range(P)]
        for q, x in enumerate(feats):
            assert set(np.unique(x)) <= {0.0, 1.0}
            assert np.all(x[148:] == 0)
            t6 = x[:144].reshape(24, 6)
            for t in range(24):
                owned = t not in d["pile"]
                assert t6[t, :4].sum() == (1 if owned else 0)
                assert t6[t, 5] == (0 if owned else 1)
                if t6[t, 4]:
                    assert owned
            for seat in range(P):
                rel = (seat - q) % P
                for t in d["rows"][seat]:
                    assert t6[t, rel] == 1
            assert x[144:148].sum() == 1 and x[144 + (d["mover"] - q) % P] == 1
        # rotating the perspective rotates the owner one-hot only
        for q in range(1, P):
            a = feats[0][:144].reshape(24, 6)
            b = feats[q][:144].reshape(24, 6)
            for t in range(24):
                for seat in range(P):
                    assert a[t, seat] == b[t, (seat - q) % P]


def _batch(orc, n, seed):
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8, phase_mix=1)
    S = orc.init_states(n, dp, seed=seed)
    rng = np.random.default_rng(seed)
    q = np.array([rng.integers(0, orc.unpack(s)["P"]) for s in S], np.int32)
    y = rng.random(n).astype(np.float32)
    return S, q, y


def test_forward_matches_numpy_route(orc):
    p = orc.vn_init(44)
    S, q, y = _batch(orc, 40, 1)
    X = np.stack([orc.vn_encode(s, int(k)) for s, k in zip(S, q)]).astype(np.float64)
    W1 = p[0:40960].reshape(256, 160).astype(np.float64)
    b1 = p[40960:41216].astype(np.float64)
    W2 = p[41216:106752].reshape(256, 256).astype(np.float64)
    b2 = p[106752:107008].astype(np.float64)
    w3 = p[107008:107264].astype(np.float64)
    b3 = float(p[107264])
    h1 = np.maximum(X @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    v = 1 / (1 + np.exp(-(h2 @ w3 + b3)))
    got = orc.vn_forward(p, S, q)
    assert np.allclose(got, v, rtol=1e-12, atol=1e-14)


def test_gradient_finite_differences(orc):
    rng = np.random.default_rng(5)
    p = orc.vn_init(44)
    # make a few biases non-zero so their derivatives are exercised too
    p[40960:41216] += rng.normal(0, 0.05, 256).astype(np.float32)
    p[107264] = 0.1
    S, q, y = _batch(orc, 24, 2)
    loss, g = orc.vn_loss_grad(p, S, q, y)
    # pick parameters in every block, with non-negligible gradients
    blocks = [(0, 40960), (40960, 41216), (41216, 106752), (106752, 107008), (107008, 107264),
              (107264, 107265)]
    checked = 0
    for lo, hi in blocks:
        cand = np.arange(lo, hi)
        cand = cand[np.abs(g[cand]) > 1e-6 * max(1e-12, np.abs(g).max())]
        for k in rng.choice(cand, size=min(6, cand.size), replace=False):
            h = 1e-3 * max(1.0, abs(float(p[k])))
            pp = p.astype(np.float64)
            # perturb in double through a float64 copy routed via two evaluations
            plus = p.copy(); plus[k] = np.float32(pp[k] + h)
            minus = p.copy(); minus[k] = np.float32(pp[k] - h)
            step = float(plus[k]) - float(minus[k])
            lp, _ = orc.vn_loss_grad(plus, S, q, y)
            lm, _ = orc.vn_loss_grad(minus, S, q, y)
            fd = (lp - lm) / step
            assert abs(fd - g[k]) <= 1e-5 * abs(g[k]) + 1e-9, (k, fd, g[k])
            checked += 1
    assert checked >= 25


def test_bf16_mirror_close_to_exact(orc):
    p = orc.vn_init(44)
    S, q, y = _batch(orc, 64, 3)
    v_exact = orc.vn_forward(p, S, q)
    v_mirror = orc.vn_forward(p, S, q, bf16_mirror=True)
    assert np.max(np.abs(v_exact - v_mirror)) < 2e-2
    _, g_exact = orc.vn_loss_grad(p, S, q, y)
    _, g_mirror = orc.vn_loss_grad(p, S, q, y, bf16_mirror=True)
    cos = g_exact @ g_mirror / (np.linalg.norm(g_exact) * np.linalg.norm(g_mirror))
    assert cos > 0.99


def test_adam_first_step_is_sign(orc):
    rng = np.random.default_rng(8)
    n = 1000
    w = rng.normal(size=n)
    w0 = w.copy()
    m = np.zeros(n)
    v = np.zeros(n)
    g = rng.normal(size=n) * 10.0 ** rng.integers(-3, 3, n)
    orc.vn_adam(w, m, v, g, 1, lr=1e-3)
    # with bias correction m_hat = g, v_hat = g^2: step = lr * g / (|g| + eps)
    expect = w0 - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(w, expect, rtol=0, atol=1e-15)
    big = np.abs(g) > 1e-3          # where eps is negligible the step is lr * sign(g)
    assert np.allclose((w0 - w)[big], 1e-3 * np.sign(g[big]), rtol=1e-4)


def test_init_bounds(orc):
    p = orc.vn_init(44)
    W1, W2, w3 = p[:40960], p[41216:106752], p[107008:107264]
    assert np.abs(W1).max() <= math.sqrt(6 / 148) and np.abs(W1).max() > 0.9 * math.sqrt(6 / 148)
    assert np.abs(W2).max() <= math.sqrt(6 / 256) and np.abs(W2).max() > 0.9 * math.sqrt(6 / 256)
    assert np.abs(w3).max() <= 1 / 16
    assert np.all(p[40960:41216] == 0) and np.all(p[106752:107008] == 0) and p[107264] == 0
    assert abs(W1.mean()) < 0.01
    assert not np.array_equal(orc.vn_init(44), orc.vn_init(45))
