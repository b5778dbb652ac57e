"""GPU value network vs the oracle (through the C ABI).

Bar: tolerance (the products run in bfloat16 on the matrix cores with
float32 accumulation in a hardware order the oracle does not reproduce).
* initialization: bit-exact float32 parameters (same Philox words);
* inference vs the oracle's bf16-mirroring forward: |dv| <= 2^-7 |v| + 1e-3;
* the gradient of one training step vs the oracle's bf16-mirroring gradient:
  cosine >= 0.999 overall and per block, magnitudes within 5% (batch 256);
  element by element at the training batch (8192 rows, every batch slice and
  chunk of the weight-gradient products): |g - g_ref| <= 2^-7 * A, where A is
  the sum of the absolute values of the element's per-row terms (the oracle
  returns it).  Both sides round the same operands to bfloat16; they differ
  where a float32 sum in another order lands on the other side of a bfloat16
  rounding boundary (one operand off by at most 2^-8 of itself) and in the
  float32 accumulation (at most about 2^-11 A over 8192 terms), so 2^-7 A
  bounds every term's operands rounded the other way with room to spare;
* Adam over three steps from fresh moments: after every step the GPU's
  weights and both moments equal the oracle's Adam (double) fed with the
  GPU's own gradients (float32 vs double: 1e-5 relative);
* training pairs: perspectives and labels bit-exact vs oracle playouts;
* a training step is deterministic (fixed-order reductions): repeated runs agree bit for bit;
* a few hundred steps on one batch drive its loss down (overfit check);
* what the network gains: a trained network predicts held-out win rates far
  better than the untrained one, and a value search agrees more often with a
  high-budget playout search than a cheaper-or-equal pure playout search does.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dvc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_10720_amd as D
    D.lib()
    return D


def _data(orc, n, seed):
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8, phase_mix=1)
    S = orc.init_states(n, dp, seed=seed)
    rng = np.random.default_rng(seed)
    q = np.array([rng.integers(0, orc.unpack(s)["P"]) for s in S], np.uint8)
    y = rng.random(n).astype(np.float32)
    return S, q, y


def _dev(S, q, y):
    return (torch.from_numpy(S.view(np.int32)).cuda(), torch.from_numpy(q).cuda(),
            torch.from_numpy(y).cuda())


def test_init_bit_exact(orc, dvc):
    net = dvc.dvc_valuenet_init(44)
    got = dvc.dvc_valuenet_get_params(net).cpu().numpy()
    ref = orc.vn_init(44)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("n", [1, 15, 16, 100, 1000])
def test_infer_vs_oracle(orc, dvc, n):
    S, q, y = _data(orc, n, 7 + n)
    params = orc.vn_init(3)
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(params).cuda())
    st, qd, _ = _dev(S, q, y)
    v = dvc.dvc_valuenet_infer(net, st, qd).cpu().numpy()
    ref = orc.vn_forward(params, S, q.astype(np.int32), bf16_mirror=True)
    assert np.all(np.abs(v - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-3), np.abs(v - ref).max()
    assert dvc.dvc_check() == 0


def test_gradient_vs_oracle(orc, dvc):
    B = 256
    S, q, y = _data(orc, B, 11)
    params = orc.vn_init(5)
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(params).cuda())
    st, qd, yd = _dev(S, q, y)
    grad = torch.zeros(dvc.VALUENET_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dvc.dvc_valuenet_train_step(net, st, qd, yd, step=1, lr=1e-3, batch=B, grad_out=grad,
                                loss_out=loss)
    g = grad.cpu().numpy().astype(np.float64)
    ref_loss, ref = orc.vn_loss_grad(params, S, q.astype(np.int32), y, bf16_mirror=True)
    assert abs(float(loss.item()) - ref_loss) <= 1e-3 * ref_loss + 1e-6
    cos = g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref))
    assert cos >= 0.999, cos
    blocks = {"W1": (0, 40960), "b1": (40960, 41216), "W2": (41216, 106752),
              "b2": (106752, 107008), "w3": (107008, 107264)}
    for name, (lo, hi) in blocks.items():
        a, b = g[lo:hi], ref[lo:hi]
        c = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30)
        assert c >= 0.999, (name, c)
        assert abs(np.linalg.norm(a) / np.linalg.norm(b) - 1) < 0.05, name
    assert abs(g[107264] - ref[107264]) <= 1e-3 * abs(ref[107264]) + 1e-7
    # Adam step: compare the updated parameters with the oracle's Adam on g
    got = dvc.dvc_valuenet_get_params(net).cpu().numpy().astype(np.float64)
    w = params.astype(np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    orc.vn_adam(w, m, v, g.copy(), 1, lr=1e-3)
    assert np.allclose(got, w, rtol=1e-5, atol=1e-7)


def test_gradient_elementwise_at_training_batch(orc, dvc):
    B = 8192
    S, q, y = _data(orc, B, 11)
    params = orc.vn_init(5)
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(params).cuda())
    st, qd, yd = _dev(S, q, y)
    grad = torch.zeros(dvc.VALUENET_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dvc.dvc_valuenet_train_step(net, st, qd, yd, step=1, lr=1e-3, batch=B, grad_out=grad,
                                loss_out=loss)
    g = grad.cpu().numpy().astype(np.float64)
    ref_loss, ref, A = orc.vn_loss_grad(params, S, q.astype(np.int32), y, bf16_mirror=True,
                                        want_abs=True)
    assert abs(float(loss.item()) - ref_loss) <= 1e-4 * ref_loss
    err = np.abs(g - ref)
    ratio = err / np.maximum(A, 1e-300)
    worst = int(np.argmax(np.where(A > 0, ratio, 0)))
    print(f"max |g - ref| / A = {ratio[worst]:.3g} at {worst}; "
          f"median {np.median(ratio[A > 0]):.3g}", flush=True)
    assert np.all(g[A == 0] == 0.0)
    assert np.all(err <= 2.0 ** -7 * A), (worst, g[worst], ref[worst], A[worst])
    cos = g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref))
    assert cos >= 0.9999, cos
    assert dvc.dvc_check() == 0


def test_adam_three_steps_vs_oracle(orc, dvc):
    B, n = 8192, 16384
    S, q, y = _data(orc, n, 12)
    params = orc.vn_init(6)
    net = dvc.dvc_valuenet_init(0)
    dvc.dvc_valuenet_set_params(net, torch.from_numpy(params).cuda())
    st, qd, yd = _dev(S, q, y)
    grad = torch.zeros(dvc.VALUENET_PARAMS, dtype=torch.float32, device="cuda")
    w = params.astype(np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    # float32 rounding of the first moment scales with the terms it adds,
    # beta1 |m| + (1 - beta1) |g|, not with m, which can cancel: A is that
    # scale (the decayed sum of |g|), and a few roundings of 2^-24 each are
    # allowed for every step
    A = np.zeros_like(w)
    prev_w = w.copy()
    ws = None
    for step in range(1, 4):
        lr = 1e-3 * step   # a different rate per step
        ws = dvc.dvc_valuenet_train_step(net, st, qd, yd, step=step, lr=lr, batch=B,
                                         perm_a=2654435761, perm_b=7, row_base=(step - 1) * B,
                                         ws=ws, grad_out=grad)
        g = grad.cpu().numpy().astype(np.float64)
        orc.vn_adam(w, m, v, g.copy(), step, lr=lr)
        A = 0.9 * A + 0.1 * np.abs(g)
        got_w = dvc.dvc_valuenet_get_params(net).cpu().numpy().astype(np.float64)
        gm, gv = (t.cpu().numpy().astype(np.float64) for t in dvc.dvc_valuenet_get_moments(net))
        err = np.abs(gm - m)
        assert np.all(err <= 2.0 ** -20 * A), (step, int(np.argmax(err / np.maximum(A, 1e-300))))
        assert np.allclose(gv, v, rtol=1e-5, atol=1e-38), step
        assert np.allclose(got_w, w, rtol=1e-5, atol=1e-7), step
        # the step moved the weights (every parameter with a nonzero first
        # moment moves)
        moved = got_w != prev_w
        assert moved.sum() > 50000, (step, moved.sum())
        prev_w = got_w
    assert dvc.dvc_check() == 0


@pytest.mark.parametrize("B", [32, 96, 8192])
def test_training_step_is_deterministic(orc, dvc, B):
    """Every reduction of a training step (split-K weight gradients over batch
    slices, bias gradients and loss over row tiles) runs in a fixed order, so
    the same steps from the same weights give bit-identical gradients, losses
    and weights, whatever the scheduling of the workgroups."""
    n = max(B, 4096)
    S, q, y = _data(orc, n, 23)
    st, qd, yd = _dev(S, q, y)
    runs = []
    for _ in range(2):
        net = dvc.dvc_valuenet_init(44)
        grad = torch.zeros(dvc.VALUENET_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        ws, out = None, []
        for step in range(1, 4):
            ws = dvc.dvc_valuenet_train_step(net, st, qd, yd, step=step, lr=1e-3, batch=B,
                                             perm_a=2654435761 if n > B else 1, perm_b=3,
                                             row_base=(step - 1) * B, ws=ws, loss_out=loss,
                                             grad_out=grad)
            out.append((grad.cpu().numpy().copy(), loss.cpu().numpy().copy()))
        runs.append((out, dvc.dvc_valuenet_get_params(net).cpu().numpy()))
    (o1, p1), (o2, p2) = runs
    for (g1, l1), (g2, l2) in zip(o1, o2):
        assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32))
        assert np.array_equal(l1.view(np.uint32), l2.view(np.uint32))
    assert np.array_equal(p1.view(np.uint32), p2.view(np.uint32))
    assert dvc.dvc_check() == 0


def test_labels_bit_exact(orc, dvc):
    n, ppl, seed = 300, 64, 9
    dp = orc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8, phase_mix=1)
    S = orc.init_states(n, dp, seed=seed, index_base=1000)
    st = torch.from_numpy(S.view(np.int32)).cuda()
    persp, labels = dvc.dvc_valuenet_labels(st, ppl, seed, tree_id=1, index_base=1000)
    _, _, wins = orc.rollout(S, ppl, seed, tree_id=1, leaf_id_base=1000)
    for i in range(n):
        P = orc.unpack(S[i])["P"]
        w = orc.philox([0, 0xFFFFFFFC, 0, 1000 + i], [seed, 0])[0]
        q = orc.mulshift(int(w), P)
        assert persp[i].item() == q
        assert labels[i].item() == np.float32(wins[i, q]) / np.float32(ppl)


def test_overfit_one_batch(orc, dvc):
    B = 512
    S, q, y = _data(orc, B, 13)
    st, qd, yd = _dev(S, q, y)
    net = dvc.dvc_valuenet_init(44)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = None
    hist = []
    for step in range(1, 401):
        ws = dvc.dvc_valuenet_train_step(net, st, qd, yd, step=step, lr=3e-3, batch=B, ws=ws,
                                         loss_out=loss)
        if step in (1, 400):
            hist.append(float(loss.item()))
    assert hist[1] < 0.25 * hist[0], hist
    assert dvc.dvc_check() == 0


def test_argument_errors(dvc):
    net = dvc.dvc_valuenet_init(1)
    st = torch.zeros((40, 4), dtype=torch.int32, device="cuda")
    q = torch.zeros(40, dtype=torch.uint8, device="cuda")
    y = torch.zeros(40, dtype=torch.float32, device="cuda")
    with pytest.raises(dvc.DvcError):
        dvc.dvc_valuenet_train_step(net, st, q, y, step=1, batch=40)   # not a multiple of 32
    with pytest.raises(dvc.DvcError):
        dvc.dvc_valuenet_train_step(net, st, q, y, step=0, batch=32)


def test_training_gains_over_the_untrained_network(dvc):
    """What the learned part adds: a network trained by the library's own kernels
    on rollout-labelled pairs predicts held-out 1024-playout win rates far better
    than the same network before training, and a search that scores every leaf
    with it (no playout fallback) agrees with the pure-playout search more often."""
    from paper_2403_10720_amd.valuenet import TrainConfig, make_data, train, TRAIN_DEAL
    cfg = TrainConfig(n_data=1 << 16, playouts=64, batch=2048, epochs=12, lr=2e-3)
    data = make_data(cfg.n_data, cfg.playouts, seed=21)
    untrained = dvc.dvc_valuenet_init(cfg.init_seed)
    trained, hist, _ = train(cfg, data=data)
    n = 2048
    states = dvc.dvc_init_states(n, dvc.deal_params(**TRAIN_DEAL), 77, index_base=1 << 27)
    persp, labels = dvc.dvc_valuenet_labels(states, 1024, 77, tree_id=0xE7A1, index_base=1 << 27)
    mse = {}
    for name, net in [("untrained", untrained), ("trained", trained)]:
        v = dvc.dvc_valuenet_infer(net, states, persp)
        mse[name] = float(((v - labels) ** 2).mean().item())
    assert mse["trained"] < 0.5 * mse["untrained"], mse

    roots = dvc.dvc_init_states(256, dvc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3),
                                                     fresh=1, root_draw=1), 5)
    ref, _ = dvc.mcts_search(roots, dvc.mcts_params(iterations=512, playouts_per_leaf=64), 5,
                             want_children=False)
    agree = {}
    for name, net in [("untrained", untrained), ("trained", trained)]:
        mp = dvc.mcts_params(iterations=512, playouts_per_leaf=1, leaf_eval=1, fallback_band=0.0,
                             fallback_playouts=64, valuenet=net)
        best, _ = dvc.mcts_search(roots, mp, 5, want_children=False)
        agree[name] = float((best == ref).float().mean().item())
    assert agree["trained"] > agree["untrained"], agree
    assert dvc.dvc_check() == 0


def test_value_search_gains_over_playout_search_at_lower_cost(dvc):
    """What the network gains over the method without it: on 1024 fresh deals,
    a value search (network leaves, 64-playout fallback within 0.05 of 1/2,
    4096 iterations, four leaves per pass, pipelined) takes less GPU time than
    a pure playout search of 2048 iterations x 64 playouts and agrees more
    often with a 16384-iteration playout search (the high-budget reference).
    Searches and training are deterministic; only the timing varies."""
    from paper_2403_10720_amd.experiments import ROOT_DEAL, median_search
    from paper_2403_10720_amd.valuenet import TrainConfig, make_data, train
    cfg = TrainConfig()
    net, _, _ = train(cfg, data=make_data(cfg.n_data, cfg.playouts, cfg.data_seed))
    n = 1024
    roots = dvc.dvc_init_states(n, dvc.deal_params(**ROOT_DEAL), 5)
    ref_mp = dvc.mcts_params(iterations=16384, playouts_per_leaf=64, max_depth=4)
    ws = torch.empty(dvc.dvc_mcts_workspace_bytes(n, ref_mp), dtype=torch.uint8, device="cuda")
    ref, _ = dvc.mcts_search(roots, ref_mp, 1001, workspace=ws, want_children=False)
    val_mp = dvc.mcts_params(iterations=4096, playouts_per_leaf=1, max_depth=4, leaf_eval=1,
                             fallback_band=0.05, fallback_playouts=64, valuenet=net,
                             leaves_per_pass=4, pipeline=1)
    roll_mp = dvc.mcts_params(iterations=2048, playouts_per_leaf=64, max_depth=4)
    best_v, t_v = median_search(roots, val_mp, 5, ws)
    best_r, t_r = median_search(roots, roll_mp, 5, ws)
    agree_v = float((best_v == ref).float().mean().item())
    agree_r = float((best_r == ref).float().mean().item())
    print(f"value {t_v * 1e3:.1f} ms, agreement {agree_v:.3f}; "
          f"playout {t_r * 1e3:.1f} ms, agreement {agree_r:.3f}", flush=True)
    assert t_v < t_r, (t_v, t_r)
    assert agree_v > agree_r + 0.03, (agree_v, agree_r)
    assert dvc.dvc_check() == 0
