"""HIP graph capture of the library's calls (through the C ABI).

The library launches only kernels on the caller's stream (no memset nodes,
no allocation once its log table exists), so a decision loop can be captured
once and replayed.  Each test captures a call with torch's graph API, replays
it three times with eager work and synchronizations between the replays, and
checks every replay bit-exactly against the eager result.
"""
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


def test_graph_rollout_step(dvc):
    n, ppl = 512, 64
    params = dvc.deal_params(p_min=2, p_max=4, pile_min=0, pile_max=16, revealed_max=8)
    states = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    winner = torch.empty(n * ppl, dtype=torch.int8, device="cuda")
    length = torch.empty(n * ppl, dtype=torch.int16, device="cuda")
    wins = torch.empty((n, 4), dtype=torch.int32, device="cuda")

    def step():
        dvc.dvc_init_states(n, params, 11, out=states)
        dvc.dvc_rollout(states, ppl, 11, 0, 0, winner=winner, length=length, seat_wins=wins)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = (states.clone(), winner.clone(), length.clone(), wins.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for _ in range(3):
        states.zero_(); winner.zero_(); length.zero_(); wins.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((states, winner, length, wins), ref):
            assert torch.equal(a, b)
    assert dvc.dvc_check() == 0


@pytest.mark.parametrize("kw", [dict(), dict(leaves_per_pass=2, playouts_per_leaf=32),
                                dict(leaves_per_pass=2, playouts_per_leaf=32, pipeline=1),
                                dict(continue_choice=1, max_depth=0, vanilla=1)])
def test_graph_batched_search(dvc, kw):
    """A captured search (sequential, leaf-batched, pipelined, un-simplified
    variants) replays to the eager result every time."""
    n = 64
    roots = dvc.dvc_init_states(n, dvc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3),
                                                   pile_min=0, pile_max=16, revealed_max=8,
                                                   root_draw=1), 3)
    args = dict(iterations=256, playouts_per_leaf=16, max_depth=4)
    args.update(kw)
    mp = dvc.mcts_params(**args)
    ws = torch.empty(dvc.dvc_mcts_workspace_bytes(n, mp), dtype=torch.uint8, device="cuda")
    best = torch.empty(n, dtype=torch.int32, device="cuda")
    kids = torch.empty((n, 864, 3), dtype=torch.int32, device="cuda")
    ref_best, ref_kids = dvc.mcts_search(roots, mp, 3, workspace=ws)   # also sizes the log table
    torch.cuda.synchronize()

    import ctypes as C
    L = dvc.lib()

    def call():
        rc = L.mcts_search(C.c_void_p(roots.data_ptr()), n, C.byref(mp), 3, 0,
                           C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(best.data_ptr()),
                           C.c_void_p(kids.data_ptr()),
                           C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for _ in range(3):
        best.fill_(-5); kids.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(best, ref_best) and torch.equal(kids, ref_kids)
    assert dvc.dvc_check() == 0
