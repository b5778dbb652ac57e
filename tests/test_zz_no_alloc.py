"""The allocation-free search entry point against mcts_search.

mcts_search_noalloc keeps its trees and its log table in the library's static
device scratch instead of a caller workspace.  Bar: bit-exact -- the same
decisions and the same root-child statistics (action, N, W bit patterns) as
mcts_search with the same arguments, on two calls in a row, the second with
a smaller batch (so that the first call's trees are still in the scratch),
and again in value mode.  Requests beyond the scratch are refused before any
device work.
"""
import ctypes as C

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


def _roots(dvc, n, seed):
    return dvc.dvc_init_states(n, dvc.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3),
                                                  pile_min=0, pile_max=16, revealed_max=8,
                                                  root_draw=1), seed)


def _same(dvc, roots, mp, seed, base):
    print(f"n={roots.shape[0]} iterations={mp.iterations} ppl={mp.playouts_per_leaf} "
          f"leaf_eval={mp.leaf_eval} lpp={mp.leaves_per_pass} pipeline={mp.pipeline}", flush=True)
    b_ref, k_ref = dvc.mcts_search(roots, mp, seed, base)
    b_got, k_got = dvc.mcts_search_noalloc(roots, mp, seed, base,
                                           kids=torch.full_like(k_ref, -7))
    torch.cuda.synchronize()
    assert dvc.dvc_check() == 0
    assert torch.equal(b_got, b_ref)
    assert torch.equal(k_got, k_ref)
    assert int((b_ref >= 0).sum().item()) == roots.shape[0]


def test_noalloc_matches_mcts_search_twice(dvc):
    big = _roots(dvc, 24, 71)
    _same(dvc, big, dvc.mcts_params(iterations=400, playouts_per_leaf=16, max_depth=4), 5, 100)
    # second call: fewer, different trees over the first call's leftovers
    small = _roots(dvc, 5, 72)
    _same(dvc, small, dvc.mcts_params(iterations=150, playouts_per_leaf=32, max_depth=3,
                                      leaves_per_pass=2), 6, 7)


def test_noalloc_value_mode(dvc):
    net = dvc.dvc_valuenet_init(44)
    roots = _roots(dvc, 12, 73)
    mp = dvc.mcts_params(iterations=300, playouts_per_leaf=1, max_depth=4, leaf_eval=1,
                         fallback_band=0.05, fallback_playouts=64, valuenet=net)
    _same(dvc, roots, mp, 8, 0)
    _same(dvc, roots[:3].contiguous(), mp, 9, 40)
    # pipelined passes: two wavefronts per tree, the same static trees
    mp4 = dvc.mcts_params(iterations=300, playouts_per_leaf=1, max_depth=4, leaf_eval=1,
                          fallback_band=0.05, fallback_playouts=64, valuenet=net,
                          leaves_per_pass=4, pipeline=1)
    _same(dvc, roots[:7].contiguous(), mp4, 10, 3)


def test_noalloc_limits(dvc):
    roots = _roots(dvc, 4, 74)
    # the trees of 512 searches of 400 iterations exceed the 64 MiB scratch
    mp = dvc.mcts_params(iterations=400, playouts_per_leaf=16, max_depth=4)
    assert dvc.dvc_mcts_workspace_bytes(512, mp) > dvc.NOALLOC_TREE_BYTES
    best = torch.empty(512, dtype=torch.int32, device="cuda")
    rc = dvc.lib().mcts_search_noalloc(C.c_void_p(roots.data_ptr()), 512, C.byref(mp), 1, 0,
                                       C.c_void_p(best.data_ptr()), None, None)
    assert rc == dvc.DVC_ETOOBIG
    # iterations x playouts beyond the static log table (2^20 entries)
    mp = dvc.mcts_params(iterations=20000, playouts_per_leaf=64, max_depth=4)
    rc = dvc.lib().mcts_search_noalloc(C.c_void_p(roots.data_ptr()), 1, C.byref(mp), 1, 0,
                                       C.c_void_p(best.data_ptr()), None, None)
    assert rc == dvc.DVC_ETOOBIG
    assert "static scratch" in dvc.status_str(dvc.DVC_ETOOBIG)
    assert dvc.dvc_check() == 0
