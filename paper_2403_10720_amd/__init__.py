"""Python binding of libdvc.so, the gfx950 Da Vinci Code MCTS engine.

Argument marshalling only: every step of the hot path runs in the HIP
kernels of ``libdvc.so``; PyTorch supplies device memory and the stream.
The functions keep the names of the C ABI in ``include/dvc.h``.

There is no CPU fallback: importing the binding without a built library, or
calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdvc.so")
MAX_ACTIONS = 864

DVC_OK, DVC_EINVAL, DVC_ESTATE, DVC_EHIP, DVC_ENOMEM, DVC_ELIMIT = 0, -1, -2, -3, -4, -5
DVC_ETOOBIG = -6
NOALLOC_TREE_BYTES = 64 << 20


class DvcError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})" if what else status_str(status))


class DealParams(C.Structure):
    _fields_ = [("p_min", C.c_int32), ("p_max", C.c_int32), ("hand", C.c_int32 * 5),
                ("pile_min", C.c_int32), ("pile_max", C.c_int32),
                ("revealed_max", C.c_int32), ("fresh", C.c_int32),
                ("root_draw", C.c_int32), ("phase_mix", C.c_int32)]


class MctsParams(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("playouts_per_leaf", C.c_int32),
                ("max_depth", C.c_int32), ("c_uct", C.c_float), ("leaf_eval", C.c_int32),
                ("fallback_band", C.c_float), ("fallback_playouts", C.c_int32),
                ("valuenet", C.c_void_p), ("continue_choice", C.c_int32), ("vanilla", C.c_int32),
                ("leaves_per_pass", C.c_int32), ("pipeline", C.c_int32)]


class MctsTuning(C.Structure):
    _fields_ = [("playouts_per_leaf", C.c_int32), ("leaves_per_pass", C.c_int32),
                ("decisions_per_s", C.c_float), ("agreement", C.c_float),
                ("self_agreement", C.c_float), ("pipeline", C.c_int32)]


def deal_params(p_min=2, p_max=2, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                revealed_max=8, fresh=0, root_draw=0, phase_mix=0) -> DealParams:
    d = DealParams()
    d.p_min, d.p_max = p_min, p_max
    for i in range(5):
        d.hand[i] = hand[i]
    d.pile_min, d.pile_max, d.revealed_max = pile_min, pile_max, revealed_max
    d.fresh, d.root_draw, d.phase_mix = fresh, root_draw, phase_mix
    return d


def mcts_params(iterations=2000, playouts_per_leaf=16, max_depth=4, c_uct=None, leaf_eval=0,
                fallback_band=0.05, fallback_playouts=64, valuenet=None, continue_choice=0,
                vanilla=0, leaves_per_pass=1, pipeline=0) -> MctsParams:
    """max_depth 0: no depth threshold; continue_choice 1: a right guess is
    followed by the same player's stop-or-guess choice; vanilla 1: sampled
    worlds are the root's children (root children come back by action id);
    leaves_per_pass B: B descents per pass, their leaves evaluated together;
    pipeline 1: a pass's wins are credited after the next pass's descents
    (one wavefront descends while another evaluates)."""
    m = MctsParams()
    m.continue_choice, m.vanilla, m.leaves_per_pass = continue_choice, vanilla, leaves_per_pass
    m.pipeline = pipeline
    m.iterations, m.playouts_per_leaf, m.max_depth = iterations, playouts_per_leaf, max_depth
    m.c_uct = float.fromhex("0x1.6a09e6p+0") if c_uct is None else c_uct  # sqrt(2) in float
    m.leaf_eval, m.fallback_band, m.fallback_playouts = leaf_eval, fallback_band, fallback_playouts
    m.valuenet = None if valuenet is None else valuenet.data_ptr()
    return m


_lib = None


def lib():
    """Load libdvc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                              "python paper_2403_10720_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, u32, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_uint64
        L.dvc_version.restype = C.c_char_p
        L.dvc_status_str.restype = C.c_char_p
        L.dvc_status_str.argtypes = [C.c_int]
        L.dvc_check.argtypes = [vp]
        L.dvc_init_states.argtypes = [vp, i64, C.POINTER(DealParams), u64, u32, vp]
        L.dvc_rollout.argtypes = [vp, i64, i32, u64, u32, u32, vp, vp, vp, vp]
        L.dvc_rollout_ex.argtypes = [vp, i64, i32, u64, u32, u32, vp, vp, vp, i32, i32, i32, i32,
                                     vp]
        L.dvc_rollout_autotune.argtypes = [vp, i64, i32, u64, u32, u32, vp, vp, vp, vp, vp]
        L.dvc_valuenet_bytes.restype = C.c_size_t
        L.dvc_valuenet_init.argtypes = [vp, u64, vp]
        L.dvc_valuenet_set_params.argtypes = [vp, vp, vp]
        L.dvc_valuenet_get_params.argtypes = [vp, vp, vp]
        L.dvc_valuenet_get_moments.argtypes = [vp, vp, vp, vp]
        L.dvc_valuenet_epoch_order.argtypes = [u64, i64, i64, C.POINTER(u32), C.POINTER(u32)]
        L.dvc_valuenet_infer.argtypes = [vp, vp, vp, i64, vp, vp]
        L.dvc_valuenet_train_workspace_bytes.restype = C.c_size_t
        L.dvc_valuenet_train_workspace_bytes.argtypes = [i64]
        L.dvc_valuenet_train_step.argtypes = [vp, vp, vp, vp, i64, u32, u32, u32, i32, i64,
                                              C.c_float, vp, C.c_size_t, vp, vp, vp]
        L.dvc_valuenet_labels.argtypes = [vp, i64, i32, u64, u32, u32, vp, vp, vp, vp]
        if hasattr(L, "mcts_search"):
            L.dvc_mcts_workspace_bytes.restype = C.c_size_t
            L.dvc_mcts_workspace_bytes.argtypes = [i64, C.POINTER(MctsParams)]
            L.mcts_search.argtypes = [vp, i64, C.POINTER(MctsParams), u64, u32, vp, C.c_size_t,
                                      vp, vp, vp]
            L.mcts_search_noalloc.argtypes = [vp, i64, C.POINTER(MctsParams), u64, u32, vp, vp,
                                              vp]
            L.mcts_search_root_parallel.argtypes = [vp, i64, i32, C.POINTER(MctsParams), u64, u32,
                                                    vp, C.c_size_t, vp, vp, vp]
            L.dvc_mcts_autotune.argtypes = [vp, i64, C.POINTER(MctsParams), u64, u32, vp,
                                            C.c_size_t, C.c_float, vp, C.POINTER(MctsTuning), vp]
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().dvc_status_str(status).decode()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_dev(t, dtype, shape=None, what=""):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {shape}, got {tuple(t.shape)}")


def _raise(rc, what):
    if rc != DVC_OK:
        raise DvcError(rc, what)


def dvc_check(stream=None) -> int:
    return lib().dvc_check(_stream(stream))


def dvc_init_states(n: int, params: DealParams, seed: int, index_base: int = 0, out=None,
                    device="cuda", stream=None) -> torch.Tensor:
    """n packed states as an int32 tensor of shape (n, 4) (bit pattern of dvc_state_t)."""
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int32, device=device)
    _check_dev(out, torch.int32, (n, 4), "out")
    rc = lib().dvc_init_states(_ptr(out), n, C.byref(params), seed & (2**64 - 1), index_base,
                               _stream(stream))
    _raise(rc, "dvc_init_states")
    return out


def dvc_rollout(leaves: torch.Tensor, playouts_per_leaf: int, seed: int, tree_id: int = 0,
                leaf_id_base: int = 0, winner=True, length=True, seat_wins=True, variant: int = 0,
                block: int = 0, grid: int = 0, accumulate: bool = False, stream=None):
    """Random playouts from every leaf.  Returns (winner int8 [n*ppl] | None,
    length int16 [n*ppl] | None, seat_wins int32 [n, 4] | None); pass
    preallocated tensors instead of True to reuse memory.  accumulate=True
    adds to the given seat_wins instead of overwriting it."""
    _check_dev(leaves, torch.int32, None, "leaves")
    if leaves.dim() != 2 or leaves.shape[1] != 4:
        raise ValueError("leaves must have shape (n, 4)")
    n = leaves.shape[0]
    dev = leaves.device
    total = n * playouts_per_leaf

    def prep(x, dtype, shape):
        if x is True:
            return torch.empty(shape, dtype=dtype, device=dev)
        if x is False or x is None:
            return None
        _check_dev(x, dtype, shape, "output")
        return x

    w = prep(winner, torch.int8, (total,))
    ln = prep(length, torch.int16, (total,))
    sw = prep(seat_wins, torch.int32, (n, 4))
    rc = lib().dvc_rollout_ex(_ptr(leaves), n, playouts_per_leaf, seed & (2**64 - 1), tree_id,
                              leaf_id_base, _ptr(w), _ptr(ln), _ptr(sw), variant, block, grid,
                              1 if accumulate else 0, _stream(stream))
    _raise(rc, "dvc_rollout")
    return w, ln, sw


def dvc_rollout_autotune(leaves: torch.Tensor, playouts_per_leaf: int, seed: int, tree_id: int = 0,
                         leaf_id_base: int = 0, winner=True, length=True, seat_wins=True,
                         stream=None):
    """Time every rollout kernel shape on this batch and remember the fastest
    for its size class (used by later calls with variant 0).  Returns
    ((variant, block, grid), (winner, length, seat_wins)) -- the outputs are
    the batch's playouts, as dvc_rollout writes them."""
    _check_dev(leaves, torch.int32, None, "leaves")
    n = leaves.shape[0]
    dev = leaves.device
    total = n * playouts_per_leaf

    def prep(x, dtype, shape):
        if x is True:
            return torch.empty(shape, dtype=dtype, device=dev)
        if x is False or x is None:
            return None
        _check_dev(x, dtype, shape, "output")
        return x

    w = prep(winner, torch.int8, (total,))
    ln = prep(length, torch.int16, (total,))
    sw = prep(seat_wins, torch.int32, (n, 4))
    chosen = (C.c_int32 * 3)()
    rc = lib().dvc_rollout_autotune(_ptr(leaves), n, playouts_per_leaf, seed & (2**64 - 1),
                                    tree_id, leaf_id_base, _ptr(w), _ptr(ln), _ptr(sw),
                                    C.cast(chosen, C.c_void_p), _stream(stream))
    _raise(rc, "dvc_rollout_autotune")
    return (chosen[0], chosen[1], chosen[2]), (w, ln, sw)


def dvc_mcts_workspace_bytes(n_trees: int, params: MctsParams) -> int:
    return int(lib().dvc_mcts_workspace_bytes(n_trees, C.byref(params)))


def mcts_search(roots: torch.Tensor, params: MctsParams, seed: int, tree_id_base: int = 0,
                workspace=None, want_children: bool = True, stream=None):
    """One decision per root.  Returns (best_action int32 [n], children
    int32 [n, 864, 3] | None) where children[..., 0] = action | pad << 16,
    [..., 1] = n (bit pattern of uint32), [..., 2] = w (bit pattern of float)."""
    _check_dev(roots, torch.int32, None, "roots")
    n = roots.shape[0]
    dev = roots.device
    need = dvc_mcts_workspace_bytes(n, params)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    best = torch.empty(n, dtype=torch.int32, device=dev)
    kids = torch.empty((n, MAX_ACTIONS, 3), dtype=torch.int32, device=dev) if want_children else None
    rc = lib().mcts_search(_ptr(roots), n, C.byref(params), seed & (2**64 - 1), tree_id_base,
                           _ptr(workspace), workspace.numel(), _ptr(best), _ptr(kids),
                           _stream(stream))
    _raise(rc, "mcts_search")
    return best, kids


def mcts_search_noalloc(roots: torch.Tensor, params: MctsParams, seed: int, tree_id_base: int = 0,
                        best=None, kids=None, stream=None):
    """mcts_search with the trees in the library's static scratch (no
    workspace, nothing allocated by the call).  Outputs as mcts_search; pass
    `best` (int32 [n]) and `kids` (int32 [n, 864, 3] or None) to reuse
    buffers."""
    _check_dev(roots, torch.int32, None, "roots")
    n = roots.shape[0]
    if best is None:
        best = torch.empty(n, dtype=torch.int32, device=roots.device)
    _check_dev(best, torch.int32, (n,), "best")
    _check_dev(kids, torch.int32, (n, MAX_ACTIONS, 3), "kids")
    rc = lib().mcts_search_noalloc(_ptr(roots), n, C.byref(params), seed & (2**64 - 1),
                                   tree_id_base, _ptr(best), _ptr(kids), _stream(stream))
    _raise(rc, "mcts_search_noalloc")
    return best, kids


def dvc_mcts_autotune(roots: torch.Tensor, params: MctsParams, seed: int, tree_id_base: int = 0,
                      tolerance: float = 0.02, workspace=None, stream=None):
    """Pick playouts per leaf x leaves per pass x pipelined passes for searches
    of this size class (see include/dvc.h).  Returns (choice dict, decisions of
    the chosen shape)."""
    _check_dev(roots, torch.int32, None, "roots")
    n = roots.shape[0]
    need = dvc_mcts_workspace_bytes(n, params)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=roots.device)
    best = torch.empty(n, dtype=torch.int32, device=roots.device)
    res = MctsTuning()
    rc = lib().dvc_mcts_autotune(_ptr(roots), n, C.byref(params), seed & (2**64 - 1), tree_id_base,
                                 _ptr(workspace), workspace.numel(), tolerance, _ptr(best),
                                 C.byref(res), _stream(stream))
    _raise(rc, "dvc_mcts_autotune")
    return ({"playouts_per_leaf": res.playouts_per_leaf, "leaves_per_pass": res.leaves_per_pass,
             "pipeline": res.pipeline, "decisions_per_s": res.decisions_per_s,
             "agreement": res.agreement,
             "self_agreement": res.self_agreement}, best)


def mcts_search_root_parallel(roots: torch.Tensor, trees_per_root: int, params: MctsParams,
                              seed: int, tree_id_base: int = 0, workspace=None,
                              want_children: bool = True, stream=None):
    """K independent trees per root amalgamated into one root (tree id
    tree_id_base + r*K + k).  Returns (best_action int32 [n], merged children
    int32 [n, 864, 3] indexed by action id | None), same encoding as
    mcts_search's children."""
    _check_dev(roots, torch.int32, None, "roots")
    n = roots.shape[0]
    dev = roots.device
    need = dvc_mcts_workspace_bytes(n * max(trees_per_root, 1), params)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    best = torch.empty(n, dtype=torch.int32, device=dev)
    kids = torch.empty((n, MAX_ACTIONS, 3), dtype=torch.int32, device=dev) if want_children else None
    rc = lib().mcts_search_root_parallel(_ptr(roots), n, trees_per_root, C.byref(params),
                                         seed & (2**64 - 1), tree_id_base, _ptr(workspace),
                                         workspace.numel(), _ptr(best), _ptr(kids),
                                         _stream(stream))
    _raise(rc, "mcts_search_root_parallel")
    return best, kids


def mcts_tree_stats(workspace: torch.Tensor, n_trees: int, params: MctsParams) -> dict:
    """Per-tree counters the search leaves at the start of each tree's workspace,
    including shader clock cycles spent in each phase of the iterations, the
    deepest leaf and the root's child count (world nodes in vanilla trees)."""
    per_tree = dvc_mcts_workspace_bytes(1, params)
    h = workspace[:n_trees * per_tree].view(n_trees, per_tree)[:, :80].contiguous().cpu()
    w = h.view(torch.int32)
    cyc = h.view(torch.int64)[:, 4:8]
    return {"nodes": w[:, 0], "overflow_blocks": w[:, 1], "root_visits": w[:, 2], "net_leaves": w[:, 3],
            "played_leaves": w[:, 4], "sampler_fallbacks": w[:, 5], "failed": w[:, 6],
            "deepest_leaf": w[:, 7], "root_children": w[:, 18],
            "cycles_sample": cyc[:, 0], "cycles_descend": cyc[:, 1], "cycles_evaluate": cyc[:, 2],
            "cycles_backprop": cyc[:, 3]}


def children_view(kids: torch.Tensor):
    """Split the raw child-statistics tensor into (action, n, w) tensors on the host."""
    k = kids.cpu()
    action = (k[..., 0] & 0xFFFF)
    n = k[..., 1].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    w = k[..., 2].view(torch.float32)
    return action, n, w


def c_uct_default() -> float:
    return float.fromhex("0x1.6a09e6p+0")


assert abs(c_uct_default() - math.sqrt(2)) < 1e-6


# ---------------------------------------------------------------------------
# value network
# ---------------------------------------------------------------------------
VALUENET_PARAMS = 107265


def dvc_valuenet_bytes() -> int:
    return int(lib().dvc_valuenet_bytes())


def dvc_valuenet_init(seed: int, net=None, device="cuda", stream=None) -> torch.Tensor:
    if net is None:
        net = torch.empty(dvc_valuenet_bytes(), dtype=torch.uint8, device=device)
    _raise(lib().dvc_valuenet_init(_ptr(net), seed & (2**64 - 1), _stream(stream)), "dvc_valuenet_init")
    return net


def dvc_valuenet_set_params(net, params: torch.Tensor, stream=None):
    _check_dev(params, torch.float32, (VALUENET_PARAMS,), "params")
    _raise(lib().dvc_valuenet_set_params(_ptr(net), _ptr(params), _stream(stream)),
           "dvc_valuenet_set_params")


def dvc_valuenet_get_params(net, stream=None) -> torch.Tensor:
    out = torch.empty(VALUENET_PARAMS, dtype=torch.float32, device=net.device)
    _raise(lib().dvc_valuenet_get_params(_ptr(net), _ptr(out), _stream(stream)),
           "dvc_valuenet_get_params")
    return out


def dvc_valuenet_get_moments(net, stream=None):
    """(m, v): the Adam moments in the flat parameter order."""
    m = torch.empty(VALUENET_PARAMS, dtype=torch.float32, device=net.device)
    v = torch.empty(VALUENET_PARAMS, dtype=torch.float32, device=net.device)
    _raise(lib().dvc_valuenet_get_moments(_ptr(net), _ptr(m), _ptr(v), _stream(stream)),
           "dvc_valuenet_get_moments")
    return m, v


def dvc_valuenet_infer(net, states: torch.Tensor, persp: torch.Tensor, out=None, stream=None):
    _check_dev(states, torch.int32, None, "states")
    _check_dev(persp, torch.uint8, (states.shape[0],), "persp")
    n = states.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=states.device)
    _raise(lib().dvc_valuenet_infer(_ptr(net), _ptr(states), _ptr(persp), n, _ptr(out),
                                    _stream(stream)), "dvc_valuenet_infer")
    return out


def dvc_valuenet_epoch_order(seed: int, epoch: int, n_data: int):
    """(perm_a, perm_b) of an epoch's batch order (Philox, see include/dvc.h)."""
    a, b = C.c_uint32(0), C.c_uint32(0)
    _raise(lib().dvc_valuenet_epoch_order(seed & (2**64 - 1), epoch, n_data, C.byref(a),
                                          C.byref(b)), "dvc_valuenet_epoch_order")
    return a.value, b.value


def dvc_valuenet_train_workspace_bytes(batch: int) -> int:
    return int(lib().dvc_valuenet_train_workspace_bytes(batch))


def dvc_valuenet_train_step(net, states, persp, labels, step: int, lr: float = 1e-3,
                            batch: int = 8192, perm_a: int = 1, perm_b: int = 0, row_base: int = 0,
                            ws=None, loss_out=None, grad_out=None, stream=None):
    n_data = states.shape[0]
    if ws is None:
        ws = torch.empty(dvc_valuenet_train_workspace_bytes(batch), dtype=torch.uint8,
                         device=states.device)
    rc = lib().dvc_valuenet_train_step(_ptr(net), _ptr(states), _ptr(persp), _ptr(labels), n_data,
                                       perm_a & 0xFFFFFFFF, perm_b & 0xFFFFFFFF,
                                       row_base & 0xFFFFFFFF, batch, step, lr, _ptr(ws),
                                       ws.numel(), _ptr(loss_out), _ptr(grad_out), _stream(stream))
    _raise(rc, "dvc_valuenet_train_step")
    return ws


def dvc_valuenet_labels(states, playouts: int, seed: int, tree_id: int = 1, index_base: int = 0,
                        stream=None):
    n = states.shape[0]
    dev = states.device
    persp = torch.empty(n, dtype=torch.uint8, device=dev)
    labels = torch.empty(n, dtype=torch.float32, device=dev)
    ws = torch.empty((n, 4), dtype=torch.int32, device=dev)
    rc = lib().dvc_valuenet_labels(_ptr(states), n, playouts, seed & (2**64 - 1), tree_id,
                                   index_base, _ptr(persp), _ptr(labels), _ptr(ws), _stream(stream))
    _raise(rc, "dvc_valuenet_labels")
    return persp, labels
