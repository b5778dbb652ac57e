"""CPU oracle of the Da Vinci Code MCTS hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it.

The arithmetic lives in plain C (``rules.c``, ``mcts.c``, ``valuenet.c``);
this module only marshals numpy arrays through ctypes.  States are
``uint32`` arrays of shape ``(n, 4)`` in the packed 16-byte interface format.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

MAX_CHILD = 864
STOP_KEY = 864          # tree key of the stop choice; a guess after a right guess is 865 + a


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


class Rows(C.Structure):
    _fields_ = [("P", C.c_int32), ("n", C.c_int32 * 4), ("tile", (C.c_int32 * 24) * 4),
                ("rev", (C.c_int32 * 24) * 4), ("pile_n", C.c_int32), ("pile", C.c_int32 * 24),
                ("mover", C.c_int32), ("phase", C.c_int32), ("drawn", C.c_int32)]

    def as_dict(self) -> dict:
        return {
            "P": self.P,
            "rows": [[int(self.tile[q][j]) for j in range(self.n[q])] for q in range(self.P)],
            "rev": [[int(self.rev[q][j]) for j in range(self.n[q])] for q in range(self.P)],
            "pile": [int(self.pile[j]) for j in range(self.pile_n)],
            "mover": self.mover, "phase": self.phase, "drawn": self.drawn,
        }


CHILD_DTYPE = np.dtype([("action", "<u2"), ("pad", "<u2"), ("n", "<u4"), ("w", "<f4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        u32p = C.POINTER(C.c_uint32)
        L.oracle_philox.argtypes = [u32p, u32p, u32p]
        L.oracle_mulshift.restype = C.c_uint32
        L.oracle_mulshift.argtypes = [C.c_uint32, C.c_uint32]
        L.oracle_validate.argtypes = [C.c_void_p]
        L.oracle_unpack.argtypes = [C.c_void_p, C.POINTER(Rows)]
        L.oracle_pack.argtypes = [C.POINTER(Rows), C.c_void_p]
        L.oracle_playout.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.POINTER(C.c_int), C.POINTER(Rows), C.POINTER(C.c_int)]
        L.oracle_rollout.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_uint32,
                                     C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_rollout_mt.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_uint32,
                                        C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.oracle_init_states.argtypes = [C.c_void_p, C.c_int64, C.POINTER(DealParams), C.c_uint64,
                                         C.c_uint32]
        L.oracle_determinize.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_void_p]
        L.oracle_legal_actions.argtypes = [C.c_void_p, C.c_void_p]
        L.oracle_apply_action.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                          C.c_uint32, C.c_void_p, C.POINTER(C.c_int),
                                          C.POINTER(C.c_int)]
        L.oracle_ln_entry.restype = C.c_float
        L.oracle_ln_entry.argtypes = [C.c_uint32]
        L.oracle_mcts_search.argtypes = [C.c_void_p, C.c_int64, C.POINTER(MctsParams), C.c_uint64,
                                         C.c_uint32, C.c_void_p, C.c_void_p]
        L.oracle_mcts_search_merged.argtypes = [C.c_void_p, C.c_int64, C.c_int32,
                                                C.POINTER(MctsParams), C.c_uint64, C.c_uint32,
                                                C.c_void_p, C.c_void_p]
        L.oracle_mcts_tree_dump.argtypes = [C.c_void_p, C.POINTER(MctsParams), C.c_uint64,
                                            C.c_uint32, C.c_void_p, C.c_void_p, C.c_int64]
        L.oracle_bf16.restype = C.c_float
        L.oracle_bf16.argtypes = [C.c_float]
        L.oracle_vn_encode.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
        L.oracle_vn_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                        C.c_void_p]
        L.oracle_vn_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                          C.c_int, C.POINTER(C.c_double), C.c_void_p, C.c_void_p]
        L.oracle_vn_adam.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double]
        L.oracle_vn_init.argtypes = [C.c_void_p, C.c_uint64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _states(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    if a.ndim == 1:
        a = a.reshape(1, 4)
    assert a.ndim == 2 and a.shape[1] == 4
    return a


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
    """valuenet: float32 numpy array of the network parameters (value mode);
    the caller keeps it alive while the search runs.  max_depth 0: no depth
    threshold; continue_choice 1: a right guess is followed by the same
    player's stop-or-guess choice; vanilla 1: the root's children are the
    sampled worlds (children then come back indexed by action id);
    leaves_per_pass B: B descents, each adding its visit counts at once, then
    their leaves are evaluated together; pipeline 1: a pass's wins are backed
    up after the next pass's descents."""
    m = MctsParams()
    m.continue_choice, m.vanilla, m.leaves_per_pass = continue_choice, vanilla, leaves_per_pass
    m.pipeline = pipeline
    m.iterations, m.playouts_per_leaf, m.max_depth = iterations, playouts_per_leaf, max_depth
    m.c_uct = float(np.float32(np.sqrt(2.0))) if c_uct is None else c_uct
    m.leaf_eval, m.fallback_band, m.fallback_playouts = leaf_eval, fallback_band, fallback_playouts
    if valuenet is not None:
        assert valuenet.dtype == np.float32 and valuenet.flags.c_contiguous
        m.valuenet = valuenet.ctypes.data
    else:
        m.valuenet = None
    return m


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def mulshift(w: int, k: int) -> int:
    return int(lib().oracle_mulshift(w, k))


def validate(state) -> int:
    s = _states(state)
    return int(lib().oracle_validate(_ptr(s)))


def unpack(state) -> dict:
    s = _states(state)
    r = Rows()
    rc = lib().oracle_unpack(_ptr(s), C.byref(r))
    if rc:
        raise ValueError(f"bad packed state (reason {rc})")
    return r.as_dict()


def pack(d: dict) -> np.ndarray:
    r = Rows()
    r.P = d["P"]
    for q in range(d["P"]):
        r.n[q] = len(d["rows"][q])
        for j, t in enumerate(d["rows"][q]):
            r.tile[q][j] = t
            r.rev[q][j] = d["rev"][q][j]
    r.pile_n = len(d["pile"])
    for j, t in enumerate(d["pile"]):
        r.pile[j] = t
    r.mover, r.phase, r.drawn = d["mover"], d["phase"], d["drawn"]
    out = np.zeros((1, 4), np.uint32)
    lib().oracle_pack(C.byref(r), _ptr(out))
    return out[0]


def playout(state, seed: int, p: int, leaf: int, tree: int, trace: bool = False):
    """One playout; returns (winner, length[, list of explicit states after each guess])."""
    s = _states(state)
    ln = C.c_int(0)
    if trace:
        buf = (Rows * 24)()
        nt = C.c_int(0)
        w = lib().oracle_playout(_ptr(s), seed, p, leaf, tree, C.byref(ln), buf, C.byref(nt))
        return w, ln.value, [buf[i].as_dict() for i in range(nt.value)]
    w = lib().oracle_playout(_ptr(s), seed, p, leaf, tree, C.byref(ln), None, None)
    return w, ln.value


def rollout(leaves, ppl: int, seed: int, tree_id: int = 0, leaf_id_base: int = 0,
            threads: int = 1, want_winner=True, want_length=True, want_wins=True):
    s = _states(leaves)
    n = s.shape[0]
    winner = np.zeros(n * ppl, np.int8) if want_winner else None
    length = np.zeros(n * ppl, np.int16) if want_length else None
    wins = np.zeros((n, 4), np.uint32) if want_wins else None
    if threads > 1:
        rc = lib().oracle_rollout_mt(_ptr(s), n, ppl, seed, tree_id, leaf_id_base, _ptr(winner),
                                     _ptr(length), _ptr(wins), threads)
    else:
        rc = lib().oracle_rollout(_ptr(s), n, ppl, seed, tree_id, leaf_id_base, _ptr(winner),
                                  _ptr(length), _ptr(wins))
    if rc:
        raise ValueError(f"oracle_rollout failed ({rc})")
    return winner, length, wins


def init_states(n: int, params: DealParams, seed: int, index_base: int = 0) -> np.ndarray:
    out = np.zeros((n, 4), np.uint32)
    rc = lib().oracle_init_states(_ptr(out), n, C.byref(params), seed, index_base)
    if rc:
        raise ValueError(f"oracle_init_states failed ({rc})")
    return out


def determinize(root, seed: int, tree: int, it: int):
    s = _states(root)
    out = np.zeros((1, 4), np.uint32)
    a = lib().oracle_determinize(_ptr(s), seed, tree, it, _ptr(out))
    if a < 0:
        raise ValueError(f"determinize failed ({a})")
    return out[0], a


def legal_actions(state) -> np.ndarray:
    s = _states(state)
    out = np.zeros(MAX_CHILD, np.uint8)
    rc = lib().oracle_legal_actions(_ptr(s), _ptr(out))
    if rc:
        raise ValueError(f"legal_actions failed ({rc})")
    return out


def apply_action(state, action: int, seed: int, tree: int, it: int, depth: int):
    s = _states(state)
    out = np.zeros((1, 4), np.uint32)
    term, win = C.c_int(0), C.c_int(-1)
    rc = lib().oracle_apply_action(_ptr(s), action, seed, tree, it, depth, _ptr(out),
                                   C.byref(term), C.byref(win))
    if rc:
        raise ValueError(f"apply_action failed ({rc})")
    return out[0], bool(term.value), win.value


def ln_entry(k: int) -> float:
    return float(lib().oracle_ln_entry(k))


def mcts_search(roots, params: MctsParams, seed: int, tree_id_base: int = 0):
    s = _states(roots)
    n = s.shape[0]
    best = np.zeros(n, np.int32)
    kids = np.zeros((n, MAX_CHILD), CHILD_DTYPE)
    rc = lib().oracle_mcts_search(_ptr(s), n, C.byref(params), seed, tree_id_base, _ptr(best),
                                  _ptr(kids))
    if rc:
        raise ValueError(f"oracle_mcts_search failed ({rc})")
    return best, kids


def mcts_search_merged(roots, trees_per_root: int, params: MctsParams, seed: int,
                       tree_id_base: int = 0):
    """Root-parallel search: (best [n], merged children [n, 864] indexed by action id)."""
    s = _states(roots)
    n = s.shape[0]
    best = np.zeros(n, np.int32)
    kids = np.zeros((n, MAX_CHILD), CHILD_DTYPE)
    rc = lib().oracle_mcts_search_merged(_ptr(s), n, trees_per_root, C.byref(params), seed,
                                         tree_id_base, _ptr(best), _ptr(kids))
    if rc:
        raise ValueError(f"oracle_mcts_search_merged failed ({rc})")
    return best, kids


TREE_NODE_DTYPE = np.dtype([("parent", np.int32), ("key", np.int32), ("chooser", np.int32),
                            ("depth", np.int32), ("n", np.uint32), ("w", np.float32),
                            ("world", np.uint64)])


def mcts_tree(root, params: MctsParams, seed: int, tree_id: int = 0):
    """(best action, every node of the searched tree in creation order as a
    TREE_NODE_DTYPE array: parent, key, chooser, depth, N, W, world key)."""
    s = _states(root)[:1]
    w_nodes = 2 * params.iterations + 1
    out = np.zeros(w_nodes, TREE_NODE_DTYPE)
    best = C.c_int32(0)
    n = lib().oracle_mcts_tree_dump(_ptr(s), C.byref(params), seed, tree_id, C.byref(best),
                                    _ptr(out), w_nodes)
    if n < 0:
        raise ValueError(f"oracle_mcts_tree_dump failed ({n})")
    return best.value, out[:n]


# ---------------------------------------------------------------------------
# value network
# ---------------------------------------------------------------------------
VN_NPARAM = 107265
VN_OFF = {"W1": (0, (256, 160)), "b1": (40960, (256,)), "W2": (41216, (256, 256)),
          "b2": (106752, (256,)), "w3": (107008, (256,)), "b3": (107264, (1,))}


def bf16(x: float) -> float:
    return float(lib().oracle_bf16(x))


def vn_encode(state, q: int) -> np.ndarray:
    s = _states(state)
    out = np.zeros(160, np.float32)
    rc = lib().oracle_vn_encode(_ptr(s), q, _ptr(out))
    if rc:
        raise ValueError(f"encode failed ({rc})")
    return out


def vn_init(seed: int) -> np.ndarray:
    p = np.zeros(VN_NPARAM, np.float32)
    lib().oracle_vn_init(_ptr(p), seed)
    return p


def vn_forward(params, states, persp, bf16_mirror: bool = False) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.float32)
    s = _states(states)
    q = np.ascontiguousarray(persp, dtype=np.int32)
    v = np.zeros(s.shape[0], np.float64)
    rc = lib().oracle_vn_forward(_ptr(p), _ptr(s), _ptr(q), s.shape[0], int(bf16_mirror), _ptr(v))
    if rc:
        raise ValueError(f"forward failed ({rc})")
    return v


def vn_loss_grad(params, states, persp, labels, bf16_mirror: bool = False,
                 want_abs: bool = False):
    """(loss, gradient), plus with want_abs the per-parameter sum of the
    absolute values of the gradient's per-row terms."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    s = _states(states)
    q = np.ascontiguousarray(persp, dtype=np.int32)
    y = np.ascontiguousarray(labels, dtype=np.float32)
    g = np.zeros(VN_NPARAM, np.float64)
    ga = np.zeros(VN_NPARAM, np.float64) if want_abs else None
    loss = C.c_double(0.0)
    rc = lib().oracle_vn_loss_grad(_ptr(p), _ptr(s), _ptr(q), _ptr(y), s.shape[0],
                                   int(bf16_mirror), C.byref(loss), _ptr(g), _ptr(ga))
    if rc:
        raise ValueError(f"loss_grad failed ({rc})")
    return (loss.value, g, ga) if want_abs else (loss.value, g)


def vn_adam(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (w, m, v, g):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().oracle_vn_adam(_ptr(w), _ptr(m), _ptr(v), _ptr(g), w.size, t, lr, b1, b2, eps)
