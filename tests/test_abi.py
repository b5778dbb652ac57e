"""Host-side checks of the C ABI library (no GPU needed).

* libdvc.so loads and exports every function include/dvc.h declares;
* status strings; argument errors are returned before any device work.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dvc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


@pytest.fixture(scope="module")
def lib():
    path = os.path.join(ROOT, "paper_2403_10720_amd", "libdvc.so")
    if not os.path.exists(path):
        from paper_2403_10720_amd import build
        build.build()
    return C.CDLL(path)


def test_header_declares_the_three_named_calls():
    names = declared_functions()
    for n in ["dvc_init_states", "dvc_rollout", "mcts_search"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    lib.dvc_status_str.restype = C.c_char_p
    assert lib.dvc_status_str(0) == b"ok"
    assert b"invalid" in lib.dvc_status_str(-1)
    assert b"malformed" in lib.dvc_status_str(-2)


def test_argument_errors_without_device(lib):
    vp = C.c_void_p
    lib.dvc_rollout_ex.argtypes = [vp, C.c_int64, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32,
                                   vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp]
    assert lib.dvc_rollout_ex(None, -1, 8, 0, 0, 0, None, None, None, 0, 0, 0, 0, None) == -1
    assert lib.dvc_rollout_ex(None, 4, 8, 0, 0, 0, None, None, None, 0, 0, 0, 0, None) == -1
    assert lib.dvc_rollout_ex(None, 0, 0, 0, 0, 0, None, None, None, 0, 0, 0, 0, None) == -1
    # unknown flag
    assert lib.dvc_rollout_ex(vp(16), 1, 8, 0, 0, 0, None, None, None, 0, 0, 0, 2, None) == -1
    # kernel variants 0-9 exist; 10 and negative ones do not; variant 9 takes
    # one or two 256-playout batches per workgroup
    for bad in (10, -1):
        assert lib.dvc_rollout_ex(vp(16), 1, 8, 0, 0, 0, None, None, None, bad, 0, 0, 0,
                                  None) == -1
    assert lib.dvc_rollout_ex(vp(16), 1, 8, 0, 0, 0, None, None, None, 9, 0, 3, 0, None) == -1
    # n * ppl must stay below 2^32
    assert lib.dvc_rollout_ex(vp(16), 1 << 20, 1 << 12, 0, 0, 0, None, None, None, 0, 0, 0, 0,
                              None) == -1
    lib.dvc_init_states.argtypes = [vp, C.c_int64, vp, C.c_uint64, C.c_uint32, vp]
    assert lib.dvc_init_states(None, -1, None, 0, 0, None) == -1


def test_root_parallel_argument_errors_without_device(lib):
    import paper_2403_10720_amd as D
    vp = C.c_void_p
    mp = D.mcts_params(iterations=10, playouts_per_leaf=4)
    lib.mcts_search_root_parallel.argtypes = [vp, C.c_int64, C.c_int32, C.POINTER(D.MctsParams),
                                              C.c_uint64, C.c_uint32, vp, C.c_size_t, vp, vp, vp]
    # no trees per root, negative roots, null buffers
    assert lib.mcts_search_root_parallel(vp(16), 2, 0, C.byref(mp), 1, 0, vp(16), 1 << 20, vp(16),
                                         None, None) == -1
    assert lib.mcts_search_root_parallel(vp(16), -1, 2, C.byref(mp), 1, 0, vp(16), 1 << 20,
                                         vp(16), None, None) == -1
    assert lib.mcts_search_root_parallel(None, 2, 2, C.byref(mp), 1, 0, vp(16), 1 << 20, vp(16),
                                         None, None) == -1
    # misaligned workspace
    assert lib.mcts_search_root_parallel(vp(16), 1, 1, C.byref(mp), 1, 0, vp(20), 1 << 30, vp(16),
                                         None, None) == -1


def test_autotune_argument_errors_without_device(lib):
    vp = C.c_void_p
    lib.dvc_rollout_autotune.argtypes = [vp, C.c_int64, C.c_int32, C.c_uint64, C.c_uint32,
                                         C.c_uint32, vp, vp, vp, vp, vp]
    assert lib.dvc_rollout_autotune(vp(16), 0, 8, 0, 0, 0, None, None, None, None, None) == -1
    assert lib.dvc_rollout_autotune(None, 4, 8, 0, 0, 0, None, None, None, None, None) == -1
    assert lib.dvc_rollout_autotune(vp(16), 4, 0, 0, 0, 0, None, None, None, None, None) == -1


def test_valuenet_alignment_errors_without_device(lib):
    vp = C.c_void_p
    lib.dvc_valuenet_init.argtypes = [vp, C.c_uint64, vp]
    lib.dvc_valuenet_infer.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
    # misaligned blobs are rejected before any device work
    assert lib.dvc_valuenet_init(vp(8), 1, None) == -1
    assert lib.dvc_valuenet_infer(vp(24), vp(16), vp(16), 4, vp(16), None) == -1


def test_tree_variant_parameters_without_device(lib):
    """Workspace sizes of the un-simplified variants (host-only), parameter
    ranges (pipelined passes keep no world nodes: not with vanilla), and
    vanilla trees refused by the root-parallel search."""
    import paper_2403_10720_amd as D
    vp = C.c_void_p
    lib.dvc_mcts_workspace_bytes.restype = C.c_size_t
    lib.dvc_mcts_workspace_bytes.argtypes = [C.c_int64, C.POINTER(D.MctsParams)]
    size = lambda **kw: lib.dvc_mcts_workspace_bytes(3, C.byref(D.mcts_params(iterations=100, **kw)))
    base, cont, van = size(), size(continue_choice=1), size(vanilla=1)
    assert base > 0 and cont > base and van > base
    assert base % 16 == 0 and cont % 16 == 0 and van % 16 == 0
    assert size(max_depth=0) == base and size(max_depth=64) == base
    for bad in (dict(max_depth=65), dict(max_depth=-1), dict(continue_choice=2), dict(vanilla=3),
                dict(leaves_per_pass=0), dict(leaves_per_pass=17), dict(pipeline=2),
                dict(pipeline=-1), dict(pipeline=1, vanilla=1)):
        assert size(**bad) == 0
    assert size(leaves_per_pass=16) == base
    assert size(pipeline=1) == base and size(pipeline=1, leaves_per_pass=16) == base
    mp = D.mcts_params(iterations=10, playouts_per_leaf=4, vanilla=1)
    lib.mcts_search_root_parallel.argtypes = [vp, C.c_int64, C.c_int32, C.POINTER(D.MctsParams),
                                              C.c_uint64, C.c_uint32, vp, C.c_size_t, vp, vp, vp]
    assert lib.mcts_search_root_parallel(vp(16), 1, 2, C.byref(mp), 1, 0, vp(16), 1 << 30, vp(16),
                                         None, None) == -1


def test_epoch_order_is_the_philox_stream(lib, orc):
    """dvc_valuenet_epoch_order (host only) takes words 0 and 1 of the Philox
    block (epoch, 0xFFFFFFFD, 0, 0): checked against the oracle's Philox, and
    the resulting map is a bijection of the rows."""
    import numpy as np
    u32 = C.c_uint32
    lib.dvc_valuenet_epoch_order.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.POINTER(u32),
                                             C.POINTER(u32)]
    for seed in (4, 2**40 + 17):
        for epoch in (0, 1, 19, 2**32 - 1):
            for n in (1, 2, 1024, 2**23, 2**32):
                a, b = u32(7), u32(7)
                assert lib.dvc_valuenet_epoch_order(seed, epoch, n, C.byref(a), C.byref(b)) == 0
                w = orc.philox([epoch, 0xFFFFFFFD, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
                if n == 1:
                    assert (a.value, b.value) == (1, 0)
                else:
                    assert a.value == (int(w[0]) | 1) % n and a.value % 2 == 1
                    assert b.value == int(w[1]) % n
                if n == 1024:
                    rows = (a.value * np.arange(n, dtype=np.int64) + b.value) % n
                    assert len(set(rows.tolist())) == n
    a, b = u32(), u32()
    assert lib.dvc_valuenet_epoch_order(4, 0, 3, C.byref(a), C.byref(b)) == -1
    assert lib.dvc_valuenet_epoch_order(4, -1, 4, C.byref(a), C.byref(b)) == -1
    assert lib.dvc_valuenet_epoch_order(4, 0, 2**33, C.byref(a), C.byref(b)) == -1
    assert lib.dvc_valuenet_epoch_order(4, 0, 4, None, C.byref(b)) == -1


def test_search_autotune_argument_errors_without_device(lib):
    """Value leaves, several leaves per pass or pipelined passes in the
    reference, no trees or a negative tolerance are refused before any device
    work; automatic shapes (playouts per leaf, leaves per pass and pipeline
    all 0) have a workspace size, a pipelined one with no shape has none."""
    import paper_2403_10720_amd as D
    L = D.lib()
    vp = C.c_void_p
    ok = D.mcts_params(iterations=64, playouts_per_leaf=8)
    auto = D.mcts_params(iterations=64, playouts_per_leaf=0, leaves_per_pass=0)
    assert L.dvc_mcts_workspace_bytes(4, C.byref(auto)) == L.dvc_mcts_workspace_bytes(4, C.byref(ok)) > 0
    half = D.mcts_params(iterations=64, playouts_per_leaf=0, leaves_per_pass=1)
    assert L.dvc_mcts_workspace_bytes(4, C.byref(half)) == 0
    big = D.mcts_params(iterations=1 << 17, playouts_per_leaf=0, leaves_per_pass=0)
    assert L.dvc_mcts_workspace_bytes(4, C.byref(big)) == 0
    res = D.MctsTuning()
    pipe_auto = D.mcts_params(iterations=64, playouts_per_leaf=0, leaves_per_pass=0, pipeline=1)
    assert L.dvc_mcts_workspace_bytes(4, C.byref(pipe_auto)) == 0
    for mp, n, tol in [(D.mcts_params(iterations=64, playouts_per_leaf=8, leaves_per_pass=2), 4, 0.0),
                       (D.mcts_params(iterations=64, playouts_per_leaf=8, pipeline=1), 4, 0.0),
                       (ok, 0, 0.0), (ok, 4, -0.1), (auto, 4, 0.0),
                       (D.mcts_params(iterations=64, playouts_per_leaf=8, leaf_eval=1), 4, 0.0)]:
        assert L.dvc_mcts_autotune(vp(16), n, C.byref(mp), 1, 0, vp(16), 1 << 30, tol, vp(16),
                                   C.byref(res), None) == -1


def test_kernels_use_no_scratch(lib, tmp_path):
    """Every kernel of the library runs without private (scratch) memory: no
    register spills, so a launch needs no scratch allocation by the runtime
    (the allocation-free search relies on it).  Read from the gfx950 code
    object's metadata, extracted from the built library."""
    import shutil
    import subprocess
    tools = "/opt/rocm/llvm/bin"
    objdump, readelf = os.path.join(tools, "llvm-objdump"), os.path.join(tools, "llvm-readelf")
    if not (os.path.exists(objdump) and os.path.exists(readelf)):
        pytest.skip("llvm-objdump / llvm-readelf not installed")
    import paper_2403_10720_amd as D
    so = tmp_path / "libdvc.so"
    shutil.copy(D.LIB_PATH, so)
    subprocess.run([objdump, "--offloading", str(so)], cwd=tmp_path, check=True,
                   capture_output=True)
    co = [p for p in tmp_path.iterdir() if "amdgcn" in p.name and "gfx950" in p.name]
    assert len(co) == 1, list(tmp_path.iterdir())
    notes = subprocess.run([readelf, "--notes", str(co[0])], check=True, capture_output=True,
                           text=True).stdout
    kernels, name = {}, None
    for line in notes.splitlines():
        line = line.strip()
        if line.startswith(".name:"):
            name = line.split(":", 1)[1].strip()
        elif line.startswith(".private_segment_fixed_size:") and name is not None:
            kernels[name] = int(line.split(":", 1)[1])
            name = None
    assert any("mcts_tree_kernel" in k for k in kernels) and any("rollout" in k for k in kernels)
    assert {k: v for k, v in kernels.items() if v} == {}
