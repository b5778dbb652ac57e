"""Measurement tools used by the benchmark, outside the engine's interface.

libvalu_probe.so (valu_probe.hip): the issue rate of each integer operation a
guess step is made of, the measured side of the integer roofline.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvalu_probe.so")
OPS = ["v_xor_b32", "v_add_u32", "v_mul_hi_u32", "v_mad_u64_u32", "v_bitop3_b32",
       "v_bcnt_u32_b32"]
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.valu_probe_launch.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def probe_valu(op: int, blocks: int, iters: int, sink, stream=None):
    """Launch `blocks` x 256 lanes, each iters * 64 operations `op` (index into
    OPS) in eight independent chains; sink: int32 device tensor [blocks * 256]."""
    import torch
    assert sink.is_cuda and sink.dtype == torch.int32 and sink.numel() == blocks * 256
    st = (stream or torch.cuda.current_stream()).cuda_stream
    rc = lib().valu_probe_launch(op, blocks, iters, C.c_void_p(sink.data_ptr()), C.c_void_p(st))
    if rc != 0:
        raise ValueError(f"valu_probe_launch failed ({rc})")
