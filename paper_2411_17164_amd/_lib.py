"""ctypes binding of libxmgn.so (the C ABI in include/xmgn.h).

Argument marshalling only: every computation runs in the library.  Importing
this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
# XMGN_LIB selects another build of the library (e.g. an instrumented one)
LIB_PATH = os.environ.get("XMGN_LIB") or os.path.join(_HERE, "libxmgn.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "xmgn.h")

XMGN_OK = 0
ERRORS = {-1: "INVALID", -2: "OOM", -3: "HIP", -4: "CAPACITY", -5: "UNSUPPORTED", -6: "STATE"}


class XmgnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"xmgn error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("n_layers", C.c_int32), ("node_in", C.c_int32),
                ("edge_in", C.c_int32), ("out_dim", C.c_int32), ("activation", C.c_int32),
                ("precision", C.c_int32), ("aggregate", C.c_int32), ("ln_eps", C.c_float)]


_p = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_pi32 = C.POINTER(C.c_int32)
_pi64 = C.POINTER(C.c_int64)
_pf = C.POINTER(C.c_float)
_pdesc = C.POINTER(Desc)

_SIGS = {
    "xmgn_last_error": (C.c_char_p, []),
    "xmgn_version": (C.c_char_p, []),
    "xmgn_param_count": (_i32, [_pdesc, _pi64]),
    "xmgn_param_offset": (_i32, [_pdesc, _i32, _i32, _i32, _pi64]),
    "xmgn_ctx_create": (_i32, [_i32, C.POINTER(_p)]),
    "xmgn_ctx_destroy": (None, [_p]),
    "xmgn_ctx_set_tiles": (_i32, [_p, _i32, _i32, _i32, _i32]),
    "xmgn_ctx_set_bwd_tiles": (_i32, [_p, _i32, _i32]),
    "xmgn_ctx_get_bwd_tiles": (_i32, [_p, _pi32, _pi32]),
    "xmgn_ctx_memory": (_i32, [_p, _pi64]),
    "xmgn_ctx_tape_serial": (_i32, [_p, _pi64]),
    "xmgn_ctx_set_tape": (_i32, [_p, _i32]),
    "xmgn_ctx_get_tape": (_i32, [_p, _pi32]),
    "xmgn_ctx_set_edge_split": (_i32, [_p, _i32]),
    "xmgn_ctx_get_edge_split": (_i32, [_p, _pi32]),
    "xmgn_ctx_host_memory": (_i32, [_p, _pi64]),
    "xmgn_ctx_set_offload": (_i32, [_p, _i32]),
    "xmgn_ctx_set_timing": (_i32, [_p, _i32]),
    "xmgn_ctx_timing_count": (_i32, [_p, _pi32]),
    "xmgn_ctx_timing_read": (_i32, [_p, _i32, C.c_char_p, _i32, C.POINTER(C.c_double), _pi64]),
    "xmgn_build_knn": (_i32, [_p, _p, _i32, _pi32, _i32, _i32, _i32, C.POINTER(_p), _p]),
    "xmgn_graph_from_csr": (_i32, [_i32, _pi32, _pi32, C.POINTER(_p)]),
    "xmgn_graph_info": (_i32, [_p, _pi32, _pi64]),
    "xmgn_graph_export": (_i32, [_p, _pi32, _pi32]),
    "xmgn_graph_destroy": (None, [_p]),
    "xmgn_partition_halo": (_i32, [_p, _pf, _i32, _pi32, _i32, C.POINTER(_p)]),
    "xmgn_partition_explicit": (_i32, [_p, _i32, _pi32, _pi32, _i32, C.POINTER(_p)]),
    "xmgn_partset_count": (_i32, [_p, _pi32, _pi32]),
    "xmgn_partset_info": (_i32, [_p, _i32, _pi32, _pi32, _pi64]),
    "xmgn_partset_export": (_i32, [_p, _i32, _pi32, _pi32, _pi32, _pi32]),
    "xmgn_partset_destroy": (None, [_p]),
    "xmgn_forward": (_i32, [_p, _pdesc, _p, _p, _pi32, _i32, _p, _p, _pf, _p, _i32, _p]),
    "xmgn_mse_grad": (_i32, [_p, _p, _p, _i64, _p, _p, _p]),
    "xmgn_backward": (_i32, [_p, _pdesc, _p, _p, _p, _p]),
    "xmgn_grad_accumulate": (_i32, [_p, _p, _i64, _p]),
    "xmgn_adam_step": (_i32, [_p, _p, _p, _p, _p, _i64, _i64, C.c_double, C.c_double, C.c_double, C.c_double,
                              C.c_double, _p, _p]),
    "xmgn_adam_step_noalloc": (_i32, [_i32, _p, _p, _p, _p, _i64, _i64, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _p, _p]),
    "xmgn_cosine_lr": (C.c_double, [_i64, _i64, C.c_double, C.c_double]),
    "xmgn_autotune": (_i32, [_p, _pdesc, _p, _p, _pi32, _i32, _p, _p, _pf, _p, _p, _p, C.c_char_p,
                             _pi32, _pi32, _pi32, _pi32, _pf, _p]),
}


def header_functions() -> list[str]:
    """Names of every function declared in include/xmgn.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xmgn_[a-z0-9_]+)\s*\(", src)))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_17164_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(code: int) -> None:
    if code != XMGN_OK:
        raise XmgnError(code, lib.xmgn_last_error().decode())
