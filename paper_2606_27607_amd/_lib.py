"""ctypes declarations of the C ABI in include/hipphylo.h (argument marshalling only).

The shared library is loaded after torch so that it binds to the HIP runtime torch
already loaded (both carry the soname libamdhip64.so.7); device memory and streams
handed to the library therefore come from the same runtime.  There is no fallback:
if the library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhipphylo.so")

HP_OK = 0
HP_ERR_ARG = -1
HP_ERR_INDEX = -2
HP_ERR_VALUE = -3
HP_ERR_UNSUPPORTED = -4
HP_ERR_WORKSPACE = -5
HP_ERR_STATE = -6
HP_ERR_DEVICE = -7
HP_ERR_NUMERIC = -8
ERROR_NAMES = {
    HP_ERR_ARG: "HP_ERR_ARG", HP_ERR_INDEX: "HP_ERR_INDEX", HP_ERR_VALUE: "HP_ERR_VALUE",
    HP_ERR_UNSUPPORTED: "HP_ERR_UNSUPPORTED", HP_ERR_WORKSPACE: "HP_ERR_WORKSPACE",
    HP_ERR_STATE: "HP_ERR_STATE", HP_ERR_DEVICE: "HP_ERR_DEVICE", HP_ERR_NUMERIC: "HP_ERR_NUMERIC",
}

PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16x3": 4}
SCALINGS = {"none": 0, "every_node": 1, "every_k": 2}


def default_scaling(n_states: int, precision: str):
    """The rescaling policy used for a state space and precision, as (scaling, period):
    every node for FP16 partials (5-bit exponent) and for more than 64 states (the
    eigensystem path, whose single-pattern partials shrink by about 1/S per tip), otherwise
    every 4 levels: FP32, BF16 and FP64 keep 8 or more exponent bits, and between rescaled
    nodes a partial combines at most 2^4 tips."""
    if precision == "f16" or n_states > 64:
        return ("every_node", 1)
    return ("every_k", 4)

HP_Q_STATE_PAD = 1
HP_Q_PATTERN_PAD = 2
HP_Q_ELEMENT_BYTES = 3
HP_Q_BLOCKS = 4
HP_Q_RUNTIME_VERSION = 5
HP_Q_TILE = 6


class hp_desc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "n_tips", "n_patterns", "n_states", "n_categories", "n_partials", "n_matrices", "n_eigen",
        "precision", "scaling", "scale_period", "device", "n_pre_partials", "flags")]


HP_FLAG_QPOST_CACHE = 1


POST_OP_FIELDS = ("dest", "child1", "mat1", "child2", "mat2", "rescale")
PRE_OP_FIELDS = ("parent_pre", "child1_post", "mat1", "child1_pre", "grad1",
                 "child2_post", "mat2", "child2_pre", "grad2")

# name -> (restype, argtypes); every function returns int
_P = ctypes.c_void_p
_I = ctypes.c_int
SIGNATURES = {
    "hp_workspace_bytes": [ctypes.POINTER(hp_desc), ctypes.POINTER(ctypes.c_size_t)],
    "hp_create": [ctypes.POINTER(hp_desc), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "hp_destroy": [_P],
    "hp_set_stream": [_P, _P],
    "hp_last_error": [_P, ctypes.c_char_p, ctypes.c_size_t],
    "hp_query": [_P, _I, ctypes.POINTER(ctypes.c_int64)],
    "hp_set_tip_states": [_P, _I, _P, _I],
    "hp_set_pattern_weights": [_P, _P],
    "hp_set_frequencies": [_P, _I, _P],
    "hp_set_category_rates": [_P, _P],
    "hp_set_category_weights": [_P, _I, _P],
    "hp_set_eigen": [_P, _I, _P, _P, _P],
    "hp_update_matrices": [_P, _I, _P, _P, _I],
    "hp_update_post": [_P, _P, _I],
    "hp_root_lnl": [_P, _I, _I, _I, _P, _P],
    "hp_root_lnl_device": [_P, _I, _I, _I, _P, _P],
    "hp_update_pre": [_P, _P, _I, _I],
    "hp_pre_gradients": [_P, _P, _I, _I, _I, _I, _P, _I],
    "hp_pre_gradients_device": [_P, _P, _I, _I, _I, _I, _P, _I],
    "hp_traverse_gradients_device": [_P, _P, _I, _I, _I, _I, _P, _I],
    "hp_set_tree": [_P, _P],
    "hp_plan_tree": [_I, _P, _I, _I, _P, _P],
    "hp_plan_pre_buffers": [_I, _P, ctypes.POINTER(ctypes.c_int)],
    "hp_evaluate": [_P, _P, _I, _P, _P],
    "hp_evaluate_device": [_P, _P, _I, _P],
    "hp_evaluate_device_noalloc": [_P, _P, _I, _P],
    "hp_gradients_device": [_P, _P],
    "hp_evaluate_rate_gradient": [_P, _P, _P, _P, _P],
    "hp_evaluate_rate_gradient_device": [_P, _P, _P],
    "hp_batch_evaluate_device": [_P, _P, _P, _I, _I, _P],
    "hp_status": [_P],
    "hp_profile": [_P, _I],
    "hp_profile_read": [_P, _P, _P],
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhipphylo.so (after torch) and declare every entry point; raises if absent."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or "
                           "python -m paper_2606_27607_amd.build")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


class HPError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code
        self.message = message


def last_error(lib, inst) -> str:
    buf = ctypes.create_string_buffer(1024)
    lib.hp_last_error(inst, buf, len(buf))
    return buf.value.decode(errors="replace")


def check(lib, rc: int, inst=None) -> int:
    if rc != HP_OK:
        raise HPError(rc, last_error(lib, inst))
    return rc


def plan_tree(children, scaling: str = "every_k", scale_period: int = 4):
    """The library's operation lists for a children table: post [N-1, 6] (post-order,
    children first, with the rescale flags of the policy) and pre [N-1, 9] (parents first)."""
    import numpy as np
    lib = load()
    ch = np.ascontiguousarray(np.asarray(children, dtype=np.int32))
    n = (ch.shape[0] + 1) // 2
    post = np.zeros((n - 1, 6), dtype=np.int32)
    pre = np.zeros((n - 1, 9), dtype=np.int32)
    check(lib, lib.hp_plan_tree(n, ctypes.c_void_p(ch.ctypes.data), SCALINGS[scaling], int(scale_period),
                                ctypes.c_void_p(post.ctypes.data), ctypes.c_void_p(pre.ctypes.data)))
    return post, pre


def plan_pre_buffers(children) -> int:
    """Pre-order buffers the whole-tree operation lists need for this children table."""
    import numpy as np
    lib = load()
    ch = np.ascontiguousarray(np.asarray(children, dtype=np.int32))
    n = ctypes.c_int()
    check(lib, lib.hp_plan_pre_buffers((ch.shape[0] + 1) // 2, ctypes.c_void_p(ch.ctypes.data),
                                       ctypes.byref(n)))
    return n.value

