"""ctypes loader for libprojprod.so and the argument types of its C ABI
(include/projprod.h).  No computation happens here."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprojprod.so")

PQ_F32, PQ_F64, PQ_BF16 = 0, 1, 2
PREC = {"default": 0, "fp32": 0, "fp64": 0, "bf16": 1, "bf16x3": 2, "bf16x6": 3}

_vp, _i64, _i32, _dbl, _sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                              ctypes.c_size_t)

# name -> (restype, argtypes), in the order of include/projprod.h
SIGNATURES = {
    "pq_version": (_i32, []),
    "pq_status_string": (ctypes.c_char_p, [_i32]),
    "pq_last_hip_error": (_i32, []),
    "pq_autotune_enable": (_i32, [_i32]),
    "pq_autotune_entries": (_i32, []),
    "pq_autotune_save": (_i32, [ctypes.c_char_p]),
    "pq_autotune_load": (_i32, [ctypes.c_char_p]),
    "pq_profile_enable": (_i32, [_i32]),
    "pq_profile_reset": (_i32, []),
    "pq_profile_query": (_i32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int)]),
    "pq_profile_names": (_i32, [ctypes.c_char_p, _sz]),
    "pq_check_q": (_i32, [_vp, _i32, _i64, _i64, _vp, _vp]),
    "pq_check_q_flag": (_i32, [_vp, _i32, _i64, _i64, _dbl, _vp, _vp, _vp]),
    "pq_hat": (_i32, [_vp, _i32, _vp, _vp, _i64, _i64, _i64, _i64, _i32, _vp]),
    "pq_unhat": (_i32, [_vp, _vp, _vp, _i32, _i64, _i64, _i64, _i64, _i32, _vp]),
    "pq_proj_workspace": (_sz, [_i64, _i64, _i64, _i64, _i32]),
    "pq_proj": (_i32, [_vp, _i32, _vp, _vp, _i64, _i64, _i64, _i64, _i32, _vp, _sz, _vp]),
    "pq_facewise": (_i32, [_vp, _vp, _vp, _i32, _i64, _i64, _i64, _i64, _i32, _vp]),
    "pq_qprod_workspace": (_sz, [_i64, _i64, _i64, _i64, _i64, _i32]),
    "pq_qprod": (_i32, [_vp, _vp, _i32, _vp, _vp, _i64, _i64, _i64, _i64, _i64, _i32, _vp, _vp,
                        _vp, _sz, _vp]),
    "pq_qprod_noalloc": (_i32, [_vp, _vp, _i32, _vp, _vp, _i64, _i64, _i64, _i64, _i64, _i32, _vp, _vp,
                                _vp]),
    "pq_qprod_backward_workspace": (_sz, [_i64, _i64, _i64, _i64, _i64, _i32]),
    "pq_qprod_backward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _i64, _i64, _i64,
                                 _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "pq_proj_backward_workspace": (_sz, [_i64, _i64, _i64, _i64, _i32]),
    "pq_proj_backward": (_i32, [_vp, _vp, _vp, _i32, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _sz,
                                _vp]),
    "pq_tsvdq_workspace": (_sz, [_i64, _i64, _i64, _i64, _i64, _i32]),
    "pq_tsvdq": (_i32, [_vp, _i32, _vp, _i64, _i64, _i64, _i64, _i64, _i32, _vp, _vp, _vp, _vp,
                        _vp, _vp, _vp, _dbl, _i32, _vp, _vp, _sz, _vp]),
    "pq_build_q": (_i32, [_i32, _i64, _i64, _i32, _vp, _vp]),
    "pq_relayout": (_i32, [_vp, _i32, _vp, _i32, _i64, _i64, _i64, _vp]),
    "pq_orthonormalize_q_workspace": (_sz, [_i64, _i64]),
    "pq_orthonormalize_q": (_i32, [_vp, _i32, _i64, _i64, _vp, _vp, _vp, _sz, _vp]),
    "pq_svdii_workspace": (_sz, [_i64, _i64, _i64, _i64, _i64, _i32]),
    "pq_svdii": (_i32, [_vp, _i32, _vp, _i64, _i64, _i64, _i64, _dbl, _i64, _i32, _vp, _vp, _vp, _vp,
                        _vp, _dbl, _i32, _vp, _vp, _sz, _vp]),
    "pq_tsvdq_backward_workspace": (_sz, [_i64, _i64, _i64, _i64, _i64, _i32]),
    "pq_tsvdq_backward": (_i32, [_vp, _i32, _vp, _i64, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _dbl,
                                 _dbl, _i32, _vp, _vp, _sz, _vp]),
    "pq_u3_workspace": (_sz, [_i64, _i64, _i64, _i64, _i32]),
    "pq_u3": (_i32, [_vp, _i32, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "pq_batched_workspace": (_i32, [_vp, _i32, _vp]),
    "pq_batched_plan": (_i32, [_vp, _i32, _i32, _dbl, _vp, _vp, _sz, _vp, _vp]),
    "pq_batched_run": (_i32, [_vp, _vp]),
    "pq_batched_destroy": (_i32, [_vp]),
}


class PQInstance(ctypes.Structure):
    """pq_instance of include/projprod.h."""
    _fields_ = [("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("n3", ctypes.c_int64),
                ("n4", ctypes.c_int64), ("p", ctypes.c_int64), ("k", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("Q", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("Uhat", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("Vhat", ctypes.c_void_p)]

_lib = None


class ProjProdError(RuntimeError):
    def __init__(self, fn, code):
        lib = load()
        msg = lib.pq_status_string(code).decode()
        if code == -9:
            msg += f" (hipError {lib.pq_last_hip_error()})"
        super().__init__(f"{fn}: {msg} [{code}]")
        self.code = code


def load():
    """Load the built library; fails loudly when it is missing (there is no
    fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built: run `python -m paper_2409_19402_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def call(name, *args):
    rc = getattr(load(), name)(*args)
    if rc != 0:
        raise ProjProdError(name, rc)
