"""ctypes binding of librdcnn.so (the C ABI declared in include/rdcnn.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  If the library has not been built this module raises at import time;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librdcnn.so")

BC = {"periodic": 0, "zeroflux": 1}
PARAM_FIELDS = ("dt", "a", "b", "eps", "c", "k3", "Du", "Dv")

OK, EINVAL, EHIP, ENONFINITE, ESTATE, ENOMEM = 0, -1, -2, -3, -4, -5


class RDCNNError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rdcnn error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    """rdcnn_params_t: the paper's gene (dt, a, b, eps, c, Du, Dv) plus k3."""
    _fields_ = [(k, ctypes.c_float) for k in PARAM_FIELDS]

    @classmethod
    def from_mapping(cls, m) -> "Params":
        return cls(*[float(m[k]) for k in PARAM_FIELDS])


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2102_10340_amd.build`")

lib = ctypes.CDLL(LIB_PATH)

_I, _LL, _P, _F = ctypes.c_int, ctypes.c_longlong, ctypes.c_void_p, ctypes.c_float
_PP = ctypes.POINTER(ctypes.c_void_p)
_PAR = ctypes.POINTER(Params)
_PI = ctypes.POINTER(ctypes.c_int)

_SIGS = {
    "rdcnn_create": [_PP, _I, _I, _I, _PAR, _P, _F, _P, _P, _P],
    "rdcnn_model_create": [_PP, _I, _I, _I, _I, _P, _I, _P, _P, _P, _P, _P],
    "rdcnn_step": [_P, _LL],
    "rdcnn_use_graph": [_P, _I],
    "rdcnn_read": [_P, _P, _P, _I],
    "rdcnn_write_state": [_P, _P, _P],
    "rdcnn_set_params": [_P, _PAR],
    "rdcnn_current": [_P, _PP],
    "rdcnn_set_kernel": [_P, _I, _I, _I, _I],
    "rdcnn_pass_config": [_P, _PI, _PI, _PI, _PI],
    "rdcnn_destroy": [_P],
    "rdcnn_step_record": [_P, _LL, _P],
    "rdcnn_adjoint": [_P, _P, _LL, _P, _P, _P],
    "rdcnn_step_record_even": [_P, _LL, _P],
    "rdcnn_adjoint_even": [_P, _P, _LL, _P, _P, _P],
    "rdcnn_step_record_sparse": [_P, _LL, _P],
    "rdcnn_step_checkpoints": [_P, _LL, _LL, _P],
    "rdcnn_step_bwd": [_P, _P, _LL, _P, _P, _P],
    "rdcnn_step_bwd_noalloc": [_P, _P, _LL, _P, _P, _P],
    "rdcnn_step_bwd_ckpt": [_P, _P, _LL, _LL, _P, _P, _P, _P],
    "rdcnn_set_check_finite": [_P, _I],
    "rdcnn_set_adjoint_kernel": [_P, _I, _I, _I],
    "rdcnn_init_backward": [_P, _LL, _F, _P, _P],
    "rdcnn_set_grad_mask": [_P, ctypes.c_uint],
    "rdcnn_batch_create": [_PP, _I, _P, _P, _P, _P, _I, _P, _P, _F, _P, _P, _LL, _P],
    "rdcnn_batch_step": [_P, _LL],
    "rdcnn_batch_current": [_P, _PP],
    "rdcnn_batch_read": [_P, _P],
    "rdcnn_batch_set_check_finite": [_P, _I],
    "rdcnn_batch_set_shared_grad": [_P, _I],
    "rdcnn_batch_set_kernel": [_P, _I, _I, _I],
    "rdcnn_batch_set_class_seg_rows": [_P, _I, _I, _I],
    "rdcnn_batch_use_graph": [_P, _I],
    "rdcnn_batch_use_lds": [_P, _I],
    "rdcnn_batch_lds_instances": [_P, ctypes.POINTER(ctypes.c_int)],
    "rdcnn_batch_stats": [_P, _P, _P, _F, _F, _P],
    "rdcnn_batch_write_state": [_P, _P],
    "rdcnn_batch_step_record": [_P, _LL, _P],
    "rdcnn_batch_set_adjoint_kernel": [_P, _I, _I, _I],
    "rdcnn_batch_adjoint": [_P, _P, _LL, _P, _P, ctypes.c_uint, _P],
    "rdcnn_batch_step_record_even": [_P, _LL, _P],
    "rdcnn_batch_adjoint_even": [_P, _P, _LL, _P, _P, ctypes.c_uint, _P],
    "rdcnn_batch_destroy": [_P],
}
for _name, _args in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int
lib.rdcnn_last_error.argtypes = []
lib.rdcnn_last_error.restype = ctypes.c_char_p


def last_error() -> str:
    return (lib.rdcnn_last_error() or b"").decode()


def check(code: int) -> int:
    if code != OK:
        raise RDCNNError(code, last_error())
    return code
