"""ctypes declarations of libwqa.so (see include/wqa.h).  Loading fails loudly when the
library has not been built: there is no other implementation to fall back to."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libwqa.so")

MASS, STIFFNESS = 0, 1
F32, F64 = 0, 1
FINAL_PLAIN, FINAL_DOT2, FINAL_F64 = 0, 1, 2

STATUS = {0: "WQA_OK", -1: "WQA_EINVAL", -2: "WQA_ESTATE", -3: "WQA_EUNSUPPORTED",
          -4: "WQA_ERULE", -5: "WQA_EHIP", -6: "WQA_ENOMEM"}


class WQAError(RuntimeError):
    """A libwqa call returned an error status."""

    def __init__(self, status, message):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {message}")


if not os.path.exists(lib_path):
    raise ImportError(f"{lib_path} is missing: build it with `python paper_1710_01048_amd/build.py` "
                      "(hipcc, gfx950)")

lib = ctypes.CDLL(lib_path)

_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i64p = _P(ctypes.c_int64)
_dp = _P(ctypes.c_double)

_SIGS = {
    "wqa_abi_version": ([], ctypes.c_int),
    "wqa_last_error": ([], ctypes.c_char_p),
    "wqa_create": ([_P(_vp), ctypes.c_int], ctypes.c_int),
    "wqa_destroy": ([_vp], None),
    "wqa_set_space": ([_vp, ctypes.c_int, ctypes.c_int, _i64p], ctypes.c_int),
    "wqa_set_knots": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "wqa_set_default_rules": ([_vp], ctypes.c_int),
    "wqa_set_rules": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double], ctypes.c_int),
    "wqa_get_rules": ([_vp, ctypes.c_int, ctypes.c_int, _dp, _dp], ctypes.c_int),
    "wqa_get_tables": ([_vp, ctypes.c_int, ctypes.c_int, _dp], ctypes.c_int),
    "wqa_query": ([_vp, _i64p, _i64p, _i64p, _i64p], ctypes.c_int),
    "wqa_set_final_mode": ([_vp, ctypes.c_int], ctypes.c_int),
    "wqa_set_dispatch_limit": ([_vp, ctypes.c_int64], ctypes.c_int),
    "wqa_set_grid_pitch": ([_vp, ctypes.c_int64], ctypes.c_int),
    "wqa_set_sample_layout": ([_vp, ctypes.c_int], ctypes.c_int),
    "wqa_assemble_mass": ([_vp, ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
    "wqa_assemble_stiffness": ([_vp, ctypes.c_int, _P(_vp), _vp, _vp], ctypes.c_int),
    "wqa_assemble_fused": ([_vp, ctypes.c_int, _vp, _P(_vp), _vp, _vp, _vp], ctypes.c_int),
    "wqa_assemble_adjoint": ([_vp, ctypes.c_int, _vp, _vp, _vp, _P(_vp), _vp], ctypes.c_int),
    "wqa_assemble_load": ([_vp, ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
    "wqa_apply_mass": ([_vp, ctypes.c_int, _vp, _vp, _vp, _vp], ctypes.c_int),
    "wqa_apply_stiffness": ([_vp, ctypes.c_int, _P(_vp), _vp, _vp, _vp], ctypes.c_int),
}

for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTS = tuple(_SIGS)


def check(status):
    if status != 0:
        msg = lib.wqa_last_error()
        raise WQAError(status, msg.decode() if msg else "")
    return status
