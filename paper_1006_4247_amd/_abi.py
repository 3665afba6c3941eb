"""ctypes declarations of the C ABI in include/hsgpt.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsgpt.so")

HSG_OK = 0
HSG_ERR_INVALID = 1
HSG_ERR_DEVICE = 2
HSG_ERR_NUMERIC = 3
HSG_ERR_UNSUPPORTED = 4
HSG_FP64 = 0
HSG_FP32 = 1
HSG_TUNE_NO_RENORM = 1

_vp = ctypes.c_void_p


class HsgEnsemble(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("n_samples", ctypes.c_int32), ("n_chains", ctypes.c_int32),
        ("n_temps", ctypes.c_int32), ("precision", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("sample_base", ctypes.c_uint32), ("chain_base", ctypes.c_uint32),
        ("slot_base", ctypes.c_uint32), ("reserved1", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("spins", _vp), ("couplings", _vp), ("betas", _vp), ("temp_of_slot", _vp),
        ("slot_of_temp", _vp), ("energy", _vp), ("sweep_ctr", _vp), ("swap_ctr", _vp),
        ("swap_stats", _vp), ("rt_state", _vp), ("rt_trips", _vp), ("guard", _vp),
        ("anneal_K", _vp), ("anneal_lambda", _vp), ("anneal_K_max", ctypes.c_int32),
        ("reserved2", ctypes.c_int32), ("scratch", _vp), ("work", _vp),
        ("Q", _vp), ("chi", _vp), ("e_temp", _vp),
    ]


class HsgTuning(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("replicas_per_block", ctypes.c_int32), ("flags", ctypes.c_int32)]


# name -> (restype, argtypes); the list is also what the export test checks
_E = ctypes.POINTER(HsgEnsemble)
_fp = ctypes.POINTER(ctypes.c_float)
_i = ctypes.c_int
SIGNATURES = {
    "hsg_abi_version": (ctypes.c_int, []),
    "hsg_last_error": (ctypes.c_char_p, []),
    "hsg_scratch_bytes": (ctypes.c_size_t, [_E]),
    "hsg_init_couplings": (_i, [_E, _i, _vp]),
    "hsg_init_spins": (_i, [_E, _i, _i, _vp]),
    "hsg_sweep": (_i, [_E, _i, _i, _i, _i, _vp]),
    "hsg_sweep_tuned": (_i, [_E, _i, _i, _i, _i, ctypes.POINTER(HsgTuning), _vp]),
    "hsg_sweep_static": (_i, [_E, _i, _i, _i, _i, _vp]),
    "hsg_energy": (_i, [_E, _i, _vp, _vp]),
    "hsg_swap": (_i, [_E, _i, _i, _vp]),
    "hsg_anneal_swap": (_i, [_E, _i, _i, _i, _i, _vp]),
    "hsg_decimate_swap": (_i, [_E, _i, _i, _vp]),
    "hsg_coolheat_swap": (_i, [_E, _i, _i, ctypes.c_double, _vp]),
    "hsg_coolheat_swap_pairs": (_i, [_E, _i, _i, _vp, _vp]),
    "hsg_measure": (_i, [_E, _i, _vp]),
    "hsg_sweep_measure": (_i, [_E, _i, _i, _i, _i, _vp]),
    "hsg_check": (_i, [_E, _i, _vp]),
    "hsg_plan_create": (_i, [_E, _i, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "hsg_plan_run": (_i, [_vp, _i, _vp]),
    "hsg_plan_destroy": (_i, [_vp]),
    "hsg_plan_next_parity": (_i, [_vp]),
    "hsg_plan_set_next_parity": (_i, [_vp, _i]),
    "hsg_mlp_forward": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _vp, _vp]),
    "hsg_mlp_backward": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _vp, _vp, _vp]),
    "hsg_mlp_mse_grad": (_i, [_vp, _vp, _vp, _i, _i, _vp, _vp, _vp]),
    "hsg_mlp_adam": (_i, [_vp, _vp, _vp, _vp, _i, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float, _i, _vp]),
    "hsg_probe_issue": (_i, [_i, _i, _i, _i, _vp, _vp]),
}

_lib = None


class HsgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hsgpt error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libhsgpt.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhsgpt.so is not built (%s); run __graft_entry__.build() or "
                              "python paper_1006_4247_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != HSG_OK:
        msg = lib().hsg_last_error()
        raise HsgError(code, msg.decode() if msg else "")
    return code
