"""ctypes mirror of include/rbffd.h (argument marshalling only)."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbffd.so")

OK, EINVAL, ESIZE, ESINGULAR, EHIP, EUNSTABLE, ESTATE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
MODE = {"FD": 0, "VFD": 1, "STAG2": 2}
BC = {"PEC": 0, "PERIODIC": 1}
ORDER = {"NONE": 0, "MORTON": 1, "RCM": 2}
DTYPE = {"f64": 0, "f32": 1, "bf16": 2}
W22 = 3            # weight storage (wdtype): compressed FP32 weights
OP_CURL_H, OP_HV_H, OP_CURL_E, OP_HV_E = 0, 1, 2, 3
ST_UNION, ST_CURL_H, ST_HV_H, ST_CURL_E, ST_HV_E = 0, 1, 2, 3, 4


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("mode", C.c_int32), ("n", C.c_int32), ("m", C.c_int32),
        ("phs_k", C.c_int32), ("hv_alpha", C.c_int32), ("n_hv", C.c_int32), ("bc", C.c_int32),
        ("reorder", C.c_int32), ("wdtype", C.c_int32), ("fdtype", C.c_int32), ("K", C.c_int32),
        ("adjoint", C.c_int32), ("pol", C.c_int32),
        ("vfd_sigma", C.c_double), ("hv_c", C.c_double), ("h", C.c_double), ("h_h", C.c_double),
        ("dt", C.c_double), ("eps0", C.c_double), ("mu0", C.c_double),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("frame_angle", C.c_double),
    ]


class Sizes(C.Structure):
    _fields_ = [
        ("N", C.c_int64), ("N_h", C.c_int64), ("n_stencil", C.c_int32), ("n_hv", C.c_int32),
        ("fe", C.c_int32), ("fh", C.c_int32), ("field_elem", C.c_int32), ("K", C.c_int32),
        ("arena_bytes", C.c_int64), ("workspace_bytes", C.c_int64), ("e_bytes", C.c_int64),
        ("h_bytes", C.c_int64), ("adjoint_ws_bytes", C.c_int64), ("dt", C.c_double), ("gamma", C.c_double),
    ]


class Fields(C.Structure):
    _fields_ = [("E", C.c_void_p * 2), ("H", C.c_void_p * 2), ("cur", C.c_int32), ("reserved", C.c_int32),
                ("eps_r", C.c_void_p)]


class RunArgs(C.Structure):
    _fields_ = [
        ("T", C.c_int32), ("energy_every", C.c_int32), ("energy_out", C.c_void_p),
        ("n_src", C.c_int32), ("n_rcv", C.c_int32), ("src_node", C.c_void_p), ("src_amp", C.c_void_p),
        ("src_wave", C.c_void_p), ("rcv_node", C.c_void_p), ("traces", C.c_void_p), ("ckpt", C.c_void_p),
        ("ckpt_every", C.c_int32), ("use_graph", C.c_int32), ("unstable_threshold", C.c_double),
        ("step0", C.c_int32), ("reserved", C.c_int32),
    ]


class AdjointArgs(C.Structure):
    _fields_ = [
        ("T", C.c_int32), ("ckpt_every", C.c_int32), ("ckpt", C.c_void_p), ("n_src", C.c_int32),
        ("n_rcv", C.c_int32), ("src_node", C.c_void_p), ("src_amp", C.c_void_p), ("src_wave", C.c_void_p),
        ("rcv_node", C.c_void_p), ("grad_traces", C.c_void_p), ("grad_eps", C.c_void_p),
        ("grad_amp", C.c_void_p), ("seg_buf", C.c_void_p), ("workspace", C.c_void_p),
    ]


class HvScanArgs(C.Structure):
    _fields_ = [
        ("E0", C.c_void_p), ("H0", C.c_void_p), ("c_lo", C.c_double), ("c_hi", C.c_double),
        ("rounds", C.c_int32), ("T", C.c_int32), ("energy_every", C.c_int32), ("reserved", C.c_int32),
        ("u_lo", C.c_double), ("u_hi", C.c_double), ("c_dev", C.c_void_p), ("energy_dev", C.c_void_p),
        ("c_host", C.c_void_p), ("umin_host", C.c_void_p), ("umax_host", C.c_void_p), ("ok_host", C.c_void_p),
        ("c_best", C.c_double), ("bracket", C.c_double * 2), ("rounds_done", C.c_int32), ("status", C.c_int32),
    ]


# name -> (restype, argtypes); the exported symbols of include/rbffd.h
PROTOTYPES = {
    "rbffd_plan_create": (C.c_int, [C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "rbffd_plan_sizes": (C.c_int, [C.c_void_p, C.POINTER(Sizes)]),
    "rbffd_set_wall_normals": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rbffd_plan_destroy": (None, [C.c_void_p]),
    "rbffd_strerror": (C.c_char_p, [C.c_int]),
    "rbffd_last_error": (C.c_char_p, [C.c_void_p]),
    "rbffd_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbffd_get_perm": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "rbffd_get_stencils": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "rbffd_get_weights": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "rbffd_set_weights": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "rbffd_permute": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                C.c_void_p]),
    "rbffd_step": (C.c_int, [C.c_void_p, C.POINTER(Fields), C.c_int32, C.c_void_p]),
    "rbffd_half": (C.c_int, [C.c_void_p, C.POINTER(Fields), C.c_int32, C.c_void_p]),
    "rbffd_run": (C.c_int, [C.c_void_p, C.POINTER(Fields), C.POINTER(RunArgs), C.c_void_p, C.c_void_p]),
    "rbffd_adjoint": (C.c_int, [C.c_void_p, C.POINTER(Fields), C.POINTER(AdjointArgs), C.c_void_p]),
    "rbffd_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "rbffd_compare": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p]),
    "rbffd_energy_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbffd_autotune": (C.c_int, [C.c_void_p, C.POINTER(Fields), C.c_int32, C.c_void_p]),
    "rbffd_autotune_cached": (C.c_int, [C.c_void_p, C.POINTER(Fields), C.c_int32, C.c_char_p,
                                        C.POINTER(C.c_int32), C.c_void_p]),
    "rbffd_get_variant": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "rbffd_set_variant": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "rbffd_set_field_hv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbffd_hv_scan": (C.c_int, [C.c_void_p, C.POINTER(Fields), C.POINTER(HvScanArgs), C.c_void_p, C.c_void_p]),
    "rbffd_stream_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
}

_lib = None


def load():
    """Load librbffd.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_18205_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class RbffdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rbffd error {code}: {msg}")
        self.code = code


def check(rc, plan=None, what=""):
    if rc != OK:
        lib = load()
        msg = lib.rbffd_strerror(rc).decode()
        if plan:
            detail = lib.rbffd_last_error(plan)
            if detail:
                msg += " -- " + detail.decode()
        raise RbffdError(rc, f"{what}: {msg}" if what else msg)
