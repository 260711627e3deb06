"""ctypes declarations of the C ABI in include/dec.h (argument marshalling only).

Loading fails loudly when libdec_hip.so has not been built: there is no
fallback implementation of any step.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdec_hip.so")

c_int = ctypes.c_int
c_i8p = ctypes.c_void_p
vp = ctypes.c_void_p
i64 = ctypes.c_int64
i64p = ctypes.POINTER(ctypes.c_int64)
dp = ctypes.POINTER(ctypes.c_double)

DEC_OK = 0
STATUS = {0: "DEC_OK", -1: "DEC_EINVAL", -2: "DEC_ENOMEM", -3: "DEC_EHIP", -4: "DEC_ENOTCONV",
          -5: "DEC_EBREAKDOWN", -6: "DEC_ETOPO", -7: "DEC_EBUDGET", -8: "DEC_ESTATE", -9: "DEC_ECANCELED"}
DEC_PREC_FP64, DEC_PREC_MIXED = 0, 1
DEC_PRECOND_JACOBI, DEC_PRECOND_FSAI, DEC_PRECOND_BLOCK = 0, 1, 2
DEC_FMT_AUTO, DEC_FMT_CSR, DEC_FMT_SELL = 0, 1, 2
DEC_NORM_RESIDUAL, DEC_NORM_ENERGY = 0, 1
DEC_NOALLOC_MAX_ROWS = 4194304

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("adaptive_final_inner", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
        ("max_iters", ctypes.c_int64),
        ("format", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("norm", ctypes.c_int32),
    ]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int64),
        ("outer_iterations", ctypes.c_int64),
        ("restarts", ctypes.c_int64),
        ("fp64_fallback", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("spmv_launches", ctypes.c_int64),
        ("spmv_ms", ctypes.c_double),
        ("spmv_bytes", ctypes.c_double),
        ("spmv_nnz", ctypes.c_int64),
        ("plain_residual", ctypes.c_double),
        ("spmv_unroll", ctypes.c_int32),
        ("spmv_nontemporal", ctypes.c_int32),
        ("spmv_col_bytes", ctypes.c_int32),
        ("spmv_band", ctypes.c_int32),
        ("spmv_order", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerCounters(ctypes.Structure):
    _fields_ = [
        ("batch_ms", ctypes.c_double),
        ("batch_bytes", ctypes.c_double),
        ("batch_iterations", ctypes.c_int64),
        ("variant", ctypes.c_int32 * 4),
        ("host_ms", ctypes.c_double * 4),
        ("steps", ctypes.c_int64),
        ("order", ctypes.c_int32 * 2),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_int64), ("xyz", vp), ("T", ctypes.c_int64), ("tets", vp), ("kappa", vp),
        ("n_cracks", ctypes.c_int32), ("cracks", vp), ("bc_type", vp), ("bc_value", vp), ("neumann_f0", vp),
        ("side", vp), ("length", ctypes.c_double), ("area", ctypes.c_double), ("dT", ctypes.c_double),
        ("T_out", vp), ("user_tag", ctypes.c_uint64), ("T0", vp), ("mesh", vp),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64), ("user_tag", ctypes.c_uint64), ("status", ctypes.c_int32),
        ("fp64_fallback", ctypes.c_int32), ("k_eff", ctypes.c_double), ("q_in", ctypes.c_double), ("q_out", ctypes.c_double),
        ("energy", ctypes.c_double), ("rel_residual", ctypes.c_double), ("inner_iterations", ctypes.c_int64),
        ("outer_iterations", ctypes.c_int64), ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
        ("t_start_ms", ctypes.c_double), ("t_finish_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double), ("adaptive_final_inner", ctypes.c_int32), ("chunk", ctypes.c_int32),
        ("max_iters", ctypes.c_int64),
    ]


# name -> (restype, argtypes); every entry point declared in include/dec.h
SIGNATURES = {
    "dec_create": (c_int, [ctypes.POINTER(vp), c_int, vp, ALLOC_FN, FREE_FN, vp]),
    "dec_destroy": (c_int, [vp]),
    "dec_status_string": (ctypes.c_char_p, [c_int]),
    "dec_last_error": (ctypes.c_char_p, [vp]),
    "dec_build_topology": (c_int, [vp, i64, vp, i64, vp, ctypes.POINTER(vp)]),
    "dec_mesh_info": (c_int, [vp, i64p, i64p, i64p, i64p, i64p, i64p]),
    "dec_get_edges": (c_int, [vp, vp]),
    "dec_get_csr": (c_int, [vp, vp, vp, vp, vp]),
    "dec_mesh_destroy": (c_int, [vp]),
    "dec_hodge1": (c_int, [vp, vp, ctypes.c_int32, vp, vp, vp]),
    "dec_assemble": (c_int, [vp, ctypes.c_uint32]),
    "dec_apply_bc": (c_int, [vp, vp, vp, vp, i64p, vp]),
    "dec_solve_opts_default": (c_int, [ctypes.POINTER(SolveOpts)]),
    "dec_solve": (c_int, [vp, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveStats)]),
    "dec_solve_noalloc": (c_int, [vp, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveStats)]),
    "dec_spmv": (c_int, [vp, ctypes.c_int32, ctypes.c_int32, vp, vp]),
    "dec_get_fsai": (c_int, [vp, i64p, vp, vp, vp]),
    "dec_flux_effective_conductivity": (c_int, [vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                dp, dp, dp, dp, vp]),
    "dec_max_flux_edge": (c_int, [vp, vp, vp, ctypes.POINTER(ctypes.c_int64), dp]),
    "dec_dual_build": (c_int, [vp, vp, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(vp),
                               ctypes.POINTER(ctypes.c_int64)]),
    "dec_dual_faces": (c_int, [vp, vp, vp, vp, vp]),
    "dec_dual_info": (c_int, [vp] + [ctypes.POINTER(ctypes.c_int64)] * 4),
    "dec_rms_error": (c_int, [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_double), dp]),
    "dec_reorder": (c_int, [vp, ctypes.c_int32, ctypes.c_int64, vp, ctypes.c_int64, vp, vp, vp, vp, vp]),
    "dec_tetgen_read": (c_int, [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64), vp, vp, vp]),
    "dec_dual_flux": (c_int, [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]),
    "dec_server_opts_default": (c_int, [ctypes.POINTER(ServerOpts)]),
    "dec_server_create": (c_int, [vp, ctypes.c_size_t, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]),
    "dec_server_submit": (c_int, [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "dec_server_step": (c_int, [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "dec_server_poll": (c_int, [vp, ctypes.POINTER(Result), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "dec_server_cancel": (c_int, [vp, ctypes.c_uint64]),
    "dec_server_stats": (c_int, [vp, vp]),
    "dec_server_destroy": (c_int, [vp]),
}

_LIB = None


def load():
    """Load libdec_hip.so (raises when it is missing: build it with __graft_entry__.build())."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
