"""ctypes binding of libpfem.so: the C ABI declared in include/pfem.h.

Argument marshalling only.  Every function here has the C name and
signature; nothing computes.  Importing this module fails loudly when the
HIP library has not been built: there is no fallback path.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfem.so")

# status codes
PFEM_OK = 0
PFEM_NOT_CONVERGED = 1
PFEM_SKIPPED_FINE = 2
PFEM_E_INVALID_ARG = -1
PFEM_E_INVALID_MESH = -2
PFEM_E_OOM = -3
PFEM_E_DEVICE = -4
PFEM_E_BREAKDOWN = -5
PFEM_E_INVERTED = -6
PFEM_E_LINESEARCH = -7
PFEM_E_CANCELLED = -8
PFEM_E_STATE = -9
# models
PFEM_LIN_PLANE_STRESS, PFEM_LIN_PLANE_STRAIN, PFEM_LIN_3D = 0, 1, 2
PFEM_NH_PLANE_STRAIN, PFEM_NH_3D = 3, 4
PFEM_PARAM_E_NU, PFEM_PARAM_LAME = 0, 1
PFEM_FP64, PFEM_FP32 = 0, 1
PFEM_KRYLOV_AUTO, PFEM_KRYLOV_CLASSIC, PFEM_KRYLOV_FUSED = 0, 1, 2
PFEM_ORDER_BLOCKS, PFEM_ORDER_RCM = 0, 1
PFEM_ELEM_P1, PFEM_ELEM_Q4, PFEM_ELEM_Q8 = 0, 1, 2
PFEM_SCATTER_OWNER, PFEM_SCATTER_COLORED, PFEM_SCATTER_ATOMIC = 0, 1, 2
PFEM_LAYOUT_USER, PFEM_LAYOUT_INTERNAL = 0, 1
PFEM_MASK_NONE, PFEM_MASK_OUT, PFEM_MASK_IN = 0, 1, 2
PFEM_Q_PERM, PFEM_Q_ELEM_ORDER, PFEM_Q_COLOR, PFEM_Q_FREE_INDEX, PFEM_Q_BLOCKS = range(5)
PFEM_Q_AGGREGATE = 5
PFEM_PRECOND_JACOBI, PFEM_PRECOND_TWO_LEVEL = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "SKIPPED_FINE", -1: "E_INVALID_ARG",
                -2: "E_INVALID_MESH", -3: "E_OOM", -4: "E_DEVICE", -5: "E_BREAKDOWN",
                -6: "E_INVERTED", -7: "E_LINESEARCH", -8: "E_CANCELLED", -9: "E_STATE"}


class pfem_mesh_info(C.Structure):
    _fields_ = [("dim", C.c_int32), ("model", C.c_int32),
                ("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("n_dof", C.c_int64),
                ("n_free", C.c_int64), ("n_colors", C.c_int32), ("n_blocks", C.c_int32),
                ("block_nodes", C.c_int32), ("bandwidth_in", C.c_int64),
                ("bandwidth_internal", C.c_int64), ("owner_elem_visits", C.c_int64),
                ("device_bytes", C.c_int64), ("solve_bytes_fp32", C.c_int64),
                ("solve_bytes_fp64", C.c_int64), ("f_ext_norm", C.c_double),
                ("band_blocks", C.c_int32), ("elem", C.c_int32),
                ("nodes_per_elem", C.c_int32)]


class pfem_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_fine", C.c_double), ("max_iter", C.c_int32),
                ("n_load_steps", C.c_int32), ("max_newton", C.c_int32), ("prec", C.c_int32),
                ("record_history", C.c_int32), ("inner_rtol", C.c_double),
                ("krylov", C.c_int32), ("precond", C.c_int32)]


class pfem_solve_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("kv_count", C.c_int32), ("pcg_iters", C.c_int32),
                ("newton_iters", C.c_int32), ("load_steps_done", C.c_int32),
                ("residual_evals", C.c_int32), ("outer_sweeps", C.c_int32),
                ("line_search_evals", C.c_int32), ("rel_residual_initial", C.c_double),
                ("rel_residual_final", C.c_double), ("history_len", C.c_int64),
                ("t_device_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pfem_kernel_stats(C.Structure):
    _fields_ = [("launches_timed", C.c_int64), ("total_ms", C.c_double),
                ("launches_run", C.c_int64), ("alg_bytes", C.c_double)]


class pfem_server_stats(C.Structure):
    _fields_ = ([(k, C.c_int64) for k in ("submitted", "completed", "live", "queued",
                                          "peak_live", "bytes_in_use", "peak_bytes",
                                          "budget", "steps", "launches")]
                + [(k, C.c_double) for k in ("admit_s", "tick_s", "complete_s")])


_VP = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_D = C.c_double
_PVP = C.POINTER(C.c_void_p)

# name -> (restype, argtypes); mirrors include/pfem.h
PROTOTYPES = {
    "pfem_ctx_create": (_I32, [C.c_int, _VP, _PVP]),
    "pfem_ctx_destroy": (None, [_VP]),
    "pfem_last_error": (C.c_char_p, []),
    "pfem_version": (C.c_char_p, []),
    "pfem_ctx_set_timing": (_I32, [_VP, C.c_int]),
    "pfem_ctx_set_timing_sample": (_I32, [_VP, C.c_int]),
    "pfem_ctx_kernel_time": (_I32, [_VP, C.c_int, C.POINTER(_I64), C.POINTER(_D)]),
    "pfem_ctx_kernel_stats": (_I32, [_VP, C.c_int, C.POINTER(pfem_kernel_stats)]),
    "pfem_ctx_reset_timing": (_I32, [_VP]),
    "pfem_ctx_synchronize": (_I32, [_VP]),
    "pfem_mesh_create": (_I32, [_VP, C.c_int, _I64, _VP, _I64, _VP, _PVP]),
    "pfem_mesh_create_quad": (_I32, [_VP, C.c_int, _I64, _VP, _I64, _VP, _PVP]),
    "pfem_mesh_set_material": (_I32, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "pfem_mesh_set_dirichlet": (_I32, [_VP, _I64, _VP, _VP, _VP]),
    "pfem_mesh_set_neumann": (_I32, [_VP, _I64, _VP, _VP]),
    "pfem_mesh_set_periodic": (_I32, [_VP, _I64, _VP, _D]),
    "pfem_mesh_set_node_order": (_I32, [_VP, C.c_int]),
    "pfem_mesh_finalize": (_I32, [_VP, C.c_int]),
    "pfem_mesh_get_info": (_I32, [_VP, C.POINTER(pfem_mesh_info)]),
    "pfem_mesh_query_int": (_I32, [_VP, C.c_int, _VP, _I64, C.POINTER(_I64)]),
    "pfem_mesh_footprint": (_I32, [_VP, C.c_int, C.POINTER(_I64)]),
    "pfem_mesh_prepare_coarse": (_I32, [_VP, C.POINTER(_I32)]),
    "pfem_mesh_upload": (_I32, [_VP, _VP]),
    "pfem_mesh_release_device": (_I32, [_VP]),
    "pfem_mesh_destroy": (None, [_VP]),
    "pfem_permute": (_I32, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "pfem_hvp": (_I32, [_VP, C.c_int, C.c_int, C.c_int, C.c_int, _VP, _VP, _VP]),
    "pfem_apply_K": (_I32, [_VP, C.c_int, C.c_int, C.c_int, C.c_int, _VP, _VP]),
    "pfem_force": (_I32, [_VP, C.c_int, C.c_int, C.c_int, _VP, _VP]),
    "pfem_energy": (_I32, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "pfem_energy_noalloc": (_I32, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "pfem_diag": (_I32, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "pfem_batch_create": (_I32, [_VP, _I32, _VP, _PVP]),
    "pfem_batch_destroy": (None, [_VP]),
    "pfem_batch_offsets": (_I32, [_VP, _VP]),
    "pfem_batch_energy": (_I32, [_VP, C.c_int, _VP, _VP]),
    "pfem_batch_force": (_I32, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "pfem_batch_hvp": (_I32, [_VP, C.c_int, C.c_int, _VP, _VP, _VP]),
    "pfem_solve_opts_default": (None, [C.POINTER(pfem_solve_opts)]),
    "pfem_solve": (_I32, [_VP, _VP, C.POINTER(pfem_solve_opts), _VP, C.c_int, _VP, _I64,
                          C.POINTER(pfem_solve_report)]),
    "pfem_homogenize": (_I32, [_VP, _VP, C.POINTER(pfem_solve_opts), _VP, C.c_int, _VP,
                               _VP]),
    "pfem_server_create": (_I32, [_VP, _I64, _I32, _PVP]),
    "pfem_server_submit": (_I32, [_VP, _VP, _VP, C.POINTER(pfem_solve_opts), _I64]),
    "pfem_server_poll": (_I32, [_VP, _VP, _I64, C.POINTER(_I64)]),
    "pfem_server_result": (_I32, [_VP, _I64, _VP, C.POINTER(pfem_solve_report),
                                  C.POINTER(_D), C.POINTER(_D), C.POINTER(_D)]),
    "pfem_server_cancel": (_I32, [_VP, _I64]),
    "pfem_server_get_stats": (_I32, [_VP, C.POINTER(pfem_server_stats)]),
    "pfem_server_set_timing": (_I32, [_VP, C.c_int]),
    "pfem_server_kernel_stats": (_I32, [_VP, C.c_int, C.POINTER(pfem_kernel_stats)]),
    "pfem_server_destroy": (None, [_VP]),
}

_lib = None


class PfemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libpfem.so (raises if it is missing: no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing; build it with "
            "`python -m paper_2601_03086_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status):
    """Raise PfemError for negative statuses; return the status otherwise."""
    if status < 0:
        msg = load().pfem_last_error().decode(errors="replace")
        raise PfemError(status, msg)
    return status


def __getattr__(name):   # module-level access to the C functions: _lib.pfem_solve(...)
    if name.startswith("pfem_"):
        return getattr(load(), name)
    raise AttributeError(name)
