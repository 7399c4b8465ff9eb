"""ctypes binding of the C-ABI in include/smg.h (argument marshalling only)."""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsmg.so")

SMG_OK = 0
SMG_EINVAL = -1
SMG_ENOMEM = -2
SMG_ENOTCONV = -3
SMG_ENONFINITE = -4
SMG_EHIP = -5
SMG_ESTATE = -6
SMG_COARSEST_CHOLESKY = 0
SMG_COARSEST_SMOOTH = 1
SMG_FP64 = 0
SMG_FP32_REFINED = 1
SMG_OUT_F64 = 0
SMG_OUT_F32 = 1
SMG_OPT_BOTTOM_KERNEL = 1
SMG_OPT_TIMED_KERNEL = 2
SMG_TIMED_FINE_PASS = 0
SMG_TIMED_LEVEL1_BLOCK_PASS = 1
SMG_TIMED_BOTTOM = 2
SMG_MAX_MODES = 32
SMG_OPT_BLOCK_TILE = 3
SMG_OPT_BLOCK_PAIRS = 4
SMG_OPT_STREAM_GROUPS = 5
SMG_TILE_AUTO = 0
SMG_TILE_4X4 = 1
SMG_TILE_4X2 = 2
SMG_TILE_8X4 = 3
SMG_BC_DEFAULT = 0
SMG_BC_PERIODIC = 1
SMG_BC_DIRICHLET_FACE = 2
SMG_STATIC_SCRATCH_BYTES = 64 * 1024 * 1024
SMG_OP_SAMPLE = 0
SMG_OP_SOLVE = 1

ERROR_NAMES = {0: "SMG_OK", -1: "SMG_EINVAL", -2: "SMG_ENOMEM", -3: "SMG_ENOTCONV",
               -4: "SMG_ENONFINITE", -5: "SMG_EHIP", -6: "SMG_ESTATE"}

EXPORTED = ["smg_create_hierarchy", "smg_hierarchy_info", "smg_bind_workspace",
            "smg_sample_field", "smg_solve", "smg_destroy_hierarchy", "smg_last_error",
            "smg_debug_smooth", "smg_debug_restrict_residual", "smg_debug_prolong_add",
            "smg_debug_coarsest", "smg_debug_host_table", "smg_set_option",
            "smg_kernel_timing", "smg_kernel_timing_read", "smg_lowest_modes",
            "smg_sample_stats", "smg_sample_batch", "smg_solve_batch",
            "smg_composite_create", "smg_composite_get_info", "smg_composite_bind",
            "smg_composite_cycle", "smg_composite_sample", "smg_composite_residual",
            "smg_composite_solve", "smg_composite_debug_pass", "smg_composite_debug_base_pass",
            "smg_composite_debug_row", "smg_composite_destroy", "smg_composite_forced_field",
            "smg_sample_field_static",
            "smg_batch_run", "smg_selm_create", "smg_selm_get_info", "smg_selm_bind",
            "smg_selm_project", "smg_selm_mobility", "smg_selm_drive", "smg_selm_step",
            "smg_selm_destroy", "smg2d_create", "smg2d_get_info", "smg2d_bind", "smg2d_sample",
            "smg2d_solve", "smg2d_destroy"]


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ncomp", ctypes.c_int32), ("h", ctypes.c_double), ("kT", ctypes.c_double),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("bc_z", ctypes.c_int32)]


class CycleParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("coarsest_max", ctypes.c_int32), ("coarsest_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("burn_in", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("state_bytes", ctypes.c_size_t),
                ("n_levels", ctypes.c_int32), ("dims", (ctypes.c_int32 * 3) * 16),
                ("coarsest_unknowns", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("relres", ctypes.c_double),
                ("last_ratio", ctypes.c_double)]


class BatchItem(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("op", ctypes.c_int32), ("nchains", ctypes.c_int32),
                ("comps_per_chain", ctypes.c_int32), ("out_dtype", ctypes.c_int32),
                ("n", ctypes.c_int64), ("seed", ctypes.c_uint64), ("first_cycle", ctypes.c_uint64),
                ("seeds", ctypes.POINTER(ctypes.c_uint64)),
                ("first_cycles", ctypes.POINTER(ctypes.c_uint64)),
                ("state", ctypes.c_void_p), ("out", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("rtol", ctypes.c_double), ("max_cycles", ctypes.c_int32),
                ("infos", ctypes.POINTER(SolveInfo)), ("status", ctypes.c_int32)]


class CompositeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("box", ctypes.c_int32 * 6), ("h", ctypes.c_double), ("kT", ctypes.c_double)]


class FACParams(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int32), ("mu1", ctypes.c_int32), ("mu2", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("coarsest_max", ctypes.c_int32),
                ("gs_only", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("row_lanes", ctypes.c_int32)]


class CompositeInfo(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("base_cells", ctypes.c_int64),
                ("fine_cells", ctypes.c_int64), ("unknowns", ctypes.c_int64),
                ("fine_dims", ctypes.c_int32 * 3), ("n_levels", ctypes.c_int32),
                ("dims", (ctypes.c_int32 * 3) * 16), ("stencils", ctypes.c_int32 * 16),
                ("block_types", ctypes.c_int32 * 16), ("layer_cells", ctypes.c_int32),
                ("coarsest_unknowns", ctypes.c_int32)]


class SelmDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double), ("mu", ctypes.c_double), ("kT", ctypes.c_double),
                ("levels", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("max_points", ctypes.c_int32)]


class SelmInfo(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("state_bytes", ctypes.c_size_t),
                ("n_levels", ctypes.c_int32)]


class Desc2D(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("ncomp", ctypes.c_int32),
                ("h", ctypes.c_double), ("kT", ctypes.c_double), ("levels", ctypes.c_int32),
                ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("coarsest_max", ctypes.c_int32), ("coarsest_mode", ctypes.c_int32),
                ("stride", ctypes.c_int32)]


class Info2D(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("n_levels", ctypes.c_int32),
                ("dims", (ctypes.c_int32 * 2) * 16)]


class SMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, code), msg))
        self.code = code


_lib = None


def load():
    """Load libsmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsmg.so not built: run __graft_entry__.build() or "
                           "python -m paper_1003_2680_amd.build")
    # torch first: the library then binds to the HIP runtime torch loaded (same soname).  Loaded
    # the other way round, torch would bring a second HIP runtime into the process, and the
    # library's calls would find no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    H = ctypes.c_void_p
    sig = {
        "smg_create_hierarchy": ([ctypes.POINTER(GridDesc), ctypes.POINTER(CycleParams),
                                  ctypes.POINTER(H)], ctypes.c_int),
        "smg_hierarchy_info": ([H, ctypes.POINTER(Info)], ctypes.c_int),
        "smg_bind_workspace": ([H, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_sample_field": ([H, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, P, P,
                              ctypes.c_int32, P], ctypes.c_int),
        "smg_solve": ([H, P, P, ctypes.c_double, ctypes.c_int32, P, ctypes.POINTER(SolveInfo)],
                      ctypes.c_int),
        "smg_sample_field_static": ([H, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, P, P,
                                     ctypes.c_int32, P], ctypes.c_int),
        "smg_destroy_hierarchy": ([H], None),
        "smg_last_error": ([], ctypes.c_char_p),
        "smg_debug_smooth": ([H, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, P], ctypes.c_int),
        "smg_debug_restrict_residual": ([H, ctypes.c_int32, P, P, P, P], ctypes.c_int),
        "smg_debug_prolong_add": ([H, ctypes.c_int32, P, P, P], ctypes.c_int),
        "smg_debug_coarsest": ([H, P, P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, P],
                               ctypes.c_int),
        "smg_debug_host_table": ([H, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_size_t],
                                 ctypes.c_int),
        "smg_set_option": ([H, ctypes.c_int32, ctypes.c_int64], ctypes.c_int),
        "smg_kernel_timing": ([H, ctypes.c_int32], ctypes.c_int),
        "smg_kernel_timing_read": ([H, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "smg_lowest_modes": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P],
                             ctypes.c_int),
        "smg_sample_stats": ([H, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, P, P,
                              ctypes.c_int32, P, ctypes.c_int32, P, P, P], ctypes.c_int),
        "smg_sample_batch": ([H, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int64, P, P,
                              ctypes.c_int32, P, ctypes.c_int32, P, P, P], ctypes.c_int),
        "smg_solve_batch": ([H, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_double,
                             ctypes.c_int32, P, P], ctypes.c_int),
        "smg_batch_run": ([ctypes.POINTER(BatchItem), ctypes.c_int32, P], ctypes.c_int),
    }
    U64, I32 = ctypes.c_uint64, ctypes.c_int32
    sig.update({
        "smg_composite_create": ([ctypes.POINTER(CompositeDesc), ctypes.POINTER(FACParams),
                                  ctypes.POINTER(H)], ctypes.c_int),
        "smg_composite_get_info": ([H, ctypes.POINTER(CompositeInfo)], ctypes.c_int),
        "smg_composite_bind": ([H, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_composite_cycle": ([H, P, P, P, P, U64, U64, I32, P], ctypes.c_int),
        "smg_composite_sample": ([H, ctypes.c_int64, U64, U64, P, P, P], ctypes.c_int),
        "smg_composite_residual": ([H, P, P, P, P, P, P, P], ctypes.c_int),
        "smg_composite_solve": ([H, P, P, P, P, ctypes.c_double, I32, P,
                                 ctypes.POINTER(SolveInfo)], ctypes.c_int),
        "smg_composite_debug_pass": ([H, I32, P, P, P, P, U64, U64, I32, I32, P], ctypes.c_int),
        "smg_composite_debug_base_pass": ([H, I32, I32, P, P, U64, U64, I32, I32, P],
                                          ctypes.c_int),
        "smg_composite_debug_row": ([H, I32, ctypes.c_int64, P, P, ctypes.POINTER(I32)],
                                    ctypes.c_int),
        "smg_composite_destroy": ([H], None),
        "smg_composite_forced_field": ([H, ctypes.c_int64, U64, U64, P, P, P, P, ctypes.c_double,
                                        I32, P, ctypes.POINTER(SolveInfo)], ctypes.c_int),
        "smg_selm_create": ([ctypes.POINTER(SelmDesc), ctypes.POINTER(H)], ctypes.c_int),
        "smg_selm_get_info": ([H, ctypes.POINTER(SelmInfo)], ctypes.c_int),
        "smg_selm_bind": ([H, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_selm_project": ([H, P, P, ctypes.c_double, P], ctypes.c_int),
        "smg_selm_mobility": ([H, I32, P, P, P, ctypes.c_double, P], ctypes.c_int),
        "smg_selm_drive": ([H, I32, P, U64, U64, P, P, ctypes.c_double, P], ctypes.c_int),
        "smg_selm_step": ([H, I32, P, P, ctypes.c_double, U64, U64, P, ctypes.c_double, P],
                          ctypes.c_int),
        "smg_selm_destroy": ([H], None),
        "smg2d_create": ([ctypes.POINTER(Desc2D), ctypes.POINTER(H)], ctypes.c_int),
        "smg2d_get_info": ([H, ctypes.POINTER(Info2D)], ctypes.c_int),
        "smg2d_bind": ([H, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg2d_sample": ([H, ctypes.c_int64, U64, U64, P, P, P], ctypes.c_int),
        "smg2d_solve": ([H, P, P, ctypes.c_double, I32, P, ctypes.POINTER(SolveInfo)],
                        ctypes.c_int),
        "smg2d_destroy": ([H], None),
    })
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc):
    if rc != SMG_OK:
        msg = load().smg_last_error()
        raise SMGError(rc, msg.decode() if msg else "")
    return rc
