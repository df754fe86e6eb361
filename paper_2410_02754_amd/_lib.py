"""ctypes declarations of the C ABI in include/chfsi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchfsi.so")

STATUS = {0: "CHFSI_OK", -1: "CHFSI_EINVAL", -2: "CHFSI_ENOMEM", -3: "CHFSI_EHIP",
          -4: "CHFSI_ENOTPD", -5: "CHFSI_ENONHERM", -6: "CHFSI_ENONFINITE", -7: "CHFSI_ESTATE"}

EXPORTED = ["chfsi_create", "chfsi_destroy", "chfsi_sizes", "chfsi_quad_points", "chfsi_set_local",
            "chfsi_set_atoms", "chfsi_apply_H", "chfsi_cheb_filter", "chfsi_chol_gs",
            "chfsi_rayleigh_ritz", "chfsi_lanczos_bounds", "chfsi_fill_random", "chfsi_sync",
            "chfsi_last_error", "chfsi_version", "chfsi_stats_enable", "chfsi_stats_read",
            "chfsi_stats_reset", "chfsi_apply_H_backward", "chfsi_filter_backward_workspace",
            "chfsi_cheb_filter_backward", "chfsi_batch_create", "chfsi_batch_filter", "chfsi_batch_tiles",
            "chfsi_batch_destroy", "chfsi_batch_last_error", "chfsi_ritz_residual", "chfsi_cheb_filter_resid",
            "chfsi_fermi_dirac", "chfsi_density", "chfsi_set_apply_form", "chfsi_batch_graph_info",
            "chfsi_cheb_filter_noalloc", "chfsi_field_inner", "chfsi_hartree", "chfsi_kerker", "chfsi_exchange",
            "chfsi_interpolate_block", "chfsi_scf_run", "chfsi_overlap", "chfsi_workspace_bytes"]

STAGES = ["cell_fp64", "cell_fp32", "nonlocal", "axpy", "gram", "rotate", "host_dense"]


class MeshDesc(C.Structure):
    _fields_ = [("n_cells", C.c_int * 3), ("box", C.c_double * 3), ("p", C.c_int),
                ("quad", C.c_int), ("n_q", C.c_int), ("n_k", C.c_int),
                ("kpts", C.POINTER(C.c_double))]


class AtomDesc(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("lmax", C.c_int), ("sigma", C.c_double),
                ("rcut", C.c_double), ("d0", C.c_double * 3), ("dso", C.c_double),
                ("delta_override", C.POINTER(C.c_double))]


class BatchTask(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("ik", C.c_int), ("X_d", C.c_void_p), ("ldx", C.c_int64),
                ("work_d", C.c_void_p), ("ldw", C.c_int64), ("n_vec", C.c_int)]


class ScfParams(C.Structure):
    _fields_ = [("n_vec", C.c_int), ("degree", C.c_int), ("passes_first", C.c_int), ("passes", C.c_int),
                ("depth", C.c_int), ("max_iter", C.c_int), ("max_coarse", C.c_int), ("lanczos_steps", C.c_int),
                ("field_max_iter", C.c_int), ("prec_mode", C.c_int), ("n_electrons", C.c_double),
                ("kT", C.c_double), ("alpha", C.c_double), ("k0", C.c_double), ("tol", C.c_double),
                ("tol_coarse", C.c_double), ("field_tol", C.c_double), ("seed", C.c_uint64),
                ("lanczos_seed", C.c_uint64), ("bounds_h", C.POINTER(C.c_double)), ("n_bounds", C.c_int),
                ("kweights_h", C.POINTER(C.c_double)), ("start_given", C.c_int)]


class ScfRecord(C.Structure):
    _fields_ = [("p", C.c_int), ("resid", C.c_double), ("mu", C.c_double), ("band_energy", C.c_double),
                ("theta0", C.c_double), ("hartree_iters", C.c_int), ("b", C.c_double)]


class StageStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("flops", C.c_double),
                ("exec_flops", C.c_double), ("bytes", C.c_double)]


class ChfsiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libchfsi.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python paper_2410_02754_amd/build.py)")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the library binds to the runtime that owns torch's memory and streams
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
    pd = C.POINTER(C.c_double)
    sig = {
        "chfsi_create": ([C.POINTER(MeshDesc), vp, C.POINTER(vp)], i32),
        "chfsi_destroy": ([vp], i32),
        "chfsi_sizes": ([vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                         C.POINTER(i32)], i32),
        "chfsi_quad_points": ([vp, pd], i32),
        "chfsi_set_local": ([vp, vp, vp], i32),
        "chfsi_set_atoms": ([vp, i32, C.POINTER(AtomDesc)], i32),
        "chfsi_apply_H": ([vp, i32, vp, i64, vp, i64, i32, i32], i32),
        "chfsi_cheb_filter": ([vp, i32, vp, i64, vp, i64, i32, i32, dbl, dbl, dbl, i32], i32),
        "chfsi_cheb_filter_noalloc": ([vp, i32, vp, i64, vp, i64, i32, i32, dbl, dbl, dbl, i32], i32),
        "chfsi_chol_gs": ([vp, vp, i64, i32, C.POINTER(i32)], i32),
        "chfsi_rayleigh_ritz": ([vp, i32, vp, i64, vp, i64, i32, pd, pd], i32),
        "chfsi_lanczos_bounds": ([vp, i32, i32, vp, pd, pd], i32),
        "chfsi_fill_random": ([vp, vp, i64, i32, i64, C.c_uint64, i64, i32, i64], i32),
        "chfsi_sync": ([vp], i32),
        "chfsi_ritz_residual": ([vp, vp, i64, vp, i64, i32, pd], i32),
        "chfsi_cheb_filter_resid": ([vp, i32, vp, i64, vp, i64, pd, vp, i64, i32, i32, dbl, dbl, dbl, i32], i32),
        "chfsi_batch_create": ([i32, C.POINTER(BatchTask), i32, i32, i32, C.POINTER(vp)], i32),
        "chfsi_batch_filter": ([vp, pd, pd, pd], i32),
        "chfsi_batch_tiles": ([vp, C.POINTER(i32), pd], i32),
        "chfsi_batch_destroy": ([vp], i32),
        "chfsi_batch_graph_info": ([vp, C.POINTER(i32), C.POINTER(i32), pd, pd], i32),
        "chfsi_batch_last_error": ([vp], C.c_char_p),
        "chfsi_apply_H_backward": ([vp, i32, vp, i64, vp, i64, vp, i64, i32, vp, vp], i32),
        "chfsi_filter_backward_workspace": ([vp, i32, i32, i32], C.c_size_t),
        "chfsi_cheb_filter_backward": ([vp, i32, vp, i64, vp, i64, vp, i64, i32, i32, dbl, dbl, dbl,
                                        i32, vp, C.c_size_t, vp, vp], i32),
        "chfsi_set_apply_form": ([vp, i32], i32),
        "chfsi_fermi_dirac": ([i32, pd, pd, dbl, dbl, pd, pd, pd], i32),
        "chfsi_density": ([vp, vp, i64, i32, pd, vp, vp], i32),
        "chfsi_field_inner": ([vp, vp, vp, vp, vp, pd], i32),
        "chfsi_overlap": ([vp, vp, i64, vp, i64, i32, pd], i32),
        "chfsi_workspace_bytes": ([vp, i32, i32, i32], C.c_size_t),
        "chfsi_hartree": ([vp, vp, vp, dbl, i32, C.POINTER(i32)], i32),
        "chfsi_kerker": ([vp, dbl, vp, vp, dbl, i32, C.POINTER(i32)], i32),
        "chfsi_exchange": ([vp, vp, vp, vp, vp], i32),
        "chfsi_interpolate_block": ([vp, vp, vp, i64, vp, i64, i32], i32),
        "chfsi_scf_run": ([vp, vp, C.POINTER(ScfParams), vp, vp, vp, vp, vp, vp, vp, i64, pd, pd,
                           C.POINTER(ScfRecord), i32, C.POINTER(i32), C.POINTER(i32)], i32),
        "chfsi_stats_enable": ([vp, i32], i32),
        "chfsi_stats_read": ([vp, C.POINTER(StageStats)], i32),
        "chfsi_stats_reset": ([vp], i32),
        "chfsi_last_error": ([vp], C.c_char_p),
        "chfsi_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(code, ctx=None):
    if code != 0:
        msg = load().chfsi_last_error(ctx).decode(errors="replace")
        raise ChfsiError(code, msg)
