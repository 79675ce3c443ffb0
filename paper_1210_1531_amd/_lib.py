"""ctypes view of libmag.so: structures and prototypes of include/mag.h."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmag.so")

MAG_OK = 0
MAG_EINVAL = -1
MAG_ENOMEM = -2
MAG_EHIP = -3
MAG_ENOTPD = -4
MAG_EBRACKET = -5
MAG_ESTATE = -6
MAG_ENONFINITE = -7
MAG_EUNSUPPORTED = -8
MAG_ENOCONV = -9
STATUS_NAMES = {
    0: "MAG_OK", -1: "MAG_EINVAL", -2: "MAG_ENOMEM", -3: "MAG_EHIP", -4: "MAG_ENOTPD",
    -5: "MAG_EBRACKET", -6: "MAG_ESTATE", -7: "MAG_ENONFINITE", -8: "MAG_EUNSUPPORTED",
    -9: "MAG_ENOCONV",
}

MAG_HOST = 0
MAG_DEVICE = 1
MAG_STATS_BUCKETS = 8
MAG_WORKFLOW_RECOMPUTE = 0
MAG_WORKFLOW_STORE = 1
MAG_WORKFLOW_AUTO = 2
MAG_SCHED_AUTO = 0
MAG_SCHED_PERSISTENT = 1
MAG_SCHED_GRID = 2
MAG_SCHED_PLAIN = 3
MAG_SCHED_GRAPH = 4
NORB = 4
NU_MAX = 48
CLUSTER_MAX = 192
BLOCKS_MAX = 32


class MagSKModel(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "es", "ep", "v_ss_sigma", "v_sp_sigma", "v_pp_sigma", "v_pp_pi",
        "s_ss_sigma", "s_sp_sigma", "s_pp_sigma", "s_pp_pi", "r0", "r_on", "r_cut")]


class MagSystem(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int64),
        ("nnz", C.c_int64),
        ("rowptr", C.c_void_p),
        ("colind", C.c_void_p),
        ("H", C.c_void_p),
        ("S", C.c_void_p),
        ("pos", C.c_void_p),
        ("cell", C.c_double * 3),
        ("r_cluster", C.c_double),
        ("clus_ptr", C.c_void_p),
        ("clus_atoms", C.c_void_p),
    ]


class MagOpts(C.Structure):
    _fields_ = [
        ("nu", C.c_int),
        ("kT", C.c_double),
        ("n_electrons", C.c_double),
        ("mu_tol", C.c_double),
        ("mu_fixed", C.c_double),
        ("breakdown", C.c_double),
        ("workflow", C.c_int),
        ("schedule", C.c_int),
        ("eig_sweeps", C.c_int),
        ("keep_exact", C.c_int),
    ]


class MagMDOpts(C.Structure):
    _fields_ = [
        ("dt", C.c_double),
        ("mass", C.c_double),
        ("phi0", C.c_double),
        ("m_rep", C.c_double),
        ("r_cluster", C.c_double),
        ("n_steps", C.c_int),
        ("exact_forces", C.c_int),
    ]


class MagStats(C.Structure):
    _fields_ = [
        ("t_set_system_ms", C.c_double),
        ("t_pass1_ms", C.c_double),
        ("t_mu_ms", C.c_double),
        ("t_pass2_ms", C.c_double),
        ("t_forces_ms", C.c_double),
        ("n_columns", C.c_int64),
        ("max_cluster", C.c_int64),
        ("sum_cluster_nnz", C.c_int64),
        ("device_bytes", C.c_int64),
        ("bisect_levels", C.c_int32),
        ("schedule_used", C.c_int32),
        ("t_krylov_ms", C.c_double),
        ("t_eig_ms", C.c_double),
        ("krylov_launches", C.c_int32),
        ("workflow_used", C.c_int32),
        ("krylov_buckets", C.c_int32),
        ("krylov_tpb", C.c_int32),
        ("autotune_ms", C.c_double),
        ("t_icohp_ms", C.c_double),
        ("t_cohp_ms", C.c_double),
        ("t_md_step_ms", C.c_double),
        ("t_cocg_ms", C.c_double),
        ("t_forces_exact_ms", C.c_double),
        ("krylov_cache_blocks", C.c_int32),
        ("plan_threads", C.c_int32 * MAG_STATS_BUCKETS),
        ("plan_rows", C.c_int32 * MAG_STATS_BUCKETS),
        ("plan_per_cu", C.c_int32 * MAG_STATS_BUCKETS),
        ("plan_cache", C.c_int32 * MAG_STATS_BUCKETS),
        ("plan_candidates", C.c_int32 * MAG_STATS_BUCKETS),
        ("plan_columns", C.c_int64 * MAG_STATS_BUCKETS),
        ("plan_us_per_col", C.c_double * MAG_STATS_BUCKETS),
    ]


P = C.c_void_p
I = C.c_int
I64 = C.c_int64
D = C.c_double
CTX = C.c_void_p

# name -> (restype, argtypes); every symbol declared in include/mag.h
PROTOTYPES = {
    "mag_create": (I, [C.POINTER(CTX), I, P]),
    "mag_destroy": (None, [CTX]),
    "mag_last_error": (C.c_char_p, [CTX]),
    "mag_version": (I, []),
    "mag_sk_build": (I, [CTX, C.POINTER(MagSKModel), I64, P, C.POINTER(D), I, C.POINTER(I64)]),
    "mag_sk_get_csr": (I, [CTX, P, P, P, P, I]),
    "mag_sk_values": (I, [CTX, P, P, P, I]),
    "mag_sk_vjp": (I, [CTX, P, P, P, P, I]),
    "mag_sk_vjp_noalloc": (I, [CTX, P, P, P, P]),
    "mag_set_system": (I, [CTX, C.POINTER(MagSystem), I]),
    "mag_update_values": (I, [CTX, P, P, I]),
    "mag_get_clusters": (I, [CTX, P, P, C.POINTER(I64), I]),
    "mag_opts_default": (None, [C.POINTER(MagOpts)]),
    "mag_solve_columns": (I, [CTX, C.POINTER(MagOpts), C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
    "mag_spectra": (I, [CTX, P, P, P, I]),
    "mag_energy": (I, [CTX, C.POINTER(D), C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
    "mag_column_spectra": (I, [CTX, C.POINTER(MagOpts), P, I64, P, P, P, I]),
    "mag_density_matrix": (I, [CTX, P, P, I]),
    "mag_cluster_columns": (I, [CTX, P, I64, P, P, I]),
    "mag_green_columns": (I, [CTX, C.POINTER(MagOpts), P, I64, P, I, P, P, I]),
    "mag_backward": (I, [CTX, D, P, P, I]),
    "mag_forces": (I, [CTX, C.POINTER(MagSKModel), P, I]),
    "mag_forces_exact": (I, [CTX, C.POINTER(MagSKModel), P, I]),
    "mag_icohp": (I, [CTX, C.POINTER(MagSKModel), P, P, P, I]),
    "mag_cohp": (I, [CTX, C.POINTER(D), I, D, P, I]),
    "mag_cocg_columns": (I, [CTX, P, I64, P, I, D, I, P, P, P, I]),
    "mag_pair_repulsion": (I, [CTX, D, D, C.POINTER(D), P, P, I]),
    "mag_md_run": (I, [CTX, C.POINTER(MagSKModel), C.POINTER(MagOpts), C.POINTER(MagMDOpts), I64,
                       C.POINTER(D), P, P, P, C.POINTER(D), I]),
    "mag_get_stats": (I, [CTX, C.POINTER(MagStats)]),
}

_lib = None


def load():
    """Load libmag.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1210_1531_amd.build` "
            "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
