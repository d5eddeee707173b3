"""ctypes declarations mirroring include/gcpush.h (same names, same layouts)."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgcpush.so")

GC_OK, GC_EINVAL, GC_ENOMEM, GC_EDEVICE, GC_ESTATE = 0, -1, -2, -3, -4
GC_F64, GC_F32, GC_F16 = 0, 1, 2
GC_PREC_F64, GC_PREC_F32_ACC64, GC_PREC_F32_KAHAN = 0, 1, 2
GC_ACTIVE, GC_EXITED, GC_FINISHED, GC_NONFINITE = 0, 1, 2, 3
GC_FLAG_BOOTSTRAP, GC_FLAG_PENDING = 1, 2
GC_ORDER_NONE, GC_ORDER_COMPACT, GC_ORDER_BIN = 0, 1, 2
GC_SOURCE_GRID, GC_SOURCE_MLP = 0, 1
GC_MLP_PARAMS = 99846


DEV_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class gc_options(C.Structure):
    _fields_ = [("hip_stream", C.c_void_p), ("device", C.c_int32), ("precision", C.c_int32),
                ("order", C.c_int32), ("chunk_steps", C.c_int32), ("bin_coarsen", C.c_int32),
                ("block_size", C.c_int32), ("persistent", C.c_int32), ("tile", C.c_int32),
                ("log_depth", C.c_int32), ("timing", C.c_int32), ("field_source", C.c_int32),
                ("tail_threshold", C.c_int32), ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN),
                ("alloc_user", C.c_void_p)]


class gc_field_desc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nth", C.c_int32), ("nph", C.c_int32), ("src_dtype", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double), ("data", C.c_void_p),
                ("store_dtype", C.c_int32), ("pad", C.c_int32), ("extra", C.c_void_p)]


class gc_inject_desc(C.Structure):
    _fields_ = [("ensemble", C.c_uint32), ("first_id", C.c_uint32), ("n", C.c_uint64), ("seed", C.c_uint64),
                ("q", C.c_double), ("m", C.c_double), ("ekin", C.c_double),
                ("r0", C.c_double), ("lat0", C.c_double), ("lon0", C.c_double),
                ("dlon", C.c_double), ("dr0", C.c_double), ("dlat", C.c_double),
                ("mu_lo", C.c_double), ("mu_hi", C.c_double), ("lambda_par", C.c_double),
                ("r_in", C.c_double), ("r_out", C.c_double), ("max_steps", C.c_int64),
                ("drift_free", C.c_int32), ("scatter_law", C.c_int32), ("rebirth_steps", C.c_int64),
                ("v_wind", C.c_double)]


class gc_moment_spec(C.Structure):
    _fields_ = [("n_rbins", C.c_int32), ("r_lo", C.c_double), ("r_hi", C.c_double),
                ("n_mubins", C.c_int32), ("sel_r_lo", C.c_double), ("sel_r_hi", C.c_double),
                ("age_lo", C.c_double), ("age_hi", C.c_double), ("min_collisions", C.c_int32),
                ("n_agebins", C.c_int32), ("age_max", C.c_double), ("n_ebins", C.c_int32),
                ("e_lo", C.c_double), ("e_hi", C.c_double), ("e_unit", C.c_double), ("len_unit", C.c_double),
                ("min_birth", C.c_uint32), ("accumulate", C.c_int32)]


STATE_DOUBLES = ("r", "th", "ph", "u", "mu", "fr", "fth", "fph", "fu", "dtp", "s", "ell", "t",
                 "cr", "cth", "cph", "cu", "ct")
STATE_U32 = ("k", "flags", "status", "step", "id", "ens", "birth")


class gc_state_view(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in STATE_DOUBLES] + [(n, C.c_void_p) for n in STATE_U32]


class gc_counters(C.Structure):
    _fields_ = [("push_ms", C.c_double), ("n_push", C.c_int64), ("reorder_ms", C.c_double),
                ("n_reorder", C.c_int64), ("particle_steps", C.c_uint64), ("form_ms", C.c_double * 3),
                ("form_launches", C.c_int64 * 3), ("form_steps", C.c_uint64 * 3)]


class gc_tune_space(C.Structure):
    _fields_ = [("n_block", C.c_int32), ("block", C.c_int32 * 3), ("n_coarsen", C.c_int32), ("coarsen", C.c_int32 * 4),
                ("n_chunk", C.c_int32), ("chunk", C.c_int32 * 6), ("n_tile", C.c_int32), ("tile", C.c_int32 * 4),
                ("probe_steps", C.c_int64), ("dt", C.c_double)]


class gc_tune_result(C.Structure):
    _fields_ = [("best", gc_options), ("best_rate", C.c_double), ("default_rate", C.c_double),
                ("n_tried", C.c_int32), ("pad", C.c_int32)]


class gc_mlp_desc(C.Structure):
    _fields_ = [("freq", (C.c_double * 3) * 64), ("r_ref", C.c_double), ("scale", C.c_double * 6),
                ("power", C.c_double * 6), ("params", C.POINTER(C.c_float))]


class gc_mlp_train_opts(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("wc", C.c_double * 6), ("beta_pair", C.c_double), ("step", C.c_int32), ("apply", C.c_int32)]


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first (python -c 'import __graft_entry__ as g; g.build()')")
    try:   # share torch's HIP runtime (same soname) when torch is present
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    L = C.CDLL(LIB_PATH)
    P, S = C.c_void_p, C.c_int
    sig = {
        "gc_default_options": (None, [C.POINTER(gc_options)]),
        "gc_create": (S, [C.POINTER(P), C.POINTER(gc_options)]),
        "gc_destroy": (None, [P]),
        "gc_last_error": (C.c_char_p, [P]),
        "gc_set_options": (S, [P, C.POINTER(gc_options)]),
        "gc_get_options": (S, [P, C.POINTER(gc_options)]),
        "gc_load_field": (S, [P, C.POINTER(gc_field_desc)]),
        "gc_inject": (S, [P, C.POINTER(gc_inject_desc)]),
        "gc_advance": (S, [P, C.c_double, C.c_int64]),
        "gc_advance_graph": (S, [P, C.c_double, C.c_int64]),
        "gc_moments_size": (C.c_int64, [C.POINTER(gc_moment_spec)]),
        "gc_moments": (S, [P, C.POINTER(gc_moment_spec), P]),
        "gc_count": (S, [P, C.POINTER(C.c_uint64)]),
        "gc_get_state": (S, [P, C.POINTER(gc_state_view)]),
        "gc_set_state": (S, [P, C.POINTER(gc_state_view), C.c_uint64]),
        "gc_get_log": (S, [P, P]),
        "gc_get_order": (S, [P, P, P, P]),
        "gc_get_counters": (S, [P, C.POINTER(gc_counters)]),
        "gc_reset_counters": (S, [P]),
        "gc_copy_probe": (S, [P, P, P, C.c_uint64]),
        "gc_gather_probe": (S, [P, C.c_double, C.c_int32, P]),
        "gc_autotune": (S, [P, C.POINTER(gc_tune_space), C.POINTER(gc_tune_result)]),
        "gc_mlp_set": (S, [P, C.POINTER(gc_mlp_desc)]),
        "gc_mlp_get_params": (S, [P, C.POINTER(C.c_float)]),
        "gc_mlp_get_grads": (S, [P, C.POINTER(C.c_float)]),
        "gc_mlp_train_step": (S, [P, P, P, C.c_int64, C.POINTER(gc_mlp_train_opts), C.POINTER(C.c_double)]),
        "gc_mlp_train_step_noalloc": (S, [P, P, P, C.c_int64, C.POINTER(gc_mlp_train_opts), C.POINTER(C.c_double)]),
        "gc_mlp_eval": (S, [P, P, C.c_int64, P]),
        "gc_field_sample": (S, [P, P, C.c_int64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


DECLARED = (
    "gc_default_options", "gc_create", "gc_destroy", "gc_last_error", "gc_set_options", "gc_get_options",
    "gc_load_field", "gc_inject", "gc_advance", "gc_advance_graph", "gc_moments_size", "gc_moments",
    "gc_count", "gc_get_state", "gc_set_state", "gc_get_log", "gc_get_order", "gc_get_counters", "gc_reset_counters",
    "gc_copy_probe", "gc_autotune", "gc_mlp_set", "gc_mlp_get_params", "gc_mlp_get_grads", "gc_mlp_train_step", "gc_mlp_train_step_noalloc",
    "gc_mlp_eval", "gc_field_sample", "gc_gather_probe",
)
