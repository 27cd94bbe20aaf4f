"""ctypes declarations of the C ABI in include/tt.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtt.so")

TT_OK, TT_ERR_INVALID_ARG, TT_ERR_DEVICE, TT_ERR_OOM, TT_ERR_NUMERIC, TT_ERR_STATE = 0, -1, -2, -3, -4, -5
TT_BC_VACUUM, TT_BC_PERIODIC, TT_BC_INFLOW, TT_BC_OUTFLOW = 0, 1, 2, 3
TT_FLUX_UPWIND, TT_FLUX_RUSANOV, TT_FLUX_HLL = 0, 1, 2
TT_FP64, TT_FP32_MIXED = 0, 1
TT_ROUND_ONCE, TT_ROUND_TWICE = 0, 1
TT_MAT_FROZEN, TT_MAT_COUPLED = 0, 1
TT_RANK_AUTO, TT_RANK_REPLAY = 0, 1

STATUS_NAMES = {0: "TT_OK", -1: "TT_ERR_INVALID_ARG", -2: "TT_ERR_DEVICE", -3: "TT_ERR_OOM",
                -4: "TT_ERR_NUMERIC", -5: "TT_ERR_STATE"}


class tt_config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ntheta", C.c_int32), ("nphi", C.c_int32),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("c", C.c_double), ("a_r", C.c_double), ("cfl", C.c_double), ("dt", C.c_double),
        ("tol", C.c_double), ("rmax", C.c_int32),
        ("bc_lo", C.c_int32 * 3), ("bc_hi", C.c_int32 * 3),
        ("precision", C.c_int32), ("schedule", C.c_int32), ("material", C.c_int32),
        ("rank_mode", C.c_int32), ("ckpt_every", C.c_int32), ("max_steps", C.c_int32),
        ("r1_cap", C.c_int32), ("r2_cap", C.c_int32),
        ("flux", C.c_int32), ("s_plus", C.c_double),
        ("hll_beta", C.c_double), ("hll_tau_threshold", C.c_double),
    ]


class tt_inflow(C.Structure):
    _fields_ = [("face", C.c_int32), ("face_w", C.POINTER(C.c_double)),
                ("theta_w", C.POINTER(C.c_double)), ("phi_w", C.POINTER(C.c_double))]


PD = C.POINTER(C.c_double)
PI = C.POINTER(C.c_int32)
VP = C.c_void_p

SIGNATURES = {
    "tt_workspace_bytes": (C.c_size_t, [C.POINTER(tt_config), C.c_int32]),
    "tt_create": (C.c_int, [C.POINTER(tt_config), PD, PD, PD, PD, C.POINTER(tt_inflow), C.c_int32,
                            PD, PD, PD, C.c_int32, C.c_int32, VP, C.c_size_t, VP, C.POINTER(VP)]),
    "tt_step": (C.c_int, [VP, C.c_int32]),
    "tt_round": (C.c_int, [VP, C.c_double, C.c_int32, PI]),
    "tt_round_randomized": (C.c_int, [VP, VP, C.c_int32, VP, C.c_int32, PI]),
    "tt_energy": (C.c_int, [VP, VP, PD, PD]),
    "tt_grad": (C.c_int, [VP, PD, C.c_double, PD, VP]),
    "tt_set_kappa": (C.c_int, [VP, VP]),
    "tt_set_scattering": (C.c_int, [VP, PD]),
    "tt_detector_loss": (C.c_int, [VP, PD, PD]),
    "tt_get_cores": (C.c_int, [VP, PD, PD, PD, PI]),
    "tt_set_cores": (C.c_int, [VP, PD, PD, PD, PI]),
    "tt_get_temperature": (C.c_int, [VP, PD]),
    "tt_get_rank_history": (C.c_int, [VP, PI, C.c_int32, PI]),
    "tt_set_rank_schedule": (C.c_int, [VP, PI, C.c_int32]),
    "tt_get_round_info": (C.c_int, [VP, PD]),
    "tt_profile_enable": (C.c_int, [VP, C.c_int32]),
    "tt_profile_read": (C.c_int, [VP, PD, PI, C.POINTER(C.c_char_p), C.c_int32, PI]),
    "tt_use_graphs": (C.c_int, [VP, C.c_int32]),
    "tt_set_gram_slices": (C.c_int, [VP, C.c_int32]),
    "tt_set_solver_limits": (C.c_int, [VP, C.c_int32]),
    "tt_last_error": (C.c_char_p, [VP]),
    "tt_kernel_eigh_workspace": (C.c_size_t, [C.c_int32]),
    "tt_kernel_eigh": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_double, VP, VP, C.c_int32, PI, VP,
                                 C.c_size_t, VP]),
    "tt_kernel_svd_workspace": (C.c_size_t, [C.c_int32, C.c_int32]),
    "tt_kernel_svd": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_int32, VP, VP, C.c_int32, PI, VP,
                                C.c_size_t, VP]),
    "tt_kernel_gram_f32_workspace": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "tt_kernel_gram_f32": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_int32, VP, C.c_int32, VP,
                                     C.c_size_t, VP]),
    "tt_kernel_gram_workspace": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "tt_kernel_gram": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_int32, VP, C.c_int32, VP, C.c_size_t, VP]),
    "tt_kernel_gram_noalloc": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_int32, VP, C.c_int32, VP]),
    "tt_kernel_gemm_tall_workspace": (C.c_size_t, []),
    "tt_kernel_gemm_tall": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_int32, VP, C.c_int32, C.c_int32,
                                      VP, C.c_int32, VP, C.c_size_t, VP]),
    "tt_kernel_gemm": (C.c_int, [VP, C.c_int32, C.c_int32, VP, C.c_int32, C.c_int32, VP, C.c_int32,
                                 C.c_int32, C.c_int32, C.c_int32, VP, C.c_size_t, VP]),
    "tt_kernel_lds_check": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "tt_kernel_microbench_workspace": (C.c_size_t, [C.c_int32, C.c_size_t]),
    "tt_kernel_microbench": (C.c_int, [C.c_int32, C.c_size_t, C.c_int32, VP, C.c_size_t, PD, VP]),
    "tt_kernel_last_error": (C.c_char_p, []),
    "tt_destroy": (None, [VP]),
}

_lib = None


def load(path=None):
    """Load libtt.so; raises if the HIP library has not been built.  The
    environment variable TT_LIBRARY names another build of the same library
    (the host-sanitizer build of the host-side checks)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or os.environ.get("TT_LIBRARY") or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is missing: run paper_2503_18056_amd.build.build()")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib
