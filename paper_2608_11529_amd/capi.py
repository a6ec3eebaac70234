"""ctypes binding of libmrpt2.so (argument marshalling only).

Every function here forwards to the C interface declared in include/mrpt2.h;
no arithmetic of the method runs in Python.  Device buffers are passed as
raw pointers (torch tensors' data_ptr()), streams as raw HIP stream handles.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrpt2.so")

MAX_SUB = 16
MAX_SETS = 4
N_CLASS = 9
CLASSES = [(2, 2), (1, 2), (0, 2), (2, 1), (1, 1), (0, 1), (2, 0), (1, 0), (0, 0)]
N_STAGE = 23
STAGES = (["factor_tables", "occupied_integrals", "reference_energy", "pair_integrals"]
          + ["sigma_%d%d" % c for c in CLASSES] + ["prep_%d%d" % c for c in CLASSES] + ["reduce"])

N_STAGE_B = 49
STAGES_B = (STAGES + ["bwd_row_%d%d" % c for c in CLASSES] + ["bwd_str_%d%d" % c for c in CLASSES]
            + ["bwd_string_fin", "bwd_reference", "bwd_couplings", "bwd_pair_integrals",
               "bwd_occupied_integrals", "bwd_tables", "bwd_outputs", "bwd_clear"])

STATUS = {
    0: "ok", 1: "invalid argument", 2: "inconsistent or unsupported sizes",
    3: "unsupported option", 4: "persistent or workspace region too small",
    5: "HIP runtime error", 6: "non-finite input or zero denominator",
}


class Mrpt2Error(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {STATUS.get(code, 'unknown')} (status {code})")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("n_frozen_core", ctypes.c_int32),
        ("n_core", ctypes.c_int32),
        ("n_virt", ctypes.c_int32),
        ("n_sub", ctypes.c_int32),
        ("sub_size", ctypes.c_int32 * MAX_SUB),
        ("sub_base", ctypes.c_int32 * MAX_SUB),
        ("max_hops", ctypes.c_int32),
        ("n_act_elec", ctypes.c_int32),
        ("q_mode", ctypes.c_int32),
        ("n_sets", ctypes.c_int32),
        ("rank", ctypes.c_int32 * MAX_SETS),
        ("weight", ctypes.c_double * MAX_SETS),
        ("precision", ctypes.c_int32),
        ("level_shift_b", ctypes.c_double),
        ("layout", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("n_orb", ctypes.c_int32),
        ("n_corr", ctypes.c_int32),
        ("n_chol", ctypes.c_int32),
        ("n_ref", ctypes.c_int64),
        ("n_ext", ctypes.c_int64),
        ("n_ext_class", ctypes.c_int64 * N_CLASS),
        ("n_strings_class", ctypes.c_int64 * N_CLASS),
        ("n_conn_class", ctypes.c_int64 * N_CLASS),
        ("flop_integral", ctypes.c_double),
        ("flop_sigma", ctypes.c_double),
        ("bytes_factors", ctypes.c_double),
        ("n_patterns_class", ctypes.c_int32 * N_CLASS),
        ("n_ref_couplings", ctypes.c_int64),
        ("kernel_class", ctypes.c_int32 * N_CLASS),
    ]


class Inputs(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_void_p),
        ("B", ctypes.c_void_p * MAX_SETS),
        ("c", ctypes.c_void_p),
    ]


class Grads(ctypes.Structure):
    _fields_ = [
        ("dh", ctypes.c_void_p),
        ("dB", ctypes.c_void_p * MAX_SETS),
        ("dc", ctypes.c_void_p),
    ]


class Tuning(ctypes.Structure):
    """Launch-shape targets of one instance per excitation class (0 = built-in rule)."""
    _fields_ = [
        ("sigma_blocks", ctypes.c_int32 * N_CLASS),
        ("bwd_blocks", ctypes.c_int32 * N_CLASS),
        ("bwd_row_blocks", ctypes.c_int32 * N_CLASS),
        ("pair_tile", ctypes.c_int32),
    ]


class Block(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("n_holes", ctypes.c_int32),
        ("hole", ctypes.c_int32 * 2),
        ("a_lo", ctypes.c_int32), ("a_hi", ctypes.c_int32),
        ("b_lo", ctypes.c_int32), ("b_hi", ctypes.c_int32),
        ("row_lo", ctypes.c_int64), ("row_hi", ctypes.c_int64),
        ("s_lo", ctypes.c_int64), ("s_hi", ctypes.c_int64),
    ]


_lib = None


def lib():
    """Load libmrpt2.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2608_11529_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, st = ctypes.c_void_p, ctypes.c_int
        L.mrpt2_plan.argtypes = [ctypes.POINTER(Desc), ctypes.c_int32, ctypes.POINTER(vp)]
        L.mrpt2_plan.restype = st
        L.mrpt2_plan_tuned.argtypes = [ctypes.POINTER(Desc), ctypes.c_int32, ctypes.POINTER(Tuning),
                                       ctypes.POINTER(vp)]
        L.mrpt2_plan_tuned.restype = st
        L.mrpt2_plan_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        L.mrpt2_plan_sizes.restype = st
        L.mrpt2_plan_upload.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.mrpt2_plan_upload.restype = st
        L.mrpt2_plan_info.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Info)]
        L.mrpt2_plan_info.restype = st
        L.mrpt2_plan_ref_strings.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
        L.mrpt2_plan_ref_strings.restype = st
        L.mrpt2_energy.argtypes = [vp, ctypes.POINTER(Inputs), vp, vp, ctypes.c_size_t, vp, vp, vp]
        L.mrpt2_energy.restype = st
        L.mrpt2_energy_async.argtypes = [vp, ctypes.POINTER(Inputs), vp, vp, ctypes.c_size_t, vp, vp, vp]
        L.mrpt2_energy_async.restype = st
        L.mrpt2_check.argtypes = [vp, vp, vp]
        L.mrpt2_check.restype = st
        L.mrpt2_delta_stats.argtypes = [vp, ctypes.POINTER(Inputs), vp, vp, ctypes.c_size_t, vp, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.mrpt2_delta_stats.restype = st
        L.mrpt2_energy_roots.argtypes = [vp, ctypes.POINTER(Inputs), ctypes.c_int32, vp, vp, ctypes.c_size_t,
                                         vp, vp, vp]
        L.mrpt2_energy_roots.restype = st
        L.mrpt2_reference_states_size.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.mrpt2_reference_states_size.restype = st
        L.mrpt2_reference_states.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Inputs), ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_int32, vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp, vp, vp,
                                             ctypes.POINTER(ctypes.c_int32)]
        L.mrpt2_reference_states.restype = st
        L.mrpt2_reference_sigma.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Inputs), ctypes.c_int32, vp, vp, vp,
                                            ctypes.c_size_t, vp, vp]
        L.mrpt2_reference_sigma.restype = st
        L.mrpt2_reference_states_direct_size.argtypes = L.mrpt2_reference_states_size.argtypes
        L.mrpt2_reference_states_direct_size.restype = st
        L.mrpt2_reference_states_direct.argtypes = L.mrpt2_reference_states.argtypes
        L.mrpt2_reference_states_direct.restype = st
        L.mrpt2_hermitian_eigh.argtypes = [ctypes.c_int32, vp, vp, vp]
        L.mrpt2_hermitian_eigh.restype = st
        L.mrpt2_energy_timed.argtypes = [vp, ctypes.POINTER(Inputs), vp, vp, ctypes.c_size_t, vp, vp, vp,
                                         ctypes.POINTER(ctypes.c_float)]
        L.mrpt2_energy_timed.restype = st
        L.mrpt2_reference_hamiltonian.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Inputs), vp, vp,
                                                  ctypes.c_size_t, vp, vp]
        L.mrpt2_reference_hamiltonian.restype = st
        L.mrpt2_plan_class_blocks.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        L.mrpt2_plan_class_blocks.restype = st
        L.mrpt2_plan_class_block.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                             ctypes.POINTER(Block)]
        L.mrpt2_plan_class_block.restype = st
        L.mrpt2_plan_class_strings.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
        L.mrpt2_plan_class_strings.restype = st
        L.mrpt2_class_partials.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.mrpt2_class_partials.restype = st
        L.mrpt2_plan_backward_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.mrpt2_plan_backward_size.restype = st
        L.mrpt2_energy_backward.argtypes = [vp, ctypes.POINTER(Inputs), vp, vp, ctypes.c_size_t, vp,
                                            ctypes.c_size_t, vp, ctypes.POINTER(Grads), vp, vp]
        L.mrpt2_energy_backward.restype = st
        L.mrpt2_energy_backward_async.argtypes = L.mrpt2_energy_backward.argtypes
        L.mrpt2_energy_backward_async.restype = st
        L.mrpt2_energy_backward_timed.argtypes = [vp, ctypes.POINTER(Inputs), vp, vp, ctypes.c_size_t, vp,
                                                  ctypes.c_size_t, vp, ctypes.POINTER(Grads), vp, vp,
                                                  ctypes.POINTER(ctypes.c_float)]
        L.mrpt2_energy_backward_timed.restype = st
        L.mrpt2_energy_static.argtypes = [vp, ctypes.POINTER(Inputs), vp, vp, vp, vp]
        L.mrpt2_energy_static.restype = st
        L.mrpt2_static_workspace_bytes.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
        L.mrpt2_static_workspace_bytes.restype = st
        L.mrpt2_plan_destroy.argtypes = [vp]
        L.mrpt2_plan_destroy.restype = None
        L.mrpt2_status_string.argtypes = [st]
        L.mrpt2_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(code, where):
    if code != 0:
        raise Mrpt2Error(code, where)


EXPORTED = [
    "mrpt2_plan", "mrpt2_plan_sizes", "mrpt2_plan_upload", "mrpt2_plan_info",
    "mrpt2_plan_ref_strings", "mrpt2_energy", "mrpt2_energy_roots", "mrpt2_reference_states_size",
    "mrpt2_reference_states", "mrpt2_hermitian_eigh", "mrpt2_energy_backward_async", "mrpt2_energy_timed", "mrpt2_reference_hamiltonian",
    "mrpt2_plan_destroy", "mrpt2_status_string", "mrpt2_plan_class_blocks", "mrpt2_plan_class_block",
    "mrpt2_plan_class_strings", "mrpt2_class_partials", "mrpt2_energy_async", "mrpt2_check",
    "mrpt2_plan_backward_size", "mrpt2_energy_backward", "mrpt2_energy_backward_timed", "mrpt2_plan_tuned",
    "mrpt2_energy_static", "mrpt2_static_workspace_bytes", "mrpt2_reference_sigma",
    "mrpt2_reference_states_direct_size", "mrpt2_reference_states_direct", "mrpt2_delta_stats",
]
