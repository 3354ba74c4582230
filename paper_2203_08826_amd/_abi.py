"""ctypes declarations of libqsv.so (include/qsv.h).  Argument marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# QSV_LIBRARY names another build of the same library (the sanitizer build
# of the host code that the CPU tests load); by default the in-tree one.
LIB_PATH = os.environ.get("QSV_LIBRARY") or os.path.join(HERE, "libqsv.so")

QSV_OK = 0
QSV_C64, QSV_C128 = 0, 1
MAX_TARGETS, MAX_CONTROLS = 6, 8
COST_FEATURES = 13

PLAN_PER_GATE, PLAN_GREEDY, PLAN_PASSES, PLAN_LEARNED = 0, 1, 2, 3

GATE_KINDS = {
    "MATRIX": 0, "UNITARY": 0, "H": 1, "X": 2, "Y": 3, "Z": 4, "SX": 5, "SY": 6, "SW": 7,
    "RX": 8, "RY": 9, "RZ": 10, "U1": 11, "SWAP": 12, "FSIM": 13, "DIAG": 14,
    # controlled names: the control comes from the gate's control list
    "CNOT": 2, "CZ": 4, "CU1": 11,
}


class QsvGate(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("k", ctypes.c_int),
        ("c", ctypes.c_int),
        ("targets", ctypes.c_int * MAX_TARGETS),
        ("controls", ctypes.c_int * MAX_CONTROLS),
        ("params", ctypes.c_double * 2),
        ("data", ctypes.c_void_p),
    ]


class QsvPlanOptions(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("kmax", ctypes.c_int), ("local_bits", ctypes.c_int),
                ("use_mfma", ctypes.c_int), ("jit", ctypes.c_int)]


class QsvPlanStats(ctypes.Structure):
    _fields_ = [("n_launches", ctypes.c_int), ("n_gate_ops", ctypes.c_int), ("n_blocks", ctypes.c_int),
                ("n_mfma_blocks", ctypes.c_int), ("n_passes", ctypes.c_int), ("mode_used", ctypes.c_int),
                ("n_jit_passes", ctypes.c_int),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double), ("predicted_s", ctypes.c_double)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_f = ctypes.c_float
_ip = ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)

SIGNATURES = {
    "qsv_abi_version": ([], _i),
    "qsv_status_string": ([_i], ctypes.c_char_p),
    "qsv_last_error": ([], ctypes.c_char_p),
    "qsv_validate": ([_i, _i, _vp, _i, _vp, _i], _i),
    "qsv_group_index_host": ([_i, _vp, _i, ctypes.c_uint64, ctypes.c_uint64, _vp], _i),
    "qsv_apply_matrix": ([_vp, _i, _i, _vp, _vp, _i, _vp, _i, _vp], _i),
    "qsv_apply_x": ([_vp, _i, _i, _i, _vp, _i, _vp], _i),
    "qsv_apply_y": ([_vp, _i, _i, _i, _vp, _i, _vp], _i),
    "qsv_apply_z": ([_vp, _i, _i, _i, _vp, _i, _vp], _i),
    "qsv_apply_swap": ([_vp, _i, _i, _i, _i, _vp, _i, _vp], _i),
    "qsv_apply_phase": ([_vp, _i, _i, _i, _d, _vp, _i, _vp], _i),
    "qsv_apply_diagonal": ([_vp, _i, _i, _vp, _vp, _i, _vp, _i, _vp], _i),
    "qsv_apply_fsim": ([_vp, _i, _i, _i, _i, _d, _d, _vp], _i),
    "qsv_scale": ([_vp, _i, _i, _d, _d, _vp], _i),
    "qsv_gate_matrix": ([_vp, _vp], _i),
    "qsv_plan_create": ([_i, _i, _vp, _i, _vp, _vp], _i),
    "qsv_plan_stats_get": ([_vp, _vp], _i),
    "qsv_plan_blocks": ([_vp, _vp, _i], _i),
    "qsv_plan_execute": ([_vp, _vp, _vp], _i),
    "qsv_plan_destroy": ([_vp], None),
    "qsv_plan_execute_ops": ([_vp, _vp, _i, _i, _vp], _i),
    "qsv_plan_op_info": ([_vp, _i, _vp, _vp, _vp], _i),
    "qsv_plan_op_program": ([_vp, _i, _vp, ctypes.c_size_t, _vp], _i),
    "qsv_plan_op_source": ([_vp, _i, _vp, ctypes.c_size_t, _vp], _i),
    "qsv_plan_op_gates": ([_vp, _i, _vp, ctypes.c_size_t, _vp], _i),
    "qsv_apply_block": ([_vp, _i, _i, _vp, _vp, _i, _vp], _i),
    "qsv_run_pass": ([_vp, _i, _i, _vp, _i, _vp, _i, _vp], _i),
    "qsv_sliced_run": ([_vp, _i, _i, _vp, _i, _i, _i, _i, _vp], _i),
    "qsv_probabilities": ([_vp, _i, _i, _vp, _i, _vp, _vp], _i),
    "qsv_probabilities_noalloc": ([_vp, _i, _i, _vp, _i, _vp, _vp], _i),
    "qsv_norm2": ([_vp, _i, _i, _vp, _vp], _i),
    "qsv_inner": ([_vp, _vp, _i, _i, _vp, _vp], _i),
    "qsv_expval_zz_x": ([_vp, _i, _i, _d, _d, _i, _vp, _vp], _i),
    "qsv_apply_tfim": ([_vp, _vp, _i, _i, _d, _d, _i, _vp], _i),
    "qsv_collapse": ([_vp, _i, _i, _vp, _i, ctypes.c_uint64, _vp, _vp], _i),
    "qsv_sample_cdf": ([_vp, _i, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp], _i),
    "qsv_sample_metropolis": ([_vp, _i, _vp, _vp, _vp, _i, ctypes.c_int64, _vp, _vp], _i),
    "qsv_dm_plan_create": ([_i, _i, _vp, _i, _vp, _vp], _i),
    "qsv_dm_apply_channel": ([_vp, _i, _i, _vp, _i, _i, _vp], _i),
    "qsv_dm_trace": ([_vp, _i, _i, _vp, _vp], _i),
    "qsv_dm_probabilities": ([_vp, _i, _i, _vp, _i, _vp, _vp], _i),
    "qsv_adjoint_grad": ([_vp, _vp, _i, _i, _vp, _i, _vp, _vp], _i),
    "qsv_mlp_forward": ([_vp, _vp, _i, _vp, _i, _vp, _vp, _vp], _i),
    "qsv_mlp_backward": ([_vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp], _i),
    "qsv_mlp_adam": ([_vp, _vp, _vp, _vp, _i, _i, _f, _f, _f, _f, _vp], _i),
    "qsv_mlp_param_count": ([_vp, _i], _i),
    "qsv_cost_model_set": ([_vp, _vp, _i, _vp, _vp], _i),
    "qsv_plan_op_features": ([_vp, _i, _vp], _i),
    "qsv_memory_stats": ([_vp, _vp, _i], _i),
}

_lib = None


class QsvError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__("%s failed with status %d: %s" % (fn, status, msg))
        self.status = status


def load():
    """Load libqsv.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libqsv.so is not built: run `python -m paper_2203_08826_amd.build` "
                              "or __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(fn_name, status):
    if status != QSV_OK:
        msg = load().qsv_last_error().decode(errors="replace")
        raise QsvError(fn_name, status, msg)
    return status
