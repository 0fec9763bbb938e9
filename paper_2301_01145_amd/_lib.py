"""ctypes binding of libhipoisson.so: the C-ABI functions under their C names.

Only argument marshalling happens here; every step of a solve runs in the
library's HIP kernels.  The library is loaded on first use and a missing or
unloadable library raises immediately -- there is no fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhipoisson.so")

HP_OK, HP_E_ARG, HP_E_UNSUPPORTED, HP_E_NOMEM, HP_E_DEVICE, HP_E_STATE = 0, -1, -2, -3, -4, -5
HP_PERIODIC, HP_DIRICHLET, HP_NEUMANN, HP_UNBOUNDED, HP_MIXED = 0, 1, 2, 3, 4
HP_REGULAR, HP_STAGGERED = 0, 1
HP_OP_PS, HP_OP_FD2, HP_G_GAUSS2 = 0, 1, 2
HP_G_GAUSS4, HP_G_GAUSS6, HP_G_GAUSS8, HP_G_GAUSS10, HP_G_SPECTRAL = 3, 4, 5, 6, 7
HP_D_NONE, HP_D_GRAD, HP_D_CURL, HP_D_DIV, HP_D_NABLA = 0, 1, 2, 3, 4
HP_F32, HP_F64 = 0, 1
HP_Q_MODEL_BYTES, HP_Q_WORKSPACE_BYTES, HP_Q_NUM_PASSES, HP_Q_NUM_OUTPUTS, HP_Q_NUM_DERIVS = 1, 2, 3, 4, 5
HP_Q_BATCH_ERROR = 6
HP_Q_TUNED_PASSES, HP_Q_TUNE_DEFAULT_MS, HP_Q_TUNE_BEST_MS, HP_Q_BATCH_TILES = 7, 8, 9, 10
HP_Q_ZERO_MODE = 11
HP_Q_BATCH_KERNEL = 12

# Every exported function of include/hipoisson.h (checked by the ABI tests).
EXPORTS = (
    "hp_plan_create", "hp_plan_create_batched", "hp_input_shape", "hp_output_shape",
    "hp_set_input", "hp_set_boundary", "hp_bind_output", "hp_bind_gradient", "hp_solve",
    "hp_solve_adjoint", "hp_get_output", "hp_get_gradient", "hp_query", "hp_plan_destroy",
    "hp_status_string", "hp_last_error", "hp_set_timing", "hp_pass_stats", "hp_autotune",
    "hp_zero_mode_noalloc", "hp_device_copy",
)


class hp_desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("ncomp", ctypes.c_int),
        ("nc", ctypes.c_int64 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int),
        ("grid", ctypes.c_int),
        ("kernel", ctypes.c_int),
        ("diff", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("inhomogeneous", ctypes.c_int),
        ("reg_sigma_cells", ctypes.c_double),
        ("bc_axis", ctypes.c_int * 3),
    ]


class HipoissonError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"hipoisson status {status}: {message}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_SIG = {
    "hp_plan_create": ([ctypes.POINTER(hp_desc), _P, ctypes.POINTER(_P)], _I),
    "hp_plan_create_batched": ([ctypes.POINTER(hp_desc), _I, _P, ctypes.POINTER(_P)], _I),
    "hp_input_shape": ([_P, _I, ctypes.POINTER(ctypes.c_int64)], _I),
    "hp_output_shape": ([_P, _I, ctypes.POINTER(ctypes.c_int64)], _I),
    "hp_set_input": ([_P, _I, _I, _P, _I], _I),
    "hp_set_boundary": ([_P, _I, _I, _I, _I, _P, _I], _I),
    "hp_bind_output": ([_P, _I, _I, _P], _I),
    "hp_bind_gradient": ([_P, _I, _I, _P], _I),
    "hp_solve": ([_P], _I),
    "hp_solve_adjoint": ([_P], _I),
    "hp_get_output": ([_P, _I, _I, _P, _I], _I),
    "hp_get_gradient": ([_P, _I, _I, _P, _I], _I),
    "hp_query": ([_P, _I, ctypes.POINTER(ctypes.c_double)], _I),
    "hp_plan_destroy": ([_P], _I),
    "hp_status_string": ([_I], ctypes.c_char_p),
    "hp_last_error": ([_P], ctypes.c_char_p),
    "hp_set_timing": ([_P, _I], _I),
    "hp_autotune": ([_P, _I], _I),
    "hp_zero_mode_noalloc": ([_P, _P], _I),
    "hp_device_copy": ([_P, _P, ctypes.c_size_t, _P], _I),
    "hp_pass_stats": ([_P, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_char_p)], _I),
}


def lib():
    """Load libhipoisson.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run __graft_entry__.build() "
                               "or python paper_2301_01145_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIG.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status, plan=None):
    if status != HP_OK:
        msg = lib().hp_last_error(plan).decode()
        raise HipoissonError(status, msg or lib().hp_status_string(status).decode())
    return status


# ----------------------------------------------------- functions, C names
def hp_plan_create(desc, stream=None):
    out = _P()
    _check(lib().hp_plan_create(ctypes.byref(desc), stream, ctypes.byref(out)))
    return out.value


def hp_plan_create_batched(descs, stream=None):
    arr = (hp_desc * len(descs))(*descs)
    out = _P()
    _check(lib().hp_plan_create_batched(arr, len(descs), stream, ctypes.byref(out)))
    return out.value


def hp_input_shape(plan, problem=0):
    s = (ctypes.c_int64 * 3)()
    _check(lib().hp_input_shape(plan, problem, s), plan)
    return tuple(s)


def hp_output_shape(plan, problem=0):
    s = (ctypes.c_int64 * 3)()
    _check(lib().hp_output_shape(plan, problem, s), plan)
    return tuple(s)


def hp_set_input(plan, problem, comp, ptr, on_device):
    _check(lib().hp_set_input(plan, problem, comp, ptr, int(on_device)), plan)


def hp_set_boundary(plan, problem, axis, side, comp, ptr, on_device):
    _check(lib().hp_set_boundary(plan, problem, axis, side, comp, ptr, int(on_device)), plan)


def hp_bind_output(plan, problem, comp, ptr):
    _check(lib().hp_bind_output(plan, problem, comp, ptr), plan)


def hp_bind_gradient(plan, problem, comp, ptr):
    _check(lib().hp_bind_gradient(plan, problem, comp, ptr), plan)


def hp_solve(plan):
    _check(lib().hp_solve(plan), plan)


def hp_solve_adjoint(plan):
    _check(lib().hp_solve_adjoint(plan), plan)


def hp_get_output(plan, problem, comp, ptr, on_device):
    _check(lib().hp_get_output(plan, problem, comp, ptr, int(on_device)), plan)


def hp_get_gradient(plan, problem, comp, ptr, on_device):
    _check(lib().hp_get_gradient(plan, problem, comp, ptr, int(on_device)), plan)


def hp_query(plan, what):
    v = ctypes.c_double()
    _check(lib().hp_query(plan, what, ctypes.byref(v)), plan)
    return v.value


def hp_plan_destroy(plan):
    _check(lib().hp_plan_destroy(plan))


def hp_autotune(plan, reps=5):
    _check(lib().hp_autotune(plan, int(reps)), plan)


def hp_set_timing(plan, enable):
    _check(lib().hp_set_timing(plan, int(enable)), plan)


def hp_pass_stats(plan, max_passes=64):
    """[(name, mean ms, model bytes)] per pass of the solves timed since the last call."""
    n = _I()
    ms = (ctypes.c_double * max_passes)()
    by = (ctypes.c_double * max_passes)()
    nm = (ctypes.c_char_p * max_passes)()
    _check(lib().hp_pass_stats(plan, max_passes, ctypes.byref(n), ms, by, nm), plan)
    return [(nm[i].decode(), ms[i], by[i]) for i in range(min(n.value, max_passes))]


def hp_status_string(status):
    return lib().hp_status_string(status).decode()


def hp_last_error(plan=None):
    return lib().hp_last_error(plan).decode()


def hp_zero_mode_noalloc(plan, out_ptr):
    """Per-component zero modes into the caller's device buffer (ncomp doubles)."""
    _check(lib().hp_zero_mode_noalloc(plan, out_ptr), plan)


def hp_device_copy(src_ptr, dst_ptr, nbytes, stream=None):
    """Plain streaming device copy (the measured bandwidth ceiling of bench.py)."""
    _check(lib().hp_device_copy(src_ptr, dst_ptr, int(nbytes), stream))
