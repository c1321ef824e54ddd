"""ctypes binding of libhsweep.so (argument marshalling only).

Every computation runs inside the HIP library; this module converts Python
arguments to the C types of include/hsweep.h and turns negative return
codes into exceptions.  Loading fails loudly if the library has not been
built: there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsweep.so")

OK = 0
EINVAL = -1
ESTATE = -2
ENOMEM = -3
EDEVICE = -4
ESINGULAR = -5
ENOCONV = -6
C128 = 0
C64 = 1
DIRECTIONS = {"+x2": 0, "-x2": 1, "+x1": 2, "-x1": 3}
EDGES = {"x1=0": 0, "x1=1": 1, "x2=0": 2, "x2=1": 3}
SIDE_ABC = -2          # pml_sides entry: the absorbing boundary condition on that side
ADMISSIBILITY = {"weak": 0, "strong": 1}

_NAMES = {EINVAL: "EINVAL", ESTATE: "ESTATE", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
          ESINGULAR: "ESINGULAR", ENOCONV: "ENOCONV"}

# Every symbol declared in include/hsweep.h.
EXPORTED = [
    "hsweep_default_opts", "hsweep_setup", "hsweep_set_opts", "hsweep_get_opts", "hsweep_plan_info",
    "hsweep_factor", "hsweep_apply", "hsweep_stencil", "hsweep_solve", "hsweep_grad_c",
    "hsweep_factor_batch", "hsweep_solve_batch", "hsweep_destroy", "hsweep_last_error", "hsweep_timings",
    "hsweep_factor_profile", "hsweep_solve_adjoint", "hsweep_workspace_bytes", "hsweep_apply_noalloc",
    "hsweep_dirichlet_forcing",
    "hsweep3_setup", "hsweep3_set_opts", "hsweep3_factor", "hsweep3_apply", "hsweep3_stencil", "hsweep3_solve",
    "hsweep3_plan_info", "hsweep3_destroy",
]
# Size of the static device scratch of hsweep_apply_noalloc (HSWEEP_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 32 << 20


class HsweepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [
        ("leaf", ctypes.c_int),
        ("rank", ctypes.c_int),
        ("rank_tol", ctypes.c_double),
        ("pml_C", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("dense", ctypes.c_int),
        ("restart", ctypes.c_int),
        ("rhs_group", ctypes.c_int),
        ("direction", ctypes.c_int),
        ("pml_sides", ctypes.c_int * 4),
        ("admissibility", ctypes.c_int),
    ]


_lib = None


def load():
    """Load libhsweep.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1007_4290_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp, i, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), \
        ctypes.c_int, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "hsweep_default_opts": (None, [ctypes.POINTER(Opts)]),
        "hsweep_setup": (i, [vp, d, i, i, pp]),
        "hsweep_set_opts": (i, [vp, ctypes.POINTER(Opts)]),
        "hsweep_get_opts": (i, [vp, ctypes.POINTER(Opts)]),
        "hsweep_plan_info": (i, [vp, ip, ip, ctypes.POINTER(ctypes.c_size_t)]),
        "hsweep_factor": (i, [vp, vp]),
        "hsweep_apply": (i, [vp, vp, vp, i, vp]),
        "hsweep_stencil": (i, [vp, vp, vp, i, vp]),
        "hsweep_solve": (i, [vp, vp, vp, i, d, i, ip, dp, vp]),
        "hsweep_grad_c": (i, [vp, vp, vp, i, vp, vp]),
        "hsweep_factor_batch": (i, [pp, i, vp]),
        "hsweep_solve_batch": (i, [pp, i, pp, pp, d, i, ip, dp, vp]),
        "hsweep_destroy": (None, [vp]),
        "hsweep_last_error": (ctypes.c_char_p, []),
        "hsweep_timings": (i, [vp, dp, i]),
        "hsweep_factor_profile": (i, [vp, vp, dp, i]),
        "hsweep_solve_adjoint": (i, [vp, vp, vp, vp, i, d, i, ip, dp, vp]),
        "hsweep_workspace_bytes": (i, [vp, i, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "hsweep_apply_noalloc": (i, [vp, vp, vp, i, vp]),
        "hsweep_dirichlet_forcing": (i, [vp, i, vp, vp, i, vp]),
        "hsweep3_setup": (i, [vp, d, i, i, pp]),
        "hsweep3_set_opts": (i, [vp, ctypes.POINTER(Opts)]),
        "hsweep3_factor": (i, [vp, vp]),
        "hsweep3_apply": (i, [vp, vp, vp, i, vp]),
        "hsweep3_stencil": (i, [vp, vp, vp, i, vp]),
        "hsweep3_solve": (i, [vp, vp, vp, i, d, i, ip, dp, vp]),
        "hsweep3_plan_info": (i, [vp, ip, ctypes.POINTER(ctypes.c_size_t)]),
        "hsweep3_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code):
    if code != OK:
        msg = load().hsweep_last_error().decode(errors="replace")
        raise HsweepError(code, msg)
    return code


def default_opts():
    o = Opts()
    load().hsweep_default_opts(ctypes.byref(o))
    return o
