"""ctypes mirror of include/ibmlbm.h.  Loads the in-tree libibmlbm.so and
raises if it is missing: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibmlbm.so")

OK, EINVAL, ENOMEM, EDEVICE, EDIVERGED, ESTATE, ERANGE = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC, BC_WALL, BC_VELOCITY, BC_PRESSURE = 0, 1, 2, 3
FP32, FP16_DEV, BF16_DEV = 0, 1, 2
ALPHA_CONST, ALPHA_SIN, ALPHA_ABS_SIN = 0, 1, 2
FIELD_RHO, FIELD_U, FIELD_FDIST = 0, 1, 2
MARKER_X, MARKER_U, MARKER_RHS, MARKER_DU, MARKER_RHO, MARKER_DA = 0, 1, 2, 3, 4, 5


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 6),
        ("tau", C.c_double),
        ("u_in", C.c_double * 3),
        ("rho_out", C.c_double),
        ("body_force", C.c_double * 3),
        ("storage", C.c_int32),
        ("check_interval", C.c_int32),
        ("u_ref", C.c_double),
        ("area_ref", C.c_double),
        ("history_steps", C.c_int64),
    ]


class Wing(C.Structure):
    _fields_ = [
        ("chord", C.c_double), ("thickness", C.c_double), ("ds", C.c_double),
        ("hinge", C.c_double * 2),
        ("pivot_frac", C.c_double), ("theta0", C.c_double), ("sense", C.c_double),
        ("alpha_shape", C.c_int32), ("pad_", C.c_int32),
        ("alpha_mean", C.c_double), ("alpha_amp", C.c_double),
        ("period_steps", C.c_double), ("phase", C.c_double),
        ("trans_amp", C.c_double), ("trans_angle", C.c_double),
    ]


Handle = C.c_void_p
_dp = C.POINTER(C.c_double)

# (name, restype, argtypes) for every symbol the header declares
SIGNATURES = [
    ("ibmlbm_workspace_bytes", C.c_size_t, [C.POINTER(Config), C.c_int32, C.POINTER(Wing)]),
    ("ibmlbm_create", C.c_int, [C.POINTER(Config), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(Handle)]),
    ("ibmlbm_create_noalloc", C.c_int, [C.POINTER(Config), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(Handle)]),
    ("ibmlbm_init_fields", C.c_int, [Handle, _dp, _dp, _dp, C.c_int64]),
    ("ibmlbm_set_kinematics", C.c_int, [Handle, C.c_int32, C.POINTER(Wing)]),
    ("ibmlbm_step", C.c_int, [Handle, C.c_int32]),
    ("ibmlbm_step_batch", C.c_int, [C.POINTER(Handle), C.c_int32, C.c_int32]),
    ("ibmlbm_set_stream", C.c_int, [Handle, C.c_void_p]),
    ("ibmlbm_step_count", C.c_int64, [Handle]),
    ("ibmlbm_forces", C.c_int, [Handle, C.c_int64, C.c_int64, _dp]),
    ("ibmlbm_fields", C.c_int, [Handle, C.c_int32, _dp]),
    ("ibmlbm_markers", C.c_int, [Handle, C.c_int32, _dp]),
    ("ibmlbm_marker_count", C.c_int32, [Handle]),
    ("ibmlbm_mass", C.c_int, [Handle, C.POINTER(C.c_int64), _dp]),
    ("ibmlbm_timing", C.c_int, [Handle, C.c_int32]),
    ("ibmlbm_read_timing", C.c_int, [Handle, _dp, C.POINTER(C.c_int64), _dp, _dp]),
    ("ibmlbm_bytes_per_cell", C.c_int32, [Handle]),
    ("ibmlbm_destroy", C.c_int, [Handle]),
    ("ibmlbm_last_error", C.c_char_p, [Handle]),
    ("ibmlbm_lattice_params", C.c_int, [C.c_double] * 5 + [_dp] * 4),
    ("ibmlbm_plate_params", C.c_int, [C.c_double] * 3 + [_dp]),
    ("ibmlbm_figure_eight_params", C.c_int, [C.c_double] * 4 + [_dp] * 2),
]

_lib = None


def _hip_runtimes():
    """Distinct libamdhip64 files mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                parts = line.split()
                if len(parts) >= 6 and "libamdhip64.so" in parts[-1]:
                    paths.add(os.path.realpath(parts[-1]))
    except OSError:
        pass
    return paths


def load():
    """Load libibmlbm.so (built in-tree by __graft_entry__.build()).

    torch ships its own HIP runtime with the same sonames as ROCm's
    (libamdhip64.so.7, libhsa-runtime64.so.1).  torch is imported first so
    that the solver binds to the runtime torch already mapped; two HIP
    runtimes in one process would each open the GPU on their own.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2102_01305_amd.build`")
    try:
        import torch  # noqa: F401  (maps torch's HIP runtime before ours)
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError(f"two HIP runtimes are mapped into this process: {sorted(runtimes)}")
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class IbmlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ibmlbm error {code}: {msg}")
        self.code = code


def check(code, handle=None):
    if code != OK:
        msg = load().ibmlbm_last_error(handle)
        raise IbmlbmError(code, msg.decode() if msg else "")
    return code
