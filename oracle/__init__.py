"""FP64 CPU oracle of the EWOD Shan-Chen D2Q9 lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library: the arithmetic lives in ``lbm_oracle.c`` (plain
loops, FP64), and this module only marshals numpy arrays through ctypes.

Every function cites the passage of the paper (arXiv:0708.4182) it follows in
``lbm_oracle.c``.  Pins against closed forms, invariants and textbook limits
live in ``tests/test_oracle_*.py``.  ``round_storage`` (numpy, here) defines
the 16-bit population storage, which is not part of the paper's model.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build() -> str:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math; the
    per-node loops run on OpenMP threads, with bitwise the same results)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("tau", C.c_double), ("rho0", C.c_double),
                ("g_axis", C.c_double), ("g_diag", C.c_double),
                ("w_axis", C.c_double), ("w_diag", C.c_double),
                ("rho_c", C.c_double), ("f_elec", C.c_double),
                ("elec_layers", C.c_int32), ("elec_walls", C.c_uint32),
                ("accel_x", C.c_double), ("accel_y", C.c_double),
                ("collision", C.c_int32), ("trt_magic", C.c_double),
                ("elec_normal", C.c_int32), ("mrt_s_e", C.c_double), ("mrt_s_eps", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER(_Params)
        dp = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        lib.orc_velocity_set.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp,
                                         C.POINTER(C.c_int32)]
        lib.orc_equilibrium.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        lib.orc_phi.argtypes = [C.c_double, C.c_double]
        lib.orc_phi.restype = C.c_double
        lib.orc_electric_layer.argtypes = [P, u8, u8, u8]
        lib.orc_flags.argtypes = [P, u8, C.POINTER(C.c_uint16)]
        lib.orc_electric_normal.argtypes = [P, u8, u8]
        lib.orc_moments.argtypes = [P, u8, dp, dp, dp, dp]
        lib.orc_forces.argtypes = [P, u8, dp, dp, dp, dp]
        lib.orc_init.argtypes = [P, u8, dp, dp, dp, dp]
        lib.orc_step.argtypes = [P, u8, dp, C.c_int64]
        lib.orc_step.restype = C.c_int
        lib.orc_step_ext.argtypes = [P, u8, dp, C.c_int64, dp]
        lib.orc_step_ext.restype = C.c_int
        lib.orc_flux.argtypes = [P, u8, dp, dp, dp]
        lib.orc_profile.argtypes = [P, u8, dp, dp]
        lib.orc_trt_omega_minus.argtypes = [C.c_double, C.c_double]
        lib.orc_trt_omega_minus.restype = C.c_double
        lib.orc_threads.argtypes = [C.c_int]
        lib.orc_threads.restype = C.c_int
        _lib = lib
    return _lib


def _params(p) -> _Params:
    return _Params(int(p.nx), int(p.ny), float(p.tau), float(p.rho0), float(p.g_axis),
                   float(p.g_diag), float(p.w_axis), float(p.w_diag), float(p.rho_c),
                   float(p.f_elec), int(p.elec_layers), int(p.elec_walls),
                   float(p.accel_x), float(p.accel_y), int(getattr(p, "collision", 0)),
                   float(getattr(p, "trt_magic", 3.0 / 16.0)), int(getattr(p, "elec_normal", 0)),
                   float(getattr(p, "mrt_s_e", 1.64)), float(getattr(p, "mrt_s_eps", 1.54)))


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _solid(p, solid):
    s = np.ascontiguousarray(solid, np.uint8)
    assert s.shape == (p.ny, p.nx)
    return s


def velocity_set():
    """(e [9,2] int, w [9], opp [9]) as the oracle builds them from the paper."""
    ex = np.zeros(9, np.int32); ey = np.zeros(9, np.int32)
    w = np.zeros(9); opp = np.zeros(9, np.int32)
    _load().orc_velocity_set(ex.ctypes.data_as(C.POINTER(C.c_int32)),
                             ey.ctypes.data_as(C.POINTER(C.c_int32)), _d(w),
                             opp.ctypes.data_as(C.POINTER(C.c_int32)))
    return np.stack([ex, ey], 1), w, opp


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    """f^eq of eq. (3) for one node."""
    out = np.zeros(9)
    _load().orc_equilibrium(float(rho), float(ux), float(uy), _d(out))
    return out


def phi(rho0: float, rho: float) -> float:
    return _load().orc_phi(float(rho0), float(rho))


def electric_normal(p, solid):
    """Direction code (0: towards the electrode; a in 1..8: along e_a) of the
    electric force per node."""
    s = _solid(p, solid)
    code = np.zeros_like(s)
    _load().orc_electric_normal(C.byref(_params(p)), _u8(s), _u8(code))
    return code


def trt_omega_minus(tau: float, magic: float) -> float:
    """omega- of the TRT operator: (tau - 1/2)(1/omega- - 1/2) = Lambda."""
    return _load().orc_trt_omega_minus(float(tau), float(magic))


def electric_layer(p, solid):
    s = _solid(p, solid)
    layer = np.zeros_like(s); top = np.zeros_like(s)
    _load().orc_electric_layer(C.byref(_params(p)), _u8(s), _u8(layer), _u8(top))
    return layer, top


def flags(p, solid) -> np.ndarray:
    """Per-node flag words (neighbour-solid bits, solid, layer, top side)."""
    s = _solid(p, solid)
    out = np.zeros(s.shape, np.uint16)
    _load().orc_flags(C.byref(_params(p)), _u8(s), out.ctypes.data_as(C.POINTER(C.c_uint16)))
    return out


def moments(p, solid, f):
    """(rho, ux, uy) of eq. (2) from populations f[9][ny][nx]."""
    s = _solid(p, solid)
    f = np.ascontiguousarray(f, np.float64)
    rho = np.zeros(s.shape); ux = np.zeros(s.shape); uy = np.zeros(s.shape)
    _load().orc_moments(C.byref(_params(p)), _u8(s), _d(f), _d(rho), _d(ux), _d(uy))
    return rho, ux, uy


def forces(p, solid, rho):
    """(Fs, Fw, Fe), each [2][ny][nx], from a density field."""
    s = _solid(p, solid)
    rho = np.ascontiguousarray(rho, np.float64)
    Fs = np.zeros((2,) + s.shape); Fw = np.zeros_like(Fs); Fe = np.zeros_like(Fs)
    _load().orc_forces(C.byref(_params(p)), _u8(s), _d(rho), _d(Fs), _d(Fw), _d(Fe))
    return Fs, Fw, Fe


def init(p, solid, rho, ux=None, uy=None) -> np.ndarray:
    """Populations at t = 0: f^eq(rho, u) on fluid nodes."""
    s = _solid(p, solid)
    rho = np.ascontiguousarray(rho, np.float64)
    ux = np.zeros(s.shape) if ux is None else np.ascontiguousarray(ux, np.float64)
    uy = np.zeros(s.shape) if uy is None else np.ascontiguousarray(uy, np.float64)
    f = np.zeros((9,) + s.shape)
    _load().orc_init(C.byref(_params(p)), _u8(s), _d(rho), _d(ux), _d(uy), _d(f))
    return f


def step(p, solid, f, nsteps: int) -> np.ndarray:
    """Advance ``nsteps`` steps in place on a float64 f[9][ny][nx]; returns f.

    Raises FloatingPointError if a fluid density became non-positive or NaN.
    """
    s = _solid(p, solid)
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (9,) + s.shape
    if _load().orc_step(C.byref(_params(p)), _u8(s), _d(f), int(nsteps)):
        raise FloatingPointError("oracle: density became non-positive or not finite")
    return f


def step_ext(p, solid, f, nsteps: int, acc) -> np.ndarray:
    """``step`` with a per-node acceleration field acc [2][ny][nx] (x plane,
    then y plane) added to the driving acceleration: body force rho (g + acc).
    Raises FloatingPointError as ``step``."""
    s = _solid(p, solid)
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (9,) + s.shape
    acc = np.ascontiguousarray(acc, np.float64)
    assert acc.shape == (2,) + s.shape
    if _load().orc_step_ext(C.byref(_params(p)), _u8(s), _d(f), int(nsteps), _d(acc)):
        raise FloatingPointError("oracle: density became non-positive or not finite")
    return f


def flux(p, solid, f):
    """(Q, M): eq. (11) flux with L = nx, and total fluid mass."""
    s = _solid(p, solid)
    f = np.ascontiguousarray(f, np.float64)
    Q = C.c_double(); M = C.c_double()
    _load().orc_flux(C.byref(_params(p)), _u8(s), _d(f), C.byref(Q), C.byref(M))
    return Q.value, M.value


def profile(p, solid, f):
    """Channel-averaged u_x per row: (1/nx) sum over the row's fluid nodes."""
    s = _solid(p, solid)
    f = np.ascontiguousarray(f, np.float64)
    out = np.zeros(p.ny)
    _load().orc_profile(C.byref(_params(p)), _u8(s), _d(f), _d(out))
    return out


def threads(n: int = 0) -> int:
    """Set the oracle's thread count (n > 0) and return the count in use."""
    return int(_load().orc_threads(int(n)))


def _round_bf16(a):
    """Nearest value with 8 significant bits (bfloat16), ties to even."""
    m, e = np.frexp(np.asarray(a, np.float64))     # a = m 2^e, 1/2 <= |m| < 1
    return np.ldexp(np.round(np.ldexp(m, 8)), e - 8)


def round_storage(p, solid, f, storage: int) -> np.ndarray:
    """The populations as a 16-bit deviation store holds them (in place; returns f).

    On every fluid node each f_a becomes w_a rho_ref + r(f_a - w_a rho_ref),
    with r rounding to the nearest FP16 (storage 1) or BF16 (storage 2) value,
    ties to even; rho_ref is p.rho_ref, or rho0 where that is 0.  Storage 0
    (FP32) leaves f unchanged: the oracle keeps FP64.  Applied after every step
    this is the FP64 model with the storage format's rounding and nothing else.
    """
    if storage == 0:
        return f
    s = _solid(p, solid)
    _, w, _ = velocity_set()
    ref = p.rho_ref if p.rho_ref > 0 else p.rho0
    off = (w * ref)[:, None, None]
    fl = (s == 0)[None, :, :]
    d = f - off
    if storage == 1:
        r = d.astype(np.float16).astype(np.float64)
    elif storage == 2:
        r = _round_bf16(d)
    else:
        raise ValueError("storage must be 0, 1 or 2")
    np.copyto(f, np.where(fl, off + r, f))
    return f


def run(case, nsteps: int):
    """Init from an inputs.Case and advance ``nsteps``; returns f."""
    f = init(case.params, case.solid, case.rho, case.ux, case.uy)
    return step(case.params, case.solid, f, nsteps)
