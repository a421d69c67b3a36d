"""ctypes binding of liblbm (include/lbm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``liblbm.so``.  PyTorch provides the device workspace (through its
caching allocator) and the HIP stream.  There is no fallback: if the library
has not been built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_LIB") or os.path.join(HERE, "liblbm.so")

LBM_F32, LBM_F16, LBM_BF16 = 0, 1, 2
KERNELS = {"fused": 0, "split": 1, "wide2": 2, "wide4": 3, "fused8": 4, "two": 5, "three": 6}
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
          -4: "LBM_EDIVERGED", -5: "LBM_ESTATE"}

# Exported symbols of include/lbm.h (checked by the CPU tests).
SYMBOLS = ("lbm_workspace_bytes", "lbm_init", "lbm_init_device", "lbm_step", "lbm_moments",
           "lbm_flux", "lbm_flux_static", "lbm_stream_copy", "lbm_round_sr", "lbm_profile", "lbm_geometry", "lbm_set_forces", "lbm_set_accel_field", "lbm_set_tile", "lbm_set_kernel",
           "lbm_set_graph",
           "lbm_get_tile",
           "lbm_autotune", "lbm_state_bytes",
           "lbm_save_state", "lbm_load_state", "lbm_steps_done", "lbm_free", "lbm_last_error",
           "lbm_status_string", "lbm_batch_workspace_bytes", "lbm_batch_init", "lbm_batch_step",
           "lbm_batch_flux", "lbm_batch_moments", "lbm_batch_profile", "lbm_batch_geometry",
           "lbm_batch_init_device",
           "lbm_batch_set_forces", "lbm_batch_retire", "lbm_batch_set_tile", "lbm_batch_set_graph",
           "lbm_batch_set_schedule", "lbm_batch_set_kernel", "lbm_batch_get_kernel",
           "lbm_batch_autotune", "lbm_batch_steps_done", "lbm_batch_free", "lbm_batch_last_error")


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Diverged(LBMError):
    pass


class lbm_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("tau", C.c_double), ("rho0", C.c_double),
                ("g_axis", C.c_double), ("g_diag", C.c_double),
                ("w_axis", C.c_double), ("w_diag", C.c_double),
                ("rho_c", C.c_double), ("f_elec", C.c_double),
                ("elec_layers", C.c_int32), ("elec_walls", C.c_uint32),
                ("accel_x", C.c_double), ("accel_y", C.c_double),
                ("storage", C.c_int32), ("rho_ref", C.c_double),
                ("collision", C.c_int32), ("trt_magic", C.c_double),
                ("elec_normal", C.c_int32), ("rounding", C.c_int32),
                ("mrt_s_e", C.c_double), ("mrt_s_eps", C.c_double)]


def to_c_params(p) -> lbm_params:
    return lbm_params(int(p.nx), int(p.ny), float(p.tau), float(p.rho0), float(p.g_axis),
                      float(p.g_diag), float(p.w_axis), float(p.w_diag), float(p.rho_c),
                      float(p.f_elec), int(p.elec_layers), int(p.elec_walls), float(p.accel_x),
                      float(p.accel_y), int(getattr(p, "storage", 0)), float(getattr(p, "rho_ref", 0.0)),
                      int(getattr(p, "collision", 0)), float(getattr(p, "trt_magic", 3.0 / 16.0)),
                      int(getattr(p, "elec_normal", 0)), int(getattr(p, "rounding", 0)),
                      float(getattr(p, "mrt_s_e", 1.64)), float(getattr(p, "mrt_s_eps", 1.54)))


_lib = None


def load_library():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0708_4182_amd/build.py")
    # torch's HIP runtime must be in the process first: the library then binds
    # to it (same soname).  Loaded the other way round, torch would add its own
    # copy of the runtime next to the system one, and memory, streams and
    # devices of one would be unknown to the other.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, P = C.c_void_p, C.POINTER(lbm_params)
    dp, fp = C.POINTER(C.c_double), C.POINTER(C.c_float)
    lib.lbm_workspace_bytes.argtypes = [P]
    lib.lbm_workspace_bytes.restype = C.c_size_t
    lib.lbm_init.argtypes = [C.POINTER(vp), P, C.POINTER(C.c_uint8), dp, dp, dp, vp, C.c_size_t, vp]
    lib.lbm_init_device.argtypes = [vp, vp, vp, vp]
    lib.lbm_step.argtypes = [vp, C.c_int64]
    lib.lbm_moments.argtypes = [vp, vp, vp, vp, C.c_int]
    lib.lbm_flux.argtypes = [vp, dp, dp]
    lib.lbm_flux_static.argtypes = [vp, dp, dp]
    lib.lbm_stream_copy.argtypes = [vp, vp, C.c_size_t, C.c_int32, vp]
    lib.lbm_stream_copy.restype = C.c_int
    lib.lbm_round_sr.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, vp]
    lib.lbm_round_sr.restype = C.c_int
    lib.lbm_geometry.argtypes = [vp, C.POINTER(C.c_uint16)]
    lib.lbm_set_forces.argtypes = [vp, C.c_double, C.c_double, C.c_double]
    lib.lbm_set_tile.argtypes = [vp, C.c_int32, C.c_int32]
    lib.lbm_set_kernel.argtypes = [vp, C.c_int32]
    lib.lbm_set_accel_field.argtypes = [vp, vp]
    lib.lbm_set_accel_field.restype = C.c_int
    lib.lbm_set_graph.argtypes = [vp, C.c_int32]
    lib.lbm_profile.argtypes = [vp, dp]
    lib.lbm_batch_profile.argtypes = [vp, C.c_int32, dp]
    lib.lbm_get_tile.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.lbm_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_float)]
    lib.lbm_state_bytes.argtypes = [vp]
    lib.lbm_state_bytes.restype = C.c_size_t
    lib.lbm_save_state.argtypes = [vp, vp, C.c_size_t]
    lib.lbm_load_state.argtypes = [vp, vp, C.c_size_t]
    lib.lbm_steps_done.argtypes = [vp]
    lib.lbm_steps_done.restype = C.c_int64
    lib.lbm_free.argtypes = [vp]
    lib.lbm_free.restype = None
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = C.c_char_p
    lib.lbm_status_string.argtypes = [C.c_int]
    lib.lbm_status_string.restype = C.c_char_p
    PP = C.POINTER(C.c_void_p)
    lib.lbm_batch_workspace_bytes.argtypes = [C.c_int32, P]
    lib.lbm_batch_workspace_bytes.restype = C.c_size_t
    lib.lbm_batch_init.argtypes = [C.POINTER(vp), C.c_int32, P, PP, PP, PP, PP, vp, C.c_size_t, vp]
    lib.lbm_batch_step.argtypes = [vp, C.c_int64]
    lib.lbm_batch_flux.argtypes = [vp, dp, dp]
    lib.lbm_batch_moments.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_int]
    lib.lbm_batch_geometry.argtypes = [vp, C.c_int32, C.POINTER(C.c_uint16)]
    lib.lbm_batch_init_device.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.lbm_batch_set_forces.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_double]
    lib.lbm_batch_retire.argtypes = [vp, C.POINTER(C.c_uint8)]
    lib.lbm_batch_set_tile.argtypes = [vp, C.c_int32, C.c_int32]
    lib.lbm_batch_set_graph.argtypes = [vp, C.c_int32]
    lib.lbm_batch_set_schedule.argtypes = [vp, C.c_int32]
    lib.lbm_batch_set_kernel.argtypes = [vp, C.c_int32]
    lib.lbm_batch_get_kernel.argtypes = [vp]
    lib.lbm_batch_get_kernel.restype = C.c_int32
    lib.lbm_batch_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_float)]
    lib.lbm_batch_steps_done.argtypes = [vp, C.c_int32]
    lib.lbm_batch_steps_done.restype = C.c_int64
    lib.lbm_batch_free.argtypes = [vp]
    lib.lbm_batch_free.restype = None
    lib.lbm_batch_last_error.argtypes = [vp]
    lib.lbm_batch_last_error.restype = C.c_char_p
    for name in ("lbm_batch_init", "lbm_batch_step", "lbm_batch_flux", "lbm_batch_moments",
                 "lbm_batch_geometry", "lbm_batch_init_device", "lbm_batch_set_forces",
                 "lbm_batch_retire", "lbm_batch_set_tile", "lbm_batch_set_graph",
                 "lbm_batch_set_schedule", "lbm_batch_set_kernel", "lbm_batch_autotune"):
        getattr(lib, name).restype = C.c_int
    for name in ("lbm_init", "lbm_init_device", "lbm_step", "lbm_moments", "lbm_flux", "lbm_flux_static",
                 "lbm_geometry", "lbm_set_forces", "lbm_set_tile", "lbm_set_kernel", "lbm_get_tile",
                 "lbm_autotune", "lbm_save_state",
                 "lbm_load_state"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def stream_copy(dst, src, per_lane: int = 1, stream=None):
    """lbm_stream_copy between two contiguous CUDA tensors of the same byte
    size (a multiple of 16), on ``stream`` (default: torch's current stream)."""
    import torch
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("stream_copy needs contiguous device tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy: sizes differ")
    st = stream if stream is not None else torch.cuda.current_stream()
    lib = load_library()
    rc = lib.lbm_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, int(per_lane),
                             C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise LBMError(rc, lib.lbm_last_error(None).decode())


def round_sr(values, bits, storage: int, stream=None):
    """lbm_round_sr: the 16-bit stochastic rounding of the step kernels applied
    to a CUDA float32 tensor with CUDA uint32 (int32 storage) random words of
    the same size; returns the 16-bit patterns as an int16 tensor."""
    import torch
    if not (values.is_cuda and bits.is_cuda and values.dtype == torch.float32 and bits.dtype == torch.int32):
        raise ValueError("round_sr needs a float32 and an int32 CUDA tensor")
    if values.numel() != bits.numel():
        raise ValueError("round_sr: sizes differ")
    v, r = values.contiguous(), bits.contiguous()
    out = torch.empty(v.numel(), dtype=torch.int16, device=v.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    lib = load_library()
    rc = lib.lbm_round_sr(C.c_void_p(v.data_ptr()), C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr()),
                          v.numel(), int(storage), C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise LBMError(rc, lib.lbm_last_error(None).decode())
    return out


def workspace_bytes(p) -> int:
    return int(load_library().lbm_workspace_bytes(C.byref(to_c_params(p))))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Simulation:
    """One lattice on one GPU: owns a torch workspace and a liblbm handle."""

    def __init__(self, params, solid, rho, ux=None, uy=None, stream=None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP GPU; torch.cuda.is_available() is False")
        lib = load_library()
        self.torch = torch
        self.params = params
        self.device = torch.device("cuda" if device is None else device)
        self.nx, self.ny = int(params.nx), int(params.ny)
        cp = to_c_params(params)
        self._cp = cp
        nbytes = int(lib.lbm_workspace_bytes(C.byref(cp)))
        if nbytes == 0:
            raise LBMError(-1, "invalid parameters (lbm_workspace_bytes returned 0)")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream() if stream is None else stream
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            solid = np.ascontiguousarray(solid, np.uint8)
            rho = np.ascontiguousarray(rho, np.float64)
            ux = None if ux is None else np.ascontiguousarray(ux, np.float64)
            uy = None if uy is None else np.ascontiguousarray(uy, np.float64)
            h = C.c_void_p()
            st = lib.lbm_init(C.byref(h), C.byref(cp), solid.ctypes.data_as(C.POINTER(C.c_uint8)),
                              _dptr(rho), None if ux is None else _dptr(ux),
                              None if uy is None else _dptr(uy), C.c_void_p(self.ws.data_ptr()),
                              nbytes, C.c_void_p(self.stream.cuda_stream))
            if st != 0:
                raise LBMError(st, lib.lbm_last_error(None).decode())
        self.h = h
        self.lib = lib

    # ------------------------------------------------------------- helpers
    def _check(self, st):
        if st != 0:
            msg = self.lib.lbm_last_error(self.h).decode()
            raise (Diverged if st == -4 else LBMError)(st, msg)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.lbm_free(h)
            self.h = None

    close = __del__

    # ------------------------------------------------------------- calls
    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self.h, int(n)))

    def moments(self):
        """(rho, ux, uy) as host float32 [ny][nx] numpy arrays (synchronizes)."""
        out = [np.empty((self.ny, self.nx), np.float32) for _ in range(3)]
        self._check(self.lib.lbm_moments(self.h, *[C.c_void_p(o.ctypes.data) for o in out], 0))
        return tuple(out)

    def moments_device(self):
        """(rho, ux, uy) as float32 torch tensors on the device (asynchronous)."""
        t = self.torch.empty((3, self.ny, self.nx), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.lbm_moments(self.h, C.c_void_p(t[0].data_ptr()),
                                         C.c_void_p(t[1].data_ptr()), C.c_void_p(t[2].data_ptr()), 1))
        return t

    def profile(self):
        """Channel-averaged u_x per row (float64 [ny]); sums to the flux Q."""
        out = np.zeros(self.ny)
        self._check(self.lib.lbm_profile(self.h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def flux(self):
        """(Q, M) of eq. (11) and the fluid mass, FP64 (synchronizes)."""
        Q, M = C.c_double(), C.c_double()
        self._check(self.lib.lbm_flux(self.h, C.byref(Q), C.byref(M)))
        return Q.value, M.value

    def set_accel_field(self, acc):
        """Per-node acceleration field: a float32 device tensor [2][ny][nx]
        (x components, then y components), or None to remove it.  The
        tensor is kept referenced while it is set."""
        if acc is None:
            self._check(self.lib.lbm_set_accel_field(self.h, None))
            self._acc = None
            return
        if (not acc.is_cuda or acc.dtype != self.torch.float32 or not acc.is_contiguous()
                or tuple(acc.shape) != (2, self.ny, self.nx)):
            raise ValueError(f"acceleration field must be a contiguous float32 device tensor [2][{self.ny}][{self.nx}]")
        self._check(self.lib.lbm_set_accel_field(self.h, C.c_void_p(acc.data_ptr())))
        self._acc = acc

    def flux_static(self):
        """flux() through lbm_flux_static: the reduction's scratch is the
        library's static device array, nothing is allocated."""
        Q, M = C.c_double(), C.c_double()
        self._check(self.lib.lbm_flux_static(self.h, C.byref(Q), C.byref(M)))
        return Q.value, M.value

    def geometry(self) -> np.ndarray:
        out = np.empty((self.ny, self.nx), np.uint16)
        self._check(self.lib.lbm_geometry(self.h, out.ctypes.data_as(C.POINTER(C.c_uint16))))
        return out

    def set_forces(self, f_elec: float, accel_x: float = 0.0, accel_y: float = 0.0):
        self._check(self.lib.lbm_set_forces(self.h, float(f_elec), float(accel_x), float(accel_y)))

    def set_tile(self, block_x: int, rows: int):
        self._check(self.lib.lbm_set_tile(self.h, int(block_x), int(rows)))

    def set_kernel(self, kernel: str):
        """'fused' (every thread loads, computes, stores its column), 'wide2' /
        'wide4' (2 or 4 adjacent columns per thread) or 'split' (a producer
        wave streams rows into LDS); all give bitwise the same results."""
        self._check(self.lib.lbm_set_kernel(self.h, KERNELS[kernel]))

    def set_graph(self, steps_per_graph: int):
        """Replay steps as hipGraphs of steps_per_graph launches (0: off)."""
        self._check(self.lib.lbm_set_graph(self.h, int(steps_per_graph)))

    def tile(self):
        """(kernel name, block_x, rows) currently in use."""
        k, bx, r = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.lbm_get_tile(self.h, C.byref(k), C.byref(bx), C.byref(r)))
        return {v: n for n, v in KERNELS.items()}[k.value], bx.value, r.value

    def autotune(self, reps: int = 5):
        """Pick the fastest tile on the device; returns (block_x, rows, us/step)."""
        bx, rows, us = C.c_int32(), C.c_int32(), C.c_float()
        self._check(self.lib.lbm_autotune(self.h, int(reps), C.byref(bx), C.byref(rows), C.byref(us)))
        return bx.value, rows.value, us.value

    def init_device(self, rho, ux=None, uy=None):
        """Re-initialise from device float32 tensors [ny][nx] (warm start)."""
        ptr = lambda t: None if t is None else C.c_void_p(t.contiguous().data_ptr())
        self._keep = (rho, ux, uy)
        self._check(self.lib.lbm_init_device(self.h, ptr(rho), ptr(ux), ptr(uy)))

    def save_state(self) -> bytes:
        n = int(self.lib.lbm_state_bytes(self.h))
        buf = C.create_string_buffer(n)
        self._check(self.lib.lbm_save_state(self.h, buf, n))
        return buf.raw

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(self.lib.lbm_load_state(self.h, buf, len(data)))

    @property
    def steps_done(self) -> int:
        return int(self.lib.lbm_steps_done(self.h))

    def synchronize(self):
        self.stream.synchronize()


def from_case(case, **kw) -> Simulation:
    """Simulation from an ``inputs.Case``."""
    return Simulation(case.params, case.solid, case.rho, case.ux, case.uy, **kw)


class Batch:
    """Many channels of uneven sizes on one GPU (lbm_batch_* of the C ABI)."""

    def __init__(self, cases, stream=None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP GPU; torch.cuda.is_available() is False")
        lib = load_library()
        self.torch = torch
        self.lib = lib
        self.n = len(cases)
        self.shapes = [(int(c.params.ny), int(c.params.nx)) for c in cases]
        self.params = [c.params for c in cases]
        self.device = torch.device("cuda" if device is None else device)
        cps = (lbm_params * self.n)(*[to_c_params(c.params) for c in cases])
        nbytes = int(lib.lbm_batch_workspace_bytes(self.n, cps))
        if nbytes == 0:
            raise LBMError(-1, "invalid batch parameters (lbm_batch_workspace_bytes returned 0)")
        keep = []

        def ptrs(arrs, dtype):
            out = (C.c_void_p * self.n)()
            for i, a in enumerate(arrs):
                if a is None:
                    out[i] = None
                else:
                    a = np.ascontiguousarray(a, dtype)
                    keep.append(a)
                    out[i] = a.ctypes.data
            return out

        solid = ptrs([c.solid for c in cases], np.uint8)
        rho = ptrs([c.rho for c in cases], np.float64)
        ux = ptrs([c.ux for c in cases], np.float64)
        uy = ptrs([c.uy for c in cases], np.float64)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream() if stream is None else stream
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            st = lib.lbm_batch_init(C.byref(h), self.n, cps, solid, rho, ux, uy,
                                    C.c_void_p(self.ws.data_ptr()), nbytes,
                                    C.c_void_p(self.stream.cuda_stream))
            if st != 0:
                raise LBMError(st, lib.lbm_batch_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != 0:
            msg = self.lib.lbm_batch_last_error(self.h).decode()
            raise (Diverged if st == -4 else LBMError)(st, msg)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.lbm_batch_free(h)
            self.h = None

    close = __del__

    def step(self, n: int = 1):
        self._check(self.lib.lbm_batch_step(self.h, int(n)))

    def profile(self, i: int):
        """Channel-averaged u_x per row of channel i (float64 [ny_i])."""
        out = np.zeros(self.shapes[i][0])
        self._check(self.lib.lbm_batch_profile(self.h, int(i), out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def flux(self):
        """(Q [n], M [n]) float64 numpy arrays; raises Diverged if any channel diverged."""
        Q = np.zeros(self.n)
        M = np.zeros(self.n)
        self._check(self.lib.lbm_batch_flux(self.h, Q.ctypes.data_as(C.POINTER(C.c_double)),
                                            M.ctypes.data_as(C.POINTER(C.c_double))))
        return Q, M

    def flux_nocheck(self):
        """(Q, M, status): like flux() but returns the status instead of raising."""
        Q = np.zeros(self.n)
        M = np.zeros(self.n)
        st = self.lib.lbm_batch_flux(self.h, Q.ctypes.data_as(C.POINTER(C.c_double)),
                                     M.ctypes.data_as(C.POINTER(C.c_double)))
        return Q, M, st

    def moments(self, i: int):
        ny, nx = self.shapes[i]
        out = [np.empty((ny, nx), np.float32) for _ in range(3)]
        self._check(self.lib.lbm_batch_moments(self.h, int(i), *[C.c_void_p(o.ctypes.data) for o in out], 0))
        return tuple(out)

    def moments_device(self, i: int):
        ny, nx = self.shapes[i]
        t = self.torch.empty((3, ny, nx), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.lbm_batch_moments(self.h, int(i), C.c_void_p(t[0].data_ptr()),
                                               C.c_void_p(t[1].data_ptr()), C.c_void_p(t[2].data_ptr()), 1))
        return t

    def geometry(self, i: int) -> np.ndarray:
        ny, nx = self.shapes[i]
        out = np.empty((ny, nx), np.uint16)
        self._check(self.lib.lbm_batch_geometry(self.h, int(i), out.ctypes.data_as(C.POINTER(C.c_uint16))))
        return out

    def init_device(self, i: int, rho, ux=None, uy=None):
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        tensors = [None if t is None else t.contiguous() for t in (rho, ux, uy)]
        self._keep = tensors
        self._check(self.lib.lbm_batch_init_device(self.h, int(i), *[ptr(t) for t in tensors]))

    def set_forces(self, i: int, f_elec: float, accel_x: float = 0.0, accel_y: float = 0.0):
        self._check(self.lib.lbm_batch_set_forces(self.h, int(i), float(f_elec), float(accel_x),
                                                  float(accel_y)))

    def retire(self, done):
        d = np.ascontiguousarray(np.asarray(done, np.uint8))
        assert d.shape == (self.n,)
        self._check(self.lib.lbm_batch_retire(self.h, d.ctypes.data_as(C.POINTER(C.c_uint8))))

    def set_tile(self, block_x: int, rows: int):
        self._check(self.lib.lbm_batch_set_tile(self.h, int(block_x), int(rows)))

    def set_schedule(self, persistent: bool):
        self._check(self.lib.lbm_batch_set_schedule(self.h, int(bool(persistent))))

    def set_kernel(self, kernel: str):
        """Steps per launch: "fused" (one), "two" or "three"."""
        if kernel not in ("fused", "two", "three"):
            raise ValueError(f"batch kernel must be fused, two or three, not {kernel!r}")
        self._check(self.lib.lbm_batch_set_kernel(self.h, KERNELS[kernel]))

    def kernel(self) -> str:
        return {v: n for n, v in KERNELS.items()}[int(self.lib.lbm_batch_get_kernel(self.h))]

    def set_graph(self, steps_per_graph: int):
        self._check(self.lib.lbm_batch_set_graph(self.h, int(steps_per_graph)))

    def autotune(self, reps: int = 3):
        bx, rows, us = C.c_int32(), C.c_int32(), C.c_float()
        self._check(self.lib.lbm_batch_autotune(self.h, int(reps), C.byref(bx), C.byref(rows), C.byref(us)))
        return bx.value, rows.value, us.value

    def steps_done(self, i: int) -> int:
        return int(self.lib.lbm_batch_steps_done(self.h, int(i)))

    def synchronize(self):
        self.stream.synchronize()

