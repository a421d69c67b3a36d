"""ctypes binding of the warm-start network (include/lbm_net.h).

Argument marshalling only: the forward pass, the gradients and the Adam update
run in the HIP kernels of ``liblbm.so``.  PyTorch provides the device
workspace and the stream; tensors handed to the calls are device tensors.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lbm

SYMBOLS = ("lbm_net_param_count", "lbm_net_workspace_bytes", "lbm_net_create", "lbm_net_set_params",
           "lbm_net_get_params", "lbm_net_forward", "lbm_net_gradient", "lbm_net_adam",
           "lbm_net_train_step", "lbm_net_free", "lbm_net_last_error")


class lbm_net_config(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("batch", C.c_int32), ("cin", C.c_int32),
                ("cout", C.c_int32), ("chans", C.c_int32 * 4), ("act_bf16", C.c_int32)]


def make_config(H, W, batch, cin=3, cout=3, chans=(32, 64, 128, 128), act_bf16=True) -> lbm_net_config:
    c = lbm_net_config()
    c.H, c.W, c.batch, c.cin, c.cout = int(H), int(W), int(batch), int(cin), int(cout)
    for i in range(4):
        c.chans[i] = int(chans[i])
    c.act_bf16 = 1 if act_bf16 else 0
    return c


def layer_shapes(cin=3, cout=3, chans=(32, 64, 128, 128)):
    """(name, cin, cout, k) of the 15 layers in parameter order (lbm_net.h)."""
    c1, c2, c3, c4 = chans
    return [("e1a", cin, c1, 3), ("e1b", c1, c1, 3), ("e2a", c1, c2, 3), ("e2b", c2, c2, 3),
            ("e3a", c2, c3, 3), ("e3b", c3, c3, 3), ("b_a", c3, c4, 3), ("b_b", c4, c4, 3),
            ("d3a", c4 + c3, c3, 3), ("d3b", c3, c3, 3), ("d2a", c3 + c2, c2, 3), ("d2b", c2, c2, 3),
            ("d1a", c2 + c1, c1, 3), ("d1b", c1, c1, 3), ("out", c1, cout, 1)]


def he_init(shapes, seed=0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; FP32 vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, k in shapes:
        parts.append(rng.standard_normal(co * ci * k * k) * np.sqrt(2.0 / (ci * k * k)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


_typed = False


def load_library():
    global _typed
    lib = lbm.load_library()
    if not _typed:
        vp, cfgp = C.c_void_p, C.POINTER(lbm_net_config)
        fp = C.POINTER(C.c_float)
        lib.lbm_net_param_count.argtypes = [cfgp]
        lib.lbm_net_param_count.restype = C.c_int64
        lib.lbm_net_workspace_bytes.argtypes = [cfgp]
        lib.lbm_net_workspace_bytes.restype = C.c_size_t
        lib.lbm_net_create.argtypes = [C.POINTER(vp), cfgp, vp, C.c_size_t, vp]
        lib.lbm_net_set_params.argtypes = [vp, fp, C.c_int64]
        lib.lbm_net_get_params.argtypes = [vp, fp, C.c_int64]
        lib.lbm_net_forward.argtypes = [vp, vp, vp, C.c_int32]
        lib.lbm_net_gradient.argtypes = [vp, vp, vp, vp, C.c_int32, C.POINTER(C.c_double), fp]
        lib.lbm_net_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
        lib.lbm_net_train_step.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.POINTER(C.c_double)]
        lib.lbm_net_free.argtypes = [vp]
        lib.lbm_net_free.restype = None
        lib.lbm_net_last_error.argtypes = [vp]
        lib.lbm_net_last_error.restype = C.c_char_p
        for n in ("lbm_net_create", "lbm_net_set_params", "lbm_net_get_params", "lbm_net_forward",
                  "lbm_net_gradient", "lbm_net_adam", "lbm_net_train_step"):
            getattr(lib, n).restype = C.c_int
        _typed = True
    return lib


def param_count(**cfg) -> int:
    return int(load_library().lbm_net_param_count(C.byref(make_config(**cfg))))


def workspace_bytes(**cfg) -> int:
    return int(load_library().lbm_net_workspace_bytes(C.byref(make_config(**cfg))))


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _dev(t):
    return C.c_void_p(t.data_ptr())


class Net:
    """The encoder-decoder on one GPU: a torch workspace and a liblbm handle."""

    def __init__(self, H, W, batch, cin=3, cout=3, chans=(32, 64, 128, 128), act_bf16=True, stream=None,
                 device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP GPU; torch.cuda.is_available() is False")
        lib = load_library()
        self.torch, self.lib = torch, lib
        self.H, self.W, self.batch, self.cin, self.cout = H, W, batch, cin, cout
        self.chans = tuple(chans)
        self.cfg = make_config(H, W, batch, cin, cout, chans, act_bf16)
        self.n_params = int(lib.lbm_net_param_count(C.byref(self.cfg)))
        nbytes = int(lib.lbm_net_workspace_bytes(C.byref(self.cfg)))
        if nbytes == 0 or self.n_params < 0:
            raise lbm.LBMError(-1, "invalid network configuration")
        self.device = torch.device("cuda" if device is None else device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream() if stream is None else stream
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            st = lib.lbm_net_create(C.byref(h), C.byref(self.cfg), _dev(self.ws), nbytes,
                                    C.c_void_p(self.stream.cuda_stream))
            if st != 0:
                raise lbm.LBMError(st, lib.lbm_net_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != 0:
            raise lbm.LBMError(st, self.lib.lbm_net_last_error(self.h).decode())

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.lbm_net_free(h)
            self.h = None

    close = __del__

    def _inputs(self, x, t=None, fluid=None):
        """Check device, layout, dtype and shape: the kernels read n x (planes x
        H x W) elements behind each pointer."""
        torch = self.torch
        n = x.shape[0] if x.dim() == 4 else -1
        want = [(x, torch.float32, (n, self.cin, self.H, self.W))]
        if t is not None:
            want.append((t, torch.float32, (n, self.cout, self.H, self.W)))
            want.append((fluid, torch.uint8, (n, self.H, self.W)))
        for a, dt, shape in want:
            if a is None or a.device.type != "cuda" or not a.is_contiguous():
                raise ValueError("network tensors must be contiguous device tensors")
            if a.dtype != dt or tuple(a.shape) != shape:
                raise ValueError(f"expected {dt} of shape {shape}, got {a.dtype} {tuple(a.shape)}")
        if not 1 <= n <= self.batch:
            raise ValueError(f"batch of {n} samples; this network takes 1..{self.batch}")
        return [a for a, _, _ in want]

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
        self._check(self.lib.lbm_net_set_params(self.h, _fptr(a), a.size))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, np.float32)
        self._check(self.lib.lbm_net_get_params(self.h, _fptr(a), a.size))
        return a

    def forward(self, x):
        """x: float32 device tensor [n][cin][H][W] -> y [n][cout][H][W] (asynchronous)."""
        (x,) = self._inputs(x)
        n = x.shape[0]
        y = self.torch.empty((n, self.cout, self.H, self.W), dtype=self.torch.float32, device=x.device)
        self._check(self.lib.lbm_net_forward(self.h, _dev(x), _dev(y), n))
        return y

    def gradient(self, x, t, fluid):
        """(loss, gradient as a host float32 vector)."""
        x, t, fluid = self._inputs(x, t, fluid)
        g = np.empty(self.n_params, np.float32)
        loss = C.c_double()
        self._check(self.lib.lbm_net_gradient(self.h, _dev(x), _dev(t), _dev(fluid), x.shape[0],
                                              C.byref(loss), _fptr(g)))
        return loss.value, g

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self._check(self.lib.lbm_net_adam(self.h, lr, b1, b2, eps))

    def train_step(self, x, t, fluid, lr=1e-3, want_loss=True):
        x, t, fluid = self._inputs(x, t, fluid)
        loss = C.c_double()
        self._check(self.lib.lbm_net_train_step(self.h, _dev(x), _dev(t), _dev(fluid), x.shape[0], lr,
                                                C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
