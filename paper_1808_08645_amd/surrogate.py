"""Binding of the trace surrogate (include/bbwadg_surrogate.h): argument marshalling only."""
import ctypes as C

import numpy as np

from .bbwadg import _check, load_library


class Surrogate:
    """c^2 on a 16^3 grid -> receiver traces; BF16 matrix-core GEMMs with FP32 accumulation."""

    def __init__(self, nout: int, max_batch: int = 32, seed: int = 0, grid: int = 16):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate needs a HIP device")
        torch.cuda.current_device()
        self._lib = load_library()
        self._h = C.c_void_p()
        _check(self._lib.bbwadg_sur_create(grid, nout, max_batch, C.c_uint64(seed), C.byref(self._h)))
        self.nout, self.max_batch, self.grid = nout, max_batch, grid
        self.num_params = int(self._lib.bbwadg_sur_num_params(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.bbwadg_sur_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream():
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _dev(self, a, shape):
        import torch
        t = torch.as_tensor(a, dtype=torch.float32, device="cuda").contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def layout(self):
        out = []
        for l in range(7):
            info = (C.c_int32 * 8)()
            _check(self._lib.bbwadg_sur_layout(self._h, l, info))
            k = list(info)
            out.append({"conv": bool(k[0]), "cin": k[1], "cout": k[2], "K": k[3], "Kp": k[4], "relu": bool(k[5]),
                        "woff": k[6], "boff": k[7]})
        return out

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _check(self._lib.bbwadg_sur_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.shape != (self.num_params,):
            raise ValueError("wrong parameter count")
        _check(self._lib.bbwadg_sur_set_params(self._h, p.ctypes.data_as(C.c_void_p)))

    def forward(self, x):
        import torch
        B = int(x.shape[0])
        x = self._dev(x, (B, self.grid, self.grid, self.grid))
        y = torch.empty((B, self.nout), dtype=torch.float32, device="cuda")
        _check(self._lib.bbwadg_sur_forward(self._h, C.c_void_p(x.data_ptr()), B, C.c_void_p(y.data_ptr()),
                                            self._stream()))
        return y

    def loss_grad(self, x, t, want_grad: bool = True):
        B = int(x.shape[0])
        x = self._dev(x, (B, self.grid, self.grid, self.grid))
        t = self._dev(t, (B, self.nout))
        loss = C.c_double()
        g = np.empty(self.num_params, dtype=np.float32) if want_grad else None
        _check(self._lib.bbwadg_sur_loss_grad(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), B,
                                              C.byref(loss), g.ctypes.data_as(C.c_void_p) if want_grad else None,
                                              self._stream()))
        return loss.value, g

    def input_grad(self, x, t):
        """(loss, dL/dx) of L = mean((f(x) - t)^2); dL/dx a device tensor shaped like x."""
        import torch
        B = int(x.shape[0])
        x = self._dev(x, (B, self.grid, self.grid, self.grid))
        t = self._dev(t, (B, self.nout))
        loss = C.c_double()
        dx = torch.empty_like(x)
        _check(self._lib.bbwadg_sur_input_grad(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), B,
                                               C.byref(loss), C.c_void_p(dx.data_ptr()), self._stream()))
        return loss.value, dx

    def train_step(self, x, t, lr: float) -> float:
        B = int(x.shape[0])
        x = self._dev(x, (B, self.grid, self.grid, self.grid))
        t = self._dev(t, (B, self.nout))
        loss = C.c_double()
        _check(self._lib.bbwadg_sur_train_step(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), B,
                                               C.c_float(lr), C.byref(loss), self._stream()))
        return loss.value
