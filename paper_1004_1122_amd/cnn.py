"""Python binding of include/lshom_cnn.h (the warm-start network).

Argument marshalling only: parameters, activations and the optimiser state
live in torch-owned device buffers handed to the library; every step runs in
the HIP kernels of liblshom.so.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int64, c_size_t, c_void_p

import numpy as np

from . import lshom as _ls

_sig_done = False


def _lib():
    global _sig_done
    lib = _ls.load()
    if not _sig_done:
        P = c_void_p
        sig = {
            "lshom_cnn_create": (c_int, [POINTER(c_void_p), c_int, P, c_int]),
            "lshom_cnn_destroy": (None, [P]),
            "lshom_cnn_last_error": (c_char_p, [P]),
            "lshom_cnn_param_size": (c_int, [P, POINTER(c_int64), POINTER(c_size_t)]),
            "lshom_cnn_set_param_buffer": (c_int, [P, P, c_size_t]),
            "lshom_cnn_set_params": (c_int, [P, POINTER(c_float), c_int64]),
            "lshom_cnn_get_params": (c_int, [P, POINTER(c_float), c_int64]),
            "lshom_cnn_get_grads": (c_int, [P, POINTER(c_float), c_int64]),
            "lshom_cnn_workspace_size": (c_int, [P, c_int, c_int, c_int, POINTER(c_size_t)]),
            "lshom_cnn_set_workspace": (c_int, [P, P, c_size_t, c_int, c_int, c_int]),
            "lshom_cnn_forward": (c_int, [P, P, P, c_int, c_int, c_int, c_int, P, P]),
            "lshom_cnn_train_step": (c_int, [P, P, P, P, c_int, c_int, c_float, c_int, POINTER(c_double)]),
            "lshom_cnn_layer_forward": (c_int, [P, c_int, P, P, P]),
            "lshom_cnn_layer_dgrad": (c_int, [P, c_int, P, P]),
            "lshom_cnn_layer_wgrad": (c_int, [P, c_int, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _sig_done = True
    return lib


class CnnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} ({status})")
        self.status = status


def layer_shapes(c0: int = 32):
    """(name, weight shape, bias length) in the compact parameter order."""
    c = [c0, 2 * c0, 4 * c0, 8 * c0]
    s = [("enc0a", (3, 3, 2, c[0])), ("enc0b", (3, 3, c[0], c[0])), ("down0", (3, 3, c[0], c[1])),
         ("enc1a", (3, 3, c[1], c[1])), ("enc1b", (3, 3, c[1], c[1])), ("down1", (3, 3, c[1], c[2])),
         ("enc2a", (3, 3, c[2], c[2])), ("enc2b", (3, 3, c[2], c[2])), ("down2", (3, 3, c[2], c[3])),
         ("bot_a", (3, 3, c[3], c[3])), ("bot_b", (3, 3, c[3], c[3]))]
    for lev in (2, 1, 0):
        s += [(f"up{lev}", (3, 3, c[lev + 1], c[lev])), (f"dec{lev}a", (3, 3, 2 * c[lev], c[lev])),
              (f"dec{lev}b", (3, 3, c[lev], c[lev]))]
    s.append(("head", (c[0], 2)))
    return [(n, shp, shp[-1]) for n, shp in s]


_LEVEL_OUT = (0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0, 0)


def layer_geometry(index: int, n: int, c0: int = 32):
    """Grids and channels of layer `index` (execution order) of a layer call
    on n x n images: (name, hi, ho, cin, cout) with cin the channels the
    kernel reads (8 for the input layer)."""
    name, shp, cout = layer_shapes(c0)[index]
    ho = n // 3 ** _LEVEL_OUT[index]
    hi = 3 * ho if name.startswith("down") else (ho // 3 if name.startswith("up") else ho)
    cin = 8 if index == 0 else shp[-2]
    return name, hi, ho, cin, cout


def he_init(c0: int = 32, seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the compact order (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, shp, nb in layer_shapes(c0):
        fan_in = int(np.prod(shp[:-1]))
        gain = 1.0 if len(shp) == 2 else 2.0
        parts.append((rng.standard_normal(shp) * np.sqrt(gain / fan_in)).ravel())
        parts.append(np.zeros(nb))
    return np.concatenate(parts).astype(np.float32)


def pack(params: dict, c0: int = 32) -> np.ndarray:
    """{name: [w, b]} (the oracle's layout) -> compact float32 vector."""
    parts = []
    for name, shp, nb in layer_shapes(c0):
        w, b = params[name]
        assert tuple(w.shape) == shp and len(b) == nb, name
        parts += [np.asarray(w, np.float64).ravel(), np.asarray(b, np.float64)]
    return np.concatenate(parts).astype(np.float32)


def unpack(vec: np.ndarray, c0: int = 32) -> dict:
    out, k = {}, 0
    for name, shp, nb in layer_shapes(c0):
        n = int(np.prod(shp))
        out[name] = [np.asarray(vec[k:k + n], np.float64).reshape(shp), np.asarray(vec[k + n:k + n + nb], np.float64)]
        k += n + nb
    return out


class WarmStartNet:
    """The U-Net of include/lshom_cnn.h on one device."""

    def __init__(self, base_channels: int = 32, device: int = 0, params=None, seed: int = 0):
        import torch
        self.torch = torch
        self.lib = _lib()
        if not torch.cuda.is_available():
            raise RuntimeError("WarmStartNet needs a GPU")
        self.c0 = base_channels
        self.device = torch.device("cuda", device)
        h = c_void_p()
        st = self.lib.lshom_cnn_create(ctypes.byref(h), device, c_void_p(torch.cuda.current_stream(self.device).cuda_stream),
                                       base_channels)
        if st != 0:
            raise CnnError(st, "lshom_cnn_create failed")
        self.h = h
        n = c_int64()
        nb = c_size_t()
        self._check(self.lib.lshom_cnn_param_size(self.h, ctypes.byref(n), ctypes.byref(nb)))
        self.n_params = int(n.value)
        self._pbuf = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        self._check(self.lib.lshom_cnn_set_param_buffer(self.h, self._aligned(self._pbuf), int(nb.value)))
        self._ws_cache = {}
        self._ws_key = None
        self.set_params(he_init(base_channels, seed) if params is None else params)

    @staticmethod
    def _aligned(t):
        return c_void_p(t.data_ptr() + ((-t.data_ptr()) % 256))

    def _check(self, st):
        if st != 0:
            msg = self.lib.lshom_cnn_last_error(self.h)
            raise CnnError(st, msg.decode() if msg else "lshom_cnn error")

    def close(self):
        if getattr(self, "h", None):
            self.lib.lshom_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # parameters ---------------------------------------------------------
    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        self._check(self.lib.lshom_cnn_set_params(self.h, v.ctypes.data_as(POINTER(c_float)), v.size))

    def get_params(self) -> np.ndarray:
        v = np.empty(self.n_params, np.float32)
        self._check(self.lib.lshom_cnn_get_params(self.h, v.ctypes.data_as(POINTER(c_float)), v.size))
        return v

    def get_grads(self) -> np.ndarray:
        v = np.empty(self.n_params, np.float32)
        self._check(self.lib.lshom_cnn_get_grads(self.h, v.ctypes.data_as(POINTER(c_float)), v.size))
        return v

    def save(self, path):
        np.savez(path, params=self.get_params(), base_channels=self.c0)

    @classmethod
    def load(cls, path, device: int = 0):
        with np.load(path, allow_pickle=False) as f:
            return cls(int(f["base_channels"]), device, params=f["params"])

    # workspace ----------------------------------------------------------
    def _ensure_ws(self, B, N, training):
        """Workspaces are kept per (batch, N, training) shape; switching
        between shapes only re-points the library."""
        key = (B, N, bool(training))
        if self._ws_key == key:
            return
        if not training and (B, N, True) in self._ws_cache:
            key = (B, N, True)  # a training workspace serves inference too
        if key not in self._ws_cache:
            sz = c_size_t()
            self._check(self.lib.lshom_cnn_workspace_size(self.h, B, N, int(key[2]), ctypes.byref(sz)))
            self._ws_cache[key] = (self.torch.empty(int(sz.value) + 256, dtype=self.torch.uint8, device=self.device),
                                   int(sz.value))
        buf, size = self._ws_cache[key]
        self._check(self.lib.lshom_cnn_set_workspace(self.h, self._aligned(buf), size, B, N, int(key[2])))
        self._ws_key = key

    def drop_workspaces(self):
        self._ws_cache.clear()
        self._ws_key = None

    def _inputs(self, phase, log10_rho):
        torch = self.torch
        ph = phase if isinstance(phase, torch.Tensor) else torch.as_tensor(np.ascontiguousarray(phase, np.uint8))
        ph = ph.to(device=self.device, dtype=torch.uint8).contiguous()
        if ph.dim() == 2:
            ph = ph[None]
        lr = torch.as_tensor(np.atleast_1d(np.asarray(log10_rho, np.float32)) if not isinstance(log10_rho, torch.Tensor)
                             else log10_rho).to(device=self.device, dtype=torch.float32).contiguous()
        if lr.numel() == 1 and ph.shape[0] > 1:
            lr = lr.expand(ph.shape[0]).contiguous()
        return ph, lr

    def forward(self, phase, log10_rho, load_axis: int = 0, want_raw: bool = False, scale: int = 1):
        """Predicted fields [B, 2, N, N] (float64, E + prediction) and
        optionally the raw output [B, N/scale, N/scale, 2] (float32)."""
        torch = self.torch
        ph, lr = self._inputs(phase, log10_rho)
        B, N = ph.shape[0], ph.shape[1]
        nc = N // scale
        self._ensure_ws(B, nc, False)
        e = torch.empty((B, 2, N, N), dtype=torch.float64, device=self.device)
        raw = torch.empty((B, nc, nc, 2), dtype=torch.float32, device=self.device) if want_raw else None
        self._check(self.lib.lshom_cnn_forward(self.h, c_void_p(ph.data_ptr()), c_void_p(lr.data_ptr()), B, N,
                                               int(load_axis), int(scale), c_void_p(e.data_ptr()),
                                               c_void_p(raw.data_ptr()) if raw is not None else None))
        return (e, raw) if want_raw else e

    def train_step(self, phase, log10_rho, e_target, lr: float = 1e-3, update: bool = True) -> float:
        """One step on a batch; e_target: FP64 [B, 2, N, N] solutions for E = e1."""
        torch = self.torch
        ph, lrho = self._inputs(phase, log10_rho)
        B, N = ph.shape[0], ph.shape[1]
        self._ensure_ws(B, N, True)
        e = e_target.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(e.shape) != (B, 2, N, N):
            raise ValueError(f"e_target must have shape {(B, 2, N, N)}, got {tuple(e.shape)}")
        loss = c_double()
        self._check(self.lib.lshom_cnn_train_step(self.h, c_void_p(ph.data_ptr()), c_void_p(lrho.data_ptr()),
                                                  c_void_p(e.data_ptr()), B, N, float(lr), int(bool(update)),
                                                  ctypes.byref(loss)))
        return float(loss.value)


    # layer calls -------------------------------------------------------
    def _layer_ws(self, B, N, training):
        self._ensure_ws(B, N, training)

    def layer_forward(self, index, x, n):
        """Layer `index` on x (bfloat16 [B, hi, hi, cin]) of n x n images:
        (y bfloat16, y float32), both [B, ho, ho, cout]."""
        torch = self.torch
        _, hi, ho, cin, cout = layer_geometry(index, n, self.c0)
        x = x.to(device=self.device, dtype=torch.bfloat16).contiguous()
        if tuple(x.shape[1:]) != (hi, hi, cin):
            raise ValueError(f"layer {index}: x must be [B, {hi}, {hi}, {cin}], got {tuple(x.shape)}")
        B = x.shape[0]
        self._layer_ws(B, n, False)
        y = torch.empty((B, ho, ho, cout), dtype=torch.bfloat16, device=self.device)
        yf = torch.empty((B, ho, ho, cout), dtype=torch.float32, device=self.device)
        self._check(self.lib.lshom_cnn_layer_forward(self.h, int(index), c_void_p(x.data_ptr()),
                                                     c_void_p(y.data_ptr()), c_void_p(yf.data_ptr())))
        return y, yf

    def layer_dgrad(self, index, gy, n):
        """Input gradient (float32 [B, hi, hi, cin]) of layer `index` for the
        pre-activation gradient gy (bfloat16 [B, ho, ho, cout8])."""
        torch = self.torch
        _, hi, ho, cin, cout = layer_geometry(index, n, self.c0)
        gy = gy.to(device=self.device, dtype=torch.bfloat16).contiguous()
        if tuple(gy.shape[1:]) != (ho, ho, (cout + 7) // 8 * 8):
            raise ValueError(f"layer {index}: gy must be [B, {ho}, {ho}, {(cout + 7) // 8 * 8}]")
        B = gy.shape[0]
        self._layer_ws(B, n, True)
        gx = torch.empty((B, hi, hi, cin), dtype=torch.float32, device=self.device)
        self._check(self.lib.lshom_cnn_layer_dgrad(self.h, int(index), c_void_p(gy.data_ptr()), c_void_p(gx.data_ptr())))
        return gx

    def layer_wgrad(self, index, x, gy, n):
        """Weight and bias gradients of layer `index` (sums over the batch's
        pixels) for input x and pre-activation gradient gy; returns the
        compact gradient vector (the other layers' entries as they were)."""
        torch = self.torch
        _, hi, ho, cin, cout = layer_geometry(index, n, self.c0)
        x = x.to(device=self.device, dtype=torch.bfloat16).contiguous()
        gy = gy.to(device=self.device, dtype=torch.bfloat16).contiguous()
        if tuple(x.shape[1:]) != (hi, hi, cin) or tuple(gy.shape[1:]) != (ho, ho, (cout + 7) // 8 * 8) \
                or x.shape[0] != gy.shape[0]:
            raise ValueError(f"layer {index}: x [B, {hi}, {hi}, {cin}] and gy [B, {ho}, {ho}, cout8] required")
        self._layer_ws(x.shape[0], n, True)
        self._check(self.lib.lshom_cnn_layer_wgrad(self.h, int(index), c_void_p(x.data_ptr()), c_void_p(gy.data_ptr())))
        return self.get_grads()


DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_unet32.npz")
