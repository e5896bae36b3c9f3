"""ctypes binding of liblshom.so: the C ABI of include/lshom.h, same names.

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides the device memory (phase image, workspace, fields) and the
stream.  ``load()`` fails loudly when the library has not been built; there is
no fallback.

High-level use::

    s = Solver(phase_gpu_uint8, cond=[1.0, 10.0])
    e, leff, info = s.solve([1.0, 0.0], tol=1e-8)
"""

from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, Structure, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblshom.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "lshom.h")

LSHOM_OK = 0
LSHOM_ERR_INVALID_ARG = -1
LSHOM_ERR_STATE = -2
LSHOM_ERR_WORKSPACE = -3
LSHOM_ERR_HIP = -4
LSHOM_ERR_NOT_CONVERGED = -5
LSHOM_ERR_BREAKDOWN = -6
LSHOM_ERR_UNSUPPORTED = -7

LSHOM_STATIC_WORKSPACE_BYTES = 64 << 20

PRECISION_FP64 = 0
PRECISION_MIXED = 1

METHOD_CG = 0
METHOD_FFTH = 1
METHOD_BICG = 2
METHOD_PIPECG = 3

NORM_RESIDUAL = 0
NORM_EQUILIBRIUM = 1


class lshom_solve_opts(Structure):
    _fields_ = [
        ("max_iter", c_int32),
        ("precision", c_int32),
        ("refresh_every", c_int32),
        ("refresh_drop", c_double),
        ("graph_block", c_int32),
        ("true_residual", c_int32),
        ("method", c_int32),
        ("norm", c_int32),
        ("history_dev", c_void_p),
        ("history_len", c_int32),
    ]


class lshom_solve_info(Structure):
    _fields_ = [
        ("iterations", c_int32),
        ("applies_fp32", c_int32),
        ("applies_fp64", c_int32),
        ("status", c_int32),
        ("warm_start_used", c_int32),
        ("refreshes", c_int32),
        ("rel_res", c_double),
        ("rel_res_true", c_double),
        ("eta_r", c_double),
        ("eta_e", c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class lshom_problem(Structure):
    _fields_ = [
        ("d", c_int32),
        ("N", c_int64 * 3),
        ("phase_dev", c_void_p),
        ("n_phases", c_int32),
        ("cond_host", POINTER(c_double)),
        ("l0", c_double),
        ("E", c_double * 3),
        ("tol", c_double),
        ("e_dev", c_void_p),
        ("cell", c_double * 3),
        ("x0_dev", c_void_p),
    ]


class lshom_schedule(Structure):
    _fields_ = [
        ("d", c_int32),
        ("N", c_int64 * 3),
        ("precision", c_int32),
        ("rows_per_block", c_int32),
        ("tile0", c_int32),
        ("tile1", c_int32),
        ("row_split", c_int32),
        ("threads_row", c_int32),
        ("threads_col", c_int32),
        ("nstages", c_int32 * 3),
        ("radix", (c_int32 * 16) * 3),
        ("ms_per_iter", c_double),
        ("tail_rows", c_int32),
    ]

    def as_dict(self):
        d = int(self.d)
        return {
            "d": d,
            "N": [int(self.N[a]) for a in range(d)],
            "precision": int(self.precision),
            "rows_per_block": int(self.rows_per_block),
            "tile0": int(self.tile0),
            "tile1": int(self.tile1),
            "row_split": int(self.row_split),
            "threads_row": int(self.threads_row),
            "threads_col": int(self.threads_col),
            "radix": [[int(self.radix[a][k]) for k in range(self.nstages[a])] for a in range(d)],
            "ms_per_iter": float(self.ms_per_iter),
            "tail_rows": int(self.tail_rows),
        }

    @classmethod
    def from_dict(cls, s):
        out = cls()
        out.d = int(s["d"])
        for a in range(3):
            out.N[a] = int(s["N"][a]) if a < out.d else 1
        out.precision = int(s["precision"])
        out.rows_per_block = int(s["rows_per_block"])
        out.tile0 = int(s["tile0"])
        out.tile1 = int(s.get("tile1", 1))
        out.row_split = int(s.get("row_split", 0))
        out.threads_row = int(s.get("threads_row", 0))
        out.threads_col = int(s.get("threads_col", 0))
        for a, rad in enumerate(s["radix"]):
            out.nstages[a] = len(rad)
            for k, r in enumerate(rad):
                out.radix[a][k] = int(r)
        out.ms_per_iter = float(s.get("ms_per_iter", 0.0))
        out.tail_rows = int(s.get("tail_rows", 0))
        return out


_lib = None


def load(path: str = LIB_PATH):
    """Load liblshom.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1004_1122_amd.build`"
                           " (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "lshom_status_string": (c_char_p, [c_int32]),
        "lshom_last_error": (c_char_p, [P]),
        "lshom_default_opts": (None, [POINTER(lshom_solve_opts)]),
        "lshom_check_problem": (c_int32, [c_int, POINTER(c_int64), c_int, POINTER(c_double), c_double,
                                          POINTER(c_double), c_double]),
        "lshom_create": (c_int32, [POINTER(c_void_p), c_int, P]),
        "lshom_destroy": (None, [P]),
        "lshom_set_microstructure": (c_int32, [P, c_int, POINTER(c_int64), P, c_int, POINTER(c_double)]),
        "lshom_set_microstructure_tensor": (c_int32, [P, c_int, POINTER(c_int64), P, c_int, POINTER(c_double)]),
        "lshom_set_reference": (c_int32, [P, c_double]),
        "lshom_set_reference_tensor": (c_int32, [P, POINTER(c_double)]),
        "lshom_set_reference_mean": (c_int32, [P]),
        "lshom_set_cell": (c_int32, [P, POINTER(c_double)]),
        "lshom_workspace_size": (c_int32, [P, c_int, POINTER(c_size_t)]),
        "lshom_workspace_size_for": (c_int32, [P, POINTER(lshom_solve_opts), POINTER(c_size_t)]),
        "lshom_set_workspace": (c_int32, [P, P, c_size_t]),
        "lshom_solve": (c_int32, [P, POINTER(c_double), c_double, POINTER(lshom_solve_opts), P, P,
                                  POINTER(c_double), POINTER(lshom_solve_info)]),
        "lshom_solve_static": (c_int32, [P, POINTER(c_double), c_double, POINTER(lshom_solve_opts), P,
                                         POINTER(c_double), POINTER(lshom_solve_info)]),
        "lshom_homogenize": (c_int32, [P, c_double, POINTER(lshom_solve_opts), POINTER(c_double),
                                       POINTER(lshom_solve_info)]),
        "lshom_apply": (c_int32, [P, P, P]),
        "lshom_time_passes": (c_int32, [P, c_int, c_int, POINTER(c_double), POINTER(c_double)]),
        "lshom_batch_workspace_size": (c_int32, [P, c_int32, POINTER(lshom_problem), c_int, POINTER(c_size_t)]),
        "lshom_solve_batched": (c_int32, [P, c_int32, POINTER(lshom_problem), POINTER(lshom_solve_opts), P,
                                          c_size_t, POINTER(c_double), POINTER(lshom_solve_info)]),
        "lshom_get_schedule": (c_int32, [P, c_int, POINTER(lshom_schedule)]),
        "lshom_set_schedule": (c_int32, [P, POINTER(lshom_schedule)]),
        "lshom_autotune": (c_int32, [P, c_int, c_int, POINTER(lshom_schedule)]),
        "lshom_autotune_batched": (c_int32, [P, c_int32, POINTER(lshom_problem), c_int, c_int, P, c_size_t,
                                             POINTER(lshom_schedule), POINTER(c_int32)]),
        "lshom_set_pass_timing": (c_int32, [P, c_int]),
        "lshom_get_pass_timing": (c_int32, [P, POINTER(c_double), POINTER(c_double), POINTER(c_int64)]),
        "lshom_save_schedules": (c_int32, [P, c_char_p]),
        "lshom_load_schedules": (c_int32, [P, c_char_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_symbols(path: str = HEADER_PATH):
    """Names of the functions include/lshom.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lshom_[a-z0-9_]+)\s*\(", text)))


# ---------------------------------------------------------------------------
# Thin wrappers with the C names
# ---------------------------------------------------------------------------

def _dbl_array(vals):
    vals = [float(v) for v in vals]
    return (c_double * max(1, len(vals)))(*vals)


def lshom_status_string(status: int) -> str:
    return load().lshom_status_string(status).decode()


def lshom_default_opts() -> lshom_solve_opts:
    o = lshom_solve_opts()
    load().lshom_default_opts(ctypes.byref(o))
    return o


def lshom_check_problem(d, N, cond, l0=0.0, E=None, tol=-1.0) -> int:
    lib = load()
    Narr = (c_int64 * max(1, len(N)))(*[int(v) for v in N])
    carr = _dbl_array(cond)
    Earr = _dbl_array(E) if E is not None else None
    return lib.lshom_check_problem(int(d), Narr, len(cond), carr, float(l0), Earr, float(tol))


class LshomError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lshom_status_string(status)} ({status}): {msg}")
        self.status = status


def _check(ctx, status, allow=()):
    if status != LSHOM_OK and status not in allow:
        msg = load().lshom_last_error(ctx).decode() if ctx else ""
        raise LshomError(status, msg)
    return status


def lshom_create(device: int = 0, stream: int | None = None) -> c_void_p:
    lib = load()
    h = c_void_p()
    _check(None, lib.lshom_create(ctypes.byref(h), int(device), c_void_p(stream or 0)))
    return h


def lshom_destroy(ctx) -> None:
    if ctx:
        load().lshom_destroy(ctx)


# ---------------------------------------------------------------------------
# High-level solver object (torch owns device memory)
# ---------------------------------------------------------------------------

PASS_NAMES = ["axis0_inverse", "axis1_inverse", "row", "axis1_forward", "axis0_forward", "update"]


def lshom_set_pass_timing(ctx, enable: bool) -> None:
    _check(ctx, load().lshom_set_pass_timing(ctx, int(bool(enable))))


def lshom_get_pass_timing(ctx):
    """{pass: (device ms, algorithmic bytes, launches)} summed over timed solves."""
    ms = (c_double * 6)()
    by = (c_double * 6)()
    n = (c_int64 * 6)()
    _check(ctx, load().lshom_get_pass_timing(ctx, ms, by, n))
    return {name: (ms[i], by[i], int(n[i])) for i, name in enumerate(PASS_NAMES) if n[i] > 0}


class Solver:
    """One microstructure on one device; owns a context and its workspace."""

    def __init__(self, phase, cond, device: int = 0, precision: int = PRECISION_MIXED, cell=None):
        """cond: one conductivity per phase, or an array [n_phases, d, d] of
        symmetric tensors; cell: side lengths of the cell (default cubic)."""
        import torch
        self.torch = torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("lshom.Solver needs a GPU")
        dev = torch.device("cuda", device)
        if not isinstance(phase, torch.Tensor):
            phase = torch.as_tensor(np.ascontiguousarray(phase, dtype=np.uint8))
        self.phase = phase.to(device=dev, dtype=torch.uint8).contiguous()
        self.shape = tuple(self.phase.shape)
        self.d = len(self.shape)
        self.nvox = int(np.prod(self.shape))
        cond_arr = np.asarray(cond, dtype=np.float64)
        self.tensor = cond_arr.ndim == 3
        self.cond = cond_arr if self.tensor else [float(c) for c in cond]
        self.device = dev
        stream = torch.cuda.current_stream(dev).cuda_stream
        self.ctx = lshom_create(device, stream)
        Narr = (c_int64 * self.d)(*self.shape)
        if self.tensor:
            if cond_arr.shape[1:] != (self.d, self.d):
                raise ValueError(f"tensor phases must have shape [n_phases, {self.d}, {self.d}]")
            _check(self.ctx, self.lib.lshom_set_microstructure_tensor(
                self.ctx, self.d, Narr, c_void_p(self.phase.data_ptr()), cond_arr.shape[0],
                _dbl_array(cond_arr.ravel())))
        else:
            _check(self.ctx, self.lib.lshom_set_microstructure(self.ctx, self.d, Narr,
                                                               c_void_p(self.phase.data_ptr()),
                                                               len(self.cond), _dbl_array(self.cond)))
        if cell is not None:
            self.set_cell(cell)
        size = c_size_t()
        _check(self.ctx, self.lib.lshom_workspace_size(self.ctx, int(precision), ctypes.byref(size)))
        self._attach_workspace(int(size.value))

    def _attach_workspace(self, nbytes):
        torch = self.torch
        self.ws_bytes = nbytes
        self._ws_raw = None
        raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws_ptr = raw.data_ptr() + off
        _check(self.ctx, self.lib.lshom_set_workspace(self.ctx, c_void_p(self.ws_ptr), self.ws_bytes))

    def _ensure_workspace(self, o):
        """Grows the workspace when the options need more (the extra fields of
        BiCG and pipelined CG)."""
        size = c_size_t()
        _check(self.ctx, self.lib.lshom_workspace_size_for(self.ctx, ctypes.byref(o), ctypes.byref(size)))
        need = int(size.value)
        if o.method in (METHOD_BICG, METHOD_PIPECG):
            # keep the FP32 part as well, so that mixed solves still fit
            mixed = lshom_default_opts()
            mixed.precision = PRECISION_MIXED
            mixed.method = METHOD_BICG
            _check(self.ctx, self.lib.lshom_workspace_size_for(self.ctx, ctypes.byref(mixed), ctypes.byref(size)))
            need = max(need, int(size.value))
        if need > self.ws_bytes:
            self._attach_workspace(need)

    def close(self):
        if getattr(self, "ctx", None):
            lshom_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_reference(self, l0):
        """Reference medium: a number l0 (L0 = l0 I), a symmetric positive
        definite d x d matrix L0, or "mean" (L0 = <L>, the Fourier-space
        Jacobi preconditioner)."""
        if isinstance(l0, str):
            if l0 != "mean":
                raise ValueError('the only named reference is "mean"')
            _check(self.ctx, self.lib.lshom_set_reference_mean(self.ctx))
        elif np.ndim(l0) == 0:
            _check(self.ctx, self.lib.lshom_set_reference(self.ctx, float(l0)))
        else:
            m = np.ascontiguousarray(l0, dtype=np.float64)
            if m.shape != (self.d, self.d):
                raise ValueError(f"L0 must be a number or a {self.d} x {self.d} matrix")
            _check(self.ctx, self.lib.lshom_set_reference_tensor(self.ctx, _dbl_array(m.ravel())))

    def set_cell(self, lengths):
        """Side lengths of the periodic cell (only their ratios matter)."""
        _check(self.ctx, self.lib.lshom_set_cell(self.ctx, _dbl_array(lengths)))

    def opts(self, **kw) -> lshom_solve_opts:
        o = lshom_default_opts()
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def solve(self, E, tol=1e-8, x0=None, want_field=True, allow_fail=False, history=0, out=None, **opt_kw):
        """Returns (e [d, *N] float64 device tensor or None, leff ndarray, info dict).

        ``out``: a contiguous FP64 device tensor of shape (d, *N) that receives
        the field (no allocation).

        ``method`` / ``norm`` select the basic scheme and the equilibrium test
        (METHOD_*, NORM_*); ``history=n`` records (eta_r, eta_e) of the first
        n iterates into ``info["history"]`` (an [m, 2] array, m the iterates
        the solve produced, at most n)."""
        torch = self.torch
        o = self.opts(**opt_kw)
        self._ensure_workspace(o)
        hist = None
        if history:
            hist = torch.full((int(history), 2), float("nan"), dtype=torch.float64, device=self.device)
            o.history_dev = hist.data_ptr()
            o.history_len = int(history)
        if out is not None:
            if (tuple(out.shape) != (self.d,) + self.shape or out.dtype != torch.float64
                    or out.device != self.device or not out.is_contiguous()):
                raise ValueError("out must be a contiguous float64 tensor of shape (d, *N) on the solver's device")
            e = out
        else:
            e = torch.empty((self.d,) + self.shape, dtype=torch.float64, device=self.device) if want_field else None
        leff = (c_double * self.d)()
        info = lshom_solve_info()
        x0p = None
        if x0 is not None:
            x0 = x0.to(device=self.device, dtype=torch.float64).contiguous()
            assert tuple(x0.shape) == (self.d,) + self.shape
            x0p = c_void_p(x0.data_ptr())
        st = self.lib.lshom_solve(self.ctx, _dbl_array(E), float(tol), ctypes.byref(o), x0p,
                                  c_void_p(e.data_ptr()) if e is not None else None, leff,
                                  ctypes.byref(info))
        allow = (LSHOM_ERR_NOT_CONVERGED, LSHOM_ERR_BREAKDOWN) if allow_fail else ()
        _check(self.ctx, st, allow)
        out = info.as_dict()
        if hist is not None:
            m = info.iterations + (1 if o.method == METHOD_CG else 0)
            out["history"] = hist[:min(m, int(history))].cpu().numpy()
        return e, np.array(leff[:]), out

    def homogenize(self, tol=1e-8, **opt_kw):
        o = self.opts(**opt_kw)
        out = (c_double * (self.d * self.d))()
        infos = (lshom_solve_info * self.d)()
        _check(self.ctx, self.lib.lshom_homogenize(self.ctx, float(tol), ctypes.byref(o), out, infos))
        return np.array(out[:]).reshape(self.d, self.d), [i.as_dict() for i in infos]

    PASS_NAMES = PASS_NAMES

    def set_pass_timing(self, enable=True):
        lshom_set_pass_timing(self.ctx, enable)

    def pass_timing(self):
        return lshom_get_pass_timing(self.ctx)

    def time_passes(self, precision=PRECISION_FP64, reps=50):
        """Average device ms and algorithmic bytes per launch of each pass kernel."""
        ms = (c_double * 6)()
        by = (c_double * 6)()
        _check(self.ctx, self.lib.lshom_time_passes(self.ctx, int(precision), int(reps), ms, by))
        return {n: (ms[i], by[i]) for i, n in enumerate(self.PASS_NAMES) if ms[i] > 0}

    def get_schedule(self, precision=PRECISION_FP64):
        s = lshom_schedule()
        _check(self.ctx, self.lib.lshom_get_schedule(self.ctx, int(precision), ctypes.byref(s)))
        return s.as_dict()

    def set_schedule(self, sched):
        s = lshom_schedule.from_dict(sched)
        _check(self.ctx, self.lib.lshom_set_schedule(self.ctx, ctypes.byref(s)))

    def autotune(self, precision=PRECISION_FP64, reps=20):
        """Tune radix orders and pass shapes on this problem; returns the schedule."""
        s = lshom_schedule()
        _check(self.ctx, self.lib.lshom_autotune(self.ctx, int(precision), int(reps), ctypes.byref(s)))
        return s.as_dict()

    def save_schedules(self, path):
        _check(self.ctx, self.lib.lshom_save_schedules(self.ctx, os.fsencode(path)))

    def load_schedules(self, path):
        _check(self.ctx, self.lib.lshom_load_schedules(self.ctx, os.fsencode(path)))

    def apply(self, p):
        """q = (I + B) p for an arbitrary real FP64 field p of shape (d, *N)."""
        torch = self.torch
        p = p.to(device=self.device, dtype=torch.float64).contiguous()
        q = torch.empty_like(p)
        _check(self.ctx, self.lib.lshom_apply(self.ctx, c_void_p(p.data_ptr()), c_void_p(q.data_ptr())))
        return q


# ---------------------------------------------------------------------------
# Many problems in one call
# ---------------------------------------------------------------------------

class BatchSolver:
    """Solves lists of problems with lshom_solve_batched on one device.

    A problem is a dict with ``phase`` (uint8 array or tensor), ``cond``,
    ``E``, ``tol`` and optionally ``l0`` (default (min + max) / 2),
    ``want_field`` (default False), ``cell`` and ``x0`` (an initial guess,
    d x N FP64, projected and kept only if its residual is the smaller).  Workspace and device copies of the
    phase images are owned by torch and kept until ``prepare`` is called with
    other problems.
    """

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("lshom.BatchSolver needs a GPU")
        self.device = torch.device("cuda", device)
        self.ctx = lshom_create(device, torch.cuda.current_stream(self.device).cuda_stream)
        self._keep = []
        self._ws = None

    def close(self):
        if getattr(self, "ctx", None):
            lshom_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, problems, precision=PRECISION_MIXED):
        """Uploads phase images, allocates fields and the workspace."""
        torch = self.torch
        n = len(problems)
        arr = (lshom_problem * n)()
        keep, fields = [], []
        for i, pr in enumerate(problems):
            ph = pr["phase"]
            if not isinstance(ph, torch.Tensor):
                ph = torch.as_tensor(np.ascontiguousarray(ph, dtype=np.uint8))
            ph = ph.to(device=self.device, dtype=torch.uint8).contiguous()
            d = ph.dim()
            cond = _dbl_array(pr["cond"])
            e = None
            if pr.get("want_field", False):
                e = torch.empty((d,) + tuple(ph.shape), dtype=torch.float64, device=self.device)
            keep += [ph, cond, e]
            fields.append(e)
            a = arr[i]
            a.d = d
            for t in range(3):
                a.N[t] = int(ph.shape[t]) if t < d else 1
                a.E[t] = float(pr["E"][t]) if t < d else 0.0
            a.phase_dev = ph.data_ptr()
            a.n_phases = len(pr["cond"])
            a.cond_host = cond
            a.l0 = float(pr.get("l0") or 0.0)
            a.tol = float(pr["tol"])
            a.e_dev = e.data_ptr() if e is not None else None
            for t in range(3):
                a.cell[t] = float(pr["cell"][t]) if pr.get("cell") is not None and t < d else 0.0
            x0 = pr.get("x0")
            if x0 is not None:
                x0 = torch.as_tensor(x0).to(device=self.device, dtype=torch.float64).contiguous()
                if tuple(x0.shape) != (d,) + tuple(ph.shape):
                    raise ValueError(f"problem {i}: x0 must have shape {(d,) + tuple(ph.shape)}")
                keep.append(x0)
            a.x0_dev = x0.data_ptr() if x0 is not None else None
        size = c_size_t()
        _check(self.ctx, self.lib.lshom_batch_workspace_size(self.ctx, n, arr, int(precision), ctypes.byref(size)))
        need = int(size.value)
        if self._ws is None or self._ws.numel() < need + 256:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        self._arr, self._keep, self._fields, self._n, self._need = arr, keep, fields, n, need
        self._precision = int(precision)
        return need

    def _ws_ptr(self):
        return c_void_p(self._ws.data_ptr() + ((-self._ws.data_ptr()) % 256))

    def autotune(self, precision=None, reps=10):
        """Tune every grid of the prepared batch on the batch itself; returns the schedules."""
        prec = self._precision if precision is None else int(precision)
        cap = c_int32(self._n)
        best = (lshom_schedule * self._n)()
        _check(self.ctx, self.lib.lshom_autotune_batched(self.ctx, self._n, self._arr, prec, int(reps),
                                                         self._ws_ptr(), self._need, best, ctypes.byref(cap)))
        return [best[i].as_dict() for i in range(min(cap.value, self._n))]

    def set_schedule(self, sched):
        s = lshom_schedule.from_dict(sched)
        _check(self.ctx, self.lib.lshom_set_schedule(self.ctx, ctypes.byref(s)))

    def save_schedules(self, path):
        _check(self.ctx, self.lib.lshom_save_schedules(self.ctx, os.fsencode(path)))

    def load_schedules(self, path):
        _check(self.ctx, self.lib.lshom_load_schedules(self.ctx, os.fsencode(path)))

    def set_pass_timing(self, enable=True):
        lshom_set_pass_timing(self.ctx, enable)

    def pass_timing(self):
        return lshom_get_pass_timing(self.ctx)

    def run(self, allow_fail=False, **opt_kw):
        """Solve the prepared problems; returns (fields, leff [n, 3], infos)."""
        o = lshom_default_opts()
        for k, v in opt_kw.items():
            setattr(o, k, v)
        n = self._n
        leff = (c_double * (3 * n))()
        infos = (lshom_solve_info * n)()
        st = self.lib.lshom_solve_batched(self.ctx, n, self._arr, ctypes.byref(o), self._ws_ptr(),
                                          self._need, leff, infos)
        allow = (LSHOM_ERR_NOT_CONVERGED, LSHOM_ERR_BREAKDOWN) if allow_fail else ()
        _check(self.ctx, st, allow)
        return self._fields, np.array(leff[:]).reshape(n, 3), [i.as_dict() for i in infos]

