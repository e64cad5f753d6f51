"""Thin ctypes binding of libisweno.so (the C ABI of include/isweno.h).

Argument marshalling only: every step of the method runs in the HIP
library.  Device buffers are torch tensors on the GPU (float64 states, SoA
(nc, ncells), x fastest); calls are enqueued on torch's current stream.
There is no fallback: if the library is missing or a call fails, an
exception is raised.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from pathlib import Path

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "_build" / "libisweno.so"

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_DEVICE, ERR_NONPHYSICAL = 0, -1, -2, -3, -4
BC_TRANSMISSIVE, BC_PERIODIC, BC_REFLECTIVE = 0, 1, 2
FP64, FP32 = 0, 1
W_MODIFIED, W_BASIC, W_MLP, W_CUTOFF = 0, 1, 2, 3
MOOD_OFF, MOOD_ON, MOOD_GATHER = 0, 1, 2
MLP_NI, MLP_H, MLP_NO = 8, 32, 9
MLP_NPARAM = 32 * 8 + 32 + 32 * 32 + 32 + 9 * 32 + 9

_ERR = {ERR_ARG: "invalid argument", ERR_UNSUPPORTED: "unsupported option",
        ERR_DEVICE: "HIP error", ERR_NONPHYSICAL: "non-physical state"}


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64 * 3),
                ("dx", C.c_double * 3), ("bc_lo", C.c_int32 * 3), ("bc_hi", C.c_int32 * 3)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("weights", C.c_int32), ("mood", C.c_int32),
                ("reserved", C.c_int32), ("eps", C.c_double), ("cfl", C.c_double),
                ("dt_max", C.c_double), ("mlp_params", C.c_void_p),
                ("mlp_conf_threshold", C.c_float), ("reserved2", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("o3", C.c_uint64 * 3), ("o1", C.c_uint64 * 3),
                ("mlp_fallback", C.c_uint64 * 3), ("status", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None
_vp = C.c_void_p

# name -> (restype, argtypes)
_SIGS = {
    "isweno_version": (C.c_char_p, []),
    "isweno_create": (C.c_int, [C.POINTER(_vp), C.c_int]),
    "isweno_destroy": (None, [_vp]),
    "isweno_rhs": (C.c_int, [_vp, C.POINTER(Grid), C.POINTER(Opts), _vp, _vp, _vp, _vp]),
    "isweno_cfl_dt": (C.c_int, [_vp, C.POINTER(Grid), C.POINTER(Opts), _vp, _vp, _vp]),
    "isweno_rk3_step": (C.c_int, [_vp, C.POINTER(Grid), C.POINTER(Opts), _vp, _vp, _vp, _vp]),
    "isweno_rk3_step_noalloc": (C.c_int, [_vp, C.POINTER(Grid), C.POINTER(Opts), _vp, _vp, _vp,
                                          _vp]),
    "isweno_batch_plan_create": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_double), C.c_int32, C.c_int32,
                                           C.POINTER(_vp)]),
    "isweno_batch_plan_destroy": (None, [_vp]),
    "isweno_batch_autotune": (C.c_int, [_vp, _vp, C.POINTER(Opts), _vp,
                                        C.POINTER(C.c_int32), _vp]),
    "isweno_batch_step": (C.c_int, [_vp, _vp, C.POINTER(Opts), _vp, _vp, C.c_int32, _vp, _vp,
                                    _vp]),
    "isweno_mlp_samples": (C.c_int, [_vp, C.POINTER(Grid), C.POINTER(Opts), _vp, _vp, _vp,
                                     C.c_int64, C.c_int64, _vp, _vp]),
    "isweno_mlp_forward": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp]),
    "isweno_mlp_infer": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp]),
    "isweno_mlp_loss_grad": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int64, _vp, _vp, _vp]),
    "isweno_mlp_adam": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int32, C.c_float, C.c_float,
                                  C.c_float, C.c_float, _vp]),
    "isweno_mlp_pack": (C.c_int, [_vp, _vp, _vp, _vp]),
    "isweno_timing_enable": (C.c_int, [_vp, C.c_int]),
    "isweno_shortcut_read": (C.c_int, [_vp, C.POINTER(C.c_int64)]),
    "isweno_timing_read": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64)]),
}

K_SWEEP_X, K_SWEEP_Y, K_SWEEP_Z, K_CFL, K_STAGE2D = 0, 1, 2, 3, 4
K_NAMES = {K_SWEEP_X: "sweep_x", K_SWEEP_Y: "sweep_y", K_SWEEP_Z: "sweep_z", K_CFL: "cfl",
           K_STAGE2D: "stage_2d"}

EXPORTED = tuple(_SIGS)


def load() -> C.CDLL:
    """Loads the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(str(LIB_PATH))
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, what: str = "") -> None:
    if code != OK:
        raise RuntimeError(f"isweno{(' ' + what) if what else ''}: "
                           f"{_ERR.get(code, 'error')} ({code})")


def version() -> str:
    return load().isweno_version().decode()


def make_grid(n, dx, bc_lo=0, bc_hi=0) -> Grid:
    n = list(n)
    ndim = len(n)
    dx = list(dx) if hasattr(dx, "__len__") else [float(dx)] * ndim
    g = Grid()
    g.ndim = ndim
    g.reserved = 0
    for a in range(3):
        g.n[a] = int(n[a]) if a < ndim else 1
        g.dx[a] = float(dx[a]) if a < ndim else 1.0
        if a < ndim:
            g.bc_lo[a] = int(bc_lo[a] if hasattr(bc_lo, "__len__") else bc_lo)
            g.bc_hi[a] = int(bc_hi[a] if hasattr(bc_hi, "__len__") else bc_hi)
        else:
            g.bc_lo[a] = g.bc_hi[a] = 0
    return g


def make_opts(precision=FP64, weights=W_MODIFIED, mood=True, eps=1e-40, cfl=0.5,
              dt_max=0.0, mlp_params=None, mlp_conf_threshold=0.5) -> Opts:
    o = Opts()
    # mood: False/True (0/1), or MOOD_GATHER (2) for the gathered redo
    o.precision, o.weights = int(precision), int(weights)
    o.mood = int(mood) if mood == MOOD_GATHER else int(bool(mood))
    o.reserved = 0
    o.eps, o.cfl, o.dt_max = float(eps), float(cfl), float(dt_max)
    o.mlp_params = None if mlp_params is None else int(mlp_params.data_ptr())
    o.mlp_conf_threshold = float(mlp_conf_threshold)
    o.reserved2 = 0
    return o


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def new_stats(device="cuda"):
    """Zeroed device isweno_stats buffer."""
    import torch
    return torch.zeros(C.sizeof(Stats), dtype=torch.uint8, device=device)


def read_stats(buf) -> Stats:
    host = bytes(buf.cpu().numpy().tobytes())
    return Stats.from_buffer_copy(host)


class Context:
    """An isweno_ctx bound to one device."""

    def __init__(self, device: int = 0):
        lib = load()
        h = _vp()
        check(lib.isweno_create(C.byref(h), int(device)), "create")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().isweno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------ operator
    def rhs(self, U, grid: Grid, opts: Opts, out=None, stats=None):
        import torch
        if out is None:
            out = torch.empty_like(U)
        check(load().isweno_rhs(self._h, C.byref(grid), C.byref(opts), _ptr(U), _ptr(out),
                                _ptr(stats), _stream()), "rhs")
        return out

    def cfl_dt(self, U, grid: Grid, opts: Opts, dt):
        check(load().isweno_cfl_dt(self._h, C.byref(grid), C.byref(opts), _ptr(U), _ptr(dt),
                                   _stream()), "cfl_dt")
        return dt

    def rk3_step(self, U, grid: Grid, opts: Opts, dt, stats=None):
        check(load().isweno_rk3_step(self._h, C.byref(grid), C.byref(opts), _ptr(U), _ptr(dt),
                                     _ptr(stats), _stream()), "rk3_step")
        return U

    def rk3_step_noalloc(self, U, grid: Grid, opts: Opts, dt, stats=None):
        """isweno_rk3_step without device allocation (library scratch of
        128 MiB for the intermediate states; see isweno.h)."""
        check(load().isweno_rk3_step_noalloc(self._h, C.byref(grid), C.byref(opts), _ptr(U),
                                             _ptr(dt), _ptr(stats), _stream()),
              "rk3_step_noalloc")
        return U

    # ------------------------------------------------------------ timing
    def timing_enable(self, on: bool = True):
        check(load().isweno_timing_enable(self._h, int(bool(on))), "timing_enable")

    def shortcut_read(self):
        """Field-sides per axis whose reconstruction took its shortcut
        (FP64: tau5 = 0, linear weights; FP32: flat stencil) since timing
        was enabled."""
        c = (C.c_int64 * 3)()
        check(load().isweno_shortcut_read(self._h, c), "shortcut_read")
        return [int(x) for x in c]

    def timing_read(self, kind: int):
        ms = C.c_double(0.0); n = C.c_int64(0)
        check(load().isweno_timing_read(self._h, int(kind), C.byref(ms), C.byref(n)), "timing_read")
        return ms.value, n.value

    # ------------------------------------------------------------ batch
    def batch_plan(self, offsets, dx, bc_lo=0, bc_hi=0) -> "BatchPlan":
        return BatchPlan(self, offsets, dx, bc_lo, bc_hi)

    # ------------------------------------------------------------ MLP
    def mlp_samples(self, U, grid: Grid, opts: Opts, X, Y, max_samples: int, stride: int, count):
        check(load().isweno_mlp_samples(self._h, C.byref(grid), C.byref(opts), _ptr(U), _ptr(X),
                                        _ptr(Y), int(max_samples), int(stride), _ptr(count),
                                        _stream()), "mlp_samples")

    def mlp_forward(self, params, X, out):
        check(load().isweno_mlp_forward(self._h, _ptr(params), _ptr(X), int(X.shape[0]),
                                        _ptr(out), _stream()), "mlp_forward")
        return out

    def mlp_infer(self, packed, X, out):
        """Logits as the solver's stage kernel computes them (packed network)."""
        check(load().isweno_mlp_infer(self._h, _ptr(packed), _ptr(X), int(X.shape[0]),
                                      _ptr(out), _stream()), "mlp_infer")
        return out

    def mlp_loss_grad(self, params, X, Y, Cc, loss, grad):
        """Cc may be None (confidence targets formed by the kernel)."""
        check(load().isweno_mlp_loss_grad(self._h, _ptr(params), _ptr(X), _ptr(Y), _ptr(Cc),
                                          int(X.shape[0]), _ptr(loss), _ptr(grad), _stream()),
              "mlp_loss_grad")

    def mlp_adam(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        check(load().isweno_mlp_adam(self._h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v),
                                     int(step), float(lr), float(beta1), float(beta2), float(eps),
                                     _stream()), "mlp_adam")

    def mlp_pack(self, params, packed):
        check(load().isweno_mlp_pack(self._h, _ptr(params), _ptr(packed), _stream()), "mlp_pack")
        return packed


class BatchPlan:
    """isweno_batch_plan for a fixed set of uneven 1D problems."""

    def __init__(self, ctx: Context, offsets, dx, bc_lo=0, bc_hi=0):
        import numpy as np
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        dxa = np.ascontiguousarray(dx, dtype=np.float64)
        self.nprob = len(dxa)
        self.total = int(off[-1])
        h = _vp()
        check(load().isweno_batch_plan_create(
            ctx.handle, self.nprob, off.ctypes.data_as(C.POINTER(C.c_int64)),
            dxa.ctypes.data_as(C.POINTER(C.c_double)), int(bc_lo), int(bc_hi), C.byref(h)),
            "batch_plan_create")
        self._h = h
        self.ctx = ctx
        self._status = None

    @property
    def status(self):
        """Per-problem status (device int32 [nprob], sticky; 0 = OK) used by
        step() when no status array is passed."""
        import torch
        if self._status is None:
            self._status = torch.zeros(self.nprob, dtype=torch.int32, device="cuda")
        return self._status

    def reset_status(self):
        self.status.zero_()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().isweno_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, U, opts: Opts) -> int:
        tile = C.c_int32(0)
        check(load().isweno_batch_autotune(self.ctx.handle, self._h, C.byref(opts), _ptr(U),
                                           C.byref(tile), _stream()), "batch_autotune")
        return tile.value

    def step(self, U, opts: Opts, dt, nsteps: int = 1, stats=None, status=None):
        st = self.status if status is None else status
        check(load().isweno_batch_step(self.ctx.handle, self._h, C.byref(opts), _ptr(U), _ptr(dt),
                                       int(nsteps), _ptr(stats), _ptr(st), _stream()),
              "batch_step")
        return U


@dataclass
class Solver:
    """Convenience driver: a grid, options and a context."""
    grid: Grid
    opts: Opts
    ctx: Context

    def run(self, U, nsteps: int | None = None, t_end: float | None = None, stats=None):
        """Advance U in place.  With t_end, the CFL time step is clipped to
        the time left (one host read of dt per step)."""
        import torch
        dt = torch.zeros(1, dtype=torch.float64, device=U.device)
        t, k = 0.0, 0
        while True:
            if nsteps is not None and k >= nsteps:
                break
            if t_end is not None and t >= t_end * (1 - 1e-14):
                break
            o = Opts.from_buffer_copy(self.opts)
            if t_end is not None:
                o.dt_max = t_end - t
            self.ctx.rk3_step(U, self.grid, o, dt, stats)
            if t_end is not None:
                t += float(dt.item())
            k += 1
        return U, t, k
