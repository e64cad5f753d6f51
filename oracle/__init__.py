"""Oracle for the WENO-IS finite-volume method of arXiv:1707.00592.

TEST INFRASTRUCTURE ONLY.  A plain FP64 C implementation of the method
(oracle.c, exact_riemann.c, mlp_ref.c) wrapped with ctypes and numpy.  Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package; the HIP library never calls it and shares no code
with it.

Array conventions match oracle.h: conservative states are float64 arrays of
shape (nc, ncells) with x fastest, nc = 4 + ndim.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
BUILD_DIR = HERE / "_build"
LIB_PATH = BUILD_DIR / "liboracle.so"
SOURCES = ["oracle.c", "exact_riemann.c", "mlp_ref.c"]

OK, ERR_ARG, ERR_NONPHYSICAL, ERR_VACUUM = 0, -1, -4, -5
BC_TRANSMISSIVE, BC_PERIODIC, BC_REFLECTIVE = 0, 1, 2
W_MODIFIED, W_BASIC, W_CUTOFF = 0, 1, 3
MLP_NI, MLP_H, MLP_NO = 8, 32, 9
MLP_NPARAM = MLP_H * MLP_NI + MLP_H + MLP_H * MLP_H + MLP_H + MLP_NO * MLP_H + MLP_NO


OPCOUNT_PATH = BUILD_DIR / "libopcount.so"


def build(verbose: bool = False) -> Path:
    """Compile the oracle with gcc (plain C11, -O2, no fused multiply-add),
    and its operation counter (the same source on a counting number type)
    with g++."""
    BUILD_DIR.mkdir(exist_ok=True)
    tmp = BUILD_DIR / f"liboracle.so.tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas",
           "-o", str(tmp)] + [str(HERE / s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    tmp = BUILD_DIR / f"libopcount.so.tmp{os.getpid()}"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden",
           "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", "-o", str(tmp),
           str(HERE / "opcount.cpp")]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, OPCOUNT_PATH)
    return LIB_PATH


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_long * 3), ("dx", C.c_double * 3),
                ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3)]


class Opts(C.Structure):
    _fields_ = [("weights", C.c_int), ("mood", C.c_int), ("eps", C.c_double),
                ("cfl", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("o3", C.c_long * 3), ("o1", C.c_long * 3), ("status", C.c_int)]


_lib = None
_dp = C.POINTER(C.c_double)


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        build()
    lib = C.CDLL(str(LIB_PATH))
    lib.or_weno_candidates.argtypes = [_dp, _dp]
    lib.or_weno_indicators.argtypes = [_dp, _dp]
    lib.or_weno_weights.argtypes = [_dp, C.c_int, C.c_double, C.c_int, _dp]
    lib.or_weno_is.argtypes = [_dp, C.c_int, C.c_double, C.c_int]
    lib.or_weno_is.restype = C.c_double
    lib.or_eigen.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.or_hllc.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
    lib.or_face.argtypes = [C.c_int, _dp, C.POINTER(Opts), _dp, _dp,
                            C.POINTER(C.c_int), _dp, _dp]
    lib.or_pos.argtypes = [C.c_int, _dp]
    lib.or_pos.restype = C.c_int
    lib.or_rhs.argtypes = [C.POINTER(Grid), C.POINTER(Opts), _dp, _dp, C.POINTER(Stats)]
    lib.or_cfl_dt.argtypes = [C.POINTER(Grid), C.POINTER(Opts), _dp, _dp]
    lib.or_rk3_step.argtypes = [C.POINTER(Grid), C.POINTER(Opts), _dp, C.c_double,
                                C.POINTER(Stats)]
    lib.or_batch_step.argtypes = [C.c_int, C.POINTER(C.c_long), _dp, C.c_int, C.c_int,
                                  C.POINTER(Opts), _dp, _dp, C.c_int, C.POINTER(Stats),
                                  C.POINTER(C.c_int)]
    lib.or_exact_star.argtypes = [_dp, _dp, _dp, _dp]
    lib.or_exact_sample.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
    lib.or_exact_sample_n.argtypes = [_dp, _dp, C.c_double, C.c_double, _dp, C.c_long, _dp]
    lib.or_mlp_forward.argtypes = [_dp, _dp, C.c_long, _dp]
    lib.or_mlp_loss_grad.argtypes = [_dp, _dp, _dp, _dp, C.c_long, _dp]
    lib.or_mlp_loss_grad.restype = C.c_double
    lib.or_threads.argtypes = [C.c_int]
    for name in ("or_rhs", "or_cfl_dt", "or_rk3_step", "or_batch_step", "or_exact_star",
                 "or_threads"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def threads(n: int = 0) -> int:
    """Threads of the oracle's OpenMP loops (set when n > 0)."""
    return int(load().or_threads(int(n)))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def make_grid(n, dx, bc_lo=0, bc_hi=0) -> Grid:
    n = list(n)
    ndim = len(n)
    dx = list(dx) if np.ndim(dx) else [float(dx)] * ndim
    g = Grid()
    g.ndim = ndim
    for a in range(3):
        g.n[a] = n[a] if a < ndim else 1
        g.dx[a] = dx[a] if a < ndim else 1.0
        if a < ndim:
            g.bc_lo[a] = int(bc_lo[a] if np.ndim(bc_lo) else bc_lo)
            g.bc_hi[a] = int(bc_hi[a] if np.ndim(bc_hi) else bc_hi)
        else:
            g.bc_lo[a] = g.bc_hi[a] = 0
    return g


def make_opts(weights=W_MODIFIED, mood=True, eps=1e-40, cfl=0.5) -> Opts:
    o = Opts()
    o.weights, o.mood, o.eps, o.cfl = int(weights), int(bool(mood)), float(eps), float(cfl)
    return o


# ---------------------------------------------------------------- pieces
def weno_candidates(v):
    v = _f64(v); out = np.zeros(4)
    load().or_weno_candidates(_ptr(v), _ptr(out))
    return out


def weno_indicators(v):
    """(beta1, beta2, beta3, beta4, beta12, tau5)."""
    v = _f64(v); out = np.zeros(6)
    load().or_weno_indicators(_ptr(v), _ptr(out))
    return out


def weno_weights(v, weights=W_MODIFIED, eps=1e-40, order=5):
    v = _f64(v); out = np.zeros(4)
    load().or_weno_weights(_ptr(v), int(weights), float(eps), int(order), _ptr(out))
    return out


def weno_is(v, weights=W_MODIFIED, eps=1e-40, order=5) -> float:
    v = _f64(v)
    return load().or_weno_is(_ptr(v), int(weights), float(eps), int(order))


def eigen(qbar, nt):
    qbar = _f64(qbar); nc = 5 + nt
    L = np.zeros((nc, nc)); R = np.zeros((nc, nc))
    load().or_eigen(int(nt), _ptr(qbar), _ptr(L), _ptr(R))
    return L, R


def hllc(ql, qr, nt):
    ql = _f64(ql); qr = _f64(qr); F = np.zeros(5 + nt); us = np.zeros(1)
    load().or_hllc(int(nt), _ptr(ql), _ptr(qr), _ptr(F), _ptr(us))
    return F, float(us[0])


def face(q6, nt, opts: Opts | None = None):
    """q6: (6, nc) face-order primitives of cells i-2..i+3."""
    q6 = _f64(q6); nc = 5 + nt
    assert q6.shape == (6, nc)
    o = opts or make_opts()
    ql = np.zeros(nc); qr = np.zeros(nc); F = np.zeros(nc); us = np.zeros(1)
    orders = (C.c_int * 2)()
    load().or_face(int(nt), _ptr(q6), C.byref(o), _ptr(ql), _ptr(qr), orders, _ptr(F), _ptr(us))
    return ql, qr, (orders[0], orders[1]), F, float(us[0])


def pos(q, nt) -> bool:
    q = _f64(q)
    return bool(load().or_pos(int(nt), _ptr(q)))


# ---------------------------------------------------------------- operator
def rhs(U, grid: Grid, opts: Opts | None = None):
    """Returns (dUdt, stats)."""
    U = _f64(U); out = np.zeros_like(U); st = Stats()
    o = opts or make_opts()
    s = load().or_rhs(C.byref(grid), C.byref(o), _ptr(U), _ptr(out), C.byref(st))
    if s == ERR_ARG:
        raise ValueError("oracle rhs: bad arguments")
    return out, st


def cfl_dt(U, grid: Grid, opts: Opts | None = None) -> float:
    U = _f64(U); dt = np.zeros(1)
    o = opts or make_opts()
    s = load().or_cfl_dt(C.byref(grid), C.byref(o), _ptr(U), _ptr(dt))
    if s != OK:
        raise ValueError("oracle cfl_dt: bad arguments")
    return float(dt[0])


def rk3_step(U, grid: Grid, dt: float, opts: Opts | None = None, stats: Stats | None = None):
    """Advances a copy of U by one RK3 step; returns (U_new, status)."""
    U = _f64(U).copy(); st = stats if stats is not None else Stats()
    o = opts or make_opts()
    s = load().or_rk3_step(C.byref(grid), C.byref(o), _ptr(U), float(dt), C.byref(st))
    if s == ERR_ARG:
        raise ValueError("oracle rk3_step: bad arguments")
    return U, s


def run(U, grid: Grid, opts: Opts, t_end: float | None = None, nsteps: int | None = None,
        dt: float | None = None):
    """Plain time loop: CFL dt from U^n each step (clipped to t_end), or a
    fixed dt.  Returns (U, t, steps, stats)."""
    U = _f64(U).copy(); st = Stats(); t = 0.0; k = 0
    while True:
        if nsteps is not None and k >= nsteps:
            break
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        h = cfl_dt(U, grid, opts) if dt is None else dt
        if t_end is not None and t + h > t_end:
            h = t_end - t
        U, s = rk3_step(U, grid, h, opts, st)
        if s != OK:
            raise RuntimeError(f"oracle: non-physical state at step {k}")
        t += h; k += 1
    return U, t, k, st


def batch_step(U, offsets, dx, opts: Opts, dt=None, nsteps=1, bc_lo=0, bc_hi=0, pstatus=None):
    """Returns (U, dt, stats, status) or, with pstatus (int array, updated in
    place), (U, dt, stats, status, pstatus)."""
    U = _f64(U).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    dxa = _f64(dx)
    nprob = len(dxa)
    dta = np.zeros(nprob) if dt is None else _f64(dt).copy()
    st = Stats()
    ps = None
    if pstatus is not None:
        ps = np.ascontiguousarray(pstatus, dtype=np.intc).copy()
    s = load().or_batch_step(nprob, off.ctypes.data_as(C.POINTER(C.c_long)), _ptr(dxa),
                             int(bc_lo), int(bc_hi), C.byref(opts), _ptr(U), _ptr(dta),
                             int(nsteps), C.byref(st),
                             None if ps is None else ps.ctypes.data_as(C.POINTER(C.c_int)))
    if s == ERR_ARG:
        raise ValueError("oracle batch_step: bad arguments")
    if ps is not None:
        return U, dta, st, s, ps
    return U, dta, st, s


# ---------------------------------------------------------------- exact
def exact_star(WL, WR):
    """W = (rho, u, p, gamma, Pinf).  Returns (p*, u*) or raises on vacuum."""
    WL = _f64(WL); WR = _f64(WR); ps = np.zeros(1); us = np.zeros(1)
    s = load().or_exact_star(_ptr(WL), _ptr(WR), _ptr(ps), _ptr(us))
    if s != OK:
        raise ValueError("vacuum")
    return float(ps[0]), float(us[0])


def exact_sample(WL, WR, xi):
    """Exact solution at x/t = xi (array) -> array (len(xi), 5)."""
    WL = _f64(WL); WR = _f64(WR)
    ps, us = exact_star(WL, WR)
    xi = _f64(np.atleast_1d(xi))
    out = np.zeros((xi.size, 5))
    load().or_exact_sample_n(_ptr(WL), _ptr(WR), ps, us, _ptr(xi), xi.size, _ptr(out))
    return out


# ---------------------------------------------------------------- MLP
def mlp_forward(params, X):
    params = _f64(params); X = _f64(X)
    n = X.shape[0]; out = np.zeros((n, MLP_NO))
    load().or_mlp_forward(_ptr(params), _ptr(X), n, _ptr(out))
    return out


def mlp_loss_grad(params, X, Y, Cc=None):
    """Cc None: confidence labels formed from the value errors."""
    params = _f64(params); X = _f64(X); Y = _f64(Y)
    cp = None if Cc is None else _ptr(_f64(Cc))
    g = np.zeros(MLP_NPARAM)
    loss = load().or_mlp_loss_grad(_ptr(params), _ptr(X), _ptr(Y), cp, X.shape[0], _ptr(g))
    return loss, g


# ------------------------------------------------------ operation counts
# Classes of opcount.cpp: additions/subtractions, multiplications,
# divisions, square roots, comparisons.
OP_CLASSES = ("add", "mul", "div", "sqrt", "cmp")
_oc = None


def load_opcount() -> C.CDLL:
    global _oc
    if _oc is not None:
        return _oc
    if not OPCOUNT_PATH.exists():
        build()
    lib = C.CDLL(str(OPCOUNT_PATH))
    lp, ip = C.POINTER(C.c_long), C.POINTER(C.c_int)
    gargs = [C.c_int, lp, _dp, ip, ip, C.c_int, C.c_int, C.c_double]
    lib.oc_face.argtypes = [C.c_int, _dp, C.c_int, C.c_int, C.c_double, lp, ip]
    lib.oc_piece.argtypes = [C.c_int, C.c_int, _dp, C.c_int, C.c_double, C.c_int, lp]
    lib.oc_prim.argtypes = [C.c_int, _dp, C.c_int, lp]
    lib.oc_line.argtypes = gargs + [_dp, C.c_int, C.c_long, lp, lp, lp]
    lib.oc_eval.argtypes = gargs + [_dp, C.c_int, C.c_double, lp, lp]
    for f in ("oc_face", "oc_piece", "oc_prim", "oc_line", "oc_eval"):
        getattr(lib, f).restype = C.c_int
    _oc = lib
    return lib


def _counts(c) -> dict:
    return dict(zip(OP_CLASSES, (int(x) for x in c)))


def _oc_check(code: int, what: str):
    if code != OK:
        raise RuntimeError(f"opcount {what}: {code}")


def opcount_face(nt: int, q6, weights=W_MODIFIED, mood=True, eps=1e-40):
    """Operations of one face (or_face) from its six primitive cell states;
    returns (counts, orders used left/right)."""
    q6 = _f64(q6).ravel(); c = (C.c_long * 5)(); o = (C.c_int * 2)()
    _oc_check(load_opcount().oc_face(nt, _ptr(q6), int(weights), int(bool(mood)), eps, c, o),
              "face")
    return _counts(c), (o[0], o[1])


def opcount_piece(kind: int, nt: int, x, weights=W_MODIFIED, eps=1e-40, order=5) -> dict:
    """kind 0: WENO-IS value from v[5]; 1: face matrices and the projection
    of six cells; 2: HLLC from (ql, qr); 3: positivity test of a state."""
    x = _f64(x).ravel(); c = (C.c_long * 5)()
    _oc_check(load_opcount().oc_piece(kind, nt, _ptr(x), int(weights), eps, order, c), "piece")
    return _counts(c)


def opcount_prim(ndim: int, u, d: int = 0) -> dict:
    u = _f64(u).ravel(); c = (C.c_long * 5)()
    _oc_check(load_opcount().oc_prim(ndim, _ptr(u), d, c), "prim")
    return _counts(c)


def _gargs(grid: Grid, opts: Opts):
    return [grid.ndim, C.cast(grid.n, C.POINTER(C.c_long)), C.cast(grid.dx, _dp),
            C.cast(grid.bc_lo, C.POINTER(C.c_int)), C.cast(grid.bc_hi, C.POINTER(C.c_int)),
            opts.weights, opts.mood, opts.eps]


def opcount_line(U, grid: Grid, opts: Opts, d: int, base: int = 0):
    """One grid line of direction d through cell `base`: (total, sum of its
    faces each counted alone, flux differences + sources + axis sum)."""
    U = _f64(U); t = (C.c_long * 5)(); f = (C.c_long * 5)(); a = (C.c_long * 5)()
    _oc_check(load_opcount().oc_line(*_gargs(grid, opts), _ptr(U), d, base, t, f, a), "line")
    return _counts(t), _counts(f), _counts(a)


def opcount_step(U, grid: Grid, opts: Opts, dt: float):
    """One RK3 step: (total, what the three stage updates add)."""
    U = _f64(U); c = (C.c_long * 5)(); u = (C.c_long * 5)()
    _oc_check(load_opcount().oc_eval(*_gargs(grid, opts), _ptr(U), 1, dt, c, u), "step")
    return _counts(c), _counts(u)


def opcount_rhs(U, grid: Grid, opts: Opts) -> dict:
    U = _f64(U); c = (C.c_long * 5)()
    _oc_check(load_opcount().oc_eval(*_gargs(grid, opts), _ptr(U), 0, 0.0, c, None), "rhs")
    return _counts(c)
