"""FP64 CPU oracle for the per-patch ideal-MHD update -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``libmhd_oracle.so`` (built from ``mhd_oracle.cpp`` by
:func:`build`).  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product library never calls it and
the two share no code.

Arrays are numpy float64, one patch = 8 fields x (Nz, Ny, Nx) padded boxes, field
order rho, rho*u, rho*v, rho*w, E, Bx, By, Bz; face fields sit on the lower face of
their cell (the staggering of the paper's Fig. 2).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhd_oracle.cpp")
_LIB = os.path.join(_HERE, "libmhd_oracle.so")

# plain IEEE FP64: no contraction into fused multiply-adds, no fast-math
CXXFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c++17",
            "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with the host C++ compiler; returns the library path."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", *CXXFLAGS, _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("rho_floor", C.c_double),
                ("p_floor", C.c_double), ("eps_deg", C.c_double), ("limiter", C.c_int32),
                ("emf_solver", C.c_int32)]


@dataclass
class Params:
    gamma: float = 5.0 / 3.0
    cfl: float = 0.4
    rho_floor: float = 1e-12
    p_floor: float = 1e-12
    eps_deg: float = 1e-10
    limiter: int = 0          # 0 = MC, 1 = minmod
    emf_solver: int = 0       # edge EMF: 0 = UCT-HLL, 1 = UCT-HLLD

    def c(self) -> _Params:
        return _Params(self.gamma, self.cfl, self.rho_floor, self.p_floor, self.eps_deg,
                       self.limiter, self.emf_solver)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp, ip, lp = P(C.c_double), P(C.c_int32), P(C.c_int64)
        L.mhd_oracle_step.argtypes = [ip, C.c_int32, dp, dp, C.c_double, dp, P(_Params), lp]
        L.mhd_oracle_step_many.argtypes = [C.c_int32, ip, C.c_int32, dp, dp, dp, dp, P(_Params), lp]
        L.mhd_oracle_cfl.argtypes = [ip, C.c_int32, dp, dp, P(_Params)]
        L.mhd_oracle_cfl.restype = C.c_double
        L.mhd_oracle_cfl_many.argtypes = [C.c_int32, ip, C.c_int32, dp, dp, P(_Params), dp]
        L.mhd_oracle_fill_guards.argtypes = [C.c_int32, ip, C.c_int32, dp, ip]
        L.mhd_oracle_step_jvp.argtypes = [ip, C.c_int32, dp, dp, dp, dp, C.c_double, dp, P(_Params)]
        L.mhd_oracle_step_jvp_many.argtypes = [C.c_int32, ip, C.c_int32, dp, dp, dp, dp, dp, dp,
                                               P(_Params)]
        up = P(C.c_uint64)
        L.mhd_oracle_step_sig_many.argtypes = [C.c_int32, ip, C.c_int32, dp, dp, dp, dp,
                                               P(_Params), up]
        L.mhd_oracle_step_ext_many.argtypes = [C.c_int32, ip, C.c_int32, C.c_void_p, C.c_void_p,
                                               dp, dp, P(_Params), up]
        L.mhd_oracle_fill_guards_ext.argtypes = [C.c_int32, ip, C.c_int32, C.c_void_p, ip]
        L.mhd_oracle_fill_guards_at.argtypes = [C.c_int32, ip, C.c_int32, dp, dp, dp, dp, ip, ip]
        L.mhd_oracle_count_ops.argtypes = [ip, C.c_int32, dp, C.c_double, dp, P(_Params), lp]
        L.mhd_oracle_hlld.argtypes = [dp, dp, P(_Params), dp, ip]
        L.mhd_oracle_hlld_fan.argtypes = [dp, dp, P(_Params), dp, ip, dp, dp]
        L.mhd_oracle_cfast.argtypes = [C.c_double] * 6
        L.mhd_oracle_cfast.restype = C.c_double
        L.mhd_oracle_limiter.argtypes = [C.c_double, C.c_double, C.c_int32]
        L.mhd_oracle_limiter.restype = C.c_double
        L.mhd_oracle_uct.argtypes = [dp, P(_Params)]
        L.mhd_oracle_uct.restype = C.c_double
        L.mhd_oracle_dqdt.argtypes = [dp, dp, ip, C.c_double, dp]
        L.mhd_oracle_threads.restype = C.c_int
        L.mhd_oracle_set_threads.argtypes = [C.c_int]
        L.mhd_oracle_set_threads.restype = None
        L.mhd_oracle_ops_per_cell.argtypes = [ip, C.c_int32, dp, C.c_double, dp, P(_Params), dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def threads() -> int:
    """OpenMP threads used by the multi-patch entry points."""
    return int(lib().mhd_oracle_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP threads of the multi-patch entry points."""
    lib().mhd_oracle_set_threads(int(n))


def step_many(U, dims, g, dt, dx, prm: Params, count_floors=False):
    """Advance every patch of the flat state U (float64) by its own dt; returns U_out
    (guards copied from U) and, if asked, floor activations per site (cell primitives,
    face states, edge-corner states)."""
    U = _f64(U)
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (P,)))
    dx = _f64(np.broadcast_to(np.asarray(dx, dtype=np.float64), (P, 3)))
    out = np.empty_like(U)
    nf = np.zeros(3, dtype=np.int64)
    p = prm.c()
    rc = lib().mhd_oracle_step_many(P, _i(dims), g, _d(U), _d(out), _d(dt), _d(dx), C.byref(p),
                                    nf.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc != 0:
        raise ValueError("mhd_oracle_step_many: invalid argument")
    return (out, nf) if count_floors else out


def step_sig_many(U, dims, g, dt, dx, prm: Params):
    """step_many (bitwise the same U_out) plus each patch's branch signature, a uint64
    hash of every comparison outcome of its update."""
    U = _f64(U)
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (P,)))
    dx = _f64(np.broadcast_to(np.asarray(dx, dtype=np.float64), (P, 3)))
    out = np.empty_like(U)
    sig = np.zeros(P, dtype=np.uint64)
    p = prm.c()
    rc = lib().mhd_oracle_step_sig_many(P, _i(dims), g, _d(U), _d(out), _d(dt), _d(dx),
                                        C.byref(p), sig.ctypes.data_as(C.POINTER(C.c_uint64)))
    if rc != 0:
        raise ValueError("mhd_oracle_step_sig_many: invalid argument")
    return out, sig


def step_ext_many(U, dims, g, dt, dx, prm: Params):
    """One update in x87 extended precision: U is np.longdouble; returns (U_out, per-patch
    branch signatures).  Same scheme and FP64 parameters as step_many."""
    assert U.dtype == np.longdouble and np.finfo(np.longdouble).nmant >= 63
    U = np.ascontiguousarray(U)
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (P,)))
    dx = _f64(np.broadcast_to(np.asarray(dx, dtype=np.float64), (P, 3)))
    out = np.empty_like(U)
    sig = np.zeros(P, dtype=np.uint64)
    p = prm.c()
    rc = lib().mhd_oracle_step_ext_many(P, _i(dims), g, U.ctypes.data, out.ctypes.data, _d(dt),
                                        _d(dx), C.byref(p),
                                        sig.ctypes.data_as(C.POINTER(C.c_uint64)))
    if rc != 0:
        raise ValueError("mhd_oracle_step_ext_many: invalid argument")
    return out, sig


def fill_guards_ext(U, dims, g, nbr):
    """fill_guards on an np.longdouble state."""
    assert U.dtype == np.longdouble and U.flags.c_contiguous
    dims = _i32(dims).reshape(-1, 3)
    nbr = _i32(nbr).reshape(-1, 27)
    if lib().mhd_oracle_fill_guards_ext(dims.shape[0], _i(dims), g, U.ctypes.data, _i(nbr)) != 0:
        raise ValueError("mhd_oracle_fill_guards_ext: inconsistent neighbour table")
    return U


def cfl_many(U, dims, g, dx, prm: Params):
    U = _f64(U)
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    dx = _f64(np.broadcast_to(np.asarray(dx, dtype=np.float64), (P, 3)))
    dt = np.empty(P, dtype=np.float64)
    p = prm.c()
    rc = lib().mhd_oracle_cfl_many(P, _i(dims), g, _d(U), _d(dx), C.byref(p), _d(dt))
    if rc != 0:
        raise ValueError("mhd_oracle_cfl_many: invalid argument")
    return dt


def fill_guards(U, dims, g, nbr):
    """In-place guard fill of the flat float64 state U from a (P, 27) neighbour table."""
    assert U.dtype == np.float64 and U.flags.c_contiguous
    dims = _i32(dims).reshape(-1, 3)
    nbr = _i32(nbr).reshape(-1, 27)
    rc = lib().mhd_oracle_fill_guards(dims.shape[0], _i(dims), g, _d(U), _i(nbr))
    if rc != 0:
        raise ValueError("mhd_oracle_fill_guards: inconsistent neighbour table")
    return U


def fill_guards_at(U, U_prev, t, t_prev, dims, g, nbr, mask=None):
    """In-place guard fill of U at each patch's own time t[p]: the owner's value linearly
    interpolated between its slices (t_prev, U_prev) and (t, U) (local time stepping)."""
    assert U.dtype == np.float64 and U.flags.c_contiguous
    U_prev = _f64(U_prev)
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    nbr = _i32(nbr).reshape(-1, 27)
    t, t_prev = _f64(t), _f64(t_prev)
    assert t.shape == (P,) and t_prev.shape == (P,) and U_prev.shape == U.shape
    m = None if mask is None else _i32(np.asarray(mask).astype(np.int32))
    rc = lib().mhd_oracle_fill_guards_at(P, _i(dims), g, _d(U), _d(U_prev), _d(t), _d(t_prev),
                                         _i(nbr), None if m is None else _i(m))
    if rc != 0:
        raise ValueError("mhd_oracle_fill_guards_at: invalid argument or neighbour table")
    return U


def lts_ready(t, t_end, nbr):
    """Patches that may advance: below t_end, and no neighbour (any of the 26 directions)
    behind them, so every guard value is an interpolation within the owner's two slices."""
    t = np.asarray(t, dtype=np.float64)
    nbr = np.asarray(nbr).reshape(-1, 27)
    ready = t < t_end
    for p in range(t.shape[0]):
        for q in nbr[p]:
            if q >= 0 and q != p and t[q] < t[p]:
                ready[p] = False
    return ready


def lts_run(U, dims, g, dx, nbr, prm: Params, t_end, dt_fixed=None, dt_quantum=0.0,
            max_steps=100000):
    """Local time stepping to t_end (§2.2 "DISPATCH": each patch advances with its own time
    step; guard zones interpolated in time from the neighbours' slices).  A step: the ready
    patches (lts_ready) fill their guards at their own time (fill_guards_at), take their own
    CFL step (or dt_fixed[p]; with dt_quantum > 0 rounded down to dt_quantum x 2^k, k an
    integer: time levels) clipped to t_end and advance (a clipped step ends exactly at t_end);
    the others stay.  The previous slice of an advanced patch is its state before the
    step.  Returns (U, t, steps per patch,
    number of steps)."""
    U = _f64(U).copy()
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    base = np.zeros(P + 1, dtype=np.int64)
    for p in range(P):
        base[p + 1] = base[p] + patch_elems_of(dims[p], g)
    Uprev = U.copy()
    t = np.zeros(P)
    tp = np.zeros(P)
    count = np.zeros(P, dtype=np.int64)
    nsteps = 0
    while np.any(t < t_end):
        if nsteps >= max_steps:
            raise RuntimeError("lts_run: step limit reached")
        ready = lts_ready(t, t_end, nbr)
        fill_guards_at(U, Uprev, t, tp, dims, g, nbr, mask=ready)
        dt = np.asarray(dt_fixed, dtype=np.float64).copy() if dt_fixed is not None else \
            cfl_many(U, dims, g, dx, prm)
        if dt_quantum > 0:
            _, e = np.frexp(dt / dt_quantum)               # dt / quantum in [2^(e-1), 2^e)
            dt = np.ldexp(np.full(P, float(dt_quantum)), e - 1)
        dt = np.where(ready, np.minimum(dt, t_end - t), 0.0)
        Un = step_many(U, dims, g, dt, dx, prm)
        for p in np.nonzero(ready)[0]:
            Uprev[base[p]:base[p + 1]] = U[base[p]:base[p + 1]]
        tp = np.where(ready, t, tp)
        t = np.where(ready & (dt >= t_end - t), t_end, t + dt)   # the last step lands on t_end
        count += ready
        U = Un
        nsteps += 1
    return U, t, count, nsteps


def patch_elems_of(n, g):
    e = 8
    for d in range(3):
        e *= int(n[d]) + 2 * g if n[d] > 1 else 1
    return e


def jvp_many(U, dU, dims, g, dt, dx, prm: Params):
    """(U_out, dU_out) = (step(U), d step(U) . dU) at fixed dt, by dual numbers."""
    U, dU = _f64(U), _f64(dU)
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (P,)))
    dx = _f64(np.broadcast_to(np.asarray(dx, dtype=np.float64), (P, 3)))
    Uo, dUo = np.empty_like(U), np.empty_like(U)
    p = prm.c()
    rc = lib().mhd_oracle_step_jvp_many(P, _i(dims), g, _d(U), _d(dU), _d(Uo), _d(dUo), _d(dt),
                                        _d(dx), C.byref(p))
    if rc != 0:
        raise ValueError("mhd_oracle_step_jvp_many: invalid argument")
    return Uo, dUo


def count_ops(U, n, g, dt, dx, prm: Params):
    """Counts of (add/sub, mul, div, sqrt, compare) performed by one patch update."""
    U = _f64(U)
    n = _i32(n)
    dx = _f64(dx)
    cnt = np.zeros(5, dtype=np.int64)
    p = prm.c()
    rc = lib().mhd_oracle_count_ops(_i(n), g, _d(U), dt, _d(dx), C.byref(p),
                                    cnt.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc != 0:
        raise ValueError("mhd_oracle_count_ops: invalid argument")
    return cnt


def ops_per_cell(U, n, g, dt, dx, prm: Params):
    """Algorithmic (add/sub, mul, div, sqrt, compare) per interior cell-update."""
    U = _f64(U)
    n = _i32(n)
    dx = _f64(dx)
    out = np.zeros(5)
    p = prm.c()
    if lib().mhd_oracle_ops_per_cell(_i(n), g, _d(U), dt, _d(dx), C.byref(p), _d(out)) != 0:
        raise ValueError("mhd_oracle_ops_per_cell: invalid argument")
    return out


def hlld(L, R, prm: Params):
    L, R = _f64(L), _f64(R)
    F = np.empty(5, dtype=np.float64)
    reg = np.zeros(1, dtype=np.int32)
    p = prm.c()
    lib().mhd_oracle_hlld(_d(L), _d(R), C.byref(p), _d(F), _i(reg))
    return F, int(reg[0])


def hlld_fan(L, R, prm: Params):
    """HLLD flux with its wave fan: (F, region, speeds (S_L, S*_L, S_M, S*_R, S_R, and
    the total pressure of the intermediate states), states (U*_L, U**_L, U**_R, U*_R) as
    rows (rho, m_n, m_t1, m_t2, E, B_n, B_t1, B_t2))."""
    L, R = _f64(L), _f64(R)
    F = np.empty(5, dtype=np.float64)
    reg = np.zeros(1, dtype=np.int32)
    sp = np.empty(6, dtype=np.float64)
    st = np.empty((4, 8), dtype=np.float64)
    p = prm.c()
    lib().mhd_oracle_hlld_fan(_d(L), _d(R), C.byref(p), _d(F), _i(reg), _d(sp), _d(st))
    return F, int(reg[0]), sp, st


def cfast(rho, p, bn, bt1, bt2, gamma):
    return lib().mhd_oracle_cfast(rho, p, bn, bt1, bt2, gamma)


def limiter(dl, dr, kind=0):
    return lib().mhd_oracle_limiter(dl, dr, kind)


def uct(W, prm: Params):
    """EMF_z from corner states W[4][8] ordered SW, SE, NW, NE."""
    W = _f64(W).reshape(4, 8)
    p = prm.c()
    return lib().mhd_oracle_uct(_d(W), C.byref(p))


def dqdt(q, D, act, gamma):
    q, D = _f64(q), _f64(D).reshape(3, 8)
    a = _i32(act)
    out = np.empty(8, dtype=np.float64)
    lib().mhd_oracle_dqdt(_d(q), _d(D), _i(a), gamma, _d(out))
    return out


def run(U, dims, g, dx, nbr, prm: Params, t_end=None, nsteps=None, dt_fixed=None,
        record_dt=False, count_floors=False):
    """Synchronous multi-patch driver: per step fill guards, take the global time step
    (minimum over patches, last step clipped to t_end), advance every patch.

    Exactly one of t_end / nsteps; dt_fixed (scalar or sequence) overrides the rule."""
    U = _f64(U).copy()
    dims = _i32(dims).reshape(-1, 3)
    P = dims.shape[0]
    t, k, dts, nfl = 0.0, 0, [], np.zeros(3, dtype=np.int64)
    while True:
        if nsteps is not None and k >= nsteps:
            break
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        fill_guards(U, dims, g, nbr)
        if dt_fixed is not None:
            dt = float(dt_fixed[k]) if np.ndim(dt_fixed) else float(dt_fixed)
        else:
            dt = float(cfl_many(U, dims, g, dx, prm).min())
            if t_end is not None and t + dt > t_end:
                dt = t_end - t
        U, nf = step_many(U, dims, g, np.full(P, dt), dx, prm, count_floors=True)
        nfl += nf
        dts.append(dt)
        t += dt
        k += 1
    fill_guards(U, dims, g, nbr)
    res = [U]
    if record_dt:
        res.append(np.array(dts))
    if count_floors:
        res.append(nfl)
    return res[0] if len(res) == 1 else tuple(res)
