"""Thin ctypes binding of libmhdbunch.so (include/mhd_bunch.h).

Functions keep the C names; they only marshal arguments.  Every step of the update
runs in the library's HIP kernels; PyTorch supplies device memory and the stream.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# MHD_PARITY_BUILD=1 loads the parity build of the same sources (no contraction, correctly
# rounded division and square root), which the parity tests use for their tightest bars
PARITY_BUILD = os.environ.get("MHD_PARITY_BUILD") == "1"
LIB_PATH = os.path.join(HERE, "libmhdbunch_strict.so" if PARITY_BUILD else "libmhdbunch.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mhd_bunch.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2508_09568_amd.build` "
        "(hipcc --offload-arch=gfx950); there is no fallback implementation")

# torch must own the process's HIP runtime before the library is loaded: the library's
# runtime dependency then resolves to the copy torch already mapped, and torch's streams
# and allocations are native objects for the library's launches.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)


def _hip_runtimes():
    try:
        maps = open("/proc/self/maps").read().splitlines()
    except OSError:
        return []
    return sorted({ln.split()[-1] for ln in maps if "libamdhip64" in ln})


if len(_hip_runtimes()) > 1:
    raise ImportError(f"two HIP runtimes are mapped in this process: {_hip_runtimes()}")

MHD_OK, MHD_EINVAL, MHD_ENOMEM, MHD_EDEVICE, MHD_ESTATE, MHD_ENONPHYS, MHD_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6


class mhd_bunch_desc(C.Structure):
    _fields_ = [
        ("n_patches", C.c_int32),
        ("dims", C.POINTER(C.c_int32)),
        ("guard", C.c_int32),
        ("precision", C.c_int32),
        ("gamma", C.c_double),
        ("cfl", C.c_double),
        ("limiter", C.c_int32),
        ("rho_floor", C.c_double),
        ("p_floor", C.c_double),
        ("eps_deg", C.c_double),
        ("max_scratch_bytes", C.c_int64),
        ("emf_solver", C.c_int32),
    ]


_h = C.c_void_p
_v = C.c_void_p
_st = C.c_void_p   # hipStream_t
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)

_SIGS = {
    "mhd_bunch_create": (C.c_int, [C.POINTER(_h), C.POINTER(mhd_bunch_desc)]),
    "mhd_bunch_destroy": (None, [_h]),
    "mhd_bunch_state_elems": (C.c_int64, [_h]),
    "mhd_bunch_state_bytes": (C.c_int64, [_h]),
    "mhd_bunch_patch_offset": (C.c_int64, [_h, C.c_int32]),
    "mhd_bunch_workspace_bytes": (C.c_int64, [_h]),
    "mhd_bunch_bind": (C.c_int, [_h, _v, _st]),
    "mhd_bunch_load": (C.c_int, [_h, _v, C.c_int32, _v, C.c_int32, _st]),
    "mhd_bunch_store": (C.c_int, [_h, _v, C.c_int32, _v, C.c_int32, _st]),
    "mhd_bunch_fill_guards": (C.c_int, [_h, _v, _v, _st]),
    "mhd_bunch_cfl": (C.c_int, [_h, _v, _v, _v, C.c_int32, _st]),
    "mhd_bunch_update": (C.c_int, [_h, _v, _v, _v, _v, _st]),
    "mhd_bunch_update_static": (C.c_int, [_h, _v, _v, _v, _v, _st]),
    "mhd_bunch_update_cfl": (C.c_int, [_h, _v, _v, _v, _v, _v, _v, _st]),
    "mhd_bunch_check": (C.c_int, [_h, _st]),
    "mhd_bunch_profile": (C.c_int, [_h, C.c_int32]),
    "mhd_bunch_profile_read": (C.c_int, [_h, C.c_int32, _dp, C.POINTER(C.c_int64)]),
    "mhd_status_string": (C.c_char_p, [C.c_int]),
    "mhd_bunch_last_error": (C.c_char_p, [_h]),
    "mhd_bunch_adjoint_workspace_bytes": (C.c_int64, [_h, _v]),
    "mhd_bunch_adjoint_bind": (C.c_int, [_h, _v, _v, _st]),
    "mhd_bunch_adjoint": (C.c_int, [_h, _v, _v, _v, _v, _v, _st]),
    "mhd_bunch_tile_count": (C.c_int32, [_h]),
    "mhd_bunch_tile_current": (C.c_int32, [_h]),
    "mhd_bunch_tile_get": (C.c_int, [_h, C.c_int32, _ip]),
    "mhd_bunch_tile_set": (C.c_int, [_h, C.c_int32]),
    "mhd_bunch_autotune": (C.c_int, [_h, _v, _v, _v, _v, C.c_int32, _st, _ip,
                                     C.POINTER(C.c_float)]),
    "mhd_bunch_graph_capture": (C.c_int, [_h, C.c_int32, _v, _v, _v, _v, _v, C.c_int32, _st]),
    "mhd_bunch_lts_step": (C.c_int, [_h, _v, _v, _v, _v, _v, _v, _v, _v, _v, C.c_double,
                                     C.c_double, _st]),
    "mhd_bunch_graph_launch": (C.c_int, [_h, _st]),
    "mhd_bunch_lts_graph_capture": (C.c_int, [_h, C.c_int32, _v, _v, _v, _v, _v, _v, _v, _v, _v,
                                             C.c_double, C.c_double, _st]),
    "mhd_bunch_set_predictor": (C.c_int, [_h, C.c_int32]),
    "mhd_bunch_predictor": (C.c_int32, [_h]),
    "mhd_bunch_predictor_count": (C.c_int32, [_h]),
    "mhd_bunch_predictor_shape": (C.c_int, [_h, C.c_int32, _v]),
    "mhd_bunch_set_solver_split": (C.c_int, [_h, C.c_int32]),
    "mhd_bunch_solver_split": (C.c_int32, [_h]),
    "mhd_stream_create": (C.c_int, [C.POINTER(_h), C.POINTER(mhd_bunch_desc), C.c_int32, C.c_int32]),
    "mhd_stream_destroy": (None, [_h]),
    "mhd_stream_device_bytes": (C.c_int64, [_h]),
    "mhd_stream_bunch_count": (C.c_int32, [_h]),
    "mhd_stream_bind": (C.c_int, [_h, _v, _st]),
    "mhd_stream_configure": (C.c_int, [_h, C.c_int32, C.c_int32, C.c_int32]),
    "mhd_stream_update": (C.c_int, [_h, _v, _v, _v, _v, _st]),
    "mhd_stream_check": (C.c_int, [_h, _st]),
    "mhd_stream_last_error": (C.c_char_p, [_h]),
}

STATIC_SCRATCH_BYTES = 128 << 20   # MHD_STATIC_SCRATCH_BYTES of include/mhd_bunch.h

KERNELS = {"prim": 0, "edge_emf_n": 1, "predict": 2, "solve": 3, "cfl": 4, "guards": 5,
           "edge": 6}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/mhd_bunch.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_\w+)\s*\(", txt)))


class MhdError(RuntimeError):
    def __init__(self, code, what, detail=""):
        msg = f"{what}: {mhd_status_string(code).decode()} ({code})"
        super().__init__(msg + (f" [{detail}]" if detail else ""))
        self.code = code


def _ok(code, what, h=None):
    if code != MHD_OK:
        detail = mhd_bunch_last_error(h).decode() if h else ""
        raise MhdError(code, what, detail)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _optr(t):
    return None if t is None else _ptr(t)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Bunch:
    """A bunch handle bound to a torch-allocated workspace on the current device.

    dims: (P, 3) interior cells per patch; precision 8 (float64) or 4 (float32).
    State buffers are flat torch tensors of `state_elems` elements (layout in
    include/mhd_bunch.h); dt (P,) and dx (P, 3) are float64 device tensors."""

    def __init__(self, dims, g=3, precision=8, gamma=5.0 / 3.0, cfl=0.4, limiter=0,
                 rho_floor=1e-12, p_floor=1e-12, eps_deg=1e-10, max_scratch_bytes=0,
                 emf_solver=0, device="cuda", stream=None):
        import numpy as np
        import torch
        self._dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 3))
        d = mhd_bunch_desc(self._dims.shape[0], self._dims.ctypes.data_as(_ip), g, precision,
                           gamma, cfl, limiter, rho_floor, p_floor, eps_deg, max_scratch_bytes,
                           emf_solver)
        h = _h()
        _ok(mhd_bunch_create(C.byref(h), C.byref(d)), "mhd_bunch_create")
        self._h = h
        self.P = int(self._dims.shape[0])
        self.g = g
        self.precision = precision
        self.dtype = torch.float64 if precision == 8 else torch.float32
        dv = torch.device(device)
        if dv.type == "cuda" and dv.index is None:
            dv = torch.device("cuda", torch.cuda.current_device())
        self.device = dv
        self.state_elems = int(mhd_bunch_state_elems(h))
        self.workspace = torch.empty(int(mhd_bunch_workspace_bytes(h)), dtype=torch.uint8,
                                     device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        _ok(mhd_bunch_bind(h, _ptr(self.workspace), _stream(stream)), "mhd_bunch_bind", h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            mhd_bunch_destroy(h)
            self._h = None

    def new_state(self):
        import torch
        return torch.zeros(self.state_elems, dtype=self.dtype, device=self.device)

    def patch_offset(self, p):
        return int(mhd_bunch_patch_offset(self._h, p))

    # The library sees plain pointers: every buffer is checked here (type, element count,
    # layout, device) so that a wrong tensor raises instead of being read out of bounds.
    def _check(self, t, dtype, n, what):
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what}: a torch tensor is required, got {type(t).__name__}")
        if t.dtype != dtype or t.numel() != n or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{what}: a contiguous {dtype} tensor of {n} elements on "
                             f"{self.device} is required, got {t.dtype} {tuple(t.shape)} on "
                             f"{t.device}{'' if t.is_contiguous() else ', not contiguous'}")

    def _check_state(self, U, what="state"):
        self._check(U, self.dtype, self.state_elems, what)

    def _check_dt(self, dt):
        self._check_dt_named(dt, "dt")

    def _check_dt_named(self, x, what):
        import torch
        self._check(x, torch.float64, self.P, what)

    def _check_dx(self, dx):
        import torch
        self._check(dx, torch.float64, 3 * self.P, "dx")

    def _check_nbr(self, nbr):
        import torch
        self._check(nbr, torch.int32, 27 * self.P, "nbr")

    def update(self, U_in, U_out, dt, dx, stream=None):
        self._check_state(U_in, "U_in")
        self._check_state(U_out, "U_out")
        self._check_dt(dt)
        self._check_dx(dx)
        _ok(mhd_bunch_update(self._h, _ptr(U_in), _ptr(U_out), _ptr(dt), _ptr(dx), _stream(stream)),
            "mhd_bunch_update", self._h)

    def update_cfl(self, U_in, U_out, dt, dx, nbr, dt_next, stream=None):
        """The update, and in the same tiles the next step's global time step of U_out as the
        guard exchange with nbr will leave it (written to every entry of dt_next)."""
        self._check_state(U_in, "U_in")
        self._check_state(U_out, "U_out")
        self._check_dt(dt)
        self._check_dt_named(dt_next, "dt_next")
        self._check_dx(dx)
        self._check_nbr(nbr)
        _ok(mhd_bunch_update_cfl(self._h, _ptr(U_in), _ptr(U_out), _ptr(dt), _ptr(dx), _ptr(nbr),
                                 _ptr(dt_next), _stream(stream)), "mhd_bunch_update_cfl", self._h)

    def update_static(self, U_in, U_out, dt, dx, stream=None):
        """The update with the library's static device scratch (allocates nothing; the bunch
        must be created with 0 < max_scratch_bytes <= STATIC_SCRATCH_BYTES)."""
        self._check_state(U_in, "U_in")
        self._check_state(U_out, "U_out")
        self._check_dt(dt)
        self._check_dx(dx)
        _ok(mhd_bunch_update_static(self._h, _ptr(U_in), _ptr(U_out), _ptr(dt), _ptr(dx),
                                    _stream(stream)), "mhd_bunch_update_static", self._h)

    def cfl(self, U, dx, dt_out, global_min=False, stream=None):
        self._check_state(U)
        self._check_dx(dx)
        self._check_dt(dt_out)
        _ok(mhd_bunch_cfl(self._h, _ptr(U), _ptr(dx), _ptr(dt_out), int(bool(global_min)),
                          _stream(stream)), "mhd_bunch_cfl", self._h)

    def fill_guards(self, U, nbr, stream=None):
        self._check_state(U)
        self._check_nbr(nbr)
        _ok(mhd_bunch_fill_guards(self._h, _ptr(U), _ptr(nbr), _stream(stream)),
            "mhd_bunch_fill_guards", self._h)

    def check(self, stream=None):
        return mhd_bunch_check(self._h, _stream(stream))

    def adjoint_bind(self, nbr_host=None, stream=None):
        """Allocate and bind the adjoint workspace.  nbr_host: (P, 27) int32 host neighbour
        table of the guard fill (guard adjoints fold onto owners), or None for frozen
        guards."""
        import numpy as np
        import torch
        self._nbr_host = None if nbr_host is None else np.ascontiguousarray(nbr_host, dtype=np.int32)
        ptr = None if self._nbr_host is None else self._nbr_host.ctypes.data_as(C.c_void_p)
        nb = int(mhd_bunch_adjoint_workspace_bytes(self._h, ptr))
        if nb < 0:
            raise MhdError(MHD_EINVAL, "mhd_bunch_adjoint_workspace_bytes")
        self.adjoint_workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        _ok(mhd_bunch_adjoint_bind(self._h, ptr, _ptr(self.adjoint_workspace), _stream(stream)),
            "mhd_bunch_adjoint_bind", self._h)

    def adjoint(self, U_in, lam_out, lam_in, dt, dx, stream=None):
        """lam_in = (dU_out/dU_in)^T lam_out for one update at fixed dt (U_in guards filled)."""
        for t, what in ((U_in, "U_in"), (lam_out, "lam_out"), (lam_in, "lam_in")):
            self._check_state(t, what)
        self._check_dt(dt)
        self._check_dx(dx)
        _ok(mhd_bunch_adjoint(self._h, _ptr(U_in), _ptr(lam_out), _ptr(lam_in), _ptr(dt), _ptr(dx),
                              _stream(stream)), "mhd_bunch_adjoint", self._h)

    def profile(self, enable=True):
        _ok(mhd_bunch_profile(self._h, int(bool(enable))), "mhd_bunch_profile")

    def profile_read(self):
        """{kernel: (total_ms, launches)} recorded since profile(True)."""
        out = {}
        for name, k in KERNELS.items():
            ms = C.c_double()
            n = C.c_int64()
            _ok(mhd_bunch_profile_read(self._h, k, C.byref(ms), C.byref(n)),
                "mhd_bunch_profile_read")
            out[name] = (ms.value, n.value)
        return out

    # ---- launch configurations, autotuning, graph-captured runs
    def tile_configs(self):
        """[(tile_x, tile_y, tile_z, mode)] of every launch configuration (mode 0 plain grid,
        1 XCD remap, 2 persistent grid + remap)."""
        out = []
        for i in range(int(mhd_bunch_tile_count(self._h))):
            cfg = (C.c_int32 * 4)()
            _ok(mhd_bunch_tile_get(self._h, i, cfg), "mhd_bunch_tile_get")
            out.append(tuple(int(v) for v in cfg))
        return out

    def tile(self):
        return int(mhd_bunch_tile_current(self._h))

    def set_tile(self, index):
        _ok(mhd_bunch_tile_set(self._h, int(index)), "mhd_bunch_tile_set")

    def set_predictor(self, mode):
        """0 = staged kernels, k >= 1 = fused tile kernel with the k-th predictor shape."""
        _ok(mhd_bunch_set_predictor(self._h, int(mode)), "mhd_bunch_set_predictor")

    def predictor(self):
        return int(mhd_bunch_predictor(self._h))

    def predictor_modes(self):
        """Tile shape of every predictor mode ((0, 0, 0) for the staged kernels)."""
        out = []
        for k in range(int(mhd_bunch_predictor_count(self._h))):
            t = (C.c_int32 * 3)()
            _ok(mhd_bunch_predictor_shape(self._h, k, C.cast(t, C.c_void_p)),
                "mhd_bunch_predictor_shape")
            out.append(tuple(int(v) for v in t))
        return out

    def set_solver_split(self, form):
        """Solver form: 0 one-phase tile, 1 two-phase tile, 2 separate edge-EMF pass, 3 that
        pass as lines of edges (3D bunches; form 2 otherwise)."""
        _ok(mhd_bunch_set_solver_split(self._h, int(form)), "mhd_bunch_set_solver_split")

    def solver_split(self):
        return int(mhd_bunch_solver_split(self._h))

    def autotune(self, U_in, U_out, dt, dx, reps=3, stream=None):
        """Time every launch configuration on these buffers and keep the fastest; returns
        (chosen index, [mean ms per update of each configuration])."""
        self._check_state(U_in, "U_in")
        self._check_state(U_out, "U_out")
        self._check_dt(dt)
        self._check_dx(dx)
        n = int(mhd_bunch_tile_count(self._h))
        ms = (C.c_float * n)()
        best = C.c_int32()
        _ok(mhd_bunch_autotune(self._h, _ptr(U_in), _ptr(U_out), _ptr(dt), _ptr(dx), int(reps),
                               _stream(stream), C.byref(best), ms), "mhd_bunch_autotune", self._h)
        return int(best.value), [float(v) for v in ms]

    def graph_capture(self, nsteps, U_a, U_b, dt, dx, nbr=None, dt_mode=0, stream=None):
        """Capture nsteps ping-pong steps (U_a -> U_b -> U_a ...) in one HIP graph;
        dt_mode 0 = dt as given, 1 = per-patch own CFL step, 2 = global minimum;
        nbr = device neighbour table to fill guards before each step, or None (frozen)."""
        self._check_state(U_a, "U_a")
        self._check_state(U_b, "U_b")
        self._check_dt(dt)
        self._check_dx(dx)
        if nbr is not None:
            self._check_nbr(nbr)
        self._graph_refs = (U_a, U_b, dt, dx, nbr)   # keep the bound buffers alive
        _ok(mhd_bunch_graph_capture(self._h, int(nsteps), _ptr(U_a), _ptr(U_b), _ptr(dt), _ptr(dx),
                                    None if nbr is None else _ptr(nbr), int(dt_mode),
                                    _stream(stream)), "mhd_bunch_graph_capture", self._h)

    def lts_step(self, U_cur, U_new, U_prev, t, t_prev, dt, dx, nbr, t_end, dt_fixed=None,
                 dt_quantum=0.0, stream=None):
        """One local time step (see include/mhd_bunch.h): ready patches fill their guards at
        their own time from the owners' two slices and advance by their own CFL step (or
        dt_fixed; rounded down to dt_quantum x 2^k if dt_quantum > 0) clipped to t_end; the
        others stay.  t, t_prev and dt (written) are (P,) float64 device tensors.  The update
        runs in place: U_new is not used (None, or any state tensor); on return U_cur holds
        every patch at its own time and U_prev the owned values of its previous slice."""
        for x, what in ((U_cur, "U_cur"), (U_new, "U_new"), (U_prev, "U_prev")):
            if x is not None or what != "U_new":
                self._check_state(x, what)
        for x, what in ((t, "t"), (t_prev, "t_prev"), (dt, "dt")):
            self._check_dt_named(x, what)
        if dt_fixed is not None:
            self._check_dt_named(dt_fixed, "dt_fixed")
        self._check_dx(dx)
        self._check_nbr(nbr)
        _ok(mhd_bunch_lts_step(self._h, _ptr(U_cur), _optr(U_new), _ptr(U_prev), _ptr(t),
                               _ptr(t_prev), _ptr(dt), None if dt_fixed is None else _ptr(dt_fixed),
                               _ptr(dx), _ptr(nbr), float(t_end), float(dt_quantum),
                               _stream(stream)),
            "mhd_bunch_lts_step", self._h)

    def lts_graph_capture(self, nsteps, U_cur, U_new, U_prev, t, t_prev, dt, dx, nbr, t_end,
                          dt_fixed=None, dt_quantum=0.0, stream=None):
        """Capture nsteps local time steps (arguments as lts_step) in the handle's HIP graph;
        graph_launch runs them."""
        for x, what in ((U_cur, "U_cur"), (U_new, "U_new"), (U_prev, "U_prev")):
            if x is not None or what != "U_new":
                self._check_state(x, what)
        for x, what in ((t, "t"), (t_prev, "t_prev"), (dt, "dt")):
            self._check_dt_named(x, what)
        if dt_fixed is not None:
            self._check_dt_named(dt_fixed, "dt_fixed")
        self._check_dx(dx)
        self._check_nbr(nbr)
        self._graph_refs = (U_cur, U_new, U_prev, t, t_prev, dt, dt_fixed, dx, nbr)
        _ok(mhd_bunch_lts_graph_capture(self._h, int(nsteps), _ptr(U_cur), _optr(U_new),
                                        _ptr(U_prev), _ptr(t), _ptr(t_prev), _ptr(dt),
                                        None if dt_fixed is None else _ptr(dt_fixed), _ptr(dx),
                                        _ptr(nbr), float(t_end), float(dt_quantum),
                                        _stream(stream)),
            "mhd_bunch_lts_graph_capture", self._h)

    def graph_launch(self, stream=None):
        _ok(mhd_bunch_graph_launch(self._h, _stream(stream)), "mhd_bunch_graph_launch", self._h)


class Stream:
    """A bunch whose state stays in host memory, streamed through the device in sub-bunches
    of at most `patches_per_bunch` patches over `slots` device slots (copy in, update, copy
    out on three streams).  State buffers are flat host tensors (pinned for overlap)."""

    def __init__(self, dims, patches_per_bunch, slots=3, g=3, precision=8, gamma=5.0 / 3.0,
                 cfl=0.4, limiter=0, rho_floor=1e-12, p_floor=1e-12, eps_deg=1e-10,
                 emf_solver=0, device="cuda", stream=None):
        import numpy as np
        import torch
        self._dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 3))
        d = mhd_bunch_desc(self._dims.shape[0], self._dims.ctypes.data_as(_ip), g, precision,
                           gamma, cfl, limiter, rho_floor, p_floor, eps_deg, 0, emf_solver)
        h = _h()
        _ok(mhd_stream_create(C.byref(h), C.byref(d), int(patches_per_bunch), int(slots)),
            "mhd_stream_create")
        self._h = h
        self.P = int(self._dims.shape[0])
        self.precision = precision
        self.dtype = torch.float64 if precision == 8 else torch.float32
        dv = torch.device(device)
        if dv.type == "cuda" and dv.index is None:
            dv = torch.device("cuda", torch.cuda.current_device())
        self.device = dv
        ncell = np.prod(np.where(self._dims > 1, self._dims + 2 * g, 1), axis=1)
        self.state_elems = int(8 * ncell.sum())
        self.buffer = torch.empty(int(mhd_stream_device_bytes(h)), dtype=torch.uint8, device=dv)
        code = mhd_stream_bind(h, _ptr(self.buffer), _stream(stream))
        if code != MHD_OK:
            raise MhdError(code, "mhd_stream_bind", mhd_stream_last_error(h).decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            mhd_stream_destroy(h)
            self._h = None

    def bunches(self):
        return int(mhd_stream_bunch_count(self._h))

    def configure(self, tile, predictor, split):
        _ok(mhd_stream_configure(self._h, int(tile), int(predictor), int(split)),
            "mhd_stream_configure")

    def _check_host(self, t, dtype, n, what):
        import torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cpu" or t.dtype != dtype \
                or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{what}: a contiguous host {dtype} tensor of {n} elements is required")

    def update(self, U_in, U_out, dt, dx, stream=None):
        import torch
        self._check_host(U_in, self.dtype, self.state_elems, "U_in")
        self._check_host(U_out, self.dtype, self.state_elems, "U_out")
        self._check_host(dt, torch.float64, self.P, "dt")
        self._check_host(dx, torch.float64, 3 * self.P, "dx")
        code = mhd_stream_update(self._h, _ptr(U_in), _ptr(U_out), _ptr(dt), _ptr(dx),
                                 _stream(stream))
        if code != MHD_OK:
            raise MhdError(code, "mhd_stream_update", mhd_stream_last_error(self._h).decode())

    def check(self, stream=None):
        return mhd_stream_check(self._h, _stream(stream))
