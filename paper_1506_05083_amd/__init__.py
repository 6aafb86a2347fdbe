"""Python binding of libmfs, the MI355X implementation of the axisymmetric
MFS scattering solver (Liu & Barnett, doubly-periodic arrays of axisymmetric
objects).  Argument marshalling only: every step of the computation runs in
the HIP kernels of libmfs.so; PyTorch provides device memory and streams.

The library must have been built (``python -m paper_1506_05083_amd.build``);
importing the computational entry points without it raises RuntimeError.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfs.so")
_lib = None

MFS_OK, MFS_EINVAL, MFS_ENOMEM, MFS_EDEVICE, MFS_ENOTCONV, MFS_ESTATE, MFS_EBUSY = range(7)
TARGETS_SURFACE, TARGETS_WALLS, TARGETS_USER = 0, 1, 2
LAYOUT_MODES, LAYOUT_ANGLE, LAYOUT_POINTS = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class C128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


_cp = C.POINTER(C128)


class Body(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("P", C.c_int32), ("q", C.c_int32),
                ("k", C.c_double), ("rho", _dp), ("z", _dp), ("nrho", _dp), ("nz", _dp),
                ("srho", _dp), ("sz", _dp), ("km", C.c_double), ("srho_out", _dp), ("sz_out", _dp)]


class PolarSpec(C.Structure):
    _fields_ = [("a", C.c_double), ("eps", C.c_double), ("j", C.c_int32), ("colloc", C.c_int32),
                ("M", C.c_int32), ("N", C.c_int32), ("tau", C.c_double)]


class CupSpec(C.Structure):
    _fields_ = [("outer", C.c_double), ("half", C.c_double), ("b", C.c_double), ("colloc", C.c_int32),
                ("M", C.c_int32), ("N", C.c_int32), ("tau", C.c_double)]


class Lattice(C.Structure):
    _fields_ = [("ex", C.c_double), ("ey", C.c_double), ("z0", C.c_double), ("p", C.c_int32),
                ("N0", C.c_double), ("M1", C.c_int32)]


class Wave(C.Structure):
    _fields_ = [("theta", C.c_double), ("phi", C.c_double)]


class Result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("resid", C.c_double), ("norders", C.c_int32),
                ("cap_orders", C.c_int32), ("m", _ip), ("n", _ip), ("kz", _cp), ("a", _cp),
                ("b", _cp), ("field", _cp), ("eps_flux", C.c_double), ("q_rank", C.c_int32),
                ("nq_cols", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("slots", C.c_int32), ("admit_batch", C.c_int32), ("queue_cap", C.c_int32),
                ("tol", C.c_double), ("maxit", C.c_int32), ("rel_cutoff", C.c_double),
                ("targets", C.POINTER(C.c_double)), ("ntargets", C.c_int32), ("q_field", C.c_int32),
                ("hbm_budget", C.c_uint64)]


class SolveTiming(C.Structure):
    _fields_ = [("rhs", C.c_double), ("periodizer", C.c_double), ("gmres", C.c_double),
                ("recover", C.c_double), ("total", C.c_double), ("nsum_avg", C.c_double),
                ("nsum_launches", C.c_int32), ("jacobi_ms", C.c_double),
                ("jacobi_launches", C.c_int32), ("jacobi_bytes", C.c_double),
                ("jacobi_flops", C.c_double), ("near_fill_ms", C.c_double),
                ("near_bytes", C.c_double), ("near_alg_bytes", C.c_double), ("near_mode", C.c_int32),
                ("q_qr_ms", C.c_double), ("q_qr_flops", C.c_double), ("q_post_ms", C.c_double)]


_SIGS = {
    "mfs_last_error": (C.c_char_p, []),
    "mfs_version": (C.c_char_p, []),
    "mfs_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "mfs_destroy": (None, [C.c_void_p]),
    "mfs_memory_stats": (C.c_int, [C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                   C.POINTER(C.c_uint64)]),
    "mfs_memory_reset_peak": (C.c_int, [C.c_int]),
    "mfs_release_cached_memory": (C.c_int, [C.c_int]),
    "mfs_polar_geometry": (C.c_int, [C.POINTER(PolarSpec), _dp, _dp, _dp, _dp, _dp, _dp]),
    "mfs_cup_geometry": (C.c_int, [C.POINTER(CupSpec), _dp, _dp, _dp, _dp, _dp, _dp]),
    "mfs_build_operator": (C.c_int, [C.c_void_p, C.POINTER(Body), C.c_int32, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    "mfs_destroy_op": (None, [C.c_void_p]),
    "mfs_op_blocks": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "mfs_factor_modes": (C.c_int, [C.c_void_p, C.c_double, _ip]),
    "mfs_op_singular_values": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "mfs_op_timing": (C.c_int, [C.c_void_p, _dp]),
    "mfs_set_near_field_budget": (C.c_int, [C.c_void_p, C.c_uint64]),
    "mfs_apply_solution_op": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                        C.c_void_p, C.c_int32, C.c_void_p]),
    "mfs_apply_solution_op_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                                C.c_void_p, C.c_int32, C.c_void_p]),
    "mfs_rhs_modes": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _dp, C.c_void_p, C.c_void_p]),
    "mfs_point_strengths": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "mfs_neighbour_sum": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Lattice), C.c_int32, C.c_int32,
                                    C.c_void_p, _cp, C.c_int32, _dp, C.c_int32, C.c_int32,
                                    C.c_void_p, C.c_void_p]),
    "mfs_field_interior": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, _dp,
                                     C.c_int32, C.c_void_p, C.c_void_p]),
    "mfs_field_free": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, _dp,
                                 C.c_int32, C.c_void_p, C.c_void_p]),
    "mfs_server_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(Lattice),
                                    C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]),
    "mfs_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Wave), C.POINTER(C.c_uint64)]),
    "mfs_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Result), _dp]),
    "mfs_server_stats": (C.c_int, [C.c_void_p, _ip, _ip, _ip, _ip]),
    "mfs_server_destroy": (None, [C.c_void_p]),
    "mfs_solve_incident": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(Lattice),
                                     C.c_int32, C.POINTER(Wave), C.c_double, C.c_int32, C.c_double,
                                     _dp, C.c_int32, C.c_int32, C.POINTER(Result),
                                     C.POINTER(SolveTiming)]),
}


def lib():
    """Load libmfs.so (raises RuntimeError if it has not been built).

    PyTorch is imported first: its ROCm build brings its own HIP runtime
    (libamdhip64.so.7), and a process must hold one HIP runtime only (two
    copies cannot both open the GPU), so libmfs's dependency on
    libamdhip64.so.7 has to resolve to the copy torch has already loaded."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1506_05083_amd.build`")
        import torch  # noqa: F401  (loads torch's HIP runtime before libmfs)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class MfsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libmfs status {status}: {msg}")
        self.status = status


def _check(st: int):
    if st != MFS_OK:
        raise MfsError(st, lib().mfs_last_error().decode())


def _ptr(a: np.ndarray, typ=_dp):
    return a.ctypes.data_as(typ)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t):
    import torch
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.complex128, "need contiguous cuda complex128"
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ API

def polar_geometry(a: float, eps: float, j: int, M: int, N: int, tau: float, colloc: str = "mid"):
    """Host geometry of a polar body (the library's own implementation)."""
    spec = PolarSpec(a, eps, j, 1 if colloc == "gauss" else 0, M, N, tau)
    out = {k: np.zeros(M) for k in ("rho", "z", "nrho", "nz")}
    out.update({k: np.zeros(N) for k in ("srho", "sz")})
    _check(lib().mfs_polar_geometry(C.byref(spec), _ptr(out["rho"]), _ptr(out["z"]), _ptr(out["nrho"]),
                                    _ptr(out["nz"]), _ptr(out["srho"]), _ptr(out["sz"])))
    return out


def cup_geometry(outer: float, half: float, b: float, M: int, N: int, tau: float, colloc: str = "mid"):
    """Host geometry of the cup of Fig. 1(c) (the library's own implementation)."""
    spec = CupSpec(outer, half, b, 1 if colloc == "gauss" else 0, M, N, tau)
    out = {k: np.zeros(M) for k in ("rho", "z", "nrho", "nz")}
    out.update({k: np.zeros(N) for k in ("srho", "sz")})
    _check(lib().mfs_cup_geometry(C.byref(spec), _ptr(out["rho"]), _ptr(out["z"]), _ptr(out["nrho"]),
                                  _ptr(out["nz"]), _ptr(out["srho"]), _ptr(out["sz"])))
    return out


def body_geometry(shape, M: int, N: int, tau: float, colloc: str = "mid"):
    """Host geometry for a shape description with fields (a, eps, j) (polar)
    or (outer, half, b) (cup)."""
    if hasattr(shape, "outer"):
        return cup_geometry(shape.outer, shape.half, shape.b, M, N, tau, colloc)
    return polar_geometry(shape.a, shape.eps, shape.j, M, N, tau, colloc)


def transmission_geometry(shape, M: int, N: int, tau: float, colloc: str = "mid"):
    """Host geometry of a transmission body: the sources of the exterior
    field inside (tau), those of the interior field outside (-tau, Sec. 3.4)."""
    g = body_geometry(shape, M, N, tau, colloc)
    go = body_geometry(shape, M, N, -tau, colloc)
    g["srho_out"], g["sz_out"] = go["srho"], go["sz"]
    return g


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().mfs_create(device, C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mfs_destroy(self.h)
            self.h = None


def create(device: int = 0) -> Context:
    return Context(device)


def memory_stats(device: int = 0) -> dict:
    """Bytes held by the library's live device buffers, their peak since
    reset_memory_peak(), and idle bytes in the library's device cache."""
    a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _check(lib().mfs_memory_stats(device, C.byref(a), C.byref(b), C.byref(c)))
    return {"in_use": a.value, "peak": b.value, "cached": c.value}


def reset_memory_peak(device: int = 0) -> None:
    _check(lib().mfs_memory_reset_peak(device))


def release_cached_memory(device: int = 0) -> None:
    """Return the idle blocks of the library's device cache to the driver."""
    _check(lib().mfs_release_cached_memory(device))


@dataclass
class BodySpec:
    """km = 0: sound-hard; km > 0: transmission, geom then also holds the
    exterior sources srho_out, sz_out (transmission_geometry)."""
    M: int
    N: int
    P: int
    q: int
    k: float
    geom: dict
    km: float = 0.0

    @property
    def rows(self) -> int:
        """Rows of one mode's system: M, or 2M for transmission."""
        return 2 * self.M if self.km > 0 else self.M

    @property
    def cols(self) -> int:
        """Columns of one mode's system: N, or 2N for transmission."""
        return 2 * self.N if self.km > 0 else self.N


class Operator:
    def __init__(self, ctx: Context, bodies: Sequence[BodySpec]):
        import torch
        self.ctx = ctx
        self.bodies = list(bodies)
        keep = []
        arr = (Body * len(bodies))()
        for i, b in enumerate(bodies):
            g = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in b.geom.items()}
            keep.append(g)
            tr = b.km > 0
            arr[i] = Body(b.M, b.N, b.P, b.q, b.k, _ptr(g["rho"]), _ptr(g["z"]), _ptr(g["nrho"]),
                          _ptr(g["nz"]), _ptr(g["srho"]), _ptr(g["sz"]), float(b.km),
                          _ptr(g["srho_out"]) if tr else None, _ptr(g["sz_out"]) if tr else None)
        torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib().mfs_build_operator(ctx.h, arr, len(bodies), _stream(), C.byref(h)))
        self.h = h
        self.ranks = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mfs_destroy_op(self.h)
            self.h = None

    def blocks(self, body: int = 0):
        import torch
        b = self.bodies[body]
        out = torch.empty((b.P // 2 + 1, b.cols, b.rows), dtype=torch.complex128, device="cuda")
        _check(lib().mfs_op_blocks(self.h, body, _dev(out), _stream()))
        torch.cuda.synchronize()
        return out

    def factor_modes(self, rel_cutoff: float = 1e-10):
        import torch
        n = sum(b.P // 2 + 1 for b in self.bodies)
        r = np.zeros(n, dtype=np.int32)
        torch.cuda.synchronize()
        _check(lib().mfs_factor_modes(self.h, rel_cutoff, _ptr(r, _ip)))
        self.ranks = r
        return r

    def set_near_field_budget(self, max_bytes: int):
        """Device-memory bound of the dense near field of later solves (0: on the fly)."""
        _check(lib().mfs_set_near_field_budget(self.h, int(max_bytes)))

    def timing(self) -> dict:
        """Fill, QR and truncation stage times (ms, HIP events)."""
        ms = np.zeros(3)
        _check(lib().mfs_op_timing(self.h, _ptr(ms)))
        return dict(fill=ms[0], qr=ms[1], svd=ms[2])

    def singular_values(self, body: int = 0) -> np.ndarray:
        b = self.bodies[body]
        out = np.zeros((b.P // 2 + 1, b.cols))
        _check(lib().mfs_op_singular_values(self.h, body, _ptr(out)))
        return out


def build_operator(ctx: Context, bodies: Sequence[BodySpec]) -> Operator:
    return Operator(ctx, bodies)


def factor_modes(op: Operator, rel_cutoff: float = 1e-10):
    return op.factor_modes(rel_cutoff)


def apply_solution_op(op: Operator, x, body: int = 0, in_layout: int = 0, out_layout: int = 0):
    """c = A'^+ x per mode.  x: cuda complex128 [nrhs][P][M] modes (in_layout
    LAYOUT_MODES) or [nrhs][M][P] angle samples (LAYOUT_ANGLE); returns
    [nrhs][P][N] modes (LAYOUT_MODES) or point strengths (LAYOUT_POINTS)."""
    import torch
    b = op.bodies[body]
    x = x.contiguous()
    ncol = b.cols if out_layout == LAYOUT_MODES else b.N
    out = torch.empty((x.shape[0], b.P, ncol), dtype=torch.complex128, device=x.device)
    _check(lib().mfs_apply_solution_op(op.h, body, x.shape[0], _dev(x), in_layout, _dev(out), out_layout,
                                       _stream()))
    return out


def apply_solution_op_noalloc(op: Operator, x, out, body: int = 0, in_layout: int = 0, out_layout: int = 0):
    """apply_solution_op into a caller-provided `out`, with no allocation by
    the library (its work memory is a static device array shared by the
    calls on one GPU)."""
    _check(lib().mfs_apply_solution_op_noalloc(op.h, body, x.shape[0], _dev(x), in_layout, _dev(out), out_layout,
                                               _stream()))
    return out


def rhs_modes(op: Operator, kvecs: np.ndarray, body: int = 0):
    import torch
    b = op.bodies[body]
    kv = np.ascontiguousarray(np.atleast_2d(kvecs), dtype=np.float64)
    out = torch.empty((kv.shape[0], b.P, b.rows), dtype=torch.complex128, device="cuda")
    _check(lib().mfs_rhs_modes(op.h, body, kv.shape[0], _ptr(kv), _dev(out), _stream()))
    return out


def point_strengths(op: Operator, c, qs: int, body: int = 0):
    import torch
    b = op.bodies[body]
    c = c.contiguous()
    out = torch.empty((c.shape[0], qs, b.N), dtype=torch.complex128, device=c.device)
    _check(lib().mfs_point_strengths(op.h, body, c.shape[0], qs, _dev(c), _dev(out), _stream()))
    return out


def neighbour_sum(op: Operator, lattice: Lattice, sigma, ab: np.ndarray, target_set: int,
                  user: Optional[np.ndarray] = None, want: int = 0, qs: Optional[int] = None,
                  body: int = 0):
    """Phased 3x3 near sum of point sources sigma [nrhs][qs][N]; ab [nrhs][2] complex."""
    import torch
    b = op.bodies[body]
    sigma = sigma.contiguous()
    nrhs = sigma.shape[0]
    qs = sigma.shape[1] if qs is None else qs
    abc = np.ascontiguousarray(ab, dtype=np.complex128).reshape(nrhs, 2)
    ab_arr = (C128 * (2 * nrhs))(*[C128(v.real, v.imag) for v in abc.reshape(-1)])
    if target_set == TARGETS_SURFACE:
        nout = b.P * b.M
    elif target_set == TARGETS_WALLS:
        nout = 8 * lattice.M1 * lattice.M1
    else:
        nout = user.shape[0]
    uptr = None
    if user is not None:
        user = np.ascontiguousarray(user, dtype=np.float64)
        uptr = _ptr(user)
    out = torch.empty((nrhs, nout), dtype=torch.complex128, device=sigma.device)
    _check(lib().mfs_neighbour_sum(op.h, body, C.byref(lattice), nrhs, qs, _dev(sigma), ab_arr,
                                   target_set, uptr, 0 if user is None else user.shape[0], want,
                                   _dev(out), _stream()))
    return out


def field_interior(op: Operator, c, qs: int, targets: np.ndarray, body: int = 0):
    """Interior field u^- of a transmission body at targets inside it."""
    c = c.contiguous()
    t = np.ascontiguousarray(targets, dtype=np.float64)
    import torch
    out = torch.empty((c.shape[0], t.shape[0]), dtype=torch.complex128, device=c.device)
    _check(lib().mfs_field_interior(op.h, body, c.shape[0], qs, _dev(c), _ptr(t), t.shape[0], _dev(out),
                                    _stream()))
    return out


def field_free(op: Operator, c, qs: int, targets: np.ndarray, body: int = 0):
    import torch
    c = c.contiguous()
    t = np.ascontiguousarray(targets, dtype=np.float64)
    out = torch.empty((c.shape[0], t.shape[0]), dtype=torch.complex128, device=c.device)
    _check(lib().mfs_field_free(op.h, body, c.shape[0], qs, _dev(c), _ptr(t), t.shape[0], _dev(out),
                                _stream()))
    return out


@dataclass
class WaveResult:
    iters: int
    resid: float
    m: np.ndarray
    n: np.ndarray
    kz: np.ndarray
    a: np.ndarray
    b: np.ndarray
    field: np.ndarray
    eps_flux: float
    q_rank: int
    nq_cols: int


def solve_incident(ctx: Context, op: Operator, lattice: Lattice, waves: Sequence, tol: float = 1e-10,
                   maxit: int = 200, rel_cutoff: float = 1e-10, targets: Optional[np.ndarray] = None,
                   q_field: Optional[int] = None, body: int = 0, cap_orders: int = 4096,
                   timing: bool = False, allow_notconv: bool = False):
    """Periodic solve of up to 16 incident waves (each (theta, phi))."""
    import torch
    b = op.bodies[body]
    W = len(waves)
    wv = (Wave * W)(*[Wave(float(t), float(p)) for (t, p) in waves])
    nt = 0 if targets is None else targets.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.float64)
    qf = q_field if q_field is not None else 2 * b.P
    keep = []
    res = (Result * W)()
    for w in range(W):
        arrs = dict(m=np.zeros(cap_orders, np.int32), n=np.zeros(cap_orders, np.int32),
                    kz=np.zeros(cap_orders, np.complex128), a=np.zeros(cap_orders, np.complex128),
                    b=np.zeros(cap_orders, np.complex128), field=np.zeros(max(nt, 1), np.complex128))
        keep.append(arrs)
        res[w].cap_orders = cap_orders
        res[w].m = _ptr(arrs["m"], _ip)
        res[w].n = _ptr(arrs["n"], _ip)
        for k in ("kz", "a", "b", "field"):
            setattr(res[w], k, arrs[k].ctypes.data_as(_cp))
    tm = SolveTiming()
    torch.cuda.synchronize()
    st = lib().mfs_solve_incident(ctx.h, op.h, body, C.byref(lattice), W, wv, tol, maxit, rel_cutoff,
                                  None if tg is None else _ptr(tg), nt, qf, res, C.byref(tm))
    if not (st == MFS_OK or (allow_notconv and st == MFS_ENOTCONV)):
        _check(st)
    out = []
    for w in range(W):
        r = res[w]
        n = r.norders
        a = keep[w]
        out.append(WaveResult(r.iters, r.resid, a["m"][:n].copy(), a["n"][:n].copy(), a["kz"][:n].copy(),
                              a["a"][:n].copy(), a["b"][:n].copy(), a["field"][:nt].copy(), r.eps_flux,
                              r.q_rank, r.nq_cols))
    if timing:
        return out, {k: getattr(tm, k) for k, _ in SolveTiming._fields_}
    return out


def _result_slot(cap_orders: int, nt: int):
    arrs = dict(m=np.zeros(cap_orders, np.int32), n=np.zeros(cap_orders, np.int32),
                kz=np.zeros(cap_orders, np.complex128), a=np.zeros(cap_orders, np.complex128),
                b=np.zeros(cap_orders, np.complex128), field=np.zeros(max(nt, 1), np.complex128))
    r = Result()
    r.cap_orders = cap_orders
    r.m = _ptr(arrs["m"], _ip)
    r.n = _ptr(arrs["n"], _ip)
    for k in ("kz", "a", "b", "field"):
        setattr(r, k, arrs[k].ctypes.data_as(_cp))
    return r, arrs


class Server:
    """Continuous-batching server of incident-wave solves on a factored operator
    (mfs_server_*): submit(theta, phi) -> ticket; poll(ticket) -> (WaveResult,
    latency ms, converged) or None while the request is in flight."""

    def __init__(self, ctx: Context, op: Operator, lattice: Lattice, slots: int = 8, admit_batch: int = 8,
                 queue_cap: int = 1 << 20, tol: float = 1e-10, maxit: int = 100, rel_cutoff: float = 1e-10,
                 targets: Optional[np.ndarray] = None, q_field: Optional[int] = None,
                 hbm_budget: int = 200 << 30, body: int = 0, cap_orders: int = 4096):
        import torch
        b = op.bodies[body]
        self.op, self.ctx, self.cap_orders = op, ctx, cap_orders
        self._tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.float64)
        self.nt = 0 if targets is None else self._tg.shape[0]
        cfg = ServerConfig(slots, admit_batch, queue_cap, tol, maxit, rel_cutoff,
                           None if self._tg is None else _ptr(self._tg), self.nt,
                           q_field if q_field is not None else 2 * b.P, int(hbm_budget))
        self._lat = lattice
        torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib().mfs_server_create(ctx.h, op.h, body, C.byref(lattice), C.byref(cfg), C.byref(h)))
        self.h = h

    def submit(self, theta: float, phi: float) -> Optional[int]:
        """Queue one wave; None if the queue is full."""
        t = C.c_uint64()
        st = lib().mfs_server_submit(self.h, C.byref(Wave(float(theta), float(phi))), C.byref(t))
        if st == MFS_EBUSY:
            return None
        _check(st)
        return int(t.value)

    def poll(self, ticket: int):
        r, arrs = _result_slot(self.cap_orders, self.nt)
        lat = C.c_double()
        st = lib().mfs_server_poll(self.h, ticket, C.byref(r), C.byref(lat))
        if st == MFS_EBUSY:
            return None
        if st not in (MFS_OK, MFS_ENOTCONV):
            _check(st)
        n = r.norders
        res = WaveResult(r.iters, r.resid, arrs["m"][:n].copy(), arrs["n"][:n].copy(), arrs["kz"][:n].copy(),
                         arrs["a"][:n].copy(), arrs["b"][:n].copy(), arrs["field"][:self.nt].copy(),
                         r.eps_flux, r.q_rank, r.nq_cols)
        return res, lat.value, st == MFS_OK

    def stats(self) -> dict:
        v = [np.zeros(1, np.int32) for _ in range(4)]
        _check(lib().mfs_server_stats(self.h, *[_ptr(x, _ip) for x in v]))
        return dict(pending=int(v[0][0]), admitting=int(v[1][0]), iterating=int(v[2][0]), finished=int(v[3][0]))

    def wait(self, ticket: int, timeout_s: float = 600.0, poll_s: float = 0.001):
        """Block (polling) until ticket finishes."""
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"ticket {ticket} not finished after {timeout_s} s")
            time.sleep(poll_s)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mfs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def lattice(ex, ey, z0, p, N0, M1) -> Lattice:
    return Lattice(ex, ey, z0, p, N0, M1)
