"""ctypes binding of the FP64 CPU oracle (``iilbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls it, and it never imports the GPU library.

Arrays: distribution fields f[9][ny][nx] float64 (C order), markers X[N][2].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iilbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SRT, MRT = 0, 1
PERIODIC, WALL, INLET, OUTLET, INLET_UNIFORM = 0, 1, 2, 3, 4
IF_NONE, IF_MEMBRANE, IF_RIGID, IF_NORMAL = 0, 1, 2, 3
II_LBM, IB_LBM, IB_LBM_GUO, II_LBM_GUO = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over lattice rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double),
                ("collision", C.c_int32), ("s", C.c_double * 9), ("bc", C.c_int32 * 4),
                ("u_max", C.c_double), ("u_wall", C.c_double * 4), ("body", C.c_double * 2),
                ("interface", C.c_int32), ("force_mode", C.c_int32), ("n_markers", C.c_int32),
                ("kappa", C.c_double), ("dX", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("radius", C.c_double), ("f_normal", C.c_double),
                ("ud", C.c_double * 3), ("theta", C.c_double), ("geometry", C.c_int32),
                ("pad2", C.c_int32)]


class BodyParams(C.Structure):
    _fields_ = [("free_dofs", C.c_int32), ("pad", C.c_int32), ("rho_star", C.c_double),
                ("spring", C.c_double * 2), ("damping", C.c_double * 2),
                ("presc_amp", C.c_double * 2), ("presc_umax", C.c_double * 2)]


class Body(C.Structure):
    _fields_ = [("c", C.c_double * 2), ("U", C.c_double * 2), ("a", C.c_double * 2),
                ("theta", C.c_double), ("W", C.c_double), ("wdot", C.c_double),
                ("Uprev", C.c_double * 2), ("Wprev", C.c_double), ("F", C.c_double * 2),
                ("T", C.c_double), ("c0", C.c_double * 2), ("n", C.c_int64)]


class Link(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("dir", C.c_int32), ("sigma", C.c_int32),
                ("seg", C.c_int32), ("pad", C.c_int32), ("q", C.c_double),
                ("theta", C.c_double), ("jp", C.c_double)]


LINK_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("dir", "<i4"), ("sigma", "<i4"),
                       ("seg", "<i4"), ("pad", "<i4"), ("q", "<f8"), ("theta", "<f8"),
                       ("jp", "<f8")])


class StepOut(C.Structure):
    _fields_ = [("U", C.c_void_p), ("G", C.c_void_p), ("nrm", C.c_void_p), ("J", C.c_void_p),
                ("jp", C.c_void_p), ("Gt", C.c_void_p), ("gx", C.c_void_p), ("gy", C.c_void_p),
                ("links", C.c_void_p), ("links_cap", C.c_int), ("n_links", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d = C.c_void_p
        P = C.POINTER(Problem)
        sig = {
            "or_d2q9": (None, [d, d, d]),
            "or_equilibrium": (None, [C.c_double, C.c_double, C.c_double, d]),
            "or_moments_node": (None, [d, d, d, d]),
            "or_moments": (None, [P, d, d, d, d]),
            "or_mrt_matrices": (None, [d, d]),
            "or_collide_node": (None, [P, d, C.c_double, C.c_double, d]),
            "or_guo_term": (None, [C.c_double, C.c_double, C.c_double, C.c_double, d]),
            "or_peskin_phi": (C.c_double, [C.c_double]),
            "or_interp": (None, [P, d, d, d, d]),
            "or_spread": (None, [P, d, d, d, d]),
            "or_marker_forces": (None, [P, d, d, d, d, d, d, d]),
            "or_cutlinks": (C.c_int, [P, d, d, d, C.c_int]),
            "or_cutlinks_bruteforce": (C.c_int, [P, d, d, C.c_int, C.c_int, C.c_int, C.c_int, d, C.c_int]),
            "or_node_inside": (C.c_int, [P, d, C.c_int, C.c_int]),
            "or_boundaries": (None, [P, d]),
            "or_step": (C.c_int, [P, d, d, C.POINTER(StepOut)]),
            "or_run": (C.c_int, [P, d, d, C.c_int, d]),
            "or_polygon_area": (C.c_double, [C.c_int, d]),
            "or_pressure_jump": (C.c_double, [P, d, d, C.c_double]),
            "or_sizeof_link": (C.c_int, []),
            "or_sizeof_problem": (C.c_int, []),
            "or_num_threads": (C.c_int, []),
            "or_set_num_threads": (None, [C.c_int]),
            "or_step_body": (C.c_int, [P, C.POINTER(BodyParams), C.POINTER(Body), d, d]),
            "or_spline": (None, [P, d, d]),
            "or_cutlinks_spline": (C.c_int, [P, d, d, d, C.c_int]),
            "or_sizeof_body": (C.c_int, []),
            "or_sizeof_body_params": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
        assert _lib.or_sizeof_link() == C.sizeof(Link) == LINK_DTYPE.itemsize
        assert _lib.or_sizeof_body() == C.sizeof(Body)
        assert _lib.or_sizeof_body_params() == C.sizeof(BodyParams)
        assert _lib.or_sizeof_problem() == C.sizeof(Problem)
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def make_problem(w) -> Problem:
    """Oracle problem from a ``workloads.Problem`` (or any object with the same fields)."""
    p = Problem()
    p.nx, p.ny, p.tau = int(w.nx), int(w.ny), float(w.tau)
    p.collision = int(w.collision)
    rates = w.rates() if hasattr(w, "rates") else [1.0 / w.tau] * 9
    for i in range(9):
        p.s[i] = float(rates[i])
    for i in range(4):
        p.bc[i] = int(w.bc[i])
        p.u_wall[i] = float(w.u_wall[i])
    p.u_max = float(w.u_max)
    p.body[0], p.body[1] = float(w.body_force[0]), float(w.body_force[1])
    p.interface = int(w.interface)
    p.force_mode = int(w.force_mode)
    p.n_markers = int(w.n_markers)
    p.kappa, p.dX = float(w.kappa), float(w.dX)
    p.cx, p.cy = float(w.center[0]), float(w.center[1])
    p.radius = float(w.radius)
    p.f_normal = float(getattr(w, "f_normal", 0.0))
    p.geometry = int(getattr(w, "geometry", 0))
    return p


# ---------------------------------------------------------------------------
# Thin numpy wrappers
# ---------------------------------------------------------------------------
def d2q9():
    ex = np.zeros(9, np.int32); ey = np.zeros(9, np.int32); w = np.zeros(9)
    lib().or_d2q9(_ptr(ex), _ptr(ey), _ptr(w))
    return ex, ey, w


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    lib().or_equilibrium(rho, ux, uy, _ptr(out))
    return out


def rest_state(p: Problem, rho: float = 1.0) -> np.ndarray:
    feq = equilibrium(rho, 0.0, 0.0)
    return np.ascontiguousarray(np.broadcast_to(feq[:, None, None], (9, p.ny, p.nx))).copy()


def moments(p: Problem, f: np.ndarray):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.zeros((p.ny, p.nx)); ux = np.zeros_like(rho); uy = np.zeros_like(rho)
    lib().or_moments(C.byref(p), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


def mrt_matrices():
    M = np.zeros((9, 9)); Mi = np.zeros((9, 9))
    lib().or_mrt_matrices(_ptr(M), _ptr(Mi))
    return M, Mi


def collide_node(p: Problem, f9, gx=0.0, gy=0.0):
    f9 = np.ascontiguousarray(f9, dtype=np.float64)
    out = np.zeros(9)
    lib().or_collide_node(C.byref(p), _ptr(f9), gx, gy, _ptr(out))
    return out


def guo_term(ux, uy, gx, gy):
    """G~_i of Guo's force term (without its relaxation factor)."""
    out = np.zeros(9)
    lib().or_guo_term(float(ux), float(uy), float(gx), float(gy), _ptr(out))
    return out


def peskin_phi(r: float) -> float:
    return lib().or_peskin_phi(float(r))


def interp(p: Problem, ux, uy, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    U = np.zeros_like(X)
    lib().or_interp(C.byref(p), _ptr(np.ascontiguousarray(ux)), _ptr(np.ascontiguousarray(uy)), _ptr(X), _ptr(U))
    return U


def spread(p: Problem, X, V):
    X = np.ascontiguousarray(X, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    gx = np.zeros((p.ny, p.nx)); gy = np.zeros((p.ny, p.nx))
    lib().or_spread(C.byref(p), _ptr(X), _ptr(V), _ptr(gx), _ptr(gy))
    return gx, gy


def marker_forces(p: Problem, X, U=None):
    X = np.ascontiguousarray(X, dtype=np.float64)
    U = np.zeros_like(X) if U is None else np.ascontiguousarray(U, dtype=np.float64)
    N = X.shape[0]
    G = np.zeros((N, 2)); n = np.zeros((N, 2)); J = np.zeros(N); jp = np.zeros(N); Gt = np.zeros((N, 2))
    lib().or_marker_forces(C.byref(p), _ptr(X), _ptr(U), _ptr(G), _ptr(n), _ptr(J), _ptr(jp), _ptr(Gt))
    return {"G": G, "n": n, "J": J, "jp": jp, "Gt": Gt}


def cutlinks(p: Problem, X, jp=None) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    N = X.shape[0]
    jp = np.zeros(N) if jp is None else np.ascontiguousarray(jp, dtype=np.float64)
    cap = 64 * N + 4096
    rec = np.zeros(cap, dtype=LINK_DTYPE)
    n = lib().or_cutlinks(C.byref(p), _ptr(X), _ptr(jp), _ptr(rec), cap)
    assert n <= cap
    return rec[:n].copy()


def spline_second_derivs(p: Problem, X) -> np.ndarray:
    """M_k of the periodic cubic spline through the markers (reading R27)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    M = np.zeros_like(X)
    lib().or_spline(C.byref(p), _ptr(X), _ptr(M))
    return M


def cutlinks_spline(p: Problem, X, G) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    cap = 64 * X.shape[0] + 4096
    rec = np.zeros(cap, dtype=LINK_DTYPE)
    n = lib().or_cutlinks_spline(C.byref(p), _ptr(X), _ptr(G), _ptr(rec), cap)
    assert n <= cap
    return rec[:n].copy()


def cutlinks_bruteforce(p: Problem, X, box, jp=None) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    N = X.shape[0]
    jp = np.zeros(N) if jp is None else np.ascontiguousarray(jp, dtype=np.float64)
    cap = 64 * N + 4096
    rec = np.zeros(cap, dtype=LINK_DTYPE)
    x0, x1, y0, y1 = box
    n = lib().or_cutlinks_bruteforce(C.byref(p), _ptr(X), _ptr(jp), x0, x1, y0, y1, _ptr(rec), cap)
    assert n <= cap
    return rec[:n].copy()


def node_inside(p: Problem, X, x: int, y: int) -> bool:
    X = np.ascontiguousarray(X, dtype=np.float64)
    return bool(lib().or_node_inside(C.byref(p), _ptr(X), int(x), int(y)))


def boundaries(p: Problem, f: np.ndarray) -> None:
    lib().or_boundaries(C.byref(p), _ptr(f))


def step(p: Problem, f: np.ndarray, X: np.ndarray, detail: bool = False):
    """One II-LBM step in place; with detail=True returns the step's marker
    quantities, the spread force planes and the cut-link records."""
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (9, p.ny, p.nx)
    N = max(int(p.n_markers), 1)
    Xp = X if X is not None else np.zeros((N, 2))
    o = StepOut()
    keep = {}
    if detail:
        for name, shape in (("U", (N, 2)), ("G", (N, 2)), ("nrm", (N, 2)), ("J", (N,)),
                            ("jp", (N,)), ("Gt", (N, 2)), ("gx", (p.ny, p.nx)), ("gy", (p.ny, p.nx))):
            keep[name] = np.zeros(shape)
            setattr(o, name, _ptr(keep[name]).value)
        cap = 64 * N + 4096
        keep["links"] = np.zeros(cap, dtype=LINK_DTYPE)
        o.links = _ptr(keep["links"]).value
        o.links_cap = cap
    rc = lib().or_step(C.byref(p), _ptr(f), _ptr(Xp), C.byref(o))
    if rc != 0:
        raise RuntimeError("oracle step: a cut link left the lattice")
    if detail:
        keep["links"] = keep["links"][:o.n_links].copy()
        return keep
    return None


def run(p: Problem, f: np.ndarray, X: np.ndarray, n_steps: int, force_hist: bool = False):
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (9, p.ny, p.nx)
    N = max(int(p.n_markers), 1)
    Xp = X if X is not None else np.zeros((N, 2))
    fh = np.zeros((n_steps, 2)) if force_hist else None
    rc = lib().or_run(C.byref(p), _ptr(f), _ptr(Xp), int(n_steps), _ptr(fh) if fh is not None else None)
    if rc != 0:
        raise RuntimeError("oracle run: a cut link left the lattice")
    return fh


def body_params(w) -> BodyParams:
    """Rigid-body parameters from a ``workloads.Problem``."""
    bp = BodyParams()
    bp.free_dofs = int(w.body_free)
    bp.rho_star = float(w.rho_star)
    for a in range(2):
        bp.spring[a], bp.damping[a] = float(w.spring[a]), float(w.damping[a])
        bp.presc_amp[a], bp.presc_umax[a] = float(w.presc_amp[a]), float(w.presc_umax[a])
    return bp


def new_body(p: Problem) -> Body:
    b = Body()
    b.c[0] = b.c0[0] = p.cx
    b.c[1] = b.c0[1] = p.cy
    return b


def run_body(p: Problem, bp: BodyParams, b: Body, f: np.ndarray, X: np.ndarray, n_steps: int):
    """Steps with a moving circle (Sec. 2.3); returns the per-step history
    [n, (cx, cy, Ux, Uy, theta, W, Fx, Fy, T)] after each step."""
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (9, p.ny, p.nx)
    hist = np.zeros((n_steps, 9))
    for s in range(n_steps):
        if lib().or_step_body(C.byref(p), C.byref(bp), C.byref(b), _ptr(f), _ptr(X)) != 0:
            raise RuntimeError("oracle run: a cut link left the lattice")
        hist[s] = (b.c[0], b.c[1], b.U[0], b.U[1], b.theta, b.W, b.F[0], b.F[1], b.T)
    return hist


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the OpenMP loops from now on (the default: every core)."""
    lib().or_set_num_threads(int(n))


def polygon_area(X) -> float:
    X = np.ascontiguousarray(X, dtype=np.float64)
    return lib().or_polygon_area(X.shape[0], _ptr(X))


def pressure_jump(p: Problem, rho, X, margin: float = 3.0) -> float:
    return lib().or_pressure_jump(C.byref(p), _ptr(np.ascontiguousarray(rho)),
                                  _ptr(np.ascontiguousarray(X, dtype=np.float64)), float(margin))
