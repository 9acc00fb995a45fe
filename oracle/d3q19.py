"""ctypes binding of the FP64 CPU oracle of the D3Q19 step (``iilbm3_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the CPU-baseline leg of
``bench.py``.  The GPU library never imports, links or calls it.

Arrays: f[19][nz][ny][nx] float64 (C order), sphere markers X[N][3]; a
triangulated surface is vertices X[nv][3] float64, triangles tri[nt][3] int32
(counter-clockwise seen from outside) and vertex jump values pv[nv].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iilbm3_oracle.c")
_LIB = os.path.join(_HERE, "liboracle3.so")


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Problem3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("force_mode", C.c_int32),
                ("tau", C.c_double), ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double),
                ("radius", C.c_double), ("f_normal", C.c_double), ("n_markers", C.c_int32),
                ("collision", C.c_int32), ("body", C.c_double * 3), ("s", C.c_double * 19)]


def mrt_rates(tau: float):
    """Relaxation rates of the 19 moments (reading R30): 0 for the conserved
    rho and j, 1/tau for the viscous stresses (3pxx, pww, pxy, pyz, pxz),
    1.19 for e, 1.4 for eps, 3pixx and piww, 1.2 for the heat fluxes q,
    1.98 for the third-order m."""
    sv = 1.0 / tau
    return [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, sv, 1.4, sv, 1.4, sv, sv, sv, 1.98, 1.98, 1.98]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d = C.c_void_p
        P = C.POINTER(Problem3)
        sig = {
            "or3_lattice": (None, [d, d, d, d]),
            "or3_equilibrium": (None, [C.c_double] * 4 + [d]),
            "or3_moments": (None, [P, d, d, d, d, d]),
            "or3_peskin": (C.c_double, [C.c_double]),
            "or3_spread": (None, [P, d, d]),
            "or3_count_cut_links": (C.c_long, [P]),
            "or3_step": (C.c_int, [P, d, d]),
            "or3_run": (C.c_int, [P, d, d, C.c_int]),
            "or3_sizeof_problem": (C.c_int, []),
            "or3_basis": (None, [d]),
            "or3_membrane_forces": (C.c_int, [C.c_int, d, C.c_int, d, C.c_double, d, d, d, d, d]),
            "or3_interp": (None, [P, d, C.c_int, d, d]),
            "or3_run_membrane": (C.c_int, [P, d, C.c_int, d, C.c_int, d, C.c_double, C.c_int, d]),
            "or3_run_surface": (C.c_int, [P, d, C.c_int, d, C.c_int, d, C.c_int, C.c_double, C.c_int, d, d]),
            "or3_run_free_sphere": (C.c_int, [P, d, C.c_int, d, C.c_int, d, C.c_double, C.c_double, d, C.c_int,
                                              d, d]),
            "or3_mesh_links": (C.c_long, [P, C.c_int, d, C.c_int, d, d, d, d, C.c_long]),
            "or3_step_mesh": (C.c_int, [P, d, C.c_int, d, C.c_int, d, d]),
            "or3_run_mesh": (C.c_int, [P, d, C.c_int, d, C.c_int, d, d, C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
        assert _lib.or3_sizeof_problem() == C.sizeof(Problem3)
    return _lib


def _ptr(a):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def make_problem(w) -> Problem3:
    p = Problem3()
    p.nx, p.ny, p.nz = int(w.nx), int(w.ny), int(w.nz)
    p.force_mode = int(w.force_mode)
    p.tau = float(w.tau)
    p.cx, p.cy, p.cz = (float(v) for v in w.center)
    p.radius, p.f_normal = float(w.radius), float(w.f_normal)
    p.n_markers = int(w.n_markers)
    for a in range(3):
        p.body[a] = float(w.body_force[a])
    p.collision = int(getattr(w, "collision", 0))
    rates = getattr(w, "mrt_s", None) or mrt_rates(p.tau)
    for k in range(19):
        p.s[k] = float(rates[k])
    return p


def basis():
    """The 19 x 19 moment matrix, row k = moment k at the 19 velocities."""
    M = np.zeros((19, 19))
    lib().or3_basis(_ptr(M))
    return M


def lattice():
    ex = np.zeros(19, np.int32); ey = np.zeros(19, np.int32); ez = np.zeros(19, np.int32)
    w = np.zeros(19)
    lib().or3_lattice(_ptr(ex), _ptr(ey), _ptr(ez), _ptr(w))
    return ex, ey, ez, w


def equilibrium(rho, ux, uy, uz):
    out = np.zeros(19)
    lib().or3_equilibrium(float(rho), float(ux), float(uy), float(uz), _ptr(out))
    return out


def rest_state(p: Problem3, rho: float = 1.0) -> np.ndarray:
    feq = equilibrium(rho, 0.0, 0.0, 0.0)
    return np.ascontiguousarray(np.broadcast_to(feq[:, None, None, None], (19, p.nz, p.ny, p.nx))).copy()


def moments(p: Problem3, f):
    n = p.nx * p.ny * p.nz
    out = [np.zeros((p.nz, p.ny, p.nx)) for _ in range(4)]
    lib().or3_moments(C.byref(p), _ptr(f), *(_ptr(o) for o in out))
    return out


def peskin(r: float) -> float:
    return lib().or3_peskin(float(r))


def spread(p: Problem3, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    g = np.zeros((3, p.nz, p.ny, p.nx))
    lib().or3_spread(C.byref(p), _ptr(X), _ptr(g))
    return g


def count_cut_links(p: Problem3) -> int:
    return int(lib().or3_count_cut_links(C.byref(p)))


def run(p: Problem3, f, X, steps: int):
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (19, p.nz, p.ny, p.nx)
    Xp = np.ascontiguousarray(X if X is not None else np.zeros((1, 3)), dtype=np.float64)
    lib().or3_run(C.byref(p), _ptr(f), _ptr(Xp), int(steps))


def _mesh_args(X, tri, pv):
    X = np.ascontiguousarray(X, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    pv = np.ascontiguousarray(np.broadcast_to(np.asarray(pv, dtype=np.float64), (len(X),)))
    return X, tri, pv


def mesh_links(p: Problem3, X, tri, pv) -> dict:
    """Cut links of a closed triangulated surface (reading R29): sending node
    (x, y, z), direction, sigma (+1 from the inside), triangle, [[p]] and the
    barycentric weights of the crossing."""
    X, tri, pv = _mesh_args(X, tri, pv)
    cap = 64 * len(tri) + 4096
    rec = np.zeros((cap, 6), np.int32)
    val = np.zeros((cap, 4))
    n = lib().or3_mesh_links(C.byref(p), len(X), _ptr(X), len(tri), _ptr(tri), _ptr(pv), _ptr(rec),
                             _ptr(val), cap)
    assert n >= 0
    r, v = rec[:n], val[:n]
    return {"x": r[:, 0], "y": r[:, 1], "z": r[:, 2], "dir": r[:, 3], "sigma": r[:, 4], "tri": r[:, 5],
            "jp": v[:, 0], "lam": v[:, 1:4]}


def run_mesh(p: Problem3, f, X, tri, pv, steps: int):
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (19, p.nz, p.ny, p.nx)
    X, tri, pv = _mesh_args(X, tri, pv)
    assert lib().or3_run_mesh(C.byref(p), _ptr(f), len(X), _ptr(X), len(tri), _ptr(tri), _ptr(pv),
                              int(steps)) == 0


def membrane_forces(X, tri, gamma: float) -> dict:
    """Surface-tension forces of a triangulated membrane (reading R31): G
    (force on the fluid per vertex), outward normals n, vertex areas A,
    [[p]] = G.n/A and the tangential parts Gt."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    nv = len(X)
    G, n, Gt = (np.zeros((nv, 3)) for _ in range(3))
    A, jp = np.zeros(nv), np.zeros(nv)
    assert lib().or3_membrane_forces(nv, _ptr(X), len(tri), _ptr(tri), float(gamma), _ptr(G), _ptr(n),
                                     _ptr(A), _ptr(jp), _ptr(Gt)) == 0
    return {"G": G, "n": n, "A": A, "jp": jp, "Gt": Gt}


def interp(p: Problem3, f, X) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    U = np.zeros_like(X)
    lib().or3_interp(C.byref(p), _ptr(f), len(X), _ptr(X), _ptr(U))
    return U


def run_membrane(p: Problem3, f, X, tri, gamma: float, steps: int) -> np.ndarray:
    """Advances f and the vertices X (in place) by steps membrane steps, II-LBM
    or (p.force_mode IB-LBM) the whole force spread; returns the last step's
    vertex velocities."""
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (19, p.nz, p.ny, p.nx)
    assert X.dtype == np.float64 and X.flags["C_CONTIGUOUS"]
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    U = np.zeros_like(X)
    law = 2 if p.force_mode == 1 else 0
    q = Problem3.from_buffer_copy(p)
    q.force_mode = 0                    # the surface's own law decides; no sphere markers
    assert lib().or3_run_surface(C.byref(q), _ptr(f), len(X), _ptr(X), len(tri), _ptr(tri), law, float(gamma),
                                 int(steps), _ptr(U), None) == 0
    return U


def run_rigid_surface(p: Problem3, f, X, tri, steps: int):
    """Steps of a fixed rigid triangulated surface with direct forcing to rest
    (reading R32); returns the last step's vertex velocities and the force on
    the surface F = -sum G."""
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (19, p.nz, p.ny, p.nx)
    X = np.ascontiguousarray(X, dtype=np.float64).copy()
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    U = np.zeros_like(X)
    F = np.zeros(3)
    assert lib().or3_run_surface(C.byref(p), _ptr(f), len(X), _ptr(X), len(tri), _ptr(tri), 1, 0.0, int(steps),
                                 _ptr(U), _ptr(F)) == 0
    return U, F


def new_body3(center, U=(0.0, 0.0, 0.0), W=(0.0, 0.0, 0.0)) -> np.ndarray:
    """State of a free sphere: c, U, a, W, wdot, Uprev, Wprev (21 doubles);
    the first step takes Uprev = U and Wprev = W."""
    b = np.zeros(21)
    b[0:3], b[3:6], b[9:12] = center, U, W
    b[15:18], b[18:21] = U, W
    return b


def run_free_sphere(p: Problem3, f, X, tri, radius: float, rho_star: float, body, steps: int):
    """Steps of a free rigid sphere (reading R33); X and body advance in
    place; returns the last step's force and torque."""
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"] and f.shape == (19, p.nz, p.ny, p.nx)
    assert X.dtype == np.float64 and X.flags["C_CONTIGUOUS"] and body.flags["C_CONTIGUOUS"]
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    F, T = np.zeros(3), np.zeros(3)
    assert lib().or3_run_free_sphere(C.byref(p), _ptr(f), len(X), _ptr(X), len(tri), _ptr(tri), float(radius),
                                     float(rho_star), _ptr(body), int(steps), _ptr(F), _ptr(T)) == 0
    return F, T
