"""Seeded synthetic workloads for the D2Q9 immersed interface-lattice Boltzmann
method (II-LBM) of Qin, Kolahdouz & Griffith, arXiv:2003.12186.

This module only describes *inputs*: lattice sizes, relaxation times, spring
constants, boundary types and the initial Lagrangian marker positions.  It holds
none of the method's arithmetic (no equilibrium, collision, delta kernel, force
law or jump), so both the GPU path and the CPU oracle can be fed from it without
sharing any code of the method itself.  It imports nothing from the rest of the
package.

Random draws come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the state advances by the
golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state passed
through the two xor-shift-multiply rounds of that paper's mixing function.  A
draw u in [0, 1) takes the top 53 bits of an output.  Stream (config, instance)
starts from the state ``config * 2**32 + instance``.

Workloads (lattice units, dx = dt = 1, Sec. 2.2):
  * ``membrane_ellipse64``  64x64 periodic, SRT tau=0.8, ellipse 12 x 8 centred at
    (32, 32), 96 markers, spring constant 0.05 (the elastic-interface relaxation
    of Sec. 4.2 on a small periodic box).
  * ``cylinder_channel``  1024x512 channel, MRT, no-slip walls, parabolic inflow
    u_max=0.05, zero-gradient outflow, rigid circle D=32 at (256, 256) with 101
    direct-forcing markers (the fixed-cylinder problem of Sec. 4.3 in a channel).
    ``cylinder_channel(small=True)`` is the 128x64, D=4 copy the oracle runs in full.
  * ``membrane_seeded``  LxL periodic (L=4096 by default), SRT with tau drawn in
    [0.55, 1.5) and kappa log-uniform in [1e-3, 1e-1) from the seed; ellipse
    0.3L x 0.2L centred, N = L markers.
  * ``membrane_batch_uneven``  512 independent periodic membrane instances with side
    L in {64, 96, ..., 512}, aspect ratio in [1, 2), kappa log-uniform in
    [1e-3, 1e-1), tau in [0.55, 1.5) and N = round(2 x ellipse perimeter).

The marker spacing Delta X is measured on the equilibrium circle of equal area,
as the paper does for its elastic ellipse (Sec. 4.2): 2*pi*sqrt(a*b)/N for a
membrane, pi*D/N for the rigid circle.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple, List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# SplitMix64
# ---------------------------------------------------------------------------
_MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


class SplitMix64:
    """SplitMix64 stream; ``uniform()`` returns top-53-bit doubles in [0, 1).

    The generator is counter based: output j of a stream is the mixing function
    applied to ``start + (j + 1) * gamma``, which ``uniform_array`` evaluates for
    many j at once with wrapping uint64 arithmetic."""

    def __init__(self, config: int, instance: int = 0):
        self.start = ((int(config) << 32) + int(instance)) & _MASK64
        self.count = 0

    @staticmethod
    def _mix(z: int) -> int:
        z = ((z ^ (z >> 30)) * _MIX1) & _MASK64
        z = ((z ^ (z >> 27)) * _MIX2) & _MASK64
        return z ^ (z >> 31)

    def next_u64(self) -> int:
        self.count += 1
        return self._mix((self.start + self.count * _GAMMA) & _MASK64)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_array(self, n: int) -> np.ndarray:
        j = np.arange(self.count + 1, self.count + 1 + n, dtype=np.uint64)
        self.count += n
        with np.errstate(over="ignore"):
            z = np.uint64(self.start) + j * np.uint64(_GAMMA)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(_MIX1)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX2)
            z = z ^ (z >> np.uint64(31))
        return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def normal_array(self, n: int) -> np.ndarray:
        """n standard normals by Box-Muller on consecutive pairs of uniforms."""
        m = (n + 1) // 2
        u = self.uniform_array(2 * m).reshape(m, 2)
        r = np.sqrt(-2.0 * np.log(np.maximum(u[:, 0], 1e-300)))
        z = np.stack([r * np.cos(2.0 * np.pi * u[:, 1]), r * np.sin(2.0 * np.pi * u[:, 1])], axis=1)
        return z.reshape(-1)[:n]


# ---------------------------------------------------------------------------
# Problem description (plain data, mirrored field by field into the C structs)
# ---------------------------------------------------------------------------
SRT, MRT = 0, 1
BC_PERIODIC, BC_WALL, BC_INLET, BC_OUTLET, BC_INLET_UNIFORM = 0, 1, 2, 3, 4
IF_NONE, IF_MEMBRANE, IF_RIGID, IF_NORMAL = 0, 1, 2, 3
FORCE_II_LBM, FORCE_IB_LBM, FORCE_IB_LBM_GUO, FORCE_II_LBM_GUO = 0, 1, 2, 3
STORE_FP32, STORE_FP16 = 0, 1
GEOM_POLYGON, GEOM_SPLINE = 0, 1
MATH_FP32, MATH_FP64 = 0, 1

# D2Q9 MRT relaxation rates printed in Sec. 2.2.1 for the non-conserved moments
# (energy, energy square, two heat fluxes); the two stress rates are 1/tau.
PAPER_MRT_RATES = {"e": 1.63, "eps": 1.14, "q": 1.92}


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    tau: float
    collision: int = SRT
    mrt_s: Optional[Sequence[float]] = None  # 9 rates in moment order, None -> paper's
    bc: Sequence[int] = (BC_PERIODIC,) * 4   # x-low, x-high, y-low, y-high
    u_max: float = 0.0                       # inlet parabola peak
    u_wall: Sequence[float] = (0.0,) * 4     # tangential wall speed per side
    body_force: Sequence[float] = (0.0, 0.0)  # uniform Eulerian force density
    interface: int = IF_NONE
    force_mode: int = FORCE_II_LBM
    n_markers: int = 0
    kappa: float = 0.0
    dX: float = 0.0
    center: Sequence[float] = (0.0, 0.0)      # rigid circle centre
    radius: float = 0.0                       # rigid circle radius
    f_normal: float = 0.0                     # prescribed normal force per unit length (IF_NORMAL)
    geometry: int = 0                         # membrane: 0 polygon through the markers, 1 cubic spline
    body_free: int = 0                        # moving circle: bit 0 x, bit 1 y, bit 2 rotation free
    rho_star: float = 1.0                     # density ratio rho_s / rho_f of the body
    spring: Sequence[float] = (0.0, 0.0)      # k_s per axis, about the initial centre
    damping: Sequence[float] = (0.0, 0.0)     # c per axis
    presc_amp: Sequence[float] = (0.0, 0.0)   # prescribed harmonic motion: amplitude A ...
    presc_umax: Sequence[float] = (0.0, 0.0)  # ... and U_max per axis (0: not prescribed)
    storage: int = STORE_FP32
    math: int = MATH_FP32                     # collision arithmetic
    name: str = ""

    def rates(self) -> List[float]:
        """The nine MRT rates in the moment order (rho, e, eps, jx, qx, jy, qy, pxx, pxy)."""
        if self.mrt_s is not None:
            return [float(v) for v in self.mrt_s]
        r = PAPER_MRT_RATES
        st = 1.0 / self.tau
        return [0.0, r["e"], r["eps"], 0.0, r["q"], 0.0, r["q"], st, st]


@dataclasses.dataclass
class Workload:
    problem: Problem
    X0: np.ndarray           # (N, 2) float64 initial markers, CCW
    steps: int
    meta: dict


def ellipse_markers(cx: float, cy: float, a: float, b: float, n: int) -> np.ndarray:
    """n markers at equal parameter angle on the ellipse, counter-clockwise."""
    k = np.arange(n, dtype=np.float64)
    th = 2.0 * np.pi * k / n
    X = np.empty((n, 2), dtype=np.float64)
    X[:, 0] = cx + a * np.cos(th)
    X[:, 1] = cy + b * np.sin(th)
    return X


def circle_markers(cx: float, cy: float, r: float, n: int) -> np.ndarray:
    return ellipse_markers(cx, cy, r, r, n)


def membrane_dX(a: float, b: float, n: int) -> float:
    """Marker spacing on the equal-area equilibrium circle (Sec. 4.2)."""
    return 2.0 * math.pi * math.sqrt(a * b) / n


def ramanujan_perimeter(a: float, b: float) -> float:
    h = ((a - b) / (a + b)) ** 2
    return math.pi * (a + b) * (1.0 + 3.0 * h / (10.0 + math.sqrt(4.0 - 3.0 * h)))


# ---------------------------------------------------------------------------
# The workloads
# ---------------------------------------------------------------------------
def membrane_ellipse64(storage: int = STORE_FP32) -> Workload:
    nx = ny = 64
    a, b, n = 12.0, 8.0, 96
    X0 = ellipse_markers(32.0, 32.0, a, b, n)
    p = Problem(nx=nx, ny=ny, tau=0.8, collision=SRT, interface=IF_MEMBRANE,
                n_markers=n, kappa=0.05, dX=membrane_dX(a, b, n), storage=storage,
                name="membrane64")
    return Workload(p, X0, 2000, {"a": a, "b": b})


def cylinder_channel(re: float = 20.0, small: bool = False, storage: int = STORE_FP32) -> Workload:
    """Channel flow past a fixed circle; tau from Re = U_mean*D/nu with U_mean = 2/3 u_max."""
    if small:
        nx, ny, D, n, cx, cy = 128, 64, 4.0, 13, 32.0, 32.0
    else:
        nx, ny, D, n, cx, cy = 1024, 512, 32.0, 101, 256.0, 256.0
    u_max = 0.05
    u_mean = 2.0 * u_max / 3.0
    # The small copy keeps the full run's tau (its own Re is then D/32 of it).
    nu = u_mean * 32.0 / re
    tau = 0.5 + 3.0 * nu
    X0 = circle_markers(cx, cy, D / 2.0, n)
    p = Problem(nx=nx, ny=ny, tau=tau, collision=MRT,
                bc=(BC_INLET, BC_OUTLET, BC_WALL, BC_WALL), u_max=u_max,
                interface=IF_RIGID, n_markers=n, kappa=0.0,
                dX=math.pi * D / n, center=(cx, cy), radius=D / 2.0, storage=storage,
                name=f"cylinder{nx}x{ny}_D{int(D)}_Re{int(re)}")
    return Workload(p, X0, 20000, {"D": D, "re": re, "u_mean": u_mean})


def normal_force_circle_e1(D: int, force_mode: int = FORCE_II_LBM, storage: int = STORE_FP32) -> Workload:
    """Uniform normal force along a fixed circle (Sec. 4.1): the fluid domain
    [-D, D]^2 ((2D+1)^2 nodes) with outflow extrapolation on every side, the
    circle of diameter D at its centre, MRT, nu = 0.05, Re = 100, U = nu Re / D,
    a force F n per unit length with F = rho U^2, run to t = D/U.  The exact
    velocity is zero.  Markers at most 1 lu apart."""
    nu, re = 0.05, 100.0
    U = nu * re / D
    n = int(math.ceil(math.pi * D - 1e-9))
    X0 = circle_markers(float(D), float(D), D / 2.0, n)
    p = Problem(nx=2 * D + 1, ny=2 * D + 1, tau=0.5 + 3.0 * nu, collision=MRT,
                bc=(BC_OUTLET,) * 4, interface=IF_NORMAL, force_mode=force_mode, n_markers=n,
                dX=math.pi * D / n, center=(float(D), float(D)), radius=D / 2.0,
                f_normal=U * U, storage=storage, name=f"normal{D}_mode{force_mode}")
    return Workload(p, X0, int(round(D / U)), {"U": U, "D": D})


def normal_force_jump_state(w: Workload) -> np.ndarray:
    """The exact solution of the normal-force circle as an initial state: the
    fluid at rest with the force's pressure jump, rho = 1 - 3 F inside the
    circle's level set (p = rho / 3) and 1 outside, f_i = w_i rho."""
    p = w.problem
    wt = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    y, x = np.mgrid[0:p.ny, 0:p.nx]
    inside = (x - p.center[0]) ** 2 + (y - p.center[1]) ** 2 - p.radius ** 2 < 0.0
    rho = np.where(inside, 1.0 - 3.0 * p.f_normal, 1.0)
    return np.ascontiguousarray(wt[:, None, None] * rho[None])


def cylinder_uniform_e3(D: int, re: float, storage: int = STORE_FP32) -> Workload:
    """Uniform flow around a fixed circular cylinder (Sec. 4.3): domain
    [0, 40D] x [0, 20D], centre (10D, 10D), uniform inflow U on the left,
    outflow on the right, the sides moving with the stream (freestream); MRT
    with the viscosity the paper gives per Re (0.1, 0.05, 0.02, 0.01 for
    Re = 20, 40, 100, 200) and U = Re nu / D.  Markers at most 1 lu apart."""
    nu = {20.0: 0.1, 40.0: 0.05, 100.0: 0.02, 200.0: 0.01}[float(re)]
    U = re * nu / D
    R = D / 2.0
    n = int(math.ceil(math.pi * D - 1e-9))
    cx = cy = 10.0 * D
    p = Problem(nx=40 * D, ny=20 * D, tau=0.5 + 3.0 * nu, collision=MRT,
                bc=(BC_INLET_UNIFORM, BC_OUTLET, BC_WALL, BC_WALL), u_max=U,
                u_wall=(0.0, 0.0, U, U), interface=IF_RIGID, n_markers=n, dX=math.pi * D / n,
                center=(cx, cy), radius=R, storage=storage, name=f"cyl_uniform{D}_Re{re:g}")
    return Workload(p, circle_markers(cx, cy, R, n), 0, {"U": U, "D": D, "re": re, "nu": nu})


def viv_cylinder_e4(D: int, u_red: float, force_mode: int = FORCE_II_LBM, re: float = 100.0,
                    U: float = 0.05, storage: int = STORE_FP32) -> Workload:
    """Vortex-induced vibration of a circular cylinder free to move across a
    uniform stream (Sec. 4.5): domain [0, 40D] x [0, 20D], centre (10D, 10D),
    uniform inflow U on the left, outflow on the right, the sides moving with
    the stream; rho* = 8/pi, no damping, spring k = m (2 pi f_N)^2 with
    U_red = U / (f_N D); MRT with nu = U D / Re.  Markers at most 1 lu apart."""
    R = D / 2.0
    n = int(math.ceil(math.pi * D - 1e-9))
    rho_star = 8.0 / math.pi
    m = rho_star * math.pi * R * R
    fN = U / (u_red * D)
    cx, cy = 10.0 * D, 10.0 * D
    p = Problem(nx=40 * D, ny=20 * D, tau=0.5 + 3.0 * U * D / re, collision=MRT,
                bc=(BC_INLET_UNIFORM, BC_OUTLET, BC_WALL, BC_WALL), u_max=U,
                u_wall=(0.0, 0.0, U, U), interface=IF_RIGID, force_mode=force_mode, n_markers=n,
                dX=math.pi * D / n, center=(cx, cy), radius=R, body_free=2, rho_star=rho_star,
                spring=(0.0, m * (2.0 * math.pi * fN) ** 2), storage=storage,
                name=f"viv{D}_ured{u_red:g}")
    return Workload(p, circle_markers(cx, cy, R, n), 0, {"U": U, "D": D, "u_red": u_red, "re": re})


@dataclasses.dataclass
class Problem3:
    """A D3Q19 box with a fixed sphere carrying a uniform normal force."""
    nx: int
    ny: int
    nz: int
    tau: float
    center: Sequence[float] = (0.0, 0.0, 0.0)
    radius: float = 0.0
    f_normal: float = 0.0                      # F per unit area along the outward normal
    force_mode: int = FORCE_II_LBM             # FORCE_II_LBM (jumps) or FORCE_IB_LBM (spread)
    n_markers: int = 0                         # IB-LBM markers on the sphere
    body_force: Sequence[float] = (0.0, 0.0, 0.0)
    collision: int = SRT                       # SRT or MRT (reading R30)


def sphere_markers(c: Sequence[float], R: float, n: int) -> np.ndarray:
    """n points spread evenly over a sphere (the Fibonacci lattice)."""
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(1.0 - z * z)
    ph = np.pi * (3.0 - math.sqrt(5.0)) * k
    return np.stack([c[0] + R * r * np.cos(ph), c[1] + R * r * np.sin(ph), c[2] + R * z], 1)


def normal_force_sphere(D: int, force_mode: int = FORCE_II_LBM,
                        re: float = 100.0) -> Tuple[Problem3, np.ndarray, dict]:
    """The uniform normal force on a fixed sphere, the three-dimensional form of
    Sec. 4.1: a periodic box of side 2D + 2 with the sphere of diameter D at
    its centre, nu = 0.05, U = nu Re / D (Re = 100 in Sec. 4.1), F = U^2, run
    to t = D/U; IB-LBM markers about 1 lu apart."""
    nu = 0.05
    U = nu * re / D
    L = 2 * D + 2
    R = D / 2.0
    n = int(math.ceil(4.0 * math.pi * R * R))
    c = (L / 2.0, L / 2.0, L / 2.0)
    p = Problem3(nx=L, ny=L, nz=L, tau=0.5 + 3.0 * nu, center=c, radius=R, f_normal=U * U,
                 force_mode=force_mode, n_markers=n if force_mode == FORCE_IB_LBM else 0)
    X = sphere_markers(c, R, n) if force_mode == FORCE_IB_LBM else np.zeros((1, 3))
    return p, X, {"U": U, "D": D, "steps": int(round(D / U))}


def normal_force_sphere_state(p: Problem3) -> np.ndarray:
    """The exact solution as a state: at rest, rho = 1 - 3 F inside the sphere's
    level set and 1 outside, f_i = w_i rho."""
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    z, y, x = np.mgrid[0:p.nz, 0:p.ny, 0:p.nx]
    c = p.center
    inside = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 - p.radius ** 2 < 0.0
    rho = np.where(inside, 1.0 - 3.0 * p.f_normal, 1.0)
    return np.ascontiguousarray(w[:, None, None, None] * rho[None])


def snap_2m16(X) -> np.ndarray:
    """Coordinates rounded to multiples of 2^-16, where a triangulated surface's
    exact side tests take its vertices."""
    return np.rint(np.asarray(X, dtype=np.float64) * 65536.0) / 65536.0


def icosphere(c: Sequence[float], R: float, max_edge: float = 2.2) -> Tuple[np.ndarray, np.ndarray]:
    """A geodesic sphere: the icosahedron's faces split into four until every
    edge is at most max_edge, vertices pushed out to radius R and snapped to
    2^-16; triangles counter-clockwise seen from outside."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0), (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
         (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    T = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]

    def longest(V, T):
        return max(np.linalg.norm(V[a] - V[b]) for t in T for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])))

    while R * longest(V, T) > max_edge:
        mid = {}

        def m(a, b):
            k = (min(a, b), max(a, b))
            if k not in mid:
                v = V[a] + V[b]
                V.append(v / np.linalg.norm(v))
                mid[k] = len(V) - 1
            return mid[k]

        T = [u for a, b, cc in T for u in ((a, m(a, b), m(cc, a)), (b, m(b, cc), m(a, b)),
                                           (cc, m(cc, a), m(b, cc)), (m(a, b), m(b, cc), m(cc, a)))]
    X = snap_2m16(np.asarray(c, float) + R * np.array(V))
    tri = np.array(T, np.int32)
    n = np.cross(X[tri[:, 1]] - X[tri[:, 0]], X[tri[:, 2]] - X[tri[:, 0]])
    assert (np.einsum("ij,ij->i", n, X[tri].mean(1) - np.asarray(c, float)) > 0).all()
    return X, tri


def box_mesh(lo: Sequence[float], hi: Sequence[float], m: int) -> Tuple[np.ndarray, np.ndarray]:
    """The surface of the box [lo, hi] with each face cut into m x m rectangles
    and each rectangle into two triangles (diagonals alternating), counter-
    clockwise seen from outside."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    verts, index, tris = [], {}, []

    def vid(ijk):
        if ijk not in index:
            index[ijk] = len(verts)
            verts.append(lo + (hi - lo) * np.array(ijk, float) / m)
        return index[ijk]

    for ax in range(3):
        u, v = (ax + 1) % 3, (ax + 2) % 3
        for side in (0, m):
            for a in range(m):
                for b in range(m):
                    q = []
                    for da, db in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        k = [0, 0, 0]
                        k[ax], k[u], k[v] = side, a + da, b + db
                        q.append(vid(tuple(k)))
                    if side == 0:
                        q = q[::-1]
                    if (a + b) % 2:
                        tris += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
                    else:
                        tris += [(q[1], q[2], q[3]), (q[1], q[3], q[0])]
    return snap_2m16(np.array(verts)), np.array(tris, np.int32)


def mesh_inside(X, tri, pts, shift=(1e-7, 0.0, 0.0), chunk: int = 0) -> np.ndarray:
    """Whether points lie inside a closed triangulated surface: the winding
    number, the sum of the triangles' solid angles (Van Oosterom and Strackee)
    over 4 pi, above one half.  ``shift`` moves the points off the faces."""
    X = np.asarray(X, float)
    A, B, Cc = X[tri[:, 0]], X[tri[:, 1]], X[tri[:, 2]]
    pts = np.asarray(pts, float) + np.asarray(shift, float)
    out = np.zeros(len(pts), bool)
    chunk = chunk or max(1, 2_000_000 // len(tri))
    for s in range(0, len(pts), chunk):
        q = pts[s:s + chunk, None, :]
        a, b, c = A[None] - q, B[None] - q, Cc[None] - q
        la, lb, lc = (np.linalg.norm(v, axis=2) for v in (a, b, c))
        num = np.einsum("pti,pti->pt", a, np.cross(b, c))
        den = (la * lb * lc + np.einsum("pti,pti->pt", a, b) * lc + np.einsum("pti,pti->pt", a, c) * lb
               + np.einsum("pti,pti->pt", b, c) * la)
        out[s:s + chunk] = (2.0 * np.arctan2(num, den)).sum(1) / (4.0 * np.pi) > 0.5
    return out


def star_mesh_inside(X, tri, c, pts, shift=(1e-7, 0.0, 0.0)) -> np.ndarray:
    """Whether points lie inside a closed surface that is star-shaped about c
    (every ray from c leaves it once): the triangle whose cone from c holds the
    point's direction, then the side of that triangle's plane.  Candidate
    triangles come from a k-d tree of the triangles' directions; a point no
    candidate holds falls back to the winding number."""
    from scipy.spatial import cKDTree
    X = np.asarray(X, float)
    c = np.asarray(c, float)
    pts = np.asarray(pts, float) + np.asarray(shift, float)
    A, B, Cc = X[tri[:, 0]] - c, X[tri[:, 1]] - c, X[tri[:, 2]] - c
    dirs = A + B + Cc
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    d = pts - c
    dn = d / np.maximum(np.linalg.norm(d, axis=1), 1e-300)[:, None]
    _, cand = cKDTree(dirs).query(dn, k=min(12, len(tri)))
    out = np.zeros(len(pts), bool)
    done = np.zeros(len(pts), bool)
    n = np.cross(B - A, Cc - A)
    for j in range(cand.shape[1]):
        t = cand[:, j]
        hold = (~done & (np.einsum("ij,ij->i", np.cross(A[t], B[t]), d) >= 0)
                & (np.einsum("ij,ij->i", np.cross(B[t], Cc[t]), d) >= 0)
                & (np.einsum("ij,ij->i", np.cross(Cc[t], A[t]), d) >= 0))
        out[hold] = np.einsum("ij,ij->i", d[hold] - A[t[hold]], n[t[hold]]) < 0
        done |= hold
    if (~done).any():
        out[~done] = mesh_inside(X, tri, pts[~done] - np.asarray(shift, float), shift)
    return out


def ellipsoid_membrane(c: Sequence[float], radii: Sequence[float], max_edge: float = 2.2):
    """A geodesic sphere stretched to the ellipsoid with semi-axes radii about
    c (vertices snapped to 2^-16): the start of a relaxing drop."""
    X, tri = icosphere((0.0, 0.0, 0.0), 1.0, max_edge / max(radii))
    X = snap_2m16(np.asarray(c, float) + X * np.asarray(radii, float))
    return X, tri


def normal_force_mesh(D: int, re: float = 100.0, offset=(0.0, 0.0, 0.0)):
    """The normal-force sphere of Sec. 4.1 in three dimensions, with the sphere
    given as a triangulated surface (edges at most 2.2 lu) carrying [[p]] = F
    at every vertex; the same box, viscosity and F = U^2 as the level-set form."""
    p, _, meta = normal_force_sphere(D, FORCE_II_LBM, re)
    c = tuple(float(a) + float(o) for a, o in zip(p.center, offset))
    X, tri = icosphere(c, D / 2.0)
    F = p.f_normal
    p.radius, p.f_normal = 0.0, 0.0                 # the jumps come from the surface only
    meta = dict(meta, F=F, center=c, R=D / 2.0)
    return p, X, tri, np.full(len(X), F), meta


def normal_force_mesh_state(p: Problem3, X, tri, F: float, center, R: float) -> np.ndarray:
    """At rest, rho = 1 - 3 F inside the triangulated sphere (vertices on the
    sphere of centre c and radius R, faces within 1 lu inside it) and 1
    outside.  Nodes more than 1 lu inside the sphere are inside, nodes outside
    it (beyond the vertices' 2^-17 snap) are outside; the shell between is
    classified through the triangle in each node's direction."""
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    z, y, x = np.mgrid[0:p.nz, 0:p.ny, 0:p.nx]
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(float)
    r = np.linalg.norm(pts - np.asarray(center, float), axis=1)
    inside = r < R - 1.0
    shell = (r >= R - 1.0) & (r <= R + 1e-4)
    inside[shell] = star_mesh_inside(X, tri, center, pts[shell])
    rho = np.where(inside, 1.0 - 3.0 * F, 1.0).reshape(p.nz, p.ny, p.nx)
    return np.ascontiguousarray(w[:, None, None, None] * rho[None])


def elastic_membrane_e2(L: int, force_mode: int = FORCE_II_LBM, storage: int = STORE_FP32) -> Workload:
    """Thin elastic membrane of Sec. 4.2: ellipse a = 0.35 L, b = 0.25^2/0.35 L
    centred in a walled L x L box, MRT, kappa_bar = kappa/(U^2 L) = 0.1,
    nu = 0.02, Re = 100, U = nu Re / L; markers at most 2 lu apart (II-LBM) or
    1/3 lu apart (IB-LBM) on the equilibrium circle of radius L/4.  Runs to
    30 L/U."""
    nu, re, kbar = 0.02, 100.0, 0.1
    U = nu * re / L
    R = 0.25 * L
    spacing = 2.0 if force_mode in (FORCE_II_LBM, FORCE_II_LBM_GUO) else 1.0 / 3.0
    n = int(math.ceil(2.0 * math.pi * R / spacing - 1e-9))   # spacing at most the paper's
    X0 = ellipse_markers(L / 2.0, L / 2.0, 0.35 * L, 0.25 ** 2 / 0.35 * L, n)
    p = Problem(nx=L, ny=L, tau=0.5 + 3.0 * nu, collision=MRT, bc=(BC_WALL,) * 4,
                interface=IF_MEMBRANE, force_mode=force_mode, n_markers=n,
                kappa=kbar * U * U * L, dX=2.0 * math.pi * R / n, storage=storage,
                name=f"elastic{L}_mode{force_mode}")
    span = int(round(L / U))
    return Workload(p, X0, 30 * span, {"U": U, "span": span, "R": R})


def membrane_seeded(L: int = 4096, seed: int = 0, storage: int = STORE_FP32,
                n_markers: Optional[int] = None) -> Workload:
    rng = SplitMix64(3, seed)
    u0, u1 = rng.uniform(), rng.uniform()
    tau = 0.55 + 0.95 * u0
    kappa = 10.0 ** (-3.0 + 2.0 * u1)
    a, b = 0.3 * L, 0.2 * L
    n = L if n_markers is None else n_markers
    X0 = ellipse_markers(L / 2.0, L / 2.0, a, b, n)
    p = Problem(nx=L, ny=L, tau=tau, collision=SRT, interface=IF_MEMBRANE,
                n_markers=n, kappa=kappa, dX=membrane_dX(a, b, n), storage=storage,
                name=f"membrane{L}_seed{seed}")
    return Workload(p, X0, 5000, {"a": a, "b": b, "seed": seed})


def membrane_batch_uneven(n_inst: int = 512, first: int = 0) -> List[Workload]:
    out = []
    for i in range(first, first + n_inst):
        rng = SplitMix64(4, i)
        u0, u1, u2, u3 = rng.uniform(), rng.uniform(), rng.uniform(), rng.uniform()
        L = 64 + 32 * int(math.floor(15.0 * u0))
        ar = 1.0 + u1
        kappa = 10.0 ** (-3.0 + 2.0 * u2)
        tau = 0.55 + 0.95 * u3
        r_eq = math.sqrt(0.06) * L
        a, b = r_eq * math.sqrt(ar), r_eq / math.sqrt(ar)
        n = int(round(2.0 * ramanujan_perimeter(a, b)))
        X0 = ellipse_markers(L / 2.0, L / 2.0, a, b, n)
        p = Problem(nx=L, ny=L, tau=tau, collision=SRT, interface=IF_MEMBRANE,
                    n_markers=n, kappa=kappa, dX=membrane_dX(a, b, n),
                    name=f"batch{i}_L{L}")
        out.append(Workload(p, X0, 4000, {"a": a, "b": b, "ar": ar, "instance": i}))
    return out


def learned_pair_coarse_fine(seed: int, L: int = 256, n_markers: int = 512) -> Tuple[Workload, Workload]:
    """Coarse/fine membrane pair for the learned correction: the seeded
    membrane generator (same seed, so the same tau and kappa draw) at L x L and at
    2L x 2L, with the fine run in diffusive scaling: the same tau (so the same
    lattice viscosity), markers at twice the coordinates (same count), half
    the lattice stiffness, four fine steps per coarse step and half the
    lattice velocity.  Coarse node (i, j) sits on fine node (2i, 2j)."""
    c = membrane_seeded(L=L, seed=seed, n_markers=n_markers)
    f = membrane_seeded(L=2 * L, seed=seed, n_markers=n_markers)
    f.problem.kappa = c.problem.kappa / 2.0
    c.steps, f.steps = 2000, 8000
    c.meta["role"], f.meta["role"] = "coarse", "fine"
    return c, f


LEARNED_TRAIN_SEEDS = range(0, 2000)
LEARNED_HELDOUT_SEEDS = range(10000, 10200)


def seeded_noise(shape, config: int, instance: int) -> np.ndarray:
    """Seeded standard-normal array of the given shape (stream (config, instance)).
    Tests scale it into perturbed distribution fields; it carries no physics."""
    rng = SplitMix64(config, instance)
    n = int(np.prod(shape))
    return rng.normal_array(n).reshape(shape)
