"""ctypes binding of ``libiilbm.so``: the same calls as ``include/ii_lbm.h``,
argument marshalling only.  Every step of the method runs in the library's
HIP kernels; there is no CPU fallback, and importing this module fails loudly
when the library has not been built.

PyTorch is used only to own device memory (the workspace) and to provide the
HIP stream the library enqueues on.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiilbm.so")

OK, EINVAL, EWORKSPACE, EDEVICE, EUNSTABLE, EGEOMETRY, ESTATE, ECAPACITY = 0, -1, -2, -3, -4, -5, -6, -7
F_RHO, F_UX, F_UY, F_P, F_DISTRIB = 1, 2, 4, 8, 16
OVERLAP_SERIAL, OVERLAP_FULL, OVERLAP_INTERP_FIRST = 0, 1, 2
DT_F32, DT_F64 = 0, 1


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double),
                ("collision", C.c_int32), ("mrt_s", C.c_double * 9), ("bc", C.c_int32 * 4),
                ("u_max", C.c_double), ("u_wall", C.c_double * 4), ("body_force", C.c_double * 2),
                ("interface_kind", C.c_int32), ("force_mode", C.c_int32), ("n_markers", C.c_int32),
                ("kappa", C.c_double), ("dX", C.c_double), ("center", C.c_double * 2),
                ("radius", C.c_double), ("storage", C.c_int32), ("fp16_log2_scale", C.c_int32),
                ("math", C.c_int32), ("f_normal", C.c_double), ("body_free", C.c_int32),
                ("rho_star", C.c_double), ("spring", C.c_double * 2), ("damping", C.c_double * 2),
                ("presc_amp", C.c_double * 2), ("presc_umax", C.c_double * 2),
                ("geometry", C.c_int32)]


class Link(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("dir", C.c_int32), ("sigma", C.c_int32),
                ("seg", C.c_int32), ("inst", C.c_int32), ("q", C.c_double),
                ("theta", C.c_double), ("jp", C.c_double)]


LINK_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("dir", "<i4"), ("sigma", "<i4"),
                       ("seg", "<i4"), ("inst", "<i4"), ("q", "<f8"), ("theta", "<f8"),
                       ("jp", "<f8")])


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("momentum", C.c_double * 2),
                ("area", C.c_double), ("force", C.c_double * 2), ("n_cut_links", C.c_int32),
                ("error_bits", C.c_int32), ("p_in", C.c_double), ("p_out", C.c_double),
                ("n_in", C.c_int64), ("n_out", C.c_int64)]


EXPORTS = [
    "ii_lbm_workspace_size", "ii_lbm_init", "ii_lbm_step", "ii_lbm_sync", "ii_lbm_markers",
    "ii_lbm_set_markers", "ii_lbm_fields", "ii_lbm_fields_noalloc", "ii_lbm_set_distrib",
    "ii_lbm_state_size",
    "ii_lbm_save_state", "ii_lbm_load_state", "ii_lbm_cutlinks", "ii_lbm_diag",
    "ii_lbm_set_timing", "ii_lbm_get_timing", "ii_lbm_sweep_bytes", "ii_lbm_set_graph",
    "ii_lbm_set_overlap", "ii_lbm_autotune", "ii_lbm_set_tile_blocks", "ii_lbm_get_schedule",
    "ii_lbm_destroy", "ii_lbm_strerror",
    "ii_lbm_set_isolation", "ii_lbm_instance_errors", "ii_lbm_body",
]

_lib = None


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2003_12186_amd.build` "
                          "(or __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that one runtime instead of pulling a
    # second copy from /opt/rocm into the process.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    v, i32, i64, sz, d = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    PP = C.POINTER(Problem)
    sig = {
        "ii_lbm_workspace_size": [PP, i32, C.POINTER(sz)],
        "ii_lbm_init": [PP, i32, C.POINTER(C.POINTER(C.c_double)), v, sz, v, C.POINTER(v)],
        "ii_lbm_step": [v, i64],
        "ii_lbm_sync": [v],
        "ii_lbm_markers": [v, i32, v, v, v],
        "ii_lbm_set_markers": [v, i32, v],
        "ii_lbm_fields": [v, i32, C.c_uint32, v, i32, i32],
        "ii_lbm_fields_noalloc": [v, i32, C.c_uint32, v, i32],
        "ii_lbm_set_distrib": [v, i32, v],
        "ii_lbm_state_size": [v, i32, C.POINTER(sz)],
        "ii_lbm_save_state": [v, i32, v, sz],
        "ii_lbm_load_state": [v, i32, v, sz],
        "ii_lbm_cutlinks": [v, i32, v, i32, C.POINTER(i32)],
        "ii_lbm_diag": [v, i32, C.POINTER(Diag)],
        "ii_lbm_set_timing": [v, i32],
        "ii_lbm_get_timing": [v, C.POINTER(d), C.POINTER(i64)],
        "ii_lbm_sweep_bytes": [v, i32, C.POINTER(d)],
        "ii_lbm_set_graph": [v, i32],
        "ii_lbm_set_isolation": [v, i32],
        "ii_lbm_instance_errors": [v, v, i32],
        "ii_lbm_body": [v, i32, v],
        "ii_lbm_set_overlap": [v, i32],
        "ii_lbm_autotune": [v, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(d)],
        "ii_lbm_set_tile_blocks": [v, i32],
        "ii_lbm_get_schedule": [v, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(d)],
        "ii_lbm_destroy": [v],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.ii_lbm_strerror.argtypes = [C.c_int]
    lib.ii_lbm_strerror.restype = C.c_char_p
    _lib = lib
    return lib


class IILBMError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = load().ii_lbm_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")


def check(code: int, where: str) -> None:
    if code != OK:
        raise IILBMError(code, where)


def make_problem(w) -> Problem:
    """C problem from a ``workloads.Problem``."""
    p = Problem()
    p.nx, p.ny, p.tau = int(w.nx), int(w.ny), float(w.tau)
    p.collision = int(w.collision)
    if w.mrt_s is not None:
        for a in range(9):
            p.mrt_s[a] = float(w.mrt_s[a])
    for s in range(4):
        p.bc[s] = int(w.bc[s])
        p.u_wall[s] = float(w.u_wall[s])
    p.u_max = float(w.u_max)
    p.body_force[0], p.body_force[1] = float(w.body_force[0]), float(w.body_force[1])
    p.interface_kind = int(w.interface)
    p.force_mode = int(w.force_mode)
    p.n_markers = int(w.n_markers)
    p.kappa, p.dX = float(w.kappa), float(w.dX)
    p.center[0], p.center[1] = float(w.center[0]), float(w.center[1])
    p.radius = float(w.radius)
    p.storage = int(w.storage)
    p.fp16_log2_scale = int(getattr(w, "fp16_log2_scale", 0))
    p.math = int(getattr(w, "math", 0))
    p.f_normal = float(getattr(w, "f_normal", 0.0))
    p.geometry = int(getattr(w, "geometry", 0))
    p.body_free = int(getattr(w, "body_free", 0))
    p.rho_star = float(getattr(w, "rho_star", 1.0))
    for a in range(2):
        p.spring[a] = float(getattr(w, "spring", (0.0, 0.0))[a])
        p.damping[a] = float(getattr(w, "damping", (0.0, 0.0))[a])
        p.presc_amp[a] = float(getattr(w, "presc_amp", (0.0, 0.0))[a])
        p.presc_umax[a] = float(getattr(w, "presc_umax", (0.0, 0.0))[a])
    return p


def workspace_size(problems: Sequence[Problem]) -> int:
    arr = (Problem * len(problems))(*problems)
    n = C.c_size_t()
    check(load().ii_lbm_workspace_size(arr, len(problems), C.byref(n)), "workspace_size")
    return n.value


class Sim:
    """A handle of the library with its torch-owned workspace and stream."""

    def __init__(self, problems: Sequence, X0: Sequence[Optional[np.ndarray]], device: str = "cuda:0",
                 stream=None):
        import torch

        lib = load()
        self.problems: List[Problem] = [p if isinstance(p, Problem) else make_problem(p) for p in problems]
        n = len(self.problems)
        self.n_inst = n
        arr = (Problem * n)(*self.problems)
        self._X0 = []
        ptrs = (C.POINTER(C.c_double) * n)()
        for j in range(n):
            x = np.zeros((1, 2)) if X0[j] is None else np.ascontiguousarray(X0[j], dtype=np.float64)
            self._X0.append(x)
            ptrs[j] = x.ctypes.data_as(C.POINTER(C.c_double))
        nbytes = workspace_size(self.problems)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        check(lib.ii_lbm_init(arr, n, ptrs, C.c_void_p(self.workspace.data_ptr()), nbytes,
                              C.c_void_p(self.stream.cuda_stream), C.byref(h)), "init")
        self.h = h

    # -- stepping ------------------------------------------------------------
    def step(self, n: int = 1) -> None:
        check(load().ii_lbm_step(self.h, int(n)), "step")

    def sync(self) -> None:
        check(load().ii_lbm_sync(self.h), "sync")

    # -- readout -------------------------------------------------------------
    def markers(self, inst: int = 0):
        N = self.problems[inst].n_markers
        X = np.zeros((N, 2)); U = np.zeros((N, 2)); G = np.zeros((N, 2))
        check(load().ii_lbm_markers(self.h, inst, X.ctypes.data, U.ctypes.data, G.ctypes.data), "markers")
        return X, U, G

    def set_markers(self, X: np.ndarray, inst: int = 0) -> None:
        X = np.ascontiguousarray(X, dtype=np.float64)
        check(load().ii_lbm_set_markers(self.h, inst, X.ctypes.data), "set_markers")

    def fields(self, what: int = F_RHO | F_UX | F_UY, inst: int = 0, dtype=np.float64) -> np.ndarray:
        p = self.problems[inst]
        planes = sum((what >> b) & 1 for b in range(4)) + (9 if what & F_DISTRIB else 0)
        out = np.zeros((planes, p.ny, p.nx), dtype=dtype)
        dt = DT_F64 if dtype == np.float64 else DT_F32
        check(load().ii_lbm_fields(self.h, inst, what, out.ctypes.data, dt, 0), "fields")
        return out

    def fields_noalloc(self, what: int = F_RHO | F_UX | F_UY, inst: int = 0,
                       dtype=np.float64) -> np.ndarray:
        """As fields(), staged through the library's static device array
        (no device allocation in the call)."""
        p = self.problems[inst]
        planes = sum((what >> b) & 1 for b in range(4)) + (9 if what & F_DISTRIB else 0)
        out = np.zeros((planes, p.ny, p.nx), dtype=dtype)
        dt = DT_F64 if dtype == np.float64 else DT_F32
        check(load().ii_lbm_fields_noalloc(self.h, inst, what, out.ctypes.data, dt),
              "fields_noalloc")
        return out

    def fields_device(self, what: int, out, inst: int = 0) -> None:
        """Write planes into a caller-owned torch CUDA tensor (float32 or float64)."""
        import torch
        dt = DT_F64 if out.dtype == torch.float64 else DT_F32
        check(load().ii_lbm_fields(self.h, inst, what, C.c_void_p(out.data_ptr()), dt, 1), "fields")

    def set_distrib(self, f: np.ndarray, inst: int = 0) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        p = self.problems[inst]
        assert f.shape == (9, p.ny, p.nx)
        check(load().ii_lbm_set_distrib(self.h, inst, f.ctypes.data), "set_distrib")

    def save_state(self, inst: int = 0) -> bytes:
        n = C.c_size_t()
        check(load().ii_lbm_state_size(self.h, inst, C.byref(n)), "state_size")
        buf = C.create_string_buffer(n.value)
        check(load().ii_lbm_save_state(self.h, inst, buf, n.value), "save_state")
        return buf.raw

    def load_state(self, blob: bytes, inst: int = 0) -> None:
        check(load().ii_lbm_load_state(self.h, inst, blob, len(blob)), "load_state")

    def cutlinks(self, inst: int = 0) -> np.ndarray:
        cnt = C.c_int32()
        check(load().ii_lbm_cutlinks(self.h, inst, None, 0, C.byref(cnt)), "cutlinks")
        out = np.zeros(max(cnt.value, 1), dtype=LINK_DTYPE)
        check(load().ii_lbm_cutlinks(self.h, inst, out.ctypes.data, len(out), C.byref(cnt)), "cutlinks")
        return out[:cnt.value].copy()

    def diag(self, inst: int = 0) -> dict:
        d = Diag()
        check(load().ii_lbm_diag(self.h, inst, C.byref(d)), "diag")
        return {"step": d.step, "mass": d.mass, "momentum": (d.momentum[0], d.momentum[1]),
                "area": d.area, "force": (d.force[0], d.force[1]), "n_cut_links": d.n_cut_links,
                "error_bits": d.error_bits, "p_in": d.p_in, "p_out": d.p_out,
                "n_in": d.n_in, "n_out": d.n_out}

    # -- timing --------------------------------------------------------------
    def set_timing(self, enable: bool) -> None:
        check(load().ii_lbm_set_timing(self.h, 1 if enable else 0), "set_timing")

    def get_timing(self):
        ms = C.c_double(); n = C.c_int64()
        check(load().ii_lbm_get_timing(self.h, C.byref(ms), C.byref(n)), "get_timing")
        return ms.value, n.value

    def set_graph(self, enable: bool, steps: int = 0) -> None:
        """HIP-graph replay on or off; steps: length of the longest graph
        (even, 0 = the library's default)."""
        check(load().ii_lbm_set_graph(self.h, (int(steps) if steps else 1) if enable else 0), "set_graph")

    def set_isolation(self, enable: bool) -> None:
        check(load().ii_lbm_set_isolation(self.h, 1 if enable else 0), "set_isolation")

    def instance_errors(self) -> np.ndarray:
        """Error bits of every instance (synchronises; 0 = healthy)."""
        out = np.zeros(self.n_inst, dtype=np.int32)
        check(load().ii_lbm_instance_errors(self.h, out.ctypes.data, self.n_inst), "instance_errors")
        return out

    def body(self, inst: int = 0) -> dict:
        """State of a moving rigid circle after the last step (synchronises)."""
        out = np.zeros(14)
        check(load().ii_lbm_body(self.h, inst, out.ctypes.data), "body")
        return {"c": out[0:2].copy(), "U": out[2:4].copy(), "theta": out[4], "W": out[5],
                "F": out[6:8].copy(), "T": out[8], "a": out[9:11].copy(), "wdot": out[11],
                "steps": int(out[12])}

    def set_overlap(self, mode: int) -> None:
        """Membrane step schedule (OVERLAP_SERIAL / _FULL / _INTERP_FIRST)."""
        check(load().ii_lbm_set_overlap(self.h, int(mode)), "set_overlap")

    def autotune(self, trials: int = 5):
        u = C.c_int32(); o = C.c_int32(); us = C.c_double()
        check(load().ii_lbm_autotune(self.h, int(trials), C.byref(u), C.byref(o), C.byref(us)), "autotune")
        out = {"unit": u.value, "order": o.value, "sweep_us": us.value}
        sch = self.schedule()
        out["tile_blocks_per_cu"] = sch["tile_blocks_per_cu"]
        out["step_us"] = sch["step_us"]
        return out

    def set_tile_blocks(self, per_cu: int) -> None:
        """Tile-pass blocks per CU of a batched handle (0: one per estimated tile)."""
        check(load().ii_lbm_set_tile_blocks(self.h, int(per_cu)), "set_tile_blocks")

    def schedule(self) -> dict:
        u = C.c_int32(); o = C.c_int32(); t = C.c_int32(); us = C.c_double()
        check(load().ii_lbm_get_schedule(self.h, C.byref(u), C.byref(o), C.byref(t), C.byref(us)),
              "get_schedule")
        return {"unit": u.value, "order": o.value, "tile_blocks_per_cu": t.value, "step_us": us.value}

    def sweep_bytes(self, inst: int = 0) -> float:
        b = C.c_double()
        check(load().ii_lbm_sweep_bytes(self.h, inst, C.byref(b)), "sweep_bytes")
        return b.value

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            load().ii_lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# The D3Q19 form (include/ii_lbm3.h).
# ---------------------------------------------------------------------------
class Problem3C(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("force_mode", C.c_int32),
                ("tau", C.c_double), ("body_force", C.c_double * 3), ("center", C.c_double * 3),
                ("radius", C.c_double), ("f_normal", C.c_double), ("n_markers", C.c_int32),
                ("collision", C.c_int32)]


EXPORTS3 = ["ii_lbm3_init", "ii_lbm3_step", "ii_lbm3_set_distrib", "ii_lbm3_fields",
            "ii_lbm3_set_timing", "ii_lbm3_get_timing", "ii_lbm3_sweep_bytes", "ii_lbm3_check_mesh",
            "ii_lbm3_set_mesh", "ii_lbm3_mesh_links", "ii_lbm3_set_membrane", "ii_lbm3_membrane",
            "ii_lbm3_set_rigid_surface", "ii_lbm3_surface_force", "ii_lbm3_set_free_sphere", "ii_lbm3_body",
            "ii_lbm3_destroy", "ii_lbm3_init_with"]

_ALLOC3 = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_RELEASE3 = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator3C(C.Structure):
    _fields_ = [("alloc", _ALLOC3), ("release", _RELEASE3), ("ctx", C.c_void_p)]


class TorchMemory:
    """Device memory of a D3Q19 handle taken from PyTorch's caching
    allocator: each buffer is a uint8 tensor held here until the library
    hands it back.  Argument marshalling only."""

    def __init__(self, device="cuda"):
        self.device = device
        self.live = {}
        self.c = Allocator3C(_ALLOC3(self._alloc), _RELEASE3(self._release), None)

    def _alloc(self, nbytes, ctx):
        try:
            import torch
            t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)
        except Exception:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _release(self, ptr, ctx):
        self.live.pop(ptr, None)

    def bytes_held(self) -> int:
        return sum(t.numel() for t in self.live.values())


def _lib3():
    lib = load()
    if not getattr(lib, "_iilbm3_sigs", False):
        v, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sigs = {
            "ii_lbm3_init": [C.POINTER(Problem3C), v, v, C.POINTER(v)],
            "ii_lbm3_step": [v, i64],
            "ii_lbm3_set_distrib": [v, v],
            "ii_lbm3_fields": [v, v],
            "ii_lbm3_set_timing": [v, i32],
            "ii_lbm3_get_timing": [v, C.POINTER(d), C.POINTER(i64)],
            "ii_lbm3_sweep_bytes": [v, C.POINTER(d)],
            "ii_lbm3_check_mesh": [C.POINTER(Problem3C), i32, v, i32, v],
            "ii_lbm3_set_mesh": [v, i32, v, i32, v, v, C.POINTER(i64)],
            "ii_lbm3_mesh_links": [v, i64, v, v, C.POINTER(i64)],
            "ii_lbm3_set_membrane": [v, i32, v, i32, v, d],
            "ii_lbm3_membrane": [v, v, v],
            "ii_lbm3_set_rigid_surface": [v, i32, v, i32, v],
            "ii_lbm3_surface_force": [v, v],
            "ii_lbm3_set_free_sphere": [v, i32, v, i32, v, v, d, d, v, v],
            "ii_lbm3_body": [v, v],
            "ii_lbm3_destroy": [v],
            "ii_lbm3_init_with": [C.POINTER(Problem3C), v, v, C.POINTER(Allocator3C), C.POINTER(v)],
        }
        for name, args in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
        lib._iilbm3_sigs = True
    return lib


def make_problem3(w) -> Problem3C:
    p = Problem3C()
    p.nx, p.ny, p.nz = int(w.nx), int(w.ny), int(w.nz)
    p.force_mode = int(w.force_mode)
    p.tau = float(w.tau)
    for a in range(3):
        p.body_force[a] = float(w.body_force[a])
        p.center[a] = float(w.center[a])
    p.radius, p.f_normal = float(w.radius), float(w.f_normal)
    p.n_markers = int(w.n_markers)
    p.collision = int(getattr(w, "collision", 0))
    return p


def _mesh3_args(X, tri, jump_p):
    X = np.ascontiguousarray(X, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    pv = np.ascontiguousarray(np.broadcast_to(np.asarray(jump_p, dtype=np.float64), (len(X),)))
    return X, tri, pv


def check_mesh3(problem, X, tri) -> int:
    """Host-only validation of a triangulated surface (no GPU); the return code."""
    p = problem if isinstance(problem, Problem3C) else make_problem3(problem)
    X, tri, _ = _mesh3_args(X, tri, 0.0)
    return int(_lib3().ii_lbm3_check_mesh(C.byref(p), len(X), X.ctypes.data, len(tri), tri.ctypes.data))


class Sim3:
    """A D3Q19 handle: a periodic box with an optional normal-force sphere.
    Its device memory comes from PyTorch's allocator (``torch_memory``, the
    default) or from the library's own hipMalloc."""

    def __init__(self, problem, X0=None, torch_memory: bool = True):
        self.p = problem if isinstance(problem, Problem3C) else make_problem3(problem)
        self.h = C.c_void_p()
        X = None if X0 is None else np.ascontiguousarray(X0, dtype=np.float64)
        self._X = X
        self.mem = TorchMemory() if torch_memory else None
        check(_lib3().ii_lbm3_init_with(C.byref(self.p), None if X is None else X.ctypes.data, None,
                                        C.byref(self.mem.c) if self.mem else None, C.byref(self.h)),
              "init3")

    def step(self, n: int) -> None:
        check(_lib3().ii_lbm3_step(self.h, int(n)), "step3")

    def set_distrib(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (19, self.p.nz, self.p.ny, self.p.nx)
        check(_lib3().ii_lbm3_set_distrib(self.h, f.ctypes.data), "set_distrib3")

    def fields(self) -> np.ndarray:
        out = np.zeros((4, self.p.nz, self.p.ny, self.p.nx))
        check(_lib3().ii_lbm3_fields(self.h, out.ctypes.data), "fields3")
        return out

    def set_timing(self, on: bool) -> None:
        check(_lib3().ii_lbm3_set_timing(self.h, 1 if on else 0), "set_timing3")

    def get_timing(self):
        ms = C.c_double(); n = C.c_int64()
        check(_lib3().ii_lbm3_get_timing(self.h, C.byref(ms), C.byref(n)), "get_timing3")
        return ms.value, n.value

    def sweep_bytes(self) -> float:
        b = C.c_double()
        check(_lib3().ii_lbm3_sweep_bytes(self.h, C.byref(b)), "sweep_bytes3")
        return b.value

    def set_mesh(self, X, tri, jump_p) -> int:
        """Installs a fixed closed triangulated surface with vertex jump values;
        returns the number of cut-link records."""
        X, tri, pv = _mesh3_args(X, tri, jump_p)
        self._mesh = (X, tri, pv)
        n = C.c_int64()
        check(_lib3().ii_lbm3_set_mesh(self.h, len(X), X.ctypes.data, len(tri), tri.ctypes.data,
                                       pv.ctypes.data, C.byref(n)), "set_mesh3")
        return n.value

    def set_membrane(self, X, tri, gamma: float) -> None:
        """Installs a deformable triangulated membrane under surface tension."""
        X, tri, _ = _mesh3_args(X, tri, 0.0)
        self._memb_nv = len(X)
        check(_lib3().ii_lbm3_set_membrane(self.h, len(X), X.ctypes.data, len(tri), tri.ctypes.data,
                                           float(gamma)), "set_membrane3")

    def set_rigid_surface(self, X, tri) -> None:
        """Installs a fixed rigid triangulated surface held at rest by direct forcing."""
        X, tri, _ = _mesh3_args(X, tri, 0.0)
        self._memb_nv = len(X)
        check(_lib3().ii_lbm3_set_rigid_surface(self.h, len(X), X.ctypes.data, len(tri), tri.ctypes.data),
              "set_rigid_surface3")

    def set_free_sphere(self, X, tri, center, radius: float, rho_star: float, U0=(0.0, 0.0, 0.0),
                        W0=(0.0, 0.0, 0.0)) -> None:
        """Installs a free rigid sphere (triangulated) with the rigid-body update."""
        X, tri, _ = _mesh3_args(X, tri, 0.0)
        self._memb_nv = len(X)
        c, u, w = (np.ascontiguousarray(v, dtype=np.float64) for v in (center, U0, W0))
        self._body_args = (c, u, w)
        check(_lib3().ii_lbm3_set_free_sphere(self.h, len(X), X.ctypes.data, len(tri), tri.ctypes.data,
                                              c.ctypes.data, float(radius), float(rho_star), u.ctypes.data,
                                              w.ctypes.data), "set_free_sphere3")

    def body(self) -> np.ndarray:
        """c, U, a, W, wdot, U^{n-1}, W^{n-1}, F, T (27 doubles)."""
        out = np.zeros(27)
        check(_lib3().ii_lbm3_body(self.h, out.ctypes.data), "body3")
        return out

    def surface_force(self) -> np.ndarray:
        F = np.zeros(3)
        check(_lib3().ii_lbm3_surface_force(self.h, F.ctypes.data), "surface_force3")
        return F

    def membrane(self):
        """The membrane's vertices and the last step's vertex velocities."""
        X = np.zeros((self._memb_nv, 3))
        U = np.zeros((self._memb_nv, 3))
        check(_lib3().ii_lbm3_membrane(self.h, X.ctypes.data, U.ctypes.data), "membrane3")
        return X, U

    def mesh_links(self) -> dict:
        n = C.c_int64()
        rc = _lib3().ii_lbm3_mesh_links(self.h, 0, None, None, C.byref(n))   # the count
        if rc not in (OK, ECAPACITY):
            check(rc, "mesh_links3")
        rec = np.zeros((max(n.value, 1), 6), np.int32)
        jp = np.zeros(max(n.value, 1))
        check(_lib3().ii_lbm3_mesh_links(self.h, n.value, rec.ctypes.data, jp.ctypes.data, C.byref(n)),
              "mesh_links3")
        r, jp = rec[:n.value], jp[:n.value]
        return {"x": r[:, 0], "y": r[:, 1], "z": r[:, 2], "dir": r[:, 3], "sigma": r[:, 4], "tri": r[:, 5],
                "jp": jp}

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            _lib3().ii_lbm3_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
