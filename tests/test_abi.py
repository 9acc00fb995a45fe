"""CPU checks of the C ABI: the library loads, exports every call the header
declares, its structs match the header's layout, and host-side validation
rejects bad problems before touching a device (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2003_12186_amd import binding as B
from paper_2003_12186_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ii_lbm.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ii_lbm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_call():
    lib = B.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTS) == names


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ii_lbm.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(ii_lbm_problem),"
        " offsetof(ii_lbm_problem, storage), offsetof(ii_lbm_problem, radius),"
        " sizeof(ii_lbm_link), offsetof(ii_lbm_link, q), sizeof(ii_lbm_diag_t),"
        " offsetof(ii_lbm_diag_t, n_cut_links));return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(B.Problem), B.Problem.storage.offset, B.Problem.radius.offset,
            C.sizeof(B.Link), B.Link.q.offset, C.sizeof(B.Diag), B.Diag.n_cut_links.offset]
    assert got == want
    assert B.LINK_DTYPE.itemsize == C.sizeof(B.Link)


def _init_rc(prob, X0):
    lib = B.load()
    arr = (B.Problem * 1)(prob)
    x = np.ascontiguousarray(X0, dtype=np.float64)
    ptrs = (C.POINTER(C.c_double) * 1)(x.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    return lib.ii_lbm_init(arr, 1, ptrs, None, 0, None, C.byref(h))


def test_workspace_size_scales_with_lattice():
    a = B.workspace_size([B.make_problem(W.membrane_ellipse64().problem)])
    b = B.workspace_size([B.make_problem(W.membrane_seeded(L=256).problem)])
    c = B.workspace_size([B.make_problem(W.membrane_seeded(L=256, storage=W.STORE_FP16).problem)])
    assert 0 < a < b
    assert c < b                                  # half-precision lattice
    two = B.workspace_size([B.make_problem(W.membrane_ellipse64().problem)] * 2)
    assert two > a


@pytest.mark.parametrize("mutate,code", [
    (lambda p, X: setattr(p, "tau", 0.5), B.EINVAL),
    (lambda p, X: setattr(p, "nx", 4), B.EINVAL),
    (lambda p, X: p.bc.__setitem__(0, W.BC_WALL), B.EINVAL),        # one side periodic only
    (lambda p, X: setattr(p, "collision", 7), B.EINVAL),
    (lambda p, X: setattr(p, "dX", 3.0), B.EINVAL),
    (lambda p, X: setattr(p, "n_markers", 2), B.EINVAL),
    (lambda p, X: setattr(p, "storage", 5), B.EINVAL),
    (lambda p, X: setattr(p, "force_mode", 4), B.EINVAL),
    (lambda p, X: setattr(p, "geometry", 2), B.EINVAL),
    (lambda p, X: (setattr(p, "interface_kind", 2), setattr(p, "radius", 8.0),
                   setattr(p, "geometry", 1)), B.EINVAL),
    (lambda p, X: (setattr(p, "interface_kind", 3), setattr(p, "radius", 0.0)), B.EINVAL),
    (lambda p, X: (setattr(p, "interface_kind", 3), setattr(p, "radius", 8.0),
                   setattr(p, "f_normal", float("nan"))), B.EINVAL),
    (lambda p, X: setattr(p, "force_mode", -1), B.EINVAL),
    (lambda p, X: X.__setitem__(slice(None), X[::-1].copy()), B.EGEOMETRY),  # clockwise
    (lambda p, X: X.__setitem__((0, 0), 61.5), B.EGEOMETRY),          # near the edge / long chord
    (lambda p, X: X.__setitem__((0, 0), X[0, 0] + 4.5), B.EGEOMETRY),  # chords over 4 lu
    (lambda p, X: X.__setitem__((5, 1), np.nan), B.EINVAL),
])
def test_init_validation_rejects_before_device_access(mutate, code):
    w = W.membrane_ellipse64()
    p = B.make_problem(w.problem)
    X = w.X0.copy()
    mutate(p, X)
    assert _init_rc(p, X) == code


def test_strerror():
    lib = B.load()
    for code in range(-7, 1):
        assert len(lib.ii_lbm_strerror(code)) > 0


LEARNED_HEADER = os.path.join(ROOT, "include", "ii_learned.h")


def test_learned_header_calls_are_exported_and_sized():
    from paper_2003_12186_amd import learned as LN
    src = open(LEARNED_HEADER).read()
    names = sorted(set(re.findall(r"\b(ii_(?:cnn|lbm_learned)_[a-z_]+|ii_lbm_set_learned)\s*\(", src)))
    lib = LN.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(LN.EXPORTS) == names
    # host-only size queries
    assert lib.ii_cnn_packed_bytes() == 2 * (25088 + 3 * 9 * 2 * 512)
    assert lib.ii_cnn_save_bytes() == 2 * (22 * 22 + 20 * 20 + 18 * 18) * 32
    assert lib.ii_cnn_work_bytes(3) == 3 * (LN.NPARAM + 1) * 4 + 256
    assert C.sizeof(LN.Scales) == 20


def test_learned_parameter_layout_round_trips_with_the_oracle():
    import oracle.learned as OL
    from paper_2003_12186_amd import learned as LN
    Wt, b = OL.init_params(seed=3)
    assert sum(w.size for w in Wt) + sum(x.size for x in b) == LN.NPARAM
    p = LN.flatten_params(Wt, b)
    W2, b2 = LN.split_params(p)
    for l in range(4):
        assert np.array_equal(W2[l], Wt[l].astype(np.float32).astype(np.float64))
        assert W2[l].shape == Wt[l].shape and b2[l].shape == b[l].shape


def test_learned_calls_reject_null_arguments_without_a_device():
    from paper_2003_12186_amd import learned as LN
    lib = LN.lib()
    assert lib.ii_cnn_pack(None, None, None) == B.EINVAL
    assert lib.ii_cnn_forward(None, None, None, 1, None, None, None) == B.EINVAL
    assert lib.ii_lbm_learned_tiles(None, 16, None, None) == B.EINVAL
    assert lib.ii_lbm_learned_infer(None, None, None, None, 16, None, None, None, None, None) == B.EINVAL
    assert lib.ii_lbm_set_learned(None, None, None, None, 16, None, None, None, None, None) == B.EINVAL


HEADER3 = os.path.join(ROOT, "include", "ii_lbm3.h")


def test_d3q19_header_calls_are_exported_and_sized(tmp_path):
    src = open(HEADER3).read()
    names = sorted(set(re.findall(r"\b(ii_lbm3_[a-z_]+)\s*\(", src)))
    lib = B.load()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTS3) == names
    prog = tmp_path / "sz3.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ii_lbm3.h"\n'
        "int main(void){printf(\"%zu %zu %zu\\n\", sizeof(ii_lbm3_problem),"
        " offsetof(ii_lbm3_problem, radius), offsetof(ii_lbm3_problem, collision));return 0;}\n")
    exe = tmp_path / "sz3"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER3), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got == [C.sizeof(B.Problem3C), B.Problem3C.radius.offset, B.Problem3C.collision.offset]


@pytest.mark.parametrize("mutate,code", [
    (lambda p: setattr(p, "nx", 4), B.EINVAL),
    (lambda p: setattr(p, "tau", 0.5), B.EINVAL),
    (lambda p: setattr(p, "force_mode", 2), B.EINVAL),
    (lambda p: setattr(p, "collision", 2), B.EINVAL),
    (lambda p: p.center.__setitem__(0, 2.0), B.EGEOMETRY),      # sphere too near a side
])
def test_d3q19_init_validation_rejects_before_device_access(mutate, code):
    prob, _, _ = W.normal_force_sphere(16, W.FORCE_II_LBM, re=20.0)
    p = B.make_problem3(prob)
    mutate(p)
    h = C.c_void_p()
    assert B._lib3().ii_lbm3_init(C.byref(p), None, None, C.byref(h)) == code


def _mesh_problem():
    from paper_2003_12186_amd import workloads as W
    return W.Problem3(nx=24, ny=24, nz=24, tau=0.8)


def test_d3q19_mesh_validation_accepts_closed_surfaces():
    from paper_2003_12186_amd import workloads as W
    p = _mesh_problem()
    X, tri = W.icosphere((12.27, 11.69, 12.13), 6.0)
    assert B.check_mesh3(p, X, tri) == B.OK
    Xb, tb = W.box_mesh((5, 5, 5), (15, 15, 15), 4)
    assert B.check_mesh3(p, Xb, tb) == B.OK


def _bad_meshes():
    from paper_2003_12186_amd import workloads as W
    X, tri = W.icosphere((12.27, 11.69, 12.13), 6.0)
    cases = {}
    cases["open"] = (X, tri[1:], B.EGEOMETRY)                     # a triangle missing
    cases["flipped_one"] = (X, np.concatenate([tri[:1, ::-1], tri[1:]]), B.EGEOMETRY)
    cases["inside_out"] = (X, np.ascontiguousarray(tri[:, ::-1]), B.EGEOMETRY)
    Xs = X.copy(); Xs[:, 0] += 6.0
    cases["near_side"] = (Xs, tri, B.EGEOMETRY)                   # x beyond n - 3
    Xb, tb = W.box_mesh((5, 5, 5), (15, 15, 15), 2)               # edges 5 and 7.1 lu
    cases["long_edge"] = (Xb, tb, B.EGEOMETRY)
    t = tri.copy(); t[0, 1] = t[0, 0]
    cases["repeated_index"] = (X, t, B.EINVAL)
    t = tri.copy(); t[3, 2] = len(X)
    cases["index_range"] = (X, t, B.EINVAL)
    Xn = X.copy(); Xn[5, 1] = np.nan
    cases["nan"] = (Xn, tri, B.EINVAL)
    return cases


@pytest.mark.parametrize("case", ["open", "flipped_one", "inside_out", "near_side", "long_edge",
                                  "repeated_index", "index_range", "nan"])
def test_d3q19_mesh_validation_rejects(case):
    X, tri, code = _bad_meshes()[case]
    assert B.check_mesh3(_mesh_problem(), X, tri) == code


def test_d3q19_mesh_needs_the_jump_force_mode():
    from paper_2003_12186_amd import workloads as W
    p = _mesh_problem()
    p.force_mode = W.FORCE_IB_LBM
    X, tri = W.icosphere((12.27, 11.69, 12.13), 6.0)
    assert B.check_mesh3(p, X, tri) == B.EINVAL
