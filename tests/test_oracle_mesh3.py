"""Pins of the oracle's triangulated-surface jumps in D3Q19 (reading R29), no
GPU: the cut-link set against the inside/outside classification of the
endpoints (half-open box rule where links graze faces, edges and vertices;
winding numbers on a geodesic sphere), the barycentric [[p]] against a linear
field evaluated at the independently computed crossing point, the step's mass
and momentum budget, and the exact state of the normal-force sphere as a
fixed point.
"""
import numpy as np
import pytest

from oracle import d3q19 as O3
from paper_2003_12186_amd import workloads as W


def _box(n=16):
    return O3.make_problem(W.Problem3(nx=n, ny=n + 1, nz=n + 2, tau=0.8))


def _link_set(L):
    return {(int(x), int(y), int(z), int(i)) for x, y, z, i in zip(L["x"], L["y"], L["z"], L["dir"])}


def _net(L):
    """Sum of sigma per link and the records of each link."""
    net, recs = {}, {}
    for k, (x, y, z, i, s, jp) in enumerate(zip(L["x"], L["y"], L["z"], L["dir"], L["sigma"], L["jp"])):
        key = (int(x), int(y), int(z), int(i))
        net[key] = net.get(key, 0) + int(s)
        recs.setdefault(key, []).append((int(s), float(jp)))
    return net, recs


def _expected(p, inside):
    """Every link P -> P + e_i whose ends are classified differently, with
    sigma = +1 when P is inside."""
    ex, ey, ez, _ = O3.lattice()
    want = {}
    for z in range(1, p.nz - 1):
        for y in range(1, p.ny - 1):
            for x in range(1, p.nx - 1):
                for i in range(1, 19):
                    a, b = inside(x, y, z), inside(x + ex[i], y + ey[i], z + ez[i])
                    if a != b:
                        want[(x, y, z, i)] = 1 if a else -1
    return want


@pytest.mark.parametrize("m", [1, 3])
def test_box_links_follow_the_half_open_rule(m):
    # Integer vertices: links lie in faces, run along edges and pass through
    # vertices.  Translating the lattice by (e, e^2, e^3) makes the box's
    # inside exactly lo <= x < hi on each axis.  A perturbed diagonal link
    # whose ends lie on two faces can run through the box between them (in
    # through one face, out through the other): two records of opposite sigma.
    # The net sigma of every link is the classification of its ends, and each
    # record's [[p]] is the linear vertex field at its own crossing point.
    lo, hi = 4, 10
    X, tri = W.box_mesh((lo,) * 3, (hi,) * 3, m)
    p = _box()
    pv = 1.0 + 0.1 * X[:, 0] - 0.05 * X[:, 2]
    L = O3.mesh_links(p, X, tri, pv)
    inside = lambda x, y, z: all(lo <= v < hi for v in (x, y, z))
    want = _expected(p, inside)
    net, recs = _net(L)
    assert {k: v for k, v in net.items() if v} == want
    clipped = [r for k, r in recs.items() if net[k] == 0]
    assert clipped and all(len(r) == 2 for r in clipped)
    assert all(len(r) == 1 for k, r in recs.items() if net[k])
    assert len(want) > 1000
    ex, ey, ez, _ = O3.lattice()
    P = np.stack([L["x"], L["y"], L["z"]], 1).astype(float)
    e = np.stack([ex[L["dir"]], ey[L["dir"]], ez[L["dir"]]], 1).astype(float)
    Xc = np.einsum("rk,rkj->rj", L["lam"], X[tri[L["tri"]]])
    s_ = np.einsum("ij,ij->i", Xc - P, e) / np.einsum("ij,ij->i", e, e)
    assert ((s_ >= -1e-15) & (s_ <= 1 + 1e-15)).all()
    assert np.abs(P + s_[:, None] * e - Xc).max() < 1e-13           # on the link
    assert np.abs(L["jp"] - (1.0 + 0.1 * Xc[:, 0] - 0.05 * Xc[:, 2])).max() < 1e-13


def test_sphere_links_match_winding_numbers():
    c, R = (8.27, 7.69, 9.13), 4.6
    X, tri = W.icosphere(c, R)
    p = _box(18)
    L = O3.mesh_links(p, X, tri, 1.0)
    z, y, x = np.mgrid[0:p.nz, 0:p.ny, 0:p.nx]
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    ins = W.mesh_inside(X, tri, pts).reshape(p.nz, p.ny, p.nx)
    want = _expected(p, lambda a, b, cc: bool(ins[cc, b, a]))
    net, recs = _net(L)
    assert {k: v for k, v in net.items() if v} == want
    # a link that grazes the polyhedron runs in and out through two faces
    assert all(len(r) == 1 for k, r in recs.items() if net[k])
    assert all(len(r) == 2 for k, r in recs.items() if not net[k])
    assert len(want) > 2000


def test_barycentric_jump_of_a_linear_field():
    # [[p]] linear in space at the vertices is the same linear function at the
    # crossing point, found here as the intersection of the link's line with
    # the triangle's plane.
    c, R = (8.27, 7.69, 9.13), 4.6
    X, tri = W.icosphere(c, R)
    a, b0 = np.array([0.3, -0.7, 0.45]), 0.2
    p = _box(18)
    L = O3.mesh_links(p, X, tri, X @ a + b0)
    ex, ey, ez, _ = O3.lattice()
    P = np.stack([L["x"], L["y"], L["z"]], 1).astype(float)
    e = np.stack([ex[L["dir"]], ey[L["dir"]], ez[L["dir"]]], 1).astype(float)
    A, B, Cc = (X[tri[L["tri"], k]] for k in range(3))
    n = np.cross(B - A, Cc - A)
    t = np.einsum("ij,ij->i", n, A - P) / np.einsum("ij,ij->i", n, e)
    assert ((t >= 0) & (t <= 1)).all()
    Xc = P + t[:, None] * e
    assert np.abs(L["jp"] - (Xc @ a + b0)).max() < 1e-12
    lam = L["lam"]
    assert np.abs(lam.sum(1) - 1).max() < 1e-14 and (lam >= 0).all()
    assert np.abs(lam[:, 0:1] * A + lam[:, 1:2] * B + lam[:, 2:3] * Cc - Xc).max() < 1e-12


def test_mesh_step_mass_and_momentum_budget():
    c, R = (8.27, 7.69, 9.13), 4.6
    X, tri = W.icosphere(c, R)
    p = _box(18)
    pv = 2e-3 * (1.0 + 0.3 * np.sin(X[:, 0]))
    ex, ey, ez, w = O3.lattice()
    f = np.ascontiguousarray(w[:, None, None, None]
                             * (1.0 + 1e-3 * W.seeded_noise((19, p.nz, p.ny, p.nx), 62, 0)))
    L = O3.mesh_links(p, X, tri, pv)
    coef = L["sigma"] * w[L["dir"]] * 3.0 * L["jp"]
    for _ in range(3):
        m0 = [a.sum() for a in O3.moments(p, f)]
        O3.run_mesh(p, f, X, tri, pv, 1)
        m1 = [a.sum() for a in O3.moments(p, f)]
        assert abs(m1[0] - m0[0]) < 1e-12
        for k, e in enumerate((ex, ey, ez)):
            assert m1[k + 1] - m0[k + 1] == pytest.approx((coef * e[L["dir"]]).sum(), abs=1e-13)


def test_exact_state_of_the_normal_force_mesh_is_fixed():
    # rho = 1 - 3 F inside the surface, u = 0: the uniform jump F on every cut
    # link carries each population across unchanged, so nothing moves.
    c, R, F = (9.27, 8.69, 10.13), 5.3, 4e-3
    X, tri = W.icosphere(c, R)
    p = O3.make_problem(W.Problem3(nx=20, ny=19, nz=21, tau=0.8))
    f = W.normal_force_mesh_state(W.Problem3(nx=20, ny=19, nz=21, tau=0.8), X, tri, F, c, R)
    f0 = f.copy()
    O3.run_mesh(p, f, X, tri, F, 6)
    assert np.abs(f - f0).max() < 1e-14
    # with the jump of the wrong sign the state is not kept
    g = f0.copy()
    O3.run_mesh(p, g, X, tri, -F, 1)
    assert np.abs(g - f0).max() > 1e-3


def test_star_shaped_inside_test_agrees_with_winding_numbers():
    # the fast classification the normal-force mesh state uses, against the
    # winding number, on every node near a geodesic sphere
    c, R = (10.27, 9.69, 11.13), 6.7
    X, tri = W.icosphere(c, R)
    z, y, x = np.mgrid[0:22, 0:21, 0:23]
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(float)
    r = np.linalg.norm(pts - np.array(c), axis=1)
    sel = pts[(r > R - 2) & (r < R + 1)]
    a = W.mesh_inside(X, tri, sel)
    b = W.star_mesh_inside(X, tri, c, sel)
    assert (a == b).all() and a.any() and (~a).any() and len(sel) > 500
