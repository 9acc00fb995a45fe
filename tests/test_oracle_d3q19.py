"""Pins of the D3Q19 oracle (reading R28), no GPU: the lattice and its
equilibrium against the closed forms the quadrature fixes, conservation and
exact acceleration on a periodic box, the sphere's level-set cut links
against brute force, the three-dimensional delta's partition of unity, and
the normal-force sphere's exact state as a fixed point of II-LBM only.
"""
import itertools

import numpy as np
import pytest

from oracle import d3q19 as O3
from paper_2003_12186_amd import workloads as W


def test_d3q19_lattice_identities():
    ex, ey, ez, w = O3.lattice()
    e = np.stack([ex, ey, ez], 1).astype(float)
    want = {(0, 0, 0)} | {v for v in itertools.product((-1, 0, 1), repeat=3)
                         if 1 <= sum(map(abs, v)) <= 2}
    assert set(map(tuple, e.astype(int))) == want and len(want) == 19
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w @ e, 0.0, atol=1e-16)
    cs2 = 1.0 / 3.0
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), cs2 * np.eye(3), atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, e, e, e), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), iso4, atol=1e-16)


def test_equilibrium_moments():
    ex, ey, ez, _ = O3.lattice()
    e = np.stack([ex, ey, ez], 1).astype(float)
    rho, u = 1.03, np.array([0.02, -0.015, 0.01])
    feq = O3.equilibrium(rho, *u)
    assert feq.sum() == pytest.approx(rho, abs=1e-15)
    assert np.allclose(feq @ e, u, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", feq, e, e), rho / 3 * np.eye(3) + np.outer(u, u),
                       atol=1e-15)


def _box(n=12, **kw):
    return W.Problem3(nx=n, ny=n + 2, nz=n + 4, tau=0.8, **kw)


def test_periodic_conservation_and_uniform_acceleration():
    p = O3.make_problem(_box())
    _, _, _, w = O3.lattice()
    f = np.ascontiguousarray(w[:, None, None, None] * (1.0 + 1e-2 * W.seeded_noise((19, 16, 14, 12), 60, 0)))
    m0 = [a.sum() for a in O3.moments(p, f)]
    O3.run(p, f, None, 20)
    m1 = [a.sum() for a in O3.moments(p, f)]
    assert np.allclose(m0, m1, atol=1e-12)
    g = (1e-5, -2e-5, 3e-5)
    p = O3.make_problem(_box(body_force=g))
    f = O3.rest_state(p)
    O3.run(p, f, None, 10)
    _, ux, uy, uz = O3.moments(p, f)
    for a, v in zip((ux, uy, uz), g):
        assert np.allclose(a, 10 * v, rtol=1e-10)


def _sphere(mode, n=24, R=5.3, F=4e-3):
    c = (n / 2 + 0.27, n / 2 - 0.31, n / 2 + 0.13)
    nm = int(np.ceil(4 * np.pi * R * R))
    prob = W.Problem3(nx=n, ny=n, nz=n, tau=0.8, center=c, radius=R, f_normal=F,
                      force_mode=mode, n_markers=nm if mode == W.FORCE_IB_LBM else 0)
    return prob, W.sphere_markers(c, R, nm)


def test_sphere_cut_links_against_brute_force():
    prob, _ = _sphere(W.FORCE_II_LBM)
    p = O3.make_problem(prob)
    ex, ey, ez, _ = O3.lattice()
    z, y, x = np.mgrid[0:p.nz, 0:p.ny, 0:p.nx].astype(float)
    phi = lambda a, b, c: (a - p.cx) ** 2 + (b - p.cy) ** 2 + (c - p.cz) ** 2 - p.radius ** 2
    inside = phi(x, y, z) < 0
    n = sum(int((inside != (phi(x + ex[i], y + ey[i], z + ez[i]) < 0)).sum()) for i in range(1, 19))
    assert O3.count_cut_links(p) == n > 500


def test_peskin_3d_partition_of_unity():
    prob, X = _sphere(W.FORCE_IB_LBM)
    p = O3.make_problem(prob)
    g = O3.spread(p, X)
    r = X - np.array([p.cx, p.cy, p.cz])
    dA = 4 * np.pi * p.radius ** 2 / len(X)
    want = p.f_normal * (r / p.radius).sum(0) * dA
    assert np.allclose(g.reshape(3, -1).sum(1), want, atol=1e-14)
    # first moment: sum_x x g(x) equals sum_k X_k G_k dA
    z, y, x = np.mgrid[0:p.nz, 0:p.ny, 0:p.nx].astype(float)
    fx = (x * g[0]).sum()
    assert fx == pytest.approx((X[:, 0] * p.f_normal * r[:, 0] / p.radius).sum() * dA, rel=1e-12)


def test_exact_state_is_a_fixed_point_of_ii_lbm_only():
    for mode in (W.FORCE_II_LBM, W.FORCE_IB_LBM):
        prob, X = _sphere(mode)
        p = O3.make_problem(prob)
        f = W.normal_force_sphere_state(prob)
        f0 = f.copy()
        O3.run(p, f, X, 8)
        _, ux, uy, uz = O3.moments(p, f)
        umax = max(np.abs(a).max() for a in (ux, uy, uz))
        if mode == W.FORCE_II_LBM:
            assert np.abs(f - f0).max() < 1e-14 and umax < 1e-14     # round-off
        else:
            assert umax > 1e-5


def test_sphere_mass_conserved_with_jumps():
    prob, X = _sphere(W.FORCE_II_LBM)
    p = O3.make_problem(prob)
    _, _, _, w = O3.lattice()
    f = np.ascontiguousarray(w[:, None, None, None] * (1.0 + 1e-3 * W.seeded_noise((19, 24, 24, 24), 61, 0)))
    m0 = O3.moments(p, f)[0].sum()
    O3.run(p, f, X, 5)
    assert abs(O3.moments(p, f)[0].sum() - m0) < 1e-11
