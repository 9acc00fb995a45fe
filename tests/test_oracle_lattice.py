"""Pins of the oracle's lattice, equilibrium, collision and streaming against
closed forms that the paper and the D2Q9 lattice fix (no GPU).

Each check is chosen so that a plausible slip (a wrong weight, a swapped
velocity, a sign in the equilibrium, a transposed MRT inverse, streaming in
the wrong direction) fails it.
"""
import numpy as np
import pytest

import oracle as O
from paper_2003_12186_amd import workloads as W


def test_d2q9_lattice_identities():
    # Sec. 2.1.1 velocities and Sec. 2.2.1 weights: the quadrature must be
    # isotropic up to fourth order with c_s^2 = 1/3.
    ex, ey, w = O.d2q9()
    e = np.stack([ex, ey], 1).astype(float)
    assert set(map(tuple, e.astype(int))) == {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1),
                                               (1, 1), (-1, 1), (-1, -1), (1, -1)}
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w @ e, 0.0, atol=1e-16)
    cs2 = 1.0 / 3.0
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), cs2 * np.eye(2), atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, e, e, e), 0.0, atol=1e-16)
    d = np.eye(2)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), iso4, atol=1e-16)
    # weights by speed: 4/9 rest, 1/9 axis, 1/36 diagonal (Sec. 2.2.1)
    for i in range(9):
        c2 = ex[i] ** 2 + ey[i] ** 2
        assert w[i] == pytest.approx({0: 4 / 9, 1: 1 / 9, 2: 1 / 36}[c2], abs=1e-16)


def test_equilibrium_moments_closed_form():
    # He-Luo incompressible equilibrium (Sec. 2.2.1): zeroth moment rho, first
    # moment u (not rho u), second moment (rho/3) I + u u.
    ex, ey, _ = O.d2q9()
    e = np.stack([ex, ey], 1).astype(float)
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(2)
        feq = O.equilibrium(rho, u[0], u[1])
        assert feq.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(feq @ e, u, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", feq, e, e)
        assert np.allclose(P, rho / 3.0 * np.eye(2) + np.outer(u, u), atol=1e-15)


def test_mrt_matrices():
    M, Mi = O.mrt_matrices()
    # independent inverse
    assert np.allclose(Mi, np.linalg.inv(M), atol=1e-14)
    assert np.allclose(M @ Mi, np.eye(9), atol=1e-14)
    # rows orthogonal
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-13)
    # conserved rows are density and momentum, in the Lallemand-Luo order
    ex, ey, _ = O.d2q9()
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[3], ex.astype(float))
    assert np.array_equal(M[5], ey.astype(float))
    # row norms of the D2Q9 basis
    assert np.allclose(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])


def _random_node_state(rng):
    _, _, w = O.d2q9()
    return w * (1.0 + 0.05 * rng.standard_normal(9))


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_collision_conserves_mass_momentum_and_adds_force(collision):
    ex, ey, _ = O.d2q9()
    prob = W.Problem(nx=4, ny=4, tau=0.7, collision=collision)
    p = O.make_problem(prob)
    rng = np.random.default_rng(1)
    for _ in range(20):
        f = _random_node_state(rng)
        g = 1e-3 * rng.standard_normal(2)
        out = O.collide_node(p, f, g[0], g[1])
        assert out.sum() == pytest.approx(f.sum(), abs=1e-15)
        # the simple force term adds exactly g to the momentum (Sec. 2.2.2)
        assert (out @ ex) == pytest.approx(f @ ex + g[0], abs=1e-15)
        assert (out @ ey) == pytest.approx(f @ ey + g[1], abs=1e-15)


def test_mrt_with_all_rates_one_over_tau_equals_srt():
    tau = 0.83
    ps = O.make_problem(W.Problem(nx=4, ny=4, tau=tau, collision=W.SRT))
    pm = O.make_problem(W.Problem(nx=4, ny=4, tau=tau, collision=W.MRT, mrt_s=[1.0 / tau] * 9))
    rng = np.random.default_rng(2)
    for _ in range(20):
        f = _random_node_state(rng)
        assert np.allclose(O.collide_node(ps, f), O.collide_node(pm, f), atol=1e-15)


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_rest_and_uniform_flow_equilibria_are_fixed_by_collision(collision):
    p = O.make_problem(W.Problem(nx=4, ny=4, tau=0.6, collision=collision))
    for rho, ux, uy in ((1.0, 0.0, 0.0), (1.02, 0.03, -0.01)):
        feq = O.equilibrium(rho, ux, uy)
        assert np.allclose(O.collide_node(p, feq), feq, atol=1e-16)


def test_srt_relaxation_closed_form():
    # SRT moves each population the fraction 1/tau of the way to equilibrium.
    p = O.make_problem(W.Problem(nx=4, ny=4, tau=2.0))
    rng = np.random.default_rng(3)
    f = _random_node_state(rng)
    rho, ux, uy = f.sum(), f @ O.d2q9()[0], f @ O.d2q9()[1]
    feq = O.equilibrium(rho, ux, uy)
    assert np.allclose(O.collide_node(p, f), 0.5 * (f + feq), atol=1e-16)


@pytest.mark.parametrize("i", range(1, 9))
def test_streaming_moves_population_i_along_e_i(i):
    # A small bump in population i, collision made negligible (huge tau):
    # after one step it sits at x0 + e_i (Sec. 2.2.1, Eq. (14) upwind form).
    ex, ey, w = O.d2q9()
    prob = W.Problem(nx=8, ny=8, tau=1e15)
    p = O.make_problem(prob)
    f = O.rest_state(p)
    f[i, 3, 4] += 1e-3
    O.step(p, f, None)
    d = f - O.rest_state(p)
    ys, xs = np.nonzero(np.abs(d[i]) > 5e-4)
    assert list(zip(xs, ys)) == [((4 + ex[i]) % 8, (3 + ey[i]) % 8)]


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_periodic_mass_and_momentum_conserved(collision):
    # P-1: with no interface and periodic sides the step is a collision that
    # conserves rho and u followed by a permutation.
    prob = W.Problem(nx=24, ny=16, tau=0.9, collision=collision)
    p = O.make_problem(prob)
    _, _, w = O.d2q9()
    f = w[:, None, None] * (1.0 + 1e-2 * W.seeded_noise((9, 16, 24), 90, 1))
    f = np.ascontiguousarray(f)
    rho0, ux0, uy0 = (a.sum() for a in O.moments(p, f))
    O.run(p, f, None, 50)
    rho1, ux1, uy1 = (a.sum() for a in O.moments(p, f))
    n = 24 * 16
    assert abs(rho1 - rho0) < 50 * n * 2e-16
    assert abs(ux1 - ux0) < 50 * n * 2e-16 and abs(uy1 - uy0) < 50 * n * 2e-16


def test_uniform_body_force_accelerates_exactly():
    # Sum of momentum grows by g per node per step with the simple force term.
    prob = W.Problem(nx=8, ny=6, tau=0.7, body_force=(1e-5, -2e-5))
    p = O.make_problem(prob)
    f = O.rest_state(p)
    O.run(p, f, None, 10)
    _, ux, uy = O.moments(p, f)
    assert np.allclose(ux, 10 * 1e-5, rtol=1e-10)
    assert np.allclose(uy, -10 * 2e-5, rtol=1e-10)


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_couette_linear_profile_with_nee_walls(collision):
    # P-4: plane Couette flow between a resting wall (y=0) and a wall moving at
    # U (y=H); the steady solution u_x = U y / H is linear, which the lattice
    # reproduces exactly; walls by non-equilibrium extrapolation.
    ny, U = 9, 0.01
    prob = W.Problem(nx=4, ny=ny, tau=0.8, collision=collision,
                     bc=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_WALL, W.BC_WALL),
                     u_wall=(0.0, 0.0, 0.0, U))
    p = O.make_problem(prob)
    f = O.rest_state(p)
    O.run(p, f, None, 6000)
    rho, ux, uy = O.moments(p, f)
    H = ny - 1
    exact = U * np.arange(ny) / H
    assert np.abs(ux - exact[:, None]).max() < 1e-13
    assert np.abs(uy).max() < 1e-14


@pytest.mark.parametrize("tau", [0.6, 0.9, 1.5])
def test_poiseuille_parabola_with_body_force_and_nee_walls(tau):
    # P-5: body-force driven channel flow between resting walls at y=0, H.
    # The interior profile must be the parabola g y (H - y) / (2 nu) with
    # nu = (tau - 1/2)/3 (Sec. 2.2.1): its second difference is -g/nu exactly,
    # which pins the force term and the viscosity relation.  The extrapolation
    # walls leave a uniform slip offset of order g/nu that the paper does not
    # fix; it is only required to be uniform, the same for SRT and MRT, and the
    # wall nodes themselves must carry u = 0.
    ny, g = 11, 1e-6
    nu = (tau - 0.5) / 3.0
    offs = []
    for coll in (W.SRT, W.MRT):
        prob = W.Problem(nx=4, ny=ny, tau=tau, collision=coll,
                         bc=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_WALL, W.BC_WALL),
                         body_force=(g, 0.0))
        p = O.make_problem(prob)
        f = O.rest_state(p)
        O.run(p, f, None, 40000)
        _, ux, uy = O.moments(p, f)
        H = ny - 1
        y = np.arange(1, ny - 1)
        prof = ux[1:-1, 0]
        d2 = prof[2:] - 2 * prof[1:-1] + prof[:-2]
        assert np.allclose(d2, -g / nu, rtol=1e-7)
        off = prof - g * y * (H - y) / (2.0 * nu)
        assert np.ptp(off) < 1e-7 * g / nu
        assert abs(ux[0, 0]) < 1e-15 and abs(ux[-1, 0]) < 1e-15
        assert np.abs(uy).max() < 1e-15
        offs.append(off.mean())
    assert offs[0] == pytest.approx(offs[1], abs=1e-8 * g / nu)
