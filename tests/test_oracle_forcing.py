"""Pins of the oracle's force modes (no GPU): Guo's force term with its
compressible equilibrium and half-force velocity (Sec. 2.2.2), the IB-LBM
comparison modes (whole force spread, no jumps), and the area conservation
comparison of the thin elastic membrane (Sec. 4.2, Table 2), against closed
forms of the D2Q9 lattice, invariants and the paper's central claim.

Each check is chosen so that a plausible slip (the force term's sign, a
missing half-force shift, the incompressible equilibrium where the
compressible one belongs, a relaxation factor (1 - s/2) on the wrong moment,
jumps left on in a comparison mode) fails one of them.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2003_12186_amd import workloads as W

GUO_MODES = (W.FORCE_IB_LBM_GUO, W.FORCE_II_LBM_GUO)


def _lattice():
    ex, ey, w = O.d2q9()
    return ex.astype(float), ey.astype(float), w


def _random_node_state(rng, amp=0.05):
    _, _, w = O.d2q9()
    return w * (1.0 + amp * rng.standard_normal(9))


def test_guo_term_moments_closed_form():
    # The bracket of Guo's term (Sec. 2.2.2) has zeroth moment 0, first moment
    # g and second moment u g + g u: with the D2Q9 isotropy
    # sum w e_a e_b = c_s^2 delta_ab and the fourth-order identity these are
    # the moments that make the force enter the momentum and stress exactly.
    ex, ey, _ = _lattice()
    rng = np.random.default_rng(11)
    for _ in range(20):
        u = 0.1 * rng.standard_normal(2)
        g = 1e-2 * rng.standard_normal(2)
        G = O.guo_term(u[0], u[1], g[0], g[1])
        assert abs(G.sum()) < 1e-17
        assert G @ ex == pytest.approx(g[0], abs=1e-17)
        assert G @ ey == pytest.approx(g[1], abs=1e-17)
        assert (G * ex * ex).sum() == pytest.approx(2 * u[0] * g[0], abs=1e-17)
        assert (G * ey * ey).sum() == pytest.approx(2 * u[1] * g[1], abs=1e-17)
        assert (G * ex * ey).sum() == pytest.approx(u[0] * g[1] + u[1] * g[0], abs=1e-17)
    # with u = 0 it reduces to the simple term w_i e_i.g / c_s^2
    _, _, w = _lattice()
    G = O.guo_term(0.0, 0.0, 3e-3, -1e-3)
    assert np.allclose(G, 3.0 * w * (ex * 3e-3 - ey * 1e-3), atol=1e-18)


@pytest.mark.parametrize("mode", GUO_MODES)
def test_guo_equilibrium_is_compressible_by_its_nine_moments(mode):
    # SRT with tau = 1 and no force returns the equilibrium itself.  Under
    # Guo's term it is w_i p/c_s^2 [...] (Sec. 2.2.2), whose nine D2Q9 moments
    # are fixed in closed form by the lattice: rho, j, rho/3 + j_a j_b / rho,
    # the third-order pair j/3 and the fourth-order rho/9 + |j|^2 / (3 rho).
    # The He-Luo equilibrium of the II-LBM differs in every j j term at rho != 1.
    ex, ey, _ = _lattice()
    p = O.make_problem(W.Problem(nx=4, ny=4, tau=1.0, force_mode=mode))
    rng = np.random.default_rng(12)
    for _ in range(20):
        f = _random_node_state(rng) * rng.uniform(0.85, 1.25)
        rho, jx, jy = f.sum(), f @ ex, f @ ey
        feq = O.collide_node(p, f)
        mom = lambda a, b: (feq * ex ** a * ey ** b).sum()
        assert mom(0, 0) == pytest.approx(rho, abs=1e-15)
        assert mom(1, 0) == pytest.approx(jx, abs=1e-15)
        assert mom(0, 1) == pytest.approx(jy, abs=1e-15)
        assert mom(2, 0) == pytest.approx(rho / 3 + jx * jx / rho, abs=1e-15)
        assert mom(0, 2) == pytest.approx(rho / 3 + jy * jy / rho, abs=1e-15)
        assert mom(1, 1) == pytest.approx(jx * jy / rho, abs=1e-15)
        assert mom(1, 2) == pytest.approx(jx / 3, abs=1e-15)
        assert mom(2, 1) == pytest.approx(jy / 3, abs=1e-15)
        assert mom(2, 2) == pytest.approx(rho / 9 + (jx * jx + jy * jy) / (3 * rho), abs=1e-15)


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
@pytest.mark.parametrize("mode", GUO_MODES)
def test_guo_collision_adds_exactly_g_for_any_rates(collision, mode):
    # The half-force velocity p/c_s^2 u = sum e f + g/2 and the factor
    # (1 - s/2) together add exactly g to the momentum, whatever the rate of
    # the momentum moments: -s (j - (j + g/2)) + (1 - s/2) g = g.  Without the
    # half-force shift the gain would be (1 - s/2) g.  Mass is untouched.
    ex, ey, _ = _lattice()
    rates = [0.0, 1.1, 1.2, 1.3, 1.4, 0.7, 1.5, 1.6, 1.7]
    p = O.make_problem(W.Problem(nx=4, ny=4, tau=1.0 / 1.6, collision=collision,
                                 force_mode=mode, mrt_s=rates))
    rng = np.random.default_rng(13)
    for _ in range(20):
        f = _random_node_state(rng) * rng.uniform(0.9, 1.1)
        g = 1e-3 * rng.standard_normal(2)
        out = O.collide_node(p, f, g[0], g[1])
        assert out.sum() == pytest.approx(f.sum(), abs=1e-15)
        assert out @ ex == pytest.approx(f @ ex + g[0], abs=1e-15)
        assert out @ ey == pytest.approx(f @ ey + g[1], abs=1e-15)


@pytest.mark.parametrize("mode", GUO_MODES)
def test_mrt_guo_with_all_rates_one_over_tau_equals_srt_guo(mode):
    # With S = I/tau, M^-1 (I - S/2) M G~ = (1 - 1/(2 tau)) G~ (Sec. 2.2.2):
    # the two forms of Guo's term and the two collisions coincide.
    tau = 0.83
    ps = O.make_problem(W.Problem(nx=4, ny=4, tau=tau, collision=W.SRT, force_mode=mode))
    pm = O.make_problem(W.Problem(nx=4, ny=4, tau=tau, collision=W.MRT, force_mode=mode,
                                  mrt_s=[1.0 / tau] * 9))
    rng = np.random.default_rng(14)
    for _ in range(20):
        f = _random_node_state(rng)
        g = 1e-3 * rng.standard_normal(2)
        assert np.allclose(O.collide_node(ps, f, *g), O.collide_node(pm, f, *g), atol=1e-15)


def test_mrt_guo_rates_act_moment_by_moment():
    # Changing the rate of one non-conserved moment changes that moment of the
    # result and no other (the force enters each moment with its own factor
    # (1 - s/2)); a transposed or mis-normalised M^-1 would leak into others.
    M, _ = O.mrt_matrices()
    base = [0.0, 1.1, 1.2, 0.0, 1.4, 0.0, 1.4, 1.6, 1.6]
    rng = np.random.default_rng(15)
    f = _random_node_state(rng)
    g = 2e-3 * rng.standard_normal(2)
    ref = M @ O.collide_node(O.make_problem(W.Problem(
        nx=4, ny=4, tau=0.625, collision=W.MRT, force_mode=W.FORCE_IB_LBM_GUO, mrt_s=base)), f, *g)
    for a in (1, 2, 4, 6, 7, 8):
        s = list(base)
        s[a] = 0.9
        m = M @ O.collide_node(O.make_problem(W.Problem(
            nx=4, ny=4, tau=0.625, collision=W.MRT, force_mode=W.FORCE_IB_LBM_GUO, mrt_s=s)), f, *g)
        others = [b for b in range(9) if b != a]
        assert np.allclose(m[others], ref[others], atol=1e-15)
        assert abs(m[a] - ref[a]) > 1e-6


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_guo_uniform_body_force_accelerates_exactly(collision):
    # A uniform force on a periodic box accelerates the fluid uniformly: after
    # n steps sum e f = n g at every node and the density stays 1.
    g = (1e-5, -2e-5)
    p = O.make_problem(W.Problem(nx=8, ny=6, tau=0.7, collision=collision,
                                 force_mode=W.FORCE_IB_LBM_GUO, body_force=g))
    f = O.rest_state(p)
    O.run(p, f, None, 10)
    rho, jx, jy = O.moments(p, f)
    assert np.allclose(rho, 1.0, atol=1e-14)
    assert np.allclose(jx, 10 * g[0], rtol=1e-10)
    assert np.allclose(jy, 10 * g[1], rtol=1e-10)


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_guo_poiseuille_parabola(collision):
    # Body-force driven channel under Guo's term: the velocity (j + g/2)/rho of
    # the interior rows has the second difference -g/nu of the parabola
    # g y (H - y) / (2 nu), nu = (tau - 1/2)/3.
    ny, g, tau = 11, 1e-6, 0.9
    nu = (tau - 0.5) / 3.0
    p = O.make_problem(W.Problem(nx=4, ny=ny, tau=tau, collision=collision,
                                 bc=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_WALL, W.BC_WALL),
                                 force_mode=W.FORCE_IB_LBM_GUO, body_force=(g, 0.0)))
    f = O.rest_state(p)
    O.run(p, f, None, 40000)
    rho, jx, jy = O.moments(p, f)
    u = (jx + 0.5 * g) / rho
    prof = u[1:-1, 0]
    d2 = prof[2:] - 2 * prof[1:-1] + prof[:-2]
    assert np.allclose(d2, -g / nu, rtol=1e-6)
    assert np.abs(jy).max() < 1e-15


def _regular(n, R, cx=32.0, cy=32.0, phase=0.0):
    th = phase + 2 * np.pi * np.arange(n) / n
    return np.stack([cx + R * np.cos(th), cy + R * np.sin(th)], 1)


@pytest.mark.parametrize("mode", [W.FORCE_II_LBM, W.FORCE_IB_LBM, W.FORCE_IB_LBM_GUO,
                                  W.FORCE_II_LBM_GUO])
def test_modes_spread_their_force_and_jump_only_with_ii_lbm(mode):
    # The delta's weights sum to one at every marker, so the spread field holds
    # sum_k F_k dX with F = G_par under II-LBM (Sec. 3.2) and F = G under
    # IB-LBM (Sec. 2.2.2); cut links (and their jumps) exist only under II-LBM.
    n, R = 64, 9.0
    X = _regular(n, R, 24.3, 23.8) * np.array([1.0, 1.0])
    X[:, 0] = 24.3 + 1.3 * (X[:, 0] - 24.3)       # an ellipse: G_par != 0
    p = O.make_problem(W.Problem(nx=48, ny=48, tau=0.8, interface=W.IF_MEMBRANE,
                                 force_mode=mode, n_markers=n, kappa=0.05,
                                 dX=2 * np.pi * R / n))
    f = O.rest_state(p)
    d = O.step(p, f, X, detail=True)
    F = d["Gt"] if mode in (W.FORCE_II_LBM, W.FORCE_II_LBM_GUO) else d["G"]
    assert d["gx"].sum() == pytest.approx(F[:, 0].sum() * p.dX, abs=1e-14)
    assert d["gy"].sum() == pytest.approx(F[:, 1].sum() * p.dX, abs=1e-14)
    assert np.abs(d["Gt"]).max() > 1e-4
    if mode in (W.FORCE_II_LBM, W.FORCE_II_LBM_GUO):
        assert len(d["links"]) > 0
    else:
        assert len(d["links"]) == 0


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_laplace_fixed_point_ii_lbm_with_guo_term(collision):
    # The two equilibria agree at rest (w_i rho), and a regular polygon has no
    # tangential force, so the Laplace state of II-LBM is a fixed point under
    # Guo's term too (Sec. 3.2: Guo's term then takes g_par).
    n, R = 96, 10.0
    X = _regular(n, R)
    p = O.make_problem(W.Problem(nx=64, ny=64, tau=0.8, collision=collision,
                                 interface=W.IF_MEMBRANE, force_mode=W.FORCE_II_LBM_GUO,
                                 n_markers=n, kappa=0.05, dX=2 * np.pi * R / n))
    jp = O.marker_forces(p, X)["jp"]
    _, _, w = O.d2q9()
    f = np.zeros((9, p.ny, p.nx))
    for y in range(p.ny):
        for x in range(p.nx):
            f[:, y, x] = w * (1.0 - 3.0 * jp.mean() if O.node_inside(p, X, x, y) else 1.0)
    f0, X0 = f.copy(), X.copy()
    O.run(p, f, X, 5)
    assert np.abs(f - f0).max() < 1e-14
    assert np.abs(X - X0).max() < 1e-14


def _e2_area_history(L, mode, spans):
    """The thin elastic membrane of Sec. 4.2 in the oracle; the enclosed area
    at the start and after each span (in L/U)."""
    w = W.elastic_membrane_e2(L, mode)
    p = O.make_problem(w.problem)
    f = O.rest_state(p)
    X = w.X0.copy()
    areas = [O.polygon_area(X)]
    for span in spans:
        O.run(p, f, X, int(round(span * w.meta["span"])))
        areas.append(O.polygon_area(X))
    return np.array(areas)


def test_area_conservation_ii_lbm_against_ib_lbm():
    # The paper's comparison (Sec. 4.2, Table 2): after the first oscillation
    # the II-LBM membrane keeps its area, while both IB-LBM membranes steadily
    # lose area.  In the comparison modes the markers move with the scheme's
    # own velocity taken from the distributions after the step's force
    # (reading R18): sum e f + g under the simple term, (sum e f + 3 g/2) / rho
    # under Guo's.  Both run ahead of the fluid (by half a force step and by a
    # whole one); the regularised force points inward, so the markers slip
    # inward and the area shrinks, about twice as fast under Guo's term.
    # Table 2 gives the loss per unit time in units of L U (the area per step
    # over L U, so the loss per L/U over L^2): 2.42e-3 (simple term) and
    # 3.70e-3 (Guo's term) at L = 80, falling as the grid is refined, Guo's
    # 1.5-2.0 times the simple term's at every L.  At L = 48, coarser than the
    # paper's coarsest grid, the rates over t = 2..5 L/U must be losses of at
    # least the paper's L = 80 rate and at most three times it (measured
    # 4.73e-3 and 9.0e-3), in a Guo-to-simple ratio within 1.4..2.2 (1.90);
    # II-LBM, with either force term, stays below 1e-5 of the area per L/U
    # (measured -4e-6 and -5e-6).
    L = 48
    rate, rate_l2 = {}, {}
    for mode in (W.FORCE_II_LBM, W.FORCE_IB_LBM, W.FORCE_IB_LBM_GUO, W.FORCE_II_LBM_GUO):
        A = _e2_area_history(L, mode, (2.0, 3.0))
        rate[mode] = (A[2] - A[1]) / A[0] / 3.0          # per L/U after t = 2 L/U
        rate_l2[mode] = -(A[2] - A[1]) / L ** 2 / 3.0     # loss per L/U over L^2
    ii = max(abs(rate[W.FORCE_II_LBM]), abs(rate[W.FORCE_II_LBM_GUO]))
    assert ii < 1e-5
    for mode, paper in ((W.FORCE_IB_LBM, 2.42e-3), (W.FORCE_IB_LBM_GUO, 3.70e-3)):
        assert rate[mode] < -100 * ii
        assert paper <= rate_l2[mode] <= 3.0 * paper, (mode, rate_l2[mode])
    assert 1.4 <= rate_l2[W.FORCE_IB_LBM_GUO] / rate_l2[W.FORCE_IB_LBM] <= 2.2
