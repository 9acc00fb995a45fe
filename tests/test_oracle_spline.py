"""Pins of the oracle's cubic-spline membrane geometry (Sec. 3.2 names a cubic
spline for flexible interfaces; reading R27), no GPU: the spline's accuracy
on a circle and its continuity, its link crossings against an independent
dense-sampling search, the jump at the crossings, and the whole step.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2003_12186_amd import workloads as W


def _segment_points(X, M, k, t):
    """S_k(t) in the standard form (1-t) X_k + t X_{k+1} +
    [((1-t)^3 - (1-t)) M_k + (t^3 - t) M_{k+1}] / 6."""
    N = len(X)
    kp = (k + 1) % N
    t = np.asarray(t)[:, None]
    return ((1 - t) * X[k] + t * X[kp]
            + (((1 - t) ** 3 - (1 - t)) * M[k] + (t ** 3 - t) * M[kp]) / 6.0)


def _problem(X, **kw):
    n = len(X)
    p = W.Problem(nx=64, ny=64, tau=0.8, interface=W.IF_MEMBRANE, n_markers=n, kappa=0.05,
                  dX=W.membrane_dX(10.0, 10.0, n), geometry=W.GEOM_SPLINE, **kw)
    return p, O.make_problem(p)


@pytest.mark.parametrize("N", [16, 32])
def test_spline_of_a_circle_is_fourth_order_and_smooth(N):
    # Markers on a circle: the spline between them stays within O(h^4) of the
    # circle while the chord's sagitta is O(h^2); halving h divides the error
    # by about 16.  The tangent is continuous across the knots.
    R, c = 10.0, np.array([32.0, 32.0])

    def err(n):
        th = 2 * np.pi * np.arange(n) / n
        X = c + R * np.stack([np.cos(th), np.sin(th)], 1)
        _, p = _problem(X)
        M = O.spline_second_derivs(p, X)
        t = np.linspace(0.0, 1.0, 41)
        return max(np.abs(np.linalg.norm(_segment_points(X, M, k, t) - c, axis=1) - R).max()
                   for k in range(n)), X, M

    e1, X, M = err(N)
    e2, _, _ = err(2 * N)
    sagitta = R * (1 - math.cos(math.pi / N))
    assert e1 < sagitta / 50
    assert 12.0 < e1 / e2 < 20.0
    h = 1e-6
    for k in range(N):
        a = (_segment_points(X, M, k, [1.0]) - _segment_points(X, M, k, [1.0 - h])) / h
        b = (_segment_points(X, M, (k + 1) % N, [h]) - _segment_points(X, M, (k + 1) % N, [0.0])) / h
        assert np.abs(a - b).max() < 1e-5


def _wobbly(n=28, seed=7):
    th = 2 * np.pi * np.arange(n) / n
    r = 9.0 + 1.2 * np.cos(3 * th + 0.4) + 0.15 * W.seeded_noise((n,), 97, seed)
    return np.stack([31.3 + r * np.cos(th), 32.6 + 0.8 * r * np.sin(th)], 1)


def test_spline_crossings_match_dense_sampling():
    # Every (link, segment) crossing: f(t) = e x (S(t) - P) sampled on a
    # fine grid, sign changes located by interpolation, kept where the link
    # parameter q lies in [0, 1).  Same set (node, direction, sign, segment)
    # as the oracle's root finder, with t to 1e-6.
    X = _wobbly()
    _, p = _problem(X)
    M = O.spline_second_derivs(p, X)
    G = O.marker_forces(p, X)["G"]
    got = O.cutlinks_spline(p, X, G)
    ex, ey, _ = O.d2q9()
    t = np.linspace(0.0, 1.0, 20001)
    want = []
    for k in range(len(X)):
        S = _segment_points(X, M, k, t)
        lo = np.floor(S.min(0)).astype(int) - 1
        hi = np.ceil(S.max(0)).astype(int) + 1
        for y in range(lo[1], hi[1] + 1):
            for x in range(lo[0], hi[0] + 1):
                for i in range(1, 9):
                    e = np.array([ex[i], ey[i]], float)
                    d = S - np.array([x, y], float)
                    f = e[0] * d[:, 1] - e[1] * d[:, 0]
                    s = f >= 0.0
                    for j in np.nonzero(s[1:] != s[:-1])[0]:
                        tt = t[j] + (t[j + 1] - t[j]) * f[j] / (f[j] - f[j + 1])
                        P = _segment_points(X, M, k, [tt])[0]
                        q = ((P - [x, y]) @ e) / (e @ e)
                        if 1e-7 < q < 1 - 1e-7:
                            want.append((x, y, i, 1 if not s[j] else -1, k, tt))
    key = lambda r: (r[0], r[1], r[2], r[3], r[4])
    g = sorted((int(r["x"]), int(r["y"]), int(r["dir"]), int(r["sigma"]), int(r["seg"]), float(r["theta"]))
               for r in got)
    w = sorted(want)
    assert [key(r) for r in g] == [key(r) for r in w]
    assert max(abs(a[5] - b[5]) for a, b in zip(g, w)) < 1e-6
    assert len(g) > 100


def test_spline_jump_on_a_tensioned_circle():
    # A regular polygon under spring tension: [[p]] at every crossing is the
    # marker value G.n/J to within the variation between markers: G is
    # linear between two force vectors 2 pi / N apart, so its length dips by
    # cos(pi / N), about (pi / N)^2 / 2, in the middle of a segment.
    n, R = 48, 10.0
    th = 2 * np.pi * np.arange(n) / n
    X = np.stack([32.0 + R * np.cos(th), 32.0 + R * np.sin(th)], 1)
    _, p = _problem(X)
    d = O.marker_forces(p, X)
    links = O.cutlinks_spline(p, X, d["G"])
    jp = links["jp"]
    assert np.ptp(d["jp"]) < 1e-12 * abs(d["jp"][0])
    assert np.abs(jp / d["jp"][0] - 1.0).max() < (math.pi / n) ** 2
    assert jp.mean() < 0.0


def test_spline_step_mass_and_momentum_budget():
    # As for the polygon: the jumps add +c and -c at the two ends of every
    # cut link (mass conserved), and the momentum change is the spread force
    # plus sigma w_i [[p]] e_i / c_s^2 summed over the crossings.
    w = W.membrane_ellipse64()
    w.problem.geometry = W.GEOM_SPLINE
    p = O.make_problem(w.problem)
    ex, ey, wt = O.d2q9()
    f = np.ascontiguousarray(wt[:, None, None] * (1.0 + 1e-3 * W.seeded_noise((9, 64, 64), 98, 0)))
    X = w.X0 + 0.3 * W.seeded_noise(w.X0.shape, 99, 0)
    for _ in range(3):
        rho0, ux0, uy0 = (a.sum() for a in O.moments(p, f))
        d = O.step(p, f, X, detail=True)
        rho1, ux1, uy1 = (a.sum() for a in O.moments(p, f))
        assert abs(rho1 - rho0) < 1e-12
        L = d["links"]
        jx = sum(r["sigma"] * wt[r["dir"]] * 3.0 * r["jp"] * ex[r["dir"]] for r in L)
        jy = sum(r["sigma"] * wt[r["dir"]] * 3.0 * r["jp"] * ey[r["dir"]] for r in L)
        assert ux1 - ux0 == pytest.approx(d["gx"].sum() + jx, abs=1e-13)
        assert uy1 - uy0 == pytest.approx(d["gy"].sum() + jy, abs=1e-13)
        assert len(L) > 50


def test_spline_membrane_obeys_laplace_law():
    # The 64 x 64 membrane with the spline geometry relaxes to a circle whose
    # pressure jump is T / R within 1 % (time average over steps 1000..2000).
    w = W.membrane_ellipse64()
    w.problem.geometry = W.GEOM_SPLINE
    p = O.make_problem(w.problem)
    f = O.rest_state(p)
    X = w.X0.copy()
    O.run(p, f, X, 1000)
    dps, trs = [], []
    for _ in range(25):
        O.run(p, f, X, 40)
        rho, _, _ = O.moments(p, f)
        A = O.polygon_area(X)
        l = np.linalg.norm(np.roll(X, -1, 0) - X, axis=1).mean()
        dps.append(O.pressure_jump(p, rho, X))
        trs.append(p.kappa * l / p.dX / math.sqrt(A / math.pi))
    assert np.mean(dps) / np.mean(trs) == pytest.approx(1.0, abs=0.01)
