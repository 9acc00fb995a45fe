"""Pins of the oracle's rigid-body dynamics of a circle (Sec. 2.3), no GPU:
the total force and torque with their interior-inertia terms, the paper's
update of velocity, position and angle, and direct forcing toward the moving
body's velocity, against invariants the scheme must keep exactly and
closed-form motions.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2003_12186_amd import workloads as W


def _body_problem(L=64, R=6.0, n=40, mode=W.FORCE_IB_LBM, **kw):
    prob = W.Problem(nx=L, ny=L, tau=0.8, collision=W.MRT, interface=W.IF_RIGID,
                     force_mode=mode, n_markers=n, dX=2 * math.pi * R / n,
                     center=(L / 2.0, L / 2.0), radius=R, **kw)
    return prob, W.circle_markers(L / 2.0, L / 2.0, R, n)


def _uniform_flow(p, V):
    feq = O.equilibrium(1.0, V[0], V[1])
    return np.ascontiguousarray(np.broadcast_to(feq[:, None, None], (9, p.ny, p.nx))).copy()


@pytest.mark.parametrize("mode", [W.FORCE_II_LBM, W.FORCE_IB_LBM])
def test_body_carried_by_uniform_flow(mode):
    # A free body moving with a uniform flow meets no relative velocity: the
    # direct forcing is zero, F and T vanish, and the centre advances by V
    # every step while the orientation stays put.
    V = (0.02, -0.01)
    prob, X = _body_problem(mode=mode, body_free=7, rho_star=1.5)
    p = O.make_problem(prob)
    f = _uniform_flow(p, V)
    b = O.new_body(p)
    b.U[0], b.U[1] = V
    h = O.run_body(p, O.body_params(prob), b, f, X, 100)
    assert h[-1, 0] == pytest.approx(32.0 + 100 * V[0], abs=1e-10)
    assert h[-1, 1] == pytest.approx(32.0 + 100 * V[1], abs=1e-10)
    assert np.abs(h[:, 2] - V[0]).max() < 1e-12 and np.abs(h[:, 3] - V[1]).max() < 1e-12
    assert np.abs(h[:, 4]).max() < 1e-12 and np.abs(h[:, 6:]).max() < 1e-12
    _, ux, uy = O.moments(p, f)
    assert np.abs(ux - V[0]).max() < 1e-12 and np.abs(uy - V[1]).max() < 1e-12


def test_momentum_of_body_and_fluid_is_invariant():
    # IB-LBM on a periodic box: the fluid gains sum G dX per step, the body
    # m dU = -sum G dX + V_s (U^n - U^{n-1}), so
    # Q^n = P_fluid^n + m U^n - V_s U^{n-1} is an exact invariant of the
    # scheme; a wrong sign, a missing dX or a wrong inertia term breaks it.
    prob, X = _body_problem(body_free=3, rho_star=2.0)
    p = O.make_problem(prob)
    _, _, w = O.d2q9()
    f = np.ascontiguousarray(w[:, None, None] * (1.0 + 1e-3 * W.seeded_noise((9, 64, 64), 95, 0)))
    b = O.new_body(p)
    b.U[0], b.U[1] = 0.01, 0.005
    bp = O.body_params(prob)
    R = prob.radius
    m, Vs = 2.0 * math.pi * R * R, math.pi * R * R

    def Q(prev):
        _, jx, jy = O.moments(p, f)
        return np.array([jx.sum() + m * b.U[0] - Vs * prev[0], jy.sum() + m * b.U[1] - Vs * prev[1]])

    q0 = Q((b.U[0], b.U[1]))
    for _ in range(150):
        prev = (b.U[0], b.U[1])
        O.run_body(p, bp, b, f, X, 1)
        q = Q(prev)
    assert np.abs(q - q0).max() < 1e-11 * max(1.0, np.abs(q0).max())
    assert abs(b.c[0] - 32.0) > 0.1              # the body did move (drag slows it)


def test_angular_momentum_of_body_and_fluid_is_invariant():
    # A spinning free body in fluid at rest (IB-LBM, before any disturbance
    # reaches the periodic sides): the fluid gains sum (X - X_c) x G dX, the
    # body I_s dW = -sum (X - X_c) x G dX + (I_s / rho*) (W^n - W^{n-1}), so
    # L_fluid + I_s W^n - (I_s / rho*) W^{n-1} is invariant.
    L = 128
    prob, X = _body_problem(L=L, body_free=4, rho_star=2.0)
    p = O.make_problem(prob)
    f = O.rest_state(p)
    b = O.new_body(p)
    b.W = 0.004
    bp = O.body_params(prob)
    R = prob.radius
    Is = 0.5 * 2.0 * math.pi * R * R * R * R
    y, x = np.mgrid[0:L, 0:L]
    rx, ry = x - L / 2.0, y - L / 2.0

    def Lq(Wprev):
        _, jx, jy = O.moments(p, f)
        return (rx * jy - ry * jx).sum() + Is * b.W - Is / 2.0 * Wprev

    q0 = Lq(b.W)
    Ws = []
    for _ in range(60):
        Wprev = b.W
        O.run_body(p, bp, b, f, X, 1)
        Ws.append(b.W)
    assert abs(Lq(Wprev) - q0) < 1e-11 * abs(q0)
    assert 0.0 < Ws[-1] < Ws[0]                  # the fluid's torque spins it down
    assert b.c[0] == 64.0 and b.c[1] == 64.0     # translation is not free


def test_spring_mounted_heavy_body_oscillates_at_its_natural_frequency():
    # A very heavy body (rho* = 1e6) on a spring k = m omega^2 hardly feels
    # the fluid: it oscillates with period 2 pi / omega (to the O(omega dt)
    # accuracy of the paper's update) and keeps its amplitude.
    om = 2 * math.pi / 200.0
    R = 6.0
    m = 1e6 * math.pi * R * R
    prob, X = _body_problem(body_free=2, rho_star=1e6, spring=(0.0, m * om * om))
    p = O.make_problem(prob)
    f = O.rest_state(p)
    b = O.new_body(p)
    b.c[1] = 32.0 + 2.0
    h = O.run_body(p, O.body_params(prob), b, f, X, 420)
    y = h[:, 1] - 32.0
    s = np.nonzero(np.diff(np.sign(y)) != 0)[0]
    period = 2.0 * (s[2] - s[1])
    assert abs(period - 200.0) <= 4.0
    assert np.abs(y).max() == pytest.approx(2.0, rel=0.05)


def test_prescribed_harmonic_motion_and_its_drag():
    # The prescribed axis follows D_c = -A sin(U_max t / A),
    # U_c = -U_max cos(U_max t / A) (Sec. 4.4) exactly; the fluid does
    # negative work on the body over the cycle.
    A, Um = 4.0, 0.02
    prob, X = _body_problem(mode=W.FORCE_II_LBM, presc_amp=(A, 0.0), presc_umax=(Um, 0.0))
    p = O.make_problem(prob)
    f = O.rest_state(p)
    b = O.new_body(p)
    n = int(round(2 * math.pi * A / Um))
    h = O.run_body(p, O.body_params(prob), b, f, X, n)
    t = np.arange(1, n + 1)            # the state after a step is that of the next step
    assert np.allclose(h[:, 0], 32.0 - A * np.sin(Um * t / A), atol=1e-13)
    assert np.allclose(h[:, 2], -Um * np.cos(Um * t / A), atol=1e-15)
    assert np.all(h[:, 1] == 32.0)
    work = (h[:, 6] * (-Um * np.cos(Um * (t - 1) / A))).sum()   # F of step s with U_c of step s
    assert work < 0.0


def test_uniform_inflow_side_carries_a_uniform_stream():
    # Uniform inflow u_max on x-low, outflow on x-high, periodic in y: the
    # steady state is the uniform stream itself.
    prob = W.Problem(nx=32, ny=8, tau=0.7, collision=W.MRT,
                     bc=(W.BC_INLET_UNIFORM, W.BC_OUTLET, W.BC_PERIODIC, W.BC_PERIODIC),
                     u_max=0.03)
    p = O.make_problem(prob)
    f = O.rest_state(p)
    O.run(p, f, None, 4000)
    _, ux, uy = O.moments(p, f)
    assert np.abs(ux - 0.03).max() < 1e-6
    assert np.abs(uy).max() < 1e-12
