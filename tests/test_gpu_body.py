"""GPU parity of the moving rigid circle (Sec. 2.3; through the C ABI)
against the FP64 CPU oracle: prescribed harmonic motion (Sec. 4.4) and a
free, spring-mounted body in a stream (the set-up of Sec. 4.5 at a small
size), with the body state, forces and velocity field compared; checkpoint
and restart of a moving body.

Tolerances: velocity field relative L2 <= 1e-6 (FP32 storage, FP64
collision arithmetic) and force to 1e-6 of its largest component.  A
prescribed path is exact.  A free body integrates its force twice, and its
lift is a small difference of stream-sized direct-forcing terms, which
carries the FP32 storage rounding of the stream (2^-24 of U per node, about
5e-6 of the lift here): measured 2.3e-6 lu after 2000 steps, so the bounds
are 1e-5 lu on the centre and 1e-3 of the largest body velocity.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2003_12186_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B(require_gpu):
    from paper_2003_12186_amd import binding
    binding.load()
    return binding


def _rel_l2(ug, vg, uo, vo):
    return np.sqrt(((ug - uo) ** 2 + (vg - vo) ** 2).sum() / (uo ** 2 + vo ** 2).sum())


def _box_body(mode, **kw):
    L, R, n = 64, 6.0, 40
    prob = W.Problem(nx=L, ny=L, tau=0.8, collision=W.MRT, interface=W.IF_RIGID,
                     force_mode=mode, n_markers=n, dX=2 * math.pi * R / n,
                     center=(L / 2.0, L / 2.0), radius=R, math=W.MATH_FP64, **kw)
    return prob, W.circle_markers(L / 2.0, L / 2.0, R, n)


def _stream_body(mode, u_red=5.0):
    """A small copy of the cylinder of Sec. 4.5: uniform stream U from the left,
    outflow on the right, the sides moving with the stream; D = 8 free in y on
    a spring with U_red = U / (f_N D), rho* = 8 / pi, no damping."""
    D, U = 8.0, 0.05
    nx, ny = 160, 80
    R = D / 2.0
    n = int(math.ceil(math.pi * D))
    nu = U * D / 100.0
    rho_star = 8.0 / math.pi
    m = rho_star * math.pi * R * R
    fN = U / (u_red * D)
    k = m * (2.0 * math.pi * fN) ** 2
    prob = W.Problem(nx=nx, ny=ny, tau=0.5 + 3.0 * nu, collision=W.MRT,
                     bc=(W.BC_INLET_UNIFORM, W.BC_OUTLET, W.BC_WALL, W.BC_WALL),
                     u_max=U, u_wall=(0.0, 0.0, U, U), interface=W.IF_RIGID, force_mode=mode,
                     n_markers=n, dX=math.pi * D / n, center=(40.0, 40.0), radius=R,
                     body_free=2, rho_star=rho_star, spring=(0.0, k), math=W.MATH_FP64)
    return prob, W.circle_markers(40.0, 40.0, R, n)


def _compare(B, prob, X0, steps, chunk):
    sim = B.Sim([prob], [X0])
    p = O.make_problem(prob)
    bp = O.body_params(prob)
    b = O.new_body(p)
    f = O.rest_state(p)
    X = X0.copy()
    worst = {"c": 0.0, "U": 0.0, "F": 0.0}
    Umax = Fmax = 1e-30
    for _ in range(steps // chunk):
        sim.step(chunk)
        h = O.run_body(p, bp, b, f, X, chunk)
        g = sim.body()
        assert g["steps"] == int(b.n)
        Umax = max(Umax, np.abs(h[:, 2:4]).max())
        Fmax = max(Fmax, np.abs(h[:, 6:8]).max())
        worst["c"] = max(worst["c"], np.abs(g["c"] - h[-1, 0:2]).max())
        worst["U"] = max(worst["U"], np.abs(g["U"] - h[-1, 2:4]).max())
        worst["F"] = max(worst["F"], np.abs(g["F"] - h[-1, 6:8]).max())
    gf = sim.fields(B.F_UX | B.F_UY)
    _, ux, uy = O.moments(p, f)
    err = _rel_l2(gf[0], gf[1], ux, uy)
    return sim, err, worst, Umax, Fmax, h


@pytest.mark.parametrize("mode", [W.FORCE_II_LBM, W.FORCE_IB_LBM])
def test_prescribed_harmonic_motion(B, mode):
    A, Um = 4.0, 0.02
    prob, X0 = _box_body(mode, presc_amp=(A, 0.0), presc_umax=(Um, 0.0))
    _say(f"prescribed harmonic motion 64^2 R=6 force_mode={mode}, 1200 steps")
    sim, err, worst, Umax, Fmax, h = _compare(B, prob, X0, 1200, 100)
    _say(f"  rel L2 u = {err:.3e}  |dc| {worst['c']:.2e}  |dU| {worst['U']:.2e}  "
         f"|dF|/Fmax {worst['F'] / Fmax:.2e}")
    assert err <= 1e-6
    assert worst["c"] <= 1e-12          # the prescribed path itself
    assert worst["F"] <= 1e-6 * Fmax
    sim.close()


@pytest.mark.parametrize("mode", [W.FORCE_II_LBM, W.FORCE_IB_LBM])
def test_spring_mounted_body_in_a_stream(B, mode):
    prob, X0 = _stream_body(mode)
    _say(f"spring-mounted circle D=8 in a stream 160x80 force_mode={mode}, 2000 steps")
    sim, err, worst, Umax, Fmax, h = _compare(B, prob, X0, 2000, 200)
    _say(f"  rel L2 u = {err:.3e}  |dc| {worst['c']:.2e}  |dU|/Umax {worst['U'] / Umax:.2e}  "
         f"|dF|/Fmax {worst['F'] / Fmax:.2e}  y-y0 {h[-1, 1] - 40.0:.4e}")
    assert err <= 1e-6
    assert worst["c"] <= 1e-5
    assert worst["U"] <= 1e-3 * Umax
    assert worst["F"] <= 1e-6 * Fmax
    assert sim.diag()["error_bits"] == 0
    sim.close()


def test_free_translation_and_rotation(B):
    # All three axes free (rho* = 1.5) in a periodic box with a noisy fluid:
    # centre, velocity and angle against the oracle.
    prob, X0 = _box_body(W.FORCE_II_LBM, body_free=7, rho_star=1.5)
    sim = B.Sim([prob], [X0])
    p = O.make_problem(prob)
    _, _, wt = O.d2q9()
    f0 = np.ascontiguousarray(wt[:, None, None] * (1.0 + 2e-3 * W.seeded_noise((9, 64, 64), 96, 0)))
    sim.set_distrib(f0)
    f = f0.copy()
    b = O.new_body(p)
    X = X0.copy()
    sim.step(600)
    h = O.run_body(p, O.body_params(prob), b, f, X, 600)
    g = sim.body()
    _say(f"free 3-DOF circle 600 steps: c {g['c']} vs {h[-1, 0:2]}, theta {g['theta']:.3e} vs {h[-1, 4]:.3e}")
    assert np.abs(g["c"] - h[-1, 0:2]).max() <= 1e-5
    assert abs(g["theta"] - h[-1, 4]) <= 1e-3 * np.abs(h[:, 4]).max() + 1e-12
    assert abs(g["W"] - h[-1, 5]) <= 1e-3 * np.abs(h[:, 5]).max() + 1e-15
    gf = sim.fields(B.F_UX | B.F_UY)
    _, ux, uy = O.moments(p, f)
    assert _rel_l2(gf[0], gf[1], ux, uy) <= 1e-6
    sim.close()


def test_moving_body_checkpoint_restart_and_fixed_body_has_no_state(B):
    prob, X0 = _stream_body(W.FORCE_II_LBM)
    a = B.Sim([prob], [X0])
    a.step(300)
    blob = a.save_state()
    a.step(300)
    b = B.Sim([prob], [X0])
    b.load_state(blob)
    b.step(300)
    assert np.array_equal(a.fields(B.F_UX | B.F_UY), b.fields(B.F_UX | B.F_UY))
    assert np.array_equal(a.body()["c"], b.body()["c"]) and a.body()["steps"] == b.body()["steps"]
    a.close()
    b.close()
    w = W.cylinder_channel(re=20.0, small=True)
    fixed = B.Sim([w.problem], [w.X0])
    with pytest.raises(B.IILBMError) as e:
        fixed.body()
    assert e.value.code == B.EINVAL
    fixed.close()


@pytest.mark.parametrize("kind", ["fixed", "prescribed"])
def test_graph_steps_report_the_last_steps_links(B, kind):
    # A graph builds the cut-link records on its last step only: after calls
    # that end on a long graph (64), a direct step (3 = pair + 1) and a pair
    # graph (66 = 64 + 2), the reported links, the field and the diagnostics
    # equal those of direct steps, each of which records.
    if kind == "fixed":
        w = W.cylinder_channel(re=20.0, small=True)
        prob, X0 = w.problem, w.X0
    else:
        prob, X0 = _box_body(W.FORCE_II_LBM, presc_amp=(4.0, 0.0), presc_umax=(0.02, 0.0))
    _say(f"rigid {kind}: graph replays against direct steps, links after 64, 67 and 133 steps")
    g = B.Sim([prob], [X0])
    g.set_graph(True)
    d = B.Sim([prob], [X0])
    d.set_graph(False)
    order = lambda r: r[np.lexsort((r["seg"], r["dir"], r["y"], r["x"]))]
    for n in (64, 3, 66):
        g.step(n)
        d.step(n)
        lg, ld = g.cutlinks(), d.cutlinks()
        assert len(lg) > 10 and np.array_equal(order(lg), order(ld))
        assert np.array_equal(g.fields(B.F_UX | B.F_UY), d.fields(B.F_UX | B.F_UY))
        assert g.diag()["n_cut_links"] == d.diag()["n_cut_links"] == len(ld)
    g.close()
    d.close()
