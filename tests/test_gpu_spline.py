"""GPU parity of the cubic-spline membrane (reading R27; through the C ABI)
against the FP64 CPU oracle: the crossings of a wobbly membrane (the same
links, signs and segments; parameters and jumps to 1e-9), and the 64 x 64
membrane over 1000 steps (relative L2 velocity <= 1e-6 with FP32 storage and
FP64 collision arithmetic, markers within 1e-6 lu).

The GPU takes the spline's second derivatives from the closed-form inverse of
the cyclic system, the oracle from a cyclic tridiagonal solve; the two agree
to rounding, so a crossing whose link parameter lies within 1e-9 of a link end
may fall on either side and is the only allowed difference.
"""
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


def _wobbly(n, seed):
    th = 2 * np.pi * np.arange(n) / n
    r = 11.0 + 1.5 * np.cos(3 * th + 0.4) + 0.2 * W.seeded_noise((n,), 97, seed)
    return np.stack([31.3 + r * np.cos(th), 32.6 + 0.8 * r * np.sin(th)], 1)


@pytest.mark.parametrize("n,seed", [(40, 1), (90, 2)])
def test_spline_crossings_match_oracle(B, n, seed):
    X = _wobbly(n, seed)
    prob = W.Problem(nx=64, ny=64, tau=0.8, interface=W.IF_MEMBRANE, n_markers=n, kappa=0.05,
                     dX=2 * np.pi * 11.0 / n, geometry=W.GEOM_SPLINE, math=W.MATH_FP64)
    sim = B.Sim([prob], [X])
    got = sim.cutlinks()
    p = O.make_problem(prob)
    want = O.cutlinks_spline(p, X, O.marker_forces(p, X)["G"])
    key = lambda r: (int(r["x"]), int(r["y"]), int(r["dir"]), int(r["sigma"]), int(r["seg"]))
    g = {key(r): r for r in got}
    w = {key(r): r for r in want}
    only = set(g) ^ set(w)
    for k in only:
        r = g.get(k, w.get(k))
        assert min(r["q"], 1.0 - r["q"]) < 1e-9, f"crossing {k} differs and is not at a link end"
    common = sorted(set(g) & set(w))
    dt = max(abs(g[k]["theta"] - w[k]["theta"]) for k in common)
    djp = max(abs(g[k]["jp"] - w[k]["jp"]) for k in common) / np.abs(want["jp"]).max()
    _say(f"spline crossings n={n}: {len(got)} gpu / {len(want)} oracle, {len(only)} at link ends, "
         f"max |dt| {dt:.2e}, max |djp|/max {djp:.2e}")
    assert len(common) > 100
    assert dt < 1e-9 and djp < 1e-9
    sim.close()


@pytest.mark.parametrize("collision", [W.SRT, W.MRT])
def test_spline_membrane64_parity_1000_steps(B, collision):
    w = W.membrane_ellipse64()
    w.problem.geometry = W.GEOM_SPLINE
    w.problem.collision = collision
    w.problem.math = W.MATH_FP64
    _say(f"spline membrane 64x64 collision={collision}, 1000 steps")
    sim = B.Sim([w.problem], [w.X0])
    sim.step(1000)
    g = sim.fields(B.F_RHO | B.F_UX | B.F_UY)
    X = sim.markers()[0]
    p = O.make_problem(w.problem)
    f = O.rest_state(p)
    Xo = w.X0.copy()
    O.run(p, f, Xo, 1000)
    rho, ux, uy = O.moments(p, f)
    err = np.sqrt(((g[1] - ux) ** 2 + (g[2] - uy) ** 2).sum() / (ux ** 2 + uy ** 2).sum())
    dX = np.abs(X - Xo).max()
    _say(f"  rel L2 u = {err:.3e}  max |dX| = {dX:.3e}")
    assert err <= 1e-6
    assert dX <= 1e-6
    assert np.abs(g[0] - rho).max() < 1e-6
    assert sim.diag()["error_bits"] == 0
    sim.close()


def test_spline_membrane_with_guo_term(B):
    w = W.membrane_ellipse64()
    w.problem.geometry = W.GEOM_SPLINE
    w.problem.force_mode = W.FORCE_II_LBM_GUO
    w.problem.math = W.MATH_FP64
    sim = B.Sim([w.problem], [w.X0])
    sim.step(400)
    g = sim.fields(B.F_UX | B.F_UY)
    p = O.make_problem(w.problem)
    f = O.rest_state(p)
    Xo = w.X0.copy()
    O.run(p, f, Xo, 400)
    _, ux, uy = O.moments(p, f)
    err = np.sqrt(((g[0] - ux) ** 2 + (g[1] - uy) ** 2).sum() / (ux ** 2 + uy ** 2).sum())
    _say(f"spline membrane, II-LBM with Guo's term, 400 steps: rel L2 u = {err:.3e}")
    assert err <= 1e-6
    assert np.abs(sim.markers()[0] - Xo).max() <= 1e-6
    sim.close()
