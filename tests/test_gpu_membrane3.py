"""GPU parity of the deformable triangulated membrane under surface tension
in D3Q19 (reading R31; through ii_lbm3_set_membrane / ii_lbm3_membrane)
against the FP64 CPU oracle: a stretched drop relaxing for 200 steps under
SRT and MRT (vertices and flow); and the stop when the surface leaves the
supported region, forced from the host with a body force.
"""
import sys

import numpy as np
import pytest

from oracle import d3q19 as O3
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


def _rel(g, o):
    return np.sqrt(sum(((g[a] - o[a]) ** 2).sum() for a in (1, 2, 3)) / sum((o[a] ** 2).sum() for a in (1, 2, 3)))


@pytest.mark.parametrize("coll,mode", [(W.SRT, W.FORCE_II_LBM), (W.MRT, W.FORCE_II_LBM),
                                       (W.SRT, W.FORCE_IB_LBM)])
def test_relaxing_drop_matches_oracle(B, coll, mode):
    n, steps, gamma = 26, 200, 0.01
    prob = W.Problem3(nx=n, ny=n + 1, nz=n + 2, tau=1.0, collision=coll, force_mode=mode)
    X0, tri = W.ellipsoid_membrane((13.1, 12.7, 13.4), (6.0, 4.5, 5.2))
    _say(f"D3Q19 membrane drop {len(X0)} vertices {len(tri)} triangles, collision={coll} force_mode={mode}, "
         f"{steps} steps")
    sim = B.Sim3(prob)
    sim.set_membrane(X0, tri, gamma)
    sim.step(steps)
    Xg, Ug = sim.membrane()
    g = sim.fields()
    p = O3.make_problem(prob)
    f = O3.rest_state(p)
    Xo = X0.copy()
    Uo = O3.run_membrane(p, f, Xo, tri, gamma, steps)
    o = O3.moments(p, f)
    err = _rel(g, o)
    dX = np.abs(Xg - Xo).max()
    dU = np.abs(Ug - Uo).max() / np.abs(Uo).max()
    moved = np.abs(Xo - X0).max()
    _say(f"  rel L2 u = {err:.3e}; max |dX| = {dX:.2e} lu (moved {moved:.3f}); max |dU|/max|U| = {dU:.2e}")
    # FP32 storage of the deviations: the velocity carries the storage's
    # 1e-7 relative rounding, as in the other D3Q19 cases; positions add up
    # 200 such velocities of at most 3e-3 lu per step
    assert err <= 1e-6
    assert dU <= 1e-5
    assert dX <= 1e-6
    assert moved > 0.05
    sim.close()


@pytest.mark.parametrize("mode", [W.FORCE_II_LBM, W.FORCE_IB_LBM])
def test_membrane_runs_are_bitwise_reproducible(B, mode):
    # The spread force field and the jumps of the cut links are summed in
    # fixed point, so two runs of the same problem agree bit for bit whatever
    # order the threads add their terms in.  A wrinkled surface (a drop with
    # a dented side) gives links cut more than once.
    n, steps, gamma = 26, 60, 0.01
    prob = W.Problem3(nx=n, ny=n + 1, nz=n + 2, tau=1.0, force_mode=mode)
    X0, tri = W.ellipsoid_membrane((13.1, 12.7, 13.4), (6.0, 4.5, 5.2))
    X0 = X0.copy()
    X0[:, 0] += 0.35 * np.sin(3.1 * X0[:, 1]) * np.cos(2.3 * X0[:, 2])
    _say(f"D3Q19 membrane force_mode={mode}: two runs of {steps} steps, bitwise")
    out = []
    for _ in range(2):
        sim = B.Sim3(prob)
        sim.set_membrane(X0, tri, gamma)
        sim.step(steps)
        Xg, Ug = sim.membrane()
        out.append((sim.fields(), Xg, Ug))
        sim.close()
    (ga, Xa, Ua), (gb, Xb, Ub) = out
    assert all(np.array_equal(ga[a], gb[a]) for a in range(len(ga)))
    assert np.array_equal(Xa, Xb) and np.array_equal(Ua, Ub)
    assert np.isfinite(Xa).all() and np.abs(Xa - X0).max() > 1e-3


def test_membrane_stops_when_it_leaves_the_region(B):
    # a uniform body force carries the drop towards the +x side; once a
    # vertex is past n - 3 the membrane stops and reports EGEOMETRY, while
    # the fluid keeps stepping
    n = 24
    prob = W.Problem3(nx=n, ny=n, nz=n, tau=0.8, body_force=(2e-4, 0.0, 0.0))
    X0, tri = W.icosphere((15.3, 12.2, 12.1), 3.5)
    sim = B.Sim3(prob)
    sim.set_membrane(X0, tri, 0.005)
    sim.step(10)
    X, _ = sim.membrane()
    assert X[:, 0].max() < n - 3
    sim.step(400)
    rc = B._lib3().ii_lbm3_membrane(sim.h, None, None)
    _say(f"D3Q19 membrane carried out of the region: code {rc}")
    assert rc == B.EGEOMETRY
    sim.step(5)
    g = sim.fields()
    assert np.isfinite(g).all() and g[1].mean() > 0.01
    sim.close()


def test_membrane_refuses_a_problem_with_a_sphere(B):
    prob, _, _ = W.normal_force_sphere(16, W.FORCE_II_LBM, re=20.0)
    X, tri = W.icosphere((10.3, 10.2, 10.1), 3.0)
    sim = B.Sim3(prob)
    Xc, tc, _ = B._mesh3_args(X, tri, 0.0)
    rc = B._lib3().ii_lbm3_set_membrane(sim.h, len(Xc), Xc.ctypes.data, len(tc), tc.ctypes.data, 0.01)
    assert rc == B.EINVAL
    sim.close()


@pytest.mark.parametrize("coll", [W.SRT, W.MRT])
def test_rigid_surface_matches_oracle(B, coll):
    # a fixed sphere held by direct forcing in a periodic box driven along x
    n, steps, g = 20, 300, 1e-5
    prob = W.Problem3(nx=n, ny=n + 1, nz=n + 2, tau=0.9, body_force=(g, 0.0, 0.0), collision=coll)
    X, tri = W.icosphere((10.27, 10.69, 11.13), 4.2)
    _say(f"D3Q19 rigid surface {len(X)} vertices, collision={coll}, {steps} steps")
    sim = B.Sim3(prob)
    sim.set_rigid_surface(X, tri)
    sim.step(steps)
    Xg, Ug = sim.membrane()
    Fg = sim.surface_force()
    gfl = sim.fields()
    p = O3.make_problem(prob)
    f = O3.rest_state(p)
    Uo, Fo = O3.run_rigid_surface(p, f, X, tri, steps)
    o = O3.moments(p, f)
    err = _rel(gfl, o)
    dF = np.abs(Fg - Fo).max() / np.abs(Fo).max()
    dU = np.abs(Ug - Uo).max() / np.abs(Uo).max()
    _say(f"  rel L2 u = {err:.3e}; force {Fg[0]:.6e} vs {Fo[0]:.6e} (rel {dF:.2e}); dU {dU:.2e}")
    assert np.abs(Xg - X).max() == 0.0
    assert err <= 1e-6
    # the force sums the vertex velocities, which carry the storage rounding
    assert dF <= 1e-5 and dU <= 1e-5
    sim.close()


def _stream3(p, U0):
    return np.ascontiguousarray(np.broadcast_to(O3.equilibrium(1.0, U0, 0.0, 0.0)[:, None, None, None],
                                                (19, p.nz, p.ny, p.nx))).copy()


@pytest.mark.parametrize("case", ["heavy_in_stream", "spinning"])
def test_free_sphere_matches_oracle(B, case):
    # the rigid-body update of Sec. 2.3 in three dimensions (reading R33)
    n, R, steps = 24, 4.0, 150
    prob = W.Problem3(nx=n, ny=n + 1, nz=n + 2, tau=0.8)
    if case == "heavy_in_stream":
        c, rs, U0, W0, ustream = (8.27, 11.69, 12.13), 4.0, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 0.01
    else:
        c, rs, U0, W0, ustream = (12.27, 11.69, 12.13), 2.0, (0.0, 0.0, 0.0), (0.001, -0.002, 0.005), 0.0
    X, tri = W.icosphere(c, R)
    p = O3.make_problem(prob)
    f0 = _stream3(p, ustream)
    _say(f"D3Q19 free sphere {case}: {len(X)} vertices, {steps} steps")
    sim = B.Sim3(prob)
    sim.set_distrib(f0)
    sim.set_free_sphere(X, tri, c, R, rs, U0, W0)
    sim.step(steps)
    bg = sim.body()
    Xg, _ = sim.membrane()
    g = sim.fields()
    f = f0.copy()
    Xo = X.copy()
    body = O3.new_body3(c, U0, W0)
    Fo, To = O3.run_free_sphere(p, f, Xo, tri, R, rs, body, steps)
    o = O3.moments(p, f)
    err = _rel(g, o)
    dc = np.abs(bg[0:3] - body[0:3]).max()
    dU = np.abs(bg[3:6] - body[3:6]).max() / max(np.abs(body[3:6]).max(), 1e-12)
    # the spin against the motion's own angular scale (a sphere carried
    # without spin keeps only a residual W of order 1e-8)
    dW = np.abs(bg[9:12] - body[9:12]).max() / max(np.abs(body[9:12]).max(), np.abs(body[3:6]).max() / R)
    _say(f"  rel L2 u = {err:.3e}; |dc| = {dc:.2e} lu; dU {dU:.2e}; dW {dW:.2e}; "
         f"U {bg[3]:.6f} W {bg[11]:.3e}; |dX| {np.abs(Xg - Xo).max():.2e}")
    assert err <= 1e-6
    assert dc <= 1e-6 and np.abs(Xg - Xo).max() <= 1e-6
    # the force sums vertex velocities that carry the FP32 storage's rounding
    assert dU <= 1e-5 and dW <= 1e-5
    sim.close()
