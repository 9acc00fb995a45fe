"""Pins of the oracle's fixed rigid triangulated surface with direct forcing
in D3Q19 (reading R32), no GPU: the force law G_v = (0 - U_v) A_v with the
jump and tangential parts it implies; and the steady momentum balance of a
periodic array of spheres driven by a uniform body force, where the force on
each sphere must carry the whole box's body force, g L^3.
"""
import numpy as np
import pytest

from oracle import d3q19 as O3
from paper_2003_12186_amd import workloads as W


def test_one_step_force_law_and_fixed_vertices():
    # from a noisy state the first step's force on the surface is
    # -sum (0 - U_v) A_v with U_v the interpolated velocity and A_v the
    # vertex areas; the vertices stay put
    n = 20
    p = O3.make_problem(W.Problem3(nx=n, ny=n, nz=n, tau=0.9))
    X, tri = W.icosphere((10.27, 9.69, 10.13), 4.2)
    _, _, _, w = O3.lattice()
    f = np.ascontiguousarray(w[:, None, None, None] * (1.0 + 1e-3 * W.seeded_noise((19, n, n, n), 72, 0)))
    U0 = O3.interp(p, f, X)
    A = O3.membrane_forces(X, tri, 0.0)["A"]
    U, F = O3.run_rigid_surface(p, f, X, tri, 1)
    assert np.abs(U - U0).max() == 0.0
    assert np.allclose(F, (U0 * A[:, None]).sum(0), rtol=1e-12, atol=1e-18)


def test_periodic_array_momentum_balance():
    # 16^3 box, sphere of radius 3.2, tau = 1, g = 1e-6 along x: after 1500
    # steps (about the viscous time L^2 / nu) the flow is steady and the force
    # on the sphere balances g L^3 within 2 % (the jumps carry the normal part
    # of sum G only up to the discretisation); the cross-stream force vanishes
    L, g = 16, 1e-6
    p = O3.make_problem(W.Problem3(nx=L, ny=L, nz=L, tau=1.0, body_force=(g, 0.0, 0.0)))
    X, tri = W.icosphere((8.27, 7.69, 8.13), 3.2)
    f = O3.rest_state(p)
    U, F = O3.run_rigid_surface(p, f, X, tri, 1500)
    assert F[0] / (g * L ** 3) == pytest.approx(1.0, abs=0.02)
    assert abs(F[1]) < 1e-3 * F[0] and abs(F[2]) < 1e-3 * F[0]
    # the surface holds the fluid back: its vertices move far slower than the mean flow
    ux = O3.moments(p, f)[1].mean()
    assert ux > 0 and np.abs(U).max() < 0.3 * ux
