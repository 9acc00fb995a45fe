"""Pins of the oracle's D3Q19 multiple-relaxation-time collision (reading
R30), no GPU: the basis rows are orthogonal and their first moments are mass
and momentum; with every rate 1/tau the collision is the SRT one; mass and
momentum are conserved; a shear wave decays at the viscosity the rate 1/tau
fixes, nu = (tau - 1/2)/3, while a different rate on the energy moments
leaves that decay alone.
"""
import math

import numpy as np
import pytest

from oracle import d3q19 as O3
from paper_2003_12186_amd import workloads as W


def test_basis_rows_are_orthogonal_and_start_with_rho_and_j():
    M = O3.basis()
    ex, ey, ez, w = O3.lattice()
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)), atol=1e-12)
    assert np.allclose(M[0], 1.0) and np.allclose(M[3], ex) and np.allclose(M[5], ey) and np.allclose(M[7], ez)
    # the rest populations are reached by rho, e and eps only
    assert np.count_nonzero(M[:, 0]) == 3
    # the viscous stress rows are traceless quadratic forms
    assert np.allclose(M[9], 3 * ex ** 2 - (ex ** 2 + ey ** 2 + ez ** 2))
    assert np.allclose(M[13], ex * ey)
    # every non-conserved moment of the equilibrium at rest is a multiple of rho
    feq = O3.equilibrium(1.0, 0.0, 0.0, 0.0)
    m = M @ feq
    assert m[0] == pytest.approx(1.0) and np.allclose(m[[3, 5, 7, 9, 11, 13, 14, 15, 16, 17, 18]], 0, atol=1e-15)


def _noisy(p, seed):
    _, _, _, w = O3.lattice()
    return np.ascontiguousarray(w[:, None, None, None]
                                * (1.0 + 1e-2 * W.seeded_noise((19, p.nz, p.ny, p.nx), 64, seed)))


def test_mrt_with_every_rate_one_over_tau_is_srt():
    tau = 0.73
    a = O3.make_problem(W.Problem3(nx=10, ny=12, nz=14, tau=tau, body_force=(1e-5, 2e-5, -1e-5)))
    b = O3.make_problem(W.Problem3(nx=10, ny=12, nz=14, tau=tau, body_force=(1e-5, 2e-5, -1e-5),
                                   collision=W.MRT))
    for k in range(19):
        b.s[k] = 1.0 / tau
    f = _noisy(a, 0)
    g = f.copy()
    O3.run(a, f, None, 5)
    O3.run(b, g, None, 5)
    assert np.abs(f - g).max() < 1e-15


def test_mrt_conserves_mass_and_momentum():
    p = O3.make_problem(W.Problem3(nx=10, ny=12, nz=14, tau=0.6, collision=W.MRT))
    f = _noisy(p, 1)
    m0 = [a.sum() for a in O3.moments(p, f)]
    O3.run(p, f, None, 10)
    m1 = [a.sum() for a in O3.moments(p, f)]
    assert np.allclose(m0, m1, atol=1e-12)
    # and it differs from SRT on the same state
    q = O3.make_problem(W.Problem3(nx=10, ny=12, nz=14, tau=0.6))
    g = _noisy(q, 1)
    O3.run(q, g, None, 10)
    assert np.abs(f - g).max() > 1e-6


def _shear_nu(L, energy_rate, tau=0.8, U=1e-4):
    """Decay rate of u_x = U sin(2 pi y / L) over the viscous time 200 (L/32)^2
    steps after 20, divided by k^2: the measured viscosity."""
    p = O3.make_problem(W.Problem3(nx=4, ny=L, nz=4, tau=tau, collision=W.MRT))
    p.s[1] = energy_rate
    y = np.arange(L)
    ux = U * np.sin(2 * np.pi * y / L)
    f = np.zeros((19, 4, L, 4))
    for j in range(L):
        f[:, :, j, :] = O3.equilibrium(1.0, ux[j], 0.0, 0.0)[:, None, None]
    f = np.ascontiguousarray(f)
    O3.run(p, f, None, 20)
    a0 = O3.moments(p, f)[1][0, :, 0] @ np.sin(2 * np.pi * y / L)
    n = int(200 * (L / 32) ** 2)
    O3.run(p, f, None, n)
    a1 = O3.moments(p, f)[1][0, :, 0] @ np.sin(2 * np.pi * y / L)
    return -math.log(a1 / a0) / (n * (2 * np.pi / L) ** 2)


def test_shear_wave_decays_at_the_viscosity_of_tau():
    # nu -> (tau - 1/2)/3 at second order in k (error / 4 when L doubles);
    # the energy moment's rate does not enter (the wave never excites it)
    tau = 0.8
    nu0 = (tau - 0.5) / 3.0
    e32, e64 = _shear_nu(32, 1.19) - nu0, _shear_nu(64, 1.19) - nu0
    assert abs(e64) < 1e-3 * nu0
    assert 3.5 < e32 / e64 < 4.5
    assert abs(_shear_nu(32, 1.6) - nu0 - e32) < 1e-12
