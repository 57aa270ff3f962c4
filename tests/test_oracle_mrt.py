"""Pins of the oracle's multiple-relaxation-time operator (the LBMRT kernels of
Sections 2.2 and 4.6; the paper gives no matrix, so the moment basis is the
D3Q19 one of d'Humieres et al. 2002, with the Guo source carried into moment
space).  What fixes it independently of the code:
  - the moments are polynomials in c; their squared norms over the 19
    velocities are counted by hand below, and distinct moments are orthogonal;
  - with every rate equal to 1/tau the operator is the single-relaxation-time
    one (Eq. 2, 7 with Guo forcing) exactly;
  - the equilibrium moments M f_eq have closed forms, worked out by hand from
    the weights (sums of w_i c_i^n over the velocity set);
  - mass is conserved, momentum grows by exactly F, a rest state stays;
  - a steady plane channel has the curvature -g/nu of the Navier-Stokes
    solution, nu = (tau - 1/2)/3, in the bulk."""
import numpy as np
import pytest

import oracle as O
from paper_1611_02445_amd import inputs as I


def test_moment_basis_orthogonal_with_counted_norms():
    M, Minv = O.mrt_matrix()
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    # squared norms counted over rest (1), axis (6) and diagonal (12) velocities:
    # rho 19; e: 30^2 + 6*11^2 + 12*8^2 = 2394; eps: 12^2 + 6*4^2 + 12 = 252;
    # j_a: 2 + 8 = 10; q_a: 2*16 + 8 = 40; 3p_xx: 2*4 + 4*1 + 8*1 + 4*4 = 36;
    # 3pi_xx: 2*16 + 4*4 + 8*1 + 4*4 = 72; p_ww: 4 + 8 = 12; pi_ww: 4*4 + 8 = 24;
    # p_ab: 4; m_a: 8
    norms = [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
    assert np.array_equal(np.diag(G), np.array(norms, dtype=float))
    assert np.abs(M @ Minv - np.eye(19)).max() <= 1e-15 * 30


@pytest.mark.parametrize("model", [0, 1])
def test_equal_rates_give_the_single_relaxation_operator(model):
    rng = np.random.default_rng(3)
    _, w, _ = O.lattice()
    tau = 0.73
    for _ in range(5):
        fin = w * (1.0 + 0.05 * rng.uniform(-1, 1, 19))
        F = rng.normal(0, 1e-4, 3)
        mrt = O.collide_mrt_rates(fin, F, np.full(19, 1.0 / tau), model=model + 2)
        bgk = O.collide_node(fin, F, tau, model=model)
        assert np.abs(mrt - bgk).max() <= 1e-15


@pytest.mark.parametrize("model", [2, 3])
def test_equilibrium_moments_closed_forms(model):
    M, _ = O.mrt_matrix()
    rng = np.random.default_rng(4)
    for _ in range(5):
        rho = 1.0 + 0.05 * rng.uniform(-1, 1)
        u = rng.normal(0, 0.03, 3)
        ux, uy, uz = u
        feq = O.feq(rho, u, model=model & 1)
        m = M @ feq
        # quadratic terms carry rho (quasi-compressible) or not (incompressible)
        r2 = rho if model == 2 else 1.0
        j = rho * u if model == 2 else u
        uu = ux * ux + uy * uy + uz * uz
        pxx = r2 * (2 * ux * ux - uy * uy - uz * uz)
        pww = r2 * (uy * uy - uz * uz)
        expect = [rho, -11 * rho + 19 * r2 * uu, 3 * rho - 5.5 * r2 * uu,
                  j[0], -2.0 / 3.0 * j[0], j[1], -2.0 / 3.0 * j[1], j[2], -2.0 / 3.0 * j[2],
                  pxx, -0.5 * pxx, pww, -0.5 * pww,
                  r2 * ux * uy, r2 * uy * uz, r2 * ux * uz, 0.0, 0.0, 0.0]
        assert np.abs(m - np.array(expect)).max() <= 1e-14


@pytest.mark.parametrize("model", [2, 3])
def test_conservation_and_rest_state(model):
    c, w, _ = O.lattice()
    rng = np.random.default_rng(5)
    tau = 0.9
    for _ in range(5):
        fin = w * (1.0 + 0.05 * rng.uniform(-1, 1, 19))
        F = rng.normal(0, 1e-4, 3)
        out = O.collide_node(fin, F, tau, model=model)
        assert abs(out.sum() - fin.sum()) <= 1e-15
        assert np.abs(c.T @ out - c.T @ fin - F).max() <= 1e-16
    # the rest state is a fixed point; the two moment transforms round it by
    # a few ulp of the largest f_i
    rest = O.collide_node(w.copy(), np.zeros(3), tau, model=model)
    assert np.abs(rest - w).max() <= 8 * 2.0 ** -53 * w.max()


@pytest.mark.parametrize("tau,model", [(0.6, 2), (0.8, 2), (1.1, 3)])
def test_plane_channel_curvature(tau, model):
    H, g = 10, 1e-6
    nu = (tau - 0.5) / 3.0
    solid = I.plane_channel(4, H, 4)
    steps = int(10 * H * H / nu)
    f = O.run(O.init(solid, model=model), solid, tau, steps, force=[g, 0, 0], periodic=7, model=model)
    _, u = O.macroscopic(f, solid, force=[g, 0, 0], model=model)
    ux = u[0][:, 1:-1, :]
    d2 = ux[:, 2:, :] - 2 * ux[:, 1:-1, :] + ux[:, :-2, :]
    assert np.abs(d2 / (-g / nu) - 1.0).max() <= 1e-8
    assert np.abs(u[1]).max() <= 1e-14 and np.abs(u[2]).max() <= 1e-14


def test_viscous_rates():
    s = O.mrt_rates(0.8)
    for k in (9, 11, 13, 14, 15):
        assert s[k] == 1.0 / 0.8
