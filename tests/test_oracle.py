"""Pins of the CPU FP64 oracle against what the paper and the mathematics fix.

Each check would fail for a plausible slip in the oracle: a dropped or wrongly
signed term of Eq. 3, a missing F/2 in the velocity, a wrong opposite
direction in the bounce-back, a wrong weight, a transposed index in the pull.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_1611_02445_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore")


# --------------------------------------------------------------------------
# lattice (Section 2.2 and Fig. 1 caption): exact rational invariants
# --------------------------------------------------------------------------
def test_lattice_invariants_exact():
    c, w, opp = O.lattice()
    wf = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12
    assert [Fraction(x).limit_denominator(100) for x in w] == wf
    assert tuple(c[3]) == (-1, 0, 0)  # e_3 = W (Fig. 1 caption)
    assert sum(wf) == 1
    for a in range(3):
        assert sum(wf[i] * c[i, a] for i in range(19)) == 0
        for b in range(3):
            m2 = sum(wf[i] * c[i, a] * c[i, b] for i in range(19))
            assert m2 == (Fraction(1, 3) if a == b else 0)
    for a in range(3):
        for b in range(3):
            for g in range(3):
                assert sum(wf[i] * c[i, a] * c[i, b] * c[i, g] for i in range(19)) == 0
                for d in range(3):
                    m4 = sum(wf[i] * c[i, a] * c[i, b] * c[i, g] * c[i, d] for i in range(19))
                    iso = Fraction((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g), 9)
                    assert m4 == iso
    for i in range(19):
        assert np.all(c[opp[i]] == -c[i])
    # 1..6 axis, 7..18 edges (weights list after Eq. 4)
    assert all(np.abs(c[i]).sum() == 1 for i in range(1, 7))
    assert all(np.abs(c[i]).sum() == 2 for i in range(7, 19))
    assert len({tuple(v) for v in c}) == 19


# --------------------------------------------------------------------------
# equilibrium (Eq. 3, Eq. 4) and forcing moments
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model", [0, 1])
def test_equilibrium_moments(model):
    c, w, _ = O.lattice()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.uniform(-1, 1)
        u = 0.05 * rng.uniform(-1, 1, 3)
        fe = O.feq(rho, u, model)
        assert abs(fe.sum() - rho) <= 1e-15 * rho
        j = c.T @ fe
        expect_j = rho * u if model == 0 else u
        assert np.abs(j - expect_j).max() <= 1e-16
        P = np.einsum("i,ia,ib->ab", fe, c, c)
        if model == 0:
            expect_P = rho / 3.0 * np.eye(3) + rho * np.outer(u, u)
        else:
            expect_P = rho / 3.0 * np.eye(3) + np.outer(u, u)
        assert np.abs(P - expect_P).max() <= 1e-15


def test_guo_source_moments():
    c, w, _ = O.lattice()
    rng = np.random.default_rng(2)
    for tau in (0.55, 0.8, 1.7):
        for _ in range(10):
            u = 0.05 * rng.uniform(-1, 1, 3)
            F = 1e-4 * rng.uniform(-1, 1, 3)
            S = O.guo(tau, u, F)
            scale = np.abs(S).max()
            assert abs(S.sum()) <= 1e-14 * scale
            assert np.abs(c.T @ S - (1 - 1 / (2 * tau)) * F).max() <= 1e-14 * scale
            # second moment: (1 - 1/2tau)(u F + F u)
            P = np.einsum("i,ia,ib->ab", S, c, c)
            expect = (1 - 1 / (2 * tau)) * (np.outer(u, F) + np.outer(F, u))
            assert np.abs(P - expect).max() <= 1e-13 * np.abs(expect).max()


def test_collision_conserves_mass_and_adds_force():
    c, w, _ = O.lattice()
    rng = np.random.default_rng(3)
    for tau in (0.6, 0.8, 1.3):
        fin = w * (1 + 0.05 * rng.uniform(-1, 1, 19))
        F = 1e-5 * rng.uniform(-1, 1, 3)
        fo = O.collide_node(fin, F, tau)
        assert abs(fo.sum() - fin.sum()) <= 1e-15
        assert np.abs(c.T @ fo - (c.T @ fin + F)).max() <= 1e-16
        # relaxation of the non-equilibrium part at rate 1/tau (no force)
        fo0 = O.collide_node(fin, [0, 0, 0], tau)
        rho = fin.sum()
        u = (c.T @ fin) / rho
        fe = O.feq(rho, u)
        assert np.abs((fo0 - fe) - (1 - 1 / tau) * (fin - fe)).max() <= 1e-16


# --------------------------------------------------------------------------
# whole-box closed forms
# --------------------------------------------------------------------------
def test_rest_state_stays_at_rest():
    solid, _ = I.sphere_pack((16, 16, 16), 0.6, 2.0, 4.0, seed=11)
    f0 = O.init(solid)
    f = O.run(f0, solid, 0.8, 1000, periodic=7)
    assert np.abs(f - f0).max() <= 1e-15


def test_free_acceleration_closed_form():
    # fully fluid periodic box from rest under uniform F: every collision adds F
    # of momentum, so u = (n - 1/2) F / rho0 after n steps (u from stored f*)
    solid = I.fluid_box(8, 8, 8)
    F = np.array([1e-5, 2e-6, -3e-6])
    n = 37
    f = O.run(O.init(solid), solid, 0.8, n, force=F, periodic=7)
    rho, u = O.macroscopic(f, solid, force=F)
    for a in range(3):
        # rounding floor of a sum of 19 terms of size ~0.05 is ~1e-16 absolute
        assert np.abs(u[a] - (n - 0.5) * F[a]).max() <= 1e-15 + 1e-13 * abs((n - 0.5) * F[a])
    assert np.abs(rho - 1.0).max() <= 1e-14


@pytest.mark.parametrize("tau,H", [(0.8, 8), (0.65, 10), (1.2, 6), (0.5 + math.sqrt(3) / 4, 8)])
def test_plane_poiseuille_closed_form(tau, H):
    # steady BGK + Guo + halfway bounce-back between walls normal to y:
    # u(y) = g/(2 nu) (H^2/4 - y^2) + g (6 nu - 1/(8 nu)),  y from the centre
    nu = (tau - 0.5) / 3.0
    g = 1e-6
    solid = I.plane_channel(4, H, 4)
    steps = int(8 * H * H / nu)
    f = O.run(O.init(solid), solid, tau, steps, force=[g, 0, 0], periodic=7)
    rho, u = O.macroscopic(f, solid, force=[g, 0, 0])
    ux = u[0][:, 1:-1, :]
    y = np.arange(H) - (H - 1) / 2.0
    exact = g / (2 * nu) * (H * H / 4 - y * y) + g * (6 * nu - 1 / (8 * nu))
    assert np.abs(ux - exact[None, :, None]).max() <= 1e-6 * exact.max()
    # no cross flow beyond the rounding floor of the moment sums
    assert np.abs(u[1]).max() <= 1e-14 and np.abs(u[2]).max() <= 1e-14
    # permeability of the box: k = nu q / g, q = superficial flux
    k_fluid = (H * H - 1) / 12.0 + 6 * nu * nu
    k = O.permeability(f, solid, tau, g, force=[g, 0, 0])
    assert abs(k - k_fluid * H / (H + 2)) <= 1e-6 * k_fluid


def duct_series(H, g, nu, t, yy, zz, terms=199):
    out = np.zeros_like(yy, dtype=np.float64)
    for m in range(1, terms + 1, 2):
        for n in range(1, terms + 1, 2):
            lam = math.pi ** 2 * (m * m + n * n) / H ** 2
            out += (16 * g / (math.pi ** 2 * m * n * nu * lam) * np.sin(m * math.pi * yy / H)
                    * np.sin(n * math.pi * zz / H) * (1 - math.exp(-nu * lam * t)))
    return out


def test_square_duct_startup_series_500_steps():
    # 32^3 box, one-node walls on the y and z faces, tau = 0.8, g_x = 1e-6,
    # 500 steps: compare with the start-up series of a duct of side 30 whose
    # walls sit half-way between the wall nodes and the first fluid nodes
    tau, g, n = 0.8, 1e-6, 500
    nu = (tau - 0.5) / 3
    solid = I.square_channel(32)
    f0 = O.init(solid)
    f = O.run(f0, solid, tau, n, force=[g, 0, 0], periodic=7)
    rho, u = O.macroscopic(f, solid, force=[g, 0, 0])
    H = 30
    coords = np.arange(1, 31) - 0.5
    zz, yy = np.meshgrid(coords, coords, indexing="ij")
    ref = duct_series(H, g, nu, n - 0.5, yy, zz)
    ux = u[0][1:31, 1:31, :]
    centre = ref.max()
    assert abs(centre - 4.163e-4) < 2e-6
    err = np.sqrt(np.mean((ux - ref[:, :, None]) ** 2))
    assert err <= 0.01 * centre
    # mass conservation (streaming permutes, collision conserves)
    fl = solid == 0
    m0 = O.macroscopic(f0, solid)[0][fl].sum()
    assert abs(rho[fl].sum() - m0) / m0 <= 1e-13


def test_mass_conserved_sparse_geometry():
    solid, _ = I.sphere_pack((20, 20, 20), 0.5, 2.0, 5.0, seed=5)
    rng = np.random.default_rng(9)
    f0 = O.init(solid) * (1 + 0.01 * rng.uniform(-1, 1, (19,) + solid.shape))
    f = O.run(f0, solid, 0.7, 200, force=[1e-5, -2e-6, 0], periodic=7)
    s0 = O.sums(f0, solid)
    s1 = O.sums(f, solid, force=[1e-5, -2e-6, 0])
    assert abs(s1[0] - s0[0]) / s0[0] <= 1e-13


def test_shear_wave_viscosity():
    # linear shear wave in a periodic fluid box decays as exp(-nu k^2 t),
    # nu = (tau - 1/2)/3 (the viscosity relation after Eq. 2)
    tau = 0.8
    nu = (tau - 0.5) / 3
    L, U = 64, 1e-4
    solid = I.fluid_box(4, L, 4)
    k = 2 * math.pi / L
    y = np.arange(L)
    f = np.zeros((19, 4, L, 4))
    for yy in range(L):
        f[:, :, yy, :] = O.feq(1.0, [U * math.sin(k * yy), 0, 0])[:, None, None]

    def amp(f):
        _, u = O.macroscopic(f, solid)
        return 2 * np.mean(u[0][0, :, 0] * np.sin(k * y))

    f1 = O.run(f, solid, tau, 100, periodic=7)
    f2 = O.run(f1, solid, tau, 900, periodic=7)
    rate = math.log(amp(f1) / amp(f2)) / 900
    assert abs(rate / (nu * k * k) - 1) <= 1e-3


def test_step_nodes_matches_full_step():
    solid, _ = I.sphere_pack((12, 12, 12), 0.5, 2.0, 3.5, seed=4)
    rng = np.random.default_rng(5)
    f0 = O.init(solid) * (1 + 0.01 * rng.uniform(-1, 1, (19,) + solid.shape))
    f1 = O.step(f0, solid, 0.7, force=[1e-5, 0, 0], periodic=7)
    nodes = rng.choice(solid.size, 50, replace=False)
    out = O.step_nodes(f0, solid, 0.7, nodes, force=[1e-5, 0, 0], periodic=7)
    ref = f1.reshape(19, -1)[:, nodes].T
    assert np.array_equal(out, ref)


def test_bounce_back_uses_opposite_slot():
    # one fluid node surrounded by solid: every read bounces back, so the
    # gathered values are s_opp(i) at the node itself
    solid = np.ones((4, 4, 4), dtype=np.uint8)
    solid[1, 2, 1] = 0
    c, w, opp = O.lattice()
    rng = np.random.default_rng(0)
    s = rng.uniform(0.01, 0.1, (19, 4, 4, 4))
    g = O.pull(s, solid)
    node = (1, 2, 1)
    for i in range(19):
        assert g[(i,) + node] == s[(opp[i],) + node]


def test_pull_reads_upstream_neighbour():
    # fully fluid periodic box: g_i(x) = s_i(x - c_i)
    c, _, _ = O.lattice()
    solid = I.fluid_box(5, 6, 7)
    rng = np.random.default_rng(0)
    s = rng.uniform(size=(19,) + solid.shape)
    g = O.pull(s, solid, periodic=7)
    for i in range(19):
        shifted = np.roll(s[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(g[i], shifted)
