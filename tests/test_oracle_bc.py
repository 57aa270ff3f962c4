"""Pins of the oracle's open boundaries (the Zou-He velocity inlet and
constant-pressure outlet the paper uses, Section 2.2), from what they must
satisfy by definition:
  - the rebuilt node has the prescribed velocity (inlet) or density and zero
    tangential velocity (outlet), and only the populations entering through
    the face change;
  - a rest state with zero inlet velocity and unit outlet density stays;
  - in a steady channel the mass flux through every cross-section is the
    same (the discrete scheme conserves mass node by node)."""
import numpy as np
import pytest

import oracle as O


def _random_node(seed):
    _, w, _ = O.lattice()
    rng = np.random.default_rng(seed)
    return w * (1.0 + 0.05 * rng.uniform(-1, 1, 19)), rng


def _code(axis, kind, n):
    """the rebuild code of a face: kind 'v' (velocity) or 'p' (pressure),
    n = c_axis of the unknown populations"""
    r = {("v", 1): 0, ("p", -1): 1, ("v", -1): 2, ("p", 1): 3}[(kind, n)]
    return 1 + 4 * axis + r


FACES = [(a, n) for a in range(3) for n in (1, -1)]


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("axis,n", FACES)
def test_inlet_rebuild_gives_the_prescribed_velocity(model, axis, n):
    c, _, _ = O.lattice()
    for seed in range(6):
        f, rng = _random_node(seed)
        u_in = rng.normal(0, 0.02, 3)
        F = rng.normal(0, 1e-4, 3)
        g = O.zou_he(f, _code(axis, "v", n), u_in=u_in, F=F, model=model)
        keep = c[:, axis] != n
        assert np.array_equal(g[keep], f[keep])
        rho, j = g.sum(), c.T @ g
        u = (j + 0.5 * F) / (rho if model == 0 else 1.0)
        assert np.abs(u - u_in).max() <= 1e-15


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("axis,n", FACES)
def test_outlet_rebuild_gives_the_prescribed_density(model, axis, n):
    c, _, _ = O.lattice()
    tang = [b for b in range(3) if b != axis]
    for seed in range(6):
        f, rng = _random_node(10 + seed)
        rho_out = 1.0 + 0.01 * rng.uniform(-1, 1)
        F = rng.normal(0, 1e-4, 3)
        g = O.zou_he(f, _code(axis, "p", n), rho_out=rho_out, F=F, model=model)
        keep = c[:, axis] != n
        assert np.array_equal(g[keep], f[keep])
        assert abs(g.sum() - rho_out) <= 1e-15
        j = c.T @ g
        assert np.abs(j[tang] + 0.5 * F[tang]).max() <= 1e-16


def test_codes_one_and_two_are_the_x_inlet_and_outlet():
    assert _code(0, "v", 1) == 1 and _code(0, "p", -1) == 2


def test_rebuild_is_covariant_under_axis_relabelling():
    """Rotating the lattice so that x goes to y maps the x-face rebuild to
    the y-face rebuild: the codes differ only by the axis."""
    c, _, _ = O.lattice()
    # permutation of the velocities for (x, y, z) -> (y, z, x)
    idx = {tuple(v): i for i, v in enumerate(c)}
    perm = np.array([idx[(v[2], v[0], v[1])] for v in c])  # direction i -> its image
    f, rng = _random_node(99)
    u_in = rng.normal(0, 0.02, 3)
    for kind, n in (("v", 1), ("p", -1), ("v", -1), ("p", 1)):
        gx = O.zou_he(f, _code(0, kind, n), u_in=u_in, rho_out=1.003)
        fy = np.empty(19)
        fy[perm] = f
        uy = np.array([u_in[2], u_in[0], u_in[1]])
        gy = O.zou_he(fy, _code(1, kind, n), u_in=uy, rho_out=1.003)
        assert np.abs(gy[perm] - gx).max() <= 1e-15


def _channel(nx, H, nz):
    """Walls (solid rows) at y = 0 and y = H + 1, periodic in z; inlet plane
    x = 0 and outlet plane x = nx - 1 on the fluid rows."""
    solid = np.zeros((nz, H + 2, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, -1, :] = 1
    bt = np.zeros_like(solid)
    bt[:, 1:-1, 0] = 1
    bt[:, 1:-1, -1] = 2
    return solid, bt


def test_rest_state_stays():
    solid, bt = _channel(16, 6, 4)
    f0 = O.init(solid)
    f = O.run_bc(f0, solid, 0.8, 200, bt, u_in=(0, 0, 0), rho_out=1.0, periodic=4)
    # a fixed point up to the rounding of the rebuild's sums (a few ulp of
    # 1/3 per step, relaxed back by the collision rather than accumulated)
    assert np.abs(f - f0).max() <= 16 * 2.0 ** -53 / 3.0


@pytest.mark.parametrize("model", [0, 2])
def test_steady_channel_flux_is_constant(model):
    # pressure waves bounce between the two open faces and die out slowly:
    # a short channel and a viscous fluid reach the steady state sooner
    nx, H, nz, tau = 16, 6, 4, 1.2
    solid, bt = _channel(nx, H, nz)
    u_in = (0.01, 0.0, 0.0)
    f = O.run_bc(O.init(solid, model=model), solid, tau, 40000, bt, u_in=u_in, rho_out=1.0, periodic=4,
                 model=model)
    rho, u = O.macroscopic(f, solid, model=model)
    flux = (rho * u[0]).sum(axis=(0, 1))  # per x plane
    inlet = rho[:, 1:-1, 0] * u_in[0]
    assert np.abs(u[0][:, 1:-1, 0] - u_in[0]).max() <= 1e-15
    assert np.abs(rho[:, 1:-1, -1] - 1.0).max() <= 1e-15
    assert np.abs(flux - inlet.sum()).max() <= 1e-9 * inlet.sum()
    assert np.abs(u[2]).max() <= 1e-14


def _couette(model, U, n=12):
    solid = np.zeros((n, 4, 4), np.uint8)
    solid[0] = 1
    bt = np.zeros_like(solid)
    bt[-1] = 11
    f = O.run_bc(O.init(solid, model=model), solid, 0.9, 6000, bt, u_in=(U, 0.0, 0.0), periodic=3,
                 model=model)
    _, u = O.macroscopic(f, solid, model=model)
    z = np.arange(1, n)
    return u, u[0][1:, 2, 2] - U * (z - 0.5) / (n - 1.5)


@pytest.mark.parametrize("model", [0, 1, 3])
def test_couette_flow_under_a_moving_velocity_layer(model):
    """Plane Couette flow: periodic in x and y, a wall below, the top layer a
    velocity node moving at U (code 11).  With halfway bounce-back the wall
    sits half a node below the first fluid layer, so the steady profile is
    u_x(z) = U (z - 1/2) / (n - 3/2) for fluid layers z = 1 .. n-1, exactly
    for both LBGK models and the incompressible LBMRT one."""
    u, dev = _couette(model, 0.03)
    assert np.abs(dev).max() <= 1e-9
    assert np.abs(u[1]).max() <= 1e-14 and np.abs(u[2]).max() <= 1e-12


def test_couette_quasi_compressible_lbmrt_deviates_at_third_order():
    """The quasi-compressible LBMRT operator carries rho into the quadratic
    equilibrium moments while its energy and normal-stress moments relax at
    their own rates, so a Couette flow picks up an O(U^2) density variation
    and an O(U^3) departure from the linear profile: halving U divides the
    departure by 8 (a first-order slip, i.e. a wrong wall or lid, would
    divide it by 2)."""
    _, d1 = _couette(2, 0.03)
    _, d2 = _couette(2, 0.015)
    ratio = np.abs(d1).max() / np.abs(d2).max()
    assert 7.0 <= ratio <= 9.0
    assert np.abs(d1).max() <= 1e-6


def _lid_amplification(model, s_m, tau, noise, steps=200, n=8):
    """Growth of a small random perturbation of the rest state over `steps`
    steps under a velocity layer at rest (code 11, u = 0) above a wall,
    periodic in x and y: max |f - f_rest| after over before."""
    solid = np.zeros((n, n, n), np.uint8)
    solid[0] = 1
    bt = np.zeros_like(solid)
    bt[-1] = 11
    rest = O.init(solid, model=model)
    rng = np.random.default_rng(1)
    f = rest * (1.0 + noise * rng.uniform(-1, 1, rest.shape))
    f[:, solid == 1] = 0.0
    d0 = np.abs(f - rest).max()
    with O.mrt_ghost_rates(s_m=s_m):
        f = O.run_bc(f, solid, tau, steps, bt, u_in=(0.0, 0.0, 0.0), periodic=3, model=model)
    return np.abs(f - rest).max() / d0


def test_velocity_layer_unstable_with_the_lbmrt_m_rate_at_small_tau():
    """The Zou-He velocity node combined with the multiple-relaxation-time
    operator has a linearly unstable mode when the rate of the third-order m
    moments is close to 2 and tau is small: at tau = 0.6 with the table's
    s_m = 1.98 a perturbation of the rest state grows ~2600-fold in 200 steps,
    by the same factor for perturbations 1000 times apart (a linear mode, not
    a nonlinear effect of the lid speed), for both equilibria.  The same layer
    damps it with s_m = 1.8, at tau = 0.8, or with the single-relaxation-time
    operator.  This is why the LBMRT rows of the dense lid-driven cavity study
    run the walled box without a lid: a lid at tau = 0.6 diverges in the oracle
    and in the kernel alike, whatever its speed."""
    a = _lid_amplification(2, 1.98, 0.6, 1e-12)
    b = _lid_amplification(2, 1.98, 0.6, 1e-9)
    assert a >= 100.0 and abs(a / b - 1.0) <= 0.01
    assert _lid_amplification(3, 1.98, 0.6, 1e-12) >= 100.0
    assert _lid_amplification(2, 1.8, 0.6, 1e-12) <= 0.1
    assert _lid_amplification(2, 1.98, 0.8, 1e-12) <= 0.1
    assert _lid_amplification(0, 1.98, 0.6, 1e-12) <= 0.1
