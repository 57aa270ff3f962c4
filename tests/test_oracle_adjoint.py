"""Pins of the oracle's discrete adjoint: transposes checked by dot products
and the whole reverse sweep checked against central finite differences of the
oracle's own forward steps."""
import numpy as np
import pytest

import oracle as O
from paper_1611_02445_amd import inputs as I


def _geom():
    solid, _ = I.sphere_pack((12, 12, 12), 0.55, 2.0, 3.5, seed=21)
    return solid


def test_pull_transpose_dot_product():
    solid = _geom()
    fl = (solid == 0)[None]
    rng = np.random.default_rng(1)
    for periodic in (7, 0, 5):
        v = rng.normal(size=(19,) + solid.shape) * fl
        w = rng.normal(size=(19,) + solid.shape) * fl
        lhs = np.sum(O.pull(v, solid, periodic) * w)
        rhs = np.sum(v * O.pull_transpose(w, solid, periodic))
        assert abs(lhs - rhs) <= 1e-14 * np.sum(np.abs(O.pull(v, solid, periodic) * w))


@pytest.mark.parametrize("model", [0, 1, 2, 3])
def test_collision_jt_against_central_differences(model):
    c, w, _ = O.lattice()
    rng = np.random.default_rng(2)
    for tau in (0.6, 0.8, 1.4):
        fin = w * (1 + 0.05 * rng.uniform(-1, 1, 19))
        F = 1e-4 * rng.uniform(-1, 1, 3)
        lam = rng.normal(size=19)
        eta, gF = O.collide_jt_node(fin, F, tau, lam, model=model)
        h = 1e-6
        for j in range(19):
            e = np.zeros(19)
            e[j] = h
            d = (O.collide_node(fin + e, F, tau, model=model) - O.collide_node(fin - e, F, tau, model=model)) / (2 * h)
            assert abs(d @ lam - eta[j]) <= 1e-8 * (1 + abs(eta[j]))
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            d = (O.collide_node(fin, F + e, tau, model=model) - O.collide_node(fin, F - e, tau, model=model)) / (2 * h)
            assert abs(d @ lam - gF[a]) <= 1e-8 * (1 + abs(gF[a]))


def test_model_jacobians_differ():
    """The four models' Jacobians are different maps (a test that passed for
    several with one formula would not pin the others)."""
    c, w, _ = O.lattice()
    rng = np.random.default_rng(4)
    fin = w * (1 + 0.05 * rng.uniform(-1, 1, 19))
    lam = rng.normal(size=19)
    e = [O.collide_jt_node(fin, np.zeros(3), 0.8, lam, model=m)[0] for m in range(4)]
    for a in range(4):
        for b in range(a):
            assert np.abs(e[a] - e[b]).max() > 1e-6 * np.abs(e[a]).max()


@pytest.mark.parametrize("model", [0, 1, 2, 3])
def test_adjoint_against_finite_differences(model):
    solid = _geom()
    tau, T = 0.8, 12
    rng = np.random.default_rng(3)
    shape = solid.shape
    fl = solid == 0
    s0 = O.init(solid, model=model) * (1 + 0.01 * rng.uniform(-1, 1, (19,) + shape))
    force = np.zeros((3,) + shape)
    force[0] = rng.normal(1e-5, 1e-6, shape) * fl
    L, gs, gF = O.adjoint(s0, solid, tau, force, T, periodic=7, model=model)

    def loss(s, ff):
        return O.loss_ux(O.run(s, solid, tau, T, force=ff, periodic=7, model=model), solid, ff, model=model)

    assert abs(loss(s0, force) - L) <= 1e-15 * abs(L) + 1e-20
    nodes = np.flatnonzero(fl.ravel())
    pick = rng.choice(nodes, 8, replace=False)
    # w.r.t. the force field (L is close to linear in F, so the truncation
    # error of a step of 1e-6 stays far below the rounding of the two runs)
    for n in pick:
        for a in (0, 1):
            eps = 1e-6
            fp = force.copy()
            fm = force.copy()
            fp.reshape(3, -1)[a, n] += eps
            fm.reshape(3, -1)[a, n] -= eps
            fd = (loss(s0, fp) - loss(s0, fm)) / (2 * eps)
            ad = gF.reshape(3, -1)[a, n]
            assert abs(fd - ad) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gF).max())
    # w.r.t. single initial distributions
    for n in pick[:5]:
        for i in (0, 1, 8, 14):
            eps = 1e-6
            sp = s0.copy()
            sm = s0.copy()
            sp.reshape(19, -1)[i, n] += eps
            sm.reshape(19, -1)[i, n] -= eps
            fd = (loss(sp, force) - loss(sm, force)) / (2 * eps)
            ad = gs.reshape(19, -1)[i, n]
            assert abs(fd - ad) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gs).max())
    # solid slots are never read: zero gradient
    assert np.all(gs[:, solid == 1] == 0)
