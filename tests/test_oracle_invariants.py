"""Pins of the FP64 oracle by invariants, brute force and finite differences.

Each check ties one oracle routine to another route the mathematics fixes:

* CRBA vs brute force: M e_k = RNEA(q, 0, e_k) - RNEA(q, 0, 0);
* M symmetric positive definite; RNEA = M qdd + RNEA(q, qd, 0);
* ABA(q, qd, RNEA(q, qd, qdd)) = qdd, and ABA equals the dense Cholesky solve;
* RNEA(q, a qd, 0) - g(q) = a^2 (RNEA(q, qd, 0) - g(q)); RNEA linear in the inertias;
* kinetic energy 1/2 qd^T M qd equals the sum of 1/2 v_i^T I_i v_i;
* g(q) is the gradient of the potential (finite differences along each velocity direction);
* power balance d/dt (T + V) = qd^T tau along a trajectory (finite differences);
* Lagrange's equations for fixed-base trees (Mdot qd - dT/dq from finite differences of M);
* change of total momentum equals the gravity wrench for a free-floating tree;
* Jacobian columns equal finite differences of FK.
"""

import numpy as np
import pytest

import synth
from oracle import OracleModel
from rigid_util import advance, gravity_wrench, system_momentum

TREES = {
    "chain7": synth.chain7,
    "humanoid_large": synth.humanoid_large,
    "humanoid_small": synth.humanoid_small,
    "quadruped_spine": synth.quadruped_spine,
    "random23": lambda: synth.random_tree(23, 3004),
}


def _setup(name, batch=6, seed=77):
    tree = TREES[name]()
    om = OracleModel.from_tree(tree)
    q, qd, qdd = synth.random_state(tree, batch, seed)
    return tree, om, q, qd, qdd


@pytest.mark.parametrize("name", list(TREES))
def test_crba_brute_force_and_spd(name):
    tree, om, q, qd, qdd = _setup(name)
    M = om.crba(q)
    nv = tree.nv
    for b in range(q.shape[0]):
        qb = np.repeat(q[b:b + 1], nv + 1, axis=0)
        acc = np.vstack([np.zeros(nv), np.eye(nv)])
        tau = om.rnea(qb, np.zeros((nv + 1, nv)), acc)
        Mbf = (tau[1:] - tau[0]).T
        np.testing.assert_allclose(M[b], Mbf, rtol=1e-12, atol=1e-11)
        np.testing.assert_allclose(M[b], M[b].T, rtol=0, atol=1e-13 * np.abs(M[b]).max())
        np.linalg.cholesky(M[b])
    bias = om.rnea(q, qd, np.zeros_like(qdd))
    tau = om.rnea(q, qd, qdd)
    np.testing.assert_allclose(tau, np.einsum("bij,bj->bi", M, qdd) + bias, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("name", list(TREES))
def test_aba_inverts_rnea(name):
    tree, om, q, qd, qdd = _setup(name)
    tau = om.rnea(q, qd, qdd)
    np.testing.assert_allclose(om.aba(q, qd, tau), qdd, rtol=1e-9, atol=1e-9)
    M = om.crba(q)
    bias = om.rnea(q, qd, np.zeros_like(qdd))
    tau2 = np.random.default_rng(3).standard_normal(tau.shape)
    ref = np.stack([np.linalg.solve(M[b], tau2[b] - bias[b]) for b in range(q.shape[0])])
    np.testing.assert_allclose(om.aba(q, qd, tau2), ref, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("name", list(TREES))
def test_velocity_scaling_and_linearity(name):
    tree, om, q, qd, qdd = _setup(name)
    z = np.zeros_like(qd)
    g = om.rnea(q, z, z)
    c1 = om.rnea(q, qd, z) - g
    c3 = om.rnea(q, 3.0 * qd, z) - g
    np.testing.assert_allclose(c3, 9.0 * c1, rtol=1e-11, atol=1e-10)
    rng = np.random.default_rng(9)
    pi1 = tree.inertia
    pi2 = tree.inertia * rng.uniform(0.5, 1.5, tree.inertia.shape)
    t1 = om.rnea(q, qd, qdd, inertia=pi1)
    t2 = om.rnea(q, qd, qdd, inertia=pi2)
    t12 = om.rnea(q, qd, qdd, inertia=pi1 + pi2)
    np.testing.assert_allclose(t12, t1 + t2, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("name", list(TREES))
def test_kinetic_energy(name):
    tree, om, q, qd, qdd = _setup(name)
    ke, _ = om.energy(q, qd)
    M = om.crba(q)
    np.testing.assert_allclose(ke, 0.5 * np.einsum("bi,bij,bj->b", qd, M, qd), rtol=1e-12)


@pytest.mark.parametrize("name", list(TREES))
def test_gravity_is_potential_gradient(name):
    tree, om, q, qd, qdd = _setup(name, batch=3)
    z = np.zeros_like(qd)
    g = om.rnea(q, z, z)
    h = 1e-6
    for b in range(q.shape[0]):
        for k in range(tree.nv):
            e = np.zeros(tree.nv)
            e[k] = h
            _, vp = om.energy(advance(tree, q[b], e)[None], z[:1])
            _, vm = om.energy(advance(tree, q[b], -e)[None], z[:1])
            assert abs((vp[0] - vm[0]) / (2 * h) - g[b, k]) < 1e-6 * (1 + abs(g[b, k]))


def _state_at(tree, q, qd, qdd, eps):
    # second-order step along the motion with constant acceleration
    return advance(tree, q, eps * qd + 0.5 * eps * eps * qdd), qd + eps * qdd


@pytest.mark.parametrize("name", list(TREES))
def test_power_balance(name):
    tree, om, q, qd, qdd = _setup(name, batch=4)
    tau = om.rnea(q, qd, qdd)
    eps = 1e-4
    for b in range(q.shape[0]):
        qp, vp = _state_at(tree, q[b], qd[b], qdd[b], eps)
        qm, vm = _state_at(tree, q[b], qd[b], qdd[b], -eps)
        kp, pp = om.energy(qp[None], vp[None])
        km, pm = om.energy(qm[None], vm[None])
        dE = ((kp[0] + pp[0]) - (km[0] + pm[0])) / (2 * eps)
        power = float(qd[b] @ tau[b])
        assert abs(dE - power) < 1e-6 * (1 + abs(power)), (dE, power)


@pytest.mark.parametrize("name", ["chain7", "quadruped_spine", "random23"])
def test_lagrange_equations_fixed_base(name):
    tree, om, q, qd, qdd = _setup(name, batch=3)
    h = 1e-6
    nv = tree.nv
    for b in range(q.shape[0]):
        M = om.crba(q[b:b + 1])[0]
        Mdot = (om.crba((q[b] + h * qd[b])[None])[0] - om.crba((q[b] - h * qd[b])[None])[0]) / (2 * h)
        dT = np.zeros(nv)
        for k in range(nv):
            e = np.zeros(nv)
            e[k] = h
            Mp = om.crba((q[b] + e)[None])[0]
            Mm = om.crba((q[b] - e)[None])[0]
            dT[k] = 0.5 * qd[b] @ ((Mp - Mm) / (2 * h)) @ qd[b]
        g = om.rnea(q[b:b + 1], np.zeros((1, nv)), np.zeros((1, nv)))[0]
        tau_lag = M @ qdd[b] + Mdot @ qd[b] - dT + g
        tau = om.rnea(q[b:b + 1], qd[b:b + 1], qdd[b:b + 1])[0]
        np.testing.assert_allclose(tau, tau_lag, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("name", ["humanoid_large", "humanoid_small"])
def test_free_floating_momentum(name):
    tree, om, q, qd, qdd = _setup(name, batch=3)
    rng = np.random.default_rng(21)
    eps = 1e-4
    for b in range(q.shape[0]):
        tau = rng.standard_normal(tree.nv)
        tau[:6] = 0.0  # nothing acts on the free root; joint torques are internal
        a = om.aba(q[b:b + 1], qd[b:b + 1], tau[None])[0]
        qp, vp = _state_at(tree, q[b], qd[b], a, eps)
        qm, vm = _state_at(tree, q[b], qd[b], a, -eps)
        dh = (system_momentum(tree, om, qp, vp) - system_momentum(tree, om, qm, vm)) / (2 * eps)
        w = gravity_wrench(tree, om, q[b])
        np.testing.assert_allclose(dh, w, rtol=1e-6, atol=1e-5 * (1 + np.abs(w).max()))


@pytest.mark.parametrize("name", list(TREES))
@pytest.mark.parametrize("frame", [0, 1])
def test_jacobian_matches_fk_differences(name, frame):
    tree, om, q, qd, qdd = _setup(name, batch=3)
    ee = tree.ee_bodies
    J = om.jacobian(q, ee, frame=frame)
    h = 1e-6
    for b in range(q.shape[0]):
        for k in range(tree.nv):
            e = np.zeros(tree.nv)
            e[k] = h
            Tp = om.fk(advance(tree, q[b], e)[None])[0]
            Tm = om.fk(advance(tree, q[b], -e)[None])[0]
            for ei, body in enumerate(ee):
                Rp, Rm = Tp[body, :, :3], Tm[body, :, :3]
                R = 0.5 * (Rp + Rm)
                W = (Rp - Rm) @ R.T / (2 * h)
                w = np.array([W[2, 1] - W[1, 2], W[0, 2] - W[2, 0], W[1, 0] - W[0, 1]]) / 2
                pdot = (Tp[body, :, 3] - Tm[body, :, 3]) / (2 * h)
                p = 0.5 * (Tp[body, :, 3] + Tm[body, :, 3])
                lin = pdot if frame == 1 else pdot - np.cross(w, p)
                col = J[b, ei, :, k]
                np.testing.assert_allclose(col[3:], w, atol=2e-8)
                np.testing.assert_allclose(col[:3], lin, atol=2e-8)
