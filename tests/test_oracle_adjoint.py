"""Pins of the oracle's reverse-mode gradients (tape AD) against FP64 central
finite differences (h = 1e-6) and, for the inertial parameters, against the
exact regressor: RNEA is linear in the 10 parameters of every body, so
d tau / d pi is obtained exactly from unit-parameter evaluations."""

import numpy as np
import pytest

import synth
from oracle import OracleModel


@pytest.mark.parametrize("name", ["quadruped_spine", "chain7", "humanoid_small"])
def test_rnea_vjp_vs_central_differences(name):
    tree = synth.tree_by_name(name)
    om = OracleModel.from_tree(tree)
    q, qd, qdd = synth.random_state(tree, 4, 123)
    tb = np.random.default_rng(4).standard_normal((4, tree.nv))
    qb, qdb, qddb, pib = om.rnea_vjp(q, qd, qdd, tb)
    h = 1e-6

    def f(qq, vv, aa, pi=None):
        return np.einsum("bi,bi->b", om.rnea(qq, vv, aa, inertia=pi), tb)

    for k in range(tree.nq):
        e = np.zeros(tree.nq)
        e[k] = h
        fd = (f(q + e, qd, qdd) - f(q - e, qd, qdd)) / (2 * h)
        np.testing.assert_allclose(qb[:, k], fd, rtol=1e-6, atol=1e-6)
    for k in range(tree.nv):
        e = np.zeros(tree.nv)
        e[k] = h
        fd = (f(q, qd + e, qdd) - f(q, qd - e, qdd)) / (2 * h)
        np.testing.assert_allclose(qdb[:, k], fd, rtol=1e-6, atol=1e-6)
        fd = (f(q, qd, qdd + e) - f(q, qd, qdd - e)) / (2 * h)
        np.testing.assert_allclose(qddb[:, k], fd, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("name", ["quadruped_spine", "humanoid_small"])
def test_rnea_inertia_gradient_is_regressor(name):
    tree = synth.tree_by_name(name)
    om = OracleModel.from_tree(tree)
    q, qd, qdd = synth.random_state(tree, 3, 321)
    tb = np.random.default_rng(8).standard_normal((3, tree.nv))
    _, _, _, pib = om.rnea_vjp(q, qd, qdd, tb)
    n = tree.n_bodies
    for j in range(10 * n):
        pi = np.zeros(10 * n)
        pi[j] = 1.0
        col = om.rnea(q, qd, qdd, inertia=pi.reshape(n, 10))  # column j of the regressor
        np.testing.assert_allclose(pib.reshape(3, -1)[:, j], np.einsum("bi,bi->b", col, tb),
                                   rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name", ["chain7", "humanoid_small", "random23"])
def test_fk_vjp_vs_central_differences(name):
    tree = synth.tree_by_name(name)
    om = OracleModel.from_tree(tree)
    q, _, _ = synth.random_state(tree, 3, 55)
    pb = np.random.default_rng(6).standard_normal((3, tree.n_bodies, 3, 4))
    qb = om.fk_vjp(q, pb)
    h = 1e-6
    for k in range(tree.nq):
        e = np.zeros(tree.nq)
        e[k] = h
        fd = (np.einsum("bnij,bnij->b", om.fk(q + e), pb) - np.einsum("bnij,bnij->b", om.fk(q - e), pb)) / (2 * h)
        np.testing.assert_allclose(qb[:, k], fd, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("name", ["chain7", "quadruped_spine", "humanoid_small", "random23"])
def test_crba_vjp_vs_central_differences(name):
    """q_bar of <M_bar, M(q)> against central differences of the oracle's
    CRBA; for a free root the mass matrix (body-frame root velocity) does not
    depend on the root's pose, so its seven coordinates get zero."""
    tree = synth.tree_by_name(name)
    om = OracleModel.from_tree(tree)
    q, _, _ = synth.random_state(tree, 3, 77)
    mb = np.random.default_rng(9).standard_normal((3, tree.nv, tree.nv))
    qb, _ = om.crba_vjp(q, mb)
    h = 1e-6
    for k in range(tree.nq):
        e = np.zeros(tree.nq)
        e[k] = h
        fd = (np.einsum("bij,bij->b", om.crba(q + e), mb) - np.einsum("bij,bij->b", om.crba(q - e), mb)) / (2 * h)
        np.testing.assert_allclose(qb[:, k], fd, rtol=1e-6, atol=1e-6)
    if tree.joint_type[0] == synth.FREE:
        assert np.abs(qb[:, :7]).max() < 1e-9


def test_crba_vjp_inertia_gradient_is_regressor():
    """M is linear in the inertial parameters: d<M_bar, M>/d pi_j is
    <M_bar, CRBA(q; e_j)> exactly."""
    tree = synth.quadruped_spine()
    om = OracleModel.from_tree(tree)
    q, _, _ = synth.random_state(tree, 2, 78)
    mb = np.random.default_rng(10).standard_normal((2, tree.nv, tree.nv))
    _, pib = om.crba_vjp(q, mb)
    n = tree.n_bodies
    for j in range(10 * n):
        pi = np.zeros(10 * n)
        pi[j] = 1.0
        col = om.crba(q, inertia=pi.reshape(n, 10))
        np.testing.assert_allclose(pib.reshape(2, -1)[:, j], np.einsum("bij,bij->b", col, mb), rtol=1e-12,
                                   atol=1e-12)


@pytest.mark.parametrize("name", ["quadruped_spine", "humanoid_small"])
def test_crba_parameter_override(name):
    """CRBA with given parameters: the default parameters reproduce M, the sum
    of the per-body mass matrices is M (linearity), and every column equals
    the unit-acceleration RNEA with the same parameters and no velocity
    (the brute-force definition M e_k = RNEA(q, 0, e_k) - RNEA(q, 0, 0))."""
    tree = synth.tree_by_name(name)
    om = OracleModel.from_tree(tree)
    q, _, _ = synth.random_state(tree, 3, 79)
    M = om.crba(q)
    np.testing.assert_array_equal(om.crba(q, inertia=tree.inertia), M)
    acc = np.zeros_like(M)
    zero = np.zeros((3, tree.nv))
    for k in range(tree.n_bodies):
        pi = np.zeros_like(tree.inertia)
        pi[k] = tree.inertia[k]
        Mk = om.crba(q, inertia=pi)
        acc += Mk
        g = om.rnea(q, zero, zero, inertia=pi)
        for j in range(tree.nv):
            e = zero.copy()
            e[:, j] = 1.0
            np.testing.assert_allclose(Mk[:, :, j], om.rnea(q, zero, e, inertia=pi) - g, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(acc, M, rtol=1e-12, atol=1e-12)
