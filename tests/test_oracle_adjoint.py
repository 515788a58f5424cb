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
