"""Pins of the FP64 oracle against closed forms (single pendulum, two-link planar arm).

The formulas here are the textbook Lagrangian results for these two systems,
written out independently of the oracle's spatial-algebra recursions.
"""

import numpy as np
import pytest

import synth
from oracle import OracleModel

G = 9.81


def _rot_x(q):
    c, s = np.cos(q), np.sin(q)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


@pytest.mark.parametrize("q", [-2.7, -0.4, 0.0, 0.9, 3.0])
def test_pendulum_fk(q):
    t = synth.pendulum()
    m = OracleModel.from_tree(t)
    T = m.fk(np.array([[q]]))[0, 0]
    np.testing.assert_allclose(T[:, :3], _rot_x(q), atol=1e-15)
    np.testing.assert_allclose(T[:, 3], 0.0, atol=1e-15)
    R = T[:, :3]
    assert abs(np.linalg.det(R) - 1) < 1e-14
    np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-15)
    # COM at [0, l sin q, -l cos q]
    l = 0.7
    com = R @ np.array([0, 0, -l]) + T[:, 3]
    np.testing.assert_allclose(com, [0, l * np.sin(q), -l * np.cos(q)], atol=1e-15)


def test_pendulum_dynamics():
    mass, l, ixx = 1.3, 0.7, 0.02
    t = synth.pendulum(m=mass, l=l, ixx=ixx)
    m = OracleModel.from_tree(t)
    rng = np.random.default_rng(5)
    q = rng.uniform(-np.pi, np.pi, (16, 1))
    qd = rng.standard_normal((16, 1))
    qdd = rng.standard_normal((16, 1))
    inertia = ixx + mass * l * l
    tau = inertia * qdd + mass * G * l * np.sin(q)
    np.testing.assert_allclose(m.rnea(q, qd, qdd), tau, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(m.crba(q)[:, 0, 0], np.full(16, inertia), rtol=1e-14)
    qdd_aba = m.aba(q, qd, tau)
    np.testing.assert_allclose(qdd_aba, qdd, rtol=1e-12, atol=1e-12)
    # pendulum forward dynamics closed form
    tau2 = rng.standard_normal((16, 1))
    np.testing.assert_allclose(m.aba(q, qd, tau2), (tau2 - mass * G * l * np.sin(q)) / inertia,
                               rtol=1e-12, atol=1e-12)


def _two_link_closed(q, qd, qdd, m1=1.5, m2=0.9, l1=0.8, lc1=0.35, lc2=0.3, i1=0.04, i2=0.025):
    c1, s1 = np.cos(q[0]), np.sin(q[0])
    c2, s2 = np.cos(q[1]), np.sin(q[1])
    c12 = np.cos(q[0] + q[1])
    M11 = i1 + i2 + m1 * lc1 ** 2 + m2 * (l1 ** 2 + lc2 ** 2 + 2 * l1 * lc2 * c2)
    M12 = i2 + m2 * (lc2 ** 2 + l1 * lc2 * c2)
    M22 = i2 + m2 * lc2 ** 2
    h = m2 * l1 * lc2 * s2
    g1 = (m1 * lc1 + m2 * l1) * G * c1 + m2 * lc2 * G * c12
    g2 = m2 * lc2 * G * c12
    tau1 = M11 * qdd[0] + M12 * qdd[1] - h * (2 * qd[0] * qd[1] + qd[1] ** 2) + g1
    tau2 = M12 * qdd[0] + M22 * qdd[1] + h * qd[0] ** 2 + g2
    return np.array([[M11, M12], [M12, M22]]), np.array([tau1, tau2])


def test_two_link_fk_and_jacobian():
    t = synth.two_link_planar()
    m = OracleModel.from_tree(t)
    l1 = 0.8
    rng = np.random.default_rng(7)
    for _ in range(8):
        q = rng.uniform(-np.pi, np.pi, 2)
        T = m.fk(q[None])[0]
        np.testing.assert_allclose(T[1, :, 3], [l1 * np.cos(q[0]), 0.0, l1 * np.sin(q[0])], atol=1e-15)
        # frame 1: velocity of body 2's origin in world axes, rows [lin; ang]
        J = m.jacobian(q[None], [1], frame=1)[0, 0]
        s1, c1 = np.sin(q[0]), np.cos(q[0])
        np.testing.assert_allclose(J[0], [-l1 * s1, 0.0], atol=1e-15)
        np.testing.assert_allclose(J[1], [0.0, 0.0], atol=1e-15)
        np.testing.assert_allclose(J[2], [l1 * c1, 0.0], atol=1e-15)
        np.testing.assert_allclose(J[3:], [[0, 0], [-1, -1], [0, 0]], atol=1e-15)
        # frame 0 (spatial): linear part = point velocity - w x p
        J0 = m.jacobian(q[None], [1], frame=0)[0, 0]
        p = T[1, :, 3]
        for k in range(2):
            np.testing.assert_allclose(J0[:3, k], J[:3, k] - np.cross(J[3:, k], p), atol=1e-15)


def test_two_link_dynamics():
    t = synth.two_link_planar()
    m = OracleModel.from_tree(t)
    rng = np.random.default_rng(11)
    q = rng.uniform(-np.pi, np.pi, (32, 2))
    qd = rng.standard_normal((32, 2))
    qdd = rng.standard_normal((32, 2))
    tau = m.rnea(q, qd, qdd)
    M = m.crba(q)
    for b in range(32):
        Mc, tc = _two_link_closed(q[b], qd[b], qdd[b])
        np.testing.assert_allclose(M[b], Mc, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(tau[b], tc, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(m.aba(q, qd, tau), qdd, rtol=1e-10, atol=1e-11)
