"""Host-side pins of the mass-identification plumbing: the affine map from
link masses to body-origin inertial parameters keeps each link's centre of
mass and its rotational inertia about it, and the loss gradient it implies
(the inertial-parameter gradient of the RNEA adjoint contracted with the map)
matches central differences of the loss.  Both use the FP64 oracle."""

import numpy as np
import pytest

import synth
from oracle import OracleModel
from paper_2605_31481_amd.sysid import mass_map


def _com_frame(pi):
    """Mass, centre of mass and rotational inertia about it from [m, h, I_O]."""
    m = pi[0]
    c = pi[1:4] / m
    io = np.array([[pi[4], pi[5], pi[7]], [pi[5], pi[6], pi[8]], [pi[7], pi[8], pi[9]]])
    # parallel-axis theorem: I_O = I_C + m (|c|^2 1 - c c^T)
    return m, c, io - m * (c @ c * np.eye(3) - np.outer(c, c))


@pytest.mark.parametrize("name", ["quadruped_spine", "chain7"])
def test_mass_map_keeps_com_and_central_inertia(name):
    tree = synth.tree_by_name(name)
    A, D, m = mass_map(tree.inertia)
    assert np.allclose(A + m[:, None] * D, tree.inertia, rtol=0, atol=1e-14)
    m2 = m * np.random.default_rng(3).uniform(0.5, 1.5, size=m.shape)
    pi2 = A + m2[:, None] * D
    for k in range(tree.n_bodies):
        ma, ca, ica = _com_frame(np.asarray(tree.inertia[k]))
        mb, cb, icb = _com_frame(pi2[k])
        assert np.isclose(mb, m2[k], rtol=1e-14)
        assert np.allclose(cb, ca, atol=1e-14)
        assert np.allclose(icb, ica, atol=1e-13)
        assert np.all(np.linalg.eigvalsh(icb) > 0)


def test_mass_gradient_matches_central_differences():
    tree = synth.quadruped_spine()
    om = OracleModel.from_tree(tree)
    q, qd, qdd = synth.sinusoid_trajectories(tree, 3, 4, seed=11)
    A, D, m0 = mass_map(tree.inertia)
    tau_meas = om.rnea(q, qd, qdd) + np.random.default_rng(2).normal(0, 0.1, size=(q.shape[0], tree.nv))
    m = m0 * (1 + 0.2 * np.random.default_rng(5).uniform(-1, 1, size=m0.shape))
    B = q.shape[0]

    def loss(mm):
        r = om.rnea(q, qd, qdd, inertia=A + mm[:, None] * D) - tau_meas
        return 0.5 * np.sum(r * r) / B

    r = om.rnea(q, qd, qdd, inertia=A + m[:, None] * D) - tau_meas
    _, _, _, pib = om.rnea_vjp(q, qd, qdd, r / B, inertia=A + m[:, None] * D)
    grad = (pib.sum(axis=0) * D).sum(axis=1)
    h = 1e-6
    for k in range(len(m)):
        e = np.zeros_like(m)
        e[k] = h
        fd = (loss(m + e) - loss(m - e)) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, grad[k], fd)
