"""Small rigid-body helpers used by the oracle's invariant tests.

These are written from first principles (matrix exponential of a twist,
momentum of a rigid body from its COM velocity) so that the invariants they
feed check the oracle through routes it does not use itself.
"""

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import synth


def hat_twist(xi):
    """4x4 matrix of a body twist [v; w]."""
    v, w = xi[:3], xi[3:]
    H = np.zeros((4, 4))
    H[:3, :3] = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    H[:3, 3] = v
    return H


def root_pose(qroot):
    T = np.eye(4)
    T[:3, :3] = Rotation.from_quat(qroot[3:7] / np.linalg.norm(qroot[3:7])).as_matrix()
    T[:3, 3] = qroot[:3]
    return T


def pose_to_qroot(T):
    return np.concatenate([T[:3, 3], Rotation.from_matrix(T[:3, :3]).as_quat()])


def advance(tree, q, dq):
    """Move the configuration by a velocity-space increment ``dq`` (length nv).

    Revolute and prismatic coordinates add; a free root composes its pose with
    exp of the body-frame twist ``dq[0:6]`` (``[v; w]``).
    """
    q = np.array(q, dtype=np.float64, copy=True)
    qo, vo = tree.q_offsets(), tree.v_offsets()
    for i, t in enumerate(tree.joint_type):
        if t == synth.FREE:
            T = root_pose(q[qo[i]:qo[i] + 7]) @ expm(hat_twist(dq[vo[i]:vo[i] + 6]))
            q[qo[i]:qo[i] + 7] = pose_to_qroot(T)
        elif t in (synth.REVOLUTE, synth.PRISMATIC):
            q[qo[i]] += dq[vo[i]]
    return q


def system_momentum(tree, om, q, qd):
    """World spatial momentum [angular about the origin; linear] of the whole tree.

    Body velocities come from the oracle's spatial Jacobian of each body, COM
    positions from the oracle's FK; the momentum of a body is m v_com and
    c x m v_com + R I_C R^T w.
    """
    n = tree.n_bodies
    T = om.fk(q[None])[0]
    J = om.jacobian(q[None], list(range(n)), frame=0)[0]
    L = np.zeros(3)
    P = np.zeros(3)
    for i in range(n):
        pi = tree.inertia[i]
        m, h = pi[0], pi[1:4]
        Io = np.array([[pi[4], pi[5], pi[7]], [pi[5], pi[6], pi[8]], [pi[7], pi[8], pi[9]]])
        c_b = h / m
        Ic = Io - m * (np.dot(c_b, c_b) * np.eye(3) - np.outer(c_b, c_b))
        R, p = T[i, :, :3], T[i, :, 3]
        twist = J[i] @ qd
        v0, w = twist[:3], twist[3:]
        c = R @ c_b + p
        vc = v0 + np.cross(w, c)
        P += m * vc
        L += np.cross(c, m * vc) + R @ Ic @ R.T @ w
    return np.concatenate([L, P])


def gravity_wrench(tree, om, q):
    """External wrench [moment about origin; force] of gravity on the tree."""
    T = om.fk(q[None])[0]
    g = tree.gravity
    n_ = np.zeros(3)
    f = np.zeros(3)
    for i in range(tree.n_bodies):
        m, h = tree.inertia[i][0], tree.inertia[i][1:4]
        c = T[i, :, :3] @ (h / m) + T[i, :, 3]
        n_ += np.cross(c, m * g)
        f += m * g
    return np.concatenate([n_, f])
