"""Seeded joint-space inputs for the synthetic trees.

Distributions (per coordinate):

* revolute q ~ U[-pi, pi]; prismatic q ~ U[-0.3, 0.3] m;
* free root: position ~ U[-1, 1]^3 m, orientation a uniform unit quaternion
  (normalised 4-D Gaussian), stored ``[x, y, z, qx, qy, qz, qw]``;
* every velocity and acceleration coordinate ~ N(0, 1).

Inputs are drawn in FP64.  ``to_fp32_grid`` rounds them to the FP32 grid so the
FP64 oracle and an FP32 kernel see exactly the same numbers.
"""

from __future__ import annotations

import numpy as np

from .trees import Tree, REVOLUTE, PRISMATIC, FREE


def random_state(tree: Tree, batch: int, seed: int):
    """Return ``(q, qd, qdd)`` as float64 arrays of shape [B, nq], [B, nv], [B, nv]."""
    rng = np.random.default_rng(seed)
    q = np.zeros((batch, tree.nq))
    qo = tree.q_offsets()
    for i, t in enumerate(tree.joint_type):
        k = qo[i]
        if t == REVOLUTE:
            q[:, k] = rng.uniform(-np.pi, np.pi, size=batch)
        elif t == PRISMATIC:
            q[:, k] = rng.uniform(-0.3, 0.3, size=batch)
        elif t == FREE:
            q[:, k:k + 3] = rng.uniform(-1.0, 1.0, size=(batch, 3))
            g = rng.standard_normal((batch, 4))
            q[:, k + 3:k + 7] = g / np.linalg.norm(g, axis=1, keepdims=True)
    qd = rng.standard_normal((batch, tree.nv))
    qdd = rng.standard_normal((batch, tree.nv))
    return q, qd, qdd


def sinusoid_trajectories(tree: Tree, n_traj: int, n_steps: int, seed: int, dt: float = 0.01):
    """Sinusoidal joint trajectories for a fixed-base revolute tree.

    ``q_j(t) = A sin(2 pi f t + phi)`` with A ~ U[0.1, 1] rad, f ~ U[0.2, 2] Hz and
    phi ~ U[0, 2 pi), drawn per trajectory and joint; velocities and
    accelerations are the analytic derivatives.  Returns float64 arrays of shape
    [n_traj * n_steps, nv], trajectory-major.
    """
    if any(int(t) == FREE for t in tree.joint_type):
        raise ValueError("sinusoid trajectories are defined for fixed-base trees")
    rng = np.random.default_rng(seed)
    nv = tree.nv
    amp = rng.uniform(0.1, 1.0, size=(n_traj, 1, nv))
    freq = rng.uniform(0.2, 2.0, size=(n_traj, 1, nv))
    phase = rng.uniform(0.0, 2 * np.pi, size=(n_traj, 1, nv))
    t = (np.arange(n_steps) * dt)[None, :, None]
    w = 2 * np.pi * freq
    arg = w * t + phase
    q = amp * np.sin(arg)
    qd = amp * w * np.cos(arg)
    qdd = -amp * w * w * np.sin(arg)
    return (q.reshape(-1, nv), qd.reshape(-1, nv), qdd.reshape(-1, nv))


def to_fp32_grid(x: np.ndarray) -> np.ndarray:
    """Round to the nearest FP32 value and return it as float64."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)
