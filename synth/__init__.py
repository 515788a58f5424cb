"""Seeded synthetic robot trees and inputs.

This module is shared by the FP64 oracle's tests and by the GPU path's tests and
benchmark. It only draws random numbers and lays them out in the arrays the
model constructor takes; it holds none of the dynamics arithmetic (no
transforms, no recursions), so neither side can borrow the other's math from it.

Conventions of the arrays (one row per body, parent before child):

* ``parent[i]``      index of the parent body, ``-1`` for a body on the world/base.
* ``joint_type[i]``  0 revolute, 1 prismatic, 2 free (6-DOF), 3 fixed.
* ``axis[i]``        unit joint axis in the joint frame.
* ``X_tree[i]``      3x4 row-major ``[R_pre | t_pre]``: pose of joint i's frame in
                     the parent body's frame.  The body frame is the joint frame
                     after the joint motion.
* ``inertia[i]``     ``[m, m*cx, m*cy, m*cz, Ixx, Ixy, Iyy, Ixz, Iyz, Izz]`` with the
                     rotational inertia taken about the body-frame origin.

A free joint has ``nq = 7`` coordinates ``[x, y, z, qx, qy, qz, qw]`` and ``nv = 6``
velocity coordinates, the body-frame twist ``[v; w]``.
"""

from .trees import (Tree, REVOLUTE, PRISMATIC, FREE, FIXED, chain7, humanoid_large,
                    humanoid_small, random_tree, multi_trees, MULTI_BATCHES, quadruped_spine,
                    pendulum, two_link_planar, random_inertia_params, tree_by_name,
                    edge_tree, EDGE_TREES)
from .inputs import random_state, sinusoid_trajectories, to_fp32_grid

__all__ = [
    "Tree", "REVOLUTE", "PRISMATIC", "FREE", "FIXED", "chain7", "humanoid_large",
    "humanoid_small", "random_tree", "multi_trees", "MULTI_BATCHES", "quadruped_spine", "pendulum", "edge_tree", "EDGE_TREES",
    "two_link_planar", "random_inertia_params", "tree_by_name", "random_state",
    "sinusoid_trajectories", "to_fp32_grid",
]
