"""Seeded synthetic kinematic trees.

The recipes stand in for the robots the paper measures (7 to 23 DOF arms,
quadrupeds and humanoids, Sec. 4.1 and Table 1); none of those robot files is
used.  Every random draw comes from ``numpy.random.Generator(PCG64(seed))`` so a
seed reproduces the same bytes on every machine.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

REVOLUTE, PRISMATIC, FREE, FIXED = 0, 1, 2, 3

_NQ = {REVOLUTE: 1, PRISMATIC: 1, FREE: 7, FIXED: 0}
_NV = {REVOLUTE: 1, PRISMATIC: 1, FREE: 6, FIXED: 0}


@dataclass
class Tree:
    """Arrays in the layout the model constructor takes (see package doc)."""

    name: str
    parent: np.ndarray          # int32 [n]
    joint_type: np.ndarray      # int32 [n]
    axis: np.ndarray            # float64 [n, 3]
    X_tree: np.ndarray          # float64 [n, 3, 4]
    inertia: np.ndarray         # float64 [n, 10]
    ee_bodies: List[int] = field(default_factory=list)
    gravity: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, -9.81]))

    @property
    def n_bodies(self) -> int:
        return int(self.parent.shape[0])

    @property
    def nq(self) -> int:
        return int(sum(_NQ[int(t)] for t in self.joint_type))

    @property
    def nv(self) -> int:
        return int(sum(_NV[int(t)] for t in self.joint_type))

    @property
    def depth(self) -> int:
        d = np.zeros(self.n_bodies, dtype=np.int64)
        for i, p in enumerate(self.parent):
            d[i] = 1 if p < 0 else d[p] + 1
        return int(d.max()) if self.n_bodies else 0

    def q_offsets(self) -> np.ndarray:
        off, k = [], 0
        for t in self.joint_type:
            off.append(k)
            k += _NQ[int(t)]
        return np.array(off, dtype=np.int64)

    def v_offsets(self) -> np.ndarray:
        off, k = [], 0
        for t in self.joint_type:
            off.append(k)
            k += _NV[int(t)]
        return np.array(off, dtype=np.int64)


def _haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation: QR of a Gaussian matrix with the sign fixed."""
    a = rng.standard_normal((3, 3))
    qm, rm = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(rm))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def random_inertia_params(rng: np.random.Generator) -> np.ndarray:
    """Mass U[0.5,5] kg, COM U[-0.1,0.1] m per axis, COM inertia R diag(a,b,c) R^T.

    The principal moments are drawn from U[0.01, 0.1] kg m^2 jointly and redrawn
    until they satisfy the triangle inequality (every pair sum >= the third).
    Returned as the 10 parameters about the body origin.
    """
    m = rng.uniform(0.5, 5.0)
    c = rng.uniform(-0.1, 0.1, size=3)
    while True:
        d = rng.uniform(0.01, 0.1, size=3)
        if d[0] + d[1] >= d[2] and d[1] + d[2] >= d[0] and d[0] + d[2] >= d[1]:
            break
    r = _haar_rotation(rng)
    ic = r @ np.diag(d) @ r.T
    io = ic + m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
    return np.array([m, m * c[0], m * c[1], m * c[2],
                     io[0, 0], io[0, 1], io[1, 1], io[0, 2], io[1, 2], io[2, 2]])


def _random_axis(rng: np.random.Generator) -> np.ndarray:
    n = rng.standard_normal(3)
    return n / np.linalg.norm(n)


def _random_offset(rng: np.random.Generator) -> np.ndarray:
    x = np.zeros((3, 4))
    x[:, :3] = np.eye(3)
    x[:, 3] = rng.uniform(-0.3, 0.3, size=3)
    return x


def _identity_offset() -> np.ndarray:
    x = np.zeros((3, 4))
    x[:, :3] = np.eye(3)
    return x


def _build(name, parents, types, rng, ee, root_identity=True) -> Tree:
    n = len(parents)
    axis = np.zeros((n, 3))
    xt = np.zeros((n, 3, 4))
    inertia = np.zeros((n, 10))
    for i in range(n):
        # Draw order per body is fixed (axis, offset, inertia) so trees are reproducible.
        axis[i] = _random_axis(rng)
        xt[i] = _random_offset(rng)
        inertia[i] = random_inertia_params(rng)
        if types[i] == FREE and root_identity:
            xt[i] = _identity_offset()
            axis[i] = np.array([0.0, 0.0, 1.0])
    return Tree(name=name, parent=np.array(parents, dtype=np.int32),
                joint_type=np.array(types, dtype=np.int32), axis=axis, X_tree=xt,
                inertia=inertia, ee_bodies=list(ee))


def chain7(seed: int = 1000) -> Tree:
    """Fixed-base 7-DOF serial chain, all revolute; the end effector is the tip."""
    rng = np.random.default_rng(seed)
    parents = [-1, 0, 1, 2, 3, 4, 5]
    return _build("chain7", parents, [REVOLUTE] * 7, rng, ee=[6])


def _humanoid(name, n_arms, n_legs, seed) -> Tree:
    # Body 0: free root (torso).  Waist w1 -> w2 -> w3 -> neck (prismatic).
    # Arms (7 revolute) hang from w1; legs (6, 4th prismatic) hang from the root.
    parents = [-1, 0, 1, 2, 3]
    types = [FREE, REVOLUTE, REVOLUTE, REVOLUTE, PRISMATIC]
    hands, feet = [], []
    for _ in range(n_arms):
        p = 1
        for _j in range(7):
            parents.append(p)
            types.append(REVOLUTE)
            p = len(parents) - 1
        hands.append(p)
    for _ in range(n_legs):
        p = 0
        for j in range(6):
            parents.append(p)
            types.append(PRISMATIC if j == 3 else REVOLUTE)
            p = len(parents) - 1
        feet.append(p)
    if n_arms == 2:
        ee = hands + feet
    else:
        ee = hands + feet + [4, 3]   # hand, foot, neck tip, waist tip
    rng = np.random.default_rng(seed)
    return _build(name, parents, types, rng, ee=ee)


def humanoid_large(seed: int = 1002) -> Tree:
    """Free root + 3-DOF waist + 1-DOF neck + two 7-DOF arms + two 6-DOF legs.

    31 bodies, nq = 37, nv = 36, depth 9, level widths 1,3,5,5,5,4,4,2,2.
    End effectors: both hands and both feet.
    """
    return _humanoid("humanoid_large", 2, 2, seed)


def humanoid_small(seed: int = 1002) -> Tree:
    """The 23-velocity-DOF companion: one arm and one leg instead of two of each.

    18 bodies, nq = 24, nv = 23, depth 9.  End effectors: hand, foot, neck, waist tip.
    """
    return _humanoid("humanoid_small", 1, 1, seed)


def random_tree(n: int, seed: int) -> Tree:
    """Fixed-base random revolute tree with n bodies and depth drawn in 4..min(10, n).

    A spine of d bodies is built from the base; each remaining body attaches to a
    uniformly chosen existing body of depth < d.  End effectors: up to the four
    deepest leaves, ties broken by the lowest index.
    """
    rng = np.random.default_rng(seed)
    d = int(rng.integers(4, min(10, n) + 1))
    parents = [-1] + list(range(d - 1))
    depth = list(range(1, d + 1))
    while len(parents) < n:
        cands = [i for i in range(len(parents)) if depth[i] < d]
        p = cands[int(rng.integers(0, len(cands)))]
        parents.append(p)
        depth.append(depth[p] + 1)
    is_leaf = [True] * n
    for p in parents:
        if p >= 0:
            is_leaf[p] = False
    leaves = sorted([i for i in range(n) if is_leaf[i]], key=lambda i: (-depth[i], i))
    return _build(f"random{n}", parents, [REVOLUTE] * n, rng, ee=leaves[:4])


def multi_trees() -> List[Tree]:
    """Five random trees of 7, 11, 12, 18 and 23 DOF (seeds 3000..3004)."""
    return [random_tree(n, 3000 + k) for k, n in enumerate([7, 11, 12, 18, 23])]


MULTI_BATCHES = [512, 1024, 2048, 4096, 8192]


def quadruped_spine(seed: int = 1004) -> Tree:
    """Fixed-base 11-DOF tree: spine s1->s2->s3, rear legs (2x2) on the base,
    front legs (2x2) on s3.  Level widths 3,3,1,2,2."""
    parents = [-1, 0, 1, -1, 3, -1, 5, 2, 7, 2, 9]
    rng = np.random.default_rng(seed)
    return _build("quadruped_spine", parents, [REVOLUTE] * 11, rng, ee=[4, 6, 8, 10])


def pendulum(m=1.3, l=0.7, ixx=0.02, iyy=0.03, izz=0.015) -> Tree:
    """Single revolute joint about x at the origin, COM at [0, 0, -l]."""
    c = np.array([0.0, 0.0, -l])
    ic = np.diag([ixx, iyy, izz])
    io = ic + m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
    inertia = np.array([[m, m * c[0], m * c[1], m * c[2],
                         io[0, 0], io[0, 1], io[1, 1], io[0, 2], io[1, 2], io[2, 2]]])
    return Tree(name="pendulum", parent=np.array([-1], dtype=np.int32),
                joint_type=np.array([REVOLUTE], dtype=np.int32),
                axis=np.array([[1.0, 0.0, 0.0]]), X_tree=_identity_offset()[None],
                inertia=inertia, ee_bodies=[0])


def two_link_planar(m1=1.5, m2=0.9, l1=0.8, lc1=0.35, lc2=0.3, i1=0.04, i2=0.025) -> Tree:
    """Planar elbow arm in the x-z plane, both axes along -y so +q lifts x toward +z.

    Link 1 has its COM at [lc1, 0, 0]; body 2's origin is at [l1, 0, 0] in body 1.
    ``i1``/``i2`` are the COM moments about the joint axis (I_yy); the other
    principal moments are set so the COM inertias stay positive definite.
    """
    def params(m, lc, iyy):
        c = np.array([lc, 0.0, 0.0])
        ic = np.diag([0.5 * iyy, iyy, 0.8 * iyy])
        io = ic + m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
        return [m, m * c[0], m * c[1], m * c[2],
                io[0, 0], io[0, 1], io[1, 1], io[0, 2], io[1, 2], io[2, 2]]
    xt = np.zeros((2, 3, 4))
    xt[0] = _identity_offset()
    xt[1] = _identity_offset()
    xt[1, 0, 3] = l1
    return Tree(name="two_link", parent=np.array([-1, 0], dtype=np.int32),
                joint_type=np.array([REVOLUTE, REVOLUTE], dtype=np.int32),
                axis=np.array([[0.0, -1.0, 0.0], [0.0, -1.0, 0.0]]), X_tree=xt,
                inertia=np.array([params(m1, lc1, i1), params(m2, lc2, i2)]),
                ee_bodies=[1])


def edge_tree(name: str) -> Tree:
    """Trees at the limits the model compiler accepts and the degenerate cases
    of the method.  Joint axes, offsets and inertias are drawn as for the
    random trees (seed 3500 + a fixed index per name).

    * ``chain64``: 64 revolute bodies in series (most bodies, depth 64).
    * ``star64``: one root body with 63 children (level width 63).
    * ``free_branches61``: free root with four 15-body branches mixing
      revolute and prismatic joints (61 bodies, nv 66).
    * ``rev1`` / ``pri1`` / ``free1``: a single revolute, prismatic or free body.
    * ``prismatic8``: eight prismatic joints in series.
    """
    specs = {
        "chain64": (list(range(-1, 63)), [REVOLUTE] * 64),
        "star64": ([-1] + [0] * 63, [REVOLUTE] * 64),
        "rev1": ([-1], [REVOLUTE]),
        "pri1": ([-1], [PRISMATIC]),
        "free1": ([-1], [FREE]),
        "prismatic8": (list(range(-1, 7)), [PRISMATIC] * 8),
    }
    if name == "free_branches61":
        parents, types = [-1], [FREE]
        for b in range(4):
            p = 0
            for j in range(15):
                parents.append(p)
                types.append(PRISMATIC if (j + b) % 4 == 3 else REVOLUTE)
                p = len(parents) - 1
        specs[name] = (parents, types)
    if name not in specs:
        raise KeyError(name)
    parents, types = specs[name]
    index = sorted(list(specs)).index(name)
    rng = np.random.default_rng(3500 + index)
    n = len(parents)
    is_leaf = [True] * n
    for q in parents:
        if q >= 0:
            is_leaf[q] = False
    depth = []
    for i, q in enumerate(parents):
        depth.append(1 if q < 0 else depth[q] + 1)
    leaves = sorted([i for i in range(n) if is_leaf[i]], key=lambda i: (-depth[i], i))
    return _build(name, parents, types, rng, ee=leaves[:4])


EDGE_TREES = ["chain64", "star64", "free_branches61", "rev1", "pri1", "free1", "prismatic8"]


def tree_by_name(name: str) -> Tree:
    table = {
        "chain7": chain7,
        "humanoid_large": humanoid_large,
        "humanoid_small": humanoid_small,
        "quadruped_spine": quadruped_spine,
    }
    if name in table:
        return table[name]()
    if name in EDGE_TREES:
        return edge_tree(name)
    if name.startswith("random"):
        n = int(name[len("random"):])
        sizes = [7, 11, 12, 18, 23]
        return random_tree(n, 3000 + sizes.index(n)) if n in sizes else random_tree(n, 3100 + n)
    raise KeyError(name)
