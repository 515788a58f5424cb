"""URDF front end: parse a robot description once into the model arrays.

The paper parses a URDF once into an immutable model holding the topology,
the spatial inertias and the precomputed constants (Fig. 1; Sec. 3.2 notes
that fixed joints are handled like the moving ones, with constants of their
own).  This module produces the arrays ``bard_model_create`` takes; the
constants are then computed by the library's model compiler.

Mapping of URDF to the model:

* ``revolute`` and ``continuous`` joints become revolute joints, ``prismatic``
  joints prismatic ones, a ``floating`` joint (or ``floating_base=True`` on a
  root link without one) the free joint of body 0.  ``planar`` joints are
  rejected.
* A joint's ``<origin>`` (xyz, rpy with R = Rz(yaw) Ry(pitch) Rx(roll)) is the
  pose of the joint frame in the parent link frame; the child link frame is the
  joint frame after the motion, and ``<axis>`` (default x) is expressed in it.
  These are the conventions of the model's ``X_tree`` and ``axis``.
* ``fixed`` joints are merged: the child link becomes part of its parent's
  body.  Its inertia is moved into the body's frame and added to the body's
  parameters (parameters about one origin add), and the joints below it are
  re-attached to the body with their origins composed with the fixed offset.
  Every link keeps a frame: ``frames[link] = (body, T)`` with T the link's
  pose in the body frame (body -1 is the world for links fixed to a
  non-floating root).
* A link's ``<inertial>`` (mass, COM origin, inertia about the COM in the COM
  frame) becomes the body-origin parameters
  ``[m, m c, I_xx, I_xy, I_yy, I_xz, I_yz, I_zz]`` with
  ``I_O = R I_C R^T + m (|c|^2 1 - c c^T)``.
* ``<mimic>`` couplings are ignored (every moving joint is a coordinate).

Bodies are numbered depth first from the root, so every parent precedes its
children.  A body whose merged links carry no mass is an error unless
``pad_massless`` gives a small mass (and an isotropic inertia of the same
magnitude, in kg m^2) to put on it.
"""

from __future__ import annotations

import xml.etree.ElementTree as ET
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

REVOLUTE, PRISMATIC, FREE = 0, 1, 2


@dataclass
class RobotModel:
    """Model arrays from a URDF (the layout ``Model.from_tree`` reads)."""

    name: str
    parent: np.ndarray        # int32 [n]
    joint_type: np.ndarray    # int32 [n]
    axis: np.ndarray          # float64 [n, 3]
    X_tree: np.ndarray        # float64 [n, 3, 4]
    inertia: np.ndarray       # float64 [n, 10]
    body_names: List[str]     # the link that starts each body
    joint_names: List[str]    # the joint of each body ("" for a free root added here)
    frames: Dict[str, Tuple[int, np.ndarray]] = field(default_factory=dict)
    gravity: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, -9.81]))

    @property
    def n_bodies(self) -> int:
        return int(self.parent.shape[0])

    def body(self, link: str) -> int:
        """Body index that carries ``link`` (-1: fixed to the world)."""
        return self.frames[link][0]


def _floats(text: Optional[str], n: int, default: float = 0.0) -> np.ndarray:
    if text is None:
        return np.full(n, default, dtype=np.float64)
    v = np.array([float(x) for x in text.split()], dtype=np.float64)
    if v.shape != (n,):
        raise ValueError(f"expected {n} numbers, got {text!r}")
    return v


def rpy_matrix(rpy) -> np.ndarray:
    """URDF fixed-axis roll-pitch-yaw: R = Rz(yaw) Ry(pitch) Rx(roll)."""
    r, p, y = rpy
    cr, sr, cp, sp, cy, sy = np.cos(r), np.sin(r), np.cos(p), np.sin(p), np.cos(y), np.sin(y)
    Rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]])
    Ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _origin(el) -> np.ndarray:
    T = np.eye(4)
    o = el.find("origin") if el is not None else None
    if o is not None:
        T[:3, :3] = rpy_matrix(_floats(o.get("rpy"), 3))
        T[:3, 3] = _floats(o.get("xyz"), 3)
    return T


def _link_params(link) -> np.ndarray:
    """Body-origin parameters of a link in its own frame (zeros without <inertial>)."""
    inl = link.find("inertial")
    if inl is None:
        return np.zeros(10)
    m_el = inl.find("mass")
    m = float(m_el.get("value")) if m_el is not None else 0.0
    T = _origin(inl)
    c, R = T[:3, 3], T[:3, :3]
    i_el = inl.find("inertia")
    g = (lambda k: float(i_el.get(k, "0"))) if i_el is not None else (lambda k: 0.0)
    Ic = np.array([[g("ixx"), g("ixy"), g("ixz")], [g("ixy"), g("iyy"), g("iyz")], [g("ixz"), g("iyz"), g("izz")]])
    return _params(m, c, R @ Ic @ R.T)


def _params(m: float, c: np.ndarray, Ic: np.ndarray) -> np.ndarray:
    Io = Ic + m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
    return np.array([m, *(m * c), Io[0, 0], Io[0, 1], Io[1, 1], Io[0, 2], Io[1, 2], Io[2, 2]])


def transform_params(pi: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Parameters of a link given in its frame, expressed in a frame where the
    link frame has pose T (rotation R, origin p)."""
    m = pi[0]
    if m == 0.0 and not np.any(pi):
        return np.zeros(10)
    R, p = T[:3, :3], T[:3, 3]
    Io = np.array([[pi[4], pi[5], pi[7]], [pi[5], pi[6], pi[8]], [pi[7], pi[8], pi[9]]])
    if m > 0:
        c = pi[1:4] / m
        Ic = Io - m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
        return _params(m, R @ c + p, R @ Ic @ R.T)
    return _params(0.0, np.zeros(3), R @ Io @ R.T)


def parse_urdf(text: str, floating_base: bool = False, pad_massless: Optional[float] = None) -> RobotModel:
    """Parse URDF text (use ``load_urdf`` for a file)."""
    root_el = ET.fromstring(text)
    if root_el.tag != "robot":
        raise ValueError("not a URDF: the root element must be <robot>")
    links = {l.get("name"): l for l in root_el.findall("link")}
    joints = []
    for j in root_el.findall("joint"):
        p_el, c_el = j.find("parent"), j.find("child")
        if p_el is None or c_el is None:
            raise ValueError(f"joint {j.get('name')!r} lacks <parent> or <child>")
        joints.append(j)
    child_joint = {}
    kids: Dict[str, List] = {name: [] for name in links}
    for j in joints:
        pl, cl = j.find("parent").get("link"), j.find("child").get("link")
        if pl not in links or cl not in links:
            raise ValueError(f"joint {j.get('name')!r} names an unknown link")
        if cl in child_joint:
            raise ValueError(f"link {cl!r} has two parent joints (not a tree)")
        child_joint[cl] = j
        kids[pl].append(j)
    roots = [l for l in links if l not in child_joint]
    if len(roots) != 1:
        raise ValueError(f"expected one root link, found {roots}")
    root = roots[0]

    parent, jtype, axis, xtree, params, body_names, joint_names = [], [], [], [], [], [], []
    frames: Dict[str, Tuple[int, np.ndarray]] = {}

    def new_body(p: int, t: int, ax, X: np.ndarray, link: str, jname: str) -> int:
        parent.append(p)
        jtype.append(t)
        axis.append(np.asarray(ax, dtype=np.float64))
        xtree.append(X[:3, :4].copy())
        params.append(np.zeros(10))
        body_names.append(link)
        joint_names.append(jname)
        return len(parent) - 1

    if floating_base:
        b0 = new_body(-1, FREE, [0.0, 0.0, 1.0], np.eye(4), root, "")
        frames[root] = (b0, np.eye(4))
    else:
        frames[root] = (-1, np.eye(4))

    def visit(link: str):
        body, T_bl = frames[link]
        if body >= 0:
            params[body] = params[body] + transform_params(_link_params(links[link]), T_bl)
        for j in kids[link]:
            child = j.find("child").get("link")
            jt = j.get("type")
            T_j = T_bl @ _origin(j)  # joint frame in the body frame
            if jt == "fixed":
                frames[child] = (body, T_j)
            elif jt in ("revolute", "continuous", "prismatic"):
                a_el = j.find("axis")
                ax = _floats(a_el.get("xyz") if a_el is not None else None, 3) if a_el is not None else np.array(
                    [1.0, 0.0, 0.0])
                if np.linalg.norm(ax) == 0:
                    raise ValueError(f"joint {j.get('name')!r} has a zero axis")
                b = new_body(body, PRISMATIC if jt == "prismatic" else REVOLUTE, ax, T_j, child, j.get("name"))
                frames[child] = (b, np.eye(4))
            elif jt == "floating":
                if body != -1 or link != root:
                    raise ValueError("a floating joint is only supported between the world root link and one child")
                b = new_body(-1, FREE, [0.0, 0.0, 1.0], T_j, child, j.get("name"))
                frames[child] = (b, np.eye(4))
            else:
                raise ValueError(f"joint {j.get('name')!r}: type {jt!r} is not supported")
            visit(child)

    visit(root)
    n = len(parent)
    if n == 0:
        raise ValueError("the URDF has no moving joint")
    pi = np.array(params)
    for i in range(n):
        if pi[i, 0] <= 0.0:
            if pad_massless is None:
                raise ValueError(f"body {i} (link {body_names[i]!r}) has no mass; give its links <inertial> "
                                 "or pass pad_massless")
            pi[i] += _params(pad_massless, np.zeros(3), pad_massless * np.eye(3))
    if FREE in jtype and jtype.index(FREE) != 0:
        raise ValueError("the free joint must be the first body")
    return RobotModel(name=root_el.get("name", ""), parent=np.array(parent, dtype=np.int32),
                      joint_type=np.array(jtype, dtype=np.int32), axis=np.array(axis),
                      X_tree=np.array(xtree), inertia=pi, body_names=body_names, joint_names=joint_names,
                      frames=frames)


def load_urdf(path: str, floating_base: bool = False, pad_massless: Optional[float] = None) -> RobotModel:
    with open(path) as f:
        return parse_urdf(f.read(), floating_base=floating_base, pad_massless=pad_massless)


def _rpy_of(R: np.ndarray) -> np.ndarray:
    """Roll, pitch, yaw with R = Rz(yaw) Ry(pitch) Rx(roll)."""
    pitch = np.arcsin(np.clip(-R[2, 0], -1.0, 1.0))
    if abs(R[2, 0]) < 1.0 - 1e-12:
        roll = np.arctan2(R[2, 1], R[2, 2])
        yaw = np.arctan2(R[1, 0], R[0, 0])
    else:  # gimbal lock: put the whole rotation about z into yaw
        roll = 0.0
        yaw = np.arctan2(-R[0, 1], R[1, 1])
    return np.array([roll, pitch, yaw])


def _num(x) -> str:
    return repr(float(x))


def _fmt(v) -> str:
    return " ".join(_num(x) for x in v)


def _inertia_xml(Ic) -> str:
    return (f'<inertia ixx="{_num(Ic[0, 0])}" ixy="{_num(Ic[0, 1])}" ixz="{_num(Ic[0, 2])}" '
            f'iyy="{_num(Ic[1, 1])}" iyz="{_num(Ic[1, 2])}" izz="{_num(Ic[2, 2])}"/>')


def to_urdf(parent, joint_type, axis, X_tree, inertia, name: str = "robot",
            extra_fixed: Optional[List[Tuple[int, np.ndarray, np.ndarray]]] = None) -> str:
    """URDF text of model arrays (revolute, prismatic, and a free body 0 written
    as a ``floating`` joint from a massless world link).  ``extra_fixed`` adds
    links on fixed joints: (body, 4x4 pose in the body frame, parameters in the
    new link's frame)."""
    n = len(parent)
    out = [f'<robot name="{name}">', '  <link name="world"/>']
    for i in range(n):
        pi = np.asarray(inertia[i], dtype=np.float64)
        m = pi[0]
        c = pi[1:4] / m
        Io = np.array([[pi[4], pi[5], pi[7]], [pi[5], pi[6], pi[8]], [pi[7], pi[8], pi[9]]])
        Ic = Io - m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
        out.append(f'  <link name="b{i}"><inertial><origin xyz="{_fmt(c)}" rpy="0 0 0"/>'
                   f'<mass value="{_num(m)}"/>{_inertia_xml(Ic)}</inertial></link>')
    for i in range(n):
        p = "world" if parent[i] < 0 else f"b{parent[i]}"
        X = np.asarray(X_tree[i])
        t = {REVOLUTE: "revolute", PRISMATIC: "prismatic", FREE: "floating"}[int(joint_type[i])]
        lim = '<limit lower="-1e9" upper="1e9" effort="1e9" velocity="1e9"/>' if t != "floating" else ""
        out.append(f'  <joint name="j{i}" type="{t}"><parent link="{p}"/><child link="b{i}"/>'
                   f'<origin xyz="{_fmt(X[:, 3])}" rpy="{_fmt(_rpy_of(X[:, :3]))}"/>'
                   f'<axis xyz="{_fmt(axis[i])}"/>{lim}</joint>')
    for k, (b, T, pi) in enumerate(extra_fixed or []):
        m = pi[0]
        c = pi[1:4] / m
        Io = np.array([[pi[4], pi[5], pi[7]], [pi[5], pi[6], pi[8]], [pi[7], pi[8], pi[9]]])
        Ic = Io - m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
        out.append(f'  <link name="f{k}"><inertial><origin xyz="{_fmt(c)}" rpy="0 0 0"/>'
                   f'<mass value="{_num(m)}"/>{_inertia_xml(Ic)}</inertial></link>')
        out.append(f'  <joint name="fj{k}" type="fixed"><parent link="b{b}"/><child link="f{k}"/>'
                   f'<origin xyz="{_fmt(T[:3, 3])}" rpy="{_fmt(_rpy_of(T[:3, :3]))}"/></joint>')
    out.append("</robot>")
    return "\n".join(out)
