"""URDF front end (CPU).

* Round trip: model arrays written as URDF and parsed back are the same
  arrays (revolute, prismatic and floating joints).
* Fixed joints are merged into their parent's body.  Pin: the same URDF with
  each fixed joint turned into a revolute joint held at q = qd = qdd = 0
  describes the same mechanism, so the oracle's torques, mass matrix and body
  poses of the merged model equal those of the unmerged one on the shared
  coordinates, and each merged link's recorded frame equals the pose of the
  corresponding unmerged body.
* Conventions: roll-pitch-yaw closed forms, an inertia given in a rotated COM
  frame, and the documented errors.
"""

import numpy as np
import pytest

import synth
from oracle import OracleModel
from paper_2605_31481_amd import urdf


def _arrays(t):
    return t.parent, t.joint_type, t.axis, t.X_tree, t.inertia


@pytest.mark.parametrize("name", ["chain7", "quadruped_spine", "humanoid_large", "random23", "prismatic8"])
def test_round_trip(name):
    t = synth.tree_by_name(name)
    text = urdf.to_urdf(*_arrays(t), name=name)
    r = urdf.parse_urdf(text)
    # bodies come back depth first: perm[k] = the original index of parsed body k
    perm = np.array([int(nm[1:]) for nm in r.body_names])
    assert sorted(perm) == list(range(t.n_bodies))
    inv = np.argsort(perm)
    assert all(r.parent[k] < k for k in range(t.n_bodies))
    np.testing.assert_array_equal(r.parent, [-1 if t.parent[o] < 0 else inv[t.parent[o]] for o in perm])
    np.testing.assert_array_equal(r.joint_type, t.joint_type[perm])
    free = t.joint_type[perm] == synth.FREE
    np.testing.assert_allclose(r.axis[~free], t.axis[perm][~free], rtol=0, atol=1e-15)
    np.testing.assert_allclose(r.X_tree, t.X_tree[perm], rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.inertia, t.inertia[perm], rtol=1e-12, atol=1e-14)


def test_rpy_closed_forms():
    np.testing.assert_allclose(urdf.rpy_matrix([0, 0, np.pi / 2]) @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(urdf.rpy_matrix([np.pi / 2, 0, 0]) @ [0, 1, 0], [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(urdf.rpy_matrix([0, np.pi / 2, 0]) @ [0, 0, 1], [1, 0, 0], atol=1e-15)
    # fixed axes: roll first, then pitch, then yaw
    r, p, y = 0.3, -0.7, 1.1
    Rx = urdf.rpy_matrix([r, 0, 0])
    Ry = urdf.rpy_matrix([0, p, 0])
    Rz = urdf.rpy_matrix([0, 0, y])
    np.testing.assert_allclose(urdf.rpy_matrix([r, p, y]), Rz @ Ry @ Rx, atol=1e-15)


def test_inertia_in_rotated_com_frame():
    text = """<robot name="r"><link name="base"/>
      <link name="a"><inertial><origin xyz="0.1 -0.2 0.3" rpy="0 0 1.5707963267948966"/><mass value="2"/>
        <inertia ixx="0.1" ixy="0" ixz="0" iyy="0.2" iyz="0" izz="0.3"/></inertial></link>
      <joint name="j" type="continuous"><parent link="base"/><child link="a"/><axis xyz="0 0 1"/></joint>
    </robot>"""
    r = urdf.parse_urdf(text)
    m, c = 2.0, np.array([0.1, -0.2, 0.3])
    Ic = np.diag([0.2, 0.1, 0.3])        # x and y principal axes swapped by the 90 degree yaw
    Io = Ic + m * (c @ c * np.eye(3) - np.outer(c, c))
    want = [m, *(m * c), Io[0, 0], Io[0, 1], Io[1, 1], Io[0, 2], Io[1, 2], Io[2, 2]]
    np.testing.assert_allclose(r.inertia[0], want, atol=1e-15)
    assert r.joint_type[0] == urdf.REVOLUTE and r.parent[0] == -1


def _fixed_case(name, seed):
    t = synth.tree_by_name(name)
    rng = np.random.default_rng(seed)
    extra = []
    for b in rng.choice(t.n_bodies, 3, replace=False):
        T = np.eye(4)
        T[:3, :3] = urdf.rpy_matrix(rng.uniform(-np.pi, np.pi, 3))
        T[:3, 3] = rng.uniform(-0.3, 0.3, 3)
        extra.append((int(b), T, synth.random_inertia_params(rng)))
    return t, urdf.to_urdf(*_arrays(t), extra_fixed=extra), extra


@pytest.mark.parametrize("name", ["quadruped_spine", "humanoid_small", "random12"])
def test_fixed_joints_merge_like_locked_joints(name):
    t, text, extra = _fixed_case(name, 11)
    merged = urdf.parse_urdf(text)
    assert merged.n_bodies == t.n_bodies
    locked = urdf.parse_urdf(text.replace('type="fixed">', 'type="revolute"><axis xyz="0 0 1"/>'))
    assert locked.n_bodies == t.n_bodies + len(extra)
    oa = OracleModel(merged.parent, merged.joint_type, merged.axis, merged.X_tree, merged.inertia)
    ob = OracleModel(locked.parent, locked.joint_type, locked.axis, locked.X_tree, locked.inertia)
    q, qd, qdd = synth.random_state(t, 5, 12)
    # coordinates of the locked model: the merged model's, zeros for the extra joints
    ia = {nm: i for i, nm in enumerate(merged.body_names)}
    qo_b, vo_b = _offsets(locked)
    qo_a, vo_a = _offsets(merged)
    qb = np.zeros((5, ob.nq))
    qdb = np.zeros((5, ob.nv))
    qddb = np.zeros((5, ob.nv))
    vmap = []
    for j, nm in enumerate(locked.body_names):
        if nm in ia:
            i = ia[nm]
            nqj = 7 if merged.joint_type[i] == urdf.FREE else 1
            nvj = 6 if merged.joint_type[i] == urdf.FREE else 1
            qb[:, qo_b[j]:qo_b[j] + nqj] = q[:, qo_a[i]:qo_a[i] + nqj]
            qdb[:, vo_b[j]:vo_b[j] + nvj] = qd[:, vo_a[i]:vo_a[i] + nvj]
            qddb[:, vo_b[j]:vo_b[j] + nvj] = qdd[:, vo_a[i]:vo_a[i] + nvj]
            vmap += list(range(vo_b[j], vo_b[j] + nvj))
    vmap = np.array(vmap)
    np.testing.assert_allclose(oa.rnea(q, qd, qdd), ob.rnea(qb, qdb, qddb)[:, vmap], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(oa.crba(q), ob.crba(qb)[:, vmap][:, :, vmap], rtol=1e-11, atol=1e-11)
    Ta, Tb = oa.fk(q), ob.fk(qb)
    for j, nm in enumerate(locked.body_names):
        if nm in ia:
            np.testing.assert_allclose(Ta[:, ia[nm]], Tb[:, j], atol=1e-12)
        else:   # a merged link: its recorded frame in the merged body
            body, T = merged.frames[nm]
            P = np.concatenate([Ta[:, body], np.tile([0, 0, 0, 1.0], (5, 1, 1))], axis=1) @ T
            np.testing.assert_allclose(P[:, :3], Tb[:, j], atol=1e-12)


def _offsets(r):
    qo, vo, a, b = [], [], 0, 0
    for t in r.joint_type:
        qo.append(a)
        vo.append(b)
        a += 7 if t == urdf.FREE else 1
        b += 6 if t == urdf.FREE else 1
    return qo, vo


def test_floating_base_option_and_errors():
    text = """<robot name="r">
      <link name="torso"><inertial><mass value="3"/><inertia ixx="0.1" iyy="0.1" izz="0.1" ixy="0" ixz="0" iyz="0"/></inertial></link>
      <link name="arm"><inertial><mass value="1"/><inertia ixx="0.01" iyy="0.01" izz="0.01" ixy="0" ixz="0" iyz="0"/></inertial></link>
      <link name="hand"/>
      <joint name="s" type="revolute"><parent link="torso"/><child link="arm"/><origin xyz="0 0.2 0"/><axis xyz="0 1 0"/></joint>
      <joint name="w" type="fixed"><parent link="arm"/><child link="hand"/><origin xyz="0.3 0 0"/></joint>
    </robot>"""
    fixed_base = urdf.parse_urdf(text)
    assert fixed_base.n_bodies == 1 and fixed_base.body("torso") == -1 and fixed_base.body("hand") == 0
    np.testing.assert_allclose(fixed_base.frames["hand"][1][:3, 3], [0.3, 0, 0])
    floating = urdf.parse_urdf(text, floating_base=True)
    assert list(floating.joint_type) == [urdf.FREE, urdf.REVOLUTE] and list(floating.parent) == [-1, 0]
    assert floating.inertia[0, 0] == 3.0
    with pytest.raises(ValueError, match="not supported"):
        urdf.parse_urdf(text.replace('type="revolute"', 'type="planar"'))
    with pytest.raises(ValueError, match="no mass"):
        urdf.parse_urdf(text.replace('<link name="arm"><inertial><mass value="1"/><inertia ixx="0.01" iyy="0.01" '
                                     'izz="0.01" ixy="0" ixz="0" iyz="0"/></inertial></link>',
                                     '<link name="arm"/>'))
    padded = urdf.parse_urdf(text.replace('<link name="arm"><inertial><mass value="1"/><inertia ixx="0.01" '
                                          'iyy="0.01" izz="0.01" ixy="0" ixz="0" iyz="0"/></inertial></link>',
                                          '<link name="arm"/>'), pad_massless=1e-4)
    assert padded.inertia[0, 0] == 1e-4
    with pytest.raises(ValueError, match="one root"):
        urdf.parse_urdf(text.replace("</robot>", '<link name="stray"/></robot>'))
