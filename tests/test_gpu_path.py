"""GPU parity of the standalone kinematics of one chain (bard_path_kinematics,
Sec. 3.1's path-only FK and Jacobian): the end effector's world pose and the
eq. (7) Jacobian columns of its root-to-body path against the FP64 oracle's
FK and Jacobian, entry by entry for the Jacobian (per column scale) and per
pose block, in both frames, FP32 and FP64, instance-minor and instance-major
layouts, at sizes spanning several workgroups with a ragged tail, on deep
(64-body chain), wide (64-body star) and free-root trees, and at 262,144
instances on sampled outputs."""

import ctypes

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from parity_util import assert_jacobian, assert_normwise, from_dev, inputs, oracle_for, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ("chain7", "float32", 4096),
    ("chain7", "float64", 65),
    ("humanoid_large", "float32", 1000),
    ("humanoid_large", "float64", 100),
    ("quadruped_spine", "float32", 513),
    ("random18", "float32", 300),
    ("chain64", "float32", 257),
    ("chain64", "float64", 65),
    ("star64", "float64", 70),
    ("free_branches61", "float32", 129),
    ("prismatic8", "float32", 129),
    ("free1", "float32", 65),
    ("rev1", "float64", 5),
    ("pri1", "float32", 3),
]


def _ees(tree):
    ee = list(tree.ee_bodies) if len(tree.ee_bodies) else []
    return sorted(set(ee + [0, tree.n_bodies - 1]))


@pytest.fixture(params=["1", "16"], ids=["lane_per_instance", "16_lanes_per_instance"])
def lanes(request, monkeypatch):
    """Both forms of the kernel whatever the batch (BARD_PATH_LANES pins one)."""
    monkeypatch.setenv("BARD_PATH_LANES", request.param)
    return request.param


@pytest.mark.parametrize("frame", [0, 1])
@pytest.mark.parametrize("name,dtype,B", CASES)
def test_path_kinematics_matches_oracle(name, dtype, B, frame, lanes):
    say(f"[gpu] path kinematics {name} {dtype} B={B} frame={frame} lanes={lanes}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    q, _, _ = inputs(tree, B, 4100, dtype)
    qd_ = to_dev(q, dtype)
    T = om.fk(q).reshape(B, tree.n_bodies, 12)
    for e in _ees(tree):
        pose, J = m.path_kinematics(qd_, e, frame=frame)
        assert_normwise(f"pose[{e}]", from_dev(pose)[:, None, :], T[:, e:e + 1], dtype)
        assert_jacobian(f"J[{e}]", from_dev(J), om.jacobian(q, [e], frame=frame), dtype)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_path_outputs_alone_layouts_and_full_tree_operators(dtype, lanes):
    """Pose only, Jacobian only, batch-major arrays, and agreement with the
    full-tree operators' blocks for the same end effector."""
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    B = 333
    q, _, _ = inputs(tree, B, 4101, dtype)
    e = tree.ee_bodies[2]
    T = om.fk(q).reshape(B, tree.n_bodies, 12)[:, e:e + 1]
    Jr = om.jacobian(q, [e], frame=1)
    pose, J = m.path_kinematics(to_dev(q, dtype), e, frame=1, jacobian=False)
    assert J is None
    assert_normwise("pose only", from_dev(pose)[:, None, :], T, dtype)
    pose, J = m.path_kinematics(to_dev(q, dtype), e, frame=1, pose=False)
    assert pose is None
    assert_jacobian("J only", from_dev(J), Jr, dtype)
    qa = to_dev(q, dtype, layout="aos")
    pose, J = m.path_kinematics(qa, e, frame=1, layout="aos")
    assert pose.shape == (B, 12) and J.shape == (B, 6 * tree.nv)
    assert_normwise("aos pose", from_dev(pose, layout="aos")[:, None, :], T, dtype)
    assert_jacobian("aos J", from_dev(J, layout="aos"), Jr, dtype)
    # the same quantities from the whole-tree kernels
    Jf = from_dev(m.jacobian(to_dev(q, dtype), [e], frame=1))
    Tf = from_dev(m.fk(to_dev(q, dtype))).reshape(B, tree.n_bodies, 12)[:, e:e + 1]
    assert_jacobian("J vs bard_jacobian", from_dev(m.path_kinematics(to_dev(q, dtype), e, frame=1)[1]),
                    Jf.reshape(Jr.shape), dtype)
    assert_normwise("pose vs bard_fk", from_dev(pose, layout="aos")[:, None, :], Tf, dtype)


@pytest.mark.parametrize("pin", [None, "16"])
def test_path_large_batch_sampled(pin, monkeypatch):
    """262,144 instances of the free-root humanoid, sampled against the
    oracle: the form the batch selects (one lane per instance, 4096
    workgroups plus the zero-column rows) and the 16-lane form (65,536
    workgroups)."""
    import torch
    if pin:
        monkeypatch.setenv("BARD_PATH_LANES", pin)
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    B = 262144
    q, _, _ = inputs(tree, B, 4102, "float32")
    e = tree.ee_bodies[0]
    say(f"[gpu] path kinematics humanoid_large float32 B={B} sampled, lanes {pin or 'by batch'}")
    pose, J = m.path_kinematics(to_dev(q, "float32"), e, frame=0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4103)
    idx = np.unique(np.concatenate([rng.choice(B, 1024, replace=False), [0, B - 1]]))
    qs = q[idx]
    pose_s = pose[:, torch.from_numpy(idx).cuda()]
    J_s = J[:, torch.from_numpy(idx).cuda()]
    assert_normwise("pose", from_dev(pose_s)[:, None, :], om.fk(qs).reshape(len(idx), -1, 12)[:, e:e + 1], "float32")
    assert_jacobian("J", from_dev(J_s), om.jacobian(qs, [e], frame=0), "float32")


def test_path_edge_arguments():
    import torch
    tree = synth.chain7()
    m = bard.Model.from_tree(tree)
    q = torch.zeros(tree.nq, 0, device="cuda")
    pose, J = m.path_kinematics(q, 3)  # B = 0: nothing launched
    assert pose.shape == (12, 0)
    q = torch.zeros(tree.nq, 8, device="cuda")
    with pytest.raises(bard.BardError) as ei:
        m.path_kinematics(q, tree.n_bodies)
    assert ei.value.status == -1
    with pytest.raises(ValueError):
        m.path_kinematics(q, 0, pose=False, jacobian=False)
    rc = bard.bard_path_kinematics(m.handle, 0, ctypes.c_void_p(q.data_ptr()), 2, 5, None, None, None, 8, None)
    assert rc == -1
