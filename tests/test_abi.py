"""Host-side tests of the C ABI (no GPU needed).

* libbard.so loads and exports every function include/bard.h declares;
* model validation returns the documented status codes;
* the model compiler's Rodrigues constants reproduce the naive parent-child
  product T_joint * R_axis(q) of eq. (1) through eqs. (4)-(5) in FP64;
* level schedules have the expected lanes per instance and depth;
* operators reject bad arguments before touching a device, and B = 0 is a no-op.
"""

import ctypes

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from paper_2605_31481_amd import bard


def test_every_declared_symbol_is_exported():
    names = bard.declared_symbols()
    assert len(names) >= 20
    lib = ctypes.CDLL(bard.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _arrays(tree):
    return (tree.parent.copy(), tree.joint_type.copy(), tree.axis.copy(), tree.X_tree.copy(),
            tree.inertia.copy())


def _create(parent, jt, axis, xt, pi):
    h = ctypes.c_void_p()
    pa = np.ascontiguousarray(parent, dtype=np.int32)
    ja = np.ascontiguousarray(jt, dtype=np.int32)
    ax = np.ascontiguousarray(axis, dtype=np.float64)
    x = np.ascontiguousarray(xt, dtype=np.float64)
    p = np.ascontiguousarray(pi, dtype=np.float64)
    rc = bard.bard_model_create(len(pa), pa.ctypes.data_as(bard._c_i32p), ja.ctypes.data_as(bard._c_i32p),
                                ax.ctypes.data_as(bard._c_dp), x.ctypes.data_as(bard._c_dp),
                                p.ctypes.data_as(bard._c_dp), ctypes.byref(h))
    if rc == 0:
        bard.bard_model_destroy(h)
    return rc


def test_valid_models_create():
    for t in [synth.chain7(), synth.humanoid_large(), synth.humanoid_small(), synth.quadruped_spine(),
              *synth.multi_trees()]:
        assert _create(*_arrays(t)) == 0, bard.bard_last_error()


@pytest.mark.parametrize("mutate,code", [
    (lambda a: a[0].__setitem__(3, 5), -2),                       # parent >= i
    (lambda a: a[0].__setitem__(3, -7), -2),                      # bad parent
    (lambda a: a[1].__setitem__(2, 3), -7),                       # fixed joint
    (lambda a: a[1].__setitem__(2, 9), -2),                       # unknown joint type
    (lambda a: a[1].__setitem__(2, 2), -2),                       # free joint not at the root
    (lambda a: a[2].__setitem__(4, 0.0), -2),                     # zero axis
    (lambda a: a[4].__setitem__((1, 0), 0.0), -3),                # zero mass
    (lambda a: a[4].__setitem__((1, 4), -1.0), -3),               # inertia not PD
    (lambda a: a[3].__setitem__((2, 0, 0), 2.0), -1),             # X_tree not a rotation
    (lambda a: a[2].__setitem__((1, 0), np.nan), -1),             # non-finite
])
def test_model_validation(mutate, code):
    a = list(_arrays(synth.chain7()))
    mutate(a)
    assert _create(*a) == code


def test_too_many_bodies():
    t = synth.random_tree(12, 5)
    par = np.arange(-1, 64, dtype=np.int32)
    n = len(par)
    ax = np.tile([0.0, 0.0, 1.0], (n, 1))
    xt = np.tile(t.X_tree[0], (n, 1, 1))
    pi = np.tile(t.inertia[0], (n, 1))
    assert _create(par, np.zeros(n, np.int32), ax, xt, pi) == -1


@pytest.mark.parametrize("name", ["chain7", "humanoid_large", "humanoid_small", "random23"])
def test_rodrigues_constants_match_naive_product(name):
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    rng = np.random.default_rng(1)
    for i in range(tree.n_bodies):
        Rp, tp = tree.X_tree[i][:, :3], tree.X_tree[i][:, 3]
        for _ in range(5):
            jt = tree.joint_type[i]
            if jt == synth.FREE:
                q = np.concatenate([rng.uniform(-1, 1, 3), rng.standard_normal(4)])
                Rj = Rotation.from_quat(q[3:] / np.linalg.norm(q[3:])).as_matrix()
                tj = q[:3]
            elif jt == synth.REVOLUTE:
                q = rng.uniform(-np.pi, np.pi, 1)
                Rj = Rotation.from_rotvec(q[0] * tree.axis[i]).as_matrix()
                tj = np.zeros(3)
            else:
                q = rng.uniform(-0.3, 0.3, 1)
                Rj = np.eye(3)
                tj = q[0] * tree.axis[i]
            # eq. (1): T_pc = T_joint * motion(q) * T_link with T_link = identity
            R_ref = Rp @ Rj
            t_ref = Rp @ tj + tp
            R, t = m.joint_transform(i, q)
            np.testing.assert_allclose(R, R_ref, rtol=0, atol=2e-15)
            np.testing.assert_allclose(t, t_ref, rtol=0, atol=2e-15)


@pytest.mark.parametrize("name,lanes,depth", [
    ("chain7", 1, 7), ("humanoid_large", 8, 9), ("humanoid_small", 4, 9), ("quadruped_spine", 4, 5)])
def test_schedule_shape(name, lanes, depth):
    m = bard.Model.from_tree(synth.tree_by_name(name))
    assert m.lanes_per_instance == lanes
    assert m.depth == depth


def test_operator_argument_errors_without_device():
    m = bard.Model.from_tree(synth.chain7())
    h = m.handle
    # B = 0 is a no-op that never touches a device
    assert bard.bard_rnea(h, None, 0, None, None, None, None, None, None, 0, 0, 0, None) == 0
    # NULL arrays with B > 0
    assert bard.bard_rnea(h, None, 0, None, None, None, None, None, None, 0, 0, 8, None) == -1
    # bad dtype
    assert bard.bard_crba(h, None, 7, None, None, None, 0, 8, None) == -1
    # negative batch
    assert bard.bard_fk(h, None, 0, None, None, None, 0, -1, None) == -1
    # bad end-effector count
    ee = (ctypes.c_int32 * 1)(6)
    assert bard.bard_jacobian(h, None, 0, None, 0, ee, 0, None, None, 0, 4, None) == -1
    assert bard.bard_jacobian(h, None, 0, None, 1, ee, 5, None, None, 0, 4, None) == -1
    assert "frame" in bard.bard_last_error().decode() or bard.bard_last_error()


def test_path_kinematics_argument_errors_without_device():
    m = bard.Model.from_tree(synth.humanoid_small())
    h = m.handle
    f = bard.bard_path_kinematics
    assert f(h, 0, None, 3, 0, None, None, None, 0, None) == 0        # B = 0
    assert f(h, 0, None, 3, 0, None, None, None, 8, None) == -1       # NULL q, no output
    assert f(h, 0, None, m.n_bodies, 0, None, None, None, 8, None) == -1  # ee_body out of range
    assert f(h, 0, None, -1, 0, None, None, None, 8, None) == -1
    assert f(h, 0, None, 3, 2, None, None, None, 8, None) == -1       # bad frame
    assert f(h, 2, None, 3, 0, None, None, None, 8, None) == -1       # bad dtype
    assert f(None, 0, None, 3, 0, None, None, None, 8, None) == -1    # NULL model


def test_workspace_capacity_checked_on_host():
    m = bard.Model.from_tree(synth.chain7())
    ws = ctypes.c_void_p()
    assert bard.bard_ws_create(m.handle, 0, 128, ctypes.byref(ws)) == 0
    assert bard.bard_crba(m.handle, ws, 0, None, None, None, 0, 129, None) == -6
    assert bard.bard_crba(m.handle, ws, 1, None, None, None, 0, 16, None) == -1
    # tier policy: any OR of the three tier bits, nothing else
    for p in range(8):
        assert bard.bard_ws_set_policy(ws, p) == 0
    for p in (8, -1, 16, 9):
        assert bard.bard_ws_set_policy(ws, p) == -1
    assert (bard.TIER_KINEMATICS, bard.TIER_MASS, bard.TIER_BIAS) == (1, 2, 4)
    assert bard.bard_ws_destroy(ws) == 0


def test_adjoint_argument_errors_without_device():
    m = bard.Model.from_tree(synth.quadruped_spine())
    h = m.handle
    # B = 0 is a no-op
    assert bard.bard_rnea_vjp(h, 0, None, None, None, None, None, None, None, None, None, None, 0, None) == 0
    assert bard.bard_fk_vjp(h, 0, None, None, None, None, 0, None) == 0
    # NULL arrays, bad dtype, negative batch
    assert bard.bard_rnea_vjp(h, 0, None, None, None, None, None, None, None, None, None, None, 8, None) == -1
    assert bard.bard_fk_vjp(h, 0, None, None, None, None, 8, None) == -1
    assert bard.bard_fk_vjp(h, 3, None, None, None, None, 8, None) == -1
    assert bard.bard_rnea_vjp(h, 0, None, None, None, None, None, None, None, None, None, None, -2, None) == -1


def test_aba_vjp_argument_errors_without_device():
    m = bard.Model.from_tree(synth.humanoid_small())
    h = m.handle
    assert bard.bard_aba_vjp(h, 0, None, None, None, None, None, None, None, None, 0, None) == 0   # B = 0
    assert bard.bard_aba_vjp(h, 0, None, None, None, None, None, None, None, None, 8, None) == -1  # NULL arrays
    assert bard.bard_aba_vjp(h, 3, None, None, None, None, None, None, None, None, 8, None) == -1  # bad dtype
    assert bard.bard_aba_vjp(None, 0, None, None, None, None, None, None, None, None, 8, None) == -1


def test_adjoints_of_free_joint_trees_check_arguments():
    """Free-root trees have adjoints; their argument errors are still caught
    on the host before any launch."""
    m = bard.Model.from_tree(synth.humanoid_small())
    h = m.handle
    assert bard.bard_rnea_vjp(h, 0, None, None, None, None, None, None, None, None, None, None, 0, None) == 0
    assert bard.bard_rnea_vjp(h, 0, None, None, None, None, None, None, None, None, None, None, 8, None) == -1
    assert bard.bard_fk_vjp(h, 0, None, None, None, None, 8, None) == -1
    assert "NULL" in bard.bard_last_error().decode()


def test_plan_host_side():
    """Plan creation, tip end effectors and configuration need no device."""
    trees = synth.multi_trees()
    ms = [bard.Model.from_tree(t) for t in trees]
    p = bard.Plan(ms, synth.MULTI_BATCHES)
    for i, t in enumerate(trees):
        assert p.ee(i) == list(t.ee_bodies)
    assert p.config == {"tile": 16, "fusion": 0, "order": 0, "lanes": 0, "from_cache": False}
    p.configure(32, 2, 1, 1)
    assert p.config["lanes"] == 1
    assert p.config["tile"] == 32 and p.config["fusion"] == 2
    with pytest.raises(bard.BardError):
        p.configure(12, 0, 0)
    p.configure(16, 3, 0)                      # the generated multi-tree kernel
    assert p.config["fusion"] == 3
    with pytest.raises(bard.BardError):
        p.configure(16, 4, 0)
    with pytest.raises(bard.BardError):
        p.configure(16, 0, 0, 2)
    # two operators have no fused kernel: only one launch per operator is valid
    p2 = bard.Plan(ms, synth.MULTI_BATCHES, op_mask=bard.PLAN_RNEA | bard.PLAN_CRBA)
    assert p2.config["fusion"] == 2
    with pytest.raises(bard.BardError):
        p2.configure(16, 0, 0)
    with pytest.raises(bard.BardError):          # the generated kernel needs all three operators
        p2.configure(16, 3, 0)
    h = ctypes.c_void_p()
    hs = (ctypes.c_void_p * 1)(ms[0].handle)
    bs = (ctypes.c_int64 * 1)(8)
    assert bard.bard_plan_create(hs, 1, bs, 0, 0, ctypes.byref(h)) == -1
    assert bard.bard_plan_create(hs, 0, bs, 7, 0, ctypes.byref(h)) == -1
    assert bard.bard_plan_create(hs, 1, bs, 7, 2, ctypes.byref(h)) == -1
    assert bard.bard_plan_run(None, None, None) == -1


def test_free_root_must_be_the_only_world_body():
    t = synth.humanoid_small()
    parent = np.array(t.parent).copy()
    parent[3] = -1          # a second body on the world next to the free root
    with pytest.raises(bard.BardError) as e:
        bard.Model(parent, t.joint_type, t.axis, t.X_tree, t.inertia)
    assert e.value.status == -2
