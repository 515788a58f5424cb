"""GPU parity of the model-specialised single-operator kernels: inverse
dynamics (bard_model_specialize_rnea), the mass matrix
(bard_model_specialize_crba), the Jacobians
(bard_model_specialize_jacobian) and the world poses
(bard_model_specialize_fk), against the FP64 oracle entry by entry on
workload and edge trees, split and whole forms, FP32 and FP64, sizes
spanning several 64-instance groups with a ragged tail; the mass matrix's
structural zeros from extra workgroups and from the lanes; routing (calls
with a workspace or an inertia override keep the generic kernel) and
unrouting."""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from parity_util import (assert_jacobian, assert_mass, assert_normwise, assert_tau, entry_scales, fk_ref_blocks,
                         from_dev, inputs, oracle_for, say, to_dev)

pytestmark = pytest.mark.gpu

CASES = [("chain7", "float32", 1000), ("chain7", "float64", 65), ("quadruped_spine", "float32", 513),
         ("random23", "float32", 300), ("humanoid_small", "float64", 40), ("humanoid_large", "float32", 1000),
         ("humanoid_large", "float64", 64), ("prismatic8", "float32", 129), ("star64", "float32", 70),
         ("free1", "float32", 65), ("rev1", "float64", 5)]


@pytest.mark.parametrize("form", ["split", "whole"])
@pytest.mark.parametrize("name,dtype,B", CASES)
def test_specialized_rnea_matches_oracle(name, dtype, B, form):
    say(f"[gpu] specialised rnea {name} {dtype} B={B} form={form}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    m.specialize_rnea(dtype=dtype, form=form)
    assert m.specialized_rnea_info(dtype=dtype, form=form)["routed"]
    om = oracle_for(tree)
    q, qd, qdd = inputs(tree, B, 6100, dtype)
    tau = from_dev(m.rnea(*(to_dev(x, dtype) for x in (q, qd, qdd))))
    st, _ = entry_scales(om, tree, q, qd, qdd, mass=False)
    assert_tau("spec rnea", tau, om.rnea(q, qd, qdd), st, dtype)


def test_specialized_rnea_routing():
    import torch
    say("[gpu] specialised rnea routing")
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    ref = bard.Model.from_tree(tree)   # never specialised: the generic kernel
    B = 777
    q, qd, qdd = inputs(tree, B, 6200, "float32")
    d = [to_dev(x, "float32") for x in (q, qd, qdd)]
    gen = ref.rnea(*d)
    m.specialize_rnea()
    spec = m.rnea(*d)
    torch.cuda.synchronize()
    assert not torch.equal(spec, gen)          # a different kernel (different rounding)
    om = oracle_for(tree)
    st, _ = entry_scales(om, tree, q, qd, qdd, mass=False)
    assert_tau("routed", from_dev(spec), om.rnea(q, qd, qdd), st, "float32")
    # with a workspace or an inertia override the generic kernel runs
    ws = bard.Workspace(m, B)
    ws.set_policy(0)
    assert torch.equal(m.rnea(*d, ws=ws), gen)
    inertia = torch.from_numpy(tree.inertia).float().cuda()
    assert torch.equal(m.rnea(*d, inertia=inertia), ref.rnea(*d, inertia=inertia))
    # the chain operator is unaffected; unrouting restores the generic results
    ee = tree.ee_bodies
    for a, b in zip(m.chain(*d, ee), ref.chain(*d, ee)):
        assert torch.equal(a, b)
    m.specialize_rnea(route=False)
    assert torch.equal(m.rnea(*d), gen)
    assert not m.specialized_rnea_info()["routed"]


def test_specialized_rnea_refuses_deep_trees():
    m = bard.Model.from_tree(synth.tree_by_name("chain64"))
    with pytest.raises(bard.BardError) as ei:
        m.specialize_rnea()
    assert ei.value.status == -7


@pytest.mark.parametrize("form", ["split", "whole"])
@pytest.mark.parametrize("name,dtype,B", CASES)
def test_specialized_crba_matches_oracle(name, dtype, B, form):
    say(f"[gpu] specialised crba {name} {dtype} B={B} form={form}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    m.specialize_op("crba", dtype=dtype, form=form)
    assert m.specialized_op_info("crba", dtype=dtype, form=form)["routed"]
    om = oracle_for(tree)
    q, _, _ = inputs(tree, B, 6300, dtype)
    M = from_dev(m.crba(to_dev(q, dtype))).reshape(B, tree.nv, tree.nv)
    _, sm = entry_scales(om, tree, q, tau=False)
    assert_mass("spec crba", M, om.crba(q), sm, dtype)
    assert (M == np.transpose(M, (0, 2, 1))).all(), "M is bitwise symmetric"


@pytest.mark.parametrize("B", [4096, 4097])
def test_specialized_crba_zero_rows(B):
    """B = 4096 instance-minor: extra workgroups write the structural zeros;
    B = 4097 (not a multiple of the 16-byte vector): the lanes do.  The
    output starts as NaN, so an unwritten entry shows."""
    import torch
    say(f"[gpu] specialised crba zero rows B={B}")
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    m.specialize_op("crba")
    q, _, _ = inputs(tree, B, 6400, "float32")
    out = torch.full((tree.nv * tree.nv, B), float("nan"), device="cuda")
    m.crba(to_dev(q, "float32"), out=out)
    torch.cuda.synchronize()
    assert not torch.isnan(out).any()
    idx = np.sort(np.random.default_rng(B).choice(B, 256, replace=False))
    om = oracle_for(tree)
    _, sm = entry_scales(om, tree, q[idx], tau=False)
    assert_mass("zero rows", from_dev(out)[idx].reshape(-1, tree.nv, tree.nv), om.crba(q[idx]), sm, "float32")


def test_specialized_crba_routing():
    import torch
    say("[gpu] specialised crba routing")
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)
    ref = bard.Model.from_tree(tree)
    B = 300
    q, qd, qdd = inputs(tree, B, 6500, "float32")
    d = [to_dev(x, "float32") for x in (q, qd, qdd)]
    gen = ref.crba(d[0])
    m.specialize_op("crba")
    m.specialize_rnea()
    assert not torch.equal(m.crba(d[0]), gen)
    ws = bard.Workspace(m, B)
    ws.set_policy(0)
    assert torch.equal(m.crba(d[0], ws=ws), gen)       # a workspace keeps the generic kernel
    m.specialize_op("crba", route=False)
    assert torch.equal(m.crba(d[0]), gen)
    assert not torch.equal(m.rnea(*d), ref.rnea(*d))  # the inverse-dynamics route stays


@pytest.mark.parametrize("form", ["split", "whole"])
@pytest.mark.parametrize("name,dtype,B", CASES)
def test_specialized_jacobian_matches_oracle(name, dtype, B, form):
    tree = synth.tree_by_name(name)
    ee = list(tree.ee_bodies) if len(tree.ee_bodies) else [tree.n_bodies - 1]
    frame = B % 2   # both frames over the cases
    say(f"[gpu] specialised jacobian {name} {dtype} B={B} form={form} frame={frame}")
    m = bard.Model.from_tree(tree)
    m.specialize_op("jacobian", dtype=dtype, form=form, ee=ee, frame=frame)
    assert m.specialized_op_info("jacobian", dtype=dtype, form=form, ee=ee, frame=frame)["routed"]
    om = oracle_for(tree)
    q, _, _ = inputs(tree, B, 6600, dtype)
    J = from_dev(m.jacobian(to_dev(q, dtype), ee, frame=frame))
    assert_jacobian("spec jacobian", J, om.jacobian(q, ee, frame=frame), dtype)


def test_specialized_jacobian_zero_rows_and_routing():
    import torch
    say("[gpu] specialised jacobian zero rows and routing")
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    ref = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    m.specialize_op("jacobian", ee=ee, frame=1)
    om = oracle_for(tree)
    for B in (4096, 4097):        # zero rows from extra workgroups, then from the lanes
        q, _, _ = inputs(tree, B, 6700 + B, "float32")
        out = torch.full((6 * tree.nv * len(ee), B), float("nan"), device="cuda")
        m.jacobian(to_dev(q, "float32"), ee, frame=1, out=out)
        torch.cuda.synchronize()
        assert not torch.isnan(out).any()
        idx = np.sort(np.random.default_rng(B).choice(B, 200, replace=False))
        assert_jacobian("zero rows", from_dev(out)[idx], om.jacobian(q[idx], ee, frame=1), "float32")
    q, _, _ = inputs(tree, 300, 6800, "float32")
    qd = to_dev(q, "float32")
    assert not torch.equal(m.jacobian(qd, ee, frame=1), ref.jacobian(qd, ee, frame=1))
    # another frame, another end-effector set or a workspace keep the generic kernel
    assert torch.equal(m.jacobian(qd, ee, frame=0), ref.jacobian(qd, ee, frame=0))
    assert torch.equal(m.jacobian(qd, ee[:2], frame=1), ref.jacobian(qd, ee[:2], frame=1))
    ws = bard.Workspace(m, 300)
    ws.set_policy(0)
    assert torch.equal(m.jacobian(qd, ee, frame=1, ws=ws), ref.jacobian(qd, ee, frame=1))
    m.specialize_op("jacobian", ee=ee, frame=1, route=False)
    assert torch.equal(m.jacobian(qd, ee, frame=1), ref.jacobian(qd, ee, frame=1))


@pytest.mark.parametrize("form", ["split", "whole"])
@pytest.mark.parametrize("name,dtype,B", CASES + [("free_branches61", "float32", 100)])
def test_specialized_fk_matches_oracle(name, dtype, B, form):
    say(f"[gpu] specialised fk {name} {dtype} B={B} form={form}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    m.specialize_op("fk", dtype=dtype, form=form)
    om = oracle_for(tree)
    q, _, _ = inputs(tree, B, 6900, dtype)
    poses = from_dev(m.fk(to_dev(q, dtype))).reshape(B, tree.n_bodies, 12)
    assert_normwise("spec fk", poses, fk_ref_blocks(om, q), dtype)


def test_specialized_fk_routing_and_batch_major():
    import torch
    say("[gpu] specialised fk routing, batch-major layout")
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    ref = bard.Model.from_tree(tree)
    m.specialize_op("fk")
    B = 513
    q, _, _ = inputs(tree, B, 7000, "float32")
    om = oracle_for(tree)
    qa = to_dev(q, "float32", layout="aos")
    out = m.fk(qa, layout="aos")
    assert_normwise("aos", from_dev(out, layout="aos").reshape(B, tree.n_bodies, 12), fk_ref_blocks(om, q), "float32")
    qs = to_dev(q, "float32")
    ws = bard.Workspace(m, B)
    ws.set_policy(0)
    assert torch.equal(m.fk(qs, ws=ws), ref.fk(qs))
    m.specialize_op("fk", route=False)
    assert torch.equal(m.fk(qs), ref.fk(qs))
