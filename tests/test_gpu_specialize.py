"""Model-specialised chain kernels (bard_model_specialize): hipRTC-compiled
per-tree code behind bard_chain, through the C ABI.

Parity: the routed chain call against the FP64 oracle under the per-entry
contract (parity_util), the three forms (split over waves by limbs, dual:
split with the torques and the mass matrix + Jacobians in two workgroups, and
whole),
FP32 and FP64, both Jacobian frames, fixed and free roots, revolute and
prismatic joints, single-body trees, batches with a ragged tail (64 instances
per workgroup), the instance-major layout, a gravity change after
compilation, joint angles past 1e5 rad, structural zeros written by extra
workgroups and by the lanes, and the headline tree at the benchmark's batches
(sampled).  Routing: without BARD_SPEC_ROUTE the generic kernel keeps the
calls (bitwise its own results); routing one form takes the calls from the
other; autotuning routes batch tiers; trees past the size bound are refused
with BARD_E_UNSUPPORTED.
"""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from parity_util import assert_chain, from_dev, inputs, oracle_for, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [("chain7", "float32", 1000, 0), ("chain7", "float64", 65, 1), ("quadruped_spine", "float32", 513, 1),
         ("random11", "float32", 300, 0), ("random18", "float64", 97, 0), ("random23", "float32", 300, 1),
         ("humanoid_small", "float32", 777, 0), ("humanoid_small", "float64", 40, 1),
         ("humanoid_large", "float32", 1000, 1), ("humanoid_large", "float64", 64, 0),
         ("prismatic8", "float32", 129, 0), ("star64", "float32", 70, 1), ("free_branches61", "float32", 100, 0),
         ("rev1", "float32", 5, 1), ("pri1", "float64", 3, 0), ("free1", "float32", 65, 1)]


TRIPLE_CASES = [("chain7", "float32", 1000, 0), ("quadruped_spine", "float32", 513, 1), ("random23", "float32", 300, 1),
                ("humanoid_small", "float64", 40, 1), ("humanoid_large", "float32", 1000, 1),
                ("humanoid_large", "float64", 64, 0), ("star64", "float32", 70, 1), ("free1", "float32", 65, 1)]


@pytest.mark.parametrize("name,dtype,B,frame,form", [c + (f,) for f in ("split", "whole", "dual") for c in CASES] +
                         [c + ("triple",) for c in TRIPLE_CASES])
def test_specialized_chain_matches_oracle(name, dtype, B, frame, form):
    say(f"[gpu] specialised chain {name} {dtype} B={B} frame={frame} form={form}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    m.specialize(ee, frame=frame, dtype=dtype, form=form)
    assert m.specialized_info(ee, frame=frame, dtype=dtype, form=form)["routed"]
    q, qd, qdd = inputs(tree, B, 5300, dtype)
    tau, M, J = m.chain(to_dev(q, dtype), to_dev(qd, dtype), to_dev(qdd, dtype), ee, frame=frame)
    assert_chain(oracle_for(tree), tree, q, qd, qdd, ee, from_dev(tau), from_dev(M), from_dev(J), dtype,
                 frame=frame, label=f"spec {name}")
    Mh = from_dev(M).reshape(B, tree.nv, tree.nv)
    assert (Mh == np.transpose(Mh, (0, 2, 1))).all(), "M is bitwise symmetric"


def test_routing_and_generic_results():
    import torch
    say("[gpu] specialised chain routing")
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    q, qd, qdd = inputs(tree, 300, 5400, "float32")
    d = [to_dev(x, "float32") for x in (q, qd, qdd)]
    generic = m.chain(*d, ee)
    m.specialize(ee, route=False)
    info = m.specialized_info(ee)
    assert not info["routed"] and info["scratch_bytes"] == 0 and info["vgprs"] > 0
    kept = m.chain(*d, ee)
    m.specialize(ee, route=True)
    spec = m.chain(*d, ee)
    m.specialize(ee, route=False)
    back = m.chain(*d, ee)
    # routing one form takes every batch from the other
    m.specialize(ee, route=True)
    m.specialize(ee, route=True, form="whole")
    assert not m.specialized_info(ee)["routed"]
    assert m.specialized_info(ee, form="whole")["route_tiers"] == 15
    whole = m.chain(*d, ee)
    torch.cuda.synchronize()
    assert_chain(oracle_for(tree), tree, q, qd, qdd, ee, *(from_dev(x) for x in whole), "float32", label="whole")
    m.specialize(ee, route=False, form="whole")
    for a, b in zip(generic, kept):
        assert torch.equal(a, b)
    for a, b in zip(generic, back):
        assert torch.equal(a, b)
    assert_chain(oracle_for(tree), tree, q, qd, qdd, ee, *(from_dev(x) for x in spec), "float32", label="routed")
    # another end-effector set or frame is not routed
    other = m.chain(*d, ee[:2])
    torch.cuda.synchronize()
    assert_chain(oracle_for(tree), tree, q, qd, qdd, ee[:2], *(from_dev(x) for x in other), "float32",
                 label="other set")


def test_instance_major_layout_and_gravity_change():
    say("[gpu] specialised chain aos layout, gravity change")
    from oracle import OracleModel
    tree = synth.quadruped_spine()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    m.specialize(ee)
    q, qd, qdd = inputs(tree, 333, 5500, "float32")
    d = [to_dev(x, "float32", "aos") for x in (q, qd, qdd)]
    out = m.chain(*d, ee, layout="aos")
    assert_chain(oracle_for(tree), tree, q, qd, qdd, ee, *(from_dev(x, "aos") for x in out), "float32",
                 label="aos")
    g = (1.0, -2.0, -9.0)
    m.set_gravity(g)
    out = m.chain(*[to_dev(x, "float32") for x in (q, qd, qdd)], ee)
    om = OracleModel(tree.parent, tree.joint_type, tree.axis, tree.X_tree, tree.inertia, gravity=g)
    assert_chain(om, tree, q, qd, qdd, ee, *(from_dev(x) for x in out), "float32", label="new gravity")


@pytest.mark.parametrize("B", [4096, 16384])
def test_headline_tree_at_benchmark_batches(B):
    say(f"[gpu] specialised chain humanoid_large B={B} (sampled)")
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    m.specialize(ee)
    q, qd, qdd = inputs(tree, B, 5600 + B, "float32")
    tau, M, J = m.chain(to_dev(q, "float32"), to_dev(qd, "float32"), to_dev(qdd, "float32"), ee)
    idx = np.sort(np.random.default_rng(B).choice(B, 256, replace=False))
    idx[-1] = B - 1
    assert_chain(oracle_for(tree), tree, q[idx], qd[idx], qdd[idx], ee, from_dev(tau)[idx], from_dev(M)[idx],
                 from_dev(J)[idx], "float32", label=f"spec B={B}")


def test_deep_tree_refused():
    say("[gpu] specialised chain refuses chain64")
    tree = synth.tree_by_name("chain64")
    m = bard.Model.from_tree(tree)
    with pytest.raises(bard.BardError) as ei:
        m.specialize(tree.ee_bodies)
    assert ei.value.status == -7


def test_autotune_routes_by_batch():
    """bard_chain_autotune times the generic kernel and both specialised forms
    and routes each batch tier to the fastest; a tier no form takes runs the
    generic kernel (bitwise its own result), and every call meets the
    contract either way."""
    import torch
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    ref = bard.Model.from_tree(tree)   # never specialised: the generic kernel
    mb = m.autotune_chain(ee)
    tiers = {f: m.specialized_info(ee, form=f)["route_tiers"] for f in bard.SPEC_FORMS}
    say(f"[gpu] autotuned chain on humanoid_small: first specialised batch {mb}, tiers " +
        ", ".join(f"{f} {t:04b}" for f, t in tiers.items()))
    assert mb in (-1,) + bard.SPEC_TIERS
    routed = 0
    for t in tiers.values():
        routed |= t
    assert sum(bin(t).count("1") for t in tiers.values()) == bin(routed).count("1")
    for B, tier in ((300, 0), (20000, 2)):
        q, qd, qdd = inputs(tree, B, 5700 + B, "float32")
        d = [to_dev(x, "float32") for x in (q, qd, qdd)]
        out = m.chain(*d, ee)
        gen = ref.chain(*d, ee)
        torch.cuda.synchronize()
        if not (routed >> tier) & 1:
            for a, b in zip(out, gen):
                assert torch.equal(a, b)
        idx = np.sort(np.random.default_rng(B).choice(B, min(B, 200), replace=False))
        assert_chain(oracle_for(tree), tree, q[idx], qd[idx], qdd[idx], ee, *(from_dev(x)[idx] for x in out),
                     "float32", label=f"autotuned B={B}")


@pytest.mark.parametrize("form", ["split", "dual", "triple"])
@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_zero_rows_from_extra_workgroups_and_from_lanes(dtype, form):
    """With instance-minor outputs, a batch that is a multiple of the 16-byte
    vector width and a grid that leaves wave slots free, the structural zeros
    of M and J come from extra workgroups; a ragged batch (B + 1) makes every
    lane write its own.  Outputs start as NaN, so an unwritten zero shows; the
    first B instances agree bitwise between the two calls."""
    import torch
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    m.specialize(ee, dtype=dtype, form=form)
    B = 4096
    q, qd, qdd = inputs(tree, B + 1, 5800, dtype)
    res = []
    for n in (B, B + 1):
        say(f"[gpu] specialised zero rows humanoid_large {dtype} {form} B={n}")
        d = [to_dev(x[:n], dtype) for x in (q, qd, qdd)]
        nan = float("nan")
        out = tuple(torch.full((k, n), nan, dtype=getattr(torch, dtype), device="cuda")
                    for k in (tree.nv, tree.nv * tree.nv, 6 * tree.nv * len(ee)))
        m.chain(*d, ee, out=out)
        torch.cuda.synchronize()
        for t in out:
            assert not torch.isnan(t).any()
        res.append(out)
    for a, b in zip(*res):
        assert torch.equal(a, b[:, :B])
    idx = np.sort(np.random.default_rng(3).choice(B + 1, 200, replace=False))
    idx[-1] = B
    assert_chain(oracle_for(tree), tree, q[idx], qd[idx], qdd[idx], ee, *(from_dev(x)[idx] for x in res[1]), dtype,
                 label="ragged")


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_large_joint_angles(dtype):
    """Angles beyond 1e5 rad take the out-of-line library sine and cosine in
    the generated code too."""
    say(f"[gpu] specialised chain, large joint angles {dtype}")
    tree = synth.chain7()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    m.specialize(ee, dtype=dtype)
    B = 96
    rng = np.random.default_rng(12)
    q = rng.uniform(-1.0, 1.0, size=(B, 7)) * np.array([1e6, 3e5, 2e5, np.pi, -np.pi, 1e5, 7e5])
    qd, qdd = rng.standard_normal((B, 7)), rng.standard_normal((B, 7))
    if dtype == "float32":
        q, qd, qdd = (synth.to_fp32_grid(x) for x in (q, qd, qdd))
    out = m.chain(*(to_dev(x, dtype) for x in (q, qd, qdd)), ee)
    assert_chain(oracle_for(tree), tree, q, qd, qdd, ee, *(from_dev(x) for x in out), dtype, label="large angles")


@pytest.mark.parametrize("name", ["star64", "free_branches61"])
def test_fp64_trees_past_the_generic_capacity(name):
    """The generic FP64 chain kernel refuses trees of 60 or more bodies
    (BARD_E_CAPACITY: its per-tile LDS); a routed specialised kernel keeps no
    per-tree state in LDS beyond the limb hand-over and serves them."""
    say(f"[gpu] specialised FP64 chain on {name}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    B = 130
    q, qd, qdd = inputs(tree, B, 5900, "float64")
    d = [to_dev(x, "float64") for x in (q, qd, qdd)]
    with pytest.raises(bard.BardError) as ei:
        m.chain(*d, ee)
    assert ei.value.status == -6  # BARD_E_CAPACITY
    m.specialize(ee, dtype="float64")
    out = m.chain(*d, ee)
    assert_chain(oracle_for(tree), tree, q, qd, qdd, ee, *(from_dev(x) for x in out), "float64", label=name)
