"""Model-specialised forward dynamics (bard_model_specialize_aba): the
hipRTC-compiled per-tree ABA kernel behind bard_aba, through the C ABI.

Parity: the routed aba call against the FP64 oracle under the backward-error
contract of the generic ABA tests (the torques the GPU's accelerations imply,
recomputed by the oracle's RNEA, against the given torques, scaled by
|tau| + |M| |qdd| + |bias|), FP32 and FP64, fixed and free roots, revolute
and prismatic joints, single-body trees, ragged batches (64 instances per
workgroup), the instance-major layout, a gravity change after compilation,
joint angles past 1e5 rad; in FP64 also element-wise against the oracle's
accelerations.  Routing: without BARD_SPEC_ROUTE the generic kernel keeps the
calls (bitwise its own results); autotuning routes batch tiers; trees deeper
than 16 are refused.
"""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from parity_util import aba_backward_error, from_dev, inputs, oracle_for, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [("chain7", "float32", 1000), ("chain7", "float64", 65), ("quadruped_spine", "float32", 513),
         ("random11", "float32", 300), ("random18", "float64", 97), ("humanoid_small", "float32", 777),
         ("humanoid_large", "float32", 1000), ("humanoid_large", "float64", 64), ("prismatic8", "float32", 129),
         ("star64", "float32", 70), ("rev1", "float32", 5), ("pri1", "float64", 3), ("free1", "float32", 65)]


def _tau(om, q, qd, qdd, dtype):
    tau = om.rnea(q, qd, qdd)
    return synth.to_fp32_grid(tau) if dtype == "float32" else tau


@pytest.mark.parametrize("name,dtype,B", CASES)
def test_specialized_aba_matches_oracle(name, dtype, B):
    say(f"[gpu] specialised aba {name} {dtype} B={B}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    m.specialize_aba(dtype=dtype)
    assert m.specialized_aba_info(dtype=dtype)["routed"]
    om = oracle_for(tree)
    q, qd, qdd = inputs(tree, B, 6300, dtype)
    tau = _tau(om, q, qd, qdd, dtype)
    out = from_dev(m.aba(to_dev(q, dtype), to_dev(qd, dtype), to_dev(tau, dtype)))
    ok, worst = aba_backward_error(om, q, qd, tau, out, dtype)
    assert ok.all(), f"backward error: {int((~ok).sum())} instances fail, worst {worst:.3g}"
    if dtype == "float64":
        ref = om.aba(q, qd, tau)
        np.testing.assert_allclose(out, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_routing_layout_gravity_and_large_angles():
    import torch
    say("[gpu] specialised aba: routing, aos layout, gravity change, large angles")
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    B = 300
    q, qd, qdd = inputs(tree, B, 6400, "float32")
    tau = _tau(om, q, qd, qdd, "float32")
    d = [to_dev(x, "float32") for x in (q, qd, tau)]
    generic = m.aba(*d)
    m.specialize_aba(route=False)
    kept = m.aba(*d)
    torch.cuda.synchronize()
    assert torch.equal(generic, kept)
    m.specialize_aba(route=True)
    out = m.aba(*[to_dev(x, "float32", "aos") for x in (q, qd, tau)], layout="aos")
    ok, worst = aba_backward_error(om, q, qd, tau, from_dev(out, "aos"), "float32")
    assert ok.all(), worst
    g = (0.5, -1.0, -9.5)
    m.set_gravity(g)
    from oracle import OracleModel
    om2 = OracleModel(tree.parent, tree.joint_type, tree.axis, tree.X_tree, tree.inertia, gravity=g)
    out = from_dev(m.aba(*d))
    ok, worst = aba_backward_error(om2, q, qd, tau, out, "float32")
    assert ok.all(), worst
    # revolute angles past 1e5 rad (the out-of-line sine and cosine)
    t7 = synth.chain7()
    m7 = bard.Model.from_tree(t7)
    m7.specialize_aba(dtype="float64")
    rng = np.random.default_rng(13)
    qb = rng.uniform(-1.0, 1.0, size=(96, 7)) * np.array([1e6, 3e5, 2e5, np.pi, -np.pi, 1e5, 7e5])
    qdb, taub = rng.standard_normal((96, 7)), rng.standard_normal((96, 7))
    om7 = oracle_for(t7)
    outb = from_dev(m7.aba(to_dev(qb, "float64"), to_dev(qdb, "float64"), to_dev(taub, "float64")))
    np.testing.assert_allclose(outb, om7.aba(qb, qdb, taub), rtol=1e-8, atol=1e-8)


def test_autotune_and_deep_tree_refused():
    import torch
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    mb = m.autotune_aba()
    tiers = m.specialized_aba_info()["route_tiers"]
    say(f"[gpu] autotuned aba on humanoid_large: first specialised batch {mb}, tiers {tiers:04b}")
    assert mb in (-1,) + bard.SPEC_TIERS
    om = oracle_for(tree)
    ref = bard.Model.from_tree(tree)
    for B, tier in ((300, 0), (20000, 2)):
        q, qd, qdd = inputs(tree, B, 6500 + B, "float32")
        tau = _tau(om, q, qd, qdd, "float32")
        d = [to_dev(x, "float32") for x in (q, qd, tau)]
        out, gen = m.aba(*d), ref.aba(*d)
        torch.cuda.synchronize()
        if not (tiers >> tier) & 1:
            assert torch.equal(out, gen)
        idx = np.sort(np.random.default_rng(B).choice(B, min(B, 200), replace=False))
        ok, worst = aba_backward_error(om, q[idx], qd[idx], tau[idx], from_dev(out)[idx], "float32")
        assert ok.all(), worst
    deep = bard.Model.from_tree(synth.tree_by_name("chain64"))
    with pytest.raises(bard.BardError) as ei:
        deep.specialize_aba()
    assert ei.value.status == -7


@pytest.mark.parametrize("name", ["star64", "free_branches61"])
def test_fp64_trees_past_the_generic_capacity(name):
    """The generic FP64 forward-dynamics kernel refuses trees of 60 or more
    bodies (BARD_E_CAPACITY); the routed specialised kernel serves them."""
    say(f"[gpu] specialised FP64 aba on {name}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    B = 130
    q, qd, qdd = inputs(tree, B, 6600, "float64")
    tau = om.rnea(q, qd, qdd)
    d = [to_dev(x, "float64") for x in (q, qd, tau)]
    with pytest.raises(bard.BardError) as ei:
        m.aba(*d)
    assert ei.value.status == -6  # BARD_E_CAPACITY
    m.specialize_aba(dtype="float64")
    out = from_dev(m.aba(*d))
    ok, worst = aba_backward_error(om, q, qd, tau, out, "float64")
    assert ok.all(), worst
    np.testing.assert_allclose(out, om.aba(q, qd, tau), rtol=1e-8, atol=1e-8 * np.abs(out).max())
