"""GPU tests of the workspace tiers (cached poses, motion subspaces and base
origin keyed by the q version tag; M; the bias forces; the binding's result
tier).

A kinematics-tier hit must give the same bits as a call that recomputes
everything, for every operator that uses the tier; a call whose tag matches
but whose q differs must return the cached state (which shows the tier was
used); tag 0, policy 0, a new batch size or an in-place change of q must
recompute.  The hit and miss counters follow the decisions."""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from oracle import OracleModel
from parity_util import (affine_rnea_ok, assert_jacobian, assert_mass, assert_normwise, assert_tau, entry_scales,
                         fk_ref_blocks, from_dev, inputs, oracle_for, say, to_dev)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,dtype,B", [("humanoid_large", "float32", 777), ("quadruped_spine", "float64", 130),
                                          ("random18", "float32", 2049), ("chain64", "float32", 65)])
def test_tier_hits_equal_cold_calls(name, dtype, B):
    """A cached result is bitwise equal to a cold recompute: every call of a
    miss/hit sequence on the kinematics tier (state stored by one operator,
    reused by the others) gives the same bits as the same operator called
    without a workspace, and those meet the per-entry contract.  The hit and
    miss counters follow the sequence."""
    import torch
    say(f"[gpu] workspace tier {name} {dtype} B={B}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    hq, hqd, hqdd = inputs(tree, B, 2700, dtype)
    q, qd, qdd = (to_dev(x, dtype) for x in (hq, hqd, hqdd))
    ee = tree.ee_bodies
    cold = {"fk": m.fk(q), "crba": m.crba(q), "rnea": m.rnea(q, qd, qdd), "jw": m.jacobian(q, ee),
            "jl": m.jacobian(q, ee, frame=bard.LOCAL_WORLD_ALIGNED)}
    torch.cuda.synchronize()
    st, sm = entry_scales(om, tree, hq, hqd, hqdd)
    assert_tau("cold rnea", from_dev(cold["rnea"]), om.rnea(hq, hqd, hqdd), st, dtype)
    assert_mass("cold crba", from_dev(cold["crba"]), om.crba(hq), sm, dtype)
    assert_jacobian("cold jw", from_dev(cold["jw"]), om.jacobian(hq, ee, frame=0), dtype)
    assert_jacobian("cold jl", from_dev(cold["jl"]), om.jacobian(hq, ee, frame=1), dtype)
    assert_normwise("cold fk", from_dev(cold["fk"]).reshape(B, tree.n_bodies, 12), fk_ref_blocks(om, hq), dtype)
    ws = bard.Workspace(m, B, dtype=getattr(torch, dtype))
    seq = [("fk", lambda: m.fk(q, ws=ws), False),                     # miss: stores poses
           ("fk", lambda: m.fk(q, ws=ws), True),                      # hit
           ("jw", lambda: m.jacobian(q, ee, ws=ws), False),           # miss (no s yet): stores s
           ("crba", lambda: m.crba(q, ws=ws), True),                  # hit: poses and s
           ("rnea", lambda: m.rnea(q, qd, qdd, ws=ws), True),         # hit: velocity sweep only
           ("jl", lambda: m.jacobian(q, ee, frame=bard.LOCAL_WORLD_ALIGNED, ws=ws), True),
           ("jw", lambda: m.jacobian(q, ee, ws=ws), True)]
    hits = misses = 0
    for key, call, hit in seq:
        out = call()
        torch.cuda.synchronize()
        assert torch.equal(out, cold[key]), f"{key} ({'hit' if hit else 'miss'}) differs from the cold call"
        hits, misses = hits + hit, misses + (not hit)
        s = ws.stats()["kinematics"]
        assert (s["hits"], s["misses"]) == (hits, misses), (key, s)


def test_result_tier_skips_unchanged_calls():
    """TIER_RESULTS: an unchanged call returns the previous output without a
    launch; an in-place change of an input or of the output recomputes."""
    import torch
    say("[gpu] workspace result tier")
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)
    hq, hqd, hqdd = inputs(tree, 300, 2750, "float32")
    q, qd, qdd = (to_dev(x, "float32") for x in (hq, hqd, hqdd))
    ws = bard.Workspace(m, 300, policy=bard.TIER_KINEMATICS | bard.TIER_RESULTS)
    t1 = m.rnea(q, qd, qdd, ws=ws)
    t2 = m.rnea(q, qd, qdd, ws=ws)
    assert t2 is t1 and ws.stats()["results"]["hits"] == 1
    qdd.mul_(2.0)                                  # input changed in place: recomputed
    t3 = m.rnea(q, qd, qdd, ws=ws)
    assert t3 is not t1
    torch.cuda.synchronize()
    assert torch.equal(t3, m.rnea(q, qd, qdd))
    t3.zero_()                                     # output changed in place: recomputed
    t4 = m.rnea(q, qd, qdd, ws=ws)
    assert t4 is not t3 and torch.equal(t4, m.rnea(q, qd, qdd))
    M1 = m.crba(q, ws=ws)
    assert m.crba(q, ws=ws) is M1
    J1 = m.jacobian(q, [3, 5], ws=ws)
    assert m.jacobian(q, [3, 5], ws=ws) is J1
    assert m.jacobian(q, [3, 6], ws=ws) is not J1     # other end effectors
    assert ws.stats()["results"]["hits"] == 3
    ws.set_policy(bard.TIER_KINEMATICS)            # off: every call launches
    assert m.crba(q, ws=ws) is not M1


def test_tier_is_used_and_invalidated():
    import torch
    say("[gpu] workspace tier use and invalidation")
    tree = synth.chain7()
    m = bard.Model.from_tree(tree)
    B = 300
    q1, _, _ = (to_dev(x, "float32") for x in inputs(tree, B, 2800, "float32"))
    q2, _, _ = (to_dev(x, "float32") for x in inputs(tree, B, 2801, "float32"))
    f1, f2 = m.fk(q1), m.fk(q2)
    ws = bard.Workspace(m, 4096)
    assert torch.equal(m.fk(q1, ws=ws, q_tag=11), f1)
    # same tag, different contents: the cached poses come back
    assert torch.equal(m.fk(q2, ws=ws, q_tag=11), f1)
    # tag 0 always recomputes; a new tag recomputes and replaces the tier
    assert torch.equal(m.fk(q2, ws=ws, q_tag=0), f2)
    assert torch.equal(m.fk(q2, ws=ws, q_tag=12), f2)
    assert torch.equal(m.fk(q1, ws=ws, q_tag=12), f2)
    # a different batch size is a miss
    assert torch.equal(m.fk(q1[:, :100].contiguous(), ws=ws, q_tag=12), f1[:, :100])
    # policy 0: the workspace is not used
    ws.set_policy(0)
    assert torch.equal(m.fk(q2, ws=ws, q_tag=11), f2)
    ws.set_policy(1)
    # automatic tags follow in-place changes of q
    qa = q1.clone()
    ws2 = bard.Workspace(m, B)
    assert torch.equal(m.fk(qa, ws=ws2), f1)
    qa.copy_(q2)
    assert torch.equal(m.fk(qa, ws=ws2), f2)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,dtype,B", [("humanoid_large", "float32", 777), ("quadruped_spine", "float64", 130),
                                          ("chain7", "float32", 4096)])
def test_mass_tier(name, dtype, B):
    """CRBA with the mass tier: the miss meets the contract and fills the
    tier, a hit returns the same bits (also into a batch-major output), and a
    hit whose q differs returns the cached matrix (the tier was used)."""
    import torch
    say(f"[gpu] mass tier {name} {dtype} B={B}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    hq, _, _ = inputs(tree, B, 3200, dtype)
    hq2, _, _ = inputs(tree, B, 3201, dtype)
    q, q2 = to_dev(hq, dtype), to_dev(hq2, dtype)
    ws = bard.Workspace(m, B, dtype=getattr(torch, dtype), policy=bard.TIER_KINEMATICS | bard.TIER_MASS)
    M1 = m.crba(q, ws=ws, q_tag=5)
    torch.cuda.synchronize()
    assert_mass("crba miss", from_dev(M1), om.crba(hq), entry_scales(om, tree, hq, tau=False)[1], dtype)
    assert torch.equal(m.crba(q, ws=ws, q_tag=5), M1)
    Ma = m.crba(to_dev(hq, dtype, "aos"), ws=ws, q_tag=5, layout="aos")
    assert torch.equal(Ma.t().contiguous(), M1)
    assert torch.equal(m.crba(q2, ws=ws, q_tag=5), M1)          # stale tag: cached M comes back
    M2 = m.crba(q2, ws=ws, q_tag=6)                              # new tag: recomputed
    torch.cuda.synchronize()
    assert_mass("crba new tag", from_dev(M2), om.crba(hq2), entry_scales(om, tree, hq2, tau=False)[1], dtype)
    hits, misses = ws.stats()["mass"]["hits"], ws.stats()["mass"]["misses"]
    assert (hits, misses) == (3, 2), ws.stats()
    ws.set_policy(bard.TIER_KINEMATICS)                         # mass tier off: no copy
    assert torch.equal(m.crba(q, ws=ws, q_tag=5), M1)


@pytest.mark.parametrize("name,dtype,B", [("humanoid_large", "float32", 777), ("quadruped_spine", "float64", 130),
                                          ("random18", "float32", 2049), ("chain64", "float32", 65)])
def test_bias_tier(name, dtype, B):
    """RNEA with the mass and bias tiers.  A miss computes tau (held to the
    contract) and b = RNEA(q, qd, 0) in one traversal; with M cached, a call
    on the same (q, qd) tags returns tau = M qdd + b, held to the affine bound
    (that of ABA's backward error).  A hit whose qd contents differ under the
    same tag evaluates with the cached b, which shows the tier was used; a
    new qd tag, an inertia override or a gravity change recompute."""
    import torch
    say(f"[gpu] bias tier {name} {dtype} B={B}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    hq, hqd, hqdd = inputs(tree, B, 3300, dtype)
    _, hqd2, hqdd2 = inputs(tree, B, 3301, dtype)
    q, qd, qdd, qd2, qdd2 = (to_dev(x, dtype) for x in (hq, hqd, hqdd, hqd2, hqdd2))

    def check(label, t, omx, x, xd, xdd):
        assert_tau(label, from_dev(t), omx.rnea(x, xd, xdd), entry_scales(omx, tree, x, xd, xdd, mass=False)[0], dtype)

    ws = bard.Workspace(m, B, dtype=getattr(torch, dtype), policy=7)
    m.crba(q, ws=ws, q_tag=1)
    t1 = m.rnea(q, qd, qdd, ws=ws, q_tag=1, qd_tag=1)        # miss: tau and b
    torch.cuda.synchronize()
    check("rnea miss", t1, om, hq, hqd, hqdd)
    t2 = m.rnea(q, qd, qdd2, ws=ws, q_tag=1, qd_tag=1)       # hit: M qdd + b
    torch.cuda.synchronize()
    ok, worst = affine_rnea_ok(om, hq, hqd, hqdd2, from_dev(t2), dtype)
    say(f"[gpu]   hit: worst error / bound {worst:.3g}")
    assert ok.all(), worst
    t3 = m.rnea(q, qd2, qdd2, ws=ws, q_tag=1, qd_tag=1)      # stale qd tag: cached b is used
    assert torch.equal(t3, t2) or tree.depth >= 32
    # the same hit into batch-major arrays: same arithmetic, same bits
    ta = m.rnea(to_dev(hq, dtype, "aos"), to_dev(hqd, dtype, "aos"), to_dev(hqdd2, dtype, "aos"), ws=ws, q_tag=1,
                qd_tag=1, layout="aos")
    assert torch.equal(ta.t().contiguous(), t2) or tree.depth >= 32
    t4 = m.rnea(q, qd2, qdd2, ws=ws, q_tag=1, qd_tag=2)      # new qd tag: recomputed
    torch.cuda.synchronize()
    check("rnea new qd", t4, om, hq, hqd2, hqdd2)
    t5 = m.rnea(q, qd2, qdd, ws=ws, q_tag=1, qd_tag=2)       # hit again with the new b
    torch.cuda.synchronize()
    ok, worst = affine_rnea_ok(om, hq, hqd2, hqdd, from_dev(t5), dtype)
    assert ok.all(), worst
    pi = torch.tensor(np.asarray(tree.inertia), dtype=getattr(torch, dtype), device="cuda").contiguous()
    t6 = m.rnea(q, qd2, qdd, inertia=pi, ws=ws, q_tag=1, qd_tag=2)   # override: never the tier
    torch.cuda.synchronize()
    check("rnea override", t6, om, hq, hqd2, hqdd)
    g = [0.3, -0.2, -3.7]
    m.set_gravity(g)
    om_g = OracleModel(tree.parent, tree.joint_type, tree.axis, tree.X_tree, tree.inertia, g)
    t7 = m.rnea(q, qd2, qdd, ws=ws, q_tag=1, qd_tag=2)       # gravity changed: b recomputed
    torch.cuda.synchronize()
    check("rnea new gravity", t7, om_g, hq, hqd2, hqdd)
