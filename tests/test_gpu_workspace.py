"""GPU tests of the workspace's kinematics tier (cached poses, motion
subspaces and base origin keyed by the q version tag).

A hit must give the same bits as a call that recomputes everything, for
every operator that uses the tier; a call whose tag matches but whose q
differs must return the cached state (which shows the tier was used); tag 0,
policy 0, a new batch size or an in-place change of q must recompute."""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from oracle import OracleModel
from parity_util import (affine_rnea_ok, assert_normwise, assert_normwise_scaled, fk_ref_blocks, from_dev, inputs,
                         oracle_for, say, term_scales, to_dev)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,dtype,B", [("humanoid_large", "float32", 777), ("quadruped_spine", "float64", 130),
                                          ("random18", "float32", 2049)])
def test_tier_hits_meet_the_contract(name, dtype, B):
    """Every call of a miss/hit sequence is checked against the oracle under
    the parity contract.  FK reloads exactly the values FK stored, so its hit
    is also bitwise equal to its miss; other operators reuse values another
    kernel instantiation stored, equal up to the compiler's contraction
    choices."""
    import torch
    say(f"[gpu] workspace tier {name} {dtype} B={B}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    hq, hqd, hqdd = inputs(tree, B, 2700, dtype)
    q, qd, qdd = (to_dev(x, dtype) for x in (hq, hqd, hqdd))
    ee = tree.ee_bodies
    ref = {"fk": fk_ref_blocks(om, hq), "crba": om.crba(hq).reshape(B, 1, -1), "rnea": om.rnea(hq, hqd, hqdd)[:, None],
           "jw": om.jacobian(hq, ee, frame=0).reshape(B, len(ee), -1),
           "jl": om.jacobian(hq, ee, frame=1).reshape(B, len(ee), -1)}
    shape = {"fk": (B, tree.n_bodies, 12), "crba": (B, 1, -1), "rnea": (B, 1, -1), "jw": (B, len(ee), -1),
             "jl": (B, len(ee), -1)}
    ws = bard.Workspace(m, B, dtype=getattr(torch, dtype))
    fk_miss = m.fk(q, ws=ws)                                   # miss: stores poses
    seq = [("fk", lambda: m.fk(q, ws=ws)),                     # hit
           ("jw", lambda: m.jacobian(q, ee, ws=ws)),           # miss (no s yet): stores s
           ("crba", lambda: m.crba(q, ws=ws)),                 # hit: poses and s
           ("rnea", lambda: m.rnea(q, qd, qdd, ws=ws)),        # hit: velocity sweep only
           ("jl", lambda: m.jacobian(q, ee, frame=bard.LOCAL_WORLD_ALIGNED, ws=ws)),  # hit
           ("jw", lambda: m.jacobian(q, ee, ws=ws))]           # hit
    for key, call in seq:
        out = call()
        torch.cuda.synchronize()
        if key == "fk":
            assert torch.equal(out, fk_miss)
        assert_normwise(f"ws {key}", from_dev(out).reshape(shape[key]), ref[key], dtype)


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
    assert_normwise("crba miss", from_dev(M1).reshape(B, 1, -1), om.crba(hq).reshape(B, 1, -1), dtype)
    assert torch.equal(m.crba(q, ws=ws, q_tag=5), M1)
    Ma = m.crba(to_dev(hq, dtype, "aos"), ws=ws, q_tag=5, layout="aos")
    assert torch.equal(Ma.t().contiguous(), M1)
    assert torch.equal(m.crba(q2, ws=ws, q_tag=5), M1)          # stale tag: cached M comes back
    M2 = m.crba(q2, ws=ws, q_tag=6)                              # new tag: recomputed
    torch.cuda.synchronize()
    assert_normwise("crba new tag", from_dev(M2).reshape(B, 1, -1), om.crba(hq2).reshape(B, 1, -1), dtype)
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
    edge = name in synth.EDGE_TREES

    def check(label, t, omx, x, xd, xdd):
        ref = omx.rnea(x, xd, xdd)[:, None]
        if edge:  # long chains: bound relative to the summed per-body terms
            assert_normwise_scaled(label, from_dev(t)[:, None], ref, term_scales(omx, tree, x, xd, xdd)[0], dtype)
        else:
            assert_normwise(label, from_dev(t)[:, None], ref, dtype)

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
