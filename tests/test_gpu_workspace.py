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
from parity_util import assert_normwise, fk_ref_blocks, from_dev, inputs, oracle_for, say, to_dev

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
