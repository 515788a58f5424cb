"""GPU reverse-mode product of CRBA (bard_crba_vjp): q_bar = d<M_bar, M(q)>/dq.

FP64 runs are checked against the oracle's tape reverse-mode AD of its CRBA
(itself pinned to central differences on the CPU) at rtol = atol = 1e-12,
normwise per instance; FP32 runs at rtol 1e-5 / atol 1e-6, normwise per
instance, the contract of every reverse-mode product.  Sizes span
several tiles and a ragged tail; the 36-DOF humanoid runs at the benchmark's
batch with sampled checks.
"""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from parity_util import TOL, assert_normwise, from_dev, inputs, oracle_for, say, to_dev

pytestmark = pytest.mark.gpu


def cot(tree, B, seed, dtype):
    x = np.random.default_rng(seed).standard_normal((B, tree.nv * tree.nv))
    return synth.to_fp32_grid(x) if dtype == "float32" else x


CASES = [("chain7", "float64", 64), ("quadruped_spine", "float64", 97), ("random23", "float64", 40),
         ("humanoid_small", "float64", 37), ("prismatic8", "float64", 20),
         ("chain7", "float32", 1000), ("quadruped_spine", "float32", 513), ("random18", "float32", 300),
         ("humanoid_small", "float32", 300), ("humanoid_large", "float32", 257)]


@pytest.mark.parametrize("name,dtype,B", CASES)
def test_crba_vjp(name, dtype, B):
    say(f"[gpu] crba_vjp {name} {dtype} B={B}")
    tree = synth.tree_by_name(name)
    m, om = bard.Model.from_tree(tree), oracle_for(tree)
    q, _, _ = inputs(tree, B, 2900, dtype)
    mb = cot(tree, B, 2901, dtype)
    g = from_dev(m.crba_vjp(to_dev(q, dtype), to_dev(mb, dtype)))
    ref, _ = om.crba_vjp(q, mb)
    assert_normwise("q_bar", g[:, None], ref[:, None], dtype)
    if tree.joint_type[0] == synth.FREE:
        assert not g[:, :7].any(), "a free root's coordinates get exact zeros"


def test_crba_vjp_full_batch_sampled_and_deterministic():
    import torch
    say("[gpu] crba_vjp humanoid_large float32 B=4096 (sampled), determinism")
    tree = synth.humanoid_large()
    m, om = bard.Model.from_tree(tree), oracle_for(tree)
    B = 4096
    q, _, _ = inputs(tree, B, 2902, "float32")
    mb = cot(tree, B, 2903, "float32")
    tq, tmb = to_dev(q, "float32"), to_dev(mb, "float32")
    a = m.crba_vjp(tq, tmb)
    b = m.crba_vjp(tq, tmb)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    idx = np.sort(np.random.default_rng(3).choice(B, 256, replace=False))
    ref, _ = om.crba_vjp(q[idx], mb[idx])
    assert_normwise("q_bar", from_dev(a)[idx][:, None], ref[:, None], "float32")


def test_crba_vjp_aos_layout_and_autograd():
    import torch
    say("[gpu] crba_vjp aos layout, autograd")
    tree = synth.tree_by_name("random12")
    m, om = bard.Model.from_tree(tree), oracle_for(tree)
    B = 77
    q, _, _ = inputs(tree, B, 2904, "float64")
    mb = cot(tree, B, 2905, "float64")
    g = from_dev(m.crba_vjp(to_dev(q, "float64", "aos"), to_dev(mb, "float64", "aos"), layout="aos"), "aos")
    ref, _ = om.crba_vjp(q, mb)
    assert_normwise("q_bar aos", g[:, None], ref[:, None], "float64")
    tq = to_dev(q, "float64").requires_grad_(True)
    M = bard.crba(m, tq)
    (M * to_dev(mb, "float64")).sum().backward()
    assert_normwise("q.grad", from_dev(tq.grad)[:, None], ref[:, None], "float64")
