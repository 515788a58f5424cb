"""GPU parity of the reverse-mode products (FK and RNEA adjoints) against the
oracle's tape reverse-mode AD.

Calls go through the C ABI.  Inputs and cotangents are seeded and rounded to
the kernel's precision; the oracle runs in FP64 on those values.  The RNEA adjoint's
per-instance gradients (q_bar, qd_bar, qdd_bar) and the FK adjoint's are held
normwise per instance (parity_util).  The inertial-parameter
gradient is a batch sum, so its bound is the per-instance bound summed over
the batch (triangle inequality): for every body,
``max_k |gpu_k - sum_b ref_bk| <= sum_b (atol + rtol * max_k |ref_bk|)``.
"""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from parity_util import TOL, assert_normwise, from_dev, inputs, oracle_for, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ("chain7", "float64", 64),
    ("chain7", "float32", 1000),
    ("quadruped_spine", "float32", 513),
    ("quadruped_spine", "float64", 97),
    ("random7", "float32", 300),
    ("random11", "float32", 300),
    ("random12", "float32", 300),
    ("random18", "float32", 300),
    ("random23", "float32", 300),
    ("random23", "float64", 40),
    # free root (quaternion coordinates)
    ("humanoid_small", "float32", 300),
    ("humanoid_small", "float64", 40),
    ("humanoid_large", "float32", 257),
]


def cotangent(shape, seed, dtype):
    x = np.random.default_rng(seed).standard_normal(shape)
    return synth.to_fp32_grid(x) if dtype == "float32" else x


def assert_param_grad(gpu, ref_per_instance, dtype):
    """gpu [n, 10]; ref_per_instance [B, n, 10]."""
    rtol, atol = TOL[dtype]
    ref = ref_per_instance.sum(axis=0)
    bound = (atol + rtol * np.abs(ref_per_instance).max(axis=2)).sum(axis=0)
    err = np.abs(gpu - ref).max(axis=1)
    worst = float((err / bound).max())
    assert (err <= bound).all(), f"inertia_bar: worst err/bound = {worst:.3g}"
    return worst


def _setup(name, dtype, B, seed=2100):
    tree = synth.tree_by_name(name)
    return tree, bard.Model.from_tree(tree), oracle_for(tree), inputs(tree, B, seed, dtype)


@pytest.mark.parametrize("name,dtype,B", CASES)
def test_rnea_vjp(name, dtype, B):
    say(f"[gpu] rnea_vjp {name} {dtype} B={B}")
    tree, m, om, (q, qd, qdd) = _setup(name, dtype, B)
    tb = cotangent((B, tree.nv), 7, dtype)
    qb, qdb, qddb, pib = m.rnea_vjp(to_dev(q, dtype), to_dev(qd, dtype), to_dev(qdd, dtype), to_dev(tb, dtype))
    rq, rqd, rqdd, rpi = om.rnea_vjp(q, qd, qdd, tb)
    assert_normwise("q_bar", from_dev(qb)[:, None], rq[:, None], dtype)
    assert_normwise("qd_bar", from_dev(qdb)[:, None], rqd[:, None], dtype)
    assert_normwise("qdd_bar", from_dev(qddb)[:, None], rqdd[:, None], dtype)
    assert_param_grad(pib.cpu().double().numpy(), rpi, dtype)


@pytest.mark.parametrize("name,dtype,B", CASES)
def test_fk_vjp(name, dtype, B):
    say(f"[gpu] fk_vjp {name} {dtype} B={B}")
    tree, m, om, (q, _, _) = _setup(name, dtype, B)
    pb = cotangent((B, tree.n_bodies * 12), 8, dtype)
    qb = m.fk_vjp(to_dev(q, dtype), to_dev(pb, dtype))
    ref = om.fk_vjp(q, pb.reshape(B, tree.n_bodies, 3, 4))
    assert_normwise("q_bar", from_dev(qb)[:, None], ref[:, None], dtype)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_rnea_vjp_inertia_override(dtype):
    """Gradients at perturbed parameters (masses scaled, as in identification)."""
    say(f"[gpu] rnea_vjp inertia override {dtype}")
    import torch
    tree, m, om, (q, qd, qdd) = _setup("quadruped_spine", dtype, 200)
    pi = tree.inertia.copy()
    pi *= np.random.default_rng(3).uniform(0.7, 1.3, size=(tree.n_bodies, 1))
    if dtype == "float32":
        pi = synth.to_fp32_grid(pi)
    tb = cotangent((200, tree.nv), 9, dtype)
    pid = torch.from_numpy(pi).to(getattr(torch, dtype)).cuda()
    qb, qdb, qddb, pib = m.rnea_vjp(to_dev(q, dtype), to_dev(qd, dtype), to_dev(qdd, dtype), to_dev(tb, dtype),
                                    inertia=pid)
    rq, rqd, rqdd, rpi = om.rnea_vjp(q, qd, qdd, tb, inertia=pi)
    assert_normwise("q_bar", from_dev(qb)[:, None], rq[:, None], dtype)
    assert_normwise("qd_bar", from_dev(qdb)[:, None], rqd[:, None], dtype)
    assert_param_grad(pib.cpu().double().numpy(), rpi, dtype)


def test_adjoints_aos_layout():
    say("[gpu] adjoints aos layout")
    dtype = "float32"
    tree, m, om, (q, qd, qdd) = _setup("random12", dtype, 333)
    tb = cotangent((333, tree.nv), 10, dtype)
    pb = cotangent((333, tree.n_bodies * 12), 11, dtype)
    d = [to_dev(x, dtype, "aos") for x in (q, qd, qdd, tb)]
    qb, qdb, qddb, pib = m.rnea_vjp(*d, layout="aos")
    rq, rqd, rqdd, rpi = om.rnea_vjp(q, qd, qdd, tb)
    assert_normwise("q_bar", from_dev(qb, "aos")[:, None], rq[:, None], dtype)
    assert_normwise("qdd_bar", from_dev(qddb, "aos")[:, None], rqdd[:, None], dtype)
    assert_param_grad(pib.cpu().double().numpy(), rpi, dtype)
    fq = m.fk_vjp(d[0], to_dev(pb, dtype, "aos"), layout="aos")
    assert_normwise("fk q_bar", from_dev(fq, "aos")[:, None],
                    om.fk_vjp(q, pb.reshape(333, -1, 3, 4))[:, None], dtype)


def test_adjoints_tiny_batches_and_determinism():
    say("[gpu] adjoints B=1, B=0, determinism")
    import torch
    dtype = "float32"
    tree, m, om, (q, qd, qdd) = _setup("quadruped_spine", dtype, 1)
    tb = cotangent((1, tree.nv), 12, dtype)
    out = m.rnea_vjp(to_dev(q, dtype), to_dev(qd, dtype), to_dev(qdd, dtype), to_dev(tb, dtype))
    rq, rqd, rqdd, rpi = om.rnea_vjp(q, qd, qdd, tb)
    assert_normwise("q_bar B=1", from_dev(out[0])[:, None], rq[:, None], dtype)
    assert_param_grad(out[3].cpu().double().numpy(), rpi, dtype)
    e = torch.empty((tree.nv, 0), dtype=torch.float32, device="cuda")
    z = m.rnea_vjp(e, e, e, e)
    assert z[0].shape == (tree.nq, 0)
    # identical bits run to run (fixed-order batch reduction)
    tree, m, om, (q, qd, qdd) = _setup("random18", dtype, 20000, seed=5)
    tb = cotangent((20000, tree.nv), 13, dtype)
    d = [to_dev(x, dtype) for x in (q, qd, qdd, tb)]
    a = m.rnea_vjp(*d)
    b = m.rnea_vjp(*d)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_rnea_vjp_identification_workload_sampled():
    """The identification workload at its full size: the 11-DOF quadruped
    with a 3-body spine, 4096 sinusoid trajectories x 200 steps = 819,200
    instances, FP32.  tau_bar is non-zero on a sampled subset only, so the
    batch-summed inertia gradient has an exact oracle over that subset; the
    other instances must return exactly zero gradients."""
    import torch
    say("[gpu] rnea_vjp identification workload 819200 (sampled)")
    tree = synth.quadruped_spine()
    m = bard.Model.from_tree(tree)
    om = oracle_for(tree)
    q, qd, qdd = (synth.to_fp32_grid(x) for x in synth.sinusoid_trajectories(tree, 4096, 200, seed=4242))
    B = q.shape[0]
    idx = np.sort(np.random.default_rng(1).choice(B, 512, replace=False))
    tb = np.zeros((B, tree.nv))
    tb[idx] = cotangent((512, tree.nv), 14, "float32")
    qb, qdb, qddb, pib = m.rnea_vjp(to_dev(q, "float32"), to_dev(qd, "float32"), to_dev(qdd, "float32"),
                                    to_dev(tb, "float32"))
    torch.cuda.synchronize()
    rq, rqd, rqdd, rpi = om.rnea_vjp(q[idx], qd[idx], qdd[idx], tb[idx])
    g = [from_dev(x) for x in (qb, qdb, qddb)]
    assert_normwise("q_bar", g[0][idx][:, None], rq[:, None], "float32")
    assert_normwise("qd_bar", g[1][idx][:, None], rqd[:, None], "float32")
    assert_normwise("qdd_bar", g[2][idx][:, None], rqdd[:, None], "float32")
    mask = np.ones(B, bool)
    mask[idx] = False
    for x in g:
        assert not x[mask].any()
    assert_param_grad(pib.cpu().double().numpy(), rpi, "float32")


def test_autograd_functions():
    """torch.autograd through bard.rnea and bard.fk returns the adjoints."""
    import torch
    say("[gpu] autograd rnea / fk")
    dtype = "float64"
    tree, m, om, (q, qd, qdd) = _setup("random11", dtype, 50)
    pi = torch.from_numpy(tree.inertia.copy()).cuda().requires_grad_(True)
    tq, tqd, tqdd = (to_dev(x, dtype).requires_grad_(True) for x in (q, qd, qdd))
    w = cotangent((50, tree.nv), 15, dtype)
    tau = bard.rnea(m, tq, tqd, tqdd, pi)
    (tau * to_dev(w, dtype)).sum().backward()
    rq, rqd, rqdd, rpi = om.rnea_vjp(q, qd, qdd, w)
    assert_normwise("q.grad", from_dev(tq.grad)[:, None], rq[:, None], dtype)
    assert_normwise("qd.grad", from_dev(tqd.grad)[:, None], rqd[:, None], dtype)
    assert_normwise("qdd.grad", from_dev(tqdd.grad)[:, None], rqdd[:, None], dtype)
    assert_param_grad(pi.grad.cpu().numpy(), rpi, dtype)
    tq2 = to_dev(q, dtype).requires_grad_(True)
    poses = bard.fk(m, tq2)
    wp = cotangent((50, tree.n_bodies * 12), 16, dtype)
    (poses * to_dev(wp, dtype)).sum().backward()
    ref = om.fk_vjp(q, wp.reshape(50, -1, 3, 4))
    assert_normwise("fk q.grad", from_dev(tq2.grad)[:, None], ref[:, None], dtype)


def _sampled_adjoint_case(name, dtype, B, n_sample, seed):
    tree = synth.tree_by_name(name)
    m, om = bard.Model.from_tree(tree), oracle_for(tree)
    q, qd, qdd = inputs(tree, B, seed, dtype)
    idx = np.sort(np.random.default_rng(seed + 1).choice(B, n_sample, replace=False))
    return tree, m, om, q, qd, qdd, idx


@pytest.mark.parametrize("name,dtype,B", [("humanoid_large", "float32", 262144), ("humanoid_small", "float64", 40000),
                                          ("quadruped_spine", "float64", 65536)])
def test_adjoints_loop_over_more_tiles_than_resident_workgroups(name, dtype, B):
    """The adjoint kernels run one workgroup per resident slot and loop over
    tiles, loading the next tile while working on the current one.  At these
    batches every workgroup runs many tiles (free root in FP32 and FP64, fixed
    base in FP64).  Cotangents are non-zero on a sampled subset, so the oracle
    checks those instances one by one, the batch-summed parameter gradient
    exactly, and every other instance must return exact zeros."""
    import torch
    say(f"[gpu] adjoint tile loop {name} {dtype} B={B}")
    tree, m, om, q, qd, qdd, idx = _sampled_adjoint_case(name, dtype, B, 256, 2150)
    tb = np.zeros((B, tree.nv))
    tb[idx] = cotangent((len(idx), tree.nv), 17, dtype)
    d = [to_dev(x, dtype) for x in (q, qd, qdd)]
    qb, qdb, qddb, pib = m.rnea_vjp(*d, to_dev(tb, dtype))
    pb = np.zeros((B, tree.n_bodies * 12))
    pb[idx] = cotangent((len(idx), tree.n_bodies * 12), 18, dtype)
    fq = m.fk_vjp(d[0], to_dev(pb, dtype))
    torch.cuda.synchronize()
    rq, rqd, rqdd, rpi = om.rnea_vjp(q[idx], qd[idx], qdd[idx], tb[idx])
    g = [from_dev(x) for x in (qb, qdb, qddb)]
    for lbl, gg, rr in zip(("q_bar", "qd_bar", "qdd_bar"), g, (rq, rqd, rqdd)):
        assert_normwise(lbl, gg[idx][:, None], rr[:, None], dtype)
    assert_param_grad(pib.cpu().double().numpy(), rpi, dtype)
    fg = from_dev(fq)
    assert_normwise("fk q_bar", fg[idx][:, None], om.fk_vjp(q[idx], pb[idx].reshape(len(idx), -1, 3, 4))[:, None],
                    dtype)
    mask = np.ones(B, bool)
    mask[idx] = False
    for x in g + [fg]:
        assert not x[mask].any()
