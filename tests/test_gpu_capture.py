"""Graph capture through the C ABI.

* A model's first call inside a graph capture would allocate its device
  tables: it returns BARD_E_CAPTURE and launches nothing, so the capture stays
  valid.
* After bard_model_upload the same calls (chain, RNEA adjoint with the
  parameter gradient) are captured and replayed; every replay, with new inputs
  and eager work between replays, matches an eager call bitwise.
* A plan that has run once is captured by the caller's graph and replays
  bitwise equal to its eager run.
"""

import numpy as np
import pytest
import torch

import synth
from paper_2605_31481_amd import bard
from parity_util import inputs, say, to_dev

pytestmark = pytest.mark.gpu


def test_first_call_under_capture_is_refused():
    say("[gpu] capture: first call of a fresh model inside a capture")
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)          # never used on the device
    q, qd, qdd = (to_dev(x, "float32") for x in inputs(tree, 64, 2700, "float32"))
    M = torch.empty((tree.nv * tree.nv, 64), device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(bard.BardError) as e:
        with torch.cuda.graph(g):
            m.crba(q, out=M)
    assert e.value.status == bard.E_CAPTURE
    # the library is still usable: the same call eagerly works
    m.crba(q, out=M)
    torch.cuda.synchronize()


def test_capture_after_upload_replays_bitwise():
    say("[gpu] capture: chain and RNEA adjoint after bard_model_upload")
    tree = synth.humanoid_large()
    B = 1000
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    m.upload(ee=ee, adjoint=True)
    host = [inputs(tree, B, 2710 + k, "float32") for k in range(3)]
    q, qd, qdd = (to_dev(x, "float32") for x in host[0])
    tb = torch.randn((tree.nv, B), device="cuda")
    tau = torch.empty((tree.nv, B), device="cuda")
    M = torch.empty((tree.nv * tree.nv, B), device="cuda")
    J = torch.empty((6 * tree.nv * len(ee), B), device="cuda")
    qb = torch.empty((tree.nq, B), device="cuda")
    qdb = torch.empty((tree.nv, B), device="cuda")
    qddb = torch.empty((tree.nv, B), device="cuda")
    pib = torch.empty((tree.n_bodies, 10), device="cuda")
    L_adj = bard._layouts([q, qd, qdd, tb, qb, qdb, qddb], "soa")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.chain(q, qd, qdd, ee, out=(tau, M, J))
        rc = bard.bard_rnea_vjp(m.handle, bard.F32, bard._ptr(q), bard._ptr(qd), bard._ptr(qdd), bard._vp(0),
                                bard._ptr(tb), bard._ptr(qb), bard._ptr(qdb), bard._ptr(qddb), bard._ptr(pib),
                                L_adj, B, bard._stream_ptr(q))
        assert rc == 0, bard.bard_last_error()
    for rep in range(3):
        hq, hqd, hqdd = host[rep]
        q.copy_(to_dev(hq, "float32"))
        qd.copy_(to_dev(hqd, "float32"))
        qdd.copy_(to_dev(hqdd, "float32"))
        (torch.randn(1 << 18, device="cuda") * 3).sum().item()     # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        et, eM, eJ = m.chain(q, qd, qdd, ee)
        eqb, eqdb, eqddb, epib = m.rnea_vjp(q, qd, qdd, tb)
        torch.cuda.synchronize()
        for a, b, nm in [(tau, et, "tau"), (M, eM, "M"), (J, eJ, "J"), (qb, eqb, "q_bar"), (qdb, eqdb, "qd_bar"),
                         (qddb, eqddb, "qdd_bar"), (pib, epib, "inertia_bar")]:
            assert torch.equal(a, b), f"replay {rep}: {nm} differs from the eager call"


def test_plan_captured_by_caller():
    say("[gpu] capture: a plan inside the caller's graph")
    trees = synth.multi_trees()
    batches = [64, 37, 129, 8, 200]
    models = [bard.Model.from_tree(t) for t in trees]
    dev = [tuple(to_dev(x, "float32") for x in inputs(t, B, 2720 + k, "float32"))
           for k, (t, B) in enumerate(zip(trees, batches))]
    plan = bard.Plan(models, batches)
    plan._outputs(dev[0][0].device)               # output tensors exist before any capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(bard.BardError) as e:      # never run: refused
        with torch.cuda.graph(g):
            plan.run(dev, stream=torch.cuda.current_stream().cuda_stream)
    assert e.value.status == bard.E_CAPTURE
    eager = [tuple(x.clone() for x in o) for o in plan.run(dev)]
    torch.cuda.synchronize()
    for o in plan.run(dev):
        for x in o:
            x.zero_()
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        outs = plan.run(dev, stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(2):
        for o in outs:
            for x in o:
                x.zero_()
        g2.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, outs):
            for x, y in zip(a, b):
                assert torch.equal(x, y), f"replay {rep} differs from the eager plan run"
