"""bard_rnea_vjp_noalloc, the RNEA adjoint for callers that cannot allocate,
through the C ABI: refused with BARD_E_STATE (nothing launched) while the
model is not on the device; afterwards bitwise equal to bard_rnea_vjp (same
kernels, same grid) on two calls in a row, the second with a smaller batch,
in FP32 and FP64, with and without the inertial-parameter gradient; and no
change of the device's free memory across a call."""

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard
from parity_util import inputs, say, to_dev

pytestmark = pytest.mark.gpu


def _outs(torch, tree, B, dtype, with_pi=True):
    t = getattr(torch, dtype)
    mk = lambda k: torch.full((k, B), 123.0, dtype=t, device="cuda")
    pib = torch.full((tree.n_bodies, 10), 123.0, dtype=t, device="cuda") if with_pi else None
    return mk(tree.nq), mk(tree.nv), mk(tree.nv), pib


def _case(tree, B, seed, dtype):
    q, qd, qdd = inputs(tree, B, seed, dtype)
    tb = np.random.default_rng(seed + 1).standard_normal((B, tree.nv))
    if dtype == "float32":
        tb = synth.to_fp32_grid(tb)
    return [to_dev(x, dtype) for x in (q, qd, qdd, tb)]


def test_refused_until_uploaded():
    import torch
    say("[gpu] rnea_vjp_noalloc refused before upload")
    tree = synth.quadruped_spine()
    m = bard.Model.from_tree(tree)
    d = _case(tree, 64, 4400, "float32")
    out = _outs(torch, tree, 64, "float32")
    with pytest.raises(bard.BardError) as ei:
        m.rnea_vjp_noalloc(*d, out)
    assert ei.value.status == bard.E_STATE
    torch.cuda.synchronize()
    for o in out:
        assert bool((o == 123.0).all()), "a refused call launched nothing"


@pytest.mark.parametrize("name,dtype,B1,B2", [("quadruped_spine", "float32", 20000, 700),
                                               ("humanoid_large", "float32", 4096, 333),
                                               ("humanoid_small", "float64", 3000, 129)])
def test_matches_rnea_vjp_on_two_calls(name, dtype, B1, B2):
    import torch
    say(f"[gpu] rnea_vjp_noalloc {name} {dtype} B={B1} then B={B2}")
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    m.upload()
    for B, seed in ((B1, 4500), (B2, 4600)):
        d = _case(tree, B, seed, dtype)
        for with_pi in (True, False):
            ref = m.rnea_vjp(*d, inertia_grad=with_pi)
            got = m.rnea_vjp_noalloc(*d, _outs(torch, tree, B, dtype, with_pi))
            torch.cuda.synchronize()
            for lbl, a, b in zip(("q_bar", "qd_bar", "qdd_bar", "inertia_bar"), got, ref):
                if b is None:
                    assert a is None
                    continue
                assert torch.equal(a, b), f"{lbl} (B={B}, inertia_bar={with_pi}) differs from bard_rnea_vjp"


def test_allocates_nothing():
    import torch
    say("[gpu] rnea_vjp_noalloc leaves the device's free memory unchanged")
    tree = synth.random_tree(18, 3601)
    warm = bard.Model.from_tree(tree)   # loads the kernels' code objects
    d = _case(tree, 5000, 4700, "float32")
    warm.rnea_vjp(*d)
    warm.rnea_vjp_noalloc(*d, _outs(torch, tree, 5000, "float32"))
    m = bard.Model.from_tree(tree)
    m.upload()
    out = _outs(torch, tree, 5000, "float32")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    m.rnea_vjp_noalloc(*d, out)
    m.rnea_vjp_noalloc(*d, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
