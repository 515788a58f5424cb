"""Host side of the model specialiser (no GPU): the generated chain source for
a tree names every dof's torque, every mass-matrix entry and every Jacobian
column once or as a structural zero, and hipRTC compiles it for gfx950
(BARD_SPEC_COMPILE_ONLY), in FP32 and FP64 and both Jacobian frames; trees
past the size bound are refused."""

import re

import pytest

import synth
from paper_2605_31481_amd import bard


@pytest.mark.parametrize("name,dtype,frame", [("chain7", "float32", 0), ("chain7", "float64", 1),
                                              ("quadruped_spine", "float32", 1), ("free1", "float64", 0)])
def test_generated_source_compiles(name, dtype, frame):
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    m.specialize(tree.ee_bodies, frame=frame, dtype=dtype, compile_only=True)


def _table(src, which):
    """The structural-zero rows of M or J listed in the generated source."""
    n = int(re.search(rf"NZ{which} = (\d+);", src).group(1))
    vals = re.search(rf"Z{which}\[\d+\] = \{{([0-9, ]*)\}}", src).group(1).split(",")
    return [int(x) for x in vals[:n]]


def test_generated_source_covers_every_output():
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    src = m.specialized_source(ee)
    nv = tree.nv
    tau = {int(k) for k in re.findall(r"&tb\[(\d+) \* st_k\]", src)}
    assert tau == set(range(nv))
    stored = [int(k) for k in re.findall(r"&Mb\[(\d+) \* sM_k\]", src)]
    zeros = _table(src, "M")
    assert sorted(stored + zeros) == list(range(nv * nv))
    jcols = [int(k) for k in re.findall(r"&Jb\[(\d+) \* sJ_k\]", src)]
    jz = _table(src, "J")
    assert sorted(jcols + jz) == list(range(len(ee) * 6 * nv))
    assert "float" in src and "double" not in src


def test_deep_tree_refused_on_the_host():
    tree = synth.tree_by_name("chain64")
    m = bard.Model.from_tree(tree)
    with pytest.raises(bard.BardError) as ei:
        m.specialize(tree.ee_bodies, compile_only=True)
    assert ei.value.status == -7
