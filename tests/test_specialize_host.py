"""Host side of the model specialiser (no GPU): the generated chain source for
a tree, in each form (split over waves by limbs, dual, whole), names every
dof's torque, every mass-matrix entry and every Jacobian column once or as a
structural zero, and hipRTC compiles it for gfx950 (BARD_SPEC_COMPILE_ONLY),
in FP32 and FP64 and both Jacobian frames; the split form gives each limb to
one wave; trees past the size bound are refused."""

import re

import numpy as np
import pytest

import synth
from paper_2605_31481_amd import bard


@pytest.mark.parametrize("name,dtype,frame,form", [("chain7", "float32", 0, "split"), ("chain7", "float64", 1, "whole"),
                                                   ("chain7", "float32", 1, "dual"),
                                                   ("quadruped_spine", "float32", 1, "split"),
                                                   ("quadruped_spine", "float64", 0, "whole"),
                                                   ("humanoid_small", "float32", 0, "dual"),
                                                   ("free1", "float64", 0, "dual"), ("star64", "float32", 0, "split"),
                                                   ("quadruped_spine", "float32", 0, "triple"),
                                                   ("humanoid_small", "float64", 1, "triple")])
def test_generated_source_compiles(name, dtype, frame, form):
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    m.specialize(tree.ee_bodies, frame=frame, dtype=dtype, compile_only=True, form=form)


def _table(src, which):
    """The structural-zero rows of M or J listed in the generated source."""
    n = int(re.search(rf"NZ{which} = (\d+);", src).group(1))
    vals = re.search(rf"Z{which}\[\d+\] = \{{([0-9, ]*)\}}", src).group(1).split(",")
    return [int(x) for x in vals[:n]]


@pytest.mark.parametrize("form", ["split", "whole", "dual", "triple"])
def test_generated_source_covers_every_output(form):
    tree = synth.humanoid_small()
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    src = m.specialized_source(ee, form=form)
    nv = tree.nv
    tau = {int(k) for k in re.findall(r"TAU\((\d+), ", src)}
    assert tau == set(range(nv))
    stored = [int(k) for k in re.findall(r"MA\((\d+), ", src)]
    zeros = _table(src, "M")
    assert sorted(stored + zeros) == list(range(nv * nv))
    jcols = [int(k) for k in re.findall(r"JA\((\d+), ", src)]
    jz = _table(src, "J")
    assert sorted(jcols + jz) == list(range(len(ee) * 6 * nv))
    assert "typedef float Real;" in src and "typedef double Real;" not in src


def test_deep_tree_refused_on_the_host():
    tree = synth.tree_by_name("chain64")
    m = bard.Model.from_tree(tree)
    with pytest.raises(bard.BardError) as ei:
        m.specialize(tree.ee_bodies, compile_only=True)
    assert ei.value.status == -7


@pytest.mark.parametrize("name,waves", [("humanoid_large", 5), ("humanoid_small", 3), ("quadruped_spine", 4),
                                        ("chain7", 1), ("free1", 1),
                                        ("star64", 8)])
def test_split_form_waves(name, waves):
    """A branched tree's split form has one wave per limb (at most 8, limbs
    dealt longest first); a chain keeps one wave; the whole form has one."""
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    src = m.specialized_source(tree.ee_bodies)
    assert int(re.search(r"NW = (\d+);", src).group(1)) == waves
    assert ("__syncthreads" in src) == (waves > 1)
    whole = m.specialized_source(tree.ee_bodies, form="whole")
    assert int(re.search(r"NW = (\d+);", whole).group(1)) == 1
    dual = m.specialized_source(tree.ee_bodies, form="dual")
    assert int(re.search(r"NW = (\d+);", dual).group(1)) == waves
    assert int(re.search(r"WG_PER_GROUP = (\d+);", dual).group(1)) == 2


@pytest.mark.parametrize("name,dtype,waves,lds,compile_", [("humanoid_large", "float32", 5, True, True),
                                                           ("humanoid_large", "float64", 1, True, False),
                                                           ("chain7", "float32", 1, True, True),
                                                           ("free1", "float64", 1, False, True),
                                                           ("quadruped_spine", "float32", 4, True, True),
                                                           ("star64", "float32", 1, True, False),
                                                           ("star64", "float64", 1, False, False)])
def test_generated_aba_source(name, dtype, waves, lds, compile_):
    """The forward-dynamics kernel's source stores every acceleration once,
    splits over waves by limbs where its LDS hand-over fits (the FP64
    humanoid and the 64-body star keep one wave), keeps the one-wave form's
    per-body W and e in LDS while they fit in 150 KB (in registers for the
    FP64 64-body star, whose copy would take 224 KB), and compiles for gfx950."""
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    src = m.specialized_aba_source(dtype=dtype)
    stored = sorted(int(k) for k in re.findall(r"QDDO\((\d+), ", src))
    assert stored == list(range(tree.nv))
    assert int(re.search(r"NW = (\d+);", src).group(1)) == waves
    assert src.count("__syncthreads") == (2 if waves > 1 and name != "chain7" else 0)
    assert ("__shared__" in src) == lds
    if compile_:  # (the one-wave forms of the large trees take minutes on the host; the GPU tests load them)
        m.specialize_aba(dtype=dtype, compile_only=True)


def test_deep_tree_refused_for_aba():
    m = bard.Model.from_tree(synth.tree_by_name("chain64"))
    with pytest.raises(bard.BardError) as ei:
        m.specialize_aba(compile_only=True)
    assert ei.value.status == -7


def test_generated_multi_tree_plan_source():
    """The plan's generated kernel (fusion 3) holds each tree's code in a
    namespace of its own, dispatches the trees' 64-instance groups (two
    workgroups each in the dual form) with trees of larger nv first, sizes
    its workgroups for the widest member, and compiles for gfx950."""
    trees = synth.multi_trees()
    models = [bard.Model.from_tree(t) for t in trees]
    plan = bard.Plan(models, synth.MULTI_BATCHES)
    src = plan.specialized_source()
    order = [int(k) for k in re.findall(r"bard_t(\d+)::run", src)]
    assert order == sorted(range(len(trees)), key=lambda k: -trees[k].nv)
    ends = [int(e) for e in re.findall(r"if \(blk < (\d+)LL\)", src)]
    groups = [(B + 63) // 64 * 2 for B in synth.MULTI_BATCHES]   # dual form: two workgroups per group
    assert ends == list(np.cumsum([groups[k] for k in order]))
    nw = [int(w) for w in re.findall(r"static constexpr int NW = (\d+);", src)]
    assert int(re.search(r"__launch_bounds__\((\d+)\) bard_spec_plan", src).group(1)) == 64 * max(nw)
    for k, t in enumerate(trees):   # every torque stored once per tree
        body = src.split(f"namespace bard_t{k} {{")[1].split(f"}}  // namespace bard_t{k}")[0]
        assert sorted(set(int(x) for x in re.findall(r"TAU\((\d+), ", body))) == list(range(t.nv))
    plan.specialized_source(compile_only=True)
    # plans without all three operators have no generated kernel
    p1 = bard.Plan(models, synth.MULTI_BATCHES, op_mask=bard.PLAN_RNEA)
    with pytest.raises(bard.BardError) as ei:
        p1.specialized_source()
    assert ei.value.status == -7


@pytest.mark.parametrize("name,form", [("humanoid_large", "split"), ("humanoid_large", "whole"),
                                       ("quadruped_spine", "split"), ("chain7", "split")])
def test_generated_rnea_only_source(name, form):
    """The inverse-dynamics-only kernel stores every torque once and no
    mass-matrix or Jacobian entry (only the accessor macros name them), and
    compiles for gfx950."""
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    src = m.specialized_rnea_source(form=form)
    tau = [int(k) for k in re.findall(r"TAU\((\d+), ", src)]
    assert sorted(tau) == list(range(tree.nv))
    assert re.findall(r"\bMA\((\d+), ", src) == [] and re.findall(r"\bJA\((\d+), ", src) == []
    assert int(re.search(r"NZM = (\d+);", src).group(1)) == 0
    m.specialize_rnea(compile_only=True, form=form)


@pytest.mark.parametrize("name,form", [("humanoid_large", "split"), ("humanoid_small", "whole"),
                                       ("quadruped_spine", "split")])
def test_generated_crba_only_source(name, form):
    """The mass-matrix-only kernel names every entry of M once, as a stored
    value or as a structural zero of its table, and no torque or Jacobian
    entry; it compiles for gfx950."""
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    src = m.specialized_op_source("crba", form=form)
    stored = [int(k) for k in re.findall(r"\bMA\((\d+), ", src)]
    assert sorted(stored + _table(src, "M")) == list(range(tree.nv * tree.nv))
    assert re.findall(r"\bTAU\((\d+), ", src) == [] and re.findall(r"\bJA\((\d+), ", src) == []
    assert "QD(" not in src.split("bard_spec_chain(")[1]     # velocities and accelerations are not read
    m.specialize_op("crba", compile_only=True, form=form)


@pytest.mark.parametrize("name,frame,form", [("humanoid_large", 0, "split"), ("humanoid_small", 1, "whole"),
                                             ("quadruped_spine", 1, "split")])
def test_generated_jacobian_only_source(name, frame, form):
    """The Jacobian-only kernel names every Jacobian entry once, as a stored
    value or an off-path zero of its table, no torque or mass-matrix entry,
    reads no velocity, has no barrier, and compiles for gfx950."""
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    ee = tree.ee_bodies
    src = m.specialized_op_source("jacobian", form=form, ee=ee, frame=frame)
    stored = [int(k) for k in re.findall(r"\bJA\((\d+), ", src)]
    assert sorted(stored + _table(src, "J")) == list(range(len(ee) * 6 * tree.nv))
    assert re.findall(r"\bTAU\((\d+), ", src) == [] and re.findall(r"\bMA\((\d+), ", src) == []
    assert "QD(" not in src.split("bard_spec_chain(")[1] and "__syncthreads" not in src
    m.specialize_op("jacobian", compile_only=True, form=form, ee=ee, frame=frame)


@pytest.mark.parametrize("name,form", [("humanoid_large", "split"), ("humanoid_small", "whole"),
                                       ("free_branches61", "split")])
def test_generated_fk_only_source(name, form):
    """The pose-only kernel stores the 12 pose values of every body once and
    nothing else, reads no velocity, has no barrier, and compiles."""
    tree = synth.tree_by_name(name)
    m = bard.Model.from_tree(tree)
    src = m.specialized_op_source("fk", form=form)
    stored = [int(k) for k in re.findall(r"\bPA\((\d+), ", src)]
    assert sorted(stored) == list(range(12 * tree.n_bodies))
    assert not re.findall(r"\b(TAU|MA|JA)\((\d+), ", src)
    assert "QD(" not in src.split("bard_spec_chain(")[1] and "__syncthreads" not in src
    if name != "free_branches61":   # (its compile takes a while on the host; the GPU tests load it)
        m.specialize_op("fk", compile_only=True, form=form)
