"""The host-side model compiler and the FP64 oracle built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer (host code only; no GPU code
is built here), run on every named synthetic tree, on seeded random trees and
on malformed trees the compiler must reject.  The drivers are in
tests/sanitize/."""

import os
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _trees():
    names = ["chain7", "humanoid_large", "humanoid_small", "quadruped_spine", "random7", "random11", "random12",
             "random18", "random23"] + synth.EDGE_TREES
    out = [(0, synth.tree_by_name(n)) for n in names]
    out += [(0, synth.random_tree(n, 5000 + n)) for n in (5, 9, 17, 33, 64)]
    out += [(0, synth.pendulum()), (0, synth.two_link_planar())]
    base = synth.random_tree(6, 5100)
    bad = []
    for kind in ("parent_not_before", "free_not_root", "zero_axis", "negative_mass", "inertia_not_pd"):
        par, jt = base.parent.copy(), base.joint_type.copy()
        ax, xt, pi = base.axis.copy(), base.X_tree.copy(), base.inertia.copy()
        if kind == "parent_not_before":
            par[3] = 4
        elif kind == "free_not_root":
            jt[2] = synth.FREE
        elif kind == "zero_axis":
            ax[1] = 0.0
        elif kind == "negative_mass":
            pi[2, 0] = -1.0
        else:
            pi[2, 4] = -5.0
        bad.append((1, (par, jt, ax, xt, pi)))
    return out, bad


def _write(path):
    good, bad = _trees()
    rows = []
    for expect, t in good:
        rows.append((expect, (t.parent, t.joint_type, t.axis, t.X_tree, t.inertia)))
    rows += bad
    with open(path, "w") as f:
        f.write(f"{len(rows)}\n")
        for expect, (par, jt, ax, xt, pi) in rows:
            f.write(f"{expect} {len(par)}\n")
            for arr in (par, jt, ax, xt, pi):
                f.write(" ".join(repr(float(x)) for x in np.asarray(arr, dtype=float).ravel()) + "\n")
    return len(rows)


def _build(name, sources, extra=()):
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, name)
    cmd = ["g++", *SAN, *extra, *sources, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.fixture(scope="module")
def tree_file():
    path = os.path.join(OUT, "trees.txt")
    os.makedirs(OUT, exist_ok=True)
    _write(path)
    return path


def test_model_compiler_under_sanitizers(tree_file):
    exe = _build("compiler_check", [os.path.join(SRC, "compiler_check.cpp"),
                                    os.path.join(ROOT, "paper_2605_31481_amd", "csrc", "compiler.cpp")])
    r = subprocess.run([exe, tree_file], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout


def test_oracle_under_sanitizers(tree_file):
    exe = _build("oracle_check", [os.path.join(SRC, "oracle_check.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp")],
                 extra=("-fopenmp",))
    r = subprocess.run([exe, tree_file], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
