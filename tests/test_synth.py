"""Seeded generators: determinism, tree shapes and inertia validity."""

import numpy as np
import pytest

import synth


def _levels(tree):
    d = np.zeros(tree.n_bodies, dtype=int)
    for i, p in enumerate(tree.parent):
        d[i] = 1 if p < 0 else d[p] + 1
    return [int((d == k).sum()) for k in range(1, d.max() + 1)]


def test_deterministic():
    a = synth.humanoid_large()
    b = synth.humanoid_large()
    for f in ("parent", "joint_type", "axis", "X_tree", "inertia"):
        assert getattr(a, f).tobytes() == getattr(b, f).tobytes()
    qa = synth.random_state(a, 16, 5)
    qb = synth.random_state(b, 16, 5)
    for x, y in zip(qa, qb):
        assert x.tobytes() == y.tobytes()


@pytest.mark.parametrize("fn,n,nq,nv,widths", [
    (synth.chain7, 7, 7, 7, [1] * 7),
    (synth.humanoid_large, 31, 37, 36, [1, 3, 5, 5, 5, 4, 4, 2, 2]),
    (synth.humanoid_small, 18, 24, 23, [1, 2, 3, 3, 3, 2, 2, 1, 1]),
    (synth.quadruped_spine, 11, 11, 11, [3, 3, 1, 2, 2]),
])
def test_shapes(fn, n, nq, nv, widths):
    t = fn()
    assert (t.n_bodies, t.nq, t.nv) == (n, nq, nv)
    assert _levels(t) == widths
    assert all(t.parent[i] < i for i in range(n))


def test_multi_trees():
    ts = synth.multi_trees()
    assert [t.nv for t in ts] == [7, 11, 12, 18, 23]
    for t in ts:
        assert 4 <= t.depth <= 10
        assert 1 <= len(t.ee_bodies) <= 4


def test_inertia_valid():
    rng = np.random.default_rng(0)
    for _ in range(200):
        p = synth.random_inertia_params(rng)
        m, h = p[0], p[1:4]
        Io = np.array([[p[4], p[5], p[7]], [p[5], p[6], p[8]], [p[7], p[8], p[9]]])
        c = h / m
        Ic = Io - m * (c @ c * np.eye(3) - np.outer(c, c))
        ev = np.linalg.eigvalsh(Ic)
        assert 0.5 <= m <= 5 and np.all(np.abs(c) <= 0.1)
        assert ev.min() > 0.0099 and ev.max() < 0.1001
        assert ev[0] + ev[1] >= ev[2] - 1e-12
