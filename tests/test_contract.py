"""CPU pins of the tolerance contract's ingredients.

* The oracle's transmitted joint forces (rnea_forces), which set the torque
  scale: a pendulum's closed form, and Newton's second law for a whole
  fixed-base tree (root joint force = sum of m_k (a_k - g) with each centre of
  mass acceleration a_k from second differences of FK, an independent route).
* Attainability: a plain single-precision evaluation of the textbook
  recursions meets the per-entry contract with a wide margin on every
  workload tree, while the sum of absolute per-body terms is not an
  attainable scale (the reason the contract does not use it).
"""

import numpy as np
import pytest

import synth
from oracle import OracleModel
from parity_util import TOL, entry_scales, inputs, mass_scales

G = 9.81


def test_pendulum_joint_force_closed_form():
    mass, l, ixx = 1.3, 0.7, 0.02
    t = synth.pendulum(m=mass, l=l, ixx=ixx)
    om = OracleModel.from_tree(t)
    rng = np.random.default_rng(11)
    q = rng.uniform(-np.pi, np.pi, (16, 1))
    qd = rng.standard_normal((16, 1))
    qdd = rng.standard_normal((16, 1))
    f = om.rnea_forces(q, qd, qdd)[:, 0]
    s, c = np.sin(q[:, 0]), np.cos(q[:, 0])
    # body frame rotates about x; COM at [0, 0, -l]: tangential +y, centripetal +z
    ft_y = mass * (l * qdd[:, 0] + G * s)
    ft_z = mass * (l * qd[:, 0] ** 2 + G * c)
    ref = np.zeros((16, 6))
    ref[:, 0] = ixx * qdd[:, 0] + l * ft_y
    ref[:, 4] = ft_y
    ref[:, 5] = ft_z
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["random11", "quadruped_spine", "chain7"])
def test_root_joint_force_is_total_momentum_rate(name):
    tree = synth.tree_by_name(name)
    assert tree.joint_type[0] != synth.FREE
    om = OracleModel.from_tree(tree)
    B = 8
    q, qd, qdd = synth.random_state(tree, B, 31)
    f0 = om.rnea_forces(q, qd, qdd)[:, 0]
    # centre of mass of every body in world coordinates along q(t) = q + t qd + t^2/2 qdd
    cl = tree.inertia[:, 1:4] / tree.inertia[:, :1]
    m = tree.inertia[:, 0]

    def coms(t):
        T = om.fk(q + t * qd + 0.5 * t * t * qdd)
        return np.einsum("bkij,kj->bki", T[:, :, :, :3], cl) + T[:, :, :, 3]

    h = 1e-3
    acc = (coms(h) - 2 * coms(0.0) + coms(-h)) / (h * h)
    g = np.asarray(tree.gravity, dtype=float)
    # the bodies carried by body 0's joint: its subtree (other roots hang from the world)
    sub = np.zeros(tree.n_bodies, bool)
    for k in range(tree.n_bodies):
        sub[k] = k == 0 or (tree.parent[k] >= 0 and sub[tree.parent[k]])
    force_world = np.einsum("k,bki->bi", m * sub, acc - g)
    R0 = om.fk(q)[:, 0, :, :3]
    force_root = np.einsum("bji,bj->bi", R0, force_world)   # R0^T f
    np.testing.assert_allclose(f0[:, 3:], force_root, rtol=1e-5, atol=1e-5 * np.abs(force_root).max())


def _attained(om, tree, q, qd, qdd):
    rt, rM = om.rnea(q, qd, qdd), om.crba(q)
    st, sm = entry_scales(om, tree, q, qd, qdd)
    rtol, atol = TOL["float32"]
    t32, M32 = om.rnea_f32(q, qd, qdd), om.crba_f32(q)
    wt = np.abs(t32 - rt) / (atol + rtol * np.maximum(np.abs(rt), st))
    B = q.shape[0]
    wm = np.abs(M32 - rM).reshape(B, -1) / (atol + rtol * np.maximum(np.abs(rM).reshape(B, -1), sm))
    return float(wt.max()), float(wm.max())


@pytest.mark.parametrize("name", ["chain7", "random18", "quadruped_spine", "humanoid_large"])
def test_single_precision_textbook_evaluation_meets_contract(name):
    tree = synth.tree_by_name(name)
    om = OracleModel.from_tree(tree)
    q, qd, qdd = inputs(tree, 128, 77, "float32")
    wt, wm = _attained(om, tree, q, qd, qdd)
    assert wt < 0.5 and wm < 0.5, (wt, wm)


def test_per_body_term_sums_are_not_an_attainable_scale():
    """Holding M_ij against the sum over bodies of |M^(k)_ij| (each body's
    parameters alone) fails even for the textbook recursion in single
    precision on the free-root humanoid: a term that is small because of how
    a vector projects still carries rounding of the vector's length."""
    tree = synth.humanoid_large()
    om = OracleModel.from_tree(tree)
    q, _, _ = inputs(tree, 128, 77, "float32")
    B = q.shape[0]
    rM = om.crba(q).reshape(B, -1)
    S = np.zeros_like(rM)
    for k in range(tree.n_bodies):
        pi = np.zeros_like(tree.inertia)
        pi[k] = tree.inertia[k]
        S += np.abs(om.crba(q, inertia=pi)).reshape(B, -1)
    rtol, atol = TOL["float32"]
    err = np.abs(om.crba_f32(q).reshape(B, -1) - rM)
    assert (err / (atol + rtol * np.maximum(np.abs(rM), S))).max() > 1.0
    # the contract's scale for M bounds every per-body term sum from above
    assert (mass_scales(rM.reshape(B, tree.nv, tree.nv)) >= S * (1 - 1e-12)).all()


@pytest.mark.parametrize("name,B", [("quadruped_spine", 300), ("humanoid_large", 129)])
def test_rounding_of_the_aba_adjoint_product_alone(name, B):
    """The FP32 ABA adjoint's second stage is q_bar = D^T c with D = dtau/dq
    and c = -M^-1 qdd_bar.  On the instances of its GPU test, the exact D and
    c rounded to single precision and the product summed in single precision
    stay within the normwise bound relative to the result: rounding of the
    product alone does not need the wider |D|^T |c| scale the GPU test uses;
    what exceeds the normwise bound there comes from the entries of D, which
    the adjoint sweeps form in single precision."""
    tree = synth.tree_by_name(name)
    om = OracleModel.from_tree(tree)
    q, qd, qdd0 = inputs(tree, B, 3700, "float32")
    tau = synth.to_fp32_grid(om.rnea(q, qd, qdd0))
    qdd = synth.to_fp32_grid(om.aba(q, qd, tau))
    cot = synth.to_fp32_grid(np.random.default_rng(3701).standard_normal((B, tree.nv)))
    c = -np.linalg.solve(om.crba(q), cot[..., None])[..., 0]
    D = np.zeros((B, tree.nv, om.nq))
    for i in range(tree.nv):
        e = np.zeros((B, tree.nv))
        e[:, i] = 1.0
        D[:, i, :] = om.rnea_vjp(q, qd, qdd, e)[0]
    g = np.einsum("bi,biq->bq", c, D)
    terms = D.astype(np.float32) * c.astype(np.float32)[:, :, None]
    g32 = np.zeros((B, om.nq), np.float32)
    for i in range(tree.nv):
        g32 = (g32 + terms[:, i, :]).astype(np.float32)
    rtol, atol = TOL["float32"]
    err = np.abs(g32 - g).max(axis=1)
    assert (err / (atol + rtol * np.abs(g).max(axis=1))).max() < 0.5
