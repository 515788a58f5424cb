"""Helpers shared by the GPU parity tests: seeded inputs on the device and the
tolerance contract.

Tolerance contract.  Inputs are rounded to the kernel's precision first and
the FP64 oracle runs on exactly those values; FP32 rtol = 1e-5, atol = 1e-6,
FP64 rtol = atol = 1e-12.  Every output entry e is held by
``|gpu_e - ref_e| <= atol + rtol * max(|ref_e|, S_e)`` with a per-entry scale
S_e fixed by the problem, not by either implementation:

* Torques: tau_i is the projection of the spatial force transmitted across
  joint i onto the joint's motion subspace.  Rounding the orientation of the
  axis or of that force by u (which any single-precision evaluation does, at
  every rotation it composes) moves the projection by u times the length of
  the projected vector, not u times the projection.  S_e is therefore the sum
  over bodies k, and over the three physical parts of the force (inertial
  M qdd, velocity products, gravity), of the length of body k's part of the
  force at joint i: the moment for a revolute dof, the force for a prismatic
  dof, and the corresponding 3-vector for a free root's angular and linear
  dofs (``entry_scales``; Higham, Accuracy and Stability of Numerical
  Algorithms, Sec. 4.2, for the sum of terms).
* Mass matrix: S_ij = sqrt(M_ii M_jj), the scaling under which a symmetric
  positive definite matrix's entries are compared (Higham, Sec. 10.1, after
  Demmel); it is invariant under a change of units of any one coordinate and
  bounds |M_ij| by Cauchy-Schwarz.
* Jacobian columns are held per column (6 rows of one end effector's column
  against that column's largest entry): a column is a rotated unit axis and
  its moment, whose rounding error follows the column's size.
* FK is held per body block (the 12 entries of [R | p]).
* ABA is held by its backward error per instance (aba_backward_error),
  because its forward error is only bounded by cond(M) times the unit
  roundoff.
* Reverse-mode products keep the normwise check per instance,
  ``max_k |gpu - ref| <= atol + rtol * max_k |ref|``: a gradient for a random
  cotangent mixes every output, so no per-entry scale follows from the
  operator's structure.

A plain single-precision evaluation of the textbook body-frame recursions
(``OracleModel.rnea_f32`` / ``crba_f32``) meets these bounds with a wide
margin (a CPU test checks it), so they are attainable and not fitted to the
kernels.
"""

import sys

import numpy as np

import synth
from oracle import OracleModel

TOL = {"float32": (1e-5, 1e-6), "float64": (1e-12, 1e-12)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def inputs(tree, B, seed, dtype):
    q, qd, qdd = synth.random_state(tree, B, seed)
    if dtype == "float32":
        q, qd, qdd = synth.to_fp32_grid(q), synth.to_fp32_grid(qd), synth.to_fp32_grid(qdd)
    return q, qd, qdd


def to_dev(x, dtype, layout="soa"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).to(getattr(torch, dtype))
    if layout == "soa":
        t = t.t().contiguous()
    return t.cuda()


def from_dev(t, layout="soa"):
    a = t.detach().cpu().double().numpy()
    return a.T.copy() if layout == "soa" else a


def normwise(gpu, ref, rtol, atol):
    """gpu, ref: [B, blocks, K].  Returns (ok mask [B, blocks], worst ratio)."""
    err = np.abs(gpu - ref).max(axis=-1)
    scale = np.abs(ref).max(axis=-1)
    bound = atol + rtol * scale
    return err <= bound, float((err / bound).max())


def assert_normwise(name, gpu, ref, dtype):
    rtol, atol = TOL[dtype]
    ok, worst = normwise(gpu, ref, rtol, atol)
    assert ok.all(), f"{name}: {int((~ok).sum())} blocks out of tolerance, worst err/bound = {worst:.3g}"
    return worst


def assert_normwise_scaled(name, gpu, ref, scale, dtype):
    """Normwise check against ``atol + rtol * max(max_k |ref|, scale)`` per
    (instance, block); ``scale`` [B] is the size of the terms the result is a
    sum of."""
    rtol, atol = TOL[dtype]
    err = np.abs(gpu - ref).max(axis=-1)
    bound = atol + rtol * np.maximum(np.abs(ref).max(axis=-1), scale[:, None])
    ok = err <= bound
    worst = float((err / bound).max())
    assert ok.all(), f"{name}: {int((~ok).sum())} blocks out of tolerance, worst err/bound = {worst:.3g}"
    return worst


def _zero_gravity(om):
    return OracleModel(om.parent, om.joint_type, om.axis, om.X_tree, om.inertia, gravity=(0.0, 0.0, 0.0))


def tau_scales(om, tree, q, qd, qdd):
    """Per-entry torque scale S_tau [B, nv] (module docstring): for every body
    k (its inertial parameters alone, from ``tree.inertia``) and every part of
    the motion, the length of the force body k's part transmits across each
    joint, summed; the length is taken of the moment (revolute dof, free-root
    angular dofs) or of the force (prismatic dof, free-root linear dofs)."""
    B = q.shape[0]
    om0 = _zero_gravity(om)
    z = np.zeros((B, tree.nv))
    W = np.zeros((B, tree.n_bodies, 2))
    for k in range(tree.n_bodies):
        pi = np.zeros_like(tree.inertia)
        pi[k] = tree.inertia[k]
        for mdl, v, a in ((om0, z, qdd), (om0, qd, z), (om, z, z)):
            f = mdl.rnea_forces(q, v, a, inertia=pi)
            W[:, :, 0] += np.linalg.norm(f[:, :, :3], axis=2)
            W[:, :, 1] += np.linalg.norm(f[:, :, 3:], axis=2)
    S = np.zeros((B, tree.nv))
    vo = tree.v_offsets()
    for i, t in enumerate(tree.joint_type):
        if t == synth.REVOLUTE:
            S[:, vo[i]] = W[:, i, 0]
        elif t == synth.PRISMATIC:
            S[:, vo[i]] = W[:, i, 1]
        elif t == synth.FREE:
            S[:, vo[i]:vo[i] + 3] = W[:, i, 1:2]   # velocity coordinates [v; w]
            S[:, vo[i] + 3:vo[i] + 6] = W[:, i, 0:1]
    return S


def mass_scales(M):
    """S_ij = sqrt(|M_ii| |M_jj|), flattened to [B, nv * nv]."""
    d = np.sqrt(np.abs(np.einsum("bii->bi", M)))
    return (d[:, :, None] * d[:, None, :]).reshape(M.shape[0], -1)


def entry_scales(om, tree, q, qd=None, qdd=None, tau=True, mass=True):
    """(S_tau [B, nv] or None, S_M [B, nv * nv] or None) for the contract."""
    st = tau_scales(om, tree, q, qd, qdd) if tau else None
    sm = mass_scales(om.crba(q, inertia=tree.inertia)) if mass else None
    return st, sm


def transpose_product_scales(om, q, qd, qdd, cot):
    """For g = D^T c with D = d tau / d(q or qd) the RNEA Jacobians: per
    instance max_j (|D|^T |c|)_j for q and for qd, the normwise size of the
    terms g sums (Higham, Sec. 3.5, matrix-vector products: the computed
    product errs by at most gamma_n |D|^T |c|)."""
    B, nv = cot.shape
    sq = np.zeros((B, om.nq))
    sqd = np.zeros((B, nv))
    for i in range(nv):
        e = np.zeros((B, nv))
        e[:, i] = 1.0
        dq, dqd, _, _ = om.rnea_vjp(q, qd, qdd, e)
        sq += np.abs(cot[:, i:i + 1]) * np.abs(dq)
        sqd += np.abs(cot[:, i:i + 1]) * np.abs(dqd)
    return sq.max(axis=1), sqd.max(axis=1)


def entrywise(gpu, ref, scale, rtol, atol):
    """Per-entry check ``|gpu - ref| <= atol + rtol * max(|ref|, scale)``.
    Returns (ok mask, worst err/bound)."""
    err = np.abs(gpu - ref)
    bound = atol + rtol * np.maximum(np.abs(ref), scale)
    ratio = err / bound
    return ratio <= 1.0, float(ratio.max()) if ratio.size else 0.0


def assert_entrywise(name, gpu, ref, scale, dtype):
    rtol, atol = TOL[dtype]
    gpu = np.asarray(gpu).reshape(ref.shape)
    ok, worst = entrywise(gpu, ref, scale.reshape(ref.shape), rtol, atol)
    assert ok.all(), f"{name}: {int((~ok).sum())} entries out of tolerance, worst err/bound = {worst:.3g}"
    return worst


def column_scale(J):
    """J [B, n_ee, 6, nv] -> per-entry scale: the largest |entry| of its column."""
    return np.broadcast_to(np.abs(J).max(axis=2, keepdims=True), J.shape)


def assert_tau(name, gpu, ref, S, dtype):
    return assert_entrywise(name, gpu, ref, S, dtype)


def assert_mass(name, gpu, ref, S, dtype):
    B = ref.shape[0]
    return assert_entrywise(name, np.asarray(gpu).reshape(B, -1), ref.reshape(B, -1), S, dtype)


def assert_jacobian(name, gpu, ref, dtype):
    """ref [B, n_ee, 6, nv]; gpu any shape of the same size."""
    return assert_entrywise(name, np.asarray(gpu).reshape(ref.shape), ref, column_scale(ref), dtype)


def assert_chain(om, tree, q, qd, qdd, ee, tau, M, J, dtype, frame=0, label="chain", ref=None, S=None):
    """Per-entry contract for the outputs of one chain evaluation (host arrays,
    instance-major; any of tau, M, J may be None)."""
    rt, rM, rJ = ref if ref is not None else om.chain(q, qd, qdd, ee, frame=frame)
    st, sm = S if S is not None else entry_scales(om, tree, q, qd, qdd, tau=tau is not None, mass=M is not None)
    w = {}
    if tau is not None:
        w["tau"] = assert_tau(f"{label}.tau", tau, rt, st, dtype)
    if M is not None:
        w["M"] = assert_mass(f"{label}.M", M, rM, sm, dtype)
    if J is not None:
        w["J"] = assert_jacobian(f"{label}.J", J, rJ, dtype)
    return w


def aba_backward_error(om, q, qd, tau, qdd_gpu, dtype):
    rtol, atol = TOL[dtype]
    res = om.rnea(q, qd, qdd_gpu) - tau
    M = om.crba(q)
    bias = om.rnea(q, qd, np.zeros_like(qd))
    scale = (np.abs(tau).max(axis=1) + np.abs(M).sum(axis=2).max(axis=1) * np.abs(qdd_gpu).max(axis=1)
             + np.abs(bias).max(axis=1))
    err = np.abs(res).max(axis=1)
    bound = atol + rtol * scale
    return err <= bound, float((err / bound).max())


def affine_rnea_ok(om, q, qd, qdd, tau_gpu, dtype):
    """Inverse dynamics evaluated as tau = M qdd + b from cached M and b: the
    error bound is that of ABA's backward error, atol + rtol (|tau| + |M| |qdd|
    + |b|) in the infinity norm, per instance."""
    rtol, atol = TOL[dtype]
    ref = om.rnea(q, qd, qdd)
    M = om.crba(q)
    bias = om.rnea(q, qd, np.zeros_like(qd))
    scale = (np.abs(ref).max(axis=1) + np.abs(M).sum(axis=2).max(axis=1) * np.abs(qdd).max(axis=1)
             + np.abs(bias).max(axis=1))
    err = np.abs(tau_gpu - ref).max(axis=1)
    bound = atol + rtol * scale
    return err <= bound, float((err / bound).max())


def fk_ref_blocks(om, q):
    T = om.fk(q)                       # [B, n, 3, 4]
    return T.reshape(T.shape[0], T.shape[1], 12)


def oracle_for(tree):
    return OracleModel.from_tree(tree)
