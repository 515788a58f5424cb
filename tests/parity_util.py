"""Helpers shared by the GPU parity tests: seeded inputs on the device and the
tolerance contract.

Tolerance contract.  Inputs are rounded to the kernel's precision first and
the FP64 oracle runs on exactly those values; FP32 rtol = 1e-5, atol = 1e-6,
FP64 rtol = atol = 1e-12.

* Torques and mass-matrix entries are held entry by entry:
  ``|gpu_e - ref_e| <= atol + rtol * max(|ref_e|, S_e)``, where S_e is the sum
  over bodies k of |the same entry computed with body k's inertial parameters
  alone| (``body_terms``).  Both quantities are linear in the parameters, so
  ref_e is the sum of those per-body terms; any evaluation that rounds each
  term to the working precision before adding them errs by about u S_e
  (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 4.2), so S_e
  is the size the entry's accuracy can be measured against.  Where nothing
  cancels S_e = |ref_e|.
* Jacobian columns are held per column (6 rows of one end effector's column
  against that column's largest entry): a column is a rotated unit axis and
  its moment, whose rounding error follows the column's size.
* FK is held per body block (the 12 entries of [R | p]).
* ABA is held by its backward error per instance (aba_backward_error),
  because its forward error is only bounded by cond(M) times the unit
  roundoff.
* Other outputs (adjoints) keep the normwise block check
  ``max_k |gpu - ref| <= atol + rtol * max_k |ref|`` unless a test states
  otherwise.
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
    sum of (see term_scales)."""
    rtol, atol = TOL[dtype]
    err = np.abs(gpu - ref).max(axis=-1)
    bound = atol + rtol * np.maximum(np.abs(ref).max(axis=-1), scale[:, None])
    ok = err <= bound
    worst = float((err / bound).max())
    assert ok.all(), f"{name}: {int((~ok).sum())} blocks out of tolerance, worst err/bound = {worst:.3g}"
    return worst


def body_terms(om, tree, q, qd=None, qdd=None, tau=True, mass=True):
    """Per-entry sums of the absolute per-body terms of the torque and the mass
    matrix: S_tau[b, i] = sum_k |RNEA_k(q, qd, qdd)_i| and
    S_M[b, i*nv + j] = sum_k |CRBA_k(q)_ij|, with RNEA_k and CRBA_k using
    body k's inertial parameters alone (zeros for every other body).  Returns
    (S_tau or None, S_M or None)."""
    B = q.shape[0]
    st = np.zeros((B, tree.nv)) if tau else None
    sm = np.zeros((B, tree.nv * tree.nv)) if mass else None
    for k in range(tree.n_bodies):
        pi = np.zeros_like(tree.inertia)
        pi[k] = tree.inertia[k]
        if tau:
            st += np.abs(om.rnea(q, qd, qdd, inertia=pi))
        if mass:
            sm += np.abs(om.crba(q, inertia=pi)).reshape(B, -1)
    return st, sm


def adjoint_body_terms(om, tree, q, qd, qdd, tau_bar):
    """Per-entry sums of the absolute per-body terms of the RNEA adjoint's
    q_bar, qd_bar and qdd_bar: for a fixed cotangent they are linear in the
    inertial parameters, as tau is."""
    B = q.shape[0]
    out = [np.zeros((B, tree.nq)), np.zeros((B, tree.nv)), np.zeros((B, tree.nv))]
    for k in range(tree.n_bodies):
        pi = np.zeros_like(tree.inertia)
        pi[k] = tree.inertia[k]
        for acc, g in zip(out, om.rnea_vjp(q, qd, qdd, tau_bar, inertia=pi)[:3]):
            acc += np.abs(g)
    return out


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
    st, sm = S if S is not None else body_terms(om, tree, q, qd, qdd, tau=tau is not None, mass=M is not None)
    w = {}
    if tau is not None:
        w["tau"] = assert_tau(f"{label}.tau", tau, rt, st, dtype)
    if M is not None:
        w["M"] = assert_mass(f"{label}.M", M, rM, sm, dtype)
    if J is not None:
        w["J"] = assert_jacobian(f"{label}.J", J, rJ, dtype)
    return w


def term_scales(om, tree, q, qd, qdd):
    """Sizes of the terms whose sums are the torque and the mass matrix.

    RNEA is linear in the inertial parameters, so tau = sum_k tau^(k) with
    tau^(k) the RNEA of body k's parameters alone, and likewise M.  Per
    instance this returns max_i sum_k |tau^(k)_i| and max_ij sum_k |M^(k)_ij|.
    An FP32 evaluation rounds the terms before it sums them, so its error is
    of the order of u times these sums (the summation bound of Higham,
    Accuracy and Stability of Numerical Algorithms, Sec. 4.2), which for a
    root carrying many children can far exceed u times the result."""
    B = q.shape[0]
    st = np.zeros((B, tree.nv))
    sm = np.zeros((B, tree.nv, tree.nv))
    zero = np.zeros((B, tree.nv))
    for k in range(tree.n_bodies):
        pi = np.zeros_like(tree.inertia)
        pi[k] = tree.inertia[k]
        st += np.abs(om.rnea(q, qd, qdd, inertia=pi))
        g = om.rnea(q, zero, zero, inertia=pi)
        for j in range(tree.nv):
            e = zero.copy()
            e[:, j] = 1.0
            sm[:, :, j] += np.abs(om.rnea(q, zero, e, inertia=pi) - g)
    return st.max(axis=1), sm.reshape(B, -1).max(axis=1)


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
