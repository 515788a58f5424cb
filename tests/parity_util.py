"""Helpers shared by the GPU parity tests: seeded inputs on the device and the
tolerance contract.

Tolerance contract.  Inputs are rounded to the kernel's precision first and
the FP64 oracle runs on exactly those values.  For FK, Jacobian, RNEA and CRBA
the check is normwise per (instance, output block):
``max_k |gpu - ref| <= atol + rtol * max_k |ref|`` with FP32 rtol = 1e-5,
atol = 1e-6 and FP64 rtol = atol = 1e-12.  ABA is checked by its backward
error, ``|RNEA_ref(q, qd, qdd_gpu) - tau|_inf <= atol + rtol * (|tau|_inf +
|M|_inf |qdd_gpu|_inf + |RNEA_ref(q, qd, 0)|_inf)``, because its forward error
is only bounded by cond(M) times the unit roundoff.  Trees whose sums are
badly conditioned (a root carrying tens of children) are checked against the
size of the summed terms instead of the result (assert_normwise_scaled).
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
