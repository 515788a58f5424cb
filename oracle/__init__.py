"""FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liboracle.so`` (built from ``oracle.cpp`` by
``oracle.buildlib.build()`` with g++), which shares no code with the GPU library.

All arrays are float64 and instance-major: ``q[B, nq]``, ``qd/qdd/tau[B, nv]``,
``poses[B, n, 3, 4]``, ``J[B, n_ee, 6, nv]`` (rows ``[linear; angular]``),
``M[B, nv, nv]``.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .buildlib import build, library_path

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(ctypes.c_int)
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.orc_model_new.restype = P
    lib.orc_model_new.argtypes = [ci, I, I, D, D, D, D]
    lib.orc_model_free.argtypes = [P]
    lib.orc_dims.argtypes = [P, I, I]
    lib.orc_fk.argtypes = [P, i64, D, D, ci]
    lib.orc_jacobian.argtypes = [P, i64, D, ci, I, ci, D, ci]
    lib.orc_rnea.argtypes = [P, i64, D, D, D, D, D, ci]
    lib.orc_crba.argtypes = [P, i64, D, D, ci]
    lib.orc_crba_pi.argtypes = [P, i64, D, D, D, ci]
    lib.orc_aba.argtypes = [P, i64, D, D, D, D, ci]
    lib.orc_chain.argtypes = [P, i64, D, D, D, ci, I, ci, D, D, D, ci]
    lib.orc_energy.argtypes = [P, i64, D, D, D, D, ci]
    lib.orc_rnea_vjp.argtypes = [P, i64, D, D, D, D, D, D, D, D, D, ci]
    lib.orc_fk_vjp.argtypes = [P, i64, D, D, D, ci]
    lib.orc_crba_vjp.argtypes = [P, i64, D, D, D, D, D, ci]
    lib.orc_rnea_forces.argtypes = [P, i64, D, D, D, D, D, ci]
    Fp = ctypes.POINTER(ctypes.c_float)
    lib.orc_rnea_f32.argtypes = [P, i64, Fp, Fp, Fp, Fp, Fp, ci]
    lib.orc_crba_f32.argtypes = [P, i64, Fp, Fp, Fp, ci]
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleModel:
    """An oracle model built from the constructor arrays of a tree."""

    def __init__(self, parent, joint_type, axis, X_tree, inertia, gravity=(0.0, 0.0, -9.81)):
        lib = _load()
        self._lib = lib
        self.parent = np.ascontiguousarray(parent, dtype=np.int32)
        self.joint_type = np.ascontiguousarray(joint_type, dtype=np.int32)
        self.axis = _f64(axis)
        self.X_tree = _f64(X_tree)
        self.inertia = _f64(inertia)
        self.gravity = _f64(gravity)
        self.n = int(self.parent.shape[0])
        self._h = lib.orc_model_new(self.n, _i(self.parent), _i(self.joint_type), _d(self.axis),
                                    _d(self.X_tree), _d(self.inertia), _d(self.gravity))
        nq, nv = ctypes.c_int(), ctypes.c_int()
        lib.orc_dims(self._h, ctypes.byref(nq), ctypes.byref(nv))
        self.nq, self.nv = nq.value, nv.value

    @classmethod
    def from_tree(cls, tree):
        return cls(tree.parent, tree.joint_type, tree.axis, tree.X_tree, tree.inertia, tree.gravity)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_model_free(h)
            self._h = None

    def fk(self, q, threads=0):
        q = _f64(q, (-1, self.nq))
        out = np.empty((q.shape[0], self.n, 3, 4))
        self._lib.orc_fk(self._h, q.shape[0], _d(q), _d(out), threads)
        return out

    def jacobian(self, q, ee, frame=0, threads=0):
        q = _f64(q, (-1, self.nq))
        ee = np.ascontiguousarray(ee, dtype=np.int32)
        out = np.empty((q.shape[0], ee.shape[0], 6, self.nv))
        self._lib.orc_jacobian(self._h, q.shape[0], _d(q), int(ee.shape[0]), _i(ee), int(frame),
                               _d(out), threads)
        return out

    def rnea(self, q, qd, qdd, inertia=None, threads=0):
        q = _f64(q, (-1, self.nq))
        qd = _f64(qd, (-1, self.nv))
        qdd = _f64(qdd, (-1, self.nv))
        out = np.empty((q.shape[0], self.nv))
        pi = None if inertia is None else _f64(inertia, (self.n, 10))
        self._lib.orc_rnea(self._h, q.shape[0], _d(q), _d(qd), _d(qdd),
                           None if pi is None else _d(pi), _d(out), threads)
        return out

    def crba(self, q, inertia=None, threads=0):
        q = _f64(q, (-1, self.nq))
        out = np.empty((q.shape[0], self.nv, self.nv))
        if inertia is None:
            self._lib.orc_crba(self._h, q.shape[0], _d(q), _d(out), threads)
        else:
            pi = _f64(inertia, (self.n, 10))
            self._lib.orc_crba_pi(self._h, q.shape[0], _d(q), _d(pi), _d(out), threads)
        return out

    def aba(self, q, qd, tau, threads=0):
        q = _f64(q, (-1, self.nq))
        qd = _f64(qd, (-1, self.nv))
        tau = _f64(tau, (-1, self.nv))
        out = np.empty((q.shape[0], self.nv))
        self._lib.orc_aba(self._h, q.shape[0], _d(q), _d(qd), _d(tau), _d(out), threads)
        return out

    def chain(self, q, qd, qdd, ee, frame=0, threads=0):
        q = _f64(q, (-1, self.nq))
        qd = _f64(qd, (-1, self.nv))
        qdd = _f64(qdd, (-1, self.nv))
        ee = np.ascontiguousarray(ee, dtype=np.int32)
        B = q.shape[0]
        tau = np.empty((B, self.nv))
        M = np.empty((B, self.nv, self.nv))
        J = np.empty((B, ee.shape[0], 6, self.nv))
        self._lib.orc_chain(self._h, B, _d(q), _d(qd), _d(qdd), int(ee.shape[0]), _i(ee), int(frame),
                            _d(tau), _d(M), _d(J), threads)
        return tau, M, J

    def energy(self, q, qd, threads=0):
        q = _f64(q, (-1, self.nq))
        qd = _f64(qd, (-1, self.nv))
        ke = np.empty(q.shape[0])
        pe = np.empty(q.shape[0])
        self._lib.orc_energy(self._h, q.shape[0], _d(q), _d(qd), _d(ke), _d(pe), threads)
        return ke, pe

    def rnea_forces(self, q, qd, qdd, inertia=None, threads=0):
        """Spatial force transmitted across each joint, [B, n, 6] = [moment; force]
        in body coordinates about the body origin (tau is its projection on the
        joint's motion subspace)."""
        q = _f64(q, (-1, self.nq))
        qd = _f64(qd, (-1, self.nv))
        qdd = _f64(qdd, (-1, self.nv))
        B = q.shape[0]
        out = np.empty((B, self.n, 6))
        pi = None if inertia is None else _f64(inertia, (self.n, 10))
        self._lib.orc_rnea_forces(self._h, B, _d(q), _d(qd), _d(qdd), None if pi is None else _d(pi), _d(out),
                                  threads)
        return out

    def rnea_f32(self, q, qd, qdd, threads=0):
        """The RNEA recursion evaluated in single precision (inputs and parameters
        rounded to float); returns float64 [B, nv].  Used only to show what a plain
        single-precision evaluation attains."""
        f = lambda a, shape: np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(shape))
        q, qd, qdd = f(q, (-1, self.nq)), f(qd, (-1, self.nv)), f(qdd, (-1, self.nv))
        pi = f(self.inertia, (self.n, 10))
        out = np.empty((q.shape[0], self.nv), dtype=np.float32)
        fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._lib.orc_rnea_f32(self._h, q.shape[0], fp(q), fp(qd), fp(qdd), fp(pi), fp(out), threads)
        return out.astype(np.float64)

    def crba_f32(self, q, threads=0):
        """CRBA evaluated in single precision; float64 [B, nv, nv]."""
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float32).reshape(-1, self.nq))
        pi = np.ascontiguousarray(np.asarray(self.inertia, dtype=np.float32).reshape(self.n, 10))
        out = np.empty((q.shape[0], self.nv, self.nv), dtype=np.float32)
        fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._lib.orc_crba_f32(self._h, q.shape[0], fp(q), fp(pi), fp(out), threads)
        return out.astype(np.float64)

    def rnea_vjp(self, q, qd, qdd, tau_bar, inertia=None, threads=0):
        """Reverse-mode gradients; inertia_bar is per instance, shape [B, n, 10]."""
        q = _f64(q, (-1, self.nq))
        qd = _f64(qd, (-1, self.nv))
        qdd = _f64(qdd, (-1, self.nv))
        tb = _f64(tau_bar, (-1, self.nv))
        B = q.shape[0]
        qb = np.empty((B, self.nq))
        qdb = np.empty((B, self.nv))
        qddb = np.empty((B, self.nv))
        pib = np.empty((B, self.n, 10))
        pi = None if inertia is None else _f64(inertia, (self.n, 10))
        self._lib.orc_rnea_vjp(self._h, B, _d(q), _d(qd), _d(qdd), None if pi is None else _d(pi),
                               _d(tb), _d(qb), _d(qdb), _d(qddb), _d(pib), threads)
        return qb, qdb, qddb, pib

    def crba_vjp(self, q, M_bar, inertia=None, threads=0):
        """Reverse-mode gradients of <M_bar, M(q)>: (q_bar [B, nq], inertia_bar [B, n, 10])."""
        q = _f64(q, (-1, self.nq))
        mb = _f64(M_bar, (-1, self.nv * self.nv))
        B = q.shape[0]
        qb = np.empty((B, self.nq))
        pib = np.empty((B, self.n, 10))
        pi = None if inertia is None else _f64(inertia, (self.n, 10))
        self._lib.orc_crba_vjp(self._h, B, _d(q), None if pi is None else _d(pi), _d(mb), _d(qb), _d(pib), threads)
        return qb, pib

    def fk_vjp(self, q, poses_bar, threads=0):
        q = _f64(q, (-1, self.nq))
        pb = _f64(poses_bar, (-1, self.n, 3, 4))
        qb = np.empty((q.shape[0], self.nq))
        self._lib.orc_fk_vjp(self._h, q.shape[0], _d(q), _d(pb), _d(qb), threads)
        return qb
