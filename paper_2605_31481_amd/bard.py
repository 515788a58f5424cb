"""ctypes binding of libbard.so.

Argument marshalling only: every step of every operator runs in the HIP
kernels of ``libbard.so``.  Device tensors come from PyTorch, which is used for
device memory and the current stream.  If the library is missing this module
raises at import time; there is no CPU fallback.

Layouts.  ``layout="soa"`` (default) means instance-minor arrays of shape
``[K, B]`` (element k of instance b at ``[k, b]``), the layout the kernels
store fastest.  ``layout="aos"`` means ``[B, K]``.  Multi-index outputs are
flattened row-major per instance (e.g. ``M`` is ``nv*nv`` per instance), and
``as_batch_major`` turns any of them into a ``[B, ...]`` view without copying.
"""

from __future__ import annotations

import ctypes
import itertools
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbard.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "bard.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with paper_2605_31481_amd.build.build() "
        "(hipcc --offload-arch=gfx950).  There is no fallback implementation.")

# PyTorch ships its own HIP runtime with the same soname as the system one that
# libbard.so links against.  Loading torch first makes libbard.so bind to the
# runtime already in the process, so one runtime owns the device and streams.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

F32, F64 = 0, 1
REVOLUTE, PRISMATIC, FREE, FIXED = 0, 1, 2, 3
WORLD, LOCAL_WORLD_ALIGNED = 0, 1
E_CAPTURE = -8  # bard_status of a call that would allocate under graph capture
E_STATE = -9  # bard_status of a call that allocates nothing and found the model not uploaded
UPLOAD_ADJOINT = 1
SPEC_ROUTE, SPEC_COMPILE_ONLY, SPEC_WHOLE, SPEC_DUAL, SPEC_TRIPLE = 1, 2, 4, 8, 16
SPEC_FORMS = ("split", "whole", "dual", "triple")


def _spec_form_flag(form: str) -> int:
    if form not in SPEC_FORMS:
        raise ValueError(f"form must be one of {SPEC_FORMS}, got {form!r}")
    return {"split": 0, "whole": SPEC_WHOLE, "dual": SPEC_DUAL, "triple": SPEC_TRIPLE}[form]
# batch tiers of the specialised-kernel routing (lower bounds)
SPEC_TIERS = (0, 4096, 16384, 65536)
# workspace tiers (bard_ws_set_policy bits); TIER_RESULTS is the binding's own
# (see Workspace)
TIER_KINEMATICS, TIER_MASS, TIER_BIAS, TIER_RESULTS = 1, 2, 4, 8

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32


class Layout(ctypes.Structure):
    _fields_ = [("stride_b", ctypes.c_int64), ("stride_k", ctypes.c_int64)]


_LP = ctypes.POINTER(Layout)


def _sig(name, argtypes, restype=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = argtypes
    f.restype = restype
    return f


bard_status_str = _sig("bard_status_str", [ctypes.c_int], ctypes.c_char_p)
bard_last_error = _sig("bard_last_error", [], ctypes.c_char_p)
bard_version = _sig("bard_version", [], ctypes.c_char_p)
bard_model_create = _sig("bard_model_create", [_i32, _c_i32p, _c_i32p, _c_dp, _c_dp, _c_dp, ctypes.POINTER(_vp)])
bard_model_set_gravity = _sig("bard_model_set_gravity", [_vp, _c_dp])
bard_model_info = _sig("bard_model_info", [_vp, _c_i32p, _c_i32p, _c_i32p, _c_i32p])
bard_model_schedule = _sig("bard_model_schedule", [_vp, _c_i32p, _c_i32p])
bard_model_joint_transform = _sig("bard_model_joint_transform", [_vp, _i32, _c_dp, _c_dp, _c_dp])
bard_model_destroy = _sig("bard_model_destroy", [_vp])
bard_model_upload = _sig("bard_model_upload", [_vp, _i32, _c_i32p, _i32])
bard_model_specialize = _sig("bard_model_specialize", [_vp, ctypes.c_int, _i32, _c_i32p, ctypes.c_int, _i32])
bard_model_specialized_info = _sig("bard_model_specialized_info",
                                   [_vp, ctypes.c_int, _i32, _c_i32p, ctypes.c_int, _i32, _c_i32p, _c_i32p,
                                    ctypes.POINTER(ctypes.c_double), _c_i32p, _c_i32p])
bard_model_specialized_source = _sig("bard_model_specialized_source",
                                     [_vp, ctypes.c_int, _i32, _c_i32p, ctypes.c_int, _i32, ctypes.c_char_p, _i64,
                                      ctypes.POINTER(_i64)])
bard_model_specialize_aba = _sig("bard_model_specialize_aba", [_vp, ctypes.c_int, _i32])
bard_model_specialized_aba_info = _sig("bard_model_specialized_aba_info",
                                       [_vp, ctypes.c_int, _c_i32p, _c_i32p, ctypes.POINTER(ctypes.c_double), _c_i32p])
bard_aba_autotune = _sig("bard_aba_autotune", [_vp, ctypes.c_int, _vp, ctypes.POINTER(_i64)])
bard_model_specialized_aba_source = _sig("bard_model_specialized_aba_source",
                                         [_vp, ctypes.c_int, ctypes.c_char_p, _i64, ctypes.POINTER(_i64)])
bard_chain_autotune = _sig("bard_chain_autotune", [_vp, ctypes.c_int, _i32, _c_i32p, ctypes.c_int, _vp,
                                                   ctypes.POINTER(_i64)])
bard_ws_create = _sig("bard_ws_create", [_vp, ctypes.c_int, _i64, ctypes.POINTER(_vp)])
bard_ws_destroy = _sig("bard_ws_destroy", [_vp])
bard_ws_set_policy = _sig("bard_ws_set_policy", [_vp, _i32])
bard_ws_stats = _sig("bard_ws_stats", [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)])
bard_fk = _sig("bard_fk", [_vp, _vp, ctypes.c_int, _vp, _vp, _LP, _u64, _i64, _vp])
bard_jacobian = _sig("bard_jacobian", [_vp, _vp, ctypes.c_int, _vp, _i32, _c_i32p, ctypes.c_int, _vp, _LP, _u64,
                                       _i64, _vp])
bard_path_kinematics = _sig("bard_path_kinematics", [_vp, ctypes.c_int, _vp, _i32, ctypes.c_int, _vp, _vp, _LP,
                                                     _i64, _vp])
bard_rnea = _sig("bard_rnea", [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _LP, _u64, _u64, _i64, _vp])
bard_crba = _sig("bard_crba", [_vp, _vp, ctypes.c_int, _vp, _vp, _LP, _u64, _i64, _vp])
bard_aba = _sig("bard_aba", [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp, _LP, _u64, _u64, _i64, _vp])
bard_chain = _sig("bard_chain", [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _i32, _c_i32p, ctypes.c_int, _vp, _vp, _vp,
                                 _LP, _i64, _vp])
bard_rnea_vjp = _sig("bard_rnea_vjp", [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _LP, _i64,
                                       _vp])
bard_rnea_vjp_noalloc = _sig("bard_rnea_vjp_noalloc", [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                                       _vp, _LP, _i64, _vp])
bard_fk_vjp = _sig("bard_fk_vjp", [_vp, ctypes.c_int, _vp, _vp, _vp, _LP, _i64, _vp])
bard_crba_vjp = _sig("bard_crba_vjp", [_vp, ctypes.c_int, _vp, _vp, _vp, _LP, _i64, _vp])
bard_aba_vjp = _sig("bard_aba_vjp", [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _LP, _i64, _vp])
bard_plan_create = _sig("bard_plan_create", [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_i64), ctypes.c_uint32,
                                             ctypes.c_int, ctypes.POINTER(_vp)])
bard_plan_autotune = _sig("bard_plan_autotune", [_vp, _vp, _i32])
bard_plan_run = _sig("bard_plan_run", [_vp, ctypes.POINTER(_vp), _vp])
bard_plan_destroy = _sig("bard_plan_destroy", [_vp])
bard_plan_configure = _sig("bard_plan_configure", [_vp, _i32, _i32, _i32, _i32])
bard_plan_get_config = _sig("bard_plan_get_config", [_vp, _c_i32p, _c_i32p, _c_i32p, _c_i32p, _c_i32p])
bard_plan_ee = _sig("bard_plan_ee", [_vp, _i32, _c_i32p, _c_i32p])
bard_model_specialize_rnea = _sig("bard_model_specialize_rnea", [_vp, ctypes.c_int, _i32])
bard_model_specialized_rnea_info = _sig("bard_model_specialized_rnea_info",
                                        [_vp, ctypes.c_int, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
bard_model_specialized_rnea_source = _sig("bard_model_specialized_rnea_source",
                                          [_vp, ctypes.c_int, _i32, ctypes.c_char_p, _i64, ctypes.POINTER(_i64)])
bard_model_specialize_crba = _sig("bard_model_specialize_crba", [_vp, ctypes.c_int, _i32])
bard_model_specialized_crba_info = _sig("bard_model_specialized_crba_info",
                                        [_vp, ctypes.c_int, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
bard_model_specialized_crba_source = _sig("bard_model_specialized_crba_source",
                                          [_vp, ctypes.c_int, _i32, ctypes.c_char_p, _i64, ctypes.POINTER(_i64)])
bard_model_specialize_fk = _sig("bard_model_specialize_fk", [_vp, ctypes.c_int, _i32])
bard_model_specialized_fk_info = _sig("bard_model_specialized_fk_info",
                                      [_vp, ctypes.c_int, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
bard_model_specialized_fk_source = _sig("bard_model_specialized_fk_source",
                                        [_vp, ctypes.c_int, _i32, ctypes.c_char_p, _i64, ctypes.POINTER(_i64)])
bard_model_specialize_jacobian = _sig("bard_model_specialize_jacobian", [_vp, ctypes.c_int, _i32, _c_i32p,
                                                                         ctypes.c_int, _i32])
bard_model_specialized_jacobian_info = _sig("bard_model_specialized_jacobian_info",
                                            [_vp, ctypes.c_int, _i32, _c_i32p, ctypes.c_int, _i32,
                                             ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32),
                                             ctypes.POINTER(_i32)])
bard_model_specialized_jacobian_source = _sig("bard_model_specialized_jacobian_source",
                                              [_vp, ctypes.c_int, _i32, _c_i32p, ctypes.c_int, _i32,
                                               ctypes.c_char_p, _i64, ctypes.POINTER(_i64)])
bard_plan_specialized_info = _sig("bard_plan_specialized_info", [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                                                 ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                                                                 ctypes.POINTER(ctypes.c_double)])
bard_plan_specialized_source = _sig("bard_plan_specialized_source", [_vp, _i32, ctypes.c_char_p, _i64,
                                                                     ctypes.POINTER(_i64)])

PLAN_RNEA, PLAN_CRBA, PLAN_JACOBIAN = 1, 2, 4


def declared_symbols() -> list:
    """Names of every function declared in include/bard.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bard_[a-z0-9_]+)\s*\(", text)))


class BardError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = bard_status_str(status).decode()
        detail = bard_last_error().decode()
        super().__init__(f"{where}: {msg}: {detail}")


def _check(rc: int, where: str):
    if rc != 0:
        raise BardError(rc, where)


def _i32arr(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int32))
    return a, a.ctypes.data_as(_c_i32p)


def _f64arr(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return a, a.ctypes.data_as(_c_dp)


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}; use float32 or float64")


def _stream_ptr(t):
    torch = _torch()
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:  # the current stream's handle without building a Stream object
        return _vp(raw(t.device.index if t.device.index is not None else torch.cuda.current_device()))
    return _vp(torch.cuda.current_stream(t.device).cuda_stream)


def _batch_of(t, K: int, layout: str) -> int:
    if layout not in ("soa", "aos"):
        raise ValueError(f"layout must be 'soa' or 'aos', got {layout!r}")
    if t.dim() != 2:
        raise ValueError("operator arrays are 2-D: [K, B] (soa) or [B, K] (aos)")
    if layout == "soa":
        if t.shape[0] != K:
            raise ValueError(f"expected [{K}, B], got {tuple(t.shape)}")
        return int(t.shape[1])
    if t.shape[1] != K:
        raise ValueError(f"expected [B, {K}], got {tuple(t.shape)}")
    return int(t.shape[0])


def _on_gpu(t, name: str):
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a GPU tensor (the kernels read device memory), got device {t.device}")


def _check_arrays(q, arrays, B: int, layout: str):
    """Every array of a call: shape [K, B] (soa) or [B, K] (aos), the dtype of
    q and the GPU device of q.  The C ABI receives bare pointers and strides,
    so a short or misplaced array would be read or written out of bounds;
    these checks run before the foreign call.  ``arrays`` holds (tensor, K,
    name) triples; a None tensor is skipped."""
    _on_gpu(q, "q")
    _dtype_code(q)
    for t, K, name in arrays:
        if t is None:
            continue
        _on_gpu(t, name)
        if t.device != q.device:
            raise ValueError(f"{name} is on device {t.device}, q on device {q.device}")
        if t.dtype != q.dtype:
            raise ValueError(f"{name} has dtype {t.dtype}, q has {q.dtype}")
        if _batch_of(t, K, layout) != B:
            raise ValueError(f"{name}: batch {_batch_of(t, K, layout)} differs from q's batch {B}")
        if min(t.stride()) < 1 and t.numel() > 0:
            raise ValueError(f"{name} has a zero stride (an expanded view); pass a materialised tensor")


def _check_inertia(q, inertia, n_bodies: int, name: str = "inertia"):
    """A shared [n_bodies, 10] parameter tensor (override or gradient)."""
    if inertia is None:
        return
    _on_gpu(inertia, name)
    if inertia.device != q.device or inertia.dtype != q.dtype:
        raise ValueError(f"{name} must be on q's device with q's dtype")
    if tuple(inertia.shape) != (n_bodies, 10) or not inertia.is_contiguous():
        raise ValueError(f"{name} must be a contiguous [{n_bodies}, 10] tensor, got {tuple(inertia.shape)}")


def _layouts(tensors, layout: str):
    arr = (Layout * len(tensors))()
    for i, t in enumerate(tensors):
        if t is None:  # an absent optional array (its pointer is NULL)
            arr[i].stride_b = arr[i].stride_k = 1
        elif layout == "soa":
            arr[i].stride_k, arr[i].stride_b = t.stride(0), t.stride(1)
        else:
            arr[i].stride_b, arr[i].stride_k = t.stride(0), t.stride(1)
    return arr


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _new(ref, K: int, B: int, layout: str):
    torch = _torch()
    shape = (K, B) if layout == "soa" else (B, K)
    return torch.empty(shape, dtype=ref.dtype, device=ref.device)


def as_batch_major(t, *shape, layout: str = "soa"):
    """View an operator array as [B, *shape] without copying."""
    if layout == "soa":
        return t.t().unflatten(1, shape)
    return t.unflatten(1, shape)


_tag_ids = itertools.count(1)


def version_tag(t) -> int:
    """A non-zero tag that changes whenever ``t`` is modified in place: an id
    given to the tensor object on first use, combined with PyTorch's version
    counter.  A new tensor (even at a recycled address) gets a new id."""
    i = getattr(t, "_bard_tag_id", None)
    if i is None:
        i = next(_tag_ids)
        t._bard_tag_id = i
    return ((i & ((1 << 43) - 1)) << 20) | (t._version & 0xFFFFF)


class Workspace:
    """Cached state of one stream (bard_ws_*): operators called with ``ws=``
    reuse what was computed for unchanged inputs, per the tiers in ``policy``
    (an OR of TIER_KINEMATICS, TIER_MASS, TIER_BIAS, TIER_RESULTS).

    TIER_RESULTS is kept by the binding: an operator call with no ``out``
    whose inputs carry the same version tags as the previous call of that
    operator on this workspace (and whose other arguments are equal) returns
    the previous output tensor without any launch, provided that tensor has
    not been modified in place since (PyTorch's version counter).  This is the
    full hit of the lazy evaluation; the library itself cannot see whether a
    caller's output buffer still holds its result."""

    def __init__(self, model: "Model", max_batch: int, dtype=None, policy: int = TIER_KINEMATICS):
        torch = _torch()
        dtype = dtype if dtype is not None else torch.float32
        code = F32 if dtype == torch.float32 else F64
        h = _vp()
        _check(bard_ws_create(model.handle, code, int(max_batch), ctypes.byref(h)), "bard_ws_create")
        self._h = h
        self.model = model
        self._results = {}
        self.skipped = 0
        self.set_policy(policy)

    def set_policy(self, policy: int):
        self.reuse_results = bool(policy & TIER_RESULTS)
        self._results.clear()
        _check(bard_ws_set_policy(self._h, int(policy) & ~TIER_RESULTS), "bard_ws_set_policy")

    def stats(self) -> dict:
        """Tier decisions so far: hits and misses per library tier, and the
        binding's full hits (calls answered without a launch)."""
        h, m = (_u64 * 3)(), (_u64 * 3)()
        _check(bard_ws_stats(self._h, h, m), "bard_ws_stats")
        names = ("kinematics", "mass", "bias")
        out = {nm: {"hits": int(h[k]), "misses": int(m[k])} for k, nm in enumerate(names)}
        out["results"] = {"hits": self.skipped}
        return out

    def _lookup(self, op: str, key):
        if not self.reuse_results:
            return None
        ent = self._results.get(op)
        if ent is not None and ent[0] == key and all(t._version == v for t, v in zip(ent[1], ent[2])):
            self.skipped += 1
            return ent[1]
        return None

    def _remember(self, op: str, key, outs):
        if self.reuse_results:
            self._results[op] = (key, outs, tuple(t._version for t in outs))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            bard_ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _T:
    """A tensor argument of a result key: keyed by its explicit tag if the
    caller gave one, else by its version tag and address."""

    def __init__(self, t, tag=None):
        self.t, self.tag = t, tag

    def key(self):
        if self.t is None:
            return None
        if self.tag is not None:
            return ("tag", int(self.tag))
        return ("v", version_tag(self.t), self.t.data_ptr())


def _result_key(ws, out, q, q_tag, B, layout, *rest):
    """Key of a call for the binding's result tier, or None when the tier is
    not in use (no workspace, TIER_RESULTS off, or a caller-given output).
    ``rest`` holds _T tensor arguments and plain values."""
    if ws is None or not ws.reuse_results or out is not None:
        return None
    return (_T(q, q_tag).key(), B, layout, q.dtype) + tuple(r.key() if isinstance(r, _T) else r for r in rest)


def _ws_args(ws, q, q_tag):
    if ws is None:
        return None, 0
    return ws.handle, (int(q_tag) if q_tag is not None else version_tag(q))


class Model:
    """A compiled kinematic tree (see include/bard.h, bard_model_create)."""

    def __init__(self, parent, joint_type, axis, X_tree, inertia, gravity=None):
        self._parent, p_parent = _i32arr(parent)
        self._jtype, p_jt = _i32arr(joint_type)
        self._axis, p_axis = _f64arr(axis)
        self._xt, p_xt = _f64arr(X_tree)
        self._pi, p_pi = _f64arr(inertia)
        n = int(self._parent.shape[0])
        h = _vp()
        _check(bard_model_create(n, p_parent, p_jt, p_axis, p_xt, p_pi, ctypes.byref(h)), "bard_model_create")
        self._h = h
        if gravity is not None:
            g, pg = _f64arr(gravity)
            _check(bard_model_set_gravity(self._h, pg), "bard_model_set_gravity")
        nq, nv, nb, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(bard_model_info(self._h, ctypes.byref(nq), ctypes.byref(nv), ctypes.byref(nb), ctypes.byref(d)),
               "bard_model_info")
        self.nq, self.nv, self.n_bodies, self.depth = nq.value, nv.value, nb.value, d.value
        lanes, levels = ctypes.c_int32(), ctypes.c_int32()
        _check(bard_model_schedule(self._h, ctypes.byref(lanes), ctypes.byref(levels)), "bard_model_schedule")
        self.lanes_per_instance = lanes.value

    @classmethod
    def from_tree(cls, tree):
        return cls(tree.parent, tree.joint_type, tree.axis, tree.X_tree, tree.inertia,
                   getattr(tree, "gravity", None))

    def set_gravity(self, gravity):
        """World-frame gravity (bard_model_set_gravity); invalidates workspace bias tiers."""
        g, pg = _f64arr(gravity)
        _check(bard_model_set_gravity(self._h, pg), "bard_model_set_gravity")

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            bard_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload(self, ee: Optional[Sequence[int]] = None, adjoint: bool = False):
        """Upload the model's device tables (and an end-effector set's table,
        and the adjoint reduction buffer) to the current device now, so that
        later calls allocate nothing and can be captured (bard_model_upload)."""
        if ee is not None and len(ee) > 0:
            ee_a, pee = _i32arr(ee)
            n = len(ee_a)
        else:
            ee_a, pee, n = None, None, 0
        _check(bard_model_upload(self._h, n, pee, UPLOAD_ADJOINT if adjoint else 0), "bard_model_upload")

    def specialize(self, ee: Sequence[int], frame: int = WORLD, dtype=None, route: bool = True,
                   compile_only: bool = False, form: str = "split"):
        """Compile the model-specialised chain kernel for (dtype, ee, frame)
        with hipRTC and load it on the current device; with route=True,
        matching chain() calls use it at every batch (bard_model_specialize).
        form: "split" (waves by limbs), "whole" (one wave over the whole
        tree) or "dual" (split, torques and mass matrix + Jacobians in two
        workgroups)."""
        ee_a, pee = _i32arr(ee)
        flags = ((SPEC_ROUTE if route else 0) | (SPEC_COMPILE_ONLY if compile_only else 0) |
                 _spec_form_flag(form))
        _check(bard_model_specialize(self._h, self._dtype_arg(dtype), len(ee_a), pee, int(frame), flags),
               "bard_model_specialize")

    def autotune_chain(self, ee: Sequence[int], frame: int = WORLD, dtype=None) -> int:
        """Time the generic chain kernel and the specialised forms
        (bard_chain_autotune) and route each batch tier to the fastest;
        returns the smallest batch a specialised form takes (-1: none)."""
        torch = _torch()
        ee_a, pee = _i32arr(ee)
        mb = _i64()
        _check(bard_chain_autotune(self._h, self._dtype_arg(dtype), len(ee_a), pee, int(frame),
                                   _vp(torch.cuda.current_stream().cuda_stream), ctypes.byref(mb)),
               "bard_chain_autotune")
        return mb.value

    def specialized_info(self, ee: Sequence[int], frame: int = WORLD, dtype=None, form: str = "split") -> dict:
        ee_a, pee = _i32arr(ee)
        vg, sc, rt, nw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cs = ctypes.c_double()
        _check(bard_model_specialized_info(self._h, self._dtype_arg(dtype), len(ee_a), pee, int(frame),
                                           _spec_form_flag(form), ctypes.byref(vg), ctypes.byref(sc),
                                           ctypes.byref(cs), ctypes.byref(rt), ctypes.byref(nw)),
               "bard_model_specialized_info")
        return {"vgprs": vg.value, "scratch_bytes": sc.value, "compile_s": cs.value, "routed": bool(rt.value),
                "route_tiers": rt.value, "waves": nw.value}

    def specialized_source(self, ee: Sequence[int], frame: int = WORLD, dtype=None, form: str = "split") -> str:
        ee_a, pee = _i32arr(ee)
        fl = _spec_form_flag(form)
        n = _i64()
        _check(bard_model_specialized_source(self._h, self._dtype_arg(dtype), len(ee_a), pee, int(frame), fl, None,
                                             0, ctypes.byref(n)), "bard_model_specialized_source")
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(bard_model_specialized_source(self._h, self._dtype_arg(dtype), len(ee_a), pee, int(frame), fl, buf,
                                             n.value + 1, ctypes.byref(n)), "bard_model_specialized_source")
        return buf.value.decode()

    def specialize_aba(self, dtype=None, route: bool = True, compile_only: bool = False):
        """Compile the model-specialised forward-dynamics kernel with hipRTC
        and load it; with route=True, aba() calls use it at every batch."""
        flags = (SPEC_ROUTE if route else 0) | (SPEC_COMPILE_ONLY if compile_only else 0)
        _check(bard_model_specialize_aba(self._h, self._dtype_arg(dtype), flags), "bard_model_specialize_aba")

    def autotune_aba(self, dtype=None) -> int:
        """Time the generic and the specialised forward-dynamics kernels and
        route each batch tier to the faster (bard_aba_autotune)."""
        torch = _torch()
        mb = _i64()
        _check(bard_aba_autotune(self._h, self._dtype_arg(dtype), _vp(torch.cuda.current_stream().cuda_stream),
                                 ctypes.byref(mb)), "bard_aba_autotune")
        return mb.value

    def specialized_aba_info(self, dtype=None) -> dict:
        vg, sc, rt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cs = ctypes.c_double()
        _check(bard_model_specialized_aba_info(self._h, self._dtype_arg(dtype), ctypes.byref(vg), ctypes.byref(sc),
                                               ctypes.byref(cs), ctypes.byref(rt)), "bard_model_specialized_aba_info")
        return {"vgprs": vg.value, "scratch_bytes": sc.value, "compile_s": cs.value, "routed": bool(rt.value),
                "route_tiers": rt.value}

    def specialized_aba_source(self, dtype=None) -> str:
        n = _i64()
        _check(bard_model_specialized_aba_source(self._h, self._dtype_arg(dtype), None, 0, ctypes.byref(n)),
               "bard_model_specialized_aba_source")
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(bard_model_specialized_aba_source(self._h, self._dtype_arg(dtype), buf, n.value + 1, ctypes.byref(n)),
               "bard_model_specialized_aba_source")
        return buf.value.decode()

    _SPEC_OP_FNS = {"rnea": ("bard_model_specialize_rnea", "bard_model_specialized_rnea_info",
                             "bard_model_specialized_rnea_source"),
                    "crba": ("bard_model_specialize_crba", "bard_model_specialized_crba_info",
                             "bard_model_specialized_crba_source"),
                    "jacobian": ("bard_model_specialize_jacobian", "bard_model_specialized_jacobian_info",
                                 "bard_model_specialized_jacobian_source"),
                    "fk": ("bard_model_specialize_fk", "bard_model_specialized_fk_info",
                           "bard_model_specialized_fk_source")}

    def _spec_op_fns(self, op: str):
        if op not in self._SPEC_OP_FNS:
            raise ValueError("op must be 'fk', 'rnea', 'crba' or 'jacobian'")
        g = globals()
        return tuple(g[n] for n in self._SPEC_OP_FNS[op])

    def _spec_op_pre(self, op: str, dtype, ee, frame):
        """Leading arguments of the op's C calls (the Jacobian's take its end
        effectors and frame)."""
        if op != "jacobian":
            return (self._h, self._dtype_arg(dtype)), ()
        if ee is None:
            raise ValueError("the Jacobian kernel needs ee")
        ee_a, pee = _i32arr(ee)
        return (self._h, self._dtype_arg(dtype), len(ee_a), pee, int(frame)), (ee_a,)

    def specialize_op(self, op: str, dtype=None, route: bool = True, compile_only: bool = False,
                      form: str = "split", ee: Optional[Sequence[int]] = None, frame: int = WORLD):
        """Compile the model-specialised kernel of one operator ("fk",
        "rnea", "crba" or "jacobian" with its end effectors ``ee`` and ``frame``;
        form "split" or "whole") with hipRTC and load it; with route=True,
        that operator's calls without a workspace (and, for rnea, without an
        inertia override; for the Jacobian, with the same ee and frame) use
        it at every batch."""
        if form not in ("split", "whole"):
            raise ValueError("form must be 'split' or 'whole'")
        flags = ((SPEC_ROUTE if route else 0) | (SPEC_COMPILE_ONLY if compile_only else 0) |
                 (SPEC_WHOLE if form == "whole" else 0))
        fn, _, _ = self._spec_op_fns(op)
        pre, keep = self._spec_op_pre(op, dtype, ee, frame)
        _check(fn(*pre, flags), fn.__name__)

    def specialized_op_info(self, op: str, dtype=None, form: str = "split", ee: Optional[Sequence[int]] = None,
                            frame: int = WORLD) -> dict:
        _, fn, _ = self._spec_op_fns(op)
        pre, keep = self._spec_op_pre(op, dtype, ee, frame)
        vg, sc, rt, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cs = ctypes.c_double()
        _check(fn(*pre, SPEC_WHOLE if form == "whole" else 0, ctypes.byref(vg), ctypes.byref(sc), ctypes.byref(cs),
                  ctypes.byref(rt), ctypes.byref(w)), fn.__name__)
        return {"vgprs": vg.value, "scratch_bytes": sc.value, "compile_s": cs.value, "routed": bool(rt.value),
                "route_tiers": rt.value, "waves": w.value}

    def specialized_op_source(self, op: str, dtype=None, form: str = "split", ee: Optional[Sequence[int]] = None,
                              frame: int = WORLD) -> str:
        _, _, fn = self._spec_op_fns(op)
        pre, keep = self._spec_op_pre(op, dtype, ee, frame)
        flags = SPEC_WHOLE if form == "whole" else 0
        n = _i64()
        _check(fn(*pre, flags, None, 0, ctypes.byref(n)), fn.__name__)
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(fn(*pre, flags, buf, n.value + 1, ctypes.byref(n)), fn.__name__)
        return buf.value.decode()

    def specialize_rnea(self, dtype=None, route: bool = True, compile_only: bool = False, form: str = "split"):
        self.specialize_op("rnea", dtype, route, compile_only, form)

    def specialized_rnea_info(self, dtype=None, form: str = "split") -> dict:
        return self.specialized_op_info("rnea", dtype, form)

    def specialized_rnea_source(self, dtype=None, form: str = "split") -> str:
        return self.specialized_op_source("rnea", dtype, form)

    @staticmethod
    def _dtype_arg(dtype) -> int:
        if dtype is None:
            return F32
        if isinstance(dtype, int):
            return dtype
        name = str(dtype)
        if name.endswith("float32"):
            return F32
        if name.endswith("float64"):
            return F64
        raise ValueError(f"dtype must be float32 or float64, got {dtype}")

    def joint_transform(self, body: int, q):
        qa, pq = _f64arr(q)
        R = np.zeros(9)
        t = np.zeros(3)
        _check(bard_model_joint_transform(self._h, int(body), pq, R.ctypes.data_as(_c_dp), t.ctypes.data_as(_c_dp)),
               "bard_model_joint_transform")
        return R.reshape(3, 3), t

    # ---------------------------------------------------------------- ops --
    def fk(self, q, out=None, layout: str = "soa", ws: Optional[Workspace] = None, q_tag=None):
        B = _batch_of(q, self.nq, layout)
        key = _result_key(ws, out, q, q_tag, B, layout)
        if key is not None and (hit := ws._lookup("fk", key)) is not None:
            return hit[0]
        out = out if out is not None else _new(q, 12 * self.n_bodies, B, layout)
        _check_arrays(q, [(out, 12 * self.n_bodies, "out")], B, layout)
        L = _layouts([q, out], layout)
        wh, tag = _ws_args(ws, q, q_tag)
        _check(bard_fk(self._h, wh, _dtype_code(q), _ptr(q), _ptr(out), L, tag, B, _stream_ptr(q)), "bard_fk")
        if key is not None:
            ws._remember("fk", key, (out,))
        return out

    def jacobian(self, q, ee: Sequence[int], frame: int = WORLD, out=None, layout: str = "soa",
                 ws: Optional[Workspace] = None, q_tag=None):
        B = _batch_of(q, self.nq, layout)
        ee_a, pee = _i32arr(ee)
        key = _result_key(ws, out, q, q_tag, B, layout, tuple(int(e) for e in ee_a), int(frame))
        if key is not None and (hit := ws._lookup("jacobian", key)) is not None:
            return hit[0]
        out = out if out is not None else _new(q, 6 * self.nv * len(ee_a), B, layout)
        _check_arrays(q, [(out, 6 * self.nv * len(ee_a), "out")], B, layout)
        L = _layouts([q, out], layout)
        wh, tag = _ws_args(ws, q, q_tag)
        _check(bard_jacobian(self._h, wh, _dtype_code(q), _ptr(q), len(ee_a), pee, int(frame), _ptr(out), L, tag, B,
                             _stream_ptr(q)), "bard_jacobian")
        if key is not None:
            ws._remember("jacobian", key, (out,))
        return out

    def path_kinematics(self, q, ee: int, frame: int = WORLD, pose: bool = True, jacobian: bool = True,
                        out_pose=None, out_J=None, layout: str = "soa"):
        """Pose [12] and Jacobian [6*nv] of one end effector from a walk of
        its root-to-body path only (bard_path_kinematics).  Returns
        (pose, J), None for an output not asked for."""
        B = _batch_of(q, self.nq, layout)
        if not (pose or jacobian):
            raise ValueError("path_kinematics needs pose or jacobian")
        po = (out_pose if out_pose is not None else _new(q, 12, B, layout)) if pose else None
        J = (out_J if out_J is not None else _new(q, 6 * self.nv, B, layout)) if jacobian else None
        _check_arrays(q, [(po, 12, "out_pose"), (J, 6 * self.nv, "out_J")], B, layout)
        L = _layouts([q, po, J], layout)
        _check(bard_path_kinematics(self._h, _dtype_code(q), _ptr(q), int(ee), int(frame), _ptr(po), _ptr(J), L, B,
                                    _stream_ptr(q)), "bard_path_kinematics")
        return po, J

    def rnea(self, q, qd, qdd, inertia=None, out=None, layout: str = "soa", ws: Optional[Workspace] = None,
             q_tag=None, qd_tag=None):
        B = _batch_of(q, self.nq, layout)
        key = _result_key(ws, out, q, q_tag, B, layout, _T(qd, qd_tag), _T(qdd), _T(inertia))
        if key is not None and (hit := ws._lookup("rnea", key)) is not None:
            return hit[0]
        out = out if out is not None else _new(q, self.nv, B, layout)
        _check_arrays(q, [(qd, self.nv, "qd"), (qdd, self.nv, "qdd"), (out, self.nv, "out")], B, layout)
        _check_inertia(q, inertia, self.n_bodies)
        L = _layouts([q, qd, qdd, out], layout)
        wh, tag = _ws_args(ws, q, q_tag)
        _, dtag = _ws_args(ws, qd, qd_tag)
        _check(bard_rnea(self._h, wh, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(qdd), _ptr(inertia), _ptr(out), L,
                         tag, dtag, B, _stream_ptr(q)), "bard_rnea")
        if key is not None:
            ws._remember("rnea", key, (out,))
        return out

    def crba(self, q, out=None, layout: str = "soa", ws: Optional[Workspace] = None, q_tag=None):
        B = _batch_of(q, self.nq, layout)
        key = _result_key(ws, out, q, q_tag, B, layout)
        if key is not None and (hit := ws._lookup("crba", key)) is not None:
            return hit[0]
        out = out if out is not None else _new(q, self.nv * self.nv, B, layout)
        _check_arrays(q, [(out, self.nv * self.nv, "out")], B, layout)
        L = _layouts([q, out], layout)
        wh, tag = _ws_args(ws, q, q_tag)
        _check(bard_crba(self._h, wh, _dtype_code(q), _ptr(q), _ptr(out), L, tag, B, _stream_ptr(q)), "bard_crba")
        if key is not None:
            ws._remember("crba", key, (out,))
        return out

    def aba(self, q, qd, tau, out=None, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        out = out if out is not None else _new(q, self.nv, B, layout)
        _check_arrays(q, [(qd, self.nv, "qd"), (tau, self.nv, "tau"), (out, self.nv, "out")], B, layout)
        L = _layouts([q, qd, tau, out], layout)
        _check(bard_aba(self._h, None, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(tau), _ptr(out), L, 0, 0, B,
                        _stream_ptr(q)), "bard_aba")
        return out

    def chain(self, q, qd, qdd, ee: Sequence[int], frame: int = WORLD, out=None, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        ee_a, pee = _i32arr(ee)
        if out is None:
            out = (_new(q, self.nv, B, layout), _new(q, self.nv * self.nv, B, layout),
                   _new(q, 6 * self.nv * len(ee_a), B, layout))
        tau, M, J = out
        _check_arrays(q, [(qd, self.nv, "qd"), (qdd, self.nv, "qdd"), (tau, self.nv, "tau"),
                          (M, self.nv * self.nv, "M"), (J, 6 * self.nv * len(ee_a), "J")], B, layout)
        L = _layouts([q, qd, qdd, tau, M, J], layout)
        _check(bard_chain(self._h, None, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(qdd), len(ee_a), pee, int(frame),
                          _ptr(tau), _ptr(M), _ptr(J), L, B, _stream_ptr(q)), "bard_chain")
        return tau, M, J

    # ----------------------------------------------------------- adjoints --
    def rnea_vjp(self, q, qd, qdd, tau_bar, inertia=None, inertia_grad: bool = True, layout: str = "soa"):
        """Reverse-mode product of RNEA: returns (q_bar, qd_bar, qdd_bar,
        inertia_bar) for the cotangent tau_bar; inertia_bar is [n_bodies, 10],
        summed over the batch (None if inertia_grad is False)."""
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(qd, self.nv, "qd"), (qdd, self.nv, "qdd"), (tau_bar, self.nv, "tau_bar")], B, layout)
        _check_inertia(q, inertia, self.n_bodies)
        qb = _new(q, self.nq, B, layout)
        qdb = _new(q, self.nv, B, layout)
        qddb = _new(q, self.nv, B, layout)
        pib = None
        if inertia_grad:
            torch = _torch()
            alloc = torch.zeros if B == 0 else torch.empty  # the sum over an empty batch
            pib = alloc((self.n_bodies, 10), dtype=q.dtype, device=q.device)
        L = _layouts([q, qd, qdd, tau_bar, qb, qdb, qddb], layout)
        _check(bard_rnea_vjp(self._h, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(qdd), _ptr(inertia), _ptr(tau_bar),
                             _ptr(qb), _ptr(qdb), _ptr(qddb), _ptr(pib), L, B, _stream_ptr(q)), "bard_rnea_vjp")
        return qb, qdb, qddb, pib

    def rnea_vjp_noalloc(self, q, qd, qdd, tau_bar, out, inertia=None, layout: str = "soa"):
        """rnea_vjp into caller-provided outputs out = (q_bar, qd_bar, qdd_bar,
        inertia_bar or None) through bard_rnea_vjp_noalloc, which allocates
        nothing (the model must already be on the device: see upload())."""
        B = _batch_of(q, self.nq, layout)
        qb, qdb, qddb, pib = out
        _check_arrays(q, [(qd, self.nv, "qd"), (qdd, self.nv, "qdd"), (tau_bar, self.nv, "tau_bar"),
                          (qb, self.nq, "q_bar"), (qdb, self.nv, "qd_bar"), (qddb, self.nv, "qdd_bar")], B, layout)
        _check_inertia(q, inertia, self.n_bodies)
        _check_inertia(q, pib, self.n_bodies, "inertia_bar")
        L = _layouts([q, qd, qdd, tau_bar, qb, qdb, qddb], layout)
        _check(bard_rnea_vjp_noalloc(self._h, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(qdd), _ptr(inertia),
                                     _ptr(tau_bar), _ptr(qb), _ptr(qdb), _ptr(qddb), _ptr(pib), L, B, _stream_ptr(q)),
               "bard_rnea_vjp_noalloc")
        return qb, qdb, qddb, pib

    def aba_vjp(self, q, qd, qdd, qdd_bar, layout: str = "soa"):
        """Reverse-mode product of forward dynamics (bard_aba_vjp): returns
        (q_bar, qd_bar, tau_bar) for the cotangent qdd_bar; qdd is the
        forward-dynamics result for (q, qd, tau)."""
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(qd, self.nv, "qd"), (qdd, self.nv, "qdd"), (qdd_bar, self.nv, "qdd_bar")], B, layout)
        qb = _new(q, self.nq, B, layout)
        qdb = _new(q, self.nv, B, layout)
        tb = _new(q, self.nv, B, layout)
        L = _layouts([q, qd, qdd, qdd_bar, qb, qdb, tb], layout)
        _check(bard_aba_vjp(self._h, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(qdd), _ptr(qdd_bar), _ptr(qb),
                            _ptr(qdb), _ptr(tb), L, B, _stream_ptr(q)), "bard_aba_vjp")
        return qb, qdb, tb

    def crba_vjp(self, q, M_bar, layout: str = "soa"):
        """Reverse-mode product of CRBA: q_bar = d<M_bar, M(q)>/dq for the
        cotangent M_bar (per instance nv*nv, row-major)."""
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(M_bar, self.nv * self.nv, "M_bar")], B, layout)
        qb = _new(q, self.nq, B, layout)
        L = _layouts([q, M_bar, qb], layout)
        _check(bard_crba_vjp(self._h, _dtype_code(q), _ptr(q), _ptr(M_bar), _ptr(qb), L, B, _stream_ptr(q)),
               "bard_crba_vjp")
        return qb

    def fk_vjp(self, q, poses_bar, layout: str = "soa"):
        """Reverse-mode product of FK: q_bar for the cotangent poses_bar (per
        body 3x4 row-major [R | p])."""
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(poses_bar, 12 * self.n_bodies, "poses_bar")], B, layout)
        qb = _new(q, self.nq, B, layout)
        L = _layouts([q, poses_bar, qb], layout)
        _check(bard_fk_vjp(self._h, _dtype_code(q), _ptr(q), _ptr(poses_bar), _ptr(qb), L, B, _stream_ptr(q)),
               "bard_fk_vjp")
        return qb

    # ------------------------------------------------------- bound calls --
    def bind_chain(self, q, qd, qdd, ee: Sequence[int], out, frame: int = WORLD, layout: str = "soa"):
        """Marshal the arguments of one chain call once; the returned callable
        only issues the foreign call (on the stream current at bind time)."""
        B = _batch_of(q, self.nq, layout)
        ee_a, pee = _i32arr(ee)
        tau, M, J = out
        _check_arrays(q, [(qd, self.nv, "qd"), (qdd, self.nv, "qdd"), (tau, self.nv, "tau"),
                          (M, self.nv * self.nv, "M"), (J, 6 * self.nv * len(ee_a), "J")], B, layout)
        L = _layouts([q, qd, qdd, tau, M, J], layout)
        args = (self._h, None, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(qdd), len(ee_a), pee, int(frame), _ptr(tau),
                _ptr(M), _ptr(J), L, B, _stream_ptr(q))
        keep = (ee_a, L, q, qd, qdd, tau, M, J)

        def call():
            rc = bard_chain(*args)
            if rc:
                raise BardError(rc, "bard_chain")
            return keep
        return call

    def bind_fk(self, q, out, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(out, 12 * self.n_bodies, "out")], B, layout)
        L = _layouts([q, out], layout)
        args = (self._h, None, _dtype_code(q), _ptr(q), _ptr(out), L, 0, B, _stream_ptr(q))
        keep = (L, q, out)

        def call():
            rc = bard_fk(*args)
            if rc:
                raise BardError(rc, "bard_fk")
            return keep
        return call

    def bind_aba(self, q, qd, tau, out, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(qd, self.nv, "qd"), (tau, self.nv, "tau"), (out, self.nv, "out")], B, layout)
        L = _layouts([q, qd, tau, out], layout)
        args = (self._h, None, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(tau), _ptr(out), L, 0, 0, B, _stream_ptr(q))
        keep = (L, q, qd, tau, out)

        def call():
            rc = bard_aba(*args)
            if rc:
                raise BardError(rc, "bard_aba")
            return keep
        return call

    def bind_rnea(self, q, qd, qdd, out, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(qd, self.nv, "qd"), (qdd, self.nv, "qdd"), (out, self.nv, "out")], B, layout)
        L = _layouts([q, qd, qdd, out], layout)
        args = (self._h, None, _dtype_code(q), _ptr(q), _ptr(qd), _ptr(qdd), _vp(0), _ptr(out), L, 0, 0, B,
                _stream_ptr(q))
        keep = (L, q, qd, qdd, out)

        def call():
            rc = bard_rnea(*args)
            if rc:
                raise BardError(rc, "bard_rnea")
            return keep
        return call

    def bind_crba(self, q, out, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(out, self.nv * self.nv, "out")], B, layout)
        L = _layouts([q, out], layout)
        args = (self._h, None, _dtype_code(q), _ptr(q), _ptr(out), L, 0, B, _stream_ptr(q))
        keep = (L, q, out)

        def call():
            rc = bard_crba(*args)
            if rc:
                raise BardError(rc, "bard_crba")
            return keep
        return call

    def bind_path_kinematics(self, q, ee: int, out_pose, out_J, frame: int = WORLD, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        _check_arrays(q, [(out_pose, 12, "out_pose"), (out_J, 6 * self.nv, "out_J")], B, layout)
        if out_pose is None and out_J is None:
            raise ValueError("path_kinematics needs an output")
        L = _layouts([q, out_pose, out_J], layout)
        args = (self._h, _dtype_code(q), _ptr(q), int(ee), int(frame), _ptr(out_pose), _ptr(out_J), L, B,
                _stream_ptr(q))
        keep = (L, q, out_pose, out_J)

        def call():
            rc = bard_path_kinematics(*args)
            if rc:
                raise BardError(rc, "bard_path_kinematics")
            return keep
        return call

    def bind_jacobian(self, q, ee: Sequence[int], out, frame: int = WORLD, layout: str = "soa"):
        B = _batch_of(q, self.nq, layout)
        ee_a, pee = _i32arr(ee)
        _check_arrays(q, [(out, 6 * self.nv * len(ee_a), "out")], B, layout)
        L = _layouts([q, out], layout)
        args = (self._h, None, _dtype_code(q), _ptr(q), len(ee_a), pee, int(frame), _ptr(out), L, 0, B,
                _stream_ptr(q))
        keep = (ee_a, L, q, out)

        def call():
            rc = bard_jacobian(*args)
            if rc:
                raise BardError(rc, "bard_jacobian")
            return keep
        return call



class Plan:
    """Several models with their own batch sizes in one launch (bard_plan_*).

    ``run(inputs)`` takes per model a tuple (q, qd, qdd) of instance-minor
    tensors and returns per model (tau, M, J) (entries the op mask does not
    produce are None).  Output tensors are allocated once per plan and reused
    by every run, so the replayed graph keeps writing to the same memory.
    ``configure(tile, fusion, order, lanes)``: fusion 0 one generic launch,
    1 one per model, 2 one per operator, 3 one generated kernel holding every
    tree's specialised code (lanes 1: each tree over at most 4 waves);
    ``autotune`` times them all and keeps the fastest.
    """

    def __init__(self, models: Sequence[Model], batches: Sequence[int], op_mask: int = 7, dtype=None):
        torch = _torch()
        self.models = list(models)
        self.batches = [int(b) for b in batches]
        self.op_mask = int(op_mask)
        self.dtype = dtype if dtype is not None else torch.float32
        code = F32 if self.dtype == torch.float32 else F64
        hs = (_vp * len(self.models))(*[m.handle for m in self.models])
        bs = (_i64 * len(self.batches))(*self.batches)
        h = _vp()
        _check(bard_plan_create(hs, len(self.models), bs, self.op_mask, code, ctypes.byref(h)), "bard_plan_create")
        self._h = h
        self._outs = None

    def close(self):
        if getattr(self, "_h", None):
            bard_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def specialized_info(self) -> dict:
        """Resources of the plan's generated multi-tree kernel (built by its
        first run in fusion 3)."""
        r, sc, w = _i32(), _i32(), _i32()
        g, c = _i64(), ctypes.c_double()
        _check(bard_plan_specialized_info(self._h, ctypes.byref(r), ctypes.byref(sc), ctypes.byref(w), ctypes.byref(g),
                                          ctypes.byref(c)), "bard_plan_specialized_info")
        return {"vgprs": r.value, "scratch_bytes": sc.value, "waves": w.value, "workgroups": g.value,
                "compile_s": c.value}

    def specialized_source(self, compile_only: bool = False) -> str:
        """Source of the plan's generated multi-tree kernel (fusion 3);
        compile_only also compiles it for gfx950 with hipRTC."""
        n = _i64()
        _check(bard_plan_specialized_source(self._h, 0, None, 0, ctypes.byref(n)), "bard_plan_specialized_source")
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(bard_plan_specialized_source(self._h, int(compile_only), buf, n.value + 1, ctypes.byref(n)),
               "bard_plan_specialized_source")
        return buf.value.decode()

    def ee(self, i: int) -> list:
        n = ctypes.c_int32()
        buf = (ctypes.c_int32 * 4)()
        _check(bard_plan_ee(self._h, int(i), ctypes.byref(n), buf), "bard_plan_ee")
        return list(buf[:n.value])

    def configure(self, tile: int, fusion: int, order: int = 0, lanes: int = 0):
        _check(bard_plan_configure(self._h, int(tile), int(fusion), int(order), int(lanes)), "bard_plan_configure")

    @property
    def config(self) -> dict:
        t, f, o, ln, c = (ctypes.c_int32() for _ in range(5))
        _check(bard_plan_get_config(self._h, ctypes.byref(t), ctypes.byref(f), ctypes.byref(o), ctypes.byref(ln),
                                    ctypes.byref(c)), "bard_plan_get_config")
        return {"tile": t.value, "fusion": f.value, "order": o.value, "lanes": ln.value, "from_cache": bool(c.value)}

    def autotune(self, budget_ms: int = 2000):
        torch = _torch()
        _check(bard_plan_autotune(self._h, _vp(torch.cuda.current_stream().cuda_stream), int(budget_ms)),
               "bard_plan_autotune")

    def _outputs(self, device):
        torch = _torch()
        if self._outs is None:
            outs = []
            for i, (m, B) in enumerate(zip(self.models, self.batches)):
                ne = len(self.ee(i))
                mk = lambda k: torch.empty((k, B), dtype=self.dtype, device=device)
                outs.append((mk(m.nv) if self.op_mask & 1 else None,
                             mk(m.nv * m.nv) if self.op_mask & 2 else None,
                             mk(6 * m.nv * ne) if self.op_mask & 4 else None))
            self._outs = outs
        return self._outs

    def run(self, inputs, stream=None):
        torch = _torch()
        if len(inputs) != len(self.models):
            raise ValueError("one (q, qd, qdd) tuple per model")
        dev = inputs[0][0].device
        if getattr(self, "_device", None) is None:
            self._device = dev
        for tup in inputs:
            for t in tup:
                if t is not None:
                    _on_gpu(t, "plan input")
                    if t.device != self._device:
                        raise ValueError(f"plan inputs must all be on {self._device}, got {t.device}")
        outs = self._outputs(dev)
        ptrs = []
        for (q, qd, qdd), (tau, M, J), m, B in zip(inputs, outs, self.models, self.batches):
            for t, K in ((q, m.nq), (qd, m.nv), (qdd, m.nv)):
                if t is not None and (tuple(t.shape) != (K, B) or not t.is_contiguous() or t.dtype != self.dtype):
                    raise ValueError(f"plan inputs must be contiguous [{K}, {B}] tensors of {self.dtype}")
            ptrs += [t.data_ptr() if t is not None else 0 for t in (q, qd, qdd, tau, M, J)]
        io = (_vp * len(ptrs))(*ptrs)
        st = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        _check(bard_plan_run(self._h, io, _vp(st)), "bard_plan_run")
        return outs

# ------------------------------------------------------------------ autograd --
class _RneaFn(torch.autograd.Function):
    """tau = RNEA(q, qd, qdd; inertia) with gradients for q, qd, qdd and the
    [n_bodies, 10] inertial parameters (summed over the batch)."""

    @staticmethod
    def forward(ctx, model, q, qd, qdd, inertia):
        ctx.model = model
        ctx.save_for_backward(q, qd, qdd, inertia)
        return model.rnea(q, qd, qdd, inertia=inertia)

    @staticmethod
    def backward(ctx, tau_bar):
        q, qd, qdd, inertia = ctx.saved_tensors
        want_pi = inertia is not None and ctx.needs_input_grad[4]
        qb, qdb, qddb, pib = ctx.model.rnea_vjp(q, qd, qdd, tau_bar.contiguous(), inertia=inertia,
                                                inertia_grad=want_pi)
        return None, qb, qdb, qddb, pib


class _FkFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, q):
        ctx.model = model
        ctx.save_for_backward(q)
        return model.fk(q)

    @staticmethod
    def backward(ctx, poses_bar):
        (q,) = ctx.saved_tensors
        return None, ctx.model.fk_vjp(q, poses_bar.contiguous())


class _CrbaFn(torch.autograd.Function):
    """M = CRBA(q) ([nv*nv, B]) with the gradient for q."""

    @staticmethod
    def forward(ctx, model, q):
        ctx.model = model
        ctx.save_for_backward(q)
        return model.crba(q)

    @staticmethod
    def backward(ctx, M_bar):
        (q,) = ctx.saved_tensors
        return None, ctx.model.crba_vjp(q, M_bar.contiguous())


class _AbaFn(torch.autograd.Function):
    """qdd = ABA(q, qd, tau) with gradients for q, qd and tau."""

    @staticmethod
    def forward(ctx, model, q, qd, tau):
        ctx.model = model
        qdd = model.aba(q, qd, tau)
        ctx.save_for_backward(q, qd, qdd)
        return qdd

    @staticmethod
    def backward(ctx, qdd_bar):
        q, qd, qdd = ctx.saved_tensors
        qb, qdb, tb = ctx.model.aba_vjp(q, qd, qdd, qdd_bar.contiguous())
        return None, qb, qdb, tb


def aba(model: Model, q, qd, tau):
    """Differentiable forward dynamics on [K, B] (instance-minor) tensors."""
    return _AbaFn.apply(model, q, qd, tau)


def rnea(model: Model, q, qd, qdd, inertia=None):
    """Differentiable inverse dynamics on [K, B] (instance-minor) tensors."""
    return _RneaFn.apply(model, q, qd, qdd, inertia)


def crba(model: Model, q):
    """Differentiable mass matrix on [nq, B] tensors; returns [nv*nv, B]."""
    return _CrbaFn.apply(model, q)


def fk(model: Model, q):
    """Differentiable forward kinematics on [nq, B] tensors; returns [12 n_bodies, B]."""
    return _FkFn.apply(model, q)
