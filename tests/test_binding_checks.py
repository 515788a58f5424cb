"""The binding's argument checks (no GPU needed).

The C ABI receives bare pointers and strides, so an array that is too short,
on the host, of another dtype or with a zero stride would be read or written
out of bounds by a kernel.  The binding rejects every such call with a
ValueError before the foreign call; these tests exercise each check with CPU
tensors (q itself on the host is the first check, so the others use a fake
device tensor that only answers the attribute queries the checks make).
"""

import numpy as np
import pytest
import torch

import synth
from paper_2605_31481_amd import bard


class FakeGpu:
    """Stand-in for a device tensor: shape, strides, dtype and device only.
    The checks raise before any pointer of it would be taken."""

    def __init__(self, shape, dtype=torch.float32, device="cuda:0", strides=None, contiguous=True):
        self.shape = tuple(shape)
        self.dtype = dtype
        self.device = torch.device(device)
        self.is_cuda = self.device.type == "cuda"
        self._strides = strides if strides is not None else (shape[1], 1)
        self._contig = contiguous

    def dim(self):
        return len(self.shape)

    def stride(self):
        return self._strides

    def numel(self):
        return int(np.prod(self.shape))

    def is_contiguous(self):
        return self._contig

    def data_ptr(self):  # never reached in these tests
        raise AssertionError("a pointer was taken before the checks rejected the call")


@pytest.fixture(scope="module")
def model():
    return bard.Model.from_tree(synth.quadruped_spine())


def test_host_q_is_rejected(model):
    q = torch.zeros(model.nq, 8)
    with pytest.raises(ValueError, match="GPU"):
        model.crba(q)


def test_short_and_mismatched_arrays_are_rejected(model):
    nq, nv, B = model.nq, model.nv, 8
    q = FakeGpu((nq, B))
    good = FakeGpu((nv, B))
    with pytest.raises(ValueError, match="batch"):
        model.rnea(q, FakeGpu((nv, B - 1)), good, out=FakeGpu((nv, B)))
    with pytest.raises(ValueError, match="expected"):
        model.rnea(q, good, FakeGpu((nv + 1, B)), out=FakeGpu((nv, B)))
    with pytest.raises(ValueError, match="dtype"):
        model.rnea(q, good, FakeGpu((nv, B), dtype=torch.float64), out=FakeGpu((nv, B)))
    with pytest.raises(ValueError, match="device"):
        model.rnea(q, good, FakeGpu((nv, B), device="cuda:1"), out=FakeGpu((nv, B)))
    with pytest.raises(ValueError, match="GPU"):
        model.rnea(q, good, FakeGpu((nv, B), device="cpu"), out=FakeGpu((nv, B)))
    with pytest.raises(ValueError, match="batch"):
        model.crba(q, out=FakeGpu((nv * nv, B - 3)))
    with pytest.raises(ValueError, match="expected"):
        model.fk(q, out=FakeGpu((12 * model.n_bodies - 1, B)))
    with pytest.raises(ValueError, match="zero stride"):
        model.aba(q, FakeGpu((nv, B), strides=(0, 1)), good, out=FakeGpu((nv, B)))


def test_chain_outputs_checked(model):
    nq, nv, B = model.nq, model.nv, 16
    q, v = FakeGpu((nq, B)), FakeGpu((nv, B))
    ee = [4, 6]
    tau, M = FakeGpu((nv, B)), FakeGpu((nv * nv, B))
    with pytest.raises(ValueError, match="expected"):
        model.chain(q, v, v, ee, out=(tau, M, FakeGpu((6 * nv * 1, B))))
    with pytest.raises(ValueError, match="batch"):
        model.chain(q, v, v, ee, out=(tau, FakeGpu((nv * nv, 2 * B)), FakeGpu((6 * nv * 2, B))))
    with pytest.raises(ValueError, match="batch"):
        model.bind_chain(q, v, v, ee, out=(FakeGpu((nv, 1)), M, FakeGpu((6 * nv * 2, B))))


def test_adjoint_inputs_checked(model):
    nq, nv, B = model.nq, model.nv, 8
    q, v = FakeGpu((nq, B)), FakeGpu((nv, B))
    with pytest.raises(ValueError, match="batch"):
        model.rnea_vjp(q, v, v, FakeGpu((nv, B + 1)))
    with pytest.raises(ValueError, match=r"\[11, 10\]"):
        model.rnea_vjp(q, v, v, v, inertia=FakeGpu((model.n_bodies - 1, 10)))
    with pytest.raises(ValueError, match="expected"):
        model.fk_vjp(q, FakeGpu((12, B)))
    with pytest.raises(ValueError, match="dtype"):
        model.aba_vjp(q, v, v, FakeGpu((nv, B), dtype=torch.float64))


def test_layout_name_checked(model):
    with pytest.raises(ValueError, match="layout"):
        model.crba(FakeGpu((8, model.nq)), layout="row")
