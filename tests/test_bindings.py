"""CPU checks of the Python binding's argument guards: a host tensor, a tensor
of the wrong type or size, or a strided view is refused before its pointer
could reach the library (no GPU and no library call needed)."""
import os
import sys

import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2301_08911_amd.hmg import Batch, Context  # noqa: E402


class _NoLib:
    def __getattr__(self, name):
        def call(*args):
            raise AssertionError(f"library entry point {name} called with a refused argument")
        return call


def _context(n=64, dtype=torch.float32):
    c = Context.__new__(Context)
    c.lib, c._h = _NoLib(), None
    c.n, c.shape, c.field_dtype = n, (4, 4, 4), dtype
    c.device = torch.device("cuda", 0)
    return c


def _batch():
    b = Batch.__new__(Batch)
    b.lib, b._h = _NoLib(), None
    b.shapes = [(4, 4, 4)]
    b.device = torch.device("cuda", 0)
    return b


@pytest.mark.parametrize("call", [
    lambda c: c.set_density(torch.zeros(64)),
    lambda c: c.oc_update(torch.zeros(64), torch.zeros(64), 0.3),
    lambda c: c.filter(torch.zeros(64), out=torch.zeros(64)),
    lambda c: c.sensitivity(torch.eye(6).numpy(), out=torch.zeros(64)),
    lambda c: c.get_displacement(out=torch.zeros(6, 3, 64)),
])
def test_context_refuses_host_tensors(call):
    with pytest.raises(ValueError):
        call(_context())


def test_context_refuses_wrong_type_size_and_strides():
    c = _context()
    meta = torch.empty(128, device="meta")
    with pytest.raises(ValueError):
        c._scalar(meta[:64])                   # not on the context's device
    with pytest.raises(ValueError):
        c._scalar(torch.zeros(64, dtype=torch.float64))
    with pytest.raises(ValueError):
        c._scalar(torch.zeros(63))
    with pytest.raises(ValueError):
        c._scalar(torch.zeros(128)[::2])
    with pytest.raises(ValueError):
        c._field(torch.zeros(6, 3, 64, dtype=torch.float64))


def test_batch_refuses_host_tensors():
    with pytest.raises(ValueError):
        _batch().set_density(0, torch.zeros(64))
