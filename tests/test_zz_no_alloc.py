"""The allocation-free convolution weight gradient against the workspace form.

hmg_conv3d_backward_weight_noalloc keeps its 64 partial sums per weight in the
library's fixed device array instead of a caller workspace; with the same
kernels and summation order it must reproduce hmg_conv3d_backward_weight.
Two calls in a row (the second smaller, so stale partials of the first stay
in the array) are compared, plus the size limit and argument errors.
"""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _inputs(B, Cin, Cout, D, seed):
    """bf16-representable operands, so the matrix cores round nothing."""
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(B, Cin, D, D, D, generator=g).to(torch.bfloat16).float().cuda()
    dz = torch.randn(B, Cout, D, D, D, generator=g).to(torch.bfloat16).float().cuda()
    return x, dz


@pytest.mark.parametrize("shapes", [[(2, 16, 32, 16), (1, 8, 16, 8)],
                                    [(1, 64, 64, 16), (3, 1, 8, 12)]])
def test_noalloc_matches_workspace_form(shapes):
    from paper_2301_08911_amd import nn
    for k, (B, Cin, Cout, D) in enumerate(shapes):
        x, dz = _inputs(B, Cin, Cout, D, 100 + k)
        dw0 = torch.full((Cout, Cin, 27), 0.25, device="cuda")
        db0 = torch.full((Cout,), -0.5, device="cuda")
        dw1, db1 = dw0.clone(), db0.clone()
        nn.conv3d_backward_weight(x, dz, dw0, db0)
        nn.conv3d_backward_weight_noalloc(x, dz, dw1, db1)
        torch.cuda.synchronize()
        a, b = dw0.cpu().numpy(), dw1.cpu().numpy()
        err = float(np.abs(a - b).max() / np.abs(a).max())
        print(f"call {k}: B {B} Cin {Cin} Cout {Cout} D {D}: max rel diff {err:.1e}", flush=True)
        assert err <= 1e-6, err
        assert np.array_equal(db0.cpu().numpy(), db1.cpu().numpy())
        # the gradient itself against the FP64 oracle of the convolution
        from oracle import nnref as N
        rw, rb = N.conv3d_backward_weight(x.double().cpu().numpy(), dz.double().cpu().numpy())
        assert np.abs((b - 0.25) - rw).max() < 1e-5 * np.abs(rw).max()
        assert np.abs((db1.cpu().numpy() + 0.5) - rb).max() < 1e-5 * np.abs(rb).max()


def test_noalloc_limit_and_arguments():
    from paper_2301_08911_amd import _lib
    lib = _lib.load()
    cap = lib.hmg_conv3d_noalloc_scratch_floats()
    assert cap == 8 << 20
    x = torch.zeros(1, 128, 4, 4, 4, device="cuda")
    dz = torch.zeros(1, 64, 4, 4, 4, device="cuda")
    dw = torch.zeros(64, 128, 27, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert lib.hmg_conv3d_workspace(1, 128, 64, 4, 4, 4) > cap
    assert lib.hmg_conv3d_backward_weight_noalloc(s, p(x), p(dz), p(dw), None, 1, 128, 64,
                                                  4, 4, 4) == 1
    assert lib.hmg_conv3d_backward_weight_noalloc(s, None, p(dz), p(dw), None, 1, 8, 8,
                                                  4, 4, 4) == 1
    assert lib.hmg_conv3d_backward_weight_noalloc(s, p(x), p(dz), p(dw), None, 0, 8, 8,
                                                  4, 4, 4) == 1
