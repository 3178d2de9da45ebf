"""GPU parity of the design-space kernels against the FP64 oracle
(oracle/design.py), through the C ABI:

* symmetry orbit averaging (Sec. 6.1) for reflect3, reflect6 and rotate3 on
  cubes and (reflect3) a ragged box, to float rounding (the sum runs in double
  over the group in the oracle's order);
* trigonometric initialization with its sigmoid projection (Sec. 6.2): the
  density within 2e-5 (the field is summed in double and stored in float
  before the projection) and its mean equal to the volume fraction;
* the density-weighted sensitivity filter (Sec. 5.3) within 1e-6 relative.
"""
import numpy as np
import pytest
import torch

from oracle import design as D
from paper_2301_08911_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def ctx_for(shape):
    from paper_2301_08911_amd.hmg import Context
    return Context(shape, precision="fp32")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).cuda()


@pytest.mark.parametrize("kind,shape", [("reflect3", (16, 16, 16)), ("reflect6", (16, 16, 16)),
                                        ("rotate3", (16, 16, 16)), ("reflect3", (12, 8, 10)),
                                        ("reflect6", (9, 9, 9)), ("rotate3", (7, 7, 7))])
def test_symmetrize_matches_oracle(kind, shape):
    n = int(np.prod(shape))
    x = I.uniform01(31, 0, n).astype(np.float32)
    ctx = ctx_for(shape)
    y = ctx.symmetrize(dev(x), kind).cpu().numpy().astype(np.float64)
    ref = D.symmetrize(x.astype(np.float64), shape, kind)
    err = np.abs(y - ref).max()
    print(kind, shape, "max abs err", err, flush=True)
    assert err <= 6e-8, err
    # the float result is still invariant to rounding: orbit members are equal
    yy = D.symmetrize(y, shape, kind)
    assert np.abs(yy - y).max() <= 1e-7


def test_symmetrize_rejects_non_cubic():
    from paper_2301_08911_amd.hmg import HmgError
    ctx = ctx_for((12, 8, 10))
    x = torch.zeros(12 * 8 * 10, device="cuda")
    with pytest.raises(HmgError):
        ctx.symmetrize(x, "reflect6")
    with pytest.raises(HmgError):
        ctx.symmetrize(x, "rotate3")


@pytest.mark.parametrize("nfreq,shape,vf,seed", [(1, (16, 16, 16), 0.3, 1), (2, (24, 20, 16), 0.1, 2),
                                                 (3, (32, 32, 32), 0.5, 3)])
def test_trig_init_matches_oracle(nfreq, shape, vf, seed):
    q, w = I.trig_init_draws(nfreq, seed)
    ctx = ctx_for(shape)
    rho, mu = ctx.trig_init(nfreq, q, w, vf)
    rho = rho.cpu().numpy().astype(np.float64)
    ref, mu_ref = D.trig_init(shape, nfreq, q, w, vf)
    err = np.abs(rho - ref).max()
    print(nfreq, shape, vf, "max abs err", err, "mu", mu, mu_ref, flush=True)
    assert err < 2e-5, err
    assert abs(rho.mean() - vf) < 1e-6
    assert abs(mu - mu_ref) < 1e-5 * max(1.0, abs(mu_ref))
    assert rho.min() >= 1e-3 - 1e-9 and rho.max() <= 1e-3 + min(1.5 * vf, 1.0) + 1e-6


def test_trig_init_rejects_bad_arguments():
    from paper_2301_08911_amd.hmg import HmgError
    ctx = ctx_for((8, 8, 8))
    q, w = I.trig_init_draws(1, 0)
    with pytest.raises(HmgError):
        ctx.trig_init(1, q, w[:-1], 0.3)
    with pytest.raises(HmgError):
        ctx.trig_init(5, q, w, 0.3)
    with pytest.raises(HmgError):
        ctx.trig_init(1, [0, 0, 0, 0], w, 0.3)


@pytest.mark.parametrize("shape", [(16, 16, 16), (66, 10, 12)])
def test_filter_sensitivity_matches_oracle(shape):
    n = int(np.prod(shape))
    x = (1e-4 + (1 - 1e-4) * I.uniform01(32, 0, n)).astype(np.float32)
    x[::17] = 1e-5
    g = (2 * I.uniform01(33, 0, n) - 1).astype(np.float32)
    ctx = ctx_for(shape)
    out = ctx.filter_sensitivity(dev(x), dev(g)).cpu().numpy().astype(np.float64)
    ref = D.filter_sensitivity(x.astype(np.float64), g.astype(np.float64), shape)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(shape, "rel err", err, flush=True)
    assert err < 1e-6, err
