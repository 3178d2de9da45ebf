"""The FP16 displacement cast before C^H and the sensitivities (Sec. 4.3).

With post_fp16 the FP32 solution is cast to FP16 and C^H and the element
sensitivities are evaluated from that copy.  C^H depends on the rounding only
to second order (the first-order term is the residual r^T du, and the solve
drives r to the tolerance), so it stays within the FP32 bar of 1e-5 of the
FP64 oracle; the sensitivities are first order in the rounding and meet the
reduced-precision bar of 1e-2 (relative L2).  The FP16 path must also agree
with the FP32 path of the same solve to those orders.
"""
import numpy as np
import pytest
import torch

from oracle import hmgref as O
from paper_2301_08911_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("shape,seed,vf", [((16, 16, 16), 3, 0.3), ((24, 16, 20), 4, 0.2)])
def test_fp16_cast_against_oracle(shape, seed, vf):
    from paper_2301_08911_amd.hmg import Context
    rho = np.asarray(I.smoothed_noise_density(shape, seed, vf, sigma=2.0),
                     dtype=np.float32).ravel()
    rd = torch.from_numpy(rho).cuda()
    out = {}
    for cast in (False, True):
        ctx = Context(shape, precision="fp32", post_fp16=cast)
        ctx.set_density(rd)
        res = ctx.solve_cases(1e-7, 3000)
        assert res.converged, res
        C = ctx.elastic_tensor()
        g = ctx.sensitivity(O.shear_weights()).cpu().numpy().astype(np.float64)
        # a second evaluation reuses the cast
        assert np.array_equal(ctx.elastic_tensor(), C)
        out[cast] = (C, g)
    s = O.simp_scale(rho.astype(np.float64))
    u, _, _ = O.solve_cases(s, shape, tol=1e-10, multigrid=True)
    K0, chi = O.element_stiffness(), O.unit_strain_displacements()
    Cref = O.elastic_tensor(s, u, shape, K0, chi)
    gref = O.sensitivity(rho.astype(np.float64), u, shape, K0, chi, O.shear_weights())
    eC16, eC32 = rel(out[True][0], Cref), rel(out[False][0], Cref)
    eg16, eg32 = rel(out[True][1], gref), rel(out[False][1], gref)
    print(shape, f"C^H fp16 {eC16:.2e} fp32 {eC32:.2e}; dF fp16 {eg16:.2e} fp32 {eg32:.2e}; "
          f"fp16 vs fp32 C^H {rel(out[True][0], out[False][0]):.2e}", flush=True)
    assert eC16 < 1e-5, eC16
    assert eg16 < 1e-2, eg16
    assert rel(out[True][0], out[False][0]) < 1e-5


@pytest.mark.parametrize("n,bound", [(32, 1e-4), (64, 3e-4)])
def test_fp16_cast_error_growth_with_resolution(n, bound):
    """The cast keeps 11 bits of u, whose magnitude grows with N (u is in element
    units) while the energy lives in element-to-element differences, so the C^H
    error of the cast grows with N.  Measured against the FP32 evaluation of
    the same solve: within the reduced-precision bar of 1e-4 at 32^3, just
    above it at 64^3 (1.1e-4 measured), which bounds where the cast is usable."""
    from paper_2301_08911_amd.hmg import Context
    shape = (n, n, n)
    rho = torch.from_numpy(np.asarray(I.smoothed_noise_density(shape, 5, 0.3, sigma=3.0),
                                      dtype=np.float32).ravel()).cuda()
    ctx = Context(shape, precision="fp32", post_fp16=True)
    ctx.set_density(rho)
    res = ctx.solve_cases(1e-6, 3000)
    assert res.converged, res
    C16 = ctx.elastic_tensor()
    ref = Context(shape, precision="fp32")
    ref.set_density(rho)
    ref.solve_cases(1e-6, 3000)
    e = rel(C16, ref.elastic_tensor())
    print(f"{n}^3: C^H of the FP16 cast vs FP32: {e:.2e}", flush=True)
    assert e < bound, e


def test_fp16_cast_needs_fp32_storage():
    from paper_2301_08911_amd.hmg import Context, HmgError
    with pytest.raises(HmgError):
        Context((8, 8, 8), precision="fp64", post_fp16=True)
