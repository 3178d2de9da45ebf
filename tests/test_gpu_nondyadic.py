"""GPU parity of non-dyadic coarsening (Sec. 4.2): the first coarse level is four
times coarser per axis, assembled from the densities with the factor-4
trilinear weights (Eq. st-level-2, st-assemb-w), and reached by the factor-4
restriction and prolongation.  Checks through the C ABI against the oracle's
factor-4 prolongation P4:

* the level-1 stencil equals P4^T K P4 (FP64, 1e-13) and deeper levels the
  dyadic Galerkin products below it;
* restriction and prolongation equal P4^T and P4;
* one Gauss-Seidel V-cycle equals the oracle's non-dyadic cycle (FP64 1e-11);
* an FP32 solve gives the oracle's C^H (1e-5).
"""
import numpy as np
import pytest
import torch

from oracle import hmgref as O
from paper_2301_08911_amd import inputs as I

pytestmark = pytest.mark.gpu

K0 = O.element_stiffness()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def ctx_for(shape, precision="fp64", **kw):
    from paper_2301_08911_amd.hmg import Context
    return Context(shape, precision=precision, nondyadic=True, **kw)


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 16, 24)])
def test_stencils_match_galerkin_products(shape):
    rho = np.asarray(I.uniform_density(shape, 5), dtype=np.float32).ravel()
    ctx = ctx_for(shape)
    ctx.set_density(dev(rho))
    K = O.assemble_stiffness(O.simp_scale(rho.astype(np.float64)), shape, K0)
    fine, factor = shape, 4
    for level in range(1, ctx.num_levels()):
        P = O.prolongation(fine, factor)
        K = (P.T @ K @ P).tocsr()
        fine = tuple(v // factor for v in fine)
        factor = 2
        assert ctx.level_dims(level) == fine
        ref = O.stencil_blocks(K, fine)
        st = ctx.get_stencil(level).cpu().numpy()
        err = np.abs(st - ref).max() / np.abs(ref).max()
        print(shape, "level", level, fine, "stencil err", err, flush=True)
        assert err < 1e-13, (level, err)


def test_transfers_match_factor4_P():
    shape = (32, 16, 16)
    ctx = ctx_for(shape)
    ctx.set_density(dev(np.full(np.prod(shape), 0.5, np.float32)))
    assert ctx.level_dims(1) == (8, 4, 4)
    P = O.prolongation(shape, 4)
    cshape = tuple(v // 4 for v in shape)
    nf, nc = int(np.prod(shape)), int(np.prod(cshape))
    e = I.random_signed_field(cshape, 6)
    r = I.random_signed_field(shape, 7)
    up = ctx.transfer(0, 1, dev(e, torch.float64)).cpu().numpy()
    dn = ctx.transfer(0, 0, dev(r, torch.float64)).cpu().numpy()
    up_ref = (P @ e.transpose(0, 2, 1).reshape(6, 3 * nc).T).T.reshape(6, nf, 3)
    dn_ref = (P.T @ r.transpose(0, 2, 1).reshape(6, 3 * nf).T).T.reshape(6, nc, 3)
    assert np.abs(up.transpose(0, 2, 1) - up_ref).max() < 1e-15
    assert np.abs(dn.transpose(0, 2, 1) - dn_ref).max() < 1e-13


@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 32, 32)])
def test_gs_vcycle_matches_oracle(shape):
    rho = (0.3 + 0.7 * I.smoothed_noise_density(shape, 8, 0.3, sigma=1.5)).astype(np.float32).ravel()
    ctx = ctx_for(shape, smoother="gs")
    ctx.set_density(dev(rho))
    x = I.random_signed_field(shape, 21)
    z = ctx.vcycle(dev(x, torch.float64)).cpu().numpy()
    K = O.assemble_stiffness(O.simp_scale(rho.astype(np.float64)), shape, K0)
    prec = O.multigrid_preconditioner(K, shape, smoother="gs", first_factor=4)
    assert prec.levels == ctx.num_levels()
    zr = prec(x.transpose(0, 2, 1)).transpose(0, 2, 1)
    err = max(rel(z[c], zr[c]) for c in range(6))
    print(shape, "levels", prec.levels, "max rel err", err, flush=True)
    assert err < 1e-11, err


def test_fp32_solve_against_oracle():
    from paper_2301_08911_amd.hmg import Context
    shape = (16, 16, 32)
    rho = np.asarray(I.smoothed_noise_density(shape, 9, 0.3, sigma=1.5), dtype=np.float32).ravel()
    iters = {}
    for nd in (True, False):
        ctx = Context(shape, precision="fp32", nondyadic=nd)
        ctx.set_density(dev(rho))
        res = ctx.solve_cases(1e-7, 3000)
        assert res.converged, res
        iters[nd] = res.iters.tolist()
        if nd:
            C = ctx.elastic_tensor()
            levels = ctx.num_levels()
    s = O.simp_scale(rho.astype(np.float64))
    u, _, _ = O.solve_cases(s, shape, tol=1e-10, multigrid=True)
    Cref = O.elastic_tensor(s, u, shape, K0, O.unit_strain_displacements())
    e = rel(C, Cref)
    print("non-dyadic levels", levels, "iters", iters[True], "dyadic", iters[False],
          f"C^H err {e:.2e}", flush=True)
    assert e < 1e-5, e


def test_nondyadic_needs_divisible_by_four():
    from paper_2301_08911_amd.hmg import Context, HmgError
    with pytest.raises(HmgError):
        Context((12, 12, 12), nondyadic=True)
