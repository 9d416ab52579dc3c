"""GPU parity of the PCG variants: the flexible (Polak-Ribiere) beta for the
non-symmetric M_2l, and the residual of Eq. residuals read literally,
||M (b - A x)|| / ||M b||, reported at exit."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import build_both, dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1801_08937_amd import mapmaker as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c1(ctx):
    p = synth.config1()
    lp, ln, op, on = build_both(ctx, p)
    b = O.rhs(op, on, p.tod)
    return p, lp, ln, op, on, b


def test_flexible_fixed_iterations_parity(ctx, c1):
    """Ten iterations with M_BD (symmetric) and with an M_2l built from the
    oracle's Z on both sides (not symmetric): the flexible iterates match the
    oracle's flexible PCG to rounding."""
    p, lp, ln, op, on, b = c1
    A = lambda v: O.apply_A(op, on, v)
    M = ctx.mbd(lp, ln)
    OM = O.mbd_build(op, on)
    x, info = ctx.solve(lp, ln, M, dev(b), tol=0.0, max_iter=10, flexible=True)
    xo, io = O.pcg(A, lambda v: O.mbd_apply(OM, v), b, 0.0, 10, flexible=True)
    assert info["iters"] == io.iters == 10
    assert rel(host(x), xo) <= 1e-10
    np.testing.assert_allclose(info["history"], io.history, rtol=1e-9)
    # symmetric M: the same iterates as Fletcher-Reeves, to rounding
    xf, _ = ctx.solve(lp, ln, M, dev(b), tol=0.0, max_iter=10)
    assert rel(host(x), host(xf)) <= 1e-10
    # M_2l from a shared Z
    OM2, _, _ = O.defl_build(op, on, OM, b, 8, 1e-8, 60)
    M2 = ctx.defl_from_Z(lp, ln, M, dev(OM2.Z))
    x2, i2 = ctx.solve(lp, ln, M2, dev(b), tol=0.0, max_iter=10, flexible=True)
    xo2, io2 = O.pcg(A, lambda v: O.m2l_apply(OM2, v), b, 0.0, 10, flexible=True)
    assert rel(host(x2), xo2) <= 1e-9
    np.testing.assert_allclose(i2["history"], io2.history, rtol=1e-8)


def test_flexible_m2l_converges(ctx, c1):
    p, lp, ln, op, on, b = c1
    M = ctx.mbd(lp, ln)
    bd = dev(b)
    M2 = ctx.defl_build(lp, ln, M, bd, k=32, eps_arn=1e-8, m_max=256)
    x1, i1 = ctx.solve(lp, ln, M2, bd, tol=1e-10, max_iter=500)
    x2, i2 = ctx.solve(lp, ln, M2, bd, tol=1e-10, max_iter=500, flexible=True)
    assert i1["converged"] and i2["converged"]
    assert rel(host(x1), host(x2)) <= 1e-7
    with pytest.raises(Exception):
        ctx.solve(lp, ln, M, dev(np.stack([b, b], 1).reshape(-1)), tol=1e-8, max_iter=10,
                  nrhs=2, block=True, flexible=True)


def test_literal_preconditioned_residual(ctx, c1):
    p, lp, ln, op, on, b = c1
    OM = O.mbd_build(op, on)
    M = ctx.mbd(lp, ln)
    for Mh, apply_M in ((M, lambda v: O.mbd_apply(OM, v)), (None, lambda v: v)):
        x, info = ctx.solve(lp, ln, Mh, dev(b), tol=1e-6, max_iter=300)
        r = b - O.apply_A(op, on, host(x))
        ref = np.linalg.norm(apply_M(r)) / np.linalg.norm(apply_M(b))
        assert abs(info["rel_res_precond"] - ref) <= 1e-9 * ref
        if Mh is None:
            assert abs(info["rel_res_precond"] - info["rel_res_true"]) <= 1e-12
    # the block solver reports it too
    B = np.stack([b, 0.5 * b + 1.0], 1)
    X, infos = ctx.solve(lp, ln, M, dev(B.reshape(-1)), tol=1e-6, max_iter=300, nrhs=2,
                         block=True)
    Xh = host(X).reshape(-1, 2)
    for c in range(2):
        r = B[:, c] - O.apply_A(op, on, Xh[:, c])
        ref = np.linalg.norm(O.mbd_apply(OM, r)) / np.linalg.norm(O.mbd_apply(OM, B[:, c]))
        assert abs(infos[c]["rel_res_precond"] - ref) <= 1e-9 * ref


def test_defl_from_prior_mbd_solve_parity(ctx, c1):
    """Ritz pairs harvested from an M_BD PCG run: the Lanczos tridiagonal's
    eigenvalues match the oracle's, the M_2l built from them satisfies
    Eq. ident and cuts the iterations."""
    p, lp, ln, op, on, b = c1
    M = ctx.mbd(lp, ln)
    OM = O.mbd_build(op, on)
    bd = dev(b)
    # 15 iterations: short of convergence (M_BD needs 18 to 1e-8), so the
    # Lanczos vectors keep their orthogonality and no Ritz value repeats
    M2 = ctx.defl_build_pcg(lp, ln, M, bd, k=8, m_max=15)
    res = O.pcg_lanczos(lambda v: O.apply_A(op, on, v), lambda v: O.mbd_apply(OM, v), b, 15)
    th_o = np.linalg.eigvalsh(res.T)
    assert M2.arnoldi_info.m == res.m == 15 and M2.arnoldi_info.k == 8
    np.testing.assert_allclose(M2.theta, th_o, rtol=1e-8)
    OM2, _, _ = O.defl_build_pcg(op, on, OM, b, 8, 15)
    import scipy.linalg
    ang = scipy.linalg.subspace_angles(host(M2.export()[0]), OM2.Z)
    assert np.max(np.sin(ang)) <= 1e-6
    Z = M2.export()[0]
    AZ = torch_stack_apply(ctx, lp, ln, Z)
    MAZ = torch_stack_precond(ctx, M2, AZ)
    assert rel(host(MAZ), host(Z)) <= 1e-9
    _, i1 = ctx.solve(lp, ln, M, bd, tol=1e-8, max_iter=500)
    _, i2 = ctx.solve(lp, ln, M2, bd, tol=1e-8, max_iter=500)
    assert i1["converged"] and i2["converged"] and i2["iters"] < i1["iters"]
    # stopped at the prior solve's tolerance: as many steps as that solve,
    # and running far past convergence still yields a valid M_2l (repeated
    # Ritz values are dropped, not an error)
    import torch
    x3 = torch.empty_like(bd)
    M3 = ctx.defl_build_pcg(lp, ln, M, bd, k=16, m_max=500, tol=1e-6, x_out=x3)
    x6, i6 = ctx.solve(lp, ln, M, bd, tol=1e-6, max_iter=500)
    assert M3.arnoldi_info.m == i6["iters"]
    np.testing.assert_array_equal(host(x3), host(x6))  # the same solve, the same bits
    M4 = ctx.defl_build_pcg(lp, ln, M, bd, k=32, m_max=120)
    assert 1 <= M4.arnoldi_info.k <= 32
    _, i4 = ctx.solve(lp, ln, M4, bd, tol=1e-8, max_iter=500)
    assert i4["converged"]


def torch_stack_apply(ctx, lp, ln, Z):
    import torch
    return torch.stack([ctx.apply_A(lp, ln, Z[:, c].contiguous()) for c in range(Z.shape[1])], 1)


def torch_stack_precond(ctx, M, V):
    import torch
    return torch.stack([ctx.precond_apply(M, V[:, c].contiguous()) for c in range(V.shape[1])], 1)
