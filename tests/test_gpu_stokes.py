"""GPU parity of the intensity-only (I) and polarisation-only (QU)
pointings, the map-making systems of a detector pair's sum and difference
streams (Eqs. d+ and d-), against the FP64 oracle through the C ABI."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import dev, host, maxrel, rel

pytestmark = pytest.mark.gpu

TOL_OP = 1e-12


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1801_08937_amd import mapmaker as mm
    c = mm.Context(0)
    yield c
    c.close()


def _both(ctx, p, stokes, prec=0, min_hits=None):
    mh = p.min_hits if min_hits is None else min_hits
    psi = None if stokes == "I" else p.psi
    lp = ctx.pointing(dev(p.pix), None if psi is None else dev(psi), p.n_pix_total, mh, prec,
                      stokes=stokes)
    ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw, 1, prec)
    op = O.pointing_build(p.pix, psi, p.n_pix_total, mh, stokes)
    on = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    return lp, ln, op, on


@pytest.mark.parametrize("stokes", ["I", "QU"])
def test_stokes_operators_parity(ctx, stokes):
    p = synth.random_problem(41, n_side=12, n_samp=30011, n_int=5, half_bw=6, n_filters=2,
                             flag_frac=0.1)
    lp, ln, op, on = _both(ctx, p, stokes)
    assert lp.n == op.n and lp.nc == len(stokes) and lp.stokes == stokes
    rng = np.random.default_rng(42)
    x = rng.standard_normal(op.n)
    y = rng.standard_normal(p.n_samp)
    assert maxrel(host(ctx.apply_P(lp, dev(x))), O.apply_P(op, x)) <= TOL_OP
    assert maxrel(host(ctx.apply_PT(lp, dev(y))), O.apply_PT(op, y)) <= TOL_OP
    Ax = host(ctx.apply_A(lp, ln, dev(x)))
    assert maxrel(Ax, O.apply_A(op, on, x)) <= TOL_OP
    assert maxrel(host(ctx.rhs(lp, ln, dev(p.tod))), O.rhs(op, on, p.tod)) <= TOL_OP
    M = ctx.mbd(lp, ln)
    Mo = O.mbd_build(op, on)
    assert maxrel(host(ctx.precond_apply(M, dev(x))), O.mbd_apply(Mo, x)) <= TOL_OP
    # four columns: a column does not depend on the others (bitwise), and
    # matches the single-column apply to rounding
    X = rng.standard_normal((op.n, 4))
    X[:, 3] = x
    AX = host(ctx.apply_A(lp, ln, dev(X.reshape(-1)), nrhs=4)).reshape(-1, 4)
    X2 = rng.standard_normal((op.n, 4))
    X2[:, 3] = x
    AX2 = host(ctx.apply_A(lp, ln, dev(X2.reshape(-1)), nrhs=4)).reshape(-1, 4)
    np.testing.assert_array_equal(AX[:, 3], AX2[:, 3])
    assert maxrel(AX[:, 3], Ax) <= 1e-13
    assert maxrel(AX, np.stack([O.apply_A(op, on, X[:, c]) for c in range(4)], 1)) <= TOL_OP


@pytest.mark.parametrize("stokes", ["I", "QU"])
def test_stokes_fp32_form(ctx, stokes):
    p = synth.random_problem(43, n_side=10, n_samp=20011, n_int=4, half_bw=5, n_filters=2)
    lp, ln, op, on = _both(ctx, p, stokes, prec=1)
    x = np.random.default_rng(44).standard_normal(op.n)
    assert rel(host(ctx.apply_A(lp, ln, dev(x))), O.apply_A(op, on, x)) <= 1e-5


@pytest.mark.parametrize("stokes", ["I", "QU"])
def test_stokes_solves_mbd_and_m2l(ctx, stokes):
    p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=10)
    lp, ln, op, on = _both(ctx, p, stokes)
    b = ctx.rhs(lp, ln, dev(p.tod))
    Mbd = ctx.mbd(lp, ln)
    x1, i1 = ctx.solve(lp, ln, Mbd, b, tol=1e-10, max_iter=2000)
    M2 = ctx.defl_build(lp, ln, Mbd, b, k=8, eps_arn=1e-10, m_max=60)
    x2, i2 = ctx.solve(lp, ln, M2, b, tol=1e-10, max_iter=2000)
    assert i1["converged"] and i2["converged"] and i2["iters"] <= i1["iters"]
    Mo = O.mbd_build(op, on)
    xo, _ = O.pcg(lambda v: O.apply_A(op, on, v), lambda v: O.mbd_apply(Mo, v),
                  O.rhs(op, on, p.tod), 1e-13, 3000)
    assert rel(host(x1), xo) <= 1e-7 and rel(host(x2), xo) <= 1e-7
    # Eq. ident on this pointing: M_2l A Z = Z
    Z = M2.export()[0]
    AZ = ctx.apply_A(lp, ln, Z[:, 0].contiguous())
    assert rel(host(ctx.precond_apply(M2, AZ)), host(Z[:, 0])) <= 1e-9


def test_pair_sum_diff_kernel(ctx):
    import torch
    rng = np.random.default_rng(45)
    a, b = rng.standard_normal(100003), rng.standard_normal(100003)
    pl, mi = ctx.pair_sum_diff(dev(a), dev(b))
    np.testing.assert_array_equal(host(pl), (a + b) * 0.5)
    np.testing.assert_array_equal(host(mi), (a - b) * 0.5)
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    pl, mi = ctx.pair_sum_diff(dev(a32), dev(b32))
    np.testing.assert_array_equal(host(pl), (a32 + b32) * np.float32(0.5))
    # in place: plus over a, minus over b
    ta, tb = dev(a), dev(b)
    ctx.pair_sum_diff(ta, tb, ta, tb)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(ta), (a + b) * 0.5)
    np.testing.assert_array_equal(host(tb), (a - b) * 0.5)


def test_pair_separation_on_gpu(ctx):
    """A detector pair with orthogonal polarisers (Sect. 4): the IQU solve of
    both detectors' streams equals the I solve of d+ = (d_A + d_B)/2 beside
    the QU solve of d- = (d_A - d_B)/2, with one banded N^-1 for both."""
    p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=10)
    n = p.n_samp
    psi_b = p.psi + 0.5 * np.pi
    d_a = p.tod
    d_b = synth.signal_tod(p.pix, psi_b, p.signal) + \
        np.random.default_rng(46).standard_normal(n)
    ist2 = np.concatenate([p.interval_start, p.interval_start[1:] + n])
    fid2 = np.concatenate([p.filter_id, p.filter_id])
    lp2 = ctx.pointing(dev(np.concatenate([p.pix, p.pix])), dev(np.concatenate([p.psi, psi_b])),
                       p.n_pix_total, 2 * p.min_hits)
    ln2 = ctx.noise(ist2, fid2, p.band, p.half_bw)
    b2 = ctx.rhs(lp2, ln2, dev(np.concatenate([d_a, d_b])))
    x2, i2 = ctx.solve(lp2, ln2, ctx.mbd(lp2, ln2), b2, tol=1e-11, max_iter=3000)
    dp, dm = ctx.pair_sum_diff(dev(d_a), dev(d_b))
    out = {}
    for stokes, d in (("I", dp), ("QU", dm)):
        lp = ctx.pointing(dev(p.pix), None if stokes == "I" else dev(p.psi), p.n_pix_total,
                          p.min_hits, stokes=stokes)
        ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw)
        b = ctx.rhs(lp, ln, d)
        x, info = ctx.solve(lp, ln, ctx.mbd(lp, ln), b, tol=1e-11, max_iter=3000)
        assert info["converged"] and lp.n_obs == lp2.n_obs
        out[stokes] = host(x)
    assert i2["converged"]
    X2 = host(x2).reshape(-1, 3)
    assert rel(X2[:, 0], out["I"]) <= 1e-8
    assert rel(X2[:, 1:].reshape(-1), out["QU"]) <= 1e-8


def test_stokes_errors(ctx):
    from paper_1801_08937_amd import mapmaker as mm
    p = synth.random_problem(47, n_side=8, n_samp=5000, n_int=3, half_bw=5, n_filters=1)
    with pytest.raises(mm.MapmakerError):
        ctx.pointing(dev(p.pix), None, p.n_pix_total, 3, stokes="QU")
    with pytest.raises(ValueError):
        ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, 3, stokes="Q")
    lpI = ctx.pointing(dev(p.pix), None, p.n_pix_total, 3, stokes="I")
    lp3 = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, 3)
    ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw)
    MI = ctx.mbd(lpI, ln)
    b = ctx.rhs(lp3, ln, dev(p.tod))
    with pytest.raises(mm.MapmakerError):
        ctx.solve(lp3, ln, MI, b, tol=1e-8, max_iter=10)
