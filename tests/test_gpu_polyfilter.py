"""GPU parity of the polynomial template filter (F = W - W B (B^T W B)^-1
B^T W, piecewise Legendre polynomials per subscan) and of A, b, M_BD and the
solvers built on it, against the FP64 oracle through the C ABI."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import build_both, dev, host, maxrel, rel

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


def _subscans(p, seed, lo=5, hi=300):
    """Ragged subscans inside every interval."""
    rng = np.random.default_rng(seed)
    starts = [0]
    for i in range(p.n_intervals):
        a, b = int(p.interval_start[i]), int(p.interval_start[i + 1])
        t = a
        while t < b:
            t = min(b, t + int(rng.integers(lo, hi)))
            starts.append(t)
    return np.array(starts, dtype=np.int64)


def _both(ctx, p, order, seed, prec=0):
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits, prec)
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    sub = _subscans(p, seed)
    w = np.random.default_rng(seed + 1).uniform(0.5, 2.0, p.n_intervals)
    lf = ctx.polyfilter(lp, p.interval_start, w, sub, order)
    of = O.polyfilter_build(op, p.interval_start, w, sub, order)
    return lp, lf, op, of


@pytest.mark.parametrize("order", [0, 1, 2, 3, 7])
def test_polyfilter_apply_parity(ctx, order):
    import torch
    p = synth.random_problem(11, n_side=12, n_samp=30011, n_int=5, half_bw=5, n_filters=2,
                             flag_frac=0.1)
    lp, lf, op, of = _both(ctx, p, order, order)
    assert lf.method == 3
    y = np.random.default_rng(2).standard_normal(p.n_samp)
    z = host(ctx.noise_apply(lf, dev(y)))
    ref = O.polyfilter_apply(of, y)
    assert maxrel(z, ref) <= TOL_OP, maxrel(z, ref)
    # columns: each equals the single apply bitwise
    Y = np.random.default_rng(3).standard_normal((p.n_samp, 4))
    Y[:, 2] = y
    Z = host(ctx.noise_apply(lf, dev(Y.reshape(-1)), nrhs=4)).reshape(-1, 4)
    np.testing.assert_array_equal(Z[:, 2], z)


def test_polyfilter_operators_and_mbd(ctx):
    p = synth.random_problem(12, n_side=10, n_samp=20011, n_int=4, half_bw=5, n_filters=2,
                             flag_frac=0.05)
    lp, lf, op, of = _both(ctx, p, 2, 12)
    x = np.random.default_rng(4).standard_normal(op.n)
    assert maxrel(host(ctx.apply_A(lp, lf, dev(x))), O.apply_A(op, of, x)) <= TOL_OP
    assert maxrel(host(ctx.rhs(lp, lf, dev(p.tod))), O.rhs(op, of, p.tod)) <= TOL_OP
    M = ctx.mbd(lp, lf)
    Mo = O.mbd_build(op, of)
    v = np.random.default_rng(5).standard_normal(op.n)
    assert maxrel(host(ctx.precond_apply(M, dev(v))), O.mbd_apply(Mo, v)) <= TOL_OP


def test_polyfilter_fp32_form(ctx):
    p = synth.random_problem(13, n_side=10, n_samp=20011, n_int=4, half_bw=5, n_filters=2,
                             flag_frac=0.05)
    lp, lf, op, of = _both(ctx, p, 2, 13, prec=1)
    y = np.random.default_rng(6).standard_normal(p.n_samp)
    z = host(ctx.noise_apply(lf, dev(y.astype(np.float32))))
    assert rel(z, O.polyfilter_apply(of, y)) <= 1e-5


def test_polyfilter_solves_m2l_beats_mbd(ctx):
    """Cross-linked scan, subscans = sweeps, quadratic polynomials removed:
    the filter leaves near-null sky modes (Sect. 4), M_BD needs many more
    iterations than M_2l; both reach the oracle's solution."""
    p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=10)
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
    lp.set_grid(p.n_side)
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    sub = np.arange(0, p.n_samp + 1, 32, dtype=np.int64)
    w = np.ones(p.n_intervals)
    lf = ctx.polyfilter(lp, p.interval_start, w, sub, 2)
    of = O.polyfilter_build(op, p.interval_start, w, sub, 2)
    d = synth.signal_tod(p.pix, p.psi, p.signal) + np.random.default_rng(0).standard_normal(p.n_samp)
    b = ctx.rhs(lp, lf, dev(d))
    Mbd = ctx.mbd(lp, lf)
    x1, i1 = ctx.solve(lp, lf, Mbd, b, tol=1e-10, max_iter=2000)
    M2 = ctx.defl_build(lp, lf, Mbd, b, k=16, eps_arn=1e-8, m_max=120)
    x2, i2 = ctx.solve(lp, lf, M2, b, tol=1e-10, max_iter=2000)
    assert i1["converged"] and i2["converged"]
    assert i2["iters"] * 2 < i1["iters"], (i1["iters"], i2["iters"])
    Mo = O.mbd_build(op, of)
    xo, io = O.pcg(lambda v: O.apply_A(op, of, v), lambda v: O.mbd_apply(Mo, v),
                   O.rhs(op, of, d), 1e-12, 3000)

    def no_monopole(v):
        # the filter leaves the intensity monopole unconstrained (A 1_I = 0):
        # solutions agree up to that null direction
        v = np.array(v, dtype=np.float64).reshape(-1, 3)
        v[:, 0] -= v[:, 0].mean()
        return v.reshape(-1)
    ref = no_monopole(xo)
    assert rel(no_monopole(host(x1)), ref) <= 1e-6 and rel(no_monopole(host(x2)), ref) <= 1e-6


def test_polyfilter_null_mode_left_out_of_Z(ctx):
    """Order 0 leaves the intensity monopole exactly unconstrained; the
    deflation space skips that null direction and E stays SPD."""
    p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=10)
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
    sub = np.arange(0, p.n_samp + 1, 32, dtype=np.int64)
    lf = ctx.polyfilter(lp, p.interval_start, np.ones(p.n_intervals), sub, 0)
    b = ctx.rhs(lp, lf, dev(synth.signal_tod(p.pix, p.psi, p.signal)))
    Mbd = ctx.mbd(lp, lf)
    M2 = ctx.defl_build(lp, lf, Mbd, b, k=8, eps_arn=1e-8, m_max=120)
    x, info = ctx.solve(lp, lf, M2, b, tol=1e-9, max_iter=1000)
    assert info["converged"]


def test_order0_null_ritz_skipped_span_vs_oracle(ctx):
    """The null-direction rule of the Ritz selection on the GPU against the
    oracle: order-0 filter, Arnoldi from a generic start vector until the
    Krylov space is invariant (a rounding-level Ritz value appears on both
    sides).  span(Z) agrees with the oracle's and with the dense
    eigenvectors of the k smallest non-null eigenvalues of M_BD A; the null
    vector stays out."""
    import scipy.linalg
    from test_oracle_pins import _pf_problem
    p, op, of = _pf_problem(0, 0)
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
    lf = ctx.polyfilter(lp, of.interval_start, of.band[:, 0], of.subscan_start, 0)
    n = op.n
    Mo = O.mbd_build(op, of)
    k = 5
    b = np.random.default_rng(5).standard_normal(n)
    OM2, res, theta = O.defl_build(op, of, Mo, b, k, 1e-10, n)
    M = ctx.mbd(lp, lf)
    M2 = ctx.defl_build(lp, lf, M, dev(b), k=k, eps_arn=1e-10, m_max=n)
    assert M2.arnoldi_info.m < n and abs(M2.arnoldi_info.m - res.m) <= 1
    Zg = host(M2.export()[0])
    assert Zg.shape[1] == k == OM2.Z.shape[1]
    assert np.max(np.sin(scipy.linalg.subspace_angles(Zg, OM2.Z))) <= 1e-6
    Bd = np.stack([O.mbd_apply(Mo, O.apply_A(op, of, e)) for e in np.eye(n)], axis=1)
    ev, V = np.linalg.eig(Bd)
    order = np.argsort(ev.real)
    V = V[:, order].real
    assert np.max(np.sin(scipy.linalg.subspace_angles(Zg, V[:, 1:1 + k]))) <= 1e-6
    u = V[:, 0] / np.linalg.norm(V[:, 0])
    assert np.linalg.norm(u - Zg @ (Zg.T @ u)) >= 0.9


def test_polyfilter_errors(ctx):
    from paper_1801_08937_amd import mapmaker as mm
    p = synth.random_problem(14, n_side=8, n_samp=5000, n_int=3, half_bw=5, n_filters=1)
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
    bad = np.array([0, int(p.interval_start[1]) + 1, p.n_samp], dtype=np.int64)
    with pytest.raises(mm.MapmakerError):
        ctx.polyfilter(lp, p.interval_start, np.ones(p.n_intervals), bad, 1)
    ok = np.array([0, p.n_samp], dtype=np.int64) if p.n_intervals == 1 else p.interval_start
    with pytest.raises(mm.MapmakerError):
        ctx.polyfilter(lp, p.interval_start, np.ones(p.n_intervals), ok, 8)
    with pytest.raises(mm.MapmakerError):
        ctx.polyfilter(lp, p.interval_start, -np.ones(p.n_intervals), ok, 1)


def _transfer_rows_np(Z, obs_from, obs_to, nc=3):
    """Rows of Z moved from one pixel set to another by global pixel id
    (0 where the source lacks the pixel), with a Python dict."""
    pos = {int(g): i for i, g in enumerate(obs_from)}
    k = Z.shape[1]
    out = np.zeros((nc * len(obs_to), k))
    for j, g in enumerate(obs_to):
        i = pos.get(int(g))
        if i is not None:
            out[nc * j:nc * j + nc] = Z[nc * i:nc * i + nc]
    return out


def test_transferred_deflation_space(ctx):
    """The "simplified" two-level preconditioner of the divide-and-conquer run
    (Sect. 7.3): Z built by Arnoldi on one subset of detectors, moved to
    another subset's pixels by the library (mm_defl_transfer), with AZ and E
    rebuilt there.  Against the oracle's M_2l built from the same moved Z:
    the rows bitwise, the M_2l apply <= 1e-10, E <= 1e-12; Eq. ident holds on
    the new subset; the solve takes the oracle's iteration count (+-1) and
    its map is within 1e-6 of the oracle's (modulo the null monopole)."""
    import torch
    p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=10)
    half = p.n_samp // 2
    ih = p.n_intervals // 2
    subs = []
    for k in range(2):
        sl = slice(k * half, (k + 1) * half)
        lp = ctx.pointing(dev(p.pix[sl]), dev(p.psi[sl]), p.n_pix_total, p.min_hits)
        op = O.pointing_build(p.pix[sl], p.psi[sl], p.n_pix_total, p.min_hits)
        ist = p.interval_start[k * ih:(k + 1) * ih + 1] - k * half
        sub = np.arange(0, half + 1, 32)
        lf = ctx.polyfilter(lp, ist, np.ones(ih), sub, 2)
        of = O.polyfilter_build(op, ist, np.ones(ih), sub, 2)
        d = synth.signal_tod(p.pix[sl], p.psi[sl], p.signal) + \
            np.random.default_rng(k).standard_normal(half)
        b = ctx.rhs(lp, lf, dev(d))
        subs.append((lp, lf, ctx.mbd(lp, lf), b, op, of, d))
    lp0, lf0, M0, b0, op0, _, _ = subs[0]
    M20 = ctx.defl_build(lp0, lf0, M0, b0, k=16, eps_arn=1e-8, m_max=120)
    Z0 = host(M20.export()[0])
    lp1, lf1, M1, b1, op1, of1, d1 = subs[1]
    Ms = ctx.defl_transfer(lp0, M20, lp1, lf1, M1)
    Zt, AZt, Et = (host(t) for t in Ms.export())
    assert set(op0.obs_pix.tolist()) != set(op1.obs_pix.tolist())   # the pixel sets differ
    Zref = _transfer_rows_np(Z0, op0.obs_pix, op1.obs_pix)
    np.testing.assert_array_equal(Zt, Zref)
    OMs = O.m2l_from_Z(op1, of1, O.mbd_build(op1, of1), Zref)
    assert maxrel(Et, OMs.E) <= 1e-12, maxrel(Et, OMs.E)
    v = np.random.default_rng(7).standard_normal(op1.n)
    e_apply = maxrel(host(ctx.precond_apply(Ms, dev(v))), O.m2l_apply(OMs, v))
    assert e_apply <= 1e-10, e_apply
    # Eq. ident on the new subset: M_2l A Z = Z
    Z1 = dev(Zt)
    AZ = torch.stack([ctx.apply_A(lp1, lf1, Z1[:, c].contiguous()) for c in range(Z1.shape[1])], 1)
    MAZ = torch.stack([ctx.precond_apply(Ms, AZ[:, c].contiguous()) for c in range(Z1.shape[1])], 1)
    assert rel(host(MAZ), Zt) <= 1e-8
    _, i_bd = ctx.solve(lp1, lf1, M1, b1, tol=1e-8, max_iter=3000)
    x_tr, i_tr = ctx.solve(lp1, lf1, Ms, b1, tol=1e-8, max_iter=3000)
    assert i_bd["converged"] and i_tr["converged"] and i_tr["iters"] < i_bd["iters"]
    bo = O.rhs(op1, of1, d1)
    xo, io = O.pcg(lambda u: O.apply_A(op1, of1, u), lambda u: O.m2l_apply(OMs, u), bo, 1e-8, 3000)
    assert io.converged and abs(io.iters - i_tr["iters"]) <= 1, (io.iters, i_tr["iters"])
    xt, _ = O.pcg(lambda u: O.apply_A(op1, of1, u), lambda u: O.m2l_apply(OMs, u), bo, 1e-12, 3000)

    def no_monopole(u):
        u = np.array(u, dtype=np.float64).reshape(-1, 3)
        u[:, 0] -= u[:, 0].mean()
        return u.reshape(-1)
    e_map = rel(no_monopole(host(x_tr)), no_monopole(xt))
    print(f"transferred M_2l: apply {e_apply:.2e}, map {e_map:.2e}, iters gpu {i_tr['iters']} "
          f"oracle {io.iters}, M_BD {i_bd['iters']}")
    assert e_map <= 1e-6


# ------------------------------------------------ ground templates (Sect. 4)

def _ground_bins(p, seed, n_bins):
    """Random azimuth bins, about a tenth of the samples in none, and (with
    two bins or more) one bin that only flagged samples fall in."""
    rng = np.random.default_rng(seed + 50)
    gb = rng.integers(0, max(n_bins - 1, 1), p.n_samp).astype(np.int32)
    gb[rng.random(p.n_samp) < 0.1] = -1
    if n_bins > 1:
        gb[np.flatnonzero(p.pix < 0)[:3]] = n_bins - 1
    return gb


def _both_ground(ctx, p, order, seed, n_bins, prec=0):
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits, prec)
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    sub = _subscans(p, seed)
    w = np.random.default_rng(seed + 1).uniform(0.5, 2.0, p.n_intervals)
    gb = _ground_bins(p, seed, n_bins)
    lf = ctx.polyfilter(lp, p.interval_start, w, sub, order, dev(gb), n_bins)
    of = O.polyfilter_build(op, p.interval_start, w, sub, order, gb, n_bins)
    return lp, lf, op, of


@pytest.mark.parametrize("order,n_bins", [(0, 5), (2, 5), (2, 61), (3, 1)])
def test_ground_filter_apply_parity(ctx, order, n_bins):
    """F = F_B W^+ F_G W^+ F_B against the oracle; with 5 bins every bin
    spans two or more chunks of the fixed-order bin sums."""
    p = synth.random_problem(21, n_side=12, n_samp=30011, n_int=5, half_bw=5, n_filters=2,
                             flag_frac=0.1)
    lp, lf, op, of = _both_ground(ctx, p, order, 20 + order, n_bins)
    y = np.random.default_rng(22).standard_normal(p.n_samp)
    z = host(ctx.noise_apply(lf, dev(y)))
    ref = O.polyfilter_apply(of, y)
    assert maxrel(z, ref) <= TOL_OP, maxrel(z, ref)
    Y = np.random.default_rng(23).standard_normal((p.n_samp, 4))
    Y[:, 1] = y
    Z = host(ctx.noise_apply(lf, dev(Y.reshape(-1)), nrhs=4)).reshape(-1, 4)
    np.testing.assert_array_equal(Z[:, 1], z)


@pytest.mark.parametrize("lo,hi,n_bins", [(5, 250, 0), (200, 500, 0), (400, 1500, 0),
                                          (5, 250, 5), (400, 1500, 5)])
def test_polyfilter_subscan_lengths(ctx, lo, hi, n_bins):
    """The apply keeps a lane's samples in registers when the longest subscan
    has at most 256 (4 per lane) or 512 (8 per lane) samples, and streams them
    otherwise: each regime, with and without ground templates, against the
    oracle, and a column of a 4-column apply bitwise equal to the single one."""
    p = synth.random_problem(31, n_side=12, n_samp=30011, n_int=5, half_bw=5, n_filters=2,
                             flag_frac=0.1)
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    sub = _subscans(p, lo + hi, lo, hi)
    assert (np.diff(sub).max() > 256) == (hi > 256)
    assert (np.diff(sub).max() > 512) == (hi > 512)
    w = np.random.default_rng(32).uniform(0.5, 2.0, p.n_intervals)
    if n_bins:
        gb = _ground_bins(p, 33, n_bins)
        lf = ctx.polyfilter(lp, p.interval_start, w, sub, 2, dev(gb), n_bins)
        of = O.polyfilter_build(op, p.interval_start, w, sub, 2, gb, n_bins)
    else:
        lf = ctx.polyfilter(lp, p.interval_start, w, sub, 2)
        of = O.polyfilter_build(op, p.interval_start, w, sub, 2)
    y = np.random.default_rng(34).standard_normal(p.n_samp)
    z = host(ctx.noise_apply(lf, dev(y)))
    ref = O.polyfilter_apply(of, y)
    assert maxrel(z, ref) <= TOL_OP, maxrel(z, ref)
    Y = np.random.default_rng(35).standard_normal((p.n_samp, 4))
    Y[:, 3] = y
    Z = host(ctx.noise_apply(lf, dev(Y.reshape(-1)), nrhs=4)).reshape(-1, 4)
    np.testing.assert_array_equal(Z[:, 3], z)


def test_ground_filter_operators_mbd_and_fp32(ctx):
    p = synth.random_problem(24, n_side=10, n_samp=20011, n_int=4, half_bw=5, n_filters=2,
                             flag_frac=0.05)
    lp, lf, op, of = _both_ground(ctx, p, 1, 24, 17)
    x = np.random.default_rng(25).standard_normal(op.n)
    assert maxrel(host(ctx.apply_A(lp, lf, dev(x))), O.apply_A(op, of, x)) <= TOL_OP
    assert maxrel(host(ctx.rhs(lp, lf, dev(p.tod))), O.rhs(op, of, p.tod)) <= TOL_OP
    v = np.random.default_rng(26).standard_normal(op.n)
    M = ctx.mbd(lp, lf)
    assert maxrel(host(ctx.precond_apply(M, dev(v))), O.mbd_apply(O.mbd_build(op, of), v)) <= TOL_OP
    lp32, lf32, _, of32 = _both_ground(ctx, p, 1, 24, 17, prec=1)
    y = np.random.default_rng(27).standard_normal(p.n_samp)
    z = host(ctx.noise_apply(lf32, dev(y.astype(np.float32))))
    assert rel(z, O.polyfilter_apply(of32, y)) <= 1e-5


def test_ground_filter_raster_m2l_beats_mbd(ctx):
    """Cross-linked scan, quadratic polynomials per sweep and azimuth-binned
    ground templates shared by the detectors of each constant-elevation
    pass: both preconditioners reach the true residual, M_2l in far fewer
    iterations."""
    p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=10)
    gb, nb = synth.raster_ground_bins(32, (4, 2), 1 << 12)
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
    lp.set_grid(p.n_side)
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    sub = np.arange(0, p.n_samp + 1, 32, dtype=np.int64)
    w = np.ones(p.n_intervals)
    lf = ctx.polyfilter(lp, p.interval_start, w, sub, 2, dev(gb), nb)
    of = O.polyfilter_build(op, p.interval_start, w, sub, 2, gb, nb)
    d = synth.signal_tod(p.pix, p.psi, p.signal) + np.random.default_rng(1).standard_normal(p.n_samp)
    b = ctx.rhs(lp, lf, dev(d))
    assert maxrel(host(b), O.rhs(op, of, d)) <= TOL_OP
    Mbd = ctx.mbd(lp, lf)
    _, i1 = ctx.solve(lp, lf, Mbd, b, tol=1e-10, max_iter=3000)
    M2 = ctx.defl_build(lp, lf, Mbd, b, k=16, eps_arn=1e-8, m_max=120)
    _, i2 = ctx.solve(lp, lf, M2, b, tol=1e-10, max_iter=3000)
    assert i1["converged"] and i2["converged"], (i1, i2)
    assert i1["rel_res_true"] <= 1e-9 and i2["rel_res_true"] <= 1e-9
    assert i2["iters"] * 2 < i1["iters"], (i1["iters"], i2["iters"])


def test_ground_filter_errors(ctx):
    from paper_1801_08937_amd import mapmaker as mm
    p = synth.random_problem(28, n_side=8, n_samp=5000, n_int=3, half_bw=5, n_filters=1)
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
    gb = _ground_bins(p, 28, 9)
    args = (lp, p.interval_start, np.ones(p.n_intervals), p.interval_start, 1)
    for bad, nb in ((np.where(gb == 3, 9, gb), 9), (np.where(gb == 3, -2, gb), 9), (gb, 0)):
        with pytest.raises(mm.MapmakerError):
            ctx.polyfilter(*args, dev(bad.astype(np.int32)), nb)
    with pytest.raises(ValueError):
        ctx.polyfilter(*args, dev(gb[:-1]), 9)


@pytest.mark.parametrize("stokes", ["I", "QU"])
def test_filter_on_stokes_subset_pointing(ctx, stokes):
    """The template filter (with ground bins) as the weight of the I-only
    and QU-only systems of a detector pair's sum and difference streams:
    A, b and M_BD (1x1 / 2x2 blocks) against the oracle, and one M_BD solve
    to the true residual."""
    p = synth.random_problem(29, n_side=10, n_samp=20011, n_int=4, half_bw=5, n_filters=2,
                             flag_frac=0.05)
    psi = None if stokes == "I" else p.psi
    lp = ctx.pointing(dev(p.pix), None if psi is None else dev(psi), p.n_pix_total,
                      p.min_hits, stokes=stokes)
    op = O.pointing_build(p.pix, psi, p.n_pix_total, p.min_hits, stokes)
    sub = _subscans(p, 30)
    w = np.random.default_rng(31).uniform(0.5, 2.0, p.n_intervals)
    gb = _ground_bins(p, 32, 13)
    lf = ctx.polyfilter(lp, p.interval_start, w, sub, 2, dev(gb), 13)
    of = O.polyfilter_build(op, p.interval_start, w, sub, 2, gb, 13)
    assert lp.nc == len(stokes) and lp.n == op.n
    x = np.random.default_rng(33).standard_normal(op.n)
    assert maxrel(host(ctx.apply_A(lp, lf, dev(x))), O.apply_A(op, of, x)) <= TOL_OP
    b = ctx.rhs(lp, lf, dev(p.tod))
    assert maxrel(host(b), O.rhs(op, of, p.tod)) <= TOL_OP
    M = ctx.mbd(lp, lf)
    assert maxrel(host(ctx.precond_apply(M, dev(x))), O.mbd_apply(O.mbd_build(op, of), x)) <= TOL_OP
    xs, info = ctx.solve(lp, lf, M, b, tol=1e-10, max_iter=3000)
    assert info["converged"] and info["rel_res_true"] <= 1e-9, info


def test_arnoldi_residual_stop_rule_vs_oracle(ctx):
    """Arnoldi under the residual stop rule (App. A: the error term of
    Eq. factoriz applied to the Arnoldi solution of B x = r_0) on a weakly
    cross-linked scan (passes 5 degrees apart) filtered by offset + slope per
    sweep: the GPU and the oracle stop at the same step (a crossing within
    1e-6 of eps may move it by one), their residual histories agree to 1e-6,
    the library's stop is the first step at or below eps, and Z spans the
    oracle's space.  The literal rule h_{j+1,j} <= eps does not stop on this
    problem (h stays near 0.2)."""
    import scipy.linalg
    p = synth.config2(n_side=16, grid=(2, 2), samp_per_det=1536, L=768, half_bw=8,
                      angles_deg=(0.0, 5.0, -5.0))
    lp, _, op, _ = build_both(ctx, p)
    sub = np.arange(0, p.n_samp + 1, 16)
    w = np.ones(p.n_intervals)
    lf = ctx.polyfilter(lp, p.interval_start, w, sub, 1)
    of = O.polyfilter_build(op, p.interval_start, w, sub, 1)
    M = ctx.mbd(lp, lf)
    OM = O.mbd_build(op, of)
    x0 = synth.rng_for(2, 31, synth.STREAM_SIGNAL).standard_normal(op.n_obs * op.nc)
    b = O.rhs(op, of, p.tod) - O.apply_A(op, of, x0)
    k = 10
    for eps in (1e-3, 1e-6, 1e-9):
        print(f"[residual rule] eps {eps:g}", flush=True)
        M2 = ctx.defl_build(lp, lf, M, dev(b), k=k, eps_arn=eps, m_max=200, stop="residual")
        OM2, res, theta = O.defl_build(op, of, OM, b, k, eps, 200, stop="residual")
        m = M2.arnoldi_info.m
        rg = M2.res_history
        assert rg.shape[0] == m and rg[-1] <= eps and np.all(rg[:-1] > eps)
        j = min(m, res.m)
        np.testing.assert_allclose(rg[:j], res.res[:j], rtol=1e-6, atol=0)
        if abs(res.res[res.m - 1] - eps) > 1e-6 * eps and \
                (res.m < 2 or abs(res.res[res.m - 2] - eps) > 1e-6 * eps):
            assert m == res.m, (eps, m, res.m)
        else:
            assert abs(m - res.m) <= 1
        th = np.sort(theta.real)
        Zg = host(M2.export()[0])
        if m == res.m and th[k] - th[k - 1] > 1e-3 * th[k]:
            s = scipy.linalg.subspace_angles(Zg, OM2.Z)
            assert np.max(np.sin(s)) <= 1e-6, (eps, np.max(np.sin(s)))
        del M2
    Mh = ctx.defl_build(lp, lf, M, dev(b), k=k, eps_arn=1e-6, m_max=200, stop="h")
    assert Mh.arnoldi_info.m == 200
    np.testing.assert_allclose(Mh.res_history[:60], res.res[:60], rtol=1e-6, atol=0)
