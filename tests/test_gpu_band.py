"""GPU parity of the direct banded N^-1 (Sect. 2: the inverse noise
correlation kept to lambda lags on each side, truncated at interval edges)
where its filter is walked in several LDS chunks: long bands with one
column, and many columns with short chunks.  Against the oracle's direct
sum, lag by lag."""
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


def _band_problem(lam, n_int, seed, n_filters=3):
    """Ragged intervals from just above 2 lambda + 1 up to several filter
    lengths, so tiles straddle interval ends and some intervals hold fewer
    samples than one tile."""
    rng = np.random.default_rng(seed)
    lo = 2 * lam + 2
    lengths = rng.integers(lo, 4 * lo, n_int).astype(np.int64)
    lengths[0] = lo
    istart = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    fid = rng.integers(0, n_filters, n_int).astype(np.int32)
    band = np.stack([synth.band_from_psd(4 * lo, lam, fk)
                     for fk in rng.uniform(0.05, 1, n_filters)])
    return istart, fid, band


@pytest.mark.parametrize("lam", [2000, 3100])
def test_band_long_filter_one_column(ctx, lam):
    """One column: FP64 chunks hold 3072 taps, so lambda 2000 takes two
    chunks and lambda 3100 three (the last a partial one)."""
    istart, fid, band = _band_problem(lam, 4, lam)
    nz = ctx.noise(istart, fid, band, lam, method=1)
    assert nz.method == 1
    on = O.noise_build(istart, fid, band, lam)
    y = np.random.default_rng(1).standard_normal(int(istart[-1]))
    z = host(ctx.noise_apply(nz, dev(y)))
    ref = O.noise_apply_direct(on, y)
    assert maxrel(z, ref) <= TOL_OP, maxrel(z, ref)


def test_band_long_filter_fp32(ctx):
    """FP32 chunks hold 7168 taps: lambda 4000 takes two."""
    lam = 4000
    istart, fid, band = _band_problem(lam, 3, 7)
    nz = ctx.noise(istart, fid, band, lam, method=1, prec=1)
    on = O.noise_build(istart, fid, band, lam)
    y = np.random.default_rng(2).standard_normal(int(istart[-1]))
    z = host(ctx.noise_apply(nz, dev(y.astype(np.float32))))
    assert rel(z, O.noise_apply_direct(on, y)) <= 1e-5


@pytest.mark.parametrize("lam,R", [(100, 64), (100, 8), (400, 8), (700, 16), (33, 32)])
def test_band_chunked_columns(ctx, lam, R):
    """R columns: the window takes R values per row, so chunks shrink (88
    taps at R = 64, 680 at R = 8).  Every column matches the oracle, and
    equals the single-column apply bitwise: each output sums its taps in
    the same order whatever R and the chunk length."""
    istart, fid, band = _band_problem(lam, 5, 100 * R + lam)
    nz = ctx.noise(istart, fid, band, lam, method=1)
    on = O.noise_build(istart, fid, band, lam)
    n = int(istart[-1])
    Y = np.random.default_rng(R).standard_normal((n, R))
    Z = host(ctx.noise_apply(nz, dev(Y.reshape(-1)), nrhs=R)).reshape(n, R)
    for c in (0, R // 2, R - 1):
        ref = O.noise_apply_direct(on, Y[:, c])
        assert maxrel(Z[:, c], ref) <= TOL_OP, (c, maxrel(Z[:, c], ref))
        z1 = host(ctx.noise_apply(nz, dev(Y[:, c].copy())))
        np.testing.assert_array_equal(Z[:, c], z1)


def test_band_columns_do_not_mix(ctx):
    """Changing the other columns leaves a column's output bitwise unchanged."""
    lam, R = 150, 32
    istart, fid, band = _band_problem(lam, 4, 11)
    nz = ctx.noise(istart, fid, band, lam, method=1)
    n = int(istart[-1])
    rng = np.random.default_rng(12)
    Y = rng.standard_normal((n, R))
    Y2 = rng.standard_normal((n, R))
    Y2[:, 5] = Y[:, 5]
    Z = host(ctx.noise_apply(nz, dev(Y.reshape(-1)), nrhs=R)).reshape(n, R)
    Z2 = host(ctx.noise_apply(nz, dev(Y2.reshape(-1)), nrhs=R)).reshape(n, R)
    np.testing.assert_array_equal(Z[:, 5], Z2[:, 5])
