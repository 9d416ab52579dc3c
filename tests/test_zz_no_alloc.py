"""mm_apply_A_noalloc (the A apply that allocates nothing, its temporaries in
the library's static per-GPU scratch array) against mm_apply_A through the C
ABI: bitwise the same on consecutive calls of different sizes and layouts,
interleaved with the allocating entry point, and oversize problems rejected."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import build_both, dev, host, maxrel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1801_08937_amd import mapmaker
    return mapmaker


def _both_applies(ctx, lp, ln, n, nrhs, seed):
    import torch
    x = dev(np.random.default_rng(seed).standard_normal(n * nrhs))
    y0 = torch.full_like(x, np.nan)
    used = ctx.apply_A_noalloc(lp, ln, x, y0, nrhs=nrhs)
    y1 = ctx.apply_A(lp, ln, x, nrhs=nrhs)
    return x, y0, y1, used


def test_noalloc_matches_apply_A_two_calls(mm):
    """Two calls in a row, the second on a smaller problem (and a different
    layout), each bitwise equal to mm_apply_A; the first also within 1e-12
    of the oracle."""
    import torch
    ctx = mm.Context(0)
    cap = mm.lib().mm_apply_A_noalloc_max_bytes()
    assert cap == 128 << 20
    # 1: config 1 with the grid hint (map copies for P, sliced P^T partial maps)
    p = synth.config1()
    lp, ln, op, on = build_both(ctx, p)
    lp.set_grid(p.n_side)
    x, y0, y1, used = _both_applies(ctx, lp, ln, op.n, 1, 1)
    print(f"config 1: scratch {used} B of {cap}")
    assert 0 < used <= cap
    assert torch.equal(y0, y1)
    assert maxrel(host(y0), O.apply_A(op, on, host(x))) <= 1e-12
    # 2: a smaller random problem (no grid): stale scratch from call 1 must not leak in
    q = synth.random_problem(3, n_side=6, n_samp=5003, n_int=3, half_bw=7, n_filters=2)
    lq, lnq, oq, onq = build_both(ctx, q)
    x, y0, y1, used2 = _both_applies(ctx, lq, lnq, oq.n, 1, 2)
    assert 0 < used2 < used
    assert torch.equal(y0, y1)
    assert maxrel(host(y0), O.apply_A(oq, onq, host(x))) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("case", ["fft", "nrhs8", "fp32", "filter"])
def test_noalloc_layouts(mm, case):
    """FFT N^-1, several columns, the FP32 form and the template filter with
    ground bins (the filter's own scratch), each bitwise equal to mm_apply_A,
    with an allocating apply in between."""
    import torch
    ctx = mm.Context(0)
    if case == "fft":
        p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=300)
        lp, ln, op, on = build_both(ctx, p, method=2)
        lp.set_grid(p.n_side)
        nrhs = 1
    elif case == "nrhs8":
        p = synth.config1()
        lp, ln, op, on = build_both(ctx, p)
        nrhs = 8
    elif case == "fp32":
        p = synth.config1()
        lp, ln, op, on = build_both(ctx, p, prec=1)
        lp.set_grid(p.n_side)
        nrhs = 1
    else:
        p = synth.random_problem(21, n_side=12, n_samp=30011, n_int=5, half_bw=5, n_filters=2,
                                 flag_frac=0.1)
        lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, p.min_hits)
        op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
        sub = np.arange(0, p.n_samp + 1, 97, dtype=np.int64)
        sub[-1] = p.n_samp
        sub = np.unique(np.concatenate([sub, p.interval_start]))
        gb = np.random.default_rng(5).integers(-1, 9, p.n_samp).astype(np.int32)
        w = np.ones(p.n_intervals)
        ln = ctx.polyfilter(lp, p.interval_start, w, sub, 2, dev(gb), 9)
        on = O.polyfilter_build(op, p.interval_start, w, sub, 2, gb, 9)
        nrhs = 1
    x, y0, y1, used = _both_applies(ctx, lp, ln, op.n, nrhs, 7)
    assert 0 < used <= mm.lib().mm_apply_A_noalloc_max_bytes()
    assert torch.equal(y0, y1)
    # an allocating apply of another vector, then the no-alloc one again
    _ = ctx.apply_A(lp, ln, dev(np.random.default_rng(8).standard_normal(op.n * nrhs)), nrhs=nrhs)
    y2 = torch.full_like(x, np.nan)
    ctx.apply_A_noalloc(lp, ln, x, y2, nrhs=nrhs)
    assert torch.equal(y2, y1)
    if nrhs == 1:
        bar = 1e-5 if case == "fp32" else 1e-11
        assert maxrel(host(y0), O.apply_A(op, on, host(x))) <= bar
    ctx.close()


def test_noalloc_allocates_nothing_and_rejects_oversize(mm):
    """On a fresh context (empty workspaces) a no-alloc apply leaves the
    device's free memory unchanged; a problem above the scratch maximum is
    rejected with MM_E_INVALID and the context stays usable."""
    import torch
    ctx = mm.Context(0)
    p = synth.config1()
    lp, ln, op, on = build_both(ctx, p)
    x = dev(np.random.default_rng(1).standard_normal(op.n))
    y = torch.empty_like(x)
    ctx.apply_A_noalloc(lp, ln, x, y)           # first launches load the kernels
    torch.cuda.synchronize()
    ctx2 = mm.Context(0)
    lp2, ln2, _, _ = build_both(ctx2, p)
    y2 = torch.empty_like(x)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx2.apply_A_noalloc(lp2, ln2, x, y2)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"free device memory before/after: {free0} / {free1}")
    assert free1 == free0
    assert torch.equal(y, y2)
    # 140,000 samples x 64 columns x 8 B x 2 TOD vectors > 128 MiB
    q = synth.random_problem(4, n_side=8, n_samp=140000, n_int=2, half_bw=4, n_filters=1)
    lq, lnq, oq, onq = build_both(ctx2, q)
    X = dev(np.zeros(oq.n * 64))
    with pytest.raises(mm.MapmakerError) as e:
        ctx2.apply_A_noalloc(lq, lnq, X, torch.empty_like(X), nrhs=64)
    assert e.value.name == "MM_E_INVALID" and "maximum" in str(e.value)
    y3 = torch.empty_like(x)
    ctx2.apply_A_noalloc(lp2, ln2, x, y3)
    assert torch.equal(y3, y)
    ctx2.close()
    ctx.close()
