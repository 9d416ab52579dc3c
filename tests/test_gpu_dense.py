"""The FP64 MFMA products of the coarse build and of block PCG (E = Z^T AZ,
Z = W_m Y, the block Gram and update products) through the C ABI, against
numpy's FP64 matrix product (a library routine) on tall skinny shapes with
ragged row counts, at the path's shapes."""
import numpy as np
import pytest

from gpu_util import dev, host, maxrel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1801_08937_amd import mapmaker as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,ka,kb", [(1, 1, 1), (77, 5, 3), (3072, 64, 64), (100003, 32, 32),
                                     (196608, 32, 17)])
def test_dense_gram(ctx, n, ka, kb):
    import torch
    rng = np.random.default_rng(n + ka)
    X = rng.standard_normal((n, ka))
    Y = rng.standard_normal((n, kb))
    ref = X.T @ Y
    # column-major storage (Z, AZ) and column-batched rows (block CG)
    Xc = dev(X.T.copy()).t()
    Yc = dev(Y.T.copy()).t()
    C1 = ctx.dense_gram(Xc, Yc)
    assert maxrel(host(C1), ref) <= 1e-12
    C2 = ctx.dense_gram(dev(X), dev(Y))
    assert maxrel(host(C2), ref) <= 1e-12
    assert torch.equal(C1, ctx.dense_gram(Xc, Yc))


@pytest.mark.parametrize("n,kin,kout", [(5, 3, 2), (3072, 256, 32), (100003, 60, 64)])
def test_dense_tall(ctx, n, kin, kout):
    rng = np.random.default_rng(kin)
    V = rng.standard_normal((n, kin))
    Y = rng.standard_normal((kin, kout))
    Z = host(ctx.dense_tall(dev(V), dev(Y)))
    assert maxrel(Z, V @ Y) <= 1e-12


@pytest.mark.parametrize("n,R", [(3, 2), (3072, 64), (50001, 16)])
def test_dense_rows(ctx, n, R):
    import torch
    rng = np.random.default_rng(R)
    In = rng.standard_normal((n, R))
    S = rng.standard_normal((R, R))
    O0 = rng.standard_normal((n, R))
    out = dev(O0)
    ctx.dense_rows(dev(In), dev(S), out=out, alpha=0.5, beta=-2.0)
    assert maxrel(host(out), -2.0 * O0 + 0.5 * In @ S) <= 1e-12
    assert maxrel(host(ctx.dense_rows(dev(In), dev(S))), In @ S) <= 1e-12


def test_dense_errors(ctx):
    import torch
    from paper_1801_08937_amd import mapmaker as mm
    X = torch.zeros(10, 65, dtype=torch.float64, device="cuda")
    with pytest.raises(mm.MapmakerError):
        ctx.dense_gram(X, X)
    with pytest.raises(mm.MapmakerError):
        ctx.dense_rows(torch.zeros(10, 3, dtype=torch.float64, device="cuda"),
                       torch.zeros(3, 3, dtype=torch.float64, device="cuda"))
