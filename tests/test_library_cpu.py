"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-only pieces (the Ritz eigensolver) are right.
No kernel is launched here."""
import ctypes
import os

import numpy as np
import pytest

from paper_1801_08937_amd import mapmaker as mm


def test_library_loads_and_exports_header_symbols():
    L = mm.lib()
    assert L.mm_version().startswith(b"mapmaker")
    syms = mm.header_symbols()
    assert len(syms) >= 25
    raw = ctypes.CDLL(mm.LIB_PATH)
    missing = [s for s in syms if not hasattr(raw, s)]
    assert not missing, missing


def test_header_is_c_compilable(tmp_path):
    """The public header compiles as plain C (no C++ or HIP types leak in)."""
    import subprocess
    src = tmp_path / "t.c"
    src.write_text('#include "mapmaker.h"\nint main(void){mm_solve_info i; (void)i; return 0;}\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I",
                        os.path.dirname(mm.HEADER), "-c", str(src), "-o", str(tmp_path / "t.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("seed,m", [(0, 5), (1, 40), (2, 120), (3, 200)])
def test_hessenberg_eig_vs_lapack(seed, m):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((m, m)), -1)
    w, V = mm.hessenberg_eig(H)
    ref = np.linalg.eigvals(H)
    # same multiset of eigenvalues, ordered by (real, imag)
    order = np.lexsort((ref.imag, ref.real))
    np.testing.assert_allclose(w, ref[order], rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    for i in range(m):
        r = np.linalg.norm(H @ V[:, i] - w[i] * V[:, i])
        assert r <= 1e-8 * np.abs(H).max(), (i, r)
        assert abs(np.linalg.norm(V[:, i]) - 1) < 1e-12


def test_hessenberg_eig_arnoldi_like_spectrum():
    """A Hessenberg matrix from an Arnoldi run on an SPD-similar operator:
    eigenvalues real, clustered near 1 with a few small ones (the M_BD A case)."""
    rng = np.random.default_rng(7)
    n = 60
    ev = np.concatenate([np.geomspace(1e-4, 1e-1, 6), 1 + 0.1 * rng.standard_normal(n - 6)])
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    S = rng.standard_normal((n, n)) * 0.05 + np.eye(n)
    B = S @ Q @ np.diag(ev) @ Q.T @ np.linalg.inv(S)
    # Arnoldi to full size
    W = np.zeros((n, n))
    H = np.zeros((n, n))
    w = rng.standard_normal(n)
    W[:, 0] = w / np.linalg.norm(w)
    for j in range(n):
        v = B @ W[:, j]
        for _ in range(2):
            h = W[:, :j + 1].T @ v
            v -= W[:, :j + 1] @ h
            H[:j + 1, j] += h
        if j + 1 < n:
            H[j + 1, j] = np.linalg.norm(v)
            W[:, j + 1] = v / H[j + 1, j]
    w_, V = mm.hessenberg_eig(H)
    np.testing.assert_allclose(np.sort(w_.real), np.sort(ev), rtol=1e-6, atol=1e-9)


def test_graft_entry_exposes_build_and_smoke(root_dir):
    import importlib.util
    spec = importlib.util.spec_from_file_location("ge", os.path.join(root_dir, "__graft_entry__.py"))
    ge = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(ge)
    assert callable(ge.build) and callable(ge.smoke)


def test_hessenberg_eig_clustered_tridiagonals():
    """Symmetric tridiagonals (Lanczos-like) with tight clusters of equal
    diagonal entries and tiny couplings, where a QR iteration with shifts
    that do not track the cluster stalls: eigenvalues against LAPACK's
    eigvalsh, eigenpair residuals small."""
    rng = np.random.default_rng(0)
    for _ in range(120):
        m = int(rng.integers(2, 160))
        d = rng.choice([1.0, 2.0, 3.0], m) + rng.standard_normal(m) * 10.0 ** rng.integers(-16, 0)
        e = rng.standard_normal(m - 1) * 10.0 ** rng.integers(-18, 0)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        w, V = mm.hessenberg_eig(T)
        ref = np.linalg.eigvalsh(T)
        tn = np.abs(T).max()
        assert np.max(np.abs(np.sort(w.real) - ref)) <= 1e-9 * tn
        assert np.max(np.abs(w.imag)) <= 1e-9 * tn
        for i in range(0, m, max(1, m // 8)):
            v = V[:, i]
            assert np.linalg.norm(T @ v - w[i] * v) <= 1e-7 * tn * np.linalg.norm(v)


def test_hessenberg_eig_converged_arnoldi_with_template_filter():
    """H from an Arnoldi run to numerical convergence on M_BD A with white
    noise and few filter templates (M_BD A = I minus a low-rank term: most
    Ritz values cluster at 1), the regime of the eps_Arn study."""
    import oracle as O
    import synth
    p = synth.config2(n_side=32, grid=(4, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=10)
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    pf = O.polyfilter_build(op, p.interval_start, np.ones(p.n_intervals),
                            np.arange(0, p.n_samp + 1, 512), 1)
    M = O.mbd_build(op, pf)
    u = np.random.default_rng(1).uniform(-1, 1, op.n)
    res = O.arnoldi(lambda w: O.mbd_apply(M, O.apply_A(op, pf, w)),
                    O.mbd_apply(M, O.apply_A(op, pf, u)), 200, 1e-14)
    assert res.m < 200 and res.h_last <= 1e-14   # numerical convergence
    for m in (res.m // 2, res.m - 5, res.m):
        H = res.H[:m, :m]
        w, V = mm.hessenberg_eig(H)
        hn = np.abs(H).max()
        ref = np.linalg.eigvals(H)
        np.testing.assert_allclose(np.sort(w.real), np.sort(ref.real), atol=1e-7 * hn)
        for i in range(m):
            assert np.linalg.norm(H @ V[:, i] - w[i] * V[:, i]) <= 1e-7 * hn
