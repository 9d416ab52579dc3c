"""Pins for the FP64 oracle: each test checks it against something other than
itself -- brute force on tiny inputs, a library routine for a special case,
a closed form, a hand-derived value or an identity the paper states.

Sizes are tiny so the whole file runs in seconds on the CPU.
"""
import json
import math
import os
from collections import defaultdict

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _setup(seed=0, **kw):
    p = synth.random_problem(seed, **kw)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    return p, pt, nz


def _dense_P_test(pix, psi, cidx):
    """P written from Eq. datamodel with math.cos/math.sin, independent of the
    oracle's vectorised gather."""
    n_obs = int(cidx.max()) + 1 if cidx.size and cidx.max() >= 0 else 0
    P = np.zeros((len(pix), 3 * n_obs))
    for t, (p, ph) in enumerate(zip(pix, psi)):
        if p >= 0 and cidx[p] >= 0:
            j = cidx[p]
            P[t, 3 * j: 3 * j + 3] = (1.0, math.cos(2 * ph), math.sin(2 * ph))
    return P


def _dense_N_scipy(p):
    """Block-diagonal N^-1 from scipy.linalg.toeplitz, one block per interval."""
    blocks = []
    for i in range(p.n_intervals):
        L = int(p.interval_start[i + 1] - p.interval_start[i])
        col = np.zeros(L)
        c = p.band[p.filter_id[i]]
        m = min(L, p.half_bw + 1)
        col[:m] = c[:m]
        blocks.append(scipy.linalg.toeplitz(col))
    return scipy.linalg.block_diag(*blocks)


# ---------------------------------------------------------------- pointing (O1)

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pointing_bruteforce(seed):
    p = synth.random_problem(seed, n_side=5, n_samp=700, flag_frac=0.1, min_hits=30)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    hits = defaultdict(int)
    for q in p.pix:
        if q >= 0:
            hits[int(q)] += 1
    assert [hits[q] for q in range(p.n_pix_total)] == pt.hits.tolist()
    obs = sorted(q for q in range(p.n_pix_total) if hits[q] >= p.min_hits)
    assert obs == pt.obs_pix.tolist()
    assert len(obs) < p.n_pix_total  # the threshold actually dropped pixels here
    pairs = sorted((obs.index(int(q)), t) for t, q in enumerate(p.pix) if q >= 0 and int(q) in obs)
    assert [t for _, t in pairs] == pt.perm.tolist()
    off = [0]
    for q in obs:
        off.append(off[-1] + hits[q])
    assert off == pt.off.tolist()
    assert pt.off[-1] == pt.perm.shape[0] == int(np.sum(pt.j >= 0))
    for t, q in enumerate(p.pix):
        exp = obs.index(int(q)) if q >= 0 and int(q) in obs else -1
        assert pt.j[t] == exp


def test_pointing_rejects_bad_pixels():
    with pytest.raises(O.OracleError):
        O.pointing_build(np.array([0, 5]), np.zeros(2), 4)
    with pytest.raises(O.OracleError):
        O.pointing_build(np.array([0, -2]), np.zeros(2), 4)


# ---------------------------------------------------------------- P, P^T (O3, O4)

@pytest.mark.parametrize("seed", [0, 3])
def test_P_PT_dense(seed):
    p, pt, nz = _setup(seed, n_side=4, n_samp=400, n_int=3, half_bw=4)
    P = _dense_P_test(p.pix, p.psi, pt.cidx)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(pt.n)
    y = rng.standard_normal(pt.n_samp)
    np.testing.assert_allclose(O.apply_P(pt, x), P @ x, rtol=1e-14, atol=1e-13)
    np.testing.assert_allclose(O.apply_PT(pt, y), P.T @ y, rtol=1e-13, atol=1e-12)


def test_P_PT_adjoint():
    p, pt, nz = _setup(4, n_side=6, n_samp=3000)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(pt.n)
    y = rng.standard_normal(pt.n_samp)
    lhs = O.apply_P(pt, x) @ y
    rhs = x @ O.apply_PT(pt, y)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_P_matches_generator_data_model():
    """Noiseless TOD from the generator's own data model equals P s."""
    p = synth.config1(noiseless=True)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    s = p.signal[pt.obs_pix].reshape(-1)
    np.testing.assert_allclose(O.apply_P(pt, s), p.tod, rtol=0, atol=1e-12)


def test_golden_one_pixel():
    g = _golden("one_pixel_binned_map.json")
    pt = O.pointing_build(np.array(g["pix"]), np.array(g["psi"]), 1, 1)
    nz = O.noise_build([0, 4], [0], [[1.0]], 0)
    np.testing.assert_allclose(O.apply_P(pt, g["iqu"]), g["tod"], atol=1e-13)
    np.testing.assert_allclose(O.apply_PT(pt, g["tod"]), g["PT_d"], atol=1e-13)
    M = O.mbd_build(pt, nz)
    np.testing.assert_allclose(M.blocks[0], g["block"], atol=1e-14)
    b = O.rhs(pt, nz, g["tod"])
    np.testing.assert_allclose(O.mbd_apply(M, b), g["binned"], atol=1e-13)


# ---------------------------------------------------------------- N^-1 (O2)

def test_golden_toeplitz():
    g = _golden("toeplitz_band_3x.json")
    nz = O.noise_build(g["interval_start"], g["filter_id"], g["band"], g["half_bw"])
    np.testing.assert_allclose(O.noise_apply_direct(nz, g["y"]), g["z"], atol=1e-15)
    np.testing.assert_allclose(O.noise_apply_fft(nz, g["y"]), g["z"], atol=1e-13)


@pytest.mark.parametrize("seed", [0, 5])
def test_noise_vs_scipy_toeplitz(seed):
    p, pt, nz = _setup(seed, n_samp=600, n_int=4, half_bw=20, n_filters=3)
    N = _dense_N_scipy(p)
    y = np.random.default_rng(seed).standard_normal(p.n_samp)
    ref = N @ y
    np.testing.assert_allclose(O.noise_apply_direct(nz, y), ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.noise_apply_fft(nz, y), ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(O.dense_Ninv(nz), N)


def test_noise_fft_vs_direct_large_band():
    p = synth.config2(n_side=32, grid=(2, 2), samp_per_det=1 << 12, L=1 << 11, half_bw=512)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    y = np.random.default_rng(0).standard_normal(p.n_samp)
    a = O.noise_apply_direct(nz, y)
    b = O.noise_apply_fft(nz, y)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_noise_symmetric_and_positive_symbol():
    p = synth.config1()
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal((2, p.n_samp))
    a = O.noise_apply_direct(nz, u) @ v
    b = u @ O.noise_apply_direct(nz, v)
    assert abs(a - b) <= 1e-12 * abs(a)
    c = p.band[0]
    lam = p.half_bw
    w = np.linspace(0, np.pi, 8 * lam + 1)
    sym = c[0] + 2 * np.sum(c[1:, None] * np.cos(np.arange(1, lam + 1)[:, None] * w[None, :]), axis=0)
    assert sym.min() > 0
    # a section's eigenvalues lie within the symbol's range
    T = scipy.linalg.toeplitz(np.concatenate([c, np.zeros(400 - lam - 1)]))
    ev = np.linalg.eigvalsh(T)
    assert ev.min() >= sym.min() * (1 - 1e-9) and ev.max() <= sym.max() * (1 + 1e-9)


def test_noise_rejects_bad_intervals():
    with pytest.raises(O.OracleError):
        O.noise_build([0, 5, 4], [0, 0], [[1.0, 0.1]], 1)
    with pytest.raises(O.OracleError):
        O.noise_build([0, 4, 8], [0, 0], [[1.0, 0.1, 0.1]], 2)


# ---------------------------------------------------------------- A, b (O5, O6)

def test_A_dense_spd():
    p, pt, nz = _setup(6, n_side=3, n_samp=480, n_int=3, half_bw=10)
    P = _dense_P_test(p.pix, p.psi, pt.cidx)
    N = _dense_N_scipy(p)
    A = P.T @ N @ P
    cols = np.stack([O.apply_A(pt, nz, e) for e in np.eye(pt.n)], axis=1)
    np.testing.assert_allclose(cols, A, rtol=1e-12, atol=1e-11 * np.abs(A).max())
    np.testing.assert_allclose(cols, cols.T, rtol=0, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_apply_A_pixels_matches_full_product():
    p, pt, nz = _setup(14, n_side=5, n_samp=1500, n_int=3, half_bw=30, flag_frac=0.1)
    x = np.random.default_rng(3).standard_normal(pt.n)
    full = O.apply_A(pt, nz, x).reshape(-1, 3)
    pix = [0, 3, pt.n_obs - 1]
    np.testing.assert_allclose(O.apply_A_pixels(pt, nz, x, pix), full[pix], rtol=1e-12,
                               atol=1e-12 * np.abs(full).max())


def test_b_noiseless_equals_A_s():
    p = synth.config1(noiseless=True)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    s = p.signal[pt.obs_pix].reshape(-1)
    b = O.rhs(pt, nz, p.tod)
    As = O.apply_A(pt, nz, s)
    assert np.linalg.norm(b - As) <= 1e-13 * np.linalg.norm(b)


def test_rhs_masks_flagged_samples():
    p, pt, nz = _setup(7, n_side=4, n_samp=500, flag_frac=0.2, n_int=2, half_bw=5)
    d = p.tod.copy()
    d[pt.j < 0] = 1e6  # garbage on flagged samples must not leak into b
    b1 = O.rhs(pt, nz, d)
    d[pt.j < 0] = 0.0
    np.testing.assert_array_equal(b1, O.rhs(pt, nz, d))


# ---------------------------------------------------------------- M_BD (O7)

def test_mbd_inverse_and_white_noise_closed_form():
    """With lambda = 0 (white noise) A = M_BD^-1, so PCG with M_BD stops after
    one iteration at the binned map B_j^-1 sum_t c0 w_t d_t (noiseless: s)."""
    p = synth.random_problem(8, n_side=4, n_samp=800, half_bw=0, n_int=2, noiseless=True)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band[:, :1], 0)
    M = O.mbd_build(pt, nz)
    for j in range(pt.n_obs):
        np.testing.assert_allclose(M.blocks[j] @ M.inv[j], np.eye(3), atol=1e-12)
    P = _dense_P_test(p.pix, p.psi, pt.cidx)
    c0 = np.concatenate([np.full(int(p.interval_start[i + 1] - p.interval_start[i]),
                                 p.band[p.filter_id[i], 0]) for i in range(p.n_intervals)])
    A_dense = P.T @ (c0[:, None] * P)
    Minv_dense = scipy.linalg.block_diag(*M.blocks)
    np.testing.assert_allclose(A_dense, Minv_dense, rtol=1e-12, atol=1e-12)
    b = O.rhs(pt, nz, p.tod)
    x, info = O.pcg(lambda v: O.apply_A(pt, nz, v), lambda v: O.mbd_apply(M, v), b, 1e-12, 50)
    assert info.iters == 1
    np.testing.assert_allclose(x, p.signal[pt.obs_pix].reshape(-1), rtol=1e-10, atol=1e-10)


def test_mbd_singular_block_detected():
    # three hits at the same angle: rank-1 block
    pix = np.array([0, 0, 0, 1, 1, 1, 1])
    psi = np.array([0.3, 0.3, 0.3, 0.0, 0.5, 1.0, 1.5])
    pt = O.pointing_build(pix, psi, 2, 3)
    nz = O.noise_build([0, 7], [0], [[1.0]], 0)
    with pytest.raises(O.OracleError) as e:
        O.mbd_build(pt, nz)
    assert e.value.code == "SINGULAR_BLOCK"


# ---------------------------------------------------------------- M_2l (O8)

def _small_c1_like():
    p = synth.config2(n_side=16, grid=(2, 2), samp_per_det=1 << 10, L=1 << 9, half_bw=32)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    return p, pt, nz


def test_arnoldi_factorisation_gives_AZ():
    """App. A, Eq. factoriz with B = M_BD A: B W_m = W_{m+1} Hbar_m, so
    A W_m = M_BD^-1 W_{m+1} Hbar_m with M_BD^-1 the assembled blocks B_j.  For
    Z = W_m Y R^-1 (Ritz vectors, orthonormalised) A Z then follows from the
    factorisation alone and equals A Z applied directly: the reading by which
    AZ of an Arnoldi-built M_2l is formed (R26).  A sign or index slip in the
    Hessenberg matrix or the basis breaks the first identity."""
    p, pt, nz = _small_c1_like()
    M = O.mbd_build(pt, nz)
    nc = M.blocks.shape[1]
    b = np.random.default_rng(11).standard_normal(pt.n)
    res = O.arnoldi(lambda w: O.mbd_apply(M, O.apply_A(pt, nz, w)), O.mbd_apply(M, b), 40, 1e-300)
    m, W, H = res.m, res.W, res.H
    assert m == 40 and W.shape[1] == m + 1

    def blocks_apply(V):
        V = V.reshape(-1, nc, V.shape[-1])
        return np.einsum("jab,jbk->jak", M.blocks, V).reshape(-1, V.shape[-1])
    AW = np.stack([O.apply_A(pt, nz, W[:, j]) for j in range(m)], axis=1)
    AW_fact = blocks_apply(W[:, :m + 1] @ H[:m + 1, :m])
    assert np.max(np.abs(AW_fact - AW)) <= 1e-10 * np.max(np.abs(AW))
    theta, Y = O.ritz_select(H[:m, :m], 8)
    V = W[:, :m] @ Y
    Z, R = np.linalg.qr(V)
    YT = Y @ np.linalg.inv(R)
    AZ_fact = blocks_apply(W[:, :m + 1] @ (H[:m + 1, :m] @ YT))
    AZ = np.stack([O.apply_A(pt, nz, Z[:, c]) for c in range(Z.shape[1])], axis=1)
    assert np.max(np.abs(AZ_fact - AZ)) <= 1e-10 * np.max(np.abs(AZ))


def test_m2l_identities():
    p, pt, nz = _small_c1_like()
    M = O.mbd_build(pt, nz)
    rng = np.random.default_rng(3)
    k = 6
    Z = rng.standard_normal((pt.n, k))
    M2 = O.m2l_from_Z(pt, nz, M, Z)
    # Eq. ident: M_2l A Z = Z
    for c in range(k):
        out = O.m2l_apply(M2, O.apply_A(pt, nz, Z[:, c]))
        assert np.linalg.norm(out - Z[:, c]) <= 1e-9 * np.linalg.norm(Z[:, c])
    # R A Z = 0 with R = 1 - A Z E^-1 Z^T
    AZ = M2.AZ
    RAZ = AZ - AZ @ np.linalg.solve(M2.E, Z.T @ AZ)
    assert np.linalg.norm(RAZ) <= 1e-10 * np.linalg.norm(AZ)
    # M_2l A y = M_BD A y for y with Z^T A y = 0
    y = rng.standard_normal(pt.n)
    y = y - Z @ np.linalg.solve(M2.E, Z.T @ O.apply_A(pt, nz, y))
    Ay = O.apply_A(pt, nz, y)
    assert np.linalg.norm(Z.T @ Ay) <= 1e-9 * np.linalg.norm(Z) * np.linalg.norm(Ay)
    np.testing.assert_allclose(O.m2l_apply(M2, Ay), O.mbd_apply(M, Ay),
                               rtol=1e-8, atol=1e-9 * np.abs(O.mbd_apply(M, Ay)).max())
    # invariance under Z -> Z G
    G = rng.standard_normal((k, k)) + 3 * np.eye(k)
    M3 = O.m2l_from_Z(pt, nz, M, Z @ G)
    v = rng.standard_normal(pt.n)
    a, b = O.m2l_apply(M2, v), O.m2l_apply(M3, v)
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(a)
    # k = 0 is M_BD
    M0 = O.m2l_from_Z(pt, nz, M, np.zeros((pt.n, 0)))
    np.testing.assert_array_equal(O.m2l_apply(M0, v), O.mbd_apply(M, v))


def test_m2l_exact_eigvecs_deflate_to_one():
    """With Z = exact eigenvectors of M_BD A, the deflated eigenvalues of
    M_2l A become 1 and the rest are unchanged."""
    p, pt, nz = _setup(9, n_side=3, n_samp=600, n_int=2, half_bw=12)
    M = O.mbd_build(pt, nz)
    B = np.stack([O.mbd_apply(M, O.apply_A(pt, nz, e)) for e in np.eye(pt.n)], axis=1)
    ev, V = np.linalg.eig(B)
    order = np.argsort(ev.real)
    ev, V = ev.real[order], V.real[:, order]
    k = 4
    M2 = O.m2l_from_Z(pt, nz, M, V[:, :k])
    C = np.stack([O.m2l_apply(M2, O.apply_A(pt, nz, e)) for e in np.eye(pt.n)], axis=1)
    ev2 = np.sort(np.linalg.eigvals(C).real)
    exp = np.sort(np.concatenate([np.ones(k), ev[k:]]))
    np.testing.assert_allclose(ev2, exp, rtol=1e-8, atol=1e-8)


def test_coarse_not_spd_detected():
    p, pt, nz = _small_c1_like()
    M = O.mbd_build(pt, nz)
    z = np.random.default_rng(0).standard_normal(pt.n)
    with pytest.raises(O.OracleError) as e:
        O.m2l_from_Z(pt, nz, M, np.stack([z, z], axis=1))
    assert e.value.code == "COARSE_NOT_SPD"


# ---------------------------------------------------------------- Arnoldi (O9)

def test_arnoldi_relations_and_full_spectrum():
    p, pt, nz = _setup(10, n_side=3, n_samp=600, n_int=2, half_bw=12)
    M = O.mbd_build(pt, nz)
    Bop = lambda w: O.mbd_apply(M, O.apply_A(pt, nz, w))
    Bd = np.stack([Bop(e) for e in np.eye(pt.n)], axis=1)
    b = O.rhs(pt, nz, p.tod)
    r0 = O.mbd_apply(M, b)
    res = O.arnoldi(Bop, r0, pt.n, 1e-300)
    m = res.m
    W = res.W
    # orthonormal basis
    G = W[:, :m].T @ W[:, :m]
    assert np.abs(G - np.eye(m)).max() <= 1e-12
    # Eq. factoriz: B W_m = W_m H_m + h_{m+1,m} w_{m+1} e_m^T
    H = res.H
    lhs = Bd @ W[:, :m]
    rhs_ = W[:, :m] @ H[:m, :m]
    if W.shape[1] > m:
        rhs_[:, m - 1] += H[m, m - 1] * W[:, m]
    assert np.abs(lhs - rhs_).max() <= 1e-12 * np.abs(Bd).max()
    # full Arnoldi: Ritz values = eigenvalues of M_BD A
    if m == pt.n:
        th = np.sort(np.linalg.eigvals(H[:m, :m]).real)
        ev = np.sort(np.linalg.eigvals(Bd).real)
        np.testing.assert_allclose(th, ev, rtol=1e-9)


def test_ritz_residual_identity():
    """||B v_i - theta_i v_i|| = |h_{m+1,m}| |e_m^T y_i| (Eq. ritz, read with
    y_i in place of v_i on the right)."""
    p, pt, nz = _small_c1_like()
    M = O.mbd_build(pt, nz)
    Bop = lambda w: O.mbd_apply(M, O.apply_A(pt, nz, w))
    b = O.rhs(pt, nz, p.tod)
    res = O.arnoldi(Bop, O.mbd_apply(M, b), 30, 1e-14)
    m = res.m
    theta, Y = np.linalg.eig(res.H[:m, :m])
    for i in range(0, m, 5):
        v = res.W[:, :m] @ Y[:, i]
        lhs = np.linalg.norm(np.array([Bop(v.real), Bop(v.imag)]).T @ np.array([1, 1j]) - theta[i] * v)
        rhs_ = abs(res.H[m, m - 1]) * abs(Y[m - 1, i])
        assert abs(lhs - rhs_) <= 1e-9 * max(1.0, np.linalg.norm(v))


def test_ritz_select_keeps_pairs():
    H = np.array([[1.0, -2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.0, 3.0]])
    theta, Y = O.ritz_select(H, 1)
    assert Y.shape[1] == 2   # the complex pair at Re = 1 is kept whole
    theta, Y = O.ritz_select(H, 3)
    assert Y.shape[1] == 3
    theta, Y = O.ritz_select(H, 0, eps_lambda=2.0)
    assert Y.shape[1] == 2


def test_fom_residual_is_the_true_residual_of_the_arnoldi_solution():
    """fom_residual (App. A, error term of Eq. factoriz applied to the
    Arnoldi solution) against r_0 - B W_j y_j formed by applying B itself,
    y_j = H_j^-1 ||r_0|| e_1, on a non-symmetric B, at every step."""
    rng = np.random.default_rng(41)
    n = 50
    B = np.eye(n) + 0.4 * rng.standard_normal((n, n)) / np.sqrt(n)
    r0 = rng.standard_normal(n)
    res = O.arnoldi(lambda w: B @ w, r0, 30, 0.0)
    beta = np.linalg.norm(r0)
    for j in range(1, res.m + 1):
        y = np.linalg.solve(res.H[:j, :j], beta * np.eye(j)[:, 0])
        true = np.linalg.norm(r0 - B @ (res.W[:, :j] @ y)) / beta
        assert abs(res.res[j - 1] - true) <= 1e-9 * max(true, 1e-6), (j, res.res[j - 1], true)
    assert res.res[-1] < 1e-8 * res.res[0]


def test_fom_residual_equals_cg_residual_on_spd():
    """For symmetric positive definite B the Arnoldi (full orthogonalisation)
    solution is the conjugate-gradient iterate, so the residual history of
    the residual stop rule must be CG's ||r_j|| / ||r_0|| step by step."""
    rng = np.random.default_rng(42)
    n = 80
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    B = Q @ np.diag(np.geomspace(1e-2, 1.0, n)) @ Q.T
    r0 = rng.standard_normal(n)
    res = O.arnoldi(lambda w: B @ w, r0, 25, 0.0)
    _, info = O.pcg(lambda x: B @ x, lambda r: r, r0, 0.0, 25)
    np.testing.assert_allclose(res.res, info.history[1:26], rtol=1e-7)


def test_arnoldi_residual_rule_stops_where_the_residual_falls():
    """stop="residual" ends at the first step whose Arnoldi-solution residual
    is <= eps_Arn; the Hessenberg entries up to there are those of the
    unstopped run; stop="h" on the same B runs on while h_{j+1,j} stays
    large (a spectrum spread over [0.01, 1] keeps h near 0.2)."""
    rng = np.random.default_rng(43)
    n = 120
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    B = Q @ np.diag(np.geomspace(1e-2, 1.0, n)) @ Q.T
    r0 = rng.standard_normal(n)
    full = O.arnoldi(lambda w: B @ w, r0, 100, 0.0)
    for eps in (1e-2, 1e-4, 1e-6):
        j = int(np.flatnonzero(full.res <= eps)[0]) + 1
        st = O.arnoldi(lambda w: B @ w, r0, 100, eps, stop="residual")
        assert st.m == j and st.res[-1] <= eps and np.all(st.res[:-1] > eps)
        np.testing.assert_allclose(st.H, full.H[:j + 1, :j], rtol=0, atol=1e-12)
        hs = O.arnoldi(lambda w: B @ w, r0, 100, eps, stop="h")
        assert hs.m > j
    with pytest.raises(O.OracleError):
        O.arnoldi(lambda w: B @ w, r0, 10, 1e-3, stop="gmres")


def _hessenberg_with_spectrum(eigs, seed, symmetric):
    """An upper Hessenberg matrix similar to diag(eigs) (scipy's Householder
    reduction of T D T^-1), and its eigenvectors as columns (U^T T)."""
    rng = np.random.default_rng(seed)
    n = len(eigs)
    if symmetric:
        T = np.linalg.qr(rng.standard_normal((n, n)))[0]
    else:
        T = np.eye(n) + 0.5 * rng.standard_normal((n, n)) / np.sqrt(n)
    S = T @ np.diag(eigs) @ np.linalg.inv(T)
    H, U = scipy.linalg.hessenberg(S, calc_q=True)
    return H, U.T @ T


@pytest.mark.parametrize("symmetric", [True, False])
def test_ritz_select_skips_exact_null_keeps_small(symmetric):
    """Reading of the Ritz selection (Sect. 6, App. A): a Ritz value at the
    rounding level is an exact null direction and stays out of Z, while a
    genuine small eigenvalue (1e-8 of the largest, and 1e-9) is kept: the k
    selected vectors span the eigenvectors of the k smallest non-zero
    eigenvalues, also with the eps_lambda rule."""
    eigs = np.array([0.0, 0.0, 4e-8, 3e-3, 0.1, 0.5, 1.0, 2.0, 3.0, 4.0])
    H, X = _hessenberg_with_spectrum(eigs, 1, symmetric)
    theta, Y = O.ritz_select(H, 2)
    assert np.max(np.abs(theta[:2])) <= 1e-14          # the two exact zeros, found by eig
    assert Y.shape[1] == 2
    assert np.max(np.sin(scipy.linalg.subspace_angles(Y, X[:, 2:4]))) <= 1e-6
    theta, Y = O.ritz_select(H, 1)
    assert Y.shape[1] == 1
    assert np.max(np.sin(scipy.linalg.subspace_angles(Y, X[:, 2:3]))) <= 1e-6
    theta, Y = O.ritz_select(H, 0, eps_lambda=0.01)   # Re theta < 0.01: 4e-8 and 3e-3 only
    assert Y.shape[1] == 2
    assert np.max(np.sin(scipy.linalg.subspace_angles(Y, X[:, 2:4]))) <= 1e-6
    # a genuine value at 1e-9 of the largest is kept too
    eigs2 = eigs.copy()
    eigs2[2] = 4e-9
    H2, X2 = _hessenberg_with_spectrum(eigs2, 2, symmetric)
    theta, Y = O.ritz_select(H2, 1)
    assert Y.shape[1] == 1
    assert np.max(np.sin(scipy.linalg.subspace_angles(Y, X2[:, 2:3]))) <= 1e-6
    # with no null direction nothing is skipped
    H3, X3 = _hessenberg_with_spectrum(eigs[2:], 3, symmetric)
    theta, Y = O.ritz_select(H3, 2)
    assert np.max(np.sin(scipy.linalg.subspace_angles(Y, X3[:, 0:2]))) <= 1e-6


def test_ritz_select_null_then_complex_pair():
    """A complex pair right after the skipped null directions is kept whole."""
    n = 8
    D = np.zeros((n, n))
    D[2, 2] = 4e-8
    D[3:5, 3:5] = [[1e-3, 2e-4], [-2e-4, 1e-3]]   # eigenvalues 1e-3 +- 2e-4 i
    for i, e in zip(range(5, n), (0.5, 1.0, 2.0)):
        D[i, i] = e
    rng = np.random.default_rng(4)
    T = np.eye(n) + 0.4 * rng.standard_normal((n, n)) / np.sqrt(n)
    H, U = scipy.linalg.hessenberg(T @ D @ np.linalg.inv(T), calc_q=True)
    X = U.T @ T                                    # columns 3, 4 span the pair's real subspace
    theta, Y = O.ritz_select(H, 2)
    assert Y.shape[1] == 3
    assert np.max(np.sin(scipy.linalg.subspace_angles(Y, X[:, 2:5]))) <= 1e-6


def test_defl_build_order0_filter_skips_the_null_mode():
    """An order-0 template filter leaves the intensity monopole unconstrained
    (A 1_I = 0).  Arnoldi from a generic start vector runs until the Krylov
    space is invariant, so a Ritz value at the rounding level appears; Z then
    spans the eigenvectors of the k smallest non-null eigenvalues of the
    dense M_BD A, and leaves the null vector out."""
    p, pt, pf = _pf_problem(0, 0)
    M = O.mbd_build(pt, pf)
    n = pt.n
    Bd = np.stack([O.mbd_apply(M, O.apply_A(pt, pf, e)) for e in np.eye(n)], axis=1)
    ev, V = np.linalg.eig(Bd)
    order = np.argsort(ev.real)
    ev, V = ev[order], V[:, order]
    assert abs(ev[0]) <= 1e-12 and ev[1].real >= 0.5   # one null mode, well separated
    k = 5
    assert ev[k + 1].real - ev[k].real >= 1e-3          # a clear gap after the k-th
    b = np.random.default_rng(5).standard_normal(n)
    M2, res, theta = O.defl_build(pt, pf, M, b, k, 1e-10, n)
    assert res.m < n and np.min(np.abs(theta)) <= 1e-12  # the null Ritz value did appear
    assert M2.Z.shape[1] == k
    Vk = np.linalg.qr(V[:, 1:1 + k].real)[0]
    assert np.max(np.sin(scipy.linalg.subspace_angles(M2.Z, Vk))) <= 1e-8
    u = V[:, 0].real / np.linalg.norm(V[:, 0].real)
    assert np.linalg.norm(u - M2.Z @ (M2.Z.T @ u)) >= 0.9   # the null vector is not in span(Z)


def test_defl_build_smallest_ritz_span():
    """With the Arnoldi run to exhaustion the selected Z spans the invariant
    subspace of the k smallest eigenvalues of M_BD A."""
    p, pt, nz = _setup(11, n_side=3, n_samp=600, n_int=2, half_bw=12)
    M = O.mbd_build(pt, nz)
    b = O.rhs(pt, nz, p.tod)
    k = 5
    M2, res, theta = O.defl_build(pt, nz, M, b, k, 1e-300, pt.n)
    Bd = np.stack([O.mbd_apply(M, O.apply_A(pt, nz, e)) for e in np.eye(pt.n)], axis=1)
    ev, V = np.linalg.eig(Bd)
    order = np.argsort(ev.real)
    Vk = np.linalg.qr(V[:, order[:k]].real)[0]
    s = scipy.linalg.subspace_angles(M2.Z, Vk)
    assert np.max(np.sin(s)) <= 1e-7


# ---------------------------------------------------------------- PCG (O10)

def test_pcg_vs_cholesky_direct():
    p, pt, nz = _setup(12, n_side=3, n_samp=600, n_int=3, half_bw=12)
    P = _dense_P_test(p.pix, p.psi, pt.cidx)
    A = P.T @ _dense_N_scipy(p) @ P
    b = O.rhs(pt, nz, p.tod)
    M = O.mbd_build(pt, nz)
    x, info = O.pcg(lambda v: O.apply_A(pt, nz, v), lambda v: O.mbd_apply(M, v), b, 1e-13, 500)
    xd = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    kappa = np.linalg.cond(A)
    assert info.converged
    assert np.linalg.norm(x - xd) <= kappa * 1e-13 * np.linalg.norm(xd) * 10
    # exact inverse as preconditioner: one iteration
    Ainv = np.linalg.inv(A)
    x1, info1 = O.pcg(lambda v: A @ v, lambda v: Ainv @ v, b, 1e-10, 10)
    assert info1.iters == 1


def test_pcg_errnorm_bound_each_iteration():
    p, pt, nz = _setup(13, n_side=3, n_samp=600, n_int=3, half_bw=12)
    P = _dense_P_test(p.pix, p.psi, pt.cidx)
    A = P.T @ _dense_N_scipy(p) @ P
    b = O.rhs(pt, nz, p.tod)
    xd = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    M = O.mbd_build(pt, nz)
    Md = scipy.linalg.block_diag(*M.inv)
    kap = np.linalg.cond(Md @ A)
    kapA = np.linalg.cond(A)
    for it in range(1, 12):
        x, info = O.pcg(lambda v: A @ v, lambda v: Md @ v, b, 0.0, it)
        err = np.linalg.norm(xd - x) / np.linalg.norm(xd)
        # unpreconditioned residual: ||e|| <= kappa(A) ||r||/||b||
        assert err <= kapA * info.rel_res_true * (1 + 1e-8)
        # preconditioned residual of Eq. residuals: ||e|| <= kappa(MA) ||M r||/||M b||
        r = b - A @ x
        assert err <= kap * np.linalg.norm(Md @ r) / np.linalg.norm(Md @ b) * (1 + 1e-8)


def test_pcg_flexible_beta():
    """Polak-Ribiere beta = r'.(z' - z)/rho.  With a symmetric M the residuals
    are M-orthogonal (r'.M r = 0), so the iterates equal the Fletcher-Reeves
    ones; with the non-symmetric M_2l it still reaches the direct solution.
    The literal preconditioned residual ||M r||/||M b|| is reported beside
    the plain one and matches its definition."""
    p, pt, nz = _setup(14, n_side=3, n_samp=600, n_int=3, half_bw=12)
    P = _dense_P_test(p.pix, p.psi, pt.cidx)
    A = P.T @ _dense_N_scipy(p) @ P
    b = O.rhs(pt, nz, p.tod)
    xd = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    M = O.mbd_build(pt, nz)
    Md = scipy.linalg.block_diag(*M.inv)
    for it in (1, 3, 6):
        x1, i1 = O.pcg(lambda v: A @ v, lambda v: Md @ v, b, 0.0, it)
        x2, i2 = O.pcg(lambda v: A @ v, lambda v: Md @ v, b, 0.0, it, flexible=True)
        assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x1)
        r = b - A @ x1
        assert abs(i1.rel_res_precond - np.linalg.norm(Md @ r) / np.linalg.norm(Md @ b)) \
            <= 1e-12 * i1.rel_res_precond
    M2, _, _ = O.defl_build(pt, nz, M, b, 4, 1e-300, 40)
    Mm = np.stack([O.m2l_apply(M2, e) for e in np.eye(pt.n)], axis=1)
    assert np.max(np.abs(Mm - Mm.T)) > 1e-6 * np.max(np.abs(Mm)), "M_2l is not symmetric"
    x3, i3 = O.pcg(lambda v: A @ v, lambda v: O.m2l_apply(M2, v), b, 1e-12, 500, flexible=True)
    assert i3.converged
    assert np.linalg.norm(x3 - xd) <= np.linalg.cond(A) * 1e-12 * np.linalg.norm(xd) * 10


def test_noiseless_recovery_config1():
    """Signal-only TOD: the solution is the input map (error-norm analogue)."""
    p = synth.config1(noiseless=True)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    M = O.mbd_build(pt, nz)
    b = O.rhs(pt, nz, p.tod)
    x, info = O.pcg(lambda v: O.apply_A(pt, nz, v), lambda v: O.mbd_apply(M, v), b, 1e-10, 500)
    s = p.signal[pt.obs_pix].reshape(-1)
    assert info.converged and info.rel_res_true <= 1e-9
    assert np.linalg.norm(x - s) / np.linalg.norm(s) <= 1e-6


def test_m2l_fewer_iterations_than_mbd():
    p = synth.config1()
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    M = O.mbd_build(pt, nz)
    b = O.rhs(pt, nz, p.tod)
    A = lambda v: O.apply_A(pt, nz, v)
    _, i1 = O.pcg(A, lambda v: O.mbd_apply(M, v), b, 1e-8, 1000)
    M2, res, th = O.defl_build(pt, nz, M, b, 32, 1e-8, 256)
    _, i2 = O.pcg(A, lambda v: O.m2l_apply(M2, v), b, 1e-8, 1000)
    assert i1.converged and i2.converged
    assert i2.iters <= i1.iters
    assert i2.rel_res_true <= 1e-8 * 1.5


# ------------------------------------------ polynomial template filter (Sect. 2)

def _pf_problem(seed=0, order=2, flag_frac=0.05):
    """A tiny problem with ragged subscans inside intervals and per-interval
    white-noise weights."""
    p = synth.random_problem(seed, n_side=8, n_samp=1600, n_int=4, half_bw=5, n_filters=2,
                             flag_frac=flag_frac)
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    rng = np.random.default_rng(seed + 100)
    starts = [0]
    for i in range(p.n_intervals):  # cut every interval into subscans of 5..120 samples
        a, b = int(p.interval_start[i]), int(p.interval_start[i + 1])
        t = a
        while t < b:
            t = min(b, t + int(rng.integers(5, 121)))
            starts.append(t)
    weight = rng.uniform(0.5, 2.0, p.n_intervals)
    pf = O.polyfilter_build(pt, p.interval_start, weight, np.array(starts), order)
    return p, pt, pf


def _F_monomial(pf):
    """F from Eq. filtnoise with an explicit monomial basis and dense algebra:
    a different basis and a different code path from the oracle's; only the
    span of the templates matters."""
    n = pf.w.shape[0]
    F = np.zeros((n, n))
    p = pf.order
    for s in range(pf.subscan_start.shape[0] - 1):
        a, b = int(pf.subscan_start[s]), int(pf.subscan_start[s + 1])
        w = pf.w[a:b]
        if np.count_nonzero(w > 0) <= p + 1:
            continue
        tt = np.arange(b - a, dtype=np.float64) / max(b - a - 1, 1)
        T = np.vander(tt, p + 1, increasing=True)
        W = np.diag(w)
        F[a:b, a:b] = W - W @ T @ np.linalg.inv(T.T @ W @ T) @ T.T @ W
    return F


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_polyfilter_matches_monomial_definition(order):
    _, _, pf = _pf_problem(1, order)
    F = O.dense_polyfilter(pf)
    Fm = _F_monomial(pf)
    assert np.max(np.abs(F - Fm)) <= 1e-9 * np.max(np.abs(Fm))


def test_polyfilter_removes_templates_and_is_a_weighted_projector():
    _, _, pf = _pf_problem(2, 2)
    rng = np.random.default_rng(3)
    # F T = 0: any piecewise polynomial of degree <= 2 is removed
    y = np.zeros(pf.w.shape[0])
    for s in range(pf.subscan_start.shape[0] - 1):
        a, b = int(pf.subscan_start[s]), int(pf.subscan_start[s + 1])
        t = np.arange(b - a, dtype=np.float64)
        y[a:b] = rng.standard_normal() + rng.standard_normal() * t + rng.standard_normal() * t * t
    assert np.max(np.abs(O.polyfilter_apply(pf, y))) <= 1e-9 * np.max(np.abs(pf.w * y))
    # symmetric, positive semi-definite, F W^+ F = F
    F = O.dense_polyfilter(pf)
    assert np.max(np.abs(F - F.T)) <= 1e-12 * np.max(np.abs(F))
    assert np.min(np.linalg.eigvalsh(F)) >= -1e-10
    Wp = np.where(pf.w > 0, 1.0 / np.where(pf.w > 0, pf.w, 1.0), 0.0)
    assert np.max(np.abs(F @ (Wp[:, None] * F) - F)) <= 1e-9 * np.max(np.abs(F))


def test_polyfilter_order0_is_weighted_mean_removal():
    _, _, pf = _pf_problem(4, 0)
    y = np.random.default_rng(5).standard_normal(pf.w.shape[0])
    z = O.polyfilter_apply(pf, y)
    for s in range(pf.subscan_start.shape[0] - 1):
        a, b = int(pf.subscan_start[s]), int(pf.subscan_start[s + 1])
        w = pf.w[a:b]
        if np.count_nonzero(w > 0) <= 1:
            assert np.all(z[a:b] == 0)
            continue
        ref = w * (y[a:b] - np.sum(w * y[a:b]) / np.sum(w))
        assert np.max(np.abs(z[a:b] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_polyfilter_flags_and_short_subscans():
    p, pt, pf = _pf_problem(6, 3, flag_frac=0.2)
    y = np.random.default_rng(7).standard_normal(pt.n_samp)
    z = O.polyfilter_apply(pf, y)
    assert np.all(z[pt.j < 0] == 0)  # flagged samples carry no weight
    # a subscan with at most order + 1 weighted samples is fitted exactly
    sub = np.array([0, 3, 10, pt.n_samp], dtype=np.int64)
    ist = np.array([0, pt.n_samp], dtype=np.int64)
    pf2 = O.polyfilter_build(pt, ist, [1.0], sub, 3)
    z2 = O.polyfilter_apply(pf2, y)
    assert np.all(z2[0:3] == 0)
    # a subscan may not cross an interval boundary
    bad = np.array([0, int(p.interval_start[1]) + 1, pt.n_samp], dtype=np.int64)
    with pytest.raises(O.OracleError):
        O.polyfilter_build(pt, p.interval_start, np.ones(p.n_intervals), bad, 1)


def test_polyfilter_degenerate_mode_of_A():
    """Sect. 4: a sky mode whose time stream lies in the template span is
    lost, P s = T y => P^T F P s = 0.  A constant intensity map is constant
    on every subscan."""
    _, pt, pf = _pf_problem(8, 1)
    s = np.zeros(3 * pt.obs_pix.shape[0])
    s[0::3] = 7.0
    As = O.apply_A(pt, pf, s)
    x = np.random.default_rng(9).standard_normal(s.shape[0])
    assert np.max(np.abs(As)) <= 1e-10 * np.max(np.abs(O.apply_A(pt, pf, x)))
    # and A = P^T F P is symmetric positive semi-definite
    P = O.dense_P(pt)
    A = P.T @ O.dense_polyfilter(pf) @ P
    assert np.max(np.abs(A - A.T)) <= 1e-10 * np.max(np.abs(A))
    assert np.min(np.linalg.eigvalsh(A)) >= -1e-8 * np.max(np.abs(A))


# ------------------------------- ground templates in the filter (Sect. 4)

def _pf_ground_problem(seed=0, order=2, flag_frac=0.1, n_bins=23):
    """_pf_problem plus azimuth bins: random bins, some samples in none, one
    bin that only flagged samples fall in, and two subscans short enough to
    be fitted exactly."""
    p, pt, pf = _pf_problem(seed, order, flag_frac)
    rng = np.random.default_rng(seed + 200)
    gb = rng.integers(0, n_bins - 1, pt.n_samp).astype(np.int32)
    gb[rng.random(pt.n_samp) < 0.1] = -1
    flagged = np.flatnonzero(pt.j < 0)
    gb[flagged[:3]] = n_bins - 1          # a bin without weight
    sub = pf.subscan_start.copy()
    a = int(sub[1])                       # split the first subscan: lengths 2, 3, rest
    sub = np.concatenate([[0, 2, 5], sub[1:]]) if a > 6 else sub
    pf = O.polyfilter_build(pt, p.interval_start, pf.band[:, 0], sub, order, gb, n_bins)
    return p, pt, pf


def _F_template_definition(pf):
    """F_B W^+ F_G W^+ F_B written out with explicit template matrices and
    pseudo-inverses: T = monomials per subscan (a different basis from the
    oracle's Legendre polynomials; only the span matters), G[t, b] = 1 for
    sample t in bin b, F_X = W - W X (X^T W X)^+ X^T W, W^+ = diag(1/w, 0
    where w = 0)."""
    n = pf.w.shape[0]
    W = np.diag(pf.w)
    Wp = np.diag(np.where(pf.w > 0, 1.0 / np.where(pf.w > 0, pf.w, 1.0), 0.0))
    p = pf.order
    n_sub = pf.subscan_start.shape[0] - 1
    B = np.zeros((n, n_sub * (p + 1)))
    for s in range(n_sub):
        a, b = int(pf.subscan_start[s]), int(pf.subscan_start[s + 1])
        tt = np.arange(b - a, dtype=np.float64) / max(b - a - 1, 1)
        B[a:b, s * (p + 1):(s + 1) * (p + 1)] = np.vander(tt, p + 1, increasing=True)
    G = np.zeros((n, pf.n_ground_bins))
    on = pf.ground_bin >= 0
    G[np.flatnonzero(on), pf.ground_bin[on]] = 1.0

    def filt(X, blocks):
        M = X.T @ W @ X
        Mp = np.zeros_like(M)
        for lo, hi in blocks:  # X^T W X is block diagonal: pseudo-invert per block
            Mp[lo:hi, lo:hi] = np.linalg.pinv(M[lo:hi, lo:hi], hermitian=True)
        return W - W @ X @ Mp @ X.T @ W

    FB = filt(B, [(s * (p + 1), (s + 1) * (p + 1)) for s in range(n_sub)])
    FG = filt(G, [(b, b + 1) for b in range(pf.n_ground_bins)])
    return FB @ Wp @ FG @ Wp @ FB, FB, B, G


@pytest.mark.parametrize("order", [0, 1, 2])
def test_template_filter_matches_definition(order):
    _, _, pf = _pf_ground_problem(11, order)
    F = O.dense_polyfilter(pf)
    Fd, _, _, _ = _F_template_definition(pf)
    assert np.max(np.abs(F - Fd)) <= 1e-9 * np.max(np.abs(Fd))


def test_template_filter_symmetric_psd_and_removes_polynomials():
    _, pt, pf = _pf_ground_problem(12, 2)
    F = O.dense_polyfilter(pf)
    _, _, B, G = _F_template_definition(pf)
    assert np.max(np.abs(F - F.T)) <= 1e-12 * np.max(np.abs(F))
    assert np.min(np.linalg.eigvalsh(F)) >= -1e-10 * np.max(np.abs(F))
    assert np.max(np.abs(F @ B)) <= 1e-9 * np.max(np.abs(F)) * np.max(np.abs(B))
    # the ground part changes the filter: G's columns are not in B's span
    Fb = O.dense_polyfilter(O.polyfilter_build(pt, pf.interval_start, pf.band[:, 0],
                                               pf.subscan_start, 2))
    assert np.max(np.abs(F - Fb)) > 1e-3 * np.max(np.abs(Fb))


def test_template_filter_ground_inside_polynomial_span_is_F_B():
    """If every bin is a whole subscan, G's columns are order-0 polynomials,
    (I - Pi_G)(I - Pi_B) = I - Pi_B and the combination reduces to F_B."""
    _, pt, pf = _pf_ground_problem(13, 1)
    sub = pf.subscan_start
    gb = (np.searchsorted(sub, np.arange(pt.n_samp), side="right") - 1).astype(np.int32)
    pfg = O.polyfilter_build(pt, pf.interval_start, pf.band[:, 0], sub, 1, gb, sub.shape[0] - 1)
    pfb = O.polyfilter_build(pt, pf.interval_start, pf.band[:, 0], sub, 1)
    y = np.random.default_rng(14).standard_normal(pt.n_samp)
    zg, zb = O.polyfilter_apply(pfg, y), O.polyfilter_apply(pfb, y)
    assert np.max(np.abs(zg - zb)) <= 1e-12 * np.max(np.abs(zb))


def test_template_filter_ground_only_is_binned_mean_removal():
    """One subscan per interval, order 0, and bins that split each interval
    into halves: F_B removes the interval's weighted mean; the ground step
    then removes each half's weighted mean, which the last F_B leaves alone
    (the residual already has zero weighted mean over the interval).  So F y
    = w (y - mean over the sample's half), a closed form."""
    p, pt, _ = _pf_problem(15, 0, flag_frac=0.1)
    ist = p.interval_start
    w_int = np.linspace(0.7, 1.6, p.n_intervals)
    gb = np.empty(pt.n_samp, dtype=np.int32)
    for i in range(p.n_intervals):
        a, b = int(ist[i]), int(ist[i + 1])
        m = (a + b) // 2
        gb[a:m], gb[m:b] = 2 * i, 2 * i + 1
    pf = O.polyfilter_build(pt, ist, w_int, ist, 0, gb, 2 * p.n_intervals)
    y = np.random.default_rng(16).standard_normal(pt.n_samp)
    z = O.polyfilter_apply(pf, y)
    ref = np.zeros_like(y)
    for b in range(2 * p.n_intervals):
        sel = gb == b
        w = pf.w[sel]
        ref[sel] = w * (y[sel] - np.sum(w * y[sel]) / np.sum(w))
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_template_filter_validation():
    _, pt, pf = _pf_ground_problem(17, 1)
    gb = pf.ground_bin.copy()
    for bad in (gb[:-1], np.where(gb == 0, -2, gb), np.where(gb == 0, 23, gb)):
        with pytest.raises(O.OracleError):
            O.polyfilter_build(pt, pf.interval_start, pf.band[:, 0], pf.subscan_start, 1,
                               bad, 23)


def test_raster_ground_bins_follow_azimuth():
    """Bins are shared across detectors of a pass and advance one per sample
    along each sweep (1-pixel bins, 1 px/sample scan)."""
    gb, nb = synth.raster_ground_bins(16, (4, 2), 2 * 256)
    assert gb.min() >= 0 and gb.max() < nb and nb == 2 * (16 + 12)
    spd = 512
    for k in range(8):
        sw = gb[k * spd:k * spd + 16]                # first sweep runs forward
        assert np.all(np.diff(sw) == 1)
        sw2 = gb[k * spd + 16:k * spd + 32]          # the next runs back
        assert np.all(np.diff(sw2) == -1)
    assert np.all(gb[256:512] >= 28) and np.all(gb[:256] < 28)   # second pass, own bins


# --------------------- intensity-only and polarisation-only maps (Eqs. d+, d-)

@pytest.mark.parametrize("stokes,cols", [("I", [0]), ("QU", [1, 2])])
def test_stokes_subsets_are_columns_of_the_IQU_pointing(stokes, cols):
    """P for the pair-sum (I) and pair-difference (QU) streams keeps the
    intensity or the polarisation columns of the IQU pointing matrix."""
    p = synth.random_problem(31, n_side=5, n_samp=900, flag_frac=0.1)
    full = O.pointing_build(p.pix, p.psi, p.n_pix_total, 1)
    sub = O.pointing_build(p.pix, None if stokes == "I" else p.psi, p.n_pix_total, 1, stokes)
    Pf = O.dense_P(full)
    keep = np.concatenate([np.arange(full.n_obs) * 3 + c for c in cols])
    keep = np.sort(keep)
    Ps = O.dense_P(sub)
    np.testing.assert_array_equal(Ps, Pf[:, keep])
    x = np.random.default_rng(32).standard_normal(sub.n)
    y = np.random.default_rng(33).standard_normal(p.n_samp)
    assert np.max(np.abs(O.apply_P(sub, x) - Ps @ x)) <= 1e-13 * np.max(np.abs(Ps @ x))
    assert np.max(np.abs(O.apply_PT(sub, y) - Ps.T @ y)) <= 1e-12 * np.max(np.abs(Ps.T @ y))


def test_intensity_only_white_noise_solution_is_the_binned_mean():
    """I-only pointing, white noise (lambda = 0): M_BD = A^-1, so PCG stops
    after one step at the weighted binned mean of each pixel's samples."""
    p = synth.random_problem(34, n_side=6, n_samp=2000, half_bw=0, n_filters=2)
    pt = O.pointing_build(p.pix, None, p.n_pix_total, 3, "I")
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, 0)
    M = O.mbd_build(pt, nz)
    b = O.rhs(pt, nz, p.tod)
    x, info = O.pcg(lambda v: O.apply_A(pt, nz, v), lambda v: O.mbd_apply(M, v), b, 1e-12, 10)
    c0 = np.empty(p.n_samp)
    for i in range(p.n_intervals):
        c0[p.interval_start[i]:p.interval_start[i + 1]] = p.band[p.filter_id[i], 0]
    ref = np.zeros(pt.n_obs)
    for j in range(pt.n_obs):
        t = pt.perm[pt.off[j]:pt.off[j + 1]]
        ref[j] = np.sum(c0[t] * p.tod[t]) / np.sum(c0[t])
    assert info.iters <= 1
    assert np.max(np.abs(x - ref)) <= 1e-12 * np.max(np.abs(ref))


def _pair_problem(seed, half_bw=4):
    """Detector pairs: B sees the same pixel as A at every sample with its
    polariser turned by 90 degrees (psi + pi/2), so d_B = I - Q c - U s +
    n_B.  Returns (p, pair pix/psi concatenated A then B, d_A, d_B)."""
    p = synth.random_problem(seed, n_side=5, n_samp=1500, n_int=3, half_bw=half_bw,
                             n_filters=2, flag_frac=0.05)
    n = p.n_samp
    psi_b = p.psi + 0.5 * np.pi
    sky = p.signal
    d_a = synth.signal_tod(p.pix, p.psi, sky) + np.random.default_rng(seed + 1).standard_normal(n)
    d_b = synth.signal_tod(p.pix, psi_b, sky) + np.random.default_rng(seed + 2).standard_normal(n)
    return p, np.concatenate([p.pix, p.pix]), np.concatenate([p.psi, psi_b]), d_a, d_b


@pytest.mark.parametrize("weight", ["band", "filter"])
def test_pair_sum_difference_separates_intensity_and_polarisation(weight):
    """Sect. 4: for a detector pair with orthogonal polarisers and the same
    noise weight, the IQU system of both detectors' data splits into an
    intensity system on d+ = (d_A + d_B)/2 with the I pointing and a
    polarisation system on d- = (d_A - d_B)/2 with the QU pointing: the cross
    terms of P_A^T W P_A + P_B^T W P_B cancel.  So the IQU solution equals
    the I and QU solutions side by side."""
    p, pix2, psi2, d_a, d_b = _pair_problem(35)
    n = p.n_samp
    full = O.pointing_build(pix2, psi2, p.n_pix_total, 2)
    ptI = O.pointing_build(p.pix, None, p.n_pix_total, 1, "I")
    ptQ = O.pointing_build(p.pix, p.psi, p.n_pix_total, 1, "QU")
    assert np.array_equal(full.obs_pix, ptI.obs_pix) and np.array_equal(full.obs_pix, ptQ.obs_pix)
    ist2 = np.concatenate([p.interval_start, p.interval_start[1:] + n])
    fid2 = np.concatenate([p.filter_id, p.filter_id])
    if weight == "band":
        nz2 = O.noise_build(ist2, fid2, p.band, p.half_bw)
        nzI = nzQ = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    else:
        sub = np.unique(np.concatenate([np.arange(0, n, 37), p.interval_start]))
        w = np.array([1.3, 0.8, 1.1])
        nz2 = O.polyfilter_build(full, ist2, np.concatenate([w, w]),
                                 np.concatenate([sub, sub[1:] + n]), 1)
        nzI = O.polyfilter_build(ptI, p.interval_start, w, sub, 1)
        nzQ = O.polyfilter_build(ptQ, p.interval_start, w, sub, 1)
    W2 = O.dense_polyfilter(nz2) if weight == "filter" else O.dense_Ninv(nz2)
    WI = O.dense_polyfilter(nzI) if weight == "filter" else O.dense_Ninv(nzI)
    WQ = O.dense_polyfilter(nzQ) if weight == "filter" else O.dense_Ninv(nzQ)
    P2, PI, PQ = O.dense_P(full), O.dense_P(ptI), O.dense_P(ptQ)
    d2 = np.concatenate([d_a, d_b])
    dp, dm = 0.5 * (d_a + d_b), 0.5 * (d_a - d_b)
    A2 = P2.T @ W2 @ P2
    # the filter leaves the intensity monopole unconstrained: solve in the
    # least-squares sense and compare modulo that direction
    x2 = np.linalg.lstsq(A2, P2.T @ W2 @ d2, rcond=1e-12)[0].reshape(-1, 3)
    xI = np.linalg.lstsq(PI.T @ WI @ PI, PI.T @ WI @ dp, rcond=1e-12)[0]
    xQ = np.linalg.solve(PQ.T @ WQ @ PQ, PQ.T @ WQ @ dm).reshape(-1, 2)
    if weight == "filter":
        x2[:, 0] -= x2[:, 0].mean()
        xI = xI - xI.mean()
    # the operator blocks themselves
    perm = np.concatenate([np.arange(full.n_obs) * 3, (np.arange(full.n_obs)[:, None] * 3
                                                        + np.array([1, 2])).reshape(-1)])
    Ap = A2[np.ix_(perm, perm)]
    nI = full.n_obs
    assert np.max(np.abs(Ap[:nI, nI:])) <= 1e-12 * np.max(np.abs(A2))
    assert np.max(np.abs(Ap[:nI, :nI] - 2 * PI.T @ WI @ PI)) <= 1e-12 * np.max(np.abs(A2))
    assert np.max(np.abs(Ap[nI:, nI:] - 2 * PQ.T @ WQ @ PQ)) <= 1e-12 * np.max(np.abs(A2))
    assert np.max(np.abs(x2[:, 0] - xI)) <= 1e-9 * np.max(np.abs(xI))
    assert np.max(np.abs(x2[:, 1:] - xQ)) <= 1e-9 * np.max(np.abs(xQ))


def test_qu_mbd_blocks_and_stokes_validation():
    p = synth.random_problem(36, n_side=5, n_samp=1200, half_bw=3)
    ptQ = O.pointing_build(p.pix, p.psi, p.n_pix_total, 3, "QU")
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    M = O.mbd_build(ptQ, nz)
    assert M.inv.shape == (ptQ.n_obs, 2, 2)
    full = O.pointing_build(p.pix, p.psi, p.n_pix_total, 3)
    Mf = O.mbd_build(full, nz)
    np.testing.assert_allclose(M.blocks, Mf.blocks[:, 1:, 1:], rtol=1e-13, atol=1e-13)
    with pytest.raises(O.OracleError):
        O.pointing_build(p.pix, None, p.n_pix_total, 3, "QU")
    with pytest.raises(O.OracleError):
        O.pointing_build(p.pix, p.psi, p.n_pix_total, 3, "Q")


# ------------------------- Ritz vectors from a prior M_BD solve (PCG-Lanczos)

def test_pcg_lanczos_relation_and_ritz_bounds():
    """The PCG coefficients define the Lanczos tridiagonal of M A: the
    vectors z_j / sqrt(rho_j) are M^-1-orthonormal, M A V_m = V_m T_m up to
    the last column, and the Ritz values lie inside the spectrum of M A and
    approach its ends as m grows."""
    p, pt, nz = _setup(15, n_side=3, n_samp=600, n_int=3, half_bw=12)
    P = _dense_P_test(p.pix, p.psi, pt.cidx)
    A = P.T @ _dense_N_scipy(p) @ P
    M = O.mbd_build(pt, nz)
    Md = scipy.linalg.block_diag(*M.inv)
    b = O.rhs(pt, nz, p.tod)
    lam = np.sort(np.linalg.eigvals(Md @ A).real)
    for m in (4, 8, 12):
        res = O.pcg_lanczos(lambda v: A @ v, lambda v: Md @ v, b, m)
        V, T = res.V, res.T
        if m == 4:  # before CG converges; later the vectors lose orthogonality
            G = V.T @ np.linalg.solve(Md, V)  # as finite-precision Lanczos does
            assert np.max(np.abs(G - np.eye(res.m))) <= 1e-10
        R = Md @ A @ V - V @ T
        assert np.max(np.abs(R[:, :-1])) <= 1e-9 * np.max(np.abs(Md @ A @ V))
        th = np.linalg.eigvalsh(T)
        assert th[0] >= lam[0] * (1 - 1e-9) and th[-1] <= lam[-1] * (1 + 1e-9)
    res = O.pcg_lanczos(lambda v: A @ v, lambda v: Md @ v, b, 20)
    th = np.linalg.eigvalsh(res.T)
    assert abs(th[0] - lam[0]) <= 1e-6 * lam[0] and abs(th[-1] - lam[-1]) <= 1e-6 * lam[-1]


def test_defl_build_from_prior_mbd_solve():
    """Z from the Ritz vectors of an M_BD solve: a valid M_2l (Eq. ident) that
    cuts the iteration count like the Arnoldi-built one."""
    p = synth.config1()
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    M = O.mbd_build(pt, nz)
    b = O.rhs(pt, nz, p.tod)
    M2, res, theta = O.defl_build_pcg(pt, nz, M, b, 16, 60)
    assert M2.Z.shape[1] == 16 and res.m == 60
    MAZ = np.stack([O.m2l_apply(M2, O.apply_A(pt, nz, M2.Z[:, c])) for c in range(16)], 1)
    assert np.max(np.abs(MAZ - M2.Z)) <= 1e-8
    A = lambda v: O.apply_A(pt, nz, v)
    _, i1 = O.pcg(A, lambda v: O.mbd_apply(M, v), b, 1e-8, 1000)
    _, i2 = O.pcg(A, lambda v: O.m2l_apply(M2, v), b, 1e-8, 1000)
    assert i1.converged and i2.converged and i2.iters < i1.iters


def test_orth_drop_removes_dependent_directions():
    rng = np.random.default_rng(40)
    A = rng.standard_normal((50, 4))
    V = np.concatenate([A, A[:, :2] * 3.0 + 1e-15 * rng.standard_normal((50, 2))], axis=1)
    Q = O.orth_drop(V)
    assert Q.shape[1] == 4
    assert np.max(np.abs(Q.T @ Q - np.eye(4))) <= 1e-13
    # same span as the independent part
    assert np.max(np.sin(scipy.linalg.subspace_angles(Q, A))) <= 1e-12


def test_pcg_lanczos_stops_at_tolerance():
    p = synth.config1()
    pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    M = O.mbd_build(pt, nz)
    b = O.rhs(pt, nz, p.tod)
    A = lambda v: O.apply_A(pt, nz, v)
    _, i1 = O.pcg(A, lambda v: O.mbd_apply(M, v), b, 1e-6, 1000)
    res = O.pcg_lanczos(A, lambda v: O.mbd_apply(M, v), b, 1000, tol=1e-6)
    assert res.m == i1.iters   # the prior solve's own iteration count


def test_stored_config1_solution_is_the_oracles():
    """tests/golden/config1_solution.json (the reference of the FP32 form's map
    error) is what its committed script computes from the oracle now."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_config1_solution", os.path.join(GOLDEN, "make_config1_solution.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    x, b, info = mod.solve()
    ref = _golden("config1_solution.json")
    assert info.rel_res_true <= 1e-12
    assert np.max(np.abs(np.array(ref["x"]) - x)) <= 1e-12 * np.max(np.abs(x))
    assert abs(ref["b_norm"] - float(np.linalg.norm(b))) <= 1e-12 * ref["b_norm"]
