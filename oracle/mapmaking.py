"""Oracle implementation (FP64, numpy).  Test infrastructure only.

Notation follows the paper: d = P s + n (Eqs. probl, datamod); a polarised
sample is d_t = I + Q cos 2phi_t + U sin 2phi_t + n_t (Eq. datamodel); the GLS
estimate solves A x = b with A = P^T W P, b = P^T W d (Eqs. estimator,
linearsystem); here W = N^-1 is a banded Toeplitz matrix per stationary
interval.  Preconditioners: M_BD (Eq. mbd) and M_2l (Eq. m2l) with E = Z^T A Z.
The deflation space comes from Ritz vectors of an Arnoldi run on B = M_BD A
(Sect. 6 and Appendix A, Alg. arnoldi, Eqs. factoriz and ritz).  The solver is
PCG (Eq. pcg) with the relative residual of the metric in Sect. 7.1.

Readings where the paper is silent or garbled (each is listed in the design doc):
  * residual: the stop test and the reported residual use the
    unpreconditioned ||b - A x|| / ||b|| (Eq. residuals mixes in M_P);
  * N^-1 is block diagonal over intervals, each block the principal section of
    the banded Toeplitz matrix (no wrap-around, nothing couples intervals);
  * flagged samples are masked out of both P and d (W = M N^-1 M);
  * M_BD uses the zero-lag coefficient c_0 of the sample's interval as
    diag(N^-1);
  * PCG uses beta = rho_new / rho for both preconditioners (M_2l is not
    symmetric; Sect. 3.2);
  * Arnoldi starts from r_0 = M_BD b_seed (b_seed = b - A x_0; b for
    x_0 = 0), orthogonalises by classical Gram-Schmidt applied twice, stops
    when h_{j+1,j} <= eps_Arn (the algorithm box) or, as a second reading of
    the error term, when the Arnoldi solution's relative residual
    h_{j+1,j} |(H_j^-1 e_1)_j| <= eps_Arn, or at j = m_max;
  * Ritz values are ordered by real part; a complex pair is never split; the
    real and imaginary parts of a pair's vector both enter Z.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Pointing", "Noise", "OracleError", "pointing_build", "apply_P", "apply_PT",
    "noise_build", "noise_apply_direct", "noise_apply_fft", "noise_apply", "fom_residual",
    "apply_A", "apply_A_pixels", "rhs", "Mbd", "mbd_build", "mbd_apply", "M2l", "m2l_from_Z",
    "m2l_apply", "arnoldi", "ritz_select", "defl_build", "pcg", "SolveInfo",
    "dense_P", "dense_Ninv", "PolyFilter", "polyfilter_build", "polyfilter_apply",
    "dense_polyfilter", "pcg_lanczos", "defl_build_pcg", "LanczosResult", "orth_drop",
]


COARSE_PIVOT_TOL = 1e-13


class OracleError(RuntimeError):
    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# O1  pointing  (Eqs. probl, datamodel; observed-pixel selection, Sect. 5)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Pointing:
    n_samp: int
    n_pix_total: int
    hits: np.ndarray      # int32[n_pix_total] samples per global pixel (unflagged)
    obs_pix: np.ndarray   # int32[n_obs] observed global ids, ascending
    cidx: np.ndarray      # int32[n_pix_total] compact index or -1
    j: np.ndarray         # int32[n_samp] compact pixel per sample, -1 = flagged
    perm: np.ndarray      # int32[n_valid] samples sorted by (j, t)
    off: np.ndarray       # int32[n_obs+1] segment offsets into perm
    cos2: np.ndarray      # f64[n_samp]
    sin2: np.ndarray      # f64[n_samp]
    stokes: str = "IQU"   # map components: "IQU", "I" or "QU"

    @property
    def n_obs(self) -> int:
        return int(self.obs_pix.shape[0])

    @property
    def nc(self) -> int:
        return len(self.stokes)

    @property
    def n(self) -> int:
        return self.nc * self.n_obs

    def weights(self) -> np.ndarray:
        """f64[n_samp, nc]: the non-zeros of each row of P.  IQU: (1, cos 2phi,
        sin 2phi) (Eq. datamodel); I: (1) for the pair-sum stream (Eq. d+);
        QU: (cos 2phi, sin 2phi) for the pair-difference stream (Eq. d-)."""
        cols = {"I": np.ones(self.n_samp), "Q": self.cos2, "U": self.sin2}
        return np.stack([cols[a] for a in self.stokes], axis=1)


def pointing_build(pix, psi, n_pix_total: int, min_hits: int = 3,
                   stokes: str = "IQU") -> Pointing:
    """P has three non-zeros per row, (1, cos 2phi_t, sin 2phi_t) at the
    sample's pixel (Eq. datamodel); with stokes = "I" or "QU" only the
    intensity or the polarisation columns (the sum and difference streams of
    a detector pair, Eqs. d+ and d-; psi may be None for "I").  Pixels seen
    fewer than min_hits times are dropped and their samples flagged (the paper
    discards samples of pixels observed without enough redundancy, Sect. 4)."""
    if stokes not in ("IQU", "I", "QU"):
        raise OracleError("INVALID", "stokes must be IQU, I or QU")
    pix = np.asarray(pix, dtype=np.int32)
    if psi is None:
        if stokes != "I":
            raise OracleError("INVALID", "psi is needed for polarisation")
        psi = np.zeros(pix.shape[0])
    psi = np.asarray(psi, dtype=np.float64)
    if pix.shape != psi.shape:
        raise OracleError("INVALID", "pix and psi differ in length")
    if np.any(pix < -1) or np.any(pix >= n_pix_total):
        raise OracleError("INVALID", "pixel index out of range")
    valid = pix >= 0
    hits = np.bincount(pix[valid], minlength=n_pix_total).astype(np.int32)
    obs_pix = np.nonzero(hits >= min_hits)[0].astype(np.int32)
    cidx = np.full(n_pix_total, -1, dtype=np.int32)
    cidx[obs_pix] = np.arange(obs_pix.shape[0], dtype=np.int32)
    j = np.full(pix.shape[0], -1, dtype=np.int32)
    j[valid] = cidx[pix[valid]]
    t_keep = np.nonzero(j >= 0)[0]
    perm = t_keep[np.argsort(j[t_keep], kind="stable")].astype(np.int32)
    off = np.zeros(obs_pix.shape[0] + 1, dtype=np.int32)
    off[1:] = np.cumsum(hits[obs_pix])
    return Pointing(n_samp=pix.shape[0], n_pix_total=n_pix_total, hits=hits,
                    obs_pix=obs_pix, cidx=cidx, j=j, perm=perm, off=off,
                    cos2=np.cos(2.0 * psi), sin2=np.sin(2.0 * psi), stokes=stokes)


def apply_P(pt: Pointing, x) -> np.ndarray:
    """y_t = I_j + Q_j cos 2phi_t + U_j sin 2phi_t at j = j_t; 0 if flagged
    (Eq. datamodel); the I or QU terms alone for those pointings.  x is the
    map, [n_obs][nc] interleaved."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, pt.nc)
    y = np.zeros(pt.n_samp)
    m = pt.j >= 0
    jj = pt.j[m]
    w = pt.weights()[m]
    for a in range(pt.nc):
        y[m] += w[:, a] * x[jj, a]
    return y


def apply_PT(pt: Pointing, z) -> np.ndarray:
    """(P^T z)_{j,a} = sum over samples t with j_t = j of w_t[a] z_t, with
    w_t the row's non-zeros (pt.weights); samples summed in time order."""
    z = np.asarray(z, dtype=np.float64)
    m = pt.j >= 0
    jj = pt.j[m]
    w = pt.weights()[m]
    out = np.empty((pt.n_obs, pt.nc))
    for a in range(pt.nc):
        out[:, a] = np.bincount(jj, weights=w[:, a] * z[m], minlength=pt.n_obs)
    return out.reshape(-1)


def dense_P(pt: Pointing) -> np.ndarray:
    """The N_t x nc n_obs pointing matrix written out (tiny inputs only)."""
    P = np.zeros((pt.n_samp, pt.n))
    cols = {"I": lambda t: 1.0, "Q": lambda t: pt.cos2[t], "U": lambda t: pt.sin2[t]}
    for t in range(pt.n_samp):
        j = pt.j[t]
        if j >= 0:
            for a, name in enumerate(pt.stokes):
                P[t, pt.nc * j + a] = cols[name](t)
    return P


# ---------------------------------------------------------------------------
# O2  N^-1: banded Toeplitz per stationary interval (W = N^-1, Sect. 2)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Noise:
    interval_start: np.ndarray  # int64[n_int+1]
    filter_id: np.ndarray       # int32[n_int]
    band: np.ndarray            # f64[n_filters, half_bw+1]
    half_bw: int

    @property
    def n_samp(self) -> int:
        return int(self.interval_start[-1])


def noise_build(interval_start, filter_id, band, half_bw: int) -> Noise:
    istart = np.asarray(interval_start, dtype=np.int64)
    fid = np.asarray(filter_id, dtype=np.int32)
    band = np.asarray(band, dtype=np.float64).reshape(-1, half_bw + 1)
    if istart[0] != 0 or np.any(np.diff(istart) <= 0):
        raise OracleError("INVALID", "intervals must tile [0, n_samp)")
    if np.any(np.diff(istart) <= 2 * half_bw):
        raise OracleError("INVALID", "half bandwidth must be < L_min/2")
    if np.any(fid < 0) or np.any(fid >= band.shape[0]):
        raise OracleError("INVALID", "filter id out of range")
    return Noise(istart, fid, band, half_bw)


def noise_apply_direct(nz: Noise, y) -> np.ndarray:
    """z_t = sum_{u in I(t), |t-u| <= lambda} c^f_{|t-u|} y_u: the definition,
    one lag at a time, truncated at interval edges."""
    y = np.asarray(y, dtype=np.float64)
    z = np.empty_like(y)
    lam = nz.half_bw
    for i in range(nz.filter_id.shape[0]):
        a, b = int(nz.interval_start[i]), int(nz.interval_start[i + 1])
        c = nz.band[nz.filter_id[i]]
        yi = y[a:b]
        zi = c[0] * yi
        for d in range(1, min(lam, b - a - 1) + 1):
            zi[d:] += c[d] * yi[:-d]
            zi[:-d] += c[d] * yi[d:]
        z[a:b] = zi
    return z


def noise_apply_fft(nz: Noise, y) -> np.ndarray:
    """Same operator by zero-padded FFT convolution: per interval of length L,
    a circular convolution of length n_f >= L + lambda with the symmetric
    kernel reproduces the truncated band exactly (no wrap-around reaches an
    output).  numpy's FFT is the library step."""
    y = np.asarray(y, dtype=np.float64)
    z = np.empty_like(y)
    lam = nz.half_bw
    cache = {}
    for i in range(nz.filter_id.shape[0]):
        a, b = int(nz.interval_start[i]), int(nz.interval_start[i + 1])
        L = b - a
        nf = 1 << int(np.ceil(np.log2(L + lam)))
        key = (nf, int(nz.filter_id[i]))
        if key not in cache:
            c = nz.band[nz.filter_id[i]]
            h = np.zeros(nf)
            h[0] = c[0]
            h[1:lam + 1] = c[1:]
            h[nf - lam:] = c[1:][::-1]
            cache[key] = np.fft.rfft(h)
        yp = np.zeros(nf)
        yp[:L] = y[a:b]
        z[a:b] = np.fft.irfft(np.fft.rfft(yp) * cache[key], n=nf)[:L]
    return z


def noise_apply(nz: Noise, y, method: str = "direct") -> np.ndarray:
    if isinstance(nz, PolyFilter):
        return polyfilter_apply(nz, y)
    return noise_apply_fft(nz, y) if method == "fft" else noise_apply_direct(nz, y)


# ---------------------------------------------------------------------------
# polynomial template filter as the weight (Sect. 2, Eqs. filt and filtnoise)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PolyFilter:
    """Template filter used as the weight (Sect. 2, Eqs. filt and filtnoise).

    Polynomial part: F_B = W - W B (B^T W B)^-1 B^T W with B the piecewise
    Legendre polynomials of degree 0..order on each subscan (Sect. 4: long
    modes filtered by low-order polynomials per subscan) and W = diag(w), w_t
    the white-noise weight of the sample's interval times the flag mask.

    Ground part (optional; Sect. 4, ground pickup): G has one column per
    azimuth bin, G[t, b] = 1 when sample t falls in bin b, and F_G is the same
    formula with G in place of B.  With both, the filter is the symmetric
    combination F_B W^-1 F_G W^-1 F_B of Sect. 4, with W^-1 read as the
    pseudo-inverse (zero on flagged samples).

    It duck-types as a Noise (interval_start, filter_id, band with half_bw =
    0, band[i, 0] = omega_i), so diag(W) enters M_BD like c_0 does (Eq. mbd)."""
    interval_start: np.ndarray   # int64[n_int+1]
    filter_id: np.ndarray        # int32[n_int] = arange
    band: np.ndarray             # f64[n_int, 1] interval weights omega_i
    half_bw: int                 # 0
    subscan_start: np.ndarray    # int64[n_sub+1]
    order: int
    w: np.ndarray                # f64[n_samp] omega of the interval x mask
    ground_bin: np.ndarray | None = None   # int32[n_samp] azimuth bin, -1 = none
    n_ground_bins: int = 0


def polyfilter_build(pt: Pointing, interval_start, weight, subscan_start, order: int,
                     ground_bin=None, n_ground_bins: int = 0) -> PolyFilter:
    istart = np.asarray(interval_start, dtype=np.int64)
    wgt = np.asarray(weight, dtype=np.float64)
    sub = np.asarray(subscan_start, dtype=np.int64)
    if istart[0] != 0 or istart[-1] != pt.n_samp or np.any(np.diff(istart) <= 0):
        raise OracleError("INVALID", "intervals must tile [0, n_samp)")
    if sub[0] != 0 or sub[-1] != pt.n_samp or np.any(np.diff(sub) <= 0):
        raise OracleError("INVALID", "subscans must tile [0, n_samp)")
    if wgt.shape[0] != istart.shape[0] - 1 or np.any(wgt < 0) or not (0 <= order <= 7):
        raise OracleError("INVALID", "one weight >= 0 per interval, order in [0, 7]")
    # every subscan lies inside one interval
    iv_a = np.searchsorted(istart, sub[:-1], side="right") - 1
    iv_b = np.searchsorted(istart, sub[1:] - 1, side="right") - 1
    if np.any(iv_a != iv_b):
        raise OracleError("INVALID", "a subscan crosses an interval boundary")
    gb = None
    if ground_bin is not None:
        gb = np.asarray(ground_bin, dtype=np.int32)
        if gb.shape != (pt.n_samp,) or n_ground_bins < 1 or np.any(gb < -1) \
                or np.any(gb >= n_ground_bins):
            raise OracleError("INVALID", "ground bins must lie in [-1, n_ground_bins)")
    w = np.empty(pt.n_samp)
    for i in range(wgt.shape[0]):
        w[istart[i]:istart[i + 1]] = wgt[i]
    w = np.where(pt.j >= 0, w, 0.0)
    return PolyFilter(istart, np.arange(wgt.shape[0], dtype=np.int32), wgt[:, None].copy(), 0,
                      sub, int(order), w, gb, int(n_ground_bins) if gb is not None else 0)


def _subscan_u(L: int) -> np.ndarray:
    """Subscan time mapped onto [-1, 1] (the Legendre interval)."""
    if L == 1:
        return np.zeros(1)
    return -1.0 + 2.0 * np.arange(L, dtype=np.float64) / (L - 1)


def _poly_residual(pf: PolyFilter, y) -> np.ndarray:
    """r = y - B (B^T W B)^-1 B^T W y, subscan by subscan.  A subscan with at
    most order + 1 weighted samples is fitted exactly by the polynomials, so
    its residual is 0 on every weighted sample; it is returned as 0 there."""
    r = np.zeros_like(y)
    p = pf.order
    for s in range(pf.subscan_start.shape[0] - 1):
        a, b = int(pf.subscan_start[s]), int(pf.subscan_start[s + 1])
        w = pf.w[a:b]
        if np.count_nonzero(w > 0) <= p + 1:
            continue
        B = np.polynomial.legendre.legvander(_subscan_u(b - a), p)
        G = B.T @ (w[:, None] * B)
        c = np.linalg.solve(G, B.T @ (w * y[a:b]))
        r[a:b] = y[a:b] - B @ c
    return r


def _ground_residual(pf: PolyFilter, y) -> np.ndarray:
    """r = y - G (G^T W G)^-1 G^T W y.  G^T W G is diagonal (a sample lies in
    at most one bin): each bin's template amplitude is the w-weighted mean of
    its samples, 0 for a bin without weight (pseudo-inverse)."""
    num = np.zeros(pf.n_ground_bins)
    den = np.zeros(pf.n_ground_bins)
    for t in range(y.shape[0]):
        b = pf.ground_bin[t]
        if b >= 0:
            num[b] += pf.w[t] * y[t]
            den[b] += pf.w[t]
    amp = np.divide(num, den, out=np.zeros_like(num), where=den > 0)
    r = y.copy()
    for t in range(y.shape[0]):
        b = pf.ground_bin[t]
        if b >= 0:
            r[t] -= amp[b]
    return r


def polyfilter_apply(pf: PolyFilter, y) -> np.ndarray:
    """z = F y.  Polynomial only: z = W (y - B (B^T W B)^-1 B^T W y).  With
    ground templates: z = F_B W^+ F_G W^+ F_B y, where W^+ F_B y = M r_B(y)
    (M the mask of weighted samples, r_B the residual above), and likewise for
    F_G."""
    y = np.asarray(y, dtype=np.float64)
    mask = pf.w > 0
    if pf.ground_bin is None:
        return pf.w * _poly_residual(pf, y)
    y1 = np.where(mask, _poly_residual(pf, y), 0.0)
    y2 = np.where(mask, _ground_residual(pf, y1), 0.0)
    return pf.w * _poly_residual(pf, y2)


def dense_polyfilter(pf: PolyFilter) -> np.ndarray:
    n = pf.w.shape[0]
    F = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        F[:, i] = polyfilter_apply(pf, e)
    return F


def dense_Ninv(nz: Noise) -> np.ndarray:
    """N^-1 written out as a block-diagonal matrix of Toeplitz sections."""
    n = nz.n_samp
    N = np.zeros((n, n))
    for i in range(nz.filter_id.shape[0]):
        a, b = int(nz.interval_start[i]), int(nz.interval_start[i + 1])
        c = nz.band[nz.filter_id[i]]
        for t in range(a, b):
            for u in range(max(a, t - nz.half_bw), min(b, t + nz.half_bw + 1)):
                N[t, u] = c[abs(t - u)]
    return N


# ---------------------------------------------------------------------------
# O5/O6  A x = P^T N^-1 P x ;  b = P^T N^-1 (mask * d)   (Eq. linearsystem)
# ---------------------------------------------------------------------------

def apply_A(pt: Pointing, nz: Noise, x, method: str = "direct") -> np.ndarray:
    return apply_PT(pt, noise_apply(nz, apply_P(pt, x), method))


def apply_A_pixels(pt: Pointing, nz: Noise, x, pixels) -> np.ndarray:
    """(A x) restricted to the listed compact pixels, each computed on its own
    from the definition: for every sample t of the pixel,
    z_t = sum_{u in I(t), |t-u| <= lambda} c_{|t-u|} (P x)_u, then
    sum_t w_t z_t.  Cost is per requested pixel, so it serves as a check at
    sizes where the whole product is too large for the oracle.
    Returns f64[len(pixels), 3] (IQU pointings only)."""
    if pt.stokes != "IQU":
        raise OracleError("INVALID", "apply_A_pixels takes IQU pointings")
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    lam = nz.half_bw
    out = np.zeros((len(pixels), 3))
    for q, j in enumerate(pixels):
        ts = pt.perm[pt.off[j]:pt.off[j + 1]]
        for t in ts:
            i = int(np.searchsorted(nz.interval_start, t, side="right") - 1)
            a, b = int(nz.interval_start[i]), int(nz.interval_start[i + 1])
            lo, hi = max(a, int(t) - lam), min(b, int(t) + lam + 1)
            u = np.arange(lo, hi)
            ju = pt.j[u]
            m = ju >= 0
            y = np.zeros(hi - lo)
            y[m] = x[ju[m], 0] + pt.cos2[u[m]] * x[ju[m], 1] + pt.sin2[u[m]] * x[ju[m], 2]
            c = nz.band[nz.filter_id[i]][np.abs(u - int(t))]
            z = float(np.dot(c, y))
            out[q] += z * np.array([1.0, pt.cos2[t], pt.sin2[t]])
    return out


def rhs(pt: Pointing, nz: Noise, d, method: str = "direct") -> np.ndarray:
    """Samples of unobserved or off-patch pixels are zeroed before weighting,
    so W = M N^-1 M with M the 0/1 mask (keeps W semi-definite, P M = P)."""
    d = np.where(pt.j >= 0, np.asarray(d, dtype=np.float64), 0.0)
    return apply_PT(pt, noise_apply(nz, d, method))


# ---------------------------------------------------------------------------
# O7  M_BD^-1 = P^T diag(N^-1) P   (Eq. mbd)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Mbd:
    blocks: np.ndarray      # f64[n_obs, nc, nc]  B_j
    inv: np.ndarray         # f64[n_obs, nc, nc]  B_j^-1
    rcond_min: float


def _diag_weight(pt: Pointing, nz: Noise) -> np.ndarray:
    """diag(N^-1)_t = c_0 of the sample's interval filter."""
    c0 = np.empty(pt.n_samp)
    for i in range(nz.filter_id.shape[0]):
        a, b = int(nz.interval_start[i]), int(nz.interval_start[i + 1])
        c0[a:b] = nz.band[nz.filter_id[i], 0]
    return c0


def mbd_build(pt: Pointing, nz: Noise, rcond_tol: float = 1e-12) -> Mbd:
    """B_j = sum_{t: j_t = j} c_0 w_t w_t^T with w_t the row's non-zeros
    ((1, cos 2phi, sin 2phi) for IQU: 3x3 blocks; 1x1 for I, 2x2 for QU);
    M_BD is the block-diagonal matrix of the B_j^-1."""
    c0 = _diag_weight(pt, nz)
    m = pt.j >= 0
    jj = pt.j[m]
    w = pt.weights()[m]
    cw = c0[m]
    nc = pt.nc
    B = np.zeros((pt.n_obs, nc, nc))
    for a in range(nc):
        for b in range(nc):
            B[:, a, b] = np.bincount(jj, weights=cw * w[:, a] * w[:, b], minlength=pt.n_obs)
    try:
        np.linalg.cholesky(B)
    except np.linalg.LinAlgError as e:
        raise OracleError("SINGULAR_BLOCK", "a pixel block is not positive definite") from e
    inv = np.linalg.inv(B)
    rc = 1.0 / (np.abs(B).sum(axis=1).max(axis=1) * np.abs(inv).sum(axis=1).max(axis=1))
    if pt.n_obs and rc.min() < rcond_tol:
        raise OracleError("SINGULAR_BLOCK", f"pixel block rcond {rc.min():.3e}")
    return Mbd(B, inv, float(rc.min()) if pt.n_obs else 1.0)


def mbd_apply(M: Mbd, v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64).reshape(-1, M.inv.shape[1])
    return np.einsum("jab,jb->ja", M.inv, v).reshape(-1)


# ---------------------------------------------------------------------------
# O8  M_2l = M_BD (1 - A Z E^-1 Z^T) + Z E^-1 Z^T,  E = Z^T A Z   (Eq. m2l)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class M2l:
    mbd: Mbd
    Z: np.ndarray      # f64[n, k]
    AZ: np.ndarray     # f64[n, k]
    E: np.ndarray      # f64[k, k] symmetrised
    L: np.ndarray      # Cholesky factor of E


def m2l_from_Z(pt: Pointing, nz: Noise, mbd: Mbd, Z, method: str = "direct") -> M2l:
    Z = np.asarray(Z, dtype=np.float64).reshape(pt.n, -1)
    k = Z.shape[1]
    AZ = np.empty_like(Z)
    for c in range(k):
        AZ[:, c] = apply_A(pt, nz, Z[:, c], method)
    E = Z.T @ AZ
    E = 0.5 * (E + E.T)
    # E must be SPD (Sect. 3.2).  A pivot below 1e-13 of the largest diagonal
    # entry is treated as a failure: E is numerically singular (Z rank deficient).
    try:
        L = np.linalg.cholesky(E) if k else np.zeros((0, 0))
    except np.linalg.LinAlgError as e:
        raise OracleError("COARSE_NOT_SPD", "E = Z^T A Z is not positive definite") from e
    if k and np.min(np.diag(L)) ** 2 <= COARSE_PIVOT_TOL * np.max(np.diag(E)):
        raise OracleError("COARSE_NOT_SPD", "E = Z^T A Z is numerically singular")
    return M2l(mbd, Z, AZ, E, L)


def m2l_apply(M: M2l, v) -> np.ndarray:
    """c = E^-1 Z^T v ; out = M_BD (v - A Z c) + Z c."""
    v = np.asarray(v, dtype=np.float64)
    if M.Z.shape[1] == 0:
        return mbd_apply(M.mbd, v)
    g = M.Z.T @ v
    c = np.linalg.solve(M.L.T, np.linalg.solve(M.L, g))
    return mbd_apply(M.mbd, v - M.AZ @ c) + M.Z @ c


# ---------------------------------------------------------------------------
# O9  Arnoldi on B = M_BD A (Alg. arnoldi), Ritz pairs (Eq. ritz), Z
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class ArnoldiResult:
    W: np.ndarray      # f64[n, m+1] orthonormal Krylov basis (last column w_{m+1})
    H: np.ndarray      # f64[m+1, m] Hessenberg matrix incl. h_{m+1,m}
    m: int
    h_last: float
    res: np.ndarray | None = None   # f64[m] fom_residual after each step


def fom_residual(H: np.ndarray, j: int) -> float:
    """||W~_j y_j|| / ||r_0|| for the Arnoldi (full orthogonalisation)
    solution of B x = r_0 in the j-step Krylov space, y_j = H_j^-1 ||r_0|| e_1:
    by Eq. factoriz the residual r_0 - B W_j y_j is -h_{j+1,j} (e_j^T y_j)
    w_{j+1}, so its relative norm is h_{j+1,j} |(H_j^-1 e_1)_j|.  Infinite if
    H_j is singular.  H holds at least j+1 rows and j columns."""
    Hj = H[:j, :j]
    e1 = np.zeros(j)
    e1[0] = 1.0
    try:
        y = np.linalg.solve(Hj, e1)
    except np.linalg.LinAlgError:
        return float("inf")
    return float(H[j, j - 1] * abs(y[j - 1]))


def arnoldi(apply_B, r0, m_max: int, eps_arn: float, reorth: bool = True,
            stop: str = "h") -> ArnoldiResult:
    """w_1 = r0/||r0||; for j: v = B w_j; h_ij = (v, w_i) for all i <= j from
    the same v (classical Gram-Schmidt); v -= sum h_ij w_i; with reorth the
    projection is repeated once and added into h (CGS2); h_{j+1,j} = ||v||;
    stop when the error term of Eq. factoriz falls to eps_arn, else
    w_{j+1} = v / h_{j+1,j}.  Two readings of that test (App. A):
    stop="h"        h_{j+1,j} <= eps_arn, as the algorithm box writes it
                    (||W~_j|| = h_{j+1,j});
    stop="residual" fom_residual(H, j) <= eps_arn, the error term applied to
                    the Arnoldi solution of B x = r_0 (the reading under
                    which tightening eps_Arn solves the system to that
                    residual, as Sect. 6 says).
    Either rule also stops on h_{j+1,j} = 0 (an invariant subspace)."""
    if stop not in ("h", "residual"):
        raise OracleError("INVALID", "stop rule is 'h' or 'residual'")
    n = r0.shape[0]
    W = np.zeros((n, m_max + 1))
    H = np.zeros((m_max + 1, m_max))
    res = np.zeros(m_max)
    W[:, 0] = r0 / np.linalg.norm(r0)
    m = 0
    h_last = 0.0
    for j in range(m_max):
        v = apply_B(W[:, j])
        h = W[:, :j + 1].T @ v
        v = v - W[:, :j + 1] @ h
        if reorth:
            h2 = W[:, :j + 1].T @ v
            v = v - W[:, :j + 1] @ h2
            h = h + h2
        H[:j + 1, j] = h
        hn = np.linalg.norm(v)
        H[j + 1, j] = hn
        m = j + 1
        h_last = hn
        res[j] = fom_residual(H, m)
        test = hn if stop == "h" else res[j]
        if test <= eps_arn or hn == 0.0:
            break
        W[:, j + 1] = v / hn
    return ArnoldiResult(W[:, :m + 1], H[:m + 1, :m], m, h_last, res[:m].copy())


NULL_RITZ_REL = 1e-10


def ritz_select(H_m: np.ndarray, k: int, eps_lambda: float = 0.0):
    """Eigenpairs of the m x m Hessenberg matrix (numpy's LAPACK eig), ordered
    by real part ascending.  Past the null directions (below), keep the k
    smallest (k+1 if that would split a conjugate pair) or, with
    eps_lambda > 0, all with Re(theta) < eps_lambda.
    Returns (theta_sorted, Y) with Y real: a complex pair contributes the real
    and imaginary parts of one of its vectors."""
    theta, Yc = np.linalg.eig(H_m)
    order = np.lexsort((theta.imag, theta.real))
    theta, Yc = theta[order], Yc[:, order]
    m = theta.shape[0]
    # Ritz values at the rounding level (|theta| <= 1e-10 max |theta|) are exact
    # null directions of M_BD A (sky modes a filter leaves unconstrained):
    # E = Z^T A Z could not be inverted with them and a consistent right-hand
    # side has no component along them, so they are left out of Z.
    first = 0
    tmax = float(np.max(np.abs(theta))) if m else 0.0
    while first < m and abs(theta[first]) <= NULL_RITZ_REL * tmax:
        first += 1
    if eps_lambda > 0:
        keep = int(np.sum(theta.real < eps_lambda))
    else:
        keep = min(first + k, m)
    if 0 < keep < m and theta[keep - 1].imag != 0 and np.conj(theta[keep - 1]) == theta[keep]:
        keep += 1
    cols = []
    i = first
    while i < keep:
        if theta[i].imag != 0 and i + 1 < m and np.conj(theta[i]) == theta[i + 1]:
            cols.append(Yc[:, i].real)
            cols.append(Yc[:, i].imag)
            i += 2
        else:
            cols.append(Yc[:, i].real)
            i += 1
    Y = np.stack(cols, axis=1) if cols else np.zeros((m, 0))
    return theta, Y


def defl_build(pt: Pointing, nz: Noise, mbd: Mbd, b_seed, k: int, eps_arn: float,
               m_max: int, eps_lambda: float = 0.0, method: str = "direct",
               reorth: bool = True, stop: str = "h"):
    """Deflation space from Ritz vectors of B = M_BD A (Sect. 6): Arnoldi from
    r_0 = M_BD b_seed (stop rule as in arnoldi), Ritz selection, V = W_m Y,
    Z = Q of a Householder QR of V (numpy's QR).
    Returns (M2l, ArnoldiResult, theta)."""
    r0 = mbd_apply(mbd, b_seed)
    res = arnoldi(lambda w: mbd_apply(mbd, apply_A(pt, nz, w, method)), r0, m_max,
                  eps_arn, reorth, stop)
    theta, Y = ritz_select(res.H[:res.m, :res.m], k, eps_lambda)
    V = res.W[:, :res.m] @ Y
    Z = np.linalg.qr(V)[0] if V.shape[1] else V
    return m2l_from_Z(pt, nz, mbd, Z, method), res, theta


@dataclasses.dataclass
class LanczosResult:
    V: np.ndarray        # f64[n, m] Lanczos vectors z_j / sqrt(rho_j)
    T: np.ndarray        # f64[m, m] symmetric tridiagonal
    m: int
    alpha: np.ndarray    # CG step lengths alpha_0..alpha_{m-1}
    beta: np.ndarray     # CG coefficients beta_0..beta_{m-1}


def pcg_lanczos(apply_A_fn, apply_M_fn, b, m: int, tol: float = 0.0) -> LanczosResult:
    """m PCG iterations from x_0 = 0 (Eq. pcg), keeping what the Lanczos
    process on M A hides in them: with z_j = M r_j and rho_j = r_j.z_j, the
    vectors v_j = z_j / sqrt(rho_j) are orthonormal in the M^-1 inner product
    (r_i.M r_j = 0 for i != j), and M A V_m = V_m T_m + (last column term),
    T_m tridiagonal with
        T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = -sqrt(beta_j)/alpha_j.
    The Ritz pairs of T_m are those of a prior M_BD solve (the reading of
    "Ritz vectors from a prior solve" that keeps the CG inner product).
    Stops after m iterations, when the solve reaches ||r||/||b|| <= tol, or if
    rho reaches 0."""
    r = np.asarray(b, dtype=np.float64).copy()
    bnorm = float(np.linalg.norm(r))
    z = apply_M_fn(r)
    rho = float(r @ z)
    p = z.copy()
    V = [z / np.sqrt(rho)]
    alpha, beta = [], []
    for j in range(m):
        q = apply_A_fn(p)
        a = rho / float(p @ q)
        r = r - a * q
        z = apply_M_fn(r)
        rho_new = float(r @ z)
        bt = rho_new / rho
        alpha.append(a)
        beta.append(bt)
        if j + 1 == m or not rho_new > 0 or float(np.linalg.norm(r)) <= tol * bnorm:
            break
        V.append(z / np.sqrt(rho_new))
        p = z + bt * p
        rho = rho_new
    mm = len(V)
    T = np.zeros((mm, mm))
    for j in range(mm):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < mm:
            T[j, j + 1] = T[j + 1, j] = -np.sqrt(beta[j]) / alpha[j]
    return LanczosResult(np.stack(V, axis=1), T, mm, np.array(alpha), np.array(beta))


DEPENDENT_REL = 1e-12


def orth_drop(V: np.ndarray) -> np.ndarray:
    """Orthonormal basis of span(V) that leaves out numerically dependent
    directions: eigenvectors of V^T V whose eigenvalue is below 1e-12 of the
    largest are dropped (finite-precision Lanczos repeats converged Ritz
    values, whose vectors then coincide), then Q of a QR."""
    if V.shape[1] == 0:
        return V
    lam, U = np.linalg.eigh(V.T @ V)
    keep = lam > DEPENDENT_REL * lam[-1]
    return np.linalg.qr(V @ (U[:, keep] / np.sqrt(lam[keep])))[0]


def defl_build_pcg(pt: Pointing, nz: Noise, mbd: Mbd, b, k: int, m: int, tol: float = 0.0,
                   eps_lambda: float = 0.0, method: str = "direct"):
    """Deflation space from the Ritz vectors of an M_BD PCG run on A x = b of
    at most m iterations, stopped at ||r||/||b|| <= tol (config 2's "Ritz
    vectors from a prior M_BD solve"): Ritz selection on T_m as for
    Arnoldi's H_m, V = V_m Y, Z = an orthonormal basis of span(V) without
    dependent directions.  Returns (M2l, LanczosResult, theta)."""
    res = pcg_lanczos(lambda v: apply_A(pt, nz, v, method), lambda v: mbd_apply(mbd, v), b, m,
                      tol)
    theta, Y = ritz_select(res.T, k, eps_lambda)
    Z = orth_drop(res.V @ Y)
    return m2l_from_Z(pt, nz, mbd, Z, method), res, theta


# ---------------------------------------------------------------------------
# O10  PCG (Eq. pcg; stop on ||b - A x|| / ||b|| <= tol, Sect. 7.1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SolveInfo:
    iters: int
    rel_res_recursive: float
    rel_res_true: float
    history: np.ndarray
    breakdown: bool = False
    converged: bool = False
    rel_res_precond: float = float("nan")   # ||M (b - A x)|| / ||M b|| at exit


def pcg(apply_A_fn, apply_M_fn, b, tol: float, max_iter: int, x0=None, flexible: bool = False):
    """Textbook preconditioned conjugate gradients:
        r = b - A x; z = M r; p = z; rho = r.z
        repeat: q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;
                z = M r; rho' = r.z; beta = rho'/rho; p = z + beta p
    until ||r|| / ||b|| <= tol or max_iter iterations.  flexible: the
    Polak-Ribiere choice beta = r'.(z' - z)/rho, which tolerates a
    preconditioner that is not symmetric (M_2l is not, Sect. 3.2); for a
    symmetric M the two coincide in exact arithmetic (r'.z = 0).
    At exit the residual is also reported in the preconditioned norm of
    Eq. residuals read literally, ||M (b - A x)|| / ||M b||."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A_fn(x)
    z = apply_M_fn(r)
    p = z.copy()
    rho = float(r @ z)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, SolveInfo(0, 0.0, 0.0, np.zeros(1), converged=True)
    hist = [float(np.linalg.norm(r)) / bnorm]
    k = 0
    breakdown = False
    while hist[-1] > tol and k < max_iter:
        q = apply_A_fn(p)
        pq = float(p @ q)
        if not pq > 0.0:
            breakdown = True
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rz_old = float(r @ z) if flexible else 0.0
        z = apply_M_fn(r)
        rho_new = float(r @ z)
        beta = (rho_new - rz_old) / rho if flexible else rho_new / rho
        p = z + beta * p
        rho = rho_new
        k += 1
        hist.append(float(np.linalg.norm(r)) / bnorm)
    r_true = b - apply_A_fn(x)
    true_res = float(np.linalg.norm(r_true)) / bnorm
    prec_res = float(np.linalg.norm(apply_M_fn(r_true))) / float(np.linalg.norm(apply_M_fn(b)))
    return x, SolveInfo(k, hist[-1], true_res, np.array(hist), breakdown,
                        converged=hist[-1] <= tol, rel_res_precond=prec_res)
