"""Seeded synthetic inputs for map-making: scans, polarisation angles, sky maps,
1/f noise and the banded inverse-noise coefficients.

This module is shared by the CPU oracle and the GPU library's tests and
benchmark.  It draws random numbers and lays out inputs; it holds none of the
map-making arithmetic (no pointing matrix, no noise weighting, no solver).

Every draw comes from ``numpy.random.default_rng(SeedSequence([cfg, realization,
stream]))`` with the stream ids below, so a given (cfg, realization) always
produces the same arrays.

The paper's own inputs (S4CMB scans of a Chilean site, HEALPix/CAMB skies,
white-noise-only TODs; Sect. 4) are not available.  These generators stand in
for them with flat-sky raster scans of the same structure: constant-elevation
back-and-forth sweeps (subscans), several detectors with focal-plane offsets,
cross-linking from rotated scan directions, a half-wave-plate angle per sample
(Eq. datamodel) and piecewise-stationary 1/f noise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STREAM_SCAN = 0
STREAM_PSI = 1
STREAM_SIGNAL = 2
STREAM_NOISE = 3
STREAM_FKNEE = 4
STREAM_ARRIVALS = 5

F_SAMP = 20.0          # Hz
NOISE_SIGMA = 1.0      # white-noise level
NOISE_ALPHA = 1.7      # 1/f slope
SIGMA_I = 100.0
SIGMA_QU = 5.0


def rng_for(cfg: int, realization: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, realization, stream]))


@dataclasses.dataclass
class Problem:
    """One map-making input set.

    pix       int32[n_samp]  global pixel id per sample, -1 = flagged (off patch)
    psi       f64[n_samp]    polarisation angle (rad) per sample
    interval_start int64[n_int+1]  stationary intervals tile [0, n_samp)
    filter_id int32[n_int]   band row used by each interval
    band      f64[n_filters, half_bw+1]  c_0..c_lambda of each banded N^-1
    signal    f64[n_pix_total, 3]  input I, Q, U per global pixel
    tod       f64[n_samp]    d = signal part + noise (noise absent if noiseless)
    """
    name: str
    n_side: int
    n_pix_total: int
    pix: np.ndarray
    psi: np.ndarray
    interval_start: np.ndarray
    filter_id: np.ndarray
    band: np.ndarray
    half_bw: int
    signal: np.ndarray
    tod: np.ndarray
    min_hits: int = 3
    noise: np.ndarray | None = None

    @property
    def n_samp(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_intervals(self) -> int:
        return int(self.filter_id.shape[0])


# ---------------------------------------------------------------------------
# noise model
# ---------------------------------------------------------------------------

def psd_1f(f, sigma=NOISE_SIGMA, fknee=0.5, alpha=NOISE_ALPHA):
    """P(f) = sigma^2 (1 + (fknee/|f|)^alpha); infinite at f = 0."""
    f = np.abs(np.asarray(f, dtype=np.float64))
    with np.errstate(divide="ignore"):
        return sigma ** 2 * (1.0 + (fknee / f) ** alpha)


def band_from_psd(L: int, half_bw: int, fknee: float, sigma=NOISE_SIGMA,
                  alpha=NOISE_ALPHA, fs=F_SAMP) -> np.ndarray:
    """Banded-Toeplitz inverse-noise coefficients c_0..c_lambda for one filter.

    The inverse PSD g_k = 1/P(f_k) on the interval's frequency grid
    f_k = k fs / L (g_0 = 0: the mean of an interval is left unconstrained) is
    turned into its time-domain autocorrelation by an inverse real DFT, then
    truncated at lag lambda with a Bartlett taper (1 - j/(lambda+1)).  The taper
    makes the band's symbol a Fejer average of g >= 0, so every interval block
    of N^-1 is positive definite.
    """
    k = np.arange(L // 2 + 1, dtype=np.float64)
    g = np.zeros(L // 2 + 1)
    g[1:] = 1.0 / psd_1f(k[1:] * fs / L, sigma, fknee, alpha)
    chat = np.fft.irfft(g, n=L)
    j = np.arange(half_bw + 1, dtype=np.float64)
    return chat[: half_bw + 1] * (1.0 - j / (half_bw + 1))


def noise_1f(rng: np.random.Generator, L: int, n_intervals: int, fknee,
             sigma=NOISE_SIGMA, alpha=NOISE_ALPHA, fs=F_SAMP) -> np.ndarray:
    """Gaussian noise with PSD psd_1f, synthesised independently per interval.

    X_k = sqrt(L P_k / 2)(a + i b), X_0 = 0, X_{L/2} = sqrt(L P_{L/2}) a,
    n = irfft(X, L).  fknee is a scalar or one value per interval.
    Returns f64[n_intervals, L].
    """
    fk = np.broadcast_to(np.asarray(fknee, dtype=np.float64), (n_intervals,))
    kf = np.arange(1, L // 2 + 1, dtype=np.float64) * fs / L
    out = np.empty((n_intervals, L))
    for i in range(n_intervals):
        P = psd_1f(kf, sigma, fk[i], alpha)
        a = rng.standard_normal(L // 2 + 1)
        b = rng.standard_normal(L // 2 + 1)
        X = np.empty(L // 2 + 1, dtype=np.complex128)
        X[0] = 0.0
        X[1:] = np.sqrt(L * P / 2.0) * (a[1:] + 1j * b[1:])
        X[-1] = np.sqrt(L * P[-1]) * a[-1]
        out[i] = np.fft.irfft(X, n=L)
    return out


# ---------------------------------------------------------------------------
# skies
# ---------------------------------------------------------------------------

def white_sky(rng: np.random.Generator, n_pix: int) -> np.ndarray:
    s = rng.standard_normal((n_pix, 3))
    s[:, 0] *= SIGMA_I
    s[:, 1:] *= SIGMA_QU
    return s


def cmb_like_sky(rng: np.random.Generator, n_side: int) -> np.ndarray:
    """Flat-sky Gaussian random field with P(k) ~ 1/(k^2+1) per Stokes map,
    rescaled to sigma_I / sigma_QU.  A stand-in for a CAMB/synfast CMB sky."""
    kx = np.fft.fftfreq(n_side) * n_side
    k2 = kx[:, None] ** 2 + kx[None, :] ** 2
    amp = np.sqrt(1.0 / (k2 + 1.0))
    out = np.empty((n_side * n_side, 3))
    for c, sig in enumerate((SIGMA_I, SIGMA_QU, SIGMA_QU)):
        w = rng.standard_normal((n_side, n_side))
        f = np.fft.ifft2(np.fft.fft2(w) * amp).real
        f = (f - f.mean()) / f.std() * sig
        out[:, c] = f.reshape(-1)
    return out


def signal_tod(pix: np.ndarray, psi: np.ndarray, sky: np.ndarray) -> np.ndarray:
    """d_t = I + Q cos 2psi + U sin 2psi at the sample's pixel; 0 if flagged.
    (The data model the inputs are drawn from, Eq. datamodel.)"""
    out = np.zeros(pix.shape[0])
    m = pix >= 0
    p = pix[m]
    out[m] = sky[p, 0] + sky[p, 1] * np.cos(2.0 * psi[m]) + sky[p, 2] * np.sin(2.0 * psi[m])
    return out


# ---------------------------------------------------------------------------
# scans
# ---------------------------------------------------------------------------

def straight_raster(n_side: int, n_det: int, n_samp_per_det: int) -> np.ndarray:
    """Back-and-forth sweeps along x at 1 px/sample, stepping 1 px in y per
    sweep; detector k starts n_side*k/n_det rows down.  Detector-major."""
    t = np.arange(n_samp_per_det, dtype=np.int64)
    q = t // n_side
    u = t % n_side
    ix = np.where(q % 2 == 0, u, n_side - 1 - u)
    out = np.empty(n_det * n_samp_per_det, dtype=np.int32)
    for k in range(n_det):
        iy = (q + (n_side * k) // n_det) % n_side
        out[k * n_samp_per_det:(k + 1) * n_samp_per_det] = iy * n_side + ix
    return out


def rotated_raster(n_side: int, grid: tuple[int, int], n_samp_per_det: int,
                   angles_deg=(0.0, 60.0, 120.0)) -> np.ndarray:
    """Cross-linked raster scans.  A pass is n_side sweeps of n_side samples;
    pass m is rotated by angles_deg[m mod len(angles_deg)] about the patch
    centre (the default, three passes 60 degrees apart, cross-links every
    pixel; a few degrees apart mimic the weak cross-linking of constant-
    elevation scans).  Detector k sits at focal-plane offset
    (2(k mod gx)-(gx-1), 2(k div gx)-(gy-1)) px.  Samples falling off the
    patch get pixel -1 (flagged)."""
    gx, gy = grid
    n_det = gx * gy
    per_pass = n_side * n_side
    assert n_samp_per_det % per_pass == 0
    s = np.arange(per_pass, dtype=np.int64)
    q = s // n_side
    u = s % n_side
    half = n_side / 2.0
    a = np.where(q % 2 == 0, u, n_side - 1 - u).astype(np.float64) + 0.5 - half
    b = q.astype(np.float64) + 0.5 - half
    rot = []
    for ang in angles_deg:
        th = math.radians(ang)
        ct, st = math.cos(th), math.sin(th)
        rot.append((half + a * ct - b * st, half + a * st + b * ct))
    n_pass = n_samp_per_det // per_pass
    out = np.empty(n_det * n_samp_per_det, dtype=np.int32)
    for k in range(n_det):
        ox = 2 * (k % gx) - (gx - 1)
        oy = 2 * (k // gx) - (gy - 1)
        for m in range(n_pass):
            x, y = rot[m % len(rot)]
            ix = np.floor(x + ox).astype(np.int64)
            iy = np.floor(y + oy).astype(np.int64)
            ok = (ix >= 0) & (ix < n_side) & (iy >= 0) & (iy < n_side)
            p = np.where(ok, iy * n_side + ix, -1)
            base = k * n_samp_per_det + m * per_pass
            out[base:base + per_pass] = p
    return out


def raster_ground_bins(n_side: int, grid: tuple[int, int], n_samp_per_det: int,
                       bin_px: float = 1.0) -> tuple[np.ndarray, int]:
    """Azimuth bins of the ground templates for rotated_raster's scans (ground
    pickup, Sect. 4).  Each pass is one constant-elevation scan whose sweeps
    run along the pass's rotated x axis, which plays the azimuth; a detector's
    azimuth is the sweep coordinate plus its focal-plane offset along the
    sweep.  The bins, bin_px pixels wide, are shared by all detectors of a
    pass.  Returns (bin int32[n_det * n_samp_per_det], n_bins)."""
    gx, gy = grid
    n_det = gx * gy
    per_pass = n_side * n_side
    assert n_samp_per_det % per_pass == 0
    n_pass = n_samp_per_det // per_pass
    s = np.arange(per_pass, dtype=np.int64)
    q = s // n_side
    u = s % n_side
    half = n_side / 2.0
    a = np.where(q % 2 == 0, u, n_side - 1 - u).astype(np.float64) + 0.5 - half
    margin = float(gx + gy)
    n_loc = int(math.ceil((n_side + 2 * margin) / bin_px))
    out = np.empty(n_det * n_samp_per_det, dtype=np.int32)
    for k in range(n_det):
        ox = 2 * (k % gx) - (gx - 1)
        oy = 2 * (k // gx) - (gy - 1)
        for m in range(n_pass):
            th = math.radians(60.0 * (m % 3))
            az = a + ox * math.cos(th) + oy * math.sin(th) + half + margin
            loc = np.clip(np.floor(az / bin_px).astype(np.int64), 0, n_loc - 1)
            base = k * n_samp_per_det + m * per_pass
            out[base:base + per_pass] = m * n_loc + loc
    return out, n_pass * n_loc


def uniform_intervals(n_samp: int, L: int) -> np.ndarray:
    assert n_samp % L == 0
    return np.arange(0, n_samp + 1, L, dtype=np.int64)


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def _finish(name, cfg, realization, n_side, pix, L, half_bw, fknee_per_det,
            samp_per_det, noiseless, sky=None, psi=None, min_hits=3):
    n_samp = pix.shape[0]
    n_pix_total = n_side * n_side
    if psi is None:
        psi = rng_for(cfg, realization, STREAM_PSI).uniform(0.0, math.pi, n_samp)
    if sky is None:
        sky = white_sky(rng_for(cfg, realization, STREAM_SIGNAL), n_pix_total)
    istart = uniform_intervals(n_samp, L)
    n_int = istart.shape[0] - 1
    int_per_det = samp_per_det // L
    fknee_per_det = np.asarray(fknee_per_det, dtype=np.float64)
    n_filters = fknee_per_det.shape[0]
    if n_filters == 1:
        filter_id = np.zeros(n_int, dtype=np.int32)
    else:
        filter_id = (np.arange(n_int) // int_per_det).astype(np.int32)
    band = np.stack([band_from_psd(L, half_bw, fk) for fk in fknee_per_det])
    d = signal_tod(pix, psi, sky)
    noise = None
    if not noiseless:
        noise = noise_1f(rng_for(cfg, realization, STREAM_NOISE), L, n_int,
                         fknee_per_det[filter_id]).reshape(-1)
        d = d + noise
    return Problem(name=name, n_side=n_side, n_pix_total=n_pix_total, pix=pix,
                   psi=psi, interval_start=istart, filter_id=filter_id, band=band,
                   half_bw=half_bw, signal=sky, tod=d, min_hits=min_hits, noise=noise)


def config1(realization: int = 0, noiseless: bool = False) -> Problem:
    """32x32 patch, 2 detectors x 65,536 samples of straight rasters (128
    hits/pixel), f_knee 0.5 Hz, intervals of 16,384, lambda = 32."""
    pix = straight_raster(32, 2, 65536)
    return _finish("c1", 1, realization, 32, pix, 16384, 32, [0.5], 65536, noiseless)


def config2(realization: int = 0, noiseless: bool = False, n_side: int = 256,
            grid=(16, 8), samp_per_det: int = 1 << 20, L: int = 1 << 16,
            half_bw: int = 4096, angles_deg=(0.0, 60.0, 120.0)) -> Problem:
    """256x256 patch, 128 detectors x 2^20 samples of cross-linked rasters,
    f_knee ~ U[0.05, 1] Hz per detector, intervals of 2^16, lambda = 4,096.
    Smaller shapes of the same structure come from the keyword arguments."""
    n_det = grid[0] * grid[1]
    pix = rotated_raster(n_side, grid, samp_per_det, angles_deg)
    fk = rng_for(2, realization, STREAM_FKNEE).uniform(0.05, 1.0, n_det)
    p = _finish("c2", 2, realization, n_side, pix, L, half_bw, fk, samp_per_det, noiseless)
    return p


def config4_realization(r: int, noiseless: bool = False) -> Problem:
    """Monte Carlo realization r on config 1's pointing (same pix and psi, same
    noise model): its own CMB-like sky and its own noise."""
    pix = straight_raster(32, 2, 65536)
    psi = rng_for(1, 0, STREAM_PSI).uniform(0.0, math.pi, pix.shape[0])
    sky = cmb_like_sky(rng_for(4, r, STREAM_SIGNAL), 32)
    return _finish("c4", 4, r, 32, pix, 16384, 32, [0.5], 65536, noiseless,
                   sky=sky, psi=psi)


# Serving strategies: (n_side, detectors grid, samples/detector, lambda)
SERVE_STRATEGIES = (
    (64, (4, 4), 1 << 16, 1024),
    (128, (8, 4), 1 << 18, 2048),
    (256, (8, 8), 1 << 20, 4096),
    (256, (16, 8), 1 << 20, 8192),
)


def serve_strategy(s: int, realization: int = 0, noiseless: bool = False,
                   shapes=None, L: int = 1 << 16) -> Problem:
    """Strategy s of the serving trace.  Pointing and noise model are fixed per
    strategy; the sky and noise realisation change with `realization`.
    `shapes` = (n_side, grid, samples/detector, lambda) overrides the table
    (smaller instances for tests)."""
    n_side, grid, spd, lam = shapes if shapes is not None else SERVE_STRATEGIES[s]
    n_det = grid[0] * grid[1]
    pix = rotated_raster(n_side, grid, spd)
    fk = rng_for(50 + s, 0, STREAM_FKNEE).uniform(0.05, 1.0, n_det)
    p = _finish(f"s{s}", 50 + s, 0, n_side, pix, L, lam, fk, spd, True)
    if realization != 0 or not noiseless:
        sky = white_sky(rng_for(50 + s, realization, STREAM_SIGNAL), p.n_pix_total)
        d = signal_tod(p.pix, p.psi, sky)
        if not noiseless:
            noise = noise_1f(rng_for(50 + s, realization, STREAM_NOISE), L,
                             p.n_intervals, fk[p.filter_id]).reshape(-1)
            d = d + noise
        p.signal, p.tod = sky, d
    return p


def poisson_arrivals(n: int, rate: float = 4.0, seed: int = 0):
    """Request arrival times (s), exponential gaps; strategy uniform over the
    four serving strategies; tolerance 1e-6 or 1e-8 with probability 1/2."""
    rng = rng_for(5, seed, STREAM_ARRIVALS)
    gaps = rng.exponential(1.0 / rate, n)
    strat = rng.integers(0, len(SERVE_STRATEGIES), n)
    tol = np.where(rng.random(n) < 0.5, 1e-6, 1e-8)
    return np.cumsum(gaps), strat, tol


def random_problem(seed: int, n_side: int = 4, n_samp: int = 2048, n_int: int = 4,
                   half_bw: int = 8, n_filters: int = 2, flag_frac: float = 0.05,
                   noiseless: bool = False, ragged: bool = True,
                   min_hits: int = 3) -> Problem:
    """Small random pointing for brute-force checks: uniform random pixels,
    some flagged samples, uneven interval lengths, several filters."""
    rng = rng_for(100, seed, STREAM_SCAN)
    n_pix_total = n_side * n_side
    pix = rng.integers(0, n_pix_total, n_samp).astype(np.int32)
    pix[rng.random(n_samp) < flag_frac] = -1
    psi = rng_for(100, seed, STREAM_PSI).uniform(0.0, math.pi, n_samp)
    if ragged and n_int > 1:
        w = rng.uniform(0.75, 1.25, n_int)
        lengths = np.floor(w / w.sum() * n_samp).astype(np.int64)
        lengths[-1] = n_samp - lengths[:-1].sum()
    else:
        lengths = np.full(n_int, n_samp // n_int, dtype=np.int64)
        lengths[-1] = n_samp - lengths[:-1].sum()
    istart = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    L_min = int(np.min(np.diff(istart)))
    assert L_min > 2 * half_bw, (L_min, half_bw)
    filter_id = rng.integers(0, n_filters, n_int).astype(np.int32)
    fk = rng_for(100, seed, STREAM_FKNEE).uniform(0.05, 1.0, n_filters)
    band = np.stack([band_from_psd(max(L_min, 2 * half_bw + 2), half_bw, f) for f in fk])
    sky = white_sky(rng_for(100, seed, STREAM_SIGNAL), n_pix_total)
    d = signal_tod(pix, psi, sky)
    noise = None
    if not noiseless:
        noise = rng_for(100, seed, STREAM_NOISE).standard_normal(n_samp)
        d = d + noise
    return Problem(name=f"rand{seed}", n_side=n_side, n_pix_total=n_pix_total, pix=pix,
                   psi=psi, interval_start=istart, filter_id=filter_id, band=band,
                   half_bw=half_bw, signal=sky, tod=d, min_hits=min_hits, noise=noise)
