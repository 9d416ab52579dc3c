"""Device-side synthesis of request data for the serving benchmark.

Each serving request needs a fresh time stream of up to 2^27 samples, which
the numpy generators would take seconds to draw.  These functions draw the
same kind of data on the GPU with torch: 1/f noise by the recipe of
``synth.noise_1f`` (a seeded complex spectrum with the model PSD, inverse real
FFT per stationary interval) and the signal part of the data model, sky values
at each sample's pixel combined with (1, cos 2psi, sin 2psi).  The draws are
seeded from the same (cfg, realization, stream) triples but come from torch's
generator, so they are not bit-identical to the numpy versions.  Nothing here
is used by the oracle or by the library.
"""
from __future__ import annotations

import numpy as np

from . import F_SAMP, NOISE_ALPHA, NOISE_SIGMA, psd_1f


def _seed(cfg: int, realization: int, stream: int) -> int:
    ss = np.random.SeedSequence([cfg, realization, stream])
    return int(ss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1))


def noise_1f(cfg: int, realization: int, stream: int, L: int, fknee_per_interval,
             device, chunk: int = 256):
    """f64[n_int * L] on `device`: independent 1/f noise per interval, PSD
    sigma^2 (1 + (fknee/f)^alpha), X_0 = 0 and a real Nyquist term."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(_seed(cfg, realization, stream))
    fk = np.asarray(fknee_per_interval, dtype=np.float64)
    n_int = fk.shape[0]
    kf = np.arange(1, L // 2 + 1, dtype=np.float64) * F_SAMP / L
    out = torch.empty(n_int * L, dtype=torch.float64, device=device)
    uniq, inv = np.unique(fk, return_inverse=True)
    amp_tab = torch.from_numpy(np.stack([np.sqrt(L * psd_1f(kf, NOISE_SIGMA, f, NOISE_ALPHA) / 2.0)
                                         for f in uniq])).to(device)
    inv_t = torch.from_numpy(inv.astype(np.int64)).to(device)
    for i0 in range(0, n_int, chunk):
        i1 = min(n_int, i0 + chunk)
        m = i1 - i0
        a = torch.randn((m, L // 2 + 1), dtype=torch.float64, device=device, generator=gen)
        b = torch.randn((m, L // 2 + 1), dtype=torch.float64, device=device, generator=gen)
        amp = amp_tab[inv_t[i0:i1]]
        X = torch.zeros((m, L // 2 + 1), dtype=torch.complex128, device=device)
        X[:, 1:] = torch.complex(amp * a[:, 1:], amp * b[:, 1:])
        X[:, -1] = torch.complex(amp[:, -1] * np.sqrt(2.0) * a[:, -1],
                                 torch.zeros(m, dtype=torch.float64, device=device))
        out[i0 * L:i1 * L] = torch.fft.irfft(X, n=L, dim=1).reshape(-1)
    return out


def signal(pix, psi, sky, device):
    """d_t = I + Q cos 2psi + U sin 2psi at the sample's pixel, 0 if flagged.
    pix int32, psi f64 (device tensors); sky f64[n_pix, 3] (numpy)."""
    import torch
    s = torch.from_numpy(np.ascontiguousarray(sky)).to(device)
    ok = pix >= 0
    j = torch.where(ok, pix, torch.zeros_like(pix)).long()
    d = s[j, 0] + torch.cos(2.0 * psi) * s[j, 1] + torch.sin(2.0 * psi) * s[j, 2]
    return torch.where(ok, d, torch.zeros_like(d))
