"""Helpers shared by the GPU tests: device tensors from numpy, and building
library objects and oracle objects from the same synthetic problem."""
import numpy as np

import oracle as O


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def build_both(ctx, p, prec=0, method=0, min_hits=None):
    """Library pointing+noise and oracle pointing+noise for one problem."""
    import torch
    mh = p.min_hits if min_hits is None else min_hits
    lp = ctx.pointing(dev(p.pix), dev(p.psi), p.n_pix_total, mh, prec)
    ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw, method, prec)
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, mh)
    on = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    return lp, ln, op, on


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
