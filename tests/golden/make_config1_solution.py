"""Writes config1_solution.json: the FP64 oracle's map for the config-1 problem
(M_BD PCG to a 1e-13 relative residual) and the right-hand side's norm, the
reference of the FP32 form's map error.  Calls only oracle/ and synth/.

    python tests/golden/make_config1_solution.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import synth  # noqa: E402


def solve():
    p = synth.config1()
    op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
    on = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
    M = O.mbd_build(op, on)
    b = O.rhs(op, on, p.tod)
    x, info = O.pcg(lambda v: O.apply_A(op, on, v), lambda v: O.mbd_apply(M, v), b, 1e-13, 5000)
    assert info.converged
    return x, b, info


if __name__ == "__main__":
    x, b, info = solve()
    out = {"what": "FP64 oracle map of config 1 (M_BD PCG to 1e-13), [n_obs][3] IQU",
           "iters": info.iters, "rel_res_true": info.rel_res_true,
           "b_norm": float(np.linalg.norm(b)), "x": [float(v) for v in x]}
    with open(os.path.join(HERE, "config1_solution.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote {len(x)} values, {info.iters} iterations, residual {info.rel_res_true:.2e}")
