"""Serving form: continuous batching of map-making solves over recurring scan
strategies (mm_server_*), through the C ABI."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu

SMALL = [(32, (4, 2), 1 << 12, 128), (64, (4, 4), 1 << 13, 256)]


def _strategy(s, r):
    return synth.serve_strategy(s, r, shapes=SMALL[s], L=1 << 11)


@pytest.fixture(scope="module")
def mm():
    import torch
    assert torch.cuda.is_available()
    from paper_1801_08937_amd import mapmaker
    return mapmaker


# A served result is compared with the oracle's solution of its own system
# (PCG to 1e-13): relative map error <= KAPPA * tol (1e-6 at tol 1e-8, 1e-4 at
# 1e-6, the bar of the other solve tests), and its true residual under the
# oracle's A <= 1.5 tol.
KAPPA = 100.0
_ORACLE = {}


def _oracle_system(s):
    if s not in _ORACLE:
        p = _strategy(s, 0)
        op = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
        on = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
        _ORACLE[s] = (p.pix, op, on, O.mbd_build(op, on))
    return _ORACLE[s]


def _check_vs_oracle(outs, infos, tols):
    """Every result against the oracle, at the bar stated above; returns the
    errors (printed by the callers)."""
    errs = []
    for (x, tod, p), info, tol in zip(outs, infos, tols):
        pix, op, on, OM = _oracle_system(int(p.name[1:]))
        assert np.array_equal(pix, p.pix)
        A = lambda v: O.apply_A(op, on, v, "fft")
        bo = O.rhs(op, on, p.tod, "fft")
        xo, io = O.pcg(A, lambda v: O.mbd_apply(OM, v), bo, 1e-13, 5000)
        assert io.converged
        xg = host(x)
        e = rel(xg, xo)
        r = float(np.linalg.norm(bo - A(xg)) / np.linalg.norm(bo))
        errs.append((e, r))
        assert info["state"] == 2 and e <= KAPPA * tol and r <= 1.5 * tol, (e, r, tol, info)
    return errs


def _server(mm, slots=4, k=8):
    srv = mm.Server(0, hbm_budget_bytes=8 << 30, slots=slots, defl_k=k, iters_per_step=3)
    for s in range(2):
        p = _strategy(s, 0)
        srv.add_strategy(s, dev(p.pix), dev(p.psi), p.n_pix_total, p.interval_start,
                         p.filter_id, p.band, p.half_bw, grid_width=p.n_side)
    return srv


def _run(srv, reqs, join_after=1):
    """reqs: list of (strategy, realization, tol); the first is submitted,
    `join_after` steps run, then the rest join mid-flight."""
    import torch
    outs, ids = [], []
    for i, (s, r, tol) in enumerate(reqs):
        p = _strategy(s, r)
        x = torch.zeros(3 * int(np.sum(np.bincount(p.pix[p.pix >= 0], minlength=p.n_pix_total)
                                       >= p.min_hits)), dtype=torch.float64, device="cuda")
        tod = dev(p.tod)
        outs.append((x, tod, p))
        ids.append(srv.submit(s, tod, x, tol=tol))
        if i == 0:
            for _ in range(join_after):
                srv.step()
    for _ in range(2000):
        run, q = srv.step()
        if run == 0 and q == 0:
            break
    return [srv.poll(i) for i in ids], outs


def test_server_result_same_alone_and_in_mix(mm):
    import torch
    srv = _server(mm)
    infos_a, outs_a = _run(srv, [(0, 1, 1e-8)])
    srv.close()
    srv = _server(mm)
    infos_b, outs_b = _run(srv, [(0, 1, 1e-8), (0, 2, 1e-6), (1, 3, 1e-8), (0, 4, 1e-8),
                                 (1, 5, 1e-6)], join_after=2)
    srv.close()
    assert infos_a[0]["state"] == 2 and all(i["state"] == 2 for i in infos_b)
    # the first request's map: bitwise the same alone and with four others joining
    assert infos_a[0]["iters"] == infos_b[0]["iters"]
    assert torch.equal(outs_a[0][0], outs_b[0][0])
    assert infos_b[0]["m2l_built"] == 1 and infos_b[1]["m2l_built"] == 0
    # the request that starts the (background) M_2l build is solved with M_BD
    assert infos_a[0]["precond"] == 0 and infos_b[0]["precond"] == 0
    errs = _check_vs_oracle(outs_b, infos_b, (1e-8, 1e-6, 1e-8, 1e-8, 1e-6))
    print("served vs oracle (map error, true residual):", errs)


def _warm(srv, strategies=(0, 1)):
    """One request per strategy, then step until every M_2l cache is ready."""
    import time
    infos, _ = _run(srv, [(s, 90 + s, 1e-6) for s in strategies])
    t0 = time.time()
    while any(srv.strategy_state(s) == 1 for s in strategies):
        srv.step()
        time.sleep(0.01)
        assert time.time() - t0 < 60, "M_2l build did not finish"
    assert all(srv.strategy_state(s) == 2 for s in strategies)
    return infos


def _run_each_alone(srv, reqs):
    """Each request by itself on the server (nothing else in flight)."""
    infos, outs = [], []
    for r in reqs:
        i, o = _run(srv, [r])
        infos += i
        outs += o
    return infos, outs


def test_server_m2l_lane_same_alone_and_in_mix(mm):
    """Once a strategy's M_2l is cached, its requests run in the M_2l session;
    every request's map is bitwise the same alone and with others joining,
    and each solves its own system (oracle bar)."""
    import torch
    reqs = [(0, 7, 1e-8), (0, 8, 1e-6), (1, 9, 1e-8), (0, 11, 1e-8), (1, 12, 1e-6)]
    srv = _server(mm)
    _warm(srv)
    infos_a, outs_a = _run_each_alone(srv, reqs)
    infos_b, outs_b = _run(srv, reqs, join_after=2)
    srv.close()
    assert all(i["state"] == 2 and i["precond"] == 1 for i in infos_a + infos_b)
    for ia, ib, oa, ob in zip(infos_a, infos_b, outs_a, outs_b):
        assert ia["iters"] == ib["iters"]
        assert torch.equal(oa[0], ob[0])
    errs = _check_vs_oracle(outs_b, infos_b, [t for _, _, t in reqs])
    print("M_2l lane vs oracle (map error, true residual):", errs)


def test_server_continuous_batching_many(mm):
    srv = _server(mm, slots=4)
    reqs = [(i % 2, 10 + i, 1e-8 if i % 3 else 1e-6) for i in range(14)]
    infos, outs = _run(srv, reqs, join_after=1)
    srv.close()
    assert all(i["state"] == 2 for i in infos)
    assert sum(i["m2l_built"] for i in infos) == 2   # one M_2l per strategy, then cached
    # more requests than slots: some waited in the queue for a slot and were admitted later
    assert max(i["queue_seconds"] for i in infos) > 0
    assert any(i["waited"] & 1 for i in infos) and not any(i["waited"] & 2 for i in infos)
    errs = _check_vs_oracle(outs, infos, [t for _, _, t in reqs])
    print("14 requests vs oracle (map error, true residual):", errs)


def test_server_budget_rejects(mm):
    srv = mm.Server(0, hbm_budget_bytes=1 << 20, slots=4, defl_k=8)
    p = _strategy(1, 0)
    with pytest.raises(mm.MapmakerError) as e:
        srv.add_strategy(1, dev(p.pix), dev(p.psi), p.n_pix_total, p.interval_start,
                         p.filter_id, p.band, p.half_bw)
    assert e.value.name == "MM_E_BUSY"
    srv.close()


def test_server_prebuilt_m2l(mm):
    """With M_2l built at registration, every request (the first included)
    runs with M_2l, a request's map is bitwise the same alone and in a mix,
    and it solves its own system."""
    import torch
    srv = mm.Server(0, hbm_budget_bytes=8 << 30, slots=4, defl_k=8, iters_per_step=3,
                    prebuild=True)
    for s in range(2):
        p = _strategy(s, 0)
        srv.add_strategy(s, dev(p.pix), dev(p.psi), p.n_pix_total, p.interval_start,
                         p.filter_id, p.band, p.half_bw, grid_width=p.n_side)
    assert all(srv.strategy_state(s) == 2 for s in range(2))
    reqs = [(0, 21, 1e-8), (1, 22, 1e-8), (0, 23, 1e-6)]
    infos_a, outs_a = _run_each_alone(srv, reqs)
    infos_b, outs_b = _run(srv, reqs, join_after=2)
    srv.close()
    assert all(i["state"] == 2 and i["precond"] == 1 and i["m2l_built"] == 0
               for i in infos_a + infos_b)
    for oa, ob in zip(outs_a, outs_b):
        assert torch.equal(oa[0], ob[0])
    errs = _check_vs_oracle(outs_b, infos_b, [t for _, _, t in reqs])
    print("prebuilt M_2l vs oracle (map error, true residual):", errs)


def test_server_admits_by_memory(mm):
    """Admission by HBM footprint: with a budget that holds both strategies'
    resident data but only one lane session, a request of the second
    strategy waits for memory -- with its lane's slots all free -- while the
    first strategy's session runs, and is admitted once that request retires
    and its idle session is evicted.  Both maps are bitwise the solo ones
    and solve their systems (oracle bar)."""
    import torch
    big = mm.Server(0, hbm_budget_bytes=8 << 30, slots=4, defl_k=0, iters_per_step=3)
    for s in range(2):
        p = _strategy(s, 0)
        big.add_strategy(s, dev(p.pix), dev(p.psi), p.n_pix_total, p.interval_start,
                         p.filter_id, p.band, p.half_bw, grid_width=p.n_side)
    mem = [big.memory(s) for s in range(2)]
    reqs = [(0, 31, 1e-8), (1, 32, 1e-8)]
    infos_a, outs_a = _run_each_alone(big, reqs)
    big.close()
    budget = mem[0]["resident"] + mem[1]["resident"] + max(m["session"] for m in mem) + 1
    assert budget < mem[0]["resident"] + mem[1]["resident"] + mem[0]["session"] + mem[1]["session"]
    srv = mm.Server(0, hbm_budget_bytes=budget, slots=4, defl_k=0, iters_per_step=3)
    for s in range(2):
        p = _strategy(s, 0)
        srv.add_strategy(s, dev(p.pix), dev(p.psi), p.n_pix_total, p.interval_start,
                         p.filter_id, p.band, p.half_bw, grid_width=p.n_side)
    assert srv.memory()["used"] == mem[0]["resident"] + mem[1]["resident"]
    infos_b, outs_b = _run(srv, reqs, join_after=0)
    assert srv.memory()["used"] <= budget
    srv.close()
    print("memory:", mem, "budget", budget, "requests:", infos_b)
    assert infos_b[0]["waited"] == 0
    assert infos_b[1]["waited"] & 2 and not infos_b[1]["waited"] & 1   # memory, not a slot
    assert infos_b[1]["queue_seconds"] > 0
    for oa, ob in zip(outs_a, outs_b):
        assert torch.equal(oa[0], ob[0])
    _check_vs_oracle(outs_b, infos_b, [t for _, _, t in reqs])


def test_server_residual_rule_m2l(mm):
    """The background M_2l built with the residual stop rule (App. A, second
    reading of the eps_Arn test; mm_server_set_arnoldi): the cache is built,
    the M_2l lane serves requests that meet the oracle bar, bitwise the same
    alone and in a mix; setting the parameters after a strategy is
    registered is refused."""
    import torch
    srv = mm.Server(0, hbm_budget_bytes=8 << 30, slots=4, defl_k=8, iters_per_step=3,
                    arnoldi=("residual", 1e-10, 128))
    for s in range(2):
        p = _strategy(s, 0)
        srv.add_strategy(s, dev(p.pix), dev(p.psi), p.n_pix_total, p.interval_start,
                         p.filter_id, p.band, p.half_bw, grid_width=p.n_side)
    from paper_1801_08937_amd.mapmaker import lib
    assert lib().mm_server_set_arnoldi(srv.h, 1, 1e-10, 128) != 0
    _warm(srv)
    reqs = [(0, 21, 1e-8), (1, 22, 1e-8), (0, 23, 1e-6)]
    infos_a, outs_a = _run_each_alone(srv, reqs)
    infos_b, outs_b = _run(srv, reqs, join_after=1)
    srv.close()
    assert all(i["state"] == 2 and i["precond"] == 1 for i in infos_a + infos_b)
    for ia, ib, oa, ob in zip(infos_a, infos_b, outs_a, outs_b):
        assert ia["iters"] == ib["iters"]
        assert torch.equal(oa[0], ob[0])
    errs = _check_vs_oracle(outs_b, infos_b, [t for _, _, t in reqs])
    print("residual-rule M_2l lane vs oracle (map error, true residual):", errs)
    with pytest.raises(mm.MapmakerError):
        mm.Server(0, hbm_budget_bytes=8 << 30, slots=4, defl_k=8, arnoldi=("residual", -1.0, 128))
