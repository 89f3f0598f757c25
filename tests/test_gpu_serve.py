"""Serving loop (libism server) on the GPU: every solve served in a mix of concurrent
requests, alone or merged with others into one batched handle, returns exactly what it
returns when served alone and what ism_iterate returns on its own handle (bitwise equal
controls), the iterates follow the oracle's plain gradient method, and admission respects
the memory budget."""
import sys

import numpy as np
import pytest

import problems
from oracle import finite as O

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mix():
    """Small requests of every served family: (problem, rho, max_iter, fid_stop, precision)."""
    base = problems.spin2(K=12, N=3)
    rng = np.random.default_rng(5)
    gate = problems.FiniteProblem("g", base.H0, base.Hc, np.eye(4, dtype=complex),
                                  problems.haar_unitary(4, rng), 1.0, 12, 3,
                                  rng.uniform(-1, 1, (1, 12, 2)), np.zeros(12), 0.5, 1,
                                  kind="gate")
    return [
        (problems.spin2(seed=7, K=200, N=8, T=2.0), 0.5, 12, 2.0, "fp64"),
        (problems.spin2(seed=8, K=150, N=5, T=2.0), 0.5, 40, 0.9, "fp32"),
        (problems.rotor(seed=9, batch=1, jmax=10, T=2.0, K=300, N=16), 1.0, 7, 2.0, "fp32"),
        (problems.rotor(seed=10, batch=1, jmax=20, T=1.0, K=257, N=19), 1.0, 5, 2.0, "fp64"),
        (problems.spin_chain_state(11, n=4, T=1.0, K=64, N=4), 0.5, 6, 2.0, "fp32"),
        (problems.gpe(seed=12, n=1024, K=120, N=6), 0.1, 4, 2.0, "fp64"),
        (gate, 0.5, 5, 2.0, "fp64"),
        (problems.spin2(seed=13, K=40, N=4), 0.5, 0, 2.0, "fp64"),          # no update at all
    ]


def _serve(items, budget=8 << 30, ipr=3, max_running=16):
    from paper_1603_01237_amd import Server
    out = {}
    with Server(budget, iters_per_round=ipr, max_running=max_running) as s:
        tickets = [s.submit(p, max_iter=mi, rho=rho, fid_stop=fs, precision=pr)
                   for (p, rho, mi, fs, pr) in items]
        for _ in range(200000):
            q, r = s.progress()
            if q == 0 and r == 0:
                break
        else:
            raise AssertionError("server did not drain")
        for k, t in enumerate(tickets):
            out[k] = s.take(t)
        stats = s.stats()
    return out, stats


def test_mix_equals_alone_and_iterate():
    from paper_1603_01237_amd import _lib
    items = _mix()
    _say("case serve mix", len(items))
    mixed, st = _serve(items)
    assert st["completed"] == len(items) and st["failed"] == 0
    for k, it in enumerate(items):
        _say("case serve alone", k)
        alone, _ = _serve([it])
        rm, um = mixed[k]
        ra, ua = alone[0]
        assert rm["state"] == _lib.REQ_DONE and ra["state"] == _lib.REQ_DONE, (rm, ra)
        assert rm["iters"] == ra["iters"]
        assert np.array_equal(um, ua)
        assert rm["F"] == ra["F"] and rm["J"] == ra["J"]
        p, rho, mi, fs, pr = it
        with _lib.from_problem(p, precision=pr) as h:
            _, done = h.iterate(mi, rho, fid_stop=fs)
            u = h.get_controls()[0]
            J, F = h.fidelity()
        assert done == rm["iters"]
        assert np.array_equal(u, um), k
        assert F[0] == rm["F"]


def test_served_iterates_follow_the_plain_gradient_method():
    from paper_1603_01237_amd import _lib
    p = problems.spin2(seed=7, K=200, N=8, T=2.0)
    _say("case serve oracle")
    res, _ = _serve([(p, 0.5, 12, 2.0, "fp64")])
    r, u = res[0]
    ref = O.plain_gradient_method(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 0.5, 12)
    assert r["iters"] == 12
    assert np.linalg.norm(u - ref["u"]) / np.linalg.norm(ref["u"]) <= 1e-10
    Fr = O.gradient(p.H0, p.Hc, p.psi0, p.target, ref["u"], p.T, p.alpha)[2]
    assert abs(r["F"] - Fr) <= 1e-10


def test_fid_stop_ends_a_request_early():
    from paper_1603_01237_amd import _lib
    p = problems.spin2(seed=8, K=100, N=4, T=2.0)
    _say("case serve fid_stop")
    res, _ = _serve([(p, 0.5, 200, 0.9, "fp64")], ipr=7)
    r, u = res[0]
    assert r["state"] == _lib.REQ_DONE
    assert 0 < r["iters"] < 200 and r["F"] >= 0.9
    with _lib.from_problem(p) as h:
        _, done = h.iterate(200, 0.5, fid_stop=0.9)
        assert done == r["iters"]
        assert np.array_equal(h.get_controls()[0], u)


def test_budget_admission_and_rejection():
    from paper_1603_01237_amd import IsmError, Server, _lib
    items = [(problems.rotor(seed=20 + i, batch=1, jmax=20, T=1.0, K=400, N=16), 1.0, 3, 2.0,
              "fp32") for i in range(4)]
    fp = _lib.footprint(21, 1, 400, 16, 1, _lib.STATE, _lib.FP32_MIXED)
    _say("case serve budget", fp)
    res, st = _serve(items, budget=int(1.5 * fp))        # one request on the device at a time
    assert st["completed"] == 4 and st["bytes_peak"] <= int(1.5 * fp)
    alone, _ = _serve(items[:1])
    assert np.array_equal(res[0][1], alone[0][1])
    with Server(fp // 2) as s:
        with pytest.raises(IsmError) as e:
            s.submit(items[0][0], max_iter=1, rho=1.0)
        assert e.value.code == _lib.ISM_E_BUDGET


def test_failed_request_reports_status_and_others_complete():
    from paper_1603_01237_amd import _lib
    good = problems.spin2(seed=30, K=50, N=5, T=2.0)
    bad = problems.spin2(seed=31, K=50, N=5, T=2.0)
    bad.Hc = bad.Hc.copy()
    bad.Hc[0, 0, 1] = 0.7              # not Hermitian: rejected when the handle is created
    _say("case serve failure")
    res, st = _serve([(bad, 0.5, 3, 2.0, "fp64"), (good, 0.5, 3, 2.0, "fp64")])
    assert res[0][0]["state"] == _lib.REQ_FAILED and res[0][0]["status"] == _lib.ISM_E_ARG
    assert res[0][1] is None
    assert res[1][0]["state"] == _lib.REQ_DONE and res[1][0]["iters"] == 3


def test_trace_replay_sample():
    """The first requests of the seeded 200 req/s trace, replayed at their arrival times
    (GPE and 256-dimensional spin requests capped to keep the test short)."""
    from paper_1603_01237_amd import Server
    from paper_1603_01237_amd.serve import latency_summary, replay
    trace = [r for r in problems.serving_trace()
             if not (r["type"] == "gpe" or (r["type"] == "spin" and r["size"] >= 64))][:12]
    items = [(r["arrival"] - trace[0]["arrival"], problems.request_problem(r),
              dict(max_iter=3, rho=problems.SERVE_RHO[r["type"]], fid_stop=0.99,
                   precision="fp32")) for r in trace]
    _say("case serve replay", len(items))
    with Server(32 << 30, iters_per_round=3, max_running=16) as s:
        recs, wall = replay(s, items, timeout=120.0)
    summ = latency_summary(recs, wall)
    _say(summ)
    assert summ["completed"] == len(items) and summ["failed"] == 0
    assert all(r["latency_s"] >= 0 and r["queue_s"] >= 0 for r in recs)


def test_merged_requests_equal_their_lone_runs():
    """Requests that differ only in the diagonal of H0 (rotors with their own rotational
    constant and initial controls; two-spin transfers with their own initial controls, frozen
    at different iterations by the fidelity rule) are admitted into one batched handle each;
    every merged request returns bitwise what it returns alone and what ism_iterate returns
    on its own handle.  Requests of another shape or stopping rule are not merged."""
    from paper_1603_01237_amd import _lib
    rot = [(problems.rotor(seed=40 + i, batch=1, jmax=20, T=1.0, K=300, N=12), 1.0, 6, 2.0,
            "fp32") for i in range(5)]
    spins = []
    for i, scale in enumerate((0.5, 1.0, 2.0, 3.0)):       # different starts: they freeze apart
        q = problems.spin2(seed=50 + i, K=100, N=4, T=2.0)
        q.u0 = q.u0 * scale
        spins.append((q, 0.5, 200, 0.9, "fp64"))
    other = [(problems.rotor(seed=60, batch=1, jmax=20, T=1.0, K=301, N=12), 1.0, 6, 2.0, "fp32"),
             (problems.rotor(seed=61, batch=1, jmax=20, T=1.0, K=300, N=12), 1.0, 5, 2.0, "fp32")]
    items = rot + spins + other
    _say("case serve merge", len(items))
    res, st = _serve(items, ipr=4)
    assert st["completed"] == len(items) and st["failed"] == 0
    assert st["merged"] == (len(rot) - 1) + (len(spins) - 1), st
    assert st["groups"] == 2 + len(other), st
    iters_spins = set()
    for k, it in enumerate(items):
        alone, _ = _serve([it], ipr=4)
        rm, um = res[k]
        ra, ua = alone[0]
        assert rm["state"] == _lib.REQ_DONE and ra["state"] == _lib.REQ_DONE
        assert rm["iters"] == ra["iters"], (k, rm, ra)
        assert np.array_equal(um, ua), k
        assert rm["F"] == ra["F"] and rm["J"] == ra["J"], k
        p, rho, mi, fs, pr = it
        with _lib.from_problem(p, precision=pr) as h:
            _, done = h.iterate(mi, rho, fid_stop=fs)
            assert done == rm["iters"]
            assert np.array_equal(h.get_controls()[0], um), k
        if len(rot) <= k < len(rot) + len(spins):
            iters_spins.add(rm["iters"])
    assert len(iters_spins) > 1           # the merged spins froze at different iterations


def test_merged_condensate_requests_equal_their_lone_runs():
    """Condensate requests on one grid, potential, time grid and stopping rule that differ
    only in their initial controls share one batched handle (one workgroup per instance in
    every kernel of the path): each returns bitwise what it returns alone and what
    ism_iterate returns on its own handle.  A request with another slice count runs apart."""
    from paper_1603_01237_amd import _lib
    same = [(problems.gpe(seed=70 + i, n=64, L=20.0, g=1.0, dt=8.0 / 256, K=256, N=8,
                          x_target=1.0), 0.1, 5, 2.0, "fp64") for i in range(3)]
    other = [(problems.gpe(seed=80, n=64, L=20.0, g=1.0, dt=8.0 / 256, K=256, N=4,
                           x_target=1.0), 0.1, 5, 2.0, "fp64")]
    items = same + other
    _say("case serve merge condensate", len(items))
    res, st = _serve(items, ipr=2)
    assert st["completed"] == len(items) and st["failed"] == 0
    assert st["merged"] == len(same) - 1, st
    assert st["groups"] == 2, st
    for k, it in enumerate(items):
        alone, _ = _serve([it], ipr=2)
        rm, um = res[k]
        ra, ua = alone[0]
        assert rm["state"] == _lib.REQ_DONE and ra["state"] == _lib.REQ_DONE
        assert rm["iters"] == ra["iters"] == it[2], (k, rm, ra)
        assert np.array_equal(um, ua), k
        assert rm["F"] == ra["F"] and rm["J"] == ra["J"], k
        p, rho, mi, fs, pr = it
        with _lib.from_problem(p, precision=pr) as h:
            _, done = h.iterate(mi, rho, fid_stop=fs)
            assert done == rm["iters"]
            assert np.array_equal(h.get_controls()[0, :, 0], np.ravel(um)), k

