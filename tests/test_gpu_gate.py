"""GPU parity of the dense gate path (batched complex GEMM on MFMA) against the FP64 oracle.

Gate synthesis: psi0 = I, target W, <A|B> = Tr(A^+ B)/d (evolution-operator form of Sec. 2).
Tolerances as for the state path: FP64 relative L2 <= 1e-12 at every size, FP32 mixed ||U_gpu(T) - U_ref(T)||_F / sqrt(d) <= 1e-4 and gradient relative L2
<= 1e-3.
"""
import sys

import numpy as np
import pytest

import problems
from oracle import finite as O

pytestmark = pytest.mark.gpu


def _P():
    from paper_1603_01237_amd import _lib
    return _lib


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gate_problem(n, K, N, seed=5, T=None):
    p = problems.spin_chain_gate(seed=seed, n=n, K=K, N=N, T=T if T is not None else K * 0.01)
    return p


def _spin2_gate(K, N, seed=3, T=1.0):
    p = problems.spin2(K=K, N=N, T=T)
    rng = np.random.default_rng(seed)
    W = problems.haar_unitary(4, rng)
    u = rng.uniform(-1, 1, size=(1, K, 2))
    return problems.FiniteProblem("spin2_gate", p.H0, p.Hc, np.eye(4, dtype=complex), W, p.T, K,
                                  N, u, np.zeros(K), 0.5, 5, kind="gate")


CASES = [
    ("spin2_gate_K24_N3", lambda: _spin2_gate(24, 3)),
    ("spin2_gate_K17_N5", lambda: _spin2_gate(17, 5)),
    ("spin2_gate_K1_N1_single_step", lambda: _spin2_gate(1, 1, T=0.1)),
    ("chain4_gate_K30_N4", lambda: _gate_problem(4, 30, 4)),
    ("chain6_gate_K13_N13", lambda: _gate_problem(6, 13, 13)),
    # slices long enough for the chunked assembly scan (local chains, carries, fix-up)
    ("chain6_gate_K300_N3_scan64", lambda: _gate_problem(6, 300, 3)),
    ("spin2_gate_K400_N1_scan32", lambda: _spin2_gate(400, 1, T=4.0)),
    # 16 or more slices: the FP64 boundaries run as a chunked scan (ragged chunks at N = 19)
    ("chain4_gate_K57_N19_bscan", lambda: _gate_problem(4, 57, 19)),
    ("spin2_gate_K40_N20_bscan", lambda: _spin2_gate(40, 20, T=2.0)),
    # d = 160: padded to 192 rows, two column blocks of the gradient (the second partly
    # filled); d = 100: padded to 128; d = 24: groups of 32 lanes with dead rows in each
    ("banded_gate_d160_K6_N2", lambda: problems.banded_gate(d=160, K=6, N=2)),
    ("banded_gate_d100_K9_N3", lambda: problems.banded_gate(seed=7, d=100, K=9, N=3, T=0.09)),
    ("banded_gate_d24_K20_N4", lambda: problems.banded_gate(seed=8, d=24, K=20, N=4, T=0.2)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gate_parity(name, mk, prec):
    _say("case", name, prec)
    P = _P()
    p = mk()
    with P.from_problem(p, precision=prec) as h:
        UT = h.forward()[0]
        J, F = h.fidelity()
        g = h.gradient()[0]
    gr, Jr, Fr, UK = O.gradient(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha)
    d = p.d
    if prec == "fp64":
        assert _rel(UT, UK) <= 1e-12
        assert abs(J[0] - Jr) <= 1e-12 and abs(F[0] - Fr) <= 1e-12
        assert _rel(g, gr) <= 1e-12, _rel(g, gr)
    else:
        assert np.linalg.norm(UT - UK) / np.sqrt(d) <= 1e-4
        assert abs(F[0] - Fr) <= 1e-4
        assert _rel(g, gr) <= 1e-3, _rel(g, gr)


def test_gate_iterate_equals_plain():
    _say("case gate iterate")
    P = _P()
    p = _gate_problem(4, 40, 6)
    ref = O.plain_gradient_method(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 0.5, 5)
    with P.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate(5, 0.5)
        u = h.get_controls()[0]
    assert done == 5
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-12
    assert _rel(u, ref["u"]) <= 1e-12


def test_gate_full_size_sampled():
    """8-spin chain gate synthesis at its full size (d=256, 16 controls, K=2000, N=64):
    U(T) against the oracle's product of step exponentials (FP64 relative 1e-12); the gradient
    at one step of every slice (FP64 relative 1e-12 per step)."""
    _say("case gate full size")
    P = _P()
    p = problems.spin_chain_gate()
    res = {}
    for prec in ("fp32", "fp64"):
        with P.from_problem(p, precision=prec) as h:
            res[prec] = (h.forward()[0], h.gradient()[0])
            _say(prec, "done")
    tau = p.T / p.K
    u = p.u0[0]
    Us = O.step_unitaries(p.H0, p.Hc, u, tau)
    psis = O.forward(Us, p.psi0)
    lams = O.backward(Us, p.target)
    UK = psis[-1]
    for prec in ("fp32", "fp64"):
        UT, g = res[prec]
        errU = np.linalg.norm(UT - UK) / np.sqrt(p.d)
        _say(prec, "U(T) err", errU)
        if prec == "fp64":
            assert _rel(UT, UK) <= 1e-12
        else:
            assert errU <= 1e-4
    # one step in every slice, at a different position in each (n mod the slice length), and
    # the last step
    s = O.slice_starts(p.K, p.N)
    steps = [int(s[n] + n % (s[n + 1] - s[n])) for n in range(p.N)] + [p.K - 1]
    worst = [0.0, 0.0]
    for j in steps:
        Hh = O.hhat(O.hamiltonian(p.H0, p.Hc, u[j]), p.Hc, tau)
        gref = np.array([np.trace(lams[j].conj().T @ Hh[c] @ psis[j]).imag / p.d
                         for c in range(p.C)])
        e64 = _rel(res["fp64"][1][j], gref)
        e32 = _rel(res["fp32"][1][j], gref)
        worst = [max(worst[0], e64), max(worst[1], e32)]
        assert e64 <= 1e-12, (j, e64)
        assert e32 <= 1e-3, (j, e32)
    _say("gradient over", len(steps), "steps: fp64 worst", worst[0], "fp32 worst", worst[1])
