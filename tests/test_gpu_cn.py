"""GPU parity of the Crank-Nicolson step map (sparse state path) against the FP64 oracle.

Tolerances as for the exponential map: FP64 relative <= 1e-12 at every size (1e-10 on iterates), FP32 mixed
||psi_gpu(T) - psi_ref(T)|| <= 1e-4 and gradient relative L2 <= 1e-3."""
import os
import sys

import numpy as np
import pytest

import problems
from oracle import finite as O

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


CASES = [
    ("spin2_K40_N3", lambda: problems.spin2(K=40, N=3)),
    ("spin2_K37_N5_ragged", lambda: problems.spin2(K=37, N=5)),
    ("spin2_K16_N16", lambda: problems.spin2(K=16, N=16)),
    ("rotor_B2_K100_N7", lambda: problems.rotor(batch=2, K=100, N=7, T=0.05)),
    ("rotor_j10_B3_K60_N6", lambda: problems.rotor(batch=3, jmax=10, K=60, N=6, T=0.05)),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_cn_parity(name, mk, prec):
    from paper_1603_01237_amd import _lib
    _say("case cn", name, prec)
    p = mk()
    with _lib.from_problem(p, precision=prec, step_map="cn") as h:
        psiT = h.forward()
        J, F = h.fidelity()
        g = h.gradient()
    for b in range(p.batch):
        gr, Jr, Fr, psiK = O.gradient_cn(p.H0_of(b), p.Hc, p.psi0, p.target, p.u0[b], p.T, p.alpha)
        if prec == "fp64":
            assert _rel(psiT[b], psiK) <= 1e-12
            assert abs(J[b] - Jr) <= 1e-12 and abs(F[b] - Fr) <= 1e-12
            assert _rel(g[b], gr) <= 1e-12, _rel(g[b], gr)
        else:
            assert np.linalg.norm(psiT[b] - psiK) <= 1e-4
            assert abs(F[b] - Fr) <= 1e-4
            assert _rel(g[b], gr) <= 1e-3, _rel(g[b], gr)


def test_cn_iterates_equal_plain_gradient():
    from paper_1603_01237_amd import _lib
    _say("case cn iterate")
    p = problems.spin2(K=200, N=8)
    ref = O.plain_gradient_method_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 0.5, 20)
    with _lib.from_problem(p, precision="fp64", step_map="cn") as h:
        Jh, done = h.iterate(20, 0.5)
        u = h.get_controls()[0]
    assert done == 20
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-10
    assert _rel(u, ref["u"]) <= 1e-10


def test_cn_out_of_series_range_is_reported():
    from paper_1603_01237_amd import _lib
    _say("case cn range")
    p = problems.spin2(K=10, N=2)
    with _lib.from_problem(p, precision="fp64", step_map="cn", set_u=False) as h:
        h.set_controls(np.full((1, 10, 2), 60.0))    # tau ||H|| / 2 ~ 3: no convergent series
        with pytest.raises(_lib.IsmError) as e:
            h.gradient()
        assert e.value.code == _lib.ISM_E_UNSUPPORTED


def test_cn_unsupported_paths():
    from paper_1603_01237_amd import _lib
    _say("case cn unsupported")
    base = problems.spin2(K=6, N=2)
    gate = problems.FiniteProblem("g", base.H0, base.Hc, np.eye(4, dtype=complex),
                                  np.eye(4, dtype=complex), 1.0, 6, 2, np.zeros((1, 6, 2)),
                                  np.zeros(6), 0.5, 1, kind="gate")
    with pytest.raises(_lib.IsmError) as e:
        _lib.from_problem(gate, step_map="cn")
    assert e.value.code == _lib.ISM_E_UNSUPPORTED
    chain = problems.spin_chain_state(3, n=4, T=0.2, K=8, N=2)      # 8 control generators
    with pytest.raises(_lib.IsmError) as e:
        _lib.from_problem(chain, step_map="cn")
    assert e.value.code == _lib.ISM_E_UNSUPPORTED


def test_cn_rotor_full_size():
    """The benchmark's rotor batch (256 rotors, K=20000, N=128) with the Crank-Nicolson map,
    FP32 mixed and FP64: psi(T), lambda(0), J and F of every instance against the oracle's
    values (tests/golden/rotor_b256_k20000.npz, from make_rotor_reference.py), the gradient of
    instances 0 and 255 against the oracle computed here.  FP64 bar 1e-12 (the oracle's own
    Crank-Nicolson rounding at this length is pinned within 5e-13 in test_oracle_long.py)."""
    from paper_1603_01237_amd import _lib
    _say("case cn rotor full size")
    p = problems.rotor()
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "rotor_b256_k20000.npz"))
    res = {}
    for prec in ("fp32", "fp64"):
        with _lib.from_problem(p, precision=prec, step_map="cn") as h:
            g = h.gradient()
            psiT = h.forward()
            lam0 = h.adjoint()
            J, F = h.fidelity()
            res[prec] = (g, psiT, lam0, J, F)
    g64, psi64, lam64, J64, F64 = res["fp64"]
    e_psi = np.linalg.norm(psi64 - ref["cn_psiT"], axis=1)
    e_lam = np.linalg.norm(lam64 - ref["cn_lam0"], axis=1)
    e32 = np.linalg.norm(res["fp32"][1] - ref["cn_psiT"], axis=1)
    _say("fp64 psi(T) max", e_psi.max(), "lambda(0) max", e_lam.max(), "J max",
         np.abs(J64 - ref["cn_J"]).max(), "| fp32 psi(T) max", e32.max())
    assert e_psi.max() <= 1e-12 and e_lam.max() <= 1e-12
    assert np.abs(J64 - ref["cn_J"]).max() <= 1e-12 and np.abs(F64 - ref["cn_F"]).max() <= 1e-12
    assert e32.max() <= 1e-4 and np.abs(res["fp32"][4] - ref["cn_F"]).max() <= 1e-4
    for b in (0, 255):
        gr, Jr, Fr, psiK = O.gradient_cn(p.H0[b], p.Hc, p.psi0, p.target, p.u0[b], p.T, p.alpha)
        _say("instance", b, "fp64 g", _rel(g64[b], gr), "fp32 g", _rel(res["fp32"][0][b], gr))
        assert _rel(g64[b], gr) <= 1e-12
        assert _rel(res["fp32"][0][b], gr) <= 1e-3
