"""GPU parity of the Crank-Nicolson step map against the FP64 oracle: the sparse state path,
and the dense path (gates and density matrices: Cayley steps formed as D_j = U_j - I by a
Neumann series, gradient Im<A y|H_c|A x> with A = (I + L_j)^{-1}).

Tolerances as for the exponential map: FP64 relative <= 1e-12 at every size (1e-10 on iterates), FP32 mixed
||psi_gpu(T) - psi_ref(T)|| <= 1e-4 and gradient relative L2 <= 1e-3."""
import os
import sys

import numpy as np
import pytest

import problems
from oracle import density as D
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


def _spin2_gate(K, N, seed=3, T=1.0):
    p = problems.spin2(K=K, N=N, T=T)
    rng = np.random.default_rng(seed)
    W = problems.haar_unitary(4, rng)
    u = rng.uniform(-1, 1, size=(1, K, 2))
    return problems.FiniteProblem("spin2_gate", p.H0, p.Hc, np.eye(4, dtype=complex), W, p.T, K,
                                  N, u, np.full(K, 0.1), 0.5, 5, kind="gate")


def _random_density(d, K, N, seed, alpha=0.0, T=0.8):
    rng = np.random.default_rng(seed)

    def herm():
        A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        return 0.5 * (A + A.conj().T)
    H0 = herm()
    Hc = np.stack([herm(), herm()])
    R0, Rf = herm(), herm()
    u0 = rng.uniform(-1, 1, size=(1, K, 2))
    return problems.FiniteProblem("density_random", H0, Hc, R0, Rf, T, K, N, u0,
                                  np.full(K, alpha), 0.1, 3, kind="density")


DENSE_CASES = [
    ("spin2_gate_K24_N3", lambda: _spin2_gate(24, 3)),
    ("spin2_gate_K17_N5_ragged", lambda: _spin2_gate(17, 5)),
    ("spin2_gate_K1_N1_single_step", lambda: _spin2_gate(1, 1, T=0.1)),
    ("chain4_gate_K30_N4", lambda: problems.spin_chain_gate(seed=5, n=4, K=30, N=4, T=0.3)),
    ("chain6_gate_K300_N3_scan64", lambda: problems.spin_chain_gate(seed=5, n=6, K=300, N=3, T=3.0)),
    ("chain4_gate_K57_N19_bscan", lambda: problems.spin_chain_gate(seed=5, n=4, K=57, N=19, T=0.57)),
    ("chain7_gate_K40_N4_d128", lambda: problems.spin_chain_gate(seed=6, n=7, K=40, N=4, T=0.4)),
    ("spin5_density_K512_N4", lambda: problems.spin5_density(K=512, N=4, u_amp=300.0)),
    ("spin5_density_K437_N5_ragged", lambda: problems.spin5_density(K=437, N=5, u_amp=300.0)),
    ("random_density_d4_K30_N3_alpha", lambda: _random_density(4, 30, 3, 7, alpha=0.2)),
    ("random_density_d4_K1_N1_single_step", lambda: _random_density(4, 1, 1, 9, T=0.02)),
]


def _dense_oracle(p):
    if p.kind == "density":
        return D.gradient_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha)
    return O.gradient_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha)


def _end_error(p, XT, XK):
    """FP32 bar quantity: ||U(T) - U_ref||_F / sqrt(d) (gates), ||rho(T) - rho_ref||_F /
    ||rho_0||_F (density matrices)."""
    if p.kind == "density":
        return np.linalg.norm(XT - XK) / np.linalg.norm(p.psi0)
    return np.linalg.norm(XT - XK) / np.sqrt(p.d)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk", DENSE_CASES, ids=[c[0] for c in DENSE_CASES])
def test_cn_dense_parity(name, mk, prec):
    from paper_1603_01237_amd import _lib
    _say("case cn dense", name, prec)
    p = mk()
    with _lib.from_problem(p, precision=prec, step_map="cn") as h:
        XT = h.forward()[0]
        J, F = h.fidelity()
        g = h.gradient()[0]
    gr, Jr, Fr, XK = _dense_oracle(p)
    if prec == "fp64":
        assert _rel(XT, XK) <= 1e-12, _rel(XT, XK)
        assert abs(J[0] - Jr) <= 1e-12 * max(1.0, abs(Jr)) and abs(F[0] - Fr) <= 1e-12
        assert _rel(g, gr) <= 1e-12, _rel(g, gr)
    else:
        assert _end_error(p, XT, XK) <= 1e-4
        assert abs(F[0] - Fr) <= 1e-4
        assert _rel(g, gr) <= 1e-3, _rel(g, gr)


@pytest.mark.parametrize("kind", ["gate", "density"])
def test_cn_dense_iterates_equal_plain(kind):
    """ism_iterate on the dense path with the Crank-Nicolson map against the oracle's plain
    gradient method (equal to the ISM iteration by Theorem 2) over 12 iterations."""
    from paper_1603_01237_amd import _lib
    _say("case cn dense iterate", kind)
    if kind == "gate":
        p = problems.spin_chain_gate(seed=5, n=4, K=60, N=5, T=0.6)
        ref = O.plain_gradient_method_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha,
                                         0.5, 12)
    else:
        p = problems.spin5_density(K=1024, N=8, u_amp=300.0)    # tau ||H|| / 2 ~ 0.07
        ref = D.plain_gradient_method_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha,
                                         30.0, 12)
    rho = 0.5 if kind == "gate" else 30.0
    with _lib.from_problem(p, precision="fp64", step_map="cn") as h:
        Jh, done = h.iterate(12, rho)
        u = h.get_controls()[0]
    assert done == 12
    _say("J", Jh[:, 0], ref["J"])
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-10 * max(1.0, np.max(np.abs(ref["J"])))
    assert _rel(u, ref["u"]) <= 1e-10


def test_cn_dense_out_of_series_range_is_reported():
    from paper_1603_01237_amd import _lib
    _say("case cn dense range")
    p = problems.spin5_density(K=64, N=4, u_amp=300.0)     # tau ||H|| / 2 ~ 1
    with _lib.from_problem(p, precision="fp64", step_map="cn") as h:
        with pytest.raises(_lib.IsmError) as e:
            h.gradient()
        assert e.value.code == _lib.ISM_E_UNSUPPORTED


def test_cn_density_five_spin_full_size():
    """The five-spin density-matrix run at the paper's size (K = 2^15, N = 8) with the
    Crank-Nicolson map: rho(T) and the gradient in FP64 (bar 1e-12) and FP32 mixed against the
    oracle, and the N = 8 gradient equal to the N = 1 one (Theorem 2) on the GPU."""
    from paper_1603_01237_amd import _lib
    _say("case cn density full size")
    p = problems.spin5_density()
    res = {}
    for prec in ("fp32", "fp64"):
        with _lib.from_problem(p, precision=prec, step_map="cn") as h:
            res[prec] = (h.gradient()[0], h.forward()[0])
    with _lib.from_problem(p, precision="fp64", step_map="cn", N=1) as h:
        g1 = h.gradient()[0]
    gr, Jr, Fr, rK = D.gradient_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha)
    n0 = np.linalg.norm(p.psi0)
    _say("fp64 g", _rel(res["fp64"][0], gr), "rho", np.linalg.norm(res["fp64"][1] - rK) / n0,
         "fp32 g", _rel(res["fp32"][0], gr), "rho", np.linalg.norm(res["fp32"][1] - rK) / n0,
         "N=1 vs N=8", _rel(g1, res["fp64"][0]))
    assert _rel(res["fp64"][0], gr) <= 1e-12
    assert np.linalg.norm(res["fp64"][1] - rK) / n0 <= 1e-12
    assert _rel(g1, res["fp64"][0]) <= 1e-12
    assert _rel(res["fp32"][0], gr) <= 1e-3
    assert np.linalg.norm(res["fp32"][1] - rK) / n0 <= 1e-4
