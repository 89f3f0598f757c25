"""GPU parity of density-matrix problems (ISM_DENSITY: rho <- U rho U^+, the five-spin
experiment of Sec. 4.A in the Liouville-von Neumann form) on the dense MFMA path against
the FP64 oracle.

Cases use the paper's control time T = 10/Jp, where J and the gradient are of order one (a
much shorter T leaves a gradient 1e-4 of its terms, and cancellation then sets the rounding),
with step counts that keep 2 tau ||H|| inside the range of the dense path's gradient series.
Tolerances: FP64 relative L2 <= 1e-12 at every size; FP32 mixed
||rho_gpu(T) - rho_ref(T)||_F / ||rho_0||_F <= 1e-4 and gradient relative L2 <= 1e-3.
"""
import sys

import numpy as np
import pytest

import problems
from oracle import density as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _random_density(d, K, N, seed, alpha=0.0, T=0.8):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    H0 = 0.5 * (A + A.conj().T)
    Hc = []
    for _ in range(2):
        B = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        Hc.append(0.5 * (B + B.conj().T))
    R0 = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)); R0 = 0.5 * (R0 + R0.conj().T)
    Rf = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)); Rf = 0.5 * (Rf + Rf.conj().T)
    u0 = rng.uniform(-1, 1, size=(1, K, 2))
    return problems.FiniteProblem("density_random", H0, np.stack(Hc), R0, Rf, T, K, N, u0,
                                  np.full(K, alpha), 0.1, 3, kind="density")


def _chain_density(n, K, N, seed=5):
    """Ising chain of the gate benchmark with I_x^(1) -> I_y^(1) + I_x^(2) as density
    matrices (reachable within a few steps, so J and the gradient are far from zero)."""
    g = problems.spin_chain_gate(seed=seed, n=n, K=K, N=N, T=K * 0.01)
    Ix, Iy, _ = problems.spin_operators(n)
    return problems.FiniteProblem("density_chain", g.H0, g.Hc, Ix[0], Iy[0] + Ix[1], g.T, K, N, g.u0,
                                  np.zeros(K), 0.1, 3, kind="density")


CASES = [
    ("spin5_K512_N4", lambda: problems.spin5_density(K=512, N=4, u_amp=300.0)),
    ("spin5_K437_N5_ragged", lambda: problems.spin5_density(K=437, N=5, u_amp=300.0)),
    ("spin5_K512_N16", lambda: problems.spin5_density(K=512, N=16, u_amp=300.0)),
    ("random_d4_K30_N3_alpha", lambda: _random_density(4, 30, 3, 7, alpha=0.2)),
    ("random_d4_K1_N1_single_step", lambda: _random_density(4, 1, 1, 9, T=0.05)),
    ("chain7_d128_K12_N3", lambda: _chain_density(7, 12, 3)),
    ("random_d4_K300_N1_scan", lambda: _random_density(4, 300, 1, 11)),
    ("chain6_d64_K200_N2_scan64", lambda: _chain_density(6, 200, 2)),
    # dimensions that leave padding rows inside the gradient's column groups (d <= 32 packs
    # 64 / lpc columns per wavefront, lpc the least power of two >= d)
    ("random_d5_K40_N3_odd", lambda: _random_density(5, 40, 3, 13, alpha=0.1)),
    ("random_d12_K64_N2_odd", lambda: _random_density(12, 64, 2, 17)),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_density_parity(name, mk, prec):
    from paper_1603_01237_amd import _lib
    _say("case density", name, prec)
    p = mk()
    with _lib.from_problem(p, precision=prec) as h:
        rhoT = h.forward()[0]
        J, F = h.fidelity()
        g = h.gradient()[0]
    gr, Jr, Fr, rK = D.gradient(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha)
    n0 = np.linalg.norm(p.psi0)
    if prec == "fp64":
        assert np.linalg.norm(rhoT - rK) / n0 <= 1e-12
        assert abs(J[0] - Jr) <= 1e-12 * max(1.0, abs(Jr)) and abs(F[0] - Fr) <= 1e-12
        assert _rel(g, gr) <= 1e-12, _rel(g, gr)
    else:
        assert np.linalg.norm(rhoT - rK) / n0 <= 1e-4
        assert abs(F[0] - Fr) <= 1e-4
        assert _rel(g, gr) <= 1e-3, _rel(g, gr)


def test_density_iterates_equal_plain():
    from paper_1603_01237_amd import _lib
    _say("case density iterate")
    p = problems.spin5_density(K=1024, N=8, u_amp=300.0)
    ref = D.plain_gradient_method(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 30.0, 4)
    with _lib.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate(4, 30.0)
        u = h.get_controls()[0]
    assert done == 4
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-10
    assert _rel(u, ref["u"]) <= 1e-10


def test_dense_path_reports_steps_beyond_its_gradient_series():
    """2 tau ||H|| ~ 4: the exact gradient's series would need more terms than the kernel
    holds, so the call reports ISM_E_UNSUPPORTED instead of a truncated gradient."""
    from paper_1603_01237_amd import _lib
    _say("case density series range")
    p = problems.spin5_density(K=64, N=4, u_amp=300.0)
    with _lib.from_problem(p, precision="fp64") as h:
        with pytest.raises(_lib.IsmError) as e:
            h.gradient()
        assert e.value.code == _lib.ISM_E_UNSUPPORTED


def test_density_rejects_non_hermitian():
    from paper_1603_01237_amd import _lib
    _say("case density args")
    p = problems.spin5_density(K=8, N=2)
    bad = np.array(p.psi0, copy=True)
    bad[0, 1] += 0.3
    q = problems.FiniteProblem("bad", p.H0, p.Hc, bad, p.target, p.T, 8, 2, p.u0, p.alpha, 1.0, 1,
                               kind="density")
    with pytest.raises(_lib.IsmError) as e:
        _lib.from_problem(q)
    assert e.value.code == _lib.ISM_E_ARG


def test_density_five_spin_full_size():
    """The five-spin density-matrix run at the paper's size (K = 2^15 steps, N = 8): one
    gradient in FP32 mixed and FP64 against the oracle, and the N = 8 gradient equal to the
    N = 1 one (Theorem 2) on the GPU.  FP64 bar 1e-12."""
    from paper_1603_01237_amd import _lib
    _say("case density full size")
    p = problems.spin5_density()
    tol64 = 1e-12
    res = {}
    for prec in ("fp32", "fp64"):
        with _lib.from_problem(p, precision=prec) as h:
            res[prec] = (h.gradient()[0], h.forward()[0])
    with _lib.from_problem(p, precision="fp64", N=1) as h:
        g1 = h.gradient()[0]
    gr, Jr, Fr, rK = D.gradient(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha)
    n0 = np.linalg.norm(p.psi0)
    _say("fp64 g", _rel(res["fp64"][0], gr), "rho", np.linalg.norm(res["fp64"][1] - rK) / n0,
         "fp32 g", _rel(res["fp32"][0], gr), "rho", np.linalg.norm(res["fp32"][1] - rK) / n0,
         "N=1 vs N=8", _rel(g1, res["fp64"][0]))
    assert _rel(res["fp64"][0], gr) <= tol64
    assert np.linalg.norm(res["fp64"][1] - rK) / n0 <= tol64
    assert _rel(g1, res["fp64"][0]) <= tol64
    assert _rel(res["fp32"][0], gr) <= 1e-3
    assert np.linalg.norm(res["fp32"][1] - rK) / n0 <= 1e-4
