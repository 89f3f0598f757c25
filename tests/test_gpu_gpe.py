"""GPU parity of the Gross-Pitaevskii path (Strang splitting with the LDS-resident FFT,
exact nonlinear adjoint, BEC-variant ISM) against the FP64 oracle.

Norms use the grid measure: ||f|| = sqrt(dx sum |f|^2).  FP64: relative <= 1e-12 (K <= 2500),
growing as 2e-14 sqrt(K) beyond; FP32 mixed: ||psi_gpu(T) - psi_ref(T)|| <= 1e-4 and gradient
relative L2 <= 1e-3.
"""
import math
import sys

import numpy as np
import pytest

import problems
from oracle import gpe as G

pytestmark = pytest.mark.gpu


def _P():
    from paper_1603_01237_amd import _lib
    return _lib


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _small(n=1024, L=40.0, K=41, N=4, g=10.0, T=0.4, seed=8, batch=1):
    x, _, dx = G.grid(n, L)
    psi0 = np.exp(-0.5 * (x + 0.3) ** 2).astype(complex)
    psi0 /= math.sqrt(dx * np.sum(abs(psi0) ** 2))
    tgt = np.exp(-0.5 * (x - 1.0) ** 2 + 0.3j * x)
    tgt /= math.sqrt(dx * np.sum(abs(tgt) ** 2))
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-1, 1, size=(batch, K, 1))
    return problems.GpeProblem("gpe_small", n, L, g, 0.5 * x ** 2, -x.copy(), 0.5, psi0, tgt, T, K,
                               N, u0, 0.1, 3)


def _norm(f, dx):
    return math.sqrt(dx * np.sum(np.abs(f) ** 2))


def _oracle(p, b=0):
    return G.adjoint_gradient(p.psi0, p.target, p.u0[b, :, 0], p.V0, p.V1, p.V2, p.g, p.L, p.T)


CASES = [
    ("n1024_K41_N4", lambda: _small()),
    ("n1024_K12_N12", lambda: _small(K=12, N=12)),
    ("n4096_K30_N1", lambda: _small(n=4096, K=30, N=1)),
    ("n1024_g0_K25_N5", lambda: _small(K=25, N=5, g=0.0)),
    ("n1024_batch2", lambda: _small(K=20, N=3, batch=2)),
    ("n1024_K1_N1_single_step", lambda: _small(K=1, N=1, T=0.01)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gpe_parity(name, mk, prec):
    _say("case", name, prec)
    P = _P()
    p = mk()
    dx = p.L / p.n
    with P.from_problem(p, precision=prec) as h:
        psiT = h.forward()
        nu0 = h.adjoint()
        J, F = h.fidelity()
        g = h.gradient()[:, :, 0]
    for b in range(p.batch):
        gr, Jr, Fr, psiK = _oracle(p, b)
        _, rec = G.strang_forward(p.psi0, p.u0[b, :, 0], p.V0, p.V1, p.V2, p.g, p.L, p.T / p.K)
        # adjoint at t=0 from the oracle's BEC-variant boundaries
        *_, nu_b = G.ism_bec_gradient(p.psi0, p.target, p.u0[b, :, 0], p.V0, p.V1, p.V2, p.g, p.L,
                                      p.T, p.N)
        eg = np.linalg.norm(g[b] - gr) / np.linalg.norm(gr)
        if prec == "fp64":
            assert _norm(psiT[b] - psiK, dx) <= 1e-12
            assert _norm(nu0[b] - nu_b[0], dx) <= 1e-12
            assert abs(J[b] - Jr) <= 1e-12 and abs(F[b] - Fr) <= 1e-12
            assert eg <= 1e-12, eg
        else:
            assert _norm(psiT[b] - psiK, dx) <= 1e-4
            assert abs(F[b] - Fr) <= 1e-4
            assert eg <= 1e-3, eg


def test_gpe_iterate_equals_plain():
    _say("case gpe iterate")
    P = _P()
    p = _small(K=30, N=5)
    ref = G.plain_gradient_method(p.psi0, p.target, p.u0[0, :, 0], p.V0, p.V1, p.V2, p.g, p.L,
                                  p.T, 0.1, 4)
    with P.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate(4, 0.1)
        u = h.get_controls()[0, :, 0]
    assert done == 4
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-12
    assert np.max(np.abs(u - ref["u"])) <= 1e-12


def test_gpe_full_size_sampled():
    """The condensate workload at its full size: n=4096 on [-20,20), g=10, K=10000, N=64,
    ground states at x0=0 and x0=5; psi(T), J, F and the gradient against the oracle."""
    _say("case gpe full size")
    P = _P()
    p = problems.gpe()
    dx = p.dx
    res = {}
    for prec in ("fp32", "fp64"):
        with P.from_problem(p, precision=prec) as h:
            psiT = h.forward()[0]
            J, F = h.fidelity()
            g = h.gradient()[0, :, 0]
        res[prec] = (psiT, J[0], F[0], g)
        _say(prec, "gpu done")
    gr, Jr, Fr, psiK = _oracle(p)
    # FP64 bar derived from the arithmetic: every transform of a step carries a fixed error
    # of at most log2(n) unit roundoffs from its rounded twiddles, the same at every step, so
    # the two implementations (this FFT and the oracle's) drift apart coherently over the
    # 2K transforms of a sweep (and 2K more in the adjoint):
    u64 = 2.0 ** -53
    tol_state = 4 * u64 * p.K * math.log2(p.n)
    # gradient g_j = dx sum dV/du Im(conj(nu') b): by Cauchy-Schwarz its error is at most
    # 2 max|dV/du| times the state error, relative to the rms gradient
    dV = np.abs(p.V1[:, None] + 2 * p.u0[0, None, :, 0] * p.V2)
    tol_g = 2 * float(dV.max()) * tol_state / float(np.sqrt(np.mean(gr ** 2)))
    for prec, (psiT, J, F, g) in res.items():
        e_psi = _norm(psiT - psiK, dx)
        e_g = np.linalg.norm(g - gr) / np.linalg.norm(gr)
        _say(prec, "psi err", e_psi, "J err", abs(J - Jr), "g rel err", e_g,
             "fp64 bars", tol_state, tol_g)
        if prec == "fp64":
            assert e_psi <= tol_state and abs(J - Jr) <= tol_state and e_g <= tol_g
        else:
            assert e_psi <= 1e-4 and abs(F - Fr) <= 1e-4 and e_g <= 1e-3
