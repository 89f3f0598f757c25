"""GPU parity of ism_iterate_inner (several gradient steps per slice problem, Algorithm 1
step (c), and the Err rule of step (e)) against the FP64 oracle, on the sparse state path
(generic and tridiagonal kernels, exponential and Crank-Nicolson maps), the dense gate path
and the Gross-Pitaevskii path.

Bars: FP64 relative <= 1e-10 on iterates (controls, J and Err after several iterations);
FP32 mixed: controls and Err relative L2 <= 1e-3 (the gradient bar), J within 1e-4.
"""
import dataclasses
import sys

import numpy as np
import pytest

import problems
from oracle import finite as O
from oracle import gpe as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _spins(K, N, alpha=0.1):
    p = problems.spin2(K=K, N=N)
    return dataclasses.replace(p, alpha=np.full(K, alpha))


def _gate(n, K, N, seed=5):
    return problems.spin_chain_gate(seed=seed, n=n, K=K, N=N, T=K * 0.01)


def _gpe(n=1024, L=40.0, K=30, N=4, g=10.0, T=0.3, seed=8, batch=1):
    x, _, dx = G.grid(n, L)
    psi0 = np.exp(-0.5 * (x + 0.3) ** 2).astype(complex)
    psi0 /= np.sqrt(dx * np.sum(abs(psi0) ** 2))
    tgt = np.exp(-0.5 * (x - 1.0) ** 2 + 0.3j * x)
    tgt /= np.sqrt(dx * np.sum(abs(tgt) ** 2))
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-1, 1, size=(batch, K, 1))
    return problems.GpeProblem("gpe_small", n, L, g, 0.5 * x ** 2, -x.copy(), 0.5, psi0, tgt, T, K,
                               N, u0, 0.1, 3)


def _finite_ref(p, b, rho, iters, ell, eta=0.0, step="exp"):
    return O.ism_iterate_inner(p.H0_of(b), p.Hc, p.psi0, p.target, p.u0[b], p.T, p.alpha, rho,
                               iters, p.N, ell, eta=eta, step=step)


def _gpe_ref(p, b, rho, iters, ell, eta=0.0):
    return G.ism_bec_iterate_inner(p.psi0, p.target, p.u0[b, :, 0], p.V0, p.V1, p.V2, p.g, p.L,
                                   p.T, rho, iters, p.N, ell, eta=eta)


def _check(prec, Jh, Eh, u, ref, b):
    n = ref["iters"]
    if prec == "fp64":
        assert np.max(np.abs(Jh[:n, b] - ref["J"])) <= 1e-10
        assert _rel(Eh[:n, b], ref["Err"]) <= 1e-10, _rel(Eh[:n, b], ref["Err"])
        assert _rel(u, ref["u"]) <= 1e-10, _rel(u, ref["u"])
    else:
        assert np.max(np.abs(Jh[:n, b] - ref["J"])) <= 1e-4
        assert _rel(Eh[:n, b], ref["Err"]) <= 1e-3, _rel(Eh[:n, b], ref["Err"])
        assert _rel(u, ref["u"]) <= 1e-3, _rel(u, ref["u"])


FINITE = [
    ("spins_K40_N4_ell3", lambda: _spins(40, 4), 3, 0.5, "exp"),
    ("spins_K37_N5_ell2_ragged", lambda: _spins(37, 5), 2, 0.5, "exp"),
    ("spins_cn_K40_N4_ell3", lambda: _spins(40, 4), 3, 0.5, "cn"),
    ("rotor_B3_K120_N6_ell2", lambda: problems.rotor(batch=3, K=120, N=6, T=0.3), 2, 2.0, "exp"),
    ("rotor_cn_B2_K100_N5_ell3", lambda: problems.rotor(batch=2, K=100, N=5, T=0.05), 3, 2.0, "cn"),
    ("gate_chain3_K24_N4_ell2", lambda: _gate(3, 24, 4), 2, 0.5, "exp"),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk,ell,rho,step", FINITE, ids=[c[0] for c in FINITE])
def test_inner_steps_parity(name, mk, ell, rho, step, prec):
    from paper_1603_01237_amd import _lib
    _say("case inner", name, prec)
    p = mk()
    iters = 4
    with _lib.from_problem(p, precision=prec, step_map=step) as h:
        Jh, Eh, done = h.iterate_inner(iters, ell, rho)
        u = h.get_controls()
    assert done == iters and Eh.shape == (iters, p.batch)
    for b in range(p.batch):
        ref = _finite_ref(p, b, rho, iters, ell, step=step)
        _check(prec, Jh, Eh, u[b], ref, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_inner_steps_parity_gpe(prec):
    from paper_1603_01237_amd import _lib
    _say("case inner gpe", prec)
    p = _gpe(K=30, N=4, batch=2)
    with _lib.from_problem(p, precision=prec) as h:
        Jh, Eh, done = h.iterate_inner(3, 3, 0.1)
        u = h.get_controls()
    assert done == 3
    for b in range(p.batch):
        ref = _gpe_ref(p, b, 0.1, 3, 3)
        _check(prec, Jh, Eh, u[b, :, 0], ref, b)


def test_one_inner_step_is_ism_iterate():
    """n_inner = 1 without the Err rule runs exactly the kernels of ism_iterate."""
    from paper_1603_01237_amd import _lib
    _say("case inner ell1")
    p = problems.rotor(batch=2, K=80, N=4, T=0.3)
    with _lib.from_problem(p, precision="fp32") as h:
        Ja, _ = h.iterate(3, 2.0)
        ua = h.get_controls()
    with _lib.from_problem(p, precision="fp32") as h:
        Jb, Eb, done = h.iterate_inner(3, 1, 2.0, record=True)
        ub = h.get_controls()
    assert done == 3
    assert np.array_equal(ua, ub) and np.array_equal(Ja, Jb)


def test_err_stop_per_instance():
    """Instances stop after their own first iteration with Err <= eta; the loop ends when
    the last one stops; frozen controls stay put."""
    from paper_1603_01237_amd import _lib
    _say("case inner err stop")
    p = problems.rotor(batch=3, K=120, N=6, T=3.0)
    ell, rho, iters = 2, 2.0, 8
    refs = [_finite_ref(p, b, rho, iters, ell) for b in range(p.batch)]
    # eta: a midpoint between recorded Err values at which some instance stops early, as far
    # from every recorded value as possible
    errs = np.sort(np.concatenate([r["Err"] for r in refs]))
    best, eta = -1.0, None
    for a, c in zip(errs[:-1], errs[1:]):
        e = 0.5 * (a + c)
        early = sum(int(np.any(r["Err"][:iters - 1] <= e)) for r in refs)
        margin = (c - a) / (2 * e)
        if 0 < early and margin > best:
            best, eta = margin, e
    assert eta is not None and best > 1e-4
    stopped = [_finite_ref(p, b, rho, iters, ell, eta=eta) for b in range(p.batch)]
    assert min(r["iters"] for r in stopped) < iters
    with _lib.from_problem(p, precision="fp64") as h:
        Jh, Eh, done = h.iterate_inner(iters, ell, rho, err_stop=eta)
        u = h.get_controls()
    assert done == max(r["iters"] for r in stopped)
    for b in range(p.batch):
        r = stopped[b]
        assert _rel(u[b], r["u"]) <= 1e-10
        assert _rel(Eh[:r["iters"], b], r["Err"]) <= 1e-10


def test_inner_argument_checks():
    from paper_1603_01237_amd import _lib
    _say("case inner args")
    p = _spins(8, 2)
    with _lib.from_problem(p) as h:
        for bad in (dict(n_inner=0), dict(err_stop=float("nan"))):
            kw = dict(n_iter=1, n_inner=2, rho=0.1, err_stop=0.0)
            kw.update(bad)
            with pytest.raises(_lib.IsmError) as e:
                h.iterate_inner(**kw)
            assert e.value.code == _lib.ISM_E_ARG


def test_inner_rotor_full_size_sampled():
    """The benchmark's rotor batch (256 rotors, K=20000, N=128), one iteration with two
    gradient steps per slice problem and Err, FP32 mixed and FP64; two instances checked
    against the oracle.  FP64 bar 1e-12, as for the single-step path at this K."""
    from paper_1603_01237_amd import _lib
    _say("case inner rotor full size")
    p = problems.rotor()
    tol64 = 1e-12
    res = {}
    for prec in ("fp32", "fp64"):
        with _lib.from_problem(p, precision=prec) as h:
            _, Eh, done = h.iterate_inner(1, 2, p.rho)
            assert done == 1
            res[prec] = (h.get_controls(), Eh[0])
    for b in (0, 255):
        r = _finite_ref(p, b, p.rho, 1, 2)
        du = {k: _rel(v[0][b] - p.u0[b], r["u"] - p.u0[b]) for k, v in res.items()}
        de = {k: abs(v[1][b] - r["Err"][0]) / r["Err"][0] for k, v in res.items()}
        _say("instance", b, "update rel", du, "Err rel", de)
        assert du["fp64"] <= tol64 and de["fp64"] <= tol64
        assert du["fp32"] <= 1e-3 and de["fp32"] <= 1e-3
