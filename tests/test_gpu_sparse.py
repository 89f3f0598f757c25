"""GPU parity of the sparse state path (path (b)) against the FP64 oracle, through the C ABI.

Tolerances (per instance, norms over the whole output):
  FP64 path      : relative L2 <= 1e-12 on psi(T), lambda(0), g, J and F at every size, the
                   benchmark's K = 20000 included; 1e-10 on the controls and J after 50
                   iterations.  The oracle's own share of the budget at K = 20000 is pinned on
                   the CPU (tests/test_oracle_long.py: within 5e-14 of an extended-precision
                   evaluation; measured 2.7e-14 over the 256 rotors).
  FP32 mixed path: ||psi_gpu(T) - psi_ref(T)||_2 <= 1e-4, ||g_gpu - g_ref|| / ||g_ref|| <= 1e-3
"""
import os
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


TOL64 = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rotor_b256_k20000.npz")


def _oracle_grad(p, b, u):
    return O.gradient(p.H0_of(b), p.Hc, p.psi0, p.target, u, p.T, p.alpha)


CASES = [
    ("spin2_K40_N3", lambda: problems.spin2(K=40, N=3)),
    ("spin2_K37_N5_ragged", lambda: problems.spin2(K=37, N=5)),
    ("spin2_K16_N16_NeqK", lambda: problems.spin2(K=16, N=16)),
    ("spin2_K25_N1", lambda: problems.spin2(K=25, N=1)),
    ("spin2_K1_N1_single_step", lambda: problems.spin2(K=1, N=1)),
    ("rotor_B2_K1_N1_single_step", lambda: problems.rotor(batch=2, K=1, N=1, T=0.01)),
    ("rotor_B3_K90_N7", lambda: problems.rotor(batch=3, K=90, N=7, T=0.5)),
    ("rotor_j40_B2_K40_N6", lambda: problems.rotor(batch=2, jmax=40, K=40, N=6, T=0.1)),
    # three-rows-per-lane layout: padded last lane (d=11), 32 items per wavefront (d=5),
    # one step per slice (N = K), slices straddling wavefronts (d=21, N=13)
    ("rotor_j10_B2_K50_N5_pad", lambda: problems.rotor(batch=2, jmax=10, K=50, N=5, T=0.2)),
    ("rotor_j4_B3_K24_N24_NeqK", lambda: problems.rotor(batch=3, jmax=4, K=24, N=24, T=0.3)),
    ("rotor_B2_K65_N13_straddle", lambda: problems.rotor(batch=2, K=65, N=13, T=0.3)),
    ("chain4_state_K21_N4", lambda: _chain_random(11, n=4, T=0.4, K=21, N=4)),
    ("chain7_state_K12_N3_block", lambda: _chain_random(12, n=7, T=0.3, K=12, N=3)),
    ("chain8_state_K10_N4_block", lambda: _chain_random(13, n=8, T=0.3, K=10, N=4)),
]


def _chain_random(seed, n, T, K, N):
    """Spin-chain Hamiltonian with seeded random initial and target states: the transfer
    |0..0> -> |1..1> at small controls has gradients of size ~(tau u)^n, far below the
    rounding scale of the terms that form them, which makes relative errors meaningless."""
    p = problems.spin_chain_state(seed, n=n, T=T, K=K, N=N)
    rng = np.random.default_rng(seed + 100)
    d = 2 ** n
    for attr in ("psi0", "target"):
        v = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        setattr(p, attr, v / np.linalg.norm(v))
    return p


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_fp64_forward_gradient_parity(name, mk):
    _say("case", name, "fp64")
    P = _P()
    p = mk()
    with P.from_problem(p, precision="fp64") as h:
        psiT = h.forward()
        chi0 = h.adjoint()
        J, F = h.fidelity()
        g = h.gradient()
    for b in range(p.batch):
        gr, Jr, Fr, psiK = _oracle_grad(p, b, p.u0[b])
        lam0 = O.backward(O.step_unitaries(p.H0_of(b), p.Hc, p.u0[b], p.T / p.K), p.target)[0]
        assert _rel(psiT[b], psiK) <= TOL64
        assert _rel(chi0[b], lam0) <= 1e-12
        assert abs(J[b] - Jr) <= 1e-12 and abs(F[b] - Fr) <= 1e-12
        assert _rel(g[b], gr) <= 1e-12, _rel(g[b], gr)


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_fp32_mixed_parity(name, mk):
    _say("case", name, "fp32")
    P = _P()
    p = mk()
    with P.from_problem(p, precision="fp32") as h:
        psiT = h.forward()
        J, F = h.fidelity()
        g = h.gradient()
    for b in range(p.batch):
        gr, Jr, Fr, psiK = _oracle_grad(p, b, p.u0[b])
        assert np.linalg.norm(psiT[b] - psiK) <= 1e-4
        assert abs(F[b] - Fr) <= 1e-4
        assert _rel(g[b], gr) <= 1e-3, _rel(g[b], gr)


def test_alpha_time_dependent_fp64():
    _say("case alpha")
    P = _P()
    p = problems.spin2(K=30, N=4)
    al = 0.3 + 0.2 * np.cos(np.arange(30))          # alpha_j per step
    with P.Problem.create(p.H0, p.Hc, p.psi0, p.target, p.T, p.K, p.N, alpha=al) as h:
        h.set_controls(p.u0)
        g = h.gradient()
        J, F = h.fidelity()
    gr, Jr, Fr, _ = O.gradient(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, al)
    assert _rel(g[0], gr) <= 1e-12
    assert abs(J[0] - Jr) <= 1e-12


def test_cfg0_iterate_equals_plain_gradient_fp64():
    """Two coupled spins, K=1000, N=8, 50 iterations, step 0.5 (the small configuration):
    the ISM iterates equal the plain gradient method's (Theorem 2)."""
    _say("case cfg0 iterate")
    P = _P()
    p = problems.spin2()
    ref = O.plain_gradient_method(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, p.rho, 50)
    with P.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate(50, p.rho)
        u = h.get_controls()
        J, F = h.fidelity()
    assert done == 50
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-10
    assert _rel(u[0], ref["u"]) <= 1e-10
    gr, Jr, Fr, _ = _oracle_grad(p, 0, ref["u"])
    assert abs(F[0] - Fr) <= 1e-10


def test_cfg0_iterate_fp32_final_fidelity():
    _say("case cfg0 iterate fp32")
    P = _P()
    p = problems.spin2()
    ref = O.plain_gradient_method(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, p.rho, 50)
    Fref = O.gradient(p.H0, p.Hc, p.psi0, p.target, ref["u"], p.T, p.alpha)[2]
    with P.from_problem(p, precision="fp32") as h:
        h.iterate(50, p.rho)
        J, F = h.fidelity()
    assert abs(F[0] - Fref) <= 1e-4


def test_fid_stop_freezes_instances():
    _say("case fid_stop")
    P = _P()
    p = problems.spin2(K=100, N=4)
    with P.from_problem(p) as h:
        Jh, done = h.iterate(200, 0.5, fid_stop=0.9)
        J, F = h.fidelity()
        u1 = h.get_controls()
        Jh2, done2 = h.iterate(5, 0.5, fid_stop=0.9)
        u2 = h.get_controls()
    assert 0 < done < 200
    assert F[0] >= 0.9
    assert done2 == 0 and np.array_equal(u1, u2)


def test_numeric_error_reported_for_nan_controls():
    _say("case nan")
    import torch
    P = _P()
    p = problems.spin2(K=20, N=2)
    u = torch.tensor(p.u0, dtype=torch.float64, device="cuda").contiguous()
    u[0, 3, 1] = float("nan")
    with P.from_problem(p, io_device=True, set_u=False) as h:
        h.set_controls(u)
        with pytest.raises(P.IsmError) as e:
            h.gradient()
        assert e.value.code == P.ISM_E_NUMERIC
        with pytest.raises(P.IsmError) as e:
            h.iterate(2, 0.1)
        assert e.value.code == P.ISM_E_NUMERIC


def test_device_io_matches_host_io():
    _say("case device io")
    import torch
    P = _P()
    p = problems.rotor(batch=2, K=50, N=5, T=0.4)
    with P.from_problem(p) as h:
        g_host = h.gradient()
        psi_host = h.forward()
    with P.from_problem(p, io_device=True, set_u=False) as h:
        h.set_controls(torch.tensor(p.u0, dtype=torch.float64, device="cuda"))
        g_dev = h.gradient()
        psi_dev = h.forward()
        torch.cuda.synchronize()
    assert np.array_equal(g_dev.cpu().numpy(), g_host)
    assert np.array_equal(psi_dev.cpu().numpy(), psi_host)


def test_rotor_full_size():
    """The benchmark's launch configuration (256 rotors, K=20000, N=128), FP32 mixed and
    FP64.  psi(T), lambda(0), J and F of every instance against the oracle's values
    (tests/golden/rotor_b256_k20000.npz, written by make_rotor_reference.py from the oracle);
    the full gradient of instances 0, 127 and 255 against the oracle computed here."""
    _say("case rotor full size")
    P = _P()
    p = problems.rotor()
    ref = np.load(GOLDEN)
    res = {}
    for prec in ("fp32", "fp64"):
        with P.from_problem(p, precision=prec) as h:
            g = h.gradient()
            psiT = h.forward()
            lam0 = h.adjoint()
            J, F = h.fidelity()
        res[prec] = (g, psiT, lam0, J, F)
    g64, psi64, lam64, J64, F64 = res["fp64"]
    g32, psi32, lam32, J32, F32 = res["fp32"]
    e_psi = np.linalg.norm(psi64 - ref["exp_psiT"], axis=1)
    e_lam = np.linalg.norm(lam64 - ref["exp_lam0"], axis=1)
    e32 = np.linalg.norm(psi32 - ref["exp_psiT"], axis=1)
    _say("fp64 psi(T) max", e_psi.max(), "lambda(0) max", e_lam.max(),
         "J max", np.abs(J64 - ref["exp_J"]).max(), "F max", np.abs(F64 - ref["exp_F"]).max(),
         "| fp32 psi(T) max", e32.max(), "F max", np.abs(F32 - ref["exp_F"]).max())
    assert e_psi.max() <= TOL64 and e_lam.max() <= TOL64
    assert np.abs(J64 - ref["exp_J"]).max() <= TOL64 and np.abs(F64 - ref["exp_F"]).max() <= TOL64
    assert e32.max() <= 1e-4 and np.abs(F32 - ref["exp_F"]).max() <= 1e-4
    for b in (0, 127, 255):
        gr, Jr, Fr, psiK = _oracle_grad(p, b, p.u0[b])
        _say("instance", b, "fp64 g", _rel(g64[b], gr), "fp32 g", _rel(g32[b], gr))
        assert _rel(g64[b], gr) <= TOL64
        assert _rel(g32[b], gr) <= 1e-3
    assert np.all(np.isfinite(g64)) and np.all(np.isfinite(g32))


def test_taylor_params_per_instance():
    """Per-instance series parameters: unavailable before a forward pass, one (m, S) per
    instance after it, the largest equal to ism_problem_info's, and the FP32 truncation
    budget (at most 1e-5 summed over the K steps) holding for every instance."""
    import math
    _say("case taylor params")
    P = _P()
    p = problems.rotor(batch=5, K=400, N=4, T=2.0)
    with P.from_problem(p, precision="fp32") as h:
        with pytest.raises(P.IsmError) as e:
            h.taylor_params()
        assert e.value.code == P.ISM_E_STATE
        h.forward(want_state=False)
        m, S = h.taylor_params()
        info = h.info()
    assert len(m) == 5 and max(m) == info["taylor_m"] and max(S) == info["taylor_S"]
    tau = p.T / p.K
    for b in range(5):
        dg = np.real(np.diag(p.H0[b]))
        bound = (np.abs(p.H0[b] - 0.5 * (dg.max() + dg.min()) * np.eye(p.d)).sum(1).max()
                 + np.abs(p.u0[b]).max() * np.abs(p.Hc[0]).sum(1).max())
        ts = tau * bound / S[b]
        # first dropped term of the sub-step series, times e^ts: the truncation per step
        drop = ts ** (m[b] + 1) / math.factorial(m[b] + 1) * math.exp(ts) * S[b]
        assert drop * p.K <= 1e-5 * 1.0001
