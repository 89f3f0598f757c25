"""GPU parity of the one-launch solve of small state problems (d <= 4, at most 4 controls
and 64 slices): every iteration of Algorithm 1 for an instance in one workgroup, in FP64
for handles of either precision.

It replaces the per-pass launch sequence in ism_iterate and in served iterations; both are
FP64 evaluations of the same iterates, so they are compared with each other and with the
oracle's plain gradient method (equal to ISM by Theorem 2): J history and controls within
1e-10 over tens of iterations (the bar of the per-pass path's iterate tests), and J, F and
the gradient at the final controls within 1e-12 of the oracle."""
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


def _qubit_pair_c4(K, N, seed, T=1.0, alpha=0.0):
    """Two spins with four controls (sx, sy on each spin), time-dependent penalty."""
    P = problems.pauli()
    H0 = (np.pi / 2) * np.kron(P["z"], P["z"]) + 0.3 * np.kron(P["x"], P["x"])
    Hc = np.stack([np.kron(P["x"], P["i"]), np.kron(P["y"], P["i"]),
                   np.kron(P["i"], P["x"]), np.kron(P["i"], P["y"])])
    psi0 = np.zeros(4, dtype=complex); psi0[0] = 1
    tgt = np.array([0, 1, 1, 0], dtype=complex) / np.sqrt(2)
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-0.5, 0.5, size=(1, K, 4))
    al = alpha * (1.0 + np.linspace(0, 1, K))
    return problems.FiniteProblem("pair_c4", H0, Hc, psi0, tgt, T, K, N, u0, al, 0.3, 10)


def _qutrit(K, N, seed, T=1.5):
    """d = 3 (padded to 4 in the kernel): a three-level ladder with two complex controls."""
    rng = np.random.default_rng(seed)
    H0 = np.diag([0.0, 1.1, 2.5]).astype(complex)
    Hc1 = np.array([[0, 1, 0], [1, 0, 1.2], [0, 1.2, 0]], dtype=complex)
    Hc2 = np.array([[0, -1j, 0], [1j, 0, -0.7j], [0, 0.7j, 0]], dtype=complex)
    psi0 = np.array([1, 0, 0], dtype=complex)
    tgt = np.array([0, 0, 1], dtype=complex)
    u0 = rng.uniform(-1, 1, size=(1, K, 2))
    return problems.FiniteProblem("qutrit", H0, np.stack([Hc1, Hc2]), psi0, tgt, T, K, N, u0,
                                  np.zeros(K), 0.4, 10)


def _single_spin(K, N, seed, T=2.0):
    P = problems.pauli()
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-1, 1, size=(1, K, 2))
    return problems.FiniteProblem("spin", 0.5 * P["z"], np.stack([P["x"], P["y"]]),
                                  np.array([1, 0], dtype=complex), np.array([0, 1], dtype=complex),
                                  T, K, N, u0, np.zeros(K), 0.5, 10)


CASES = [
    ("cfg0_spin2_K1000_N8", lambda: problems.spin2(), 50),
    ("spin2_K37_N5_ragged", lambda: problems.spin2(K=37, N=5, seed=3), 20),
    ("spin2_K64_N64", lambda: problems.spin2(K=64, N=64, seed=4), 15),
    ("spin2_K1_N1", lambda: problems.spin2(K=1, N=1, seed=5, T=0.2), 10),
    ("pair_c4_K300_N16_alpha", lambda: _qubit_pair_c4(300, 16, 6, alpha=0.05), 20),
    ("qutrit_K200_N7", lambda: _qutrit(200, 7, 7), 20),
    ("spin_d2_K150_N10", lambda: _single_spin(150, 10, 8), 20),
]


@pytest.mark.parametrize("name,mk,iters", CASES, ids=[c[0] for c in CASES])
def test_one_launch_iterates_equal_plain_gradient(name, mk, iters):
    from paper_1603_01237_amd import _lib
    _say("case small", name)
    p = mk()
    al = p.alpha
    ref = O.plain_gradient_method(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, al, p.rho, iters)
    with _lib.from_problem(p, precision="fp64") as h:
        Jh, done = h.iterate(iters, p.rho)
        u = h.get_controls()[0]
        J, F = h.fidelity()
        g = h.gradient()[0]                 # after the one-launch solve: per-pass slice kernel
    with _lib.from_problem(p, precision="fp64", launch_per_pass=True) as h:
        Jp, donep = h.iterate(iters, p.rho)
        up = h.get_controls()[0]
    assert done == iters and donep == iters
    scale = max(1.0, float(np.max(np.abs(ref["J"]))))
    _say("J", np.max(np.abs(Jh[:, 0] - ref["J"])), "u", _rel(u, ref["u"]), "vs per-pass",
         np.max(np.abs(Jh - Jp)), _rel(u, up))
    assert np.max(np.abs(Jh[:, 0] - ref["J"])) <= 1e-10 * scale
    assert _rel(u, ref["u"]) <= 1e-10
    assert np.max(np.abs(Jh - Jp)) <= 1e-10 * scale and _rel(u, up) <= 1e-10
    gr, Jr, Fr, _ = O.gradient(p.H0, p.Hc, p.psi0, p.target, ref["u"], p.T, al)
    assert abs(J[0] - Jr) <= 1e-10 * scale and abs(F[0] - Fr) <= 1e-10
    # the gradient at the library's final controls: near an optimum it is a small difference
    # of O(1) terms, so it is compared at the same point and on the terms' scale
    gu, Ju, Fu, _ = O.gradient(p.H0, p.Hc, p.psi0, p.target, u, p.T, al)
    assert np.max(np.abs(g - gu)) <= 1e-12 * max(1.0, float(np.max(np.abs(gu))))
    assert abs(J[0] - Ju) <= 1e-12 * scale and abs(F[0] - Fu) <= 1e-12


def test_one_launch_runs_as_one_launch():
    from paper_1603_01237_amd import _lib
    _say("case small launches")
    p = problems.spin2()
    with _lib.from_problem(p, precision="fp64") as h:
        h.set_timing(True)
        h.iterate(50, p.rho)
        kt = h.kernel_times()
    assert set(kt) == {"small_solve"} and kt["small_solve"][0] == 1, kt


def test_fp32_handle_takes_the_fp64_one_launch_solve():
    """An FP32 mixed handle of a small problem iterates through the same FP64 one-launch
    solve as the FP64 handle (same inputs, same kernel: bitwise the same J history and
    controls); with launch_per_pass its FP32 per-pass loop stays within the FP32 bar."""
    from paper_1603_01237_amd import _lib
    _say("case small fp32 handle")
    p = problems.spin2()
    res = {}
    for prec, lpp in (("fp64", False), ("fp32", False), ("fp32", True)):
        with _lib.from_problem(p, precision=prec, launch_per_pass=lpp) as h:
            h.set_timing(True)
            Jh, done = h.iterate(20, p.rho)
            kt = h.kernel_times()
            res[(prec, lpp)] = (Jh[:, 0].copy(), done, h.get_controls()[0].copy(), set(kt))
    J64, d64, u64, k64 = res[("fp64", False)]
    J32, d32, u32, k32 = res[("fp32", False)]
    Jp, dp, up, kp = res[("fp32", True)]
    assert k64 == k32 == {"small_solve"} and "small_solve" not in kp
    assert d32 == d64 and np.array_equal(J32, J64) and np.array_equal(u32, u64)
    assert dp == d64 and np.max(np.abs(Jp - J64)) <= 1e-4
    assert _rel(up, u64) <= 1e-4


def test_one_launch_batch_with_freezing():
    """Three instances (batched H0, different starting controls), fid_stop = 0.9: each
    freezes at its own iteration; done, the J rows and the final controls equal the
    per-pass loop's."""
    from paper_1603_01237_amd import _lib
    _say("case small batch freeze")
    base = problems.spin2(K=100, N=4, T=2.0)
    B = 3
    H0 = np.stack([base.H0 * (1.0 + 0.05 * b) for b in range(B)])
    rng = np.random.default_rng(11)
    u0 = np.stack([base.u0[0] * (0.6 + 0.4 * b) + rng.uniform(-0.01, 0.01, base.u0[0].shape)
                   for b in range(B)])
    p = problems.FiniteProblem("spin2_b3", H0, base.Hc, base.psi0, base.target, base.T, base.K,
                               base.N, u0, np.zeros(base.K), 0.5, 10)
    res = {}
    for lpp in (False, True):
        with _lib.from_problem(p, precision="fp64", launch_per_pass=lpp) as h:
            Jh, done = h.iterate(200, 0.5, fid_stop=0.9)
            res[lpp] = (Jh, done, h.get_controls(), h.fidelity())
    (J1, d1, u1, (Jf1, F1)), (J2, d2, u2, (Jf2, F2)) = res[False], res[True]
    _say("done", d1, d2, "F", F1, F2)
    assert d1 == d2 and 0 < d1 < 200
    rows = min(200, d1 + 1)
    assert np.max(np.abs(J1[:rows] - J2[:rows])) <= 1e-10
    assert _rel(u1, u2) <= 1e-10
    assert np.all(F1 >= 0.9) and np.max(np.abs(F1 - F2)) <= 1e-10
    for b in range(B):
        # each instance alone reaches the same controls (its own freeze iteration)
        q = problems.FiniteProblem("one", H0[b], base.Hc, base.psi0, base.target, base.T, base.K,
                                   base.N, u0[b:b + 1], np.zeros(base.K), 0.5, 10)
        with _lib.from_problem(q, precision="fp64") as h:
            h.iterate(200, 0.5, fid_stop=0.9)
            assert np.array_equal(h.get_controls()[0], u1[b])


def test_one_launch_reports_out_of_range_controls():
    from paper_1603_01237_amd import _lib
    _say("case small range")
    p = problems.spin2(K=10, N=2)
    with _lib.from_problem(p, precision="fp64", set_u=False) as h:
        h.set_controls(np.full((1, 10, 2), 1e5))     # tau ||H|| ~ 4e4: beyond 512
        with pytest.raises(_lib.IsmError) as e:
            h.iterate(2, 0.1)
        assert e.value.code == _lib.ISM_E_UNSUPPORTED
