"""Pins of the Crank-Nicolson oracle (Sec. 3 step map U = (I + L)^{-1}(I - L), L = i tau H/2)
against mathematics that does not go through the oracle's own formulas."""
import numpy as np
import pytest

import problems
from oracle import finite as O

SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
SZ = np.array([[1, 0], [0, -1]], dtype=complex)


def _rand_herm(rng, d):
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    return 0.5 * (A + A.conj().T)


def test_cn_single_spin_closed_form():
    """H = (omega/2) n.sigma: with b = tau omega / 4, (I + i b n.sigma)^{-1}(I - i b n.sigma)
    = ((1 - b^2) I - 2 i b n.sigma) / (1 + b^2), since (n.sigma)^2 = I."""
    rng = np.random.default_rng(31)
    for _ in range(20):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        om, tau = rng.uniform(0.1, 5.0), rng.uniform(0.01, 0.5)
        ns = n[0] * SX + n[1] * SY + n[2] * SZ
        b = tau * om / 4
        ref = ((1 - b * b) * np.eye(2) - 2j * b * ns) / (1 + b * b)
        U = O.step_unitary_cn(0.5 * om * ns, tau)
        assert np.max(np.abs(U - ref)) <= 1e-15


def test_cn_unitary_and_second_order():
    rng = np.random.default_rng(32)
    H = _rand_herm(rng, 6)
    for tau in (0.3, 0.05):
        U = O.step_unitary_cn(H, tau)
        assert np.max(np.abs(U.conj().T @ U - np.eye(6))) <= 1e-14
    # Cayley transform vs exp: e^x - (1 + x/2)/(1 - x/2) = -x^3/12 + O(x^4), so halving tau
    # divides the difference by 8
    e1 = np.linalg.norm(O.step_unitary_cn(H, 0.02) - O.step_unitary(H, 0.02), 2)
    e2 = np.linalg.norm(O.step_unitary_cn(H, 0.01) - O.step_unitary(H, 0.01), 2)
    assert 7.5 < e1 / e2 < 8.5
    hn = np.linalg.norm(H, 2)
    assert e1 <= 1.05 * (0.02 * hn) ** 3 / 12


def test_cn_midpoint_identity():
    """psi_j + psi_{j+1} = 2 (I - L)^{-1} psi_{j+1}: from (I + L) psi_{j+1} = (I - L) psi_j."""
    rng = np.random.default_rng(33)
    H = _rand_herm(rng, 5)
    psi = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    nxt = O.step_unitary_cn(H, 0.2) @ psi
    L = O.cn_generator(H, 0.2)
    rhs = 2 * np.linalg.solve(np.eye(5) - L, nxt)
    assert np.max(np.abs(psi + nxt - rhs)) <= 1e-14


def _fd(fun, u, eps=1e-5):
    g = np.zeros_like(u)
    for idx in np.ndindex(u.shape):
        up, um = u.copy(), u.copy()
        up[idx] += eps
        um[idx] -= eps
        g[idx] = (fun(up) - fun(um)) / (2 * eps)
    return g


@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_cn_gradient_vs_finite_differences(alpha):
    p = problems.spin2(K=8, N=2)
    rng = np.random.default_rng(34)
    u = rng.uniform(-1, 1, (8, 2))
    al = np.full(8, alpha)
    tau = p.T / 8

    def J(uu):
        Us = O.step_unitaries_cn(p.H0, p.Hc, uu, tau)
        return O.objective(O.forward(Us, p.psi0)[-1], p.target, uu, al, tau)[0]

    g, *_ = O.gradient_cn(p.H0, p.Hc, p.psi0, p.target, u, p.T, al)
    fd = _fd(J, u)
    assert np.linalg.norm(tau * g - fd) / np.linalg.norm(fd) <= 1e-8


def test_cn_gate_gradient_vs_finite_differences():
    base = problems.spin2(K=6, N=2)
    rng = np.random.default_rng(35)
    W = problems.haar_unitary(4, rng)
    u = rng.uniform(-1, 1, (6, 2))
    tau = 1.0 / 6
    al = np.zeros(6)

    def J(uu):
        Us = O.step_unitaries_cn(base.H0, base.Hc, uu, tau)
        return O.objective(O.forward(Us, np.eye(4, dtype=complex))[-1], W, uu, al, tau)[0]

    g, *_ = O.gradient_cn(base.H0, base.Hc, np.eye(4, dtype=complex), W, u, 1.0, al)
    fd = _fd(J, u)
    assert np.linalg.norm(tau * g - fd) / np.linalg.norm(fd) <= 1e-8


@pytest.mark.parametrize("N", [1, 3, 8])
def test_cn_ism_equals_plain(N):
    p = problems.spin2(K=37, N=N)
    rng = np.random.default_rng(36)
    u = rng.uniform(-1, 1, (37, 2))
    g, J, F, _ = O.gradient_cn(p.H0, p.Hc, p.psi0, p.target, u, p.T, p.alpha)
    gi, Ji, Fi, phi, _, _ = O.ism_gradient_cn(p.H0, p.Hc, p.psi0, p.target, u, p.T, p.alpha, N)
    assert np.max(np.abs(g - gi)) <= 1e-12 * max(1.0, np.max(np.abs(g)))
    assert abs(J - Ji) <= 1e-12
    assert np.max(np.abs(phi[0] - p.psi0)) == 0 and np.max(np.abs(phi[-1] - p.target)) == 0


def test_cn_ism_iterates_equal_plain():
    p = problems.spin2(K=40, N=6)
    ref = O.plain_gradient_method_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 0.5, 30)
    ism = O.ism_iterate_cn(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 0.5, 30, 6)
    assert np.max(np.abs(ref["u"] - ism["u"])) <= 1e-10
    assert np.max(np.abs(ref["J"] - ism["J"])) <= 1e-10
    assert ref["J"][-1] > ref["J"][0]


def test_cn_dropped_solve_is_detected(monkeypatch):
    """Planting a mistake (chi_j = lambda_{j+1}, the (I - L_j) solve left out) breaks the
    finite-difference pin."""
    real_solve = np.linalg.solve

    def fake(A, b):
        return b if b.ndim == 1 else real_solve(A, b)

    monkeypatch.setattr(O.np.linalg, "solve", fake)
    with pytest.raises(AssertionError):
        test_cn_gradient_vs_finite_differences(0.0)
