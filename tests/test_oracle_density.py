"""Pins of the density-matrix oracle (Liouville-von Neumann form of the five-spin
experiment, Sec. 4.A) against mathematics that does not go through its own formulas: the
Liouville-space vectorisation run through the (separately pinned) state oracle, central
finite differences with scipy's expm, product-operator closed forms, invariants.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import problems
from oracle import density as D
from oracle import finite as O


def _liouville(H):
    """Superoperator of [H, .] on row-major vec: vec(A X B) = (A (x) B^T) vec(X)."""
    d = H.shape[0]
    return np.kron(H, np.eye(d)) - np.kron(np.eye(d), H.T)


def _tiny(seed=41, d=4, C=2, K=16, T=0.9):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    H0 = 0.5 * (A + A.conj().T)
    Hc = []
    for _ in range(C):
        B = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        Hc.append(0.5 * (B + B.conj().T))
    R0 = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)); R0 = R0 + R0.conj().T
    Rf = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)); Rf = Rf + Rf.conj().T
    u = rng.uniform(-1, 1, size=(K, C))
    return H0, np.stack(Hc), R0, Rf, u, T


@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_liouville_vectorisation(alpha):
    """The density problem is the state problem of dimension d^2 with Hamiltonian
    superoperators and <a|b> = sum conj(a) b on vec(rho) = Tr(A^+ B)."""
    H0, Hc, R0, Rf, u, T = _tiny()
    al = np.full(u.shape[0], alpha)
    g, J, F, rhoK = D.gradient(H0, Hc, R0, Rf, u, T, al)
    gv, Jv, Fv, vK = O.gradient(_liouville(H0), np.stack([_liouville(h) for h in Hc]),
                                R0.reshape(-1), Rf.reshape(-1), u, T, al)
    assert np.max(np.abs(rhoK.reshape(-1) - vK)) <= 1e-12
    assert abs(J - Jv) <= 1e-12
    assert np.max(np.abs(g - gv)) <= 1e-11 * max(1.0, np.max(np.abs(gv)))
    # the oracle's F is the squared overlap normalised by the two norms
    assert abs(F - Fv / (np.vdot(R0, R0).real * np.vdot(Rf, Rf).real)) <= 1e-13


def test_gradient_fd():
    H0, Hc, R0, Rf, u, T = _tiny(seed=42, K=10)
    al = np.full(10, 0.2)
    g, *_ = D.gradient(H0, Hc, R0, Rf, u, T, al)
    tau, eps = T / 10, 1e-6

    def Jof(v):
        rho = R0.astype(complex)
        for j in range(10):
            U = sla.expm(-1j * tau * (H0 + v[j, 0] * Hc[0] + v[j, 1] * Hc[1]))
            rho = U @ rho @ U.conj().T
        return np.trace(rho.conj().T @ Rf).real - 0.5 * tau * np.sum(al[:, None] * v ** 2)
    for j in range(10):
        for c in range(2):
            up = u.copy(); up[j, c] += eps
            um = u.copy(); um[j, c] -= eps
            assert abs((Jof(up) - Jof(um)) / (2 * eps) - tau * g[j, c]) <= 1e-8


@pytest.mark.parametrize("N", [1, 2, 3, 7])
def test_ism_equals_plain(N):
    H0, Hc, R0, Rf, u, T = _tiny(seed=43, K=21)
    al = np.full(21, 0.1)
    g, J, F, _ = D.gradient(H0, Hc, R0, Rf, u, T, al)
    gi, Ji, Fi, phi, Psi, Lam = D.ism_gradient(H0, Hc, R0, Rf, u, T, al, N)
    assert np.max(np.abs(gi - g)) <= 1e-11 * max(1.0, np.max(np.abs(g)))
    assert abs(Ji - J) <= 1e-12 and abs(Fi - F) <= 1e-12
    a = D.plain_gradient_method(H0, Hc, R0, Rf, u, T, al, 0.02, 6)
    b = D.ism_iterate(H0, Hc, R0, Rf, u, T, al, 0.02, 6, N)
    assert np.max(np.abs(a["u"] - b["u"])) <= 1e-10 * np.max(np.abs(a["u"]))


def test_five_spin_free_evolution_product_operators():
    """Under H0 = 2 pi J sum I_z I_z alone, <I_x^(k)> of I_x^(k) decays as the product of
    cos(pi J_kl t) over the partners l of spin k (product-operator formalism): spin 1 couples
    to 2 and 3, spin 5 only to 2."""
    p = problems.spin5_density(K=64, T=0.013)
    Jp = p.meta["Jp"]
    Ix, _, _ = problems.spin_operators(5)
    tau = p.T / p.K
    Us = O.step_unitaries(p.H0, p.Hc, np.zeros((p.K, 10)), tau)
    rho = D.forward(Us, Ix[0])
    rho5 = D.forward(Us, Ix[4])
    nrm = np.trace(Ix[0] @ Ix[0]).real
    for j in (0, 17, 64):
        t = j * tau
        assert abs(np.trace(Ix[0] @ rho[j]).real / nrm - math.cos(math.pi * Jp * t) ** 2) <= 1e-12
        assert abs(np.trace(Ix[4] @ rho5[j]).real / nrm - math.cos(math.pi * Jp * t)) <= 1e-12


def test_purity_conserved_and_hermitian():
    p = problems.spin5_density(K=40, T=0.01, u_amp=300.0)
    Us = O.step_unitaries(p.H0, p.Hc, p.u0[0], p.T / p.K)
    rho = D.forward(Us, p.psi0)
    for r in (rho[0], rho[13], rho[-1]):
        assert abs(np.trace(r @ r).real - np.trace(p.psi0 @ p.psi0).real) <= 1e-12
        assert np.max(np.abs(r - r.conj().T)) <= 1e-13


# --- Crank-Nicolson conjugation map (Sec. 3 Cayley step applied as rho <- U rho U^+) ------

def _J_cn_direct(H0, Hc, R0, Rf, u, T, al):
    """J_tau of the Cayley conjugation map, each step solved directly with numpy's dense
    solver on the inputs (no oracle routine)."""
    K = u.shape[0]
    tau = T / K
    d = H0.shape[0]
    I = np.eye(d)
    rho = R0.astype(complex)
    for j in range(K):
        H = H0 + sum(u[j, c] * Hc[c] for c in range(Hc.shape[0]))
        U = np.linalg.solve(I + 0.5j * tau * H, I - 0.5j * tau * H)
        rho = U @ rho @ U.conj().T
    return float(np.vdot(Rf, rho).real) - 0.5 * tau * float(np.sum(al[:, None] * u ** 2))


@pytest.mark.parametrize("alpha", [0.0, 0.25])
def test_cn_gradient_fd(alpha):
    """tau g of the Crank-Nicolson conjugation map against central finite differences of J
    computed by direct dense solves (rel 1e-8)."""
    H0, Hc, R0, Rf, u, T = _tiny(seed=44, K=12, T=1.1)
    al = np.full(12, alpha)
    g, J, *_ = D.gradient_cn(H0, Hc, R0, Rf, u, T, al)
    assert abs(J - _J_cn_direct(H0, Hc, R0, Rf, u, T, al)) <= 1e-12
    tau, eps = T / 12, 1e-6
    fd = np.zeros_like(u)
    for j in range(12):
        for c in range(Hc.shape[0]):
            up, um = u.copy(), u.copy()
            up[j, c] += eps
            um[j, c] -= eps
            fd[j, c] = (_J_cn_direct(H0, Hc, R0, Rf, up, T, al) -
                        _J_cn_direct(H0, Hc, R0, Rf, um, T, al)) / (2 * eps)
    assert np.linalg.norm(tau * g - fd) / np.linalg.norm(fd) <= 1e-8


def test_cn_gradient_is_not_the_exponential_one():
    """Guard: the exponential map's gradient evaluated on the same controls misses the
    Crank-Nicolson finite differences at this step size, so the pin above tells them apart."""
    H0, Hc, R0, Rf, u, T = _tiny(seed=44, K=12, T=1.1)
    al = np.zeros(12)
    g_exp, *_ = D.gradient(H0, Hc, R0, Rf, u, T, al)
    g_cn, *_ = D.gradient_cn(H0, Hc, R0, Rf, u, T, al)
    assert np.linalg.norm(g_exp - g_cn) / np.linalg.norm(g_cn) > 1e-3


@pytest.mark.parametrize("N", [1, 3, 5])
def test_cn_ism_equals_plain(N):
    """Theorem 2 with the Cayley conjugation map: the ISM slice gradients (non-divisible K
    included) equal the plain gradient per call, and the iterates over several steps."""
    H0, Hc, R0, Rf, u, T = _tiny(seed=45, K=17, T=0.8)
    al = np.full(17, 0.1)
    g, J, F, _ = D.gradient_cn(H0, Hc, R0, Rf, u, T, al)
    gi, Ji, Fi, *_ = D.ism_gradient_cn(H0, Hc, R0, Rf, u, T, al, N)
    assert np.max(np.abs(gi - g)) <= 1e-12 * max(1.0, np.max(np.abs(g)))
    assert abs(Ji - J) <= 1e-13 and abs(Fi - F) <= 1e-13
    a = D.plain_gradient_method_cn(H0, Hc, R0, Rf, u, T, al, 0.05, 6)
    b = D.ism_iterate_cn(H0, Hc, R0, Rf, u, T, al, 0.05, 6, N)
    assert np.max(np.abs(a["u"] - b["u"])) <= 1e-10
    assert np.max(np.abs(a["J"] - b["J"])) <= 1e-10


def test_cn_conjugation_preserves_purity():
    """Each Cayley step is unitary, so Tr(rho^2) and hermiticity are conserved."""
    H0, Hc, R0, Rf, u, T = _tiny(seed=46, K=40, T=2.0)
    Us = O.step_unitaries_cn(H0, Hc, u, T / 40)
    rho = D.forward(Us, R0)
    p0 = np.trace(R0 @ R0).real
    for r in rho:
        assert abs(np.trace(r @ r).real - p0) <= 1e-12 * p0
        assert np.max(np.abs(r - r.conj().T)) <= 1e-12
