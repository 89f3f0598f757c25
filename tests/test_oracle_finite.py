"""Pins of the finite-dimensional oracle against mathematics the paper fixes.

Each test names the passage it pins.  None of these compares the oracle with
itself: closed forms, library routines that compute the same object by a
different algorithm (scipy's expm / expm_frechet), central finite differences,
brute-force linear solves and invariants are used instead.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import problems
from oracle import finite as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
SZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2)


def _tiny_problem(seed=7, d=4, C=2, K=24, T=1.3, alpha=0.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    H0 = 0.5 * (A + A.conj().T)
    Hc = []
    for _ in range(C):
        B = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        Hc.append(0.5 * (B + B.conj().T))
    Hc = np.stack(Hc)
    psi0 = rng.standard_normal(d) + 1j * rng.standard_normal(d); psi0 /= np.linalg.norm(psi0)
    tgt = rng.standard_normal(d) + 1j * rng.standard_normal(d); tgt /= np.linalg.norm(tgt)
    u = rng.uniform(-1, 1, size=(K, C))
    al = np.full(K, alpha)
    return H0, Hc, psi0, tgt, u, T, al


# --- P1: closed-form single-spin propagator (Sec. 4.A spin operators) -----------------

def test_p1_single_spin_closed_form_random():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = rng.standard_normal(3); n /= np.linalg.norm(n)
        theta = rng.uniform(-7, 7)
        ns = n[0] * SX + n[1] * SY + n[2] * SZ
        U = O.step_unitary(ns, theta / 2)      # exp(-i (theta/2) n.sigma)
        ref = math.cos(theta / 2) * I2 - 1j * math.sin(theta / 2) * ns
        assert np.max(np.abs(U - ref)) <= 1e-15 * 4


def test_p1_golden_rotations():
    with open(os.path.join(GOLD, "spin_rotations.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for row in rows:
        lhs, rhs = row.split("|")
        th, nx, ny, nz = map(float, lhs.split())
        v = list(map(float, rhs.split()))
        ref = np.array([[v[0] + 1j * v[1], v[2] + 1j * v[3]], [v[4] + 1j * v[5], v[6] + 1j * v[7]]])
        U = O.step_unitary(nx * SX + ny * SY + nz * SZ, th / 2)
        assert np.max(np.abs(U - ref)) <= 2e-15


def test_p1_exp_vs_eigendecomposition():
    """The step map against the spectral form V diag(e^{-i tau w}) V^dagger of the same
    exponential (numpy's eigh), an independent evaluation."""
    H0, Hc, *_ = _tiny_problem(d=6)
    w, V = np.linalg.eigh(H0)
    for tau in (1e-3, 0.1, 0.7):
        ref = (V * np.exp(-1j * tau * w)[None, :]) @ V.conj().T
        assert np.max(np.abs(O.step_unitary(H0, tau) - ref)) <= 1e-13


# --- P2: product form, cfg0 Hamiltonian with the zz coupling off ----------------------

def test_p2_two_spin_product():
    p = problems.spin2()
    rng = np.random.default_rng(2)
    for _ in range(20):
        ux, uy = rng.uniform(-3, 3, 2)
        tau = rng.uniform(1e-3, 0.5)
        H = O.hamiltonian(0 * p.H0, p.Hc, np.array([ux, uy]))
        U = O.step_unitary(H, tau)
        r = math.hypot(ux, uy)
        R = math.cos(tau * r) * I2 - 1j * math.sin(tau * r) * (ux * SX + uy * SY) / r
        assert np.max(np.abs(U - np.kron(R, R))) <= 1e-15 * 8


# --- P3/P4/P5: unitarity, norm, reversibility, overlap invariant (Sec. 3 norm remark) ----

def test_p3_p4_p5_invariants():
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(K=200, T=3.0)
    tau = T / u.shape[0]
    Us = O.step_unitaries(H0, Hc, u, tau)
    for U in Us:
        assert np.max(np.abs(U.conj().T @ U - np.eye(4))) <= 1e-14
    psis = O.forward(Us, psi0)
    assert abs(np.linalg.norm(psis[-1]) - 1) <= 200 * 1e-15
    back = O.backward(Us, psis[-1])
    assert np.max(np.abs(back[0] - psi0)) <= 1e-13
    lams = O.backward(Us, tgt)
    z = np.vdot(psis[-1], tgt)
    for j in range(len(Us) + 1):
        assert abs(np.vdot(psis[j], lams[j]) - z) <= 1e-13


# --- P6: exact discrete gradient vs central differences (Sec. 3: exact differentiability) ---

@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_p6_gradient_fd(alpha):
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(K=12, alpha=alpha)
    al = al * np.linspace(0.5, 1.5, al.shape[0])      # time-dependent alpha (Sec. 4.B)
    tau = T / u.shape[0]
    g, J, F, _ = O.gradient(H0, Hc, psi0, tgt, u, T, al)

    def Jof(v):
        Us = O.step_unitaries(H0, Hc, v, tau)
        return O.objective(O.forward(Us, psi0)[-1], tgt, v, al, tau)[0]

    eps = 1e-5
    fd = np.zeros_like(u)
    for j in range(u.shape[0]):
        for c in range(u.shape[1]):
            up = u.copy(); up[j, c] += eps
            um = u.copy(); um[j, c] -= eps
            fd[j, c] = (Jof(up) - Jof(um)) / (2 * eps)
    rel = np.max(np.abs(tau * g - fd)) / np.max(np.abs(fd))
    assert rel <= 1e-8


def test_p6_first_order_formula_is_not_exact():
    """Guard: the first-order form Im<lambda|H_c|psi> (no step averaging) must NOT pass
    the FD bar at this step size, so the FD pin can tell the two apart."""
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(K=6, T=3.0)
    tau = T / u.shape[0]
    g, *_ = O.gradient(H0, Hc, psi0, tgt, u, T, al)
    Us = O.step_unitaries(H0, Hc, u, tau)
    ps, ls = O.forward(Us, psi0), O.backward(Us, tgt)
    g1 = np.array([[np.vdot(ls[j], Hc[c] @ ps[j]).imag for c in range(2)] for j in range(6)])
    assert np.max(np.abs(g1 - g)) / np.max(np.abs(g)) > 1e-3


# --- P7: step average vs scipy's Frechet derivative of expm ---------------------------

def test_p7_hhat_vs_expm_frechet():
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(d=5, C=3)
    for tau in (1e-3, 0.05, 0.4):
        H = O.hamiltonian(H0, Hc, u[0])
        U = O.step_unitary(H, tau)
        Hh = O.hhat(H, Hc, tau)
        for c in range(3):
            _, L = sla.expm_frechet(-1j * tau * H, -1j * tau * Hc[c])
            assert np.max(np.abs(-1j * tau * U @ Hh[c] - L)) <= 1e-13


def test_p7_hhat_degenerate_spectrum():
    """phi1 series branch: H with repeated eigenvalues (x = 0 on the whole diagonal)."""
    H = np.diag([1.0, 1.0, -2.0, -2.0]).astype(complex)
    Hc = np.stack([np.kron(SX, I2)])
    tau = 0.3
    _, L = sla.expm_frechet(-1j * tau * H, -1j * tau * Hc[0])
    U = O.step_unitary(H, tau)
    assert np.max(np.abs(-1j * tau * U @ O.hhat(H, Hc, tau)[0] - L)) <= 1e-14


# --- P8: ISM == plain gradient iterates (Theorem 2; Sec. 4.A: same values for all N) ----

@pytest.mark.parametrize("N", [1, 2, 3, 8])
def test_p8_ism_equals_plain_one_call(N):
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(K=26, alpha=0.2)
    g, J, F, *_ = O.gradient(H0, Hc, psi0, tgt, u, T, al)
    gi, Ji, Fi, phi, Psi, Lam = O.ism_gradient(H0, Hc, psi0, tgt, u, T, al, N)
    assert np.max(np.abs(gi - g)) <= 1e-12 * max(1, np.max(np.abs(g)))
    assert abs(Ji - J) <= 1e-13 and abs(Fi - F) <= 1e-13


@pytest.mark.parametrize("N", [2, 3, 8])
def test_p8_ism_equals_plain_iterates(N):
    p = problems.spin2(K=40)
    kw = dict(H0=p.H0, Hc=p.Hc, psi0=p.psi0, target=p.target, u0=p.u0[0], T=p.T,
              alpha=p.alpha, rho=p.rho, iters=50)
    a = O.plain_gradient_method(**kw)
    b = O.ism_iterate(N=N, **kw)
    assert np.max(np.abs(a["u"] - b["u"])) <= 1e-10
    assert np.max(np.abs(a["J"] - b["J"])) <= 1e-10


def test_p8_gate_form_ism_equals_plain_and_fd():
    """Gate synthesis (evolution operators, Sec. 2 remark): psi0 = I, target W, <A|B> = Tr(A^+B)/d."""
    rng = np.random.default_rng(3)
    d, K, T = 4, 10, 1.0
    p = problems.spin2()
    W = problems.haar_unitary(d, rng)
    u = rng.uniform(-1, 1, size=(K, 2)); al = np.zeros(K)
    g, J, F, UK = O.gradient(p.H0, p.Hc, np.eye(d), W, u, T, al)
    assert abs(J - np.trace(W.conj().T @ UK).real / d) <= 1e-14
    assert abs(F - abs(np.trace(W.conj().T @ UK)) ** 2 / d ** 2) <= 1e-14
    for N in (2, 3):
        gi, Ji, *_ = O.ism_gradient(p.H0, p.Hc, np.eye(d), W, u, T, al, N)
        assert np.max(np.abs(gi - g)) <= 1e-12
    tau = T / K
    eps = 1e-5

    def Jof(v):
        Us = O.step_unitaries(p.H0, p.Hc, v, tau)
        return O.objective(O.forward(Us, np.eye(d))[-1], W, v, al, tau)[0]
    for j in (0, 4, 9):
        for c in (0, 1):
            up = u.copy(); up[j, c] += eps
            um = u.copy(); um[j, c] -= eps
            assert abs((Jof(up) - Jof(um)) / (2 * eps) - tau * g[j, c]) <= 1e-9


# --- P9: Theorem 1 (value up to the constant; argmax) --------------------------------

@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_p9_theorem1(N):
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(K=15, alpha=0.4)
    K = u.shape[0]
    tau = T / K
    s = O.slice_starts(K, N)
    Us = O.step_unitaries(H0, Hc, u, tau)
    Ms = O.assemble(Us, s)
    Psi, Lam = O.boundaries(Ms, psi0, tgt)
    phi = O.intermediate_states(Psi, Lam, s, K)
    J, _ = O.objective(Psi[-1], tgt, u, al, tau)
    assert abs(O.theorem1_functional(Ms, phi, u, al, s, K, T) - (J - 1.0)) <= 1e-12
    star = O.theorem1_argmax(Ms, psi0, tgt, s, K)
    for n in range(N + 1):
        assert np.max(np.abs(star[n] - phi[n])) <= 1e-12
    if N > 1:       # any perturbation of an interior phi lowers J_par
        rng = np.random.default_rng(9)
        pert = [x.copy() for x in phi]
        pert[1] = pert[1] + 1e-3 * (rng.standard_normal(4) + 1j * rng.standard_normal(4))
        assert O.theorem1_functional(Ms, pert, u, al, s, K, T) < O.theorem1_functional(Ms, phi, u, al, s, K, T)


# --- P10: Theorem 2 per slice, both end conditions ----------------------------------

def test_p10_theorem2_per_slice():
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(K=24)
    K, N = 24, 5
    tau = T / K
    s = O.slice_starts(K, N)
    Us = O.step_unitaries(H0, Hc, u, tau)
    Hh = [O.hhat(O.hamiltonian(H0, Hc, u[j]), Hc, tau) for j in range(K)]
    ps, ls = O.forward(Us, psi0), O.backward(Us, tgt)
    Psi, Lam = O.boundaries(O.assemble(Us, s), psi0, tgt)
    phi = O.intermediate_states(Psi, Lam, s, K)
    for n in range(N):
        beta = K / (s[n + 1] - s[n])
        psi_n = [phi[n]]
        for j in range(s[n], s[n + 1]):
            psi_n.append(Us[j] @ psi_n[-1])
        for endc in ("re", "sq"):
            end = phi[n + 1] if endc == "re" else phi[n + 1] - psi_n[-1]
            chi = [end]
            for j in range(s[n + 1] - 1, s[n] - 1, -1):
                chi.append(Us[j].conj().T @ chi[-1])
            chi = chi[::-1]
            for j in range(s[n], s[n + 1]):
                for c in range(2):
                    lhs = beta * np.vdot(chi[j - s[n]], Hh[j][c] @ psi_n[j - s[n]]).imag
                    rhs = np.vdot(ls[j], Hh[j][c] @ ps[j]).imag
                    assert abs(lhs - rhs) <= 1e-12


# --- P11: propagator assembling == sequential propagation ---------------------------

def test_p11_assembly():
    H0, Hc, psi0, tgt, u, T, al = _tiny_problem(K=23)
    K, N = 23, 4
    tau = T / K
    s = O.slice_starts(K, N)
    assert list(s) == [0, 5, 11, 17, 23]
    Us = O.step_unitaries(H0, Hc, u, tau)
    Psi, Lam = O.boundaries(O.assemble(Us, s), psi0, tgt)
    ps, ls = O.forward(Us, psi0), O.backward(Us, tgt)
    for n in range(N + 1):
        assert np.max(np.abs(Psi[n] - ps[s[n]])) <= 1e-13
        assert np.max(np.abs(Lam[n] - ls[s[n]])) <= 1e-13
    phi = O.intermediate_states(Psi, Lam, s, K)
    assert np.max(np.abs(phi[0] - psi0)) == 0.0
    assert np.max(np.abs(phi[N] - tgt)) == 0.0


def test_slice_starts_edges():
    assert list(O.slice_starts(5, 5)) == [0, 1, 2, 3, 4, 5]
    assert list(O.slice_starts(7, 1)) == [0, 7]
    s = O.slice_starts(20000, 128)
    L = np.diff(s)
    assert set(L.tolist()) == {156, 157} and s[-1] == 20000
    with pytest.raises(ValueError):
        O.slice_starts(4, 5)
    with pytest.raises(ValueError):
        O.slice_starts(4, 0)


# --- P12: cfg0 swap symmetry ------------------------------------------------------

def test_p12_singlet_stays_zero():
    p = problems.spin2(K=200)
    tau = p.T / p.K
    Us = O.step_unitaries(p.H0, p.Hc, p.u0[0], tau)
    singlet = np.array([0, 1, -1, 0]) / math.sqrt(2)
    for psi in O.forward(Us, p.psi0):
        assert abs(np.vdot(singlet, psi)) <= 1e-14


# --- P13/P14: rotor operator and free rotor --------------------------------------

def test_p13_rotor_cos_gauss_legendre():
    with open(os.path.join(GOLD, "legendre_p5_roots.txt")) as f:
        roots = np.array([float(l) for l in f if l.strip() and not l.startswith("#")])
    C = problems.rotor_cos_matrix(20)
    w = np.linalg.eigvalsh(C[:5, :5])
    assert np.max(np.abs(np.sort(w) - roots)) <= 1e-14
    for m in (3, 8, 21):
        nodes, _ = np.polynomial.legendre.leggauss(m)
        assert np.max(np.abs(np.linalg.eigvalsh(C[:m, :m]) - nodes)) <= 1e-13
    t = problems.rotor_target(20)
    assert abs(np.vdot(t, C @ t).real - roots[-1]) <= 1e-14
    assert t[0].real > 0 and np.max(np.abs(t[5:])) == 0


def test_p14_free_rotor():
    p = problems.rotor(batch=2, K=50, T=0.7)
    tau = p.T / p.K
    rng = np.random.default_rng(4)
    psi0 = rng.standard_normal(21) + 1j * rng.standard_normal(21)
    B = p.meta["B"][1]
    Us = O.step_unitaries(p.H0[1], p.Hc, np.zeros((p.K, 1)), tau)
    psiK = O.forward(Us, psi0)[-1]
    j = np.arange(21)
    assert np.max(np.abs(psiK - np.exp(-1j * B * j * (j + 1) * p.T) * psi0)) <= 1e-13


# --- P20: ascent sanity ----------------------------------------------------------

def test_p20_ascent_monotone_small_step():
    p = problems.spin2(K=50)
    r = O.plain_gradient_method(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 0.05, 15)
    assert np.all(np.diff(r["J"]) > 0)
    assert np.all(np.diff(r["Err"]) != 0)
