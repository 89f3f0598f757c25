"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins catch them.

Each case patches one oracle routine with a wrong variant (dropped term, wrong sign,
swapped weights, missing adjoint, missing factor) and asserts that the relevant
pin's error exceeds that pin's tolerance.
"""
import math

import numpy as np
import pytest

from oracle import finite as O
from oracle import gpe as G


def _tiny(seed=11, d=4, C=2, K=18, T=1.1):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    H0 = 0.5 * (A + A.conj().T)
    Hc = []
    for _ in range(C):
        B = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        Hc.append(0.5 * (B + B.conj().T))
    psi0 = rng.standard_normal(d) + 1j * rng.standard_normal(d); psi0 /= np.linalg.norm(psi0)
    tgt = rng.standard_normal(d) + 1j * rng.standard_normal(d); tgt /= np.linalg.norm(tgt)
    u = rng.uniform(-1, 1, size=(K, C))
    return H0, np.stack(Hc), psi0, tgt, u, T, np.full(K, 0.1)


def _fd_error():
    H0, Hc, psi0, tgt, u, T, al = _tiny()
    tau = T / u.shape[0]
    g, *_ = O.gradient(H0, Hc, psi0, tgt, u, T, al)
    eps = 1e-5
    fd = np.zeros_like(u)
    for j in range(u.shape[0]):
        for c in range(u.shape[1]):
            up = u.copy(); up[j, c] += eps
            um = u.copy(); um[j, c] -= eps
            Jp = O.objective(O.forward(O.step_unitaries(H0, Hc, up, tau), psi0)[-1], tgt, up, al, tau)[0]
            Jm = O.objective(O.forward(O.step_unitaries(H0, Hc, um, tau), psi0)[-1], tgt, um, al, tau)[0]
            fd[j, c] = (Jp - Jm) / (2 * eps)
    return np.max(np.abs(tau * g - fd)) / np.max(np.abs(fd))


def _ism_error(N=3):
    H0, Hc, psi0, tgt, u, T, al = _tiny()
    g, *_ = O.gradient(H0, Hc, psi0, tgt, u, T, al)
    gi, *_ = O.ism_gradient(H0, Hc, psi0, tgt, u, T, al, N)
    return np.max(np.abs(gi - g))


def test_unmutated_pins_pass():
    assert _fd_error() <= 1e-8
    assert _ism_error() <= 1e-12


def test_mutation_first_order_hhat(monkeypatch):
    monkeypatch.setattr(O, "hhat", lambda H, Hcs, tau: np.array(Hcs))
    assert _fd_error() > 1e-8


def test_mutation_gradient_sign(monkeypatch):
    real = O.inner
    monkeypatch.setattr(O, "inner", lambda a, b: np.conj(real(a, b)))
    assert _fd_error() > 1e-8


def test_mutation_phi_weights_swapped(monkeypatch):
    def bad(Psi, Lam, s, K):
        return [(s[n] / K) * Psi[n] + (1.0 - s[n] / K) * Lam[n] for n in range(len(s))]
    monkeypatch.setattr(O, "intermediate_states", bad)
    assert _ism_error() > 1e-12


def test_mutation_missing_beta(monkeypatch):
    real = O.ism_slice_gradient

    def bad(Us, Hh, u, alpha, a, b, sn, sn1, K):
        g, e = real(Us, Hh, u, alpha, a, b, sn, sn1, K)
        return g * (sn1 - sn) / K, e
    monkeypatch.setattr(O, "ism_slice_gradient", bad)
    assert _ism_error() > 1e-12


def test_mutation_adjoint_boundary_without_dagger(monkeypatch):
    def bad(Ms, psi0, target):
        N = len(Ms)
        Psi = [np.array(psi0)]
        for n in range(N):
            Psi.append(Ms[n] @ Psi[-1])
        Lam = [None] * (N + 1)
        Lam[N] = np.array(target)
        for n in range(N - 1, -1, -1):
            Lam[n] = Ms[n] @ Lam[n + 1]
        return Psi, Lam
    monkeypatch.setattr(O, "boundaries", bad)
    assert _ism_error() > 1e-12


def test_mutation_phi_time_off_by_one(monkeypatch):
    """phi_n weighted with t_{n}+tau while the slice starts at t_n (an index slip)."""
    def bad(Psi, Lam, s, K):
        w = [min(s[n] + (1 if 0 < n < len(s) - 1 else 0), K) / K for n in range(len(s))]
        return [(1.0 - w[n]) * Psi[n] + w[n] * Lam[n] for n in range(len(s))]
    monkeypatch.setattr(O, "intermediate_states", bad)
    assert _ism_error() > 1e-12


def _gpe_fd_error():
    n, L, K, T, gnl = 32, 12.0, 10, 0.3, 10.0
    x, _, dx = G.grid(n, L)
    psi0 = np.exp(-0.5 * (x + 0.5) ** 2).astype(complex); psi0 /= math.sqrt(dx * np.sum(abs(psi0) ** 2))
    tgt = np.exp(-0.5 * (x - 1) ** 2 + 0.2j * x); tgt /= math.sqrt(dx * np.sum(abs(tgt) ** 2))
    u = np.linspace(-1, 1, K)
    V0, V1, V2 = 0.5 * x ** 2, -x, 0.5
    g, *_ = G.adjoint_gradient(psi0, tgt, u, V0, V1, V2, gnl, L, T)
    eps = 1e-5
    fd = np.zeros(K)
    for j in range(K):
        up = u.copy(); up[j] += eps
        um = u.copy(); um[j] -= eps
        fd[j] = (G.adjoint_gradient(psi0, tgt, up, V0, V1, V2, gnl, L, T)[1]
                 - G.adjoint_gradient(psi0, tgt, um, V0, V1, V2, gnl, L, T)[1]) / (2 * eps)
    return np.max(np.abs((T / K) * g - fd)) / np.max(np.abs(fd))


def test_gpe_unmutated_and_dropped_potential_derivative(monkeypatch):
    assert _gpe_fd_error() <= 1e-6
    monkeypatch.setattr(G, "dpotential", lambda V1, V2, u: V1)    # drop the 2 u V2 term
    assert _gpe_fd_error() > 1e-6


def test_gpe_mutation_kinetic_sign(monkeypatch):
    real_grid = G.grid
    calls = {"n": 0}

    def bad_adjoint(nu, rec, u, V1, V2, gnl, L, tau, j_lo, j_hi, dx):
        # same as the oracle's adjoint but with the forward (not conjugate) kinetic phase
        n = nu.shape[0]
        _, k, _ = real_grid(n, L)
        half = np.exp(-1j * tau * k ** 2 / 4)
        g = np.zeros(j_hi - j_lo)
        for j in range(j_hi - 1, j_lo - 1, -1):
            a, b, th = rec["a"][j], rec["b"][j], rec["theta"][j]
            nup = np.fft.ifft(half * np.fft.fft(nu))
            g[j - j_lo] = dx * float(np.sum(G.dpotential(V1, V2, u[j]) * np.imag(np.conj(nup) * b)))
            w = np.exp(1j * th) * nup
            mu = w + 2.0 * tau * gnl * np.imag(np.conj(w) * a) * a
            nu = np.fft.ifft(half * np.fft.fft(mu))
        return nu, g
    monkeypatch.setattr(G, "_adjoint_steps", bad_adjoint)
    assert _gpe_fd_error() > 1e-6


def test_mutation_inner_step_without_beta(monkeypatch):
    """An inner step that forgets the beta_n scale is no longer the plain step for ell = 1."""
    H0, Hc, psi0, tgt, u, T, al = _tiny()
    kw = dict(H0=H0, Hc=Hc, psi0=psi0, target=tgt, u0=u, T=T, alpha=al, rho=0.3, iters=3)
    plain = O.plain_gradient_method(**kw)
    ok = O.ism_iterate_inner(N=4, ell=1, **kw)
    assert np.max(np.abs(ok["u"] - plain["u"])) <= 1e-10
    orig = O.subproblem_gradient

    def unscaled(H0_, Hc_, v, al_, phi_n, phi_n1, sn, sn1, T_, step="exp"):
        return orig(H0_, Hc_, v, al_, phi_n, phi_n1, sn, sn1, T_, step) * (sn1 - sn) / v.shape[0]
    monkeypatch.setattr(O, "subproblem_gradient", unscaled)
    bad = O.ism_iterate_inner(N=4, ell=1, **kw)
    assert np.max(np.abs(bad["u"] - plain["u"])) > 1e-3


def test_mutation_density_one_sided_adjoint(monkeypatch):
    """An adjoint propagated as U^+ lambda (state rule) instead of U^+ lambda U is caught by
    the Liouville-space vectorisation pin."""
    from oracle import density as D
    rng = np.random.default_rng(4)
    d, K, T = 3, 8, 0.7
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)); H0 = A + A.conj().T
    B = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)); Hc = np.stack([B + B.conj().T])
    R0 = np.diag([1.0, -0.5, 0.2]).astype(complex); Rf = np.roll(R0, 1, axis=0) + np.roll(R0, 1, axis=0).T
    u = rng.uniform(-1, 1, size=(K, 1)); al = np.zeros(K)

    def lv(H):
        return np.kron(H, np.eye(d)) - np.kron(np.eye(d), H.T)

    def err():
        g, *_ = D.gradient(H0, Hc, R0, Rf, u, T, al)
        gv, *_ = O.gradient(lv(H0), np.stack([lv(Hc[0])]), R0.reshape(-1), Rf.reshape(-1), u, T, al)
        return np.max(np.abs(g - gv))
    assert err() <= 1e-11

    def one_sided(Us, target):
        out = [None] * (len(Us) + 1)
        out[-1] = np.array(target, dtype=np.complex128)
        for j in range(len(Us) - 1, -1, -1):
            out[j] = Us[j].conj().T @ out[j + 1]
        return out
    monkeypatch.setattr(D, "backward", one_sided)
    assert err() > 1e-3
