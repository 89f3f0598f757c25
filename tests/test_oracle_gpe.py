"""Pins of the GPE oracle (Strang splitting, exact discrete adjoint, BEC-variant ISM)."""
import math

import numpy as np
import pytest

import problems
from oracle import gpe as G


def _gauss(x, x0, p0=0.0, w=1.0):
    psi = np.exp(-0.5 * ((x - x0) / w) ** 2 + 1j * p0 * x)
    return psi


def _normed(psi, dx):
    return psi / math.sqrt(dx * np.sum(np.abs(psi) ** 2))


# --- P15: g = 0 ground state is the oscillator Gaussian ---------------------------

def test_p15_ground_state_g0():
    n, L = 256, 20.0
    x, _, dx = G.grid(n, L)
    for x0 in (0.0, 1.5):
        gs = problems.gpe_ground_state(n, L, 0.0, x0, tol=1e-12)
        ref = math.pi ** -0.25 * np.exp(-0.5 * (x - x0) ** 2)
        assert np.max(np.abs(gs - ref)) <= 1e-6


# --- P16 / P17: Ehrenfest leapfrog and norm, per Strang step ---------------------

def _moments(psi, x, k, dx):
    nx = dx * np.sum(np.abs(psi) ** 2)
    mx = dx * np.sum(x * np.abs(psi) ** 2) / nx
    ph = np.fft.fft(psi)
    mp = np.sum(k * np.abs(ph) ** 2) / np.sum(np.abs(ph) ** 2)
    return nx, mx, mp


@pytest.mark.parametrize("gnl", [0.0, 10.0])
def test_p16_p17_ehrenfest_and_norm(gnl):
    n, L, tau, K = 1024, 40.0, 1e-3, 200
    x, k, dx = G.grid(n, L)
    psi0 = _normed(_gauss(x, 0.7, p0=0.3).astype(complex), dx)
    rng = np.random.default_rng(5)
    u = rng.uniform(-2, 2, size=K)
    V0, V1, V2 = 0.5 * x ** 2, -x, 0.5
    _, rec = G.strang_forward(psi0, u, V0, V1, V2, gnl, L, tau)
    n0, mx, mp = _moments(psi0, x, k, dx)
    for j in range(K):
        mx = mx + tau * mp / 2
        mp = mp - tau * (mx - u[j])
        mx = mx + tau * mp / 2
        nj, ax, ap = _moments(rec["psi"][j + 1], x, k, dx)
        assert abs(ax - mx) <= 1e-11 and abs(ap - mp) <= 1e-11
        assert abs(nj - n0) <= (j + 1) * 1e-15 + 1e-15


# --- P19: adjoint gradient vs central differences -------------------------------

@pytest.mark.parametrize("gnl", [0.0, 10.0])
def test_p19_gpe_gradient_fd(gnl):
    n, L, K, T = 64, 16.0, 20, 0.4
    x, _, dx = G.grid(n, L)
    psi0 = _normed(_gauss(x, -0.5).astype(complex), dx)
    tgt = _normed(_gauss(x, 1.0, p0=0.2).astype(complex), dx)
    rng = np.random.default_rng(6)
    u = rng.uniform(-1, 1, size=K)
    V0, V1, V2 = 0.5 * x ** 2, -x, 0.5
    g, J, F, _ = G.adjoint_gradient(psi0, tgt, u, V0, V1, V2, gnl, L, T)
    tau = T / K
    eps = 1e-5
    fd = np.zeros(K)
    for j in range(K):
        up = u.copy(); up[j] += eps
        um = u.copy(); um[j] -= eps
        Jp = G.adjoint_gradient(psi0, tgt, up, V0, V1, V2, gnl, L, T)[1]
        Jm = G.adjoint_gradient(psi0, tgt, um, V0, V1, V2, gnl, L, T)[1]
        fd[j] = (Jp - Jm) / (2 * eps)
    assert np.max(np.abs(tau * g - fd)) / np.max(np.abs(fd)) <= 1e-6


def test_p19_nonlinear_term_matters():
    """Guard for the FD pin: dropping the 2 tau g Im(conj(w) a) a term is detectable."""
    n, L, K, T, gnl = 64, 16.0, 20, 0.4, 10.0
    x, k, dx = G.grid(n, L)
    psi0 = _normed(_gauss(x, -0.5).astype(complex), dx)
    tgt = _normed(_gauss(x, 1.0, p0=0.2).astype(complex), dx)
    u = np.linspace(-1, 1, K)
    V0, V1, V2 = 0.5 * x ** 2, -x, 0.5
    g_full, *_ = G.adjoint_gradient(psi0, tgt, u, V0, V1, V2, gnl, L, T)
    g_lin_adj = G.adjoint_gradient(psi0, tgt, u, V0, V1, V2, 0.0, L, T)[0]
    assert np.max(np.abs(g_full - g_lin_adj)) > 1e-3 * np.max(np.abs(g_full))


# --- P18: BEC-variant ISM == plain -------------------------------------------

@pytest.mark.parametrize("N", [1, 4, 7])
def test_p18_ism_bec_equals_plain(N):
    n, L, K, T, gnl = 64, 16.0, 30, 0.6, 10.0
    x, _, dx = G.grid(n, L)
    psi0 = _normed(_gauss(x, 0.0).astype(complex), dx)
    tgt = _normed(_gauss(x, 1.0).astype(complex), dx)
    u = np.linspace(0, 1, K)
    V0, V1, V2 = 0.5 * x ** 2, -x, 0.5
    g, J, F, _ = G.adjoint_gradient(psi0, tgt, u, V0, V1, V2, gnl, L, T)
    gi, Ji, Fi, psi_b, nu_b = G.ism_bec_gradient(psi0, tgt, u, V0, V1, V2, gnl, L, T, N)
    assert np.max(np.abs(gi - g)) <= 1e-12 * max(1.0, np.max(np.abs(g)))
    assert Ji == J
    assert np.max(np.abs(psi_b[0] - psi0)) == 0 and np.max(np.abs(nu_b[N] - tgt)) == 0
