"""Pins of the oracle's multi-step slice solves and of the Err stopping rule (Algorithm 1
steps (c) and (e), Eq. (gradStep) iterated), against mathematics that does not go through
the oracle's own formulas: central finite differences of the slice functional J_n computed
with scipy's expm (or a dense linear solve for Crank-Nicolson), the plain gradient method,
and the reduction of the N = 1 slice problem to the original problem.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import problems
from oracle import finite as O
from oracle import gpe as G


def _tiny(seed=21, d=4, C=2, K=18, T=1.1, alpha=0.15):
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
    return H0, np.stack(Hc), psi0, tgt, u, T, np.full(K, alpha)


def _step(H, tau, step):
    if step == "cn":
        L = 0.5j * tau * H
        return np.linalg.solve(np.eye(H.shape[0]) + L, np.eye(H.shape[0]) - L)
    return sla.expm(-1j * tau * H)


def _Jn_direct(H0, Hc, u, al, phi_n, phi_n1, a, b, T, step):
    """J_n = Re<psi_n(t_{n+1})|phi_{n+1}> - alpha_n/2 tau sum |u_j|^2 by scipy propagation."""
    K = u.shape[0]
    tau = T / K
    beta = K / (b - a)
    psi = phi_n.copy()
    for j in range(a, b):
        H = H0 + np.einsum("c,cij->ij", u[j], Hc)
        psi = _step(H, tau, step) @ psi
    ov = np.vdot(psi, phi_n1) if psi.ndim == 1 else np.trace(psi.conj().T @ phi_n1) / psi.shape[0]
    return ov.real - 0.5 * tau * np.sum((al[a:b] / beta)[:, None] * u[a:b] ** 2)


def _phi(H0, Hc, psi0, tgt, u, T, N, step):
    K = u.shape[0]
    maps = O.step_unitaries_cn if step == "cn" else O.step_unitaries
    s = O.slice_starts(K, N)
    Psi, Lam = O.boundaries(O.assemble(maps(H0, Hc, u, T / K), s), psi0, tgt)
    return s, O.intermediate_states(Psi, Lam, s, K)


# --- slice-problem gradient vs central finite differences of J_n -------------------------

@pytest.mark.parametrize("step", ["exp", "cn"])
def test_subproblem_gradient_fd(step):
    H0, Hc, psi0, tgt, u, T, al = _tiny()
    N = 3
    s, phi = _phi(H0, Hc, psi0, tgt, u, T, N, step)
    # move the controls away from those that produced phi: the slice problem is solved at
    # controls other than u^(k) from the second inner step on
    v = u + 0.3 * np.random.default_rng(5).uniform(-1, 1, size=u.shape)
    K = u.shape[0]
    tau = T / K
    eps = 1e-5
    for n in range(N):
        a, b = s[n], s[n + 1]
        beta = K / (b - a)
        g = O.subproblem_gradient(H0, Hc, v, al, phi[n], phi[n + 1], a, b, T, step)
        assert np.allclose(O.subproblem_objective(H0, Hc, v, al, phi[n], phi[n + 1], a, b, T, step),
                           _Jn_direct(H0, Hc, v, al, phi[n], phi[n + 1], a, b, T, step), atol=1e-13)
        for j in range(a, b):
            for c in range(u.shape[1]):
                up = v.copy(); up[j, c] += eps
                um = v.copy(); um[j, c] -= eps
                fd = (_Jn_direct(H0, Hc, up, al, phi[n], phi[n + 1], a, b, T, step)
                      - _Jn_direct(H0, Hc, um, al, phi[n], phi[n + 1], a, b, T, step)) / (2 * eps)
                # g = beta_n grad J_n and grad J_n = (1/tau) dJ_n/du_j
                assert abs(tau * g[j - a, c] / beta - fd) <= 1e-9


def test_subproblem_gradient_fd_gate():
    rng = np.random.default_rng(8)
    d, K, T, N = 4, 12, 1.0, 3
    p = problems.spin2()
    W = problems.haar_unitary(d, rng)
    u = rng.uniform(-1, 1, size=(K, 2)); al = np.full(K, 0.05)
    s, phi = _phi(p.H0, p.Hc, np.eye(d, dtype=complex), W, u, T, N, "exp")
    v = u + 0.2 * rng.uniform(-1, 1, size=u.shape)
    eps, tau = 1e-5, T / K
    n = 1
    a, b = s[n], s[n + 1]
    g = O.subproblem_gradient(p.H0, p.Hc, v, al, phi[n], phi[n + 1], a, b, T)
    for j in range(a, b):
        for c in range(2):
            up = v.copy(); up[j, c] += eps
            um = v.copy(); um[j, c] -= eps
            fd = (_Jn_direct(p.H0, p.Hc, up, al, phi[n], phi[n + 1], a, b, T, "exp")
                  - _Jn_direct(p.H0, p.Hc, um, al, phi[n], phi[n + 1], a, b, T, "exp")) / (2 * eps)
            assert abs(tau * g[j - a, c] * (b - a) / K - fd) <= 1e-9


# --- ell = 1 is the plain gradient method (Theorem 2) ----------------------------------

@pytest.mark.parametrize("step", ["exp", "cn"])
@pytest.mark.parametrize("N", [2, 5])
def test_one_inner_step_equals_plain(step, N):
    p = problems.spin2(K=30)
    kw = dict(H0=p.H0, Hc=p.Hc, psi0=p.psi0, target=p.target, u0=p.u0[0], T=p.T,
              alpha=np.full(30, 0.1), rho=p.rho, iters=12)
    plain = (O.plain_gradient_method_cn if step == "cn" else O.plain_gradient_method)(**kw)
    r = O.ism_iterate_inner(N=N, ell=1, step=step, **kw)
    assert np.max(np.abs(r["u"] - plain["u"])) <= 1e-10
    assert np.max(np.abs(r["J"] - plain["J"])) <= 1e-10
    assert r["iters"] == 12


# --- N = 1: the slice problem is the original problem, so ell inner steps == ell plain steps

@pytest.mark.parametrize("step", ["exp", "cn"])
def test_single_slice_inner_steps_equal_plain(step):
    p = problems.spin2(K=24)
    al = np.full(24, 0.1)
    kw = dict(H0=p.H0, Hc=p.Hc, psi0=p.psi0, target=p.target, T=p.T, alpha=al, rho=p.rho)
    plain = (O.plain_gradient_method_cn if step == "cn" else O.plain_gradient_method)(
        u0=p.u0[0], iters=12, **kw)
    r = O.ism_iterate_inner(u0=p.u0[0], iters=4, N=1, ell=3, step=step, **kw)
    assert np.max(np.abs(r["u"] - plain["u"])) <= 1e-10
    # J^(k) of the outer loop is the plain method's J at iterations 0, 3, 6, 9
    assert np.max(np.abs(r["J"] - plain["J"][::3])) <= 1e-10


# --- Err against finite differences of J_n at u^(k+1) with the old phi ---------------------

@pytest.mark.parametrize("step", ["exp", "cn"])
def test_err_fd(step):
    H0, Hc, psi0, tgt, u, T, al = _tiny(seed=23, K=15)
    N, ell, rho = 3, 2, 0.4
    K = u.shape[0]
    tau = T / K
    r = O.ism_iterate_inner(H0, Hc, psi0, tgt, u, T, al, rho, 1, N, ell, step=step)
    s, phi = _phi(H0, Hc, psi0, tgt, u, T, N, step)
    v = r["u"]
    eps = 1e-6
    err = 0.0
    for n in range(N):
        a, b = s[n], s[n + 1]
        for j in range(a, b):
            gj = np.zeros(u.shape[1])
            for c in range(u.shape[1]):
                up = v.copy(); up[j, c] += eps
                um = v.copy(); um[j, c] -= eps
                gj[c] = (_Jn_direct(H0, Hc, up, al, phi[n], phi[n + 1], a, b, T, step)
                         - _Jn_direct(H0, Hc, um, al, phi[n], phi[n + 1], a, b, T, step)) / (2 * eps) / tau
            err += tau * math.sqrt(float(np.sum(gj ** 2)))
    assert abs(r["Err"][0] - err) <= 1e-7 * max(1.0, err)


def test_inner_steps_increase_slice_functional():
    """Small constant steps are ascent steps on every slice problem: J_n grows with ell."""
    H0, Hc, psi0, tgt, u, T, al = _tiny(seed=24, K=16)
    N = 4
    s, phi = _phi(H0, Hc, psi0, tgt, u, T, N, "exp")
    for ell in (1, 2, 3):
        prev = None
        r = O.ism_iterate_inner(H0, Hc, psi0, tgt, u, T, al, 0.05, 1, N, ell)
        vals = [_Jn_direct(H0, Hc, r["u"], al, phi[n], phi[n + 1], s[n], s[n + 1], T, "exp")
                for n in range(N)]
        base = [_Jn_direct(H0, Hc, u, al, phi[n], phi[n + 1], s[n], s[n + 1], T, "exp")
                for n in range(N)]
        assert all(v > b0 for v, b0 in zip(vals, base))
        if prev is not None:
            assert all(v > p0 for v, p0 in zip(vals, prev))
        prev = vals


def test_err_stop():
    """The loop stops after the first iteration whose Err is <= eta."""
    p = problems.spin2(K=20)
    kw = dict(H0=p.H0, Hc=p.Hc, psi0=p.psi0, target=p.target, u0=p.u0[0], T=p.T,
              alpha=np.zeros(20), rho=p.rho, N=4, ell=2)
    full = O.ism_iterate_inner(iters=10, **kw)
    eta = 0.5 * (full["Err"][3] + full["Err"][4])
    assert full["Err"][3] > eta >= full["Err"][4] or full["Err"][4] > eta >= full["Err"][3]
    first = int(np.argmax(full["Err"] <= eta))
    r = O.ism_iterate_inner(iters=10, eta=eta, **kw)
    assert r["iters"] == first + 1
    assert np.array_equal(r["Err"], full["Err"][:first + 1])


# --- GPE (BEC variant) --------------------------------------------------------------------

def _gpe_case(n=64, L=16.0, K=24, T=0.48, gnl=10.0):
    x, _, dx = G.grid(n, L)
    psi0 = np.exp(-0.5 * x ** 2).astype(complex)
    psi0 /= math.sqrt(dx * np.sum(np.abs(psi0) ** 2))
    tgt = np.exp(-0.5 * (x - 1.0) ** 2).astype(complex)
    tgt /= math.sqrt(dx * np.sum(np.abs(tgt) ** 2))
    u = np.linspace(0.0, 1.0, K)
    return psi0, tgt, u, 0.5 * x ** 2, -x, 0.5, gnl, L, T


def test_bec_subproblem_gradient_fd():
    psi0, tgt, u, V0, V1, V2, gnl, L, T = _gpe_case()
    N = 3
    K = u.shape[0]
    tau = T / K
    _, _, _, psi_b, nu_b = G.ism_bec_gradient(psi0, tgt, u, V0, V1, V2, gnl, L, T, N)
    s = [(i * K) // N for i in range(N + 1)]
    v = u + 0.2 * np.sin(np.arange(K))
    eps = 1e-6
    n = 1
    a, b = s[n], s[n + 1]
    g = G.bec_subproblem_gradient(psi_b[n], nu_b[n + 1], v[a:b], V0, V1, V2, gnl, L, tau)
    for j in range(b - a):
        up = v[a:b].copy(); up[j] += eps
        um = v[a:b].copy(); um[j] -= eps
        fd = (G.bec_subproblem_objective(psi_b[n], nu_b[n + 1], up, V0, V1, V2, gnl, L, tau)
              - G.bec_subproblem_objective(psi_b[n], nu_b[n + 1], um, V0, V1, V2, gnl, L, tau)) / (2 * eps)
        assert abs(tau * g[j] - fd) <= 1e-8


def test_bec_inner_equals_plain_cases():
    psi0, tgt, u, V0, V1, V2, gnl, L, T = _gpe_case()
    kw = dict(psi0=psi0, target=tgt, V0=V0, V1=V1, V2=V2, gnl=gnl, L=L, T=T, rho=0.5)
    plain = G.plain_gradient_method(u0=u, iters=6, **kw)
    one = G.ism_bec_iterate_inner(u0=u, iters=6, N=4, ell=1, **kw)
    assert np.max(np.abs(one["u"] - plain["u"])) <= 1e-10
    single = G.ism_bec_iterate_inner(u0=u, iters=2, N=1, ell=3, **kw)
    assert np.max(np.abs(single["u"] - plain["u"])) <= 1e-10
    assert np.max(np.abs(single["J"] - plain["J"][::3])) <= 1e-10


def test_bec_err_fd():
    psi0, tgt, u, V0, V1, V2, gnl, L, T = _gpe_case(K=12, T=0.24)
    N, K = 3, 12
    tau = T / K
    r = G.ism_bec_iterate_inner(psi0, tgt, u, V0, V1, V2, gnl, L, T, 0.5, 1, N, 2)
    _, _, _, psi_b, nu_b = G.ism_bec_gradient(psi0, tgt, u, V0, V1, V2, gnl, L, T, N)
    s = [(i * K) // N for i in range(N + 1)]
    v = r["u"]
    eps = 1e-6
    err = 0.0
    for n in range(N):
        a, b = s[n], s[n + 1]
        for j in range(b - a):
            up = v[a:b].copy(); up[j] += eps
            um = v[a:b].copy(); um[j] -= eps
            fd = (G.bec_subproblem_objective(psi_b[n], nu_b[n + 1], up, V0, V1, V2, gnl, L, tau)
                  - G.bec_subproblem_objective(psi_b[n], nu_b[n + 1], um, V0, V1, V2, gnl, L, tau)) / (2 * eps)
            err += abs(fd)
    assert abs(r["Err"][0] - err) <= 1e-6 * max(1.0, err)
