"""Oracle, density-matrix (Liouville-von Neumann) problems (TEST INFRASTRUCTURE ONLY).

The five-spin experiment of Sec. 4.A moves to the density-matrix formalism: the state is a
Hermitian operator rho, evolving as i d/dt rho = [H(u), rho].  With the controls constant on
each step, one step is the conjugation

    rho_{j+1} = U_j rho_j U_j^dagger,   U_j = exp(-i tau H(u_j)),

which is exactly the exponential of the Liouvillian superoperator (no splitting error).
Inner product: the Hilbert-Schmidt form <A|B> = Tr(A^dagger B).

* objective J_tau = Re<rho_K|rho_f> - tau/2 sum_j alpha_j |u_j|^2, and the normalised
  fidelity F = |<rho_K|rho_f>|^2 / (<rho_0|rho_0><rho_f|rho_f>)
* adjoint   lambda_K = rho_f, lambda_j = U_j^dagger lambda_{j+1} U_j
* gradient  g_{j,c} = (1/tau) dJ_tau/du_{j,c} = Im Tr(Hhat_{c,j} [rho_j, lambda_j]) - alpha_j u_{j,c}
  (Hhat the step average of H_c, dU_j/du_c = -i tau U_j Hhat_{c,j})
* ISM (Algorithm 1): slice propagators W_n = U_{s_{n+1}-1} ... U_{s_n}; boundaries
  Psi_{n+1} = W_n Psi_n W_n^dagger, Lambda_n = W_n^dagger Lambda_{n+1} W_n; intermediate
  states phi_n = (1 - t_n/T) Psi_n + (t_n/T) Lambda_n (Eq. (cible)); per slice the forward
  trajectory from phi_n, the adjoint from phi_{n+1} and beta_n times the slice gradient
  (Theorem 2).

Pins (tests/test_oracle_density.py): the Liouville-space vectorisation (a state problem of
dimension d^2 with the superoperators H (x) I - I (x) H^T, run through the state oracle),
central finite differences of J_tau with scipy's expm, ISM == plain, product-operator closed
forms of the free evolution under the five-spin coupling topology, conservation of Tr(rho^2).
No function here is parity-unpinned.
"""
from __future__ import annotations

import numpy as np

from . import finite as _F

__all__ = ["inner_hs", "forward", "backward", "objective", "gradient", "plain_gradient_method",
           "assemble", "boundaries", "ism_gradient", "ism_iterate", "forward_cn", "backward_cn",
           "gradient_cn", "objective_cn", "ism_gradient_cn", "plain_gradient_method_cn",
           "ism_iterate_cn"]


def inner_hs(a: np.ndarray, b: np.ndarray) -> complex:
    """<A|B> = Tr(A^dagger B)."""
    return complex(np.vdot(a, b))


def forward(Us, rho0):
    """rho_0 = rho0, rho_{j+1} = U_j rho_j U_j^dagger; returns rho_0..rho_K."""
    out = [np.array(rho0, dtype=np.complex128)]
    for U in Us:
        out.append(U @ out[-1] @ U.conj().T)
    return out


def backward(Us, target):
    """lambda_K = rho_f, lambda_j = U_j^dagger lambda_{j+1} U_j; returns lambda_0..lambda_K."""
    out = [None] * (len(Us) + 1)
    out[-1] = np.array(target, dtype=np.complex128)
    for j in range(len(Us) - 1, -1, -1):
        out[j] = Us[j].conj().T @ out[j + 1] @ Us[j]
    return out


def objective(rhoK, rho0, target, u, alpha, tau):
    z = inner_hs(rhoK, target)
    J = z.real - 0.5 * tau * float(np.sum(alpha[:, None] * u ** 2))
    F = abs(z) ** 2 / (inner_hs(rho0, rho0).real * inner_hs(target, target).real)
    return J, F


def _step_grad(Hhats_j, rho_j, lam_j):
    comm = rho_j @ lam_j - lam_j @ rho_j
    return np.array([np.trace(Hh @ comm).imag for Hh in Hhats_j])


def gradient(H0, Hc, rho0, target, u, T, alpha):
    """Exact (1/tau) dJ_tau/du of the conjugation step map, with J and F at u."""
    K = u.shape[0]
    tau = T / K
    Us = _F.step_unitaries(H0, Hc, u, tau)
    rho = forward(Us, rho0)
    lam = backward(Us, target)
    g = np.zeros_like(u)
    for j in range(K):
        Hh = _F.hhat(_F.hamiltonian(H0, Hc, u[j]), Hc, tau)
        g[j] = _step_grad(Hh, rho[j], lam[j]) - alpha[j] * u[j]
    J, F = objective(rho[-1], rho0, target, u, alpha, tau)
    return g, J, F, rho[-1]


def plain_gradient_method(H0, Hc, rho0, target, u0, T, alpha, rho, iters):
    """Constant-step gradient ascent u <- u + rho g (Eq. (gradStep))."""
    u = np.array(u0, dtype=np.float64, copy=True)
    Js, Fs = [], []
    for _ in range(iters):
        g, J, F, _ = gradient(H0, Hc, rho0, target, u, T, alpha)
        Js.append(J); Fs.append(F)
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}


def assemble(Us, s):
    """Hilbert-space slice propagators W_n = U_{s_{n+1}-1} ... U_{s_n}: the slice map of the
    density matrix is rho -> W_n rho W_n^dagger (propagator assembling, Sec. 3)."""
    return _F.assemble(Us, s)


def boundaries(Ws, rho0, target):
    """Psi_0 = rho0, Psi_{n+1} = W_n Psi_n W_n^dagger; Lambda_N = rho_f,
    Lambda_n = W_n^dagger Lambda_{n+1} W_n."""
    N = len(Ws)
    Psi = [np.array(rho0, dtype=np.complex128)]
    for n in range(N):
        Psi.append(Ws[n] @ Psi[-1] @ Ws[n].conj().T)
    Lam = [None] * (N + 1)
    Lam[N] = np.array(target, dtype=np.complex128)
    for n in range(N - 1, -1, -1):
        Lam[n] = Ws[n].conj().T @ Lam[n + 1] @ Ws[n]
    return Psi, Lam


def ism_gradient(H0, Hc, rho0, target, u, T, alpha, N):
    """ISM gradient (Algorithm 1 steps (a)-(c)) in the density-matrix formalism.
    Returns (g[K, C], J, F, phi, Psi, Lam)."""
    K = u.shape[0]
    tau = T / K
    s = _F.slice_starts(K, N)
    Us = _F.step_unitaries(H0, Hc, u, tau)
    Psi, Lam = boundaries(assemble(Us, s), rho0, target)
    phi = _F.intermediate_states(Psi, Lam, s, K)
    g = np.zeros_like(u)
    for n in range(N):
        sn, sn1 = s[n], s[n + 1]
        beta = K / (sn1 - sn)
        rho = forward(Us[sn:sn1], phi[n])
        lam = backward(Us[sn:sn1], phi[n + 1])
        for j in range(sn, sn1):
            Hh = _F.hhat(_F.hamiltonian(H0, Hc, u[j]), Hc, tau)
            gj = _step_grad(Hh, rho[j - sn], lam[j - sn])
            g[j] = beta * (gj - (alpha[j] / beta) * u[j])
    J, F = objective(Psi[-1], rho0, target, u, alpha, tau)
    return g, J, F, phi, Psi, Lam


def ism_iterate(H0, Hc, rho0, target, u0, T, alpha, rho, iters, N):
    """ISM with one constant-step gradient step per slice (Algorithm 1)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    Js, Fs = [], []
    for _ in range(iters):
        g, J, F, *_ = ism_gradient(H0, Hc, rho0, target, u, T, alpha, N)
        Js.append(J); Fs.append(F)
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}


# ----------------------------------------------------------------------------
# Crank-Nicolson step map on the density matrix (Sec. 3 applied to the conjugation form):
# rho_{j+1} = U_j rho_j U_j^dagger with U_j = (I + L_j)^{-1} (I - L_j), L_j = (i tau/2) H_j,
# the Hilbert-space Cayley step of the paper's finite-dimensional scheme.
# ----------------------------------------------------------------------------

def _cn_difference(H, tau):
    """D_j = U_j - I = -2 (I + L_j)^{-1} L_j for the Cayley step U_j = (I + L_j)^{-1}(I - L_j).

    The same map as U_j, written without forming I + D_j: at tau ||H|| ~ 3e-3 the entries of
    U_j near 1 carry a rounding of about 1e-16 that is nearly the same at every step, and
    conjugating by the rounded U_j drifted coherently over the 2^15 steps of the five-spin run
    (1.8e-12 on rho(T)).  Over the first 1024 steps, against an extended-precision evaluation,
    the D_j form stays within 1.8e-15 and the U_j form drifts to 6.4e-14."""
    L = _F.cn_generator(H, tau)
    I = np.eye(L.shape[0], dtype=np.complex128)
    return -2.0 * np.linalg.solve(I + L, L)


def _conj_diff(Dm, x):
    """(I + D) x (I + D)^dagger = x + (D x + x D^dagger) + D x D^dagger."""
    Dh = Dm.conj().T
    return x + (Dm @ x + x @ Dh) + Dm @ x @ Dh


def _cn_differences(H0, Hc, u, tau):
    return [_cn_difference(_F.hamiltonian(H0, Hc, u[j]), tau) for j in range(u.shape[0])]


def forward_cn(Ds, rho0):
    """rho_{j+1} = U_j rho_j U_j^dagger with U_j = I + D_j; returns rho_0..rho_K."""
    out = [np.array(rho0, dtype=np.complex128)]
    for Dm in Ds:
        out.append(_conj_diff(Dm, out[-1]))
    return out


def backward_cn(Ds, target):
    """lambda_K = rho_f, lambda_j = U_j^dagger lambda_{j+1} U_j with U_j = I + D_j."""
    out = [None] * (len(Ds) + 1)
    out[-1] = np.array(target, dtype=np.complex128)
    for j in range(len(Ds) - 1, -1, -1):
        out[j] = _conj_diff(Ds[j].conj().T, out[j + 1])
    return out


def _cn_step_grad(H, Hc, tau, rho_j, lam_j):
    """(1/tau) dJ/du_{j,c} of one Crank-Nicolson conjugation step, without the penalty:
        g_{j,c} = 2 Im Tr( lambda_j (I - L_j)^{-1} H_c (I + L_j)^{-1} rho_j ).
    From dU/du_c = -(i tau/2) (I+L)^{-1} H_c (I + U): dJ = 2 Re Tr(lambda_{j+1} dU rho_j U^+),
    U^+ lambda_{j+1} = lambda_j U^+, U^+ (I+L)^{-1} = (I-L)^{-1} and I + U = 2 (I+L)^{-1}."""
    L = _F.cn_generator(H, tau)
    I = np.eye(L.shape[0], dtype=np.complex128)
    a = np.linalg.solve(I + L, rho_j)                     # (I + L)^{-1} rho_j
    b = np.linalg.solve((I - L).conj().T, lam_j.conj().T).conj().T   # lambda_j (I - L)^{-1}
    return np.array([2.0 * np.trace(b @ Hc[c] @ a).imag for c in range(Hc.shape[0])])


def gradient_cn(H0, Hc, rho0, target, u, T, alpha):
    """Exact (1/tau) dJ_tau/du of the Crank-Nicolson conjugation map, with J and F at u."""
    K = u.shape[0]
    tau = T / K
    Ds = _cn_differences(H0, Hc, u, tau)
    rho = forward_cn(Ds, rho0)
    lam = backward_cn(Ds, target)
    g = np.zeros_like(u)
    for j in range(K):
        H = _F.hamiltonian(H0, Hc, u[j])
        g[j] = _cn_step_grad(H, Hc, tau, rho[j], lam[j]) - alpha[j] * u[j]
    J, F = objective(rho[-1], rho0, target, u, alpha, tau)
    return g, J, F, rho[-1]


def objective_cn(H0, Hc, rho0, target, u, T, alpha):
    """J_tau and F of the Crank-Nicolson conjugation map at u."""
    K = u.shape[0]
    rhoK = forward_cn(_cn_differences(H0, Hc, u, T / K), rho0)[-1]
    return objective(rhoK, rho0, target, u, alpha, T / K)


def ism_gradient_cn(H0, Hc, rho0, target, u, T, alpha, N):
    """ISM gradient (Algorithm 1 steps (a)-(c)) with the Crank-Nicolson conjugation map:
    slice maps W_n from the Cayley steps, boundaries, intermediate states (Eq. (cible)), and
    per slice beta_n [ 2 Im Tr(lambda^n_j (I-L_j)^{-1} H_c (I+L_j)^{-1} rho^n_j)
    - alpha_{n,j} u_{j,c} ].  Returns (g, J, F, phi, Psi, Lam)."""
    K = u.shape[0]
    tau = T / K
    s = _F.slice_starts(K, N)
    Ds = _cn_differences(H0, Hc, u, tau)
    I = np.eye(Ds[0].shape[0], dtype=np.complex128)
    Psi, Lam = boundaries(assemble([I + Dm for Dm in Ds], s), rho0, target)
    phi = _F.intermediate_states(Psi, Lam, s, K)
    g = np.zeros_like(u)
    for n in range(N):
        sn, sn1 = s[n], s[n + 1]
        beta = K / (sn1 - sn)
        rho = forward_cn(Ds[sn:sn1], phi[n])
        lam = backward_cn(Ds[sn:sn1], phi[n + 1])
        for j in range(sn, sn1):
            H = _F.hamiltonian(H0, Hc, u[j])
            gj = _cn_step_grad(H, Hc, tau, rho[j - sn], lam[j - sn])
            g[j] = beta * (gj - (alpha[j] / beta) * u[j])
    J, F = objective(Psi[-1], rho0, target, u, alpha, tau)
    return g, J, F, phi, Psi, Lam


def plain_gradient_method_cn(H0, Hc, rho0, target, u0, T, alpha, rho, iters):
    """Constant-step gradient ascent (Eq. (gradStep)) with the Crank-Nicolson map."""
    u = np.array(u0, dtype=np.float64, copy=True)
    Js, Fs = [], []
    for _ in range(iters):
        g, J, F, _ = gradient_cn(H0, Hc, rho0, target, u, T, alpha)
        Js.append(J); Fs.append(F)
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}


def ism_iterate_cn(H0, Hc, rho0, target, u0, T, alpha, rho, iters, N):
    """ISM with one constant-step gradient step per slice (Algorithm 1), Crank-Nicolson map."""
    u = np.array(u0, dtype=np.float64, copy=True)
    Js, Fs = [], []
    for _ in range(iters):
        g, J, F, *_ = ism_gradient_cn(H0, Hc, rho0, target, u, T, alpha, N)
        Js.append(J); Fs.append(F)
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}
