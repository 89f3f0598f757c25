"""Oracle, 1-D Gross-Pitaevskii problem (TEST INFRASTRUCTURE ONLY).

Model (Sec. 4.C, with the equation's missing factor i restored and the density
written |psi|^2):  i d/dt psi = (-1/2 d_xx + V(x,u) + g |psi|^2) psi  on a periodic
grid x_m = -L/2 + m dx, dx = L/n, and V(x,u) = V0(x) + u V1(x) + u^2 V2.

Step map: Strang splitting (Eq. (OS)) with the kinetic half steps done exactly in
Fourier space (e^{-i tau k^2/4}; each half step F^-1 e^{-i tau k^2/4} F is evaluated in
extended precision and rounded once to FP64) and the potential-plus-density phase in real
space:
    a       = F^-1 e^{-i tau k^2/4} F psi_j
    theta_m = tau (V(x_m,u_j) + g |a_m|^2)
    b       = e^{-i theta} a
    psi_{j+1} = F^-1 e^{-i tau k^2/4} F b
Objective J = Re<psi_K|psi_f> with <a|b> = dx sum conj(a) b, alpha = 0 (Sec. 4.C).

Exact discrete adjoint (the splitting is exactly differentiable for a scalar
control, Sec. 3), for the real inner product Re<.|.>: nu_K = psi_f and, for
j = K-1..0,
    nu'  = F^-1 e^{+i tau k^2/4} F nu_{j+1}
    g_j  = dx sum_m dV/du(x_m,u_j) Im(conj(nu'_m) b_m)      (= (1/tau) dJ/du_j)
    w    = e^{+i theta} nu'
    mu   = w + 2 tau g Im(conj(w) a) a
    nu_j = F^-1 e^{+i tau k^2/4} F mu
(mu is the real-linear adjoint of a -> e^{-i tau (V + g|a|^2)} a).

BEC variant of ISM (Sec. 4.C): the slice start states are psi(t_n) taken on the
forward trajectory and the slice targets are taken on the adjoint trajectory,
J_n = Re<psi_n(t_{n+1})|nu(t_{n+1})>; the boundary sequences are produced by one
sequential forward and one sequential adjoint sweep (propagator assembling is
not defined for a nonlinear map), so each slice gradient equals the plain
gradient on that slice by the chain rule (weight 1, no beta_n).

Several gradient steps per slice (Algorithm 1 step (c), Eq. (gradStep) iterated ell times on
max J_n with psi(t_n) and nu(t_{n+1}) held fixed): u_n <- u_n + rho grad J_n, ell times;
Err = sum_n tau sum_{j in slice n} |grad J_n[u^(k+1)]_j| (Algorithm 1 step (e)).

Pins (tests/test_oracle_gpe.py, tests/test_oracle_inner.py): g=0 ground state is the harmonic-oscillator
Gaussian, norm conservation, Ehrenfest leapfrog identities per step, adjoint
gradient vs central finite differences, ISM == plain, slice-problem gradient and Err vs
central finite differences of J_n, ell = 1 == plain, N = 1 with ell steps == plain.  No
function here is parity-unpinned.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as _sfft

__all__ = ["grid", "potential", "dpotential", "strang_forward", "adjoint_gradient",
           "objective", "plain_gradient_method", "ism_bec_gradient", "ism_bec_iterate",
           "bec_subproblem_objective", "bec_subproblem_gradient", "ism_bec_iterate_inner"]


def grid(n, L):
    dx = L / n
    x = -L / 2 + dx * np.arange(n)
    k = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    return x, k, dx


def _kinetic(f, tau, k, sign=-1):
    """Kinetic half step F^-1 diag(e^{sign i tau k^2/4}) F f (sign = -1 forward, +1 in the
    adjoint), evaluated in extended precision (numpy.longdouble, 64-bit significand) from the
    FP64 tau and k and rounded once to FP64.  In FP64 both the FFT's rounding (fixed by its
    twiddle factors) and the rounding of the factor e^{-i tau k^2/4} are the same at every half
    step, so they add up coherently: over the 2 x 10^4 half steps of a condensate trajectory
    (n = 4096, K = 10000) an FP64 evaluation drifts 1.9e-11 from the exact result."""
    kl = np.asarray(k).astype(np.longdouble)
    fac = np.exp(sign * 1j * np.longdouble(tau) * kl * kl / 4)
    out = _sfft.ifft(fac * _sfft.fft(np.asarray(f).astype(np.clongdouble)))
    return out.astype(np.complex128)


def potential(V0, V1, V2, u):
    return V0 + u * V1 + (u * u) * V2


def dpotential(V1, V2, u):
    """dV/du = V1 + 2 u V2."""
    return V1 + 2.0 * u * V2


def _strang_step(psi, k, V, gnl, tau):
    a = _kinetic(psi, tau, k)
    theta = tau * (V + gnl * np.abs(a) ** 2)
    b = np.exp(-1j * theta) * a
    nxt = _kinetic(b, tau, k)
    return nxt, a, b, theta


def strang_forward(psi0, u, V0, V1, V2, gnl, L, tau, keep=True):
    """Forward Strang sweep.  Returns psi_K and (if keep) lists of psi_j, a_j, b_j, theta_j."""
    n = psi0.shape[0]
    _, k, _ = grid(n, L)
    psi = np.array(psi0, dtype=np.complex128)
    rec = {"psi": [psi], "a": [], "b": [], "theta": []}
    for j in range(u.shape[0]):
        psi, a, b, th = _strang_step(psi, k, potential(V0, V1, V2, u[j]), gnl, tau)
        if keep:
            rec["psi"].append(psi); rec["a"].append(a); rec["b"].append(b); rec["theta"].append(th)
    return psi, rec


def objective(psiK, target, dx):
    z = dx * np.vdot(psiK, target)
    return float(z.real), float(abs(z) ** 2)


def _adjoint_steps(nu, rec, u, V1, V2, gnl, L, tau, j_lo, j_hi, dx):
    """Run the exact adjoint from nu (at step j_hi) down to j_lo; returns (nu_{j_lo}, g[j_lo:j_hi])."""
    n = nu.shape[0]
    _, k, _ = grid(n, L)
    g = np.zeros(j_hi - j_lo)
    for j in range(j_hi - 1, j_lo - 1, -1):
        a, b, th = rec["a"][j], rec["b"][j], rec["theta"][j]
        nup = _kinetic(nu, tau, k, +1)
        g[j - j_lo] = dx * float(np.sum(dpotential(V1, V2, u[j]) * np.imag(np.conj(nup) * b)))
        w = np.exp(1j * th) * nup
        mu = w + 2.0 * tau * gnl * np.imag(np.conj(w) * a) * a
        nu = _kinetic(mu, tau, k, +1)
    return nu, g


def adjoint_gradient(psi0, target, u, V0, V1, V2, gnl, L, T):
    """Plain gradient: forward sweep, exact adjoint sweep.  u has shape (K,).
    Returns (g[K], J, F, psi_K)."""
    K = u.shape[0]
    tau = T / K
    n = psi0.shape[0]
    dx = L / n
    psiK, rec = strang_forward(psi0, u, V0, V1, V2, gnl, L, tau)
    _, g = _adjoint_steps(np.array(target, dtype=np.complex128), rec, u, V1, V2, gnl, L, tau, 0, K, dx)
    J, F = objective(psiK, target, dx)
    return g, J, F, psiK


def plain_gradient_method(psi0, target, u0, V0, V1, V2, gnl, L, T, rho, iters):
    u = np.array(u0, dtype=np.float64, copy=True)
    Js, Fs = [], []
    for _ in range(iters):
        g, J, F, _ = adjoint_gradient(psi0, target, u, V0, V1, V2, gnl, L, T)
        Js.append(J); Fs.append(F)
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}


def ism_bec_gradient(psi0, target, u, V0, V1, V2, gnl, L, T, N):
    """BEC-variant ISM gradient (Sec. 4.C).

    Boundaries: psi(t_n) from a sequential forward sweep and nu(t_n) from a sequential
    adjoint sweep.  Then, per slice n independently: forward from psi(t_n) over the slice,
    adjoint from nu(t_{n+1}) back over the slice, gradient on the slice."""
    K = u.shape[0]
    tau = T / K
    n = psi0.shape[0]
    dx = L / n
    s = np.array([(i * K) // N for i in range(N + 1)])
    psiK, rec = strang_forward(psi0, u, V0, V1, V2, gnl, L, tau)
    psi_b = [rec["psi"][s[i]] for i in range(N + 1)]
    # sequential adjoint sweep, recording nu at the slice boundaries
    nu_b = [None] * (N + 1)
    nu = np.array(target, dtype=np.complex128)
    nu_b[N] = nu
    for i in range(N - 1, -1, -1):
        nu, _ = _adjoint_steps(nu, rec, u, V1, V2, gnl, L, tau, s[i], s[i + 1], dx)
        nu_b[i] = nu
    g = np.zeros(K)
    for i in range(N):
        _, srec = strang_forward(psi_b[i], u[s[i]:s[i + 1]], V0, V1, V2, gnl, L, tau)
        _, gi = _adjoint_steps(nu_b[i + 1], srec, u[s[i]:s[i + 1]], V1, V2, gnl, L, tau,
                               0, s[i + 1] - s[i], dx)
        g[s[i]:s[i + 1]] = gi
    J, F = objective(psiK, target, dx)
    return g, J, F, psi_b, nu_b


def ism_bec_iterate(psi0, target, u0, V0, V1, V2, gnl, L, T, rho, iters, N):
    u = np.array(u0, dtype=np.float64, copy=True)
    Js, Fs = [], []
    for _ in range(iters):
        g, J, F, _, _ = ism_bec_gradient(psi0, target, u, V0, V1, V2, gnl, L, T, N)
        Js.append(J); Fs.append(F)
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}


def bec_subproblem_objective(psi_n, nu_n1, u_slice, V0, V1, V2, gnl, L, tau):
    """BEC slice functional (Sec. 4.C): J_n = Re<psi_n(t_{n+1})|nu(t_{n+1})>, psi_n propagated
    from psi(t_n) = psi_n under the slice controls u_slice."""
    dx = L / psi_n.shape[0]
    end, _ = strang_forward(psi_n, u_slice, V0, V1, V2, gnl, L, tau, keep=False)
    return float((dx * np.vdot(end, nu_n1)).real)


def bec_subproblem_gradient(psi_n, nu_n1, u_slice, V0, V1, V2, gnl, L, tau):
    """(1/tau) dJ_n/du_j on the slice: forward from psi(t_n), exact adjoint from nu(t_{n+1})."""
    dx = L / psi_n.shape[0]
    _, rec = strang_forward(psi_n, u_slice, V0, V1, V2, gnl, L, tau)
    _, g = _adjoint_steps(np.array(nu_n1, dtype=np.complex128), rec, u_slice, V1, V2, gnl, L,
                          tau, 0, u_slice.shape[0], dx)
    return g


def ism_bec_iterate_inner(psi0, target, u0, V0, V1, V2, gnl, L, T, rho, iters, N, ell,
                          eta=0.0):
    """BEC-variant ISM with ell gradient steps per slice problem and the Err rule.

    Iteration k: sequential sweeps give psi(t_n) and nu(t_n) at u^(k); each slice takes ell
    steps u_n <- u_n + rho grad J_n; Err^(k) = sum_n tau sum_j |grad J_n[u^(k+1)]_j|.  The
    loop stops after the iteration whose Err is <= eta (eta <= 0: never).  Returns
    {"u", "J", "F", "Err", "iters"} as the finite-dimensional version."""
    u = np.array(u0, dtype=np.float64, copy=True)
    K = u.shape[0]
    tau = T / K
    Js, Fs, Errs = [], [], []
    for _ in range(iters):
        _, J, F, psi_b, nu_b = ism_bec_gradient(psi0, target, u, V0, V1, V2, gnl, L, T, N)
        Js.append(J); Fs.append(F)
        s = [(i * K) // N for i in range(N + 1)]
        err = 0.0
        for i in range(N):
            a, b = s[i], s[i + 1]
            for _l in range(ell):
                g = bec_subproblem_gradient(psi_b[i], nu_b[i + 1], u[a:b], V0, V1, V2, gnl, L, tau)
                u[a:b] = u[a:b] + rho * g
            g = bec_subproblem_gradient(psi_b[i], nu_b[i + 1], u[a:b], V0, V1, V2, gnl, L, tau)
            err += tau * float(np.sum(np.abs(g)))
        Errs.append(err)
        if eta > 0 and err <= eta:
            break
    return {"u": u, "J": np.array(Js), "F": np.array(Fs), "Err": np.array(Errs),
            "iters": len(Errs)}
