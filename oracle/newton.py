"""Oracle, Newton slice solver (TEST INFRASTRUCTURE ONLY: imported by tests/, never by the
library).

Sec. 4.B runs Algorithm 1 with Step (c) done by one iteration of Newton's method on every
slice problem  max_{u_n} J_n[u_n, phi^(k)],  matrix-free, the Newton system being solved by
GMRES.  The paper prints no further detail; the readings taken here:

  * the Newton system of slice n is  A_n delta_n = -G_n,  G_n = beta_n grad J_n[u_n, phi^(k)]
    the slice gradient (finite.subproblem_gradient, the quantity the library's slice kernels
    compute) and A_n its Jacobian with respect to u_n (a constant factor such as beta_n or
    1/tau changes neither the system's solution nor GMRES's iterates);
  * A_n v by the central difference of slice gradients,
        A_n v ~ (G_n(u_n + eps v) - G_n(u_n - eps v)) / (2 eps),   ||v|| = 1,
    with phi^(k) held (the matrix-free form);
  * GMRES from delta_n = 0 in the Euclidean inner product over the slice's (step, control)
    entries: m Arnoldi steps with modified Gram-Schmidt, no restart, ending early only at a
    breakdown (h_{i+1,i} <= 1e-14 ||A v_i||), then the (i+1) x i least-squares problem;
  * the full Newton step u_n <- u_n + delta_n, no damping or line search (the paper reports
    the method failing to converge for N = 1 and 2, which an undamped step explains).

Pins (tests/test_oracle_newton.py): GMRES at m = dim equals a direct solve of the assembled
difference Jacobian; the difference Jacobian is symmetric and agrees with second differences
of the slice functional itself; the Newton step converges quadratically near a maximum of a
slice problem; with N = 1 the slice problem is the whole problem (phi_0 = psi0,
phi_1 = psi_f).
"""
from __future__ import annotations

import numpy as np

from . import finite as _F

__all__ = ["slice_hvp", "gmres", "newton_slice_step", "ism_newton_iterate"]


def slice_hvp(grad_fn, un, v, eps):
    """(G(u_n + eps v) - G(u_n - eps v)) / (2 eps): the Jacobian of the slice gradient applied
    to v (matrix-free, central difference)."""
    return (grad_fn(un + eps * v) - grad_fn(un - eps * v)) / (2.0 * eps)


def gmres(apply_a, b, m):
    """m steps of GMRES for A x = b from x = 0 (Arnoldi with modified Gram-Schmidt, no
    restart; a breakdown ends it early).  b and the iterates are flat vectors."""
    n = b.size
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros(n)
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    V[0] = b / beta
    k = m
    for i in range(m):
        w = apply_a(V[i])
        wn = float(np.linalg.norm(w))
        for l in range(i + 1):
            H[l, i] = float(np.dot(V[l], w))
            w = w - H[l, i] * V[l]
        H[i + 1, i] = float(np.linalg.norm(w))
        if H[i + 1, i] <= 1e-14 * wn:
            k = i + 1
            break
        V[i + 1] = w / H[i + 1, i]
    e1 = np.zeros(k + 1)
    e1[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
    return V[:k].T @ y


def newton_slice_step(H0, Hc, u, alpha, phi_n, phi_n1, sn, sn1, T, m, eps, step="exp"):
    """delta_n of one Newton step on slice n (controls u of the whole interval, the slice's
    entries u[sn:sn1] varied)."""
    shape = u[sn:sn1].shape

    def grad_fn(flat):
        w = np.array(u, copy=True)
        w[sn:sn1] = flat.reshape(shape)
        return _F.subproblem_gradient(H0, Hc, w, alpha, phi_n, phi_n1, sn, sn1, T, step).ravel()

    un = u[sn:sn1].ravel()
    g = grad_fn(un)
    delta = gmres(lambda v: slice_hvp(grad_fn, un, v, eps), -g, m)
    return delta.reshape(shape)


def ism_newton_iterate(H0, Hc, psi0, target, u0, T, alpha, iters, N, m, eps=1e-5,
                       step="exp"):
    """Algorithm 1 with Step (c) = one Newton-GMRES step per slice problem (Sec. 4.B).

    Iteration k: boundaries and intermediate states phi^(k) at u^(k) (steps (a)-(b)); every
    slice takes its Newton step with phi^(k) held (steps (c)-(d)).  Returns {"u", "J", "F"}
    with J^(k), F^(k) at u^(k) for every iteration."""
    u = np.array(u0, dtype=np.float64, copy=True)
    K = u.shape[0]
    tau = T / K
    s = _F.slice_starts(K, N)
    maps = _F.step_unitaries_cn if step == "cn" else _F.step_unitaries
    Js, Fs = [], []
    for _ in range(iters):
        Psi, Lam = _F.boundaries(_F.assemble(maps(H0, Hc, u, tau), s), psi0, target)
        phi = _F.intermediate_states(Psi, Lam, s, K)
        J, F = _F.objective(Psi[-1], target, u, alpha, tau)
        Js.append(J); Fs.append(F)
        deltas = [newton_slice_step(H0, Hc, u, alpha, phi[n], phi[n + 1], s[n], s[n + 1], T,
                                    m, eps, step) for n in range(N)]
        for n in range(N):
            u[s[n]:s[n + 1]] += deltas[n]
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}
