"""Oracle, frozen-density propagator assembling for the condensate (TEST INFRASTRUCTURE ONLY:
imported by tests/, never by the library).

Sec. 4.C builds the BEC variant's boundary sequences psi(t_n) (forward trajectory) and
nu(t_n) (adjoint trajectory) by the propagator assembling of Sec. 3, which a nonlinear step
map does not define.  Reading taken: the nonlinearity is frozen at the previous iteration.

  * Forward.  With the density of the intermediate state a_j frozen, one Strang step
        S_j psi = Kh e^{-i theta_j} Kh psi,   theta_j = tau (V(x, u_j) + g |a_j|^2),
    Kh = F^-1 e^{-i tau k^2/4} F, is linear and unitary, so slice propagators
    M_n = S_{s_{n+1}-1} ... S_{s_n} (n x n complex) exist.
  * Adjoint.  The exact discrete adjoint step (oracle/gpe.py), linearised at the frozen a_j,
        R_j nu = Kh^+ [w + 2 tau g Im(conj(w) a_j) a_j],   w = e^{+i theta_j} Kh^+ nu,
    is real-linear; the slice map A_n = R_{s_n} ... R_{s_{n+1}-1} is kept as its images of
    the 2n real basis vectors e_m and i e_m, and applied to nu by real weights:
    A_n nu = sum_m Re(nu_m) A_n(e_m) + Im(nu_m) A_n(i e_m).
  * Boundaries: Psi_0 = psi0, Psi_{n+1} = M_n Psi_n; Lambda_N = psi_f, Lambda_n = A_n Lambda_{n+1}.
  * Iteration k (lagged ISM): (a)-(b) the boundaries above with the maps at u^(k) and the
    a_j of iteration k-1's slice trajectories (iteration 0: one exact sequential forward and
    adjoint sweep at u^(0), as in the exact BEC variant); J^(k), F^(k) from Psi_N;
    (c)-(d) every slice solves its BEC slice problem from Psi_n with target Lambda_{n+1}
    exactly (nonlinear forward, exact adjoint, u_n <- u_n + rho grad J_n), and its forward
    trajectory (at u^(k)) supplies the a_j frozen for iteration k+1.
At a fixed point the slice trajectories start on the exact trajectory, so the frozen maps
are the exact ones and the lagged iteration has the plain method's fixed points; before
that its iterates differ from the plain method's, which the exact BEC variant does not.

Pins (tests/test_oracle_gpe_frozen.py): S_j and R_j at the exact trajectory's a_j reproduce
the exact forward and adjoint steps; with the exact trajectory's a_j the assembled
boundaries equal the sequential sweeps'; M_n is unitary and A_n is the real transpose of
the linearised forward slice map; the lagged iteration approaches the plain method's limit.
"""
from __future__ import annotations

import numpy as np

from . import gpe as G

__all__ = ["frozen_forward_step", "frozen_adjoint_step", "assemble_forward", "assemble_adjoint",
           "apply_adjoint_map", "frozen_boundaries", "ism_bec_frozen_iterate"]


def frozen_forward_step(psi, a_frozen, k, V, gnl, tau):
    """S_j psi with the density |a_frozen|^2 frozen (psi: one state, or states stacked along
    the first axis)."""
    a = G._kinetic(psi, tau, k)
    theta = tau * (V + gnl * np.abs(a_frozen) ** 2)
    return G._kinetic(np.exp(-1j * theta) * a, tau, k)


def frozen_adjoint_step(nu, a_frozen, k, V, gnl, tau):
    """R_j nu: the exact adjoint step of oracle/gpe.py at the frozen a_j (real-linear; nu:
    one state, or states stacked along the first axis)."""
    theta = tau * (V + gnl * np.abs(a_frozen) ** 2)
    nup = G._kinetic(nu, tau, k, +1)
    w = np.exp(1j * theta) * nup
    mu = w + 2.0 * tau * gnl * np.imag(np.conj(w) * a_frozen) * a_frozen
    return G._kinetic(mu, tau, k, +1)


def assemble_forward(a_fr, u, V0, V1, V2, gnl, L, tau, s):
    """M_n, n = 0..N-1 (columns: the slice's frozen steps applied to the basis vectors)."""
    n = a_fr[0].shape[0]
    _, k, _ = G.grid(n, L)
    Ms = []
    for i in range(len(s) - 1):
        X = np.eye(n, dtype=np.complex128)          # row c: the image of e_c
        for j in range(s[i], s[i + 1]):
            X = frozen_forward_step(X, a_fr[j], k, G.potential(V0, V1, V2, u[j]), gnl, tau)
        Ms.append(X.T.copy())
    return Ms


def assemble_adjoint(a_fr, u, V0, V1, V2, gnl, L, tau, s):
    """A_n, n = 0..N-1, as (n x 2n) complex arrays: column m is A_n(e_m), column n + m is
    A_n(i e_m) (the slice's frozen adjoint steps from its last step down to its first)."""
    n = a_fr[0].shape[0]
    _, k, _ = G.grid(n, L)
    As = []
    for i in range(len(s) - 1):
        # row c: the image of e_c (c < n) or of i e_{c-n}
        X = np.concatenate([np.eye(n), 1j * np.eye(n)], axis=0).astype(np.complex128)
        for j in range(s[i + 1] - 1, s[i] - 1, -1):
            X = frozen_adjoint_step(X, a_fr[j], k, G.potential(V0, V1, V2, u[j]), gnl, tau)
        As.append(X.T.copy())
    return As


def apply_adjoint_map(A, nu):
    n = nu.shape[0]
    return A[:, :n] @ nu.real + A[:, n:] @ nu.imag


def frozen_boundaries(Ms, As, psi0, target):
    """Psi_0 = psi0, Psi_{n+1} = M_n Psi_n; Lambda_N = psi_f, Lambda_n = A_n Lambda_{n+1}."""
    N = len(Ms)
    Psi = [np.array(psi0, dtype=np.complex128)]
    for i in range(N):
        Psi.append(Ms[i] @ Psi[-1])
    Lam = [None] * (N + 1)
    Lam[N] = np.array(target, dtype=np.complex128)
    for i in range(N - 1, -1, -1):
        Lam[i] = apply_adjoint_map(As[i], Lam[i + 1])
    return Psi, Lam


def ism_bec_frozen_iterate(psi0, target, u0, V0, V1, V2, gnl, L, T, rho, iters, N):
    """Lagged ISM for the condensate (see the module text).  Returns {"u", "J", "F"} with
    J^(k), F^(k) from the boundary chain of iteration k."""
    u = np.array(u0, dtype=np.float64, copy=True)
    K = u.shape[0]
    tau = T / K
    n = psi0.shape[0]
    dx = L / n
    s = [(i * K) // N for i in range(N + 1)]
    Js, Fs = [], []
    a_fr = None
    for _ in range(iters):
        if a_fr is None:
            # first iteration: exact sequential sweeps (the exact BEC variant's boundaries)
            _, J, F, Psi, Lam = G.ism_bec_gradient(psi0, target, u, V0, V1, V2, gnl, L, T, N)
        else:
            Ms = assemble_forward(a_fr, u, V0, V1, V2, gnl, L, tau, s)
            As = assemble_adjoint(a_fr, u, V0, V1, V2, gnl, L, tau, s)
            Psi, Lam = frozen_boundaries(Ms, As, psi0, target)
            J, F = G.objective(Psi[N], target, dx)
        Js.append(J); Fs.append(F)
        a_next = [None] * K
        for i in range(N):
            lo, hi = s[i], s[i + 1]
            _, rec = G.strang_forward(Psi[i], u[lo:hi], V0, V1, V2, gnl, L, tau)
            a_next[lo:hi] = rec["a"]
            _, g = G._adjoint_steps(np.array(Lam[i + 1], dtype=np.complex128), rec, u[lo:hi],
                                    V1, V2, gnl, L, tau, 0, hi - lo, dx)
            u[lo:hi] = u[lo:hi] + rho * g
        a_fr = a_next
    return {"u": u, "J": np.array(Js), "F": np.array(Fs)}
