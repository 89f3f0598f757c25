"""Oracle, finite-dimensional problems (TEST INFRASTRUCTURE ONLY).

Notation follows the paper (Sec. 2 and Sec. 3):

* dynamics  i d/dt psi = H(u) psi,  H(u) = H0 + sum_c u_c H_c        (Eq. (dir))
* objective J[u] = Re<psi(T)|psi_f> - alpha/2 int u^2                 (Sec. 2)
* K steps of length tau = T/K, control u_j constant on step j         (Sec. 3, time grid)
* step map  psi_{j+1} = exp(-i tau H(u_j)) psi_j  (exact exponential of the
  piecewise-constant Hamiltonian, evaluated by scipy's expm; the paper's Crank-Nicolson
  map is the separate *_cn family below)
* discrete objective J_tau = Re<psi_K|psi_f> - tau/2 sum_j alpha_j |u_j|^2
* adjoint  lambda_K = psi_f, lambda_j = U_j^dagger lambda_{j+1}      (discrete Eq. (adj))
* gradient g_{j,c} = (1/tau) dJ_tau/du_{j,c}
           = Im<lambda_j| Hhat_{c,j} |psi_j> - alpha_j u_{j,c}
  where Hhat_{c,j} = (1/tau) int_0^tau e^{isH_j} H_c e^{-isH_j} ds is the
  step average of H_c, so that dU_j/du_c = -i tau U_j Hhat_{c,j}.  This is
  the exact discrete counterpart of Eq. (gradJ); the paper's own discrete
  formula (Sec. 3, end) is for Crank-Nicolson and is garbled in print.
* plain method  u <- u + rho g   (Eq. (gradStep), read as ascent since J is
  maximised)
* ISM (Algorithm 1, one gradient step per slice): slices s_n = floor(nK/N),
  t_n = s_n tau, intermediate states
      phi_n = (T - t_n)/T psi(t_n) + t_n/T chi(t_n)                  (Eq. (cible))
  slice functional J_n with alpha_n = alpha (t_{n+1}-t_n)/T, beta_n = T/(t_{n+1}-t_n),
  slice trajectories psi^n from phi_n and chi^n from phi_{n+1}, slice gradient
  beta_n grad J_n = grad J (Theorem 2), boundaries by propagator assembling
  M_n = U_{s_{n+1}-1} ... U_{s_n} and 2N matrix-vector products (Sec. 3).

Inner products: states <a|b> = sum conj(a) b; gates <A|B> = Tr(A^dagger B)/d.

Crank-Nicolson map (Sec. 3): U_j = (I + L_j)^{-1}(I - L_j), L_j = (i tau/2) H_j, with the
exact gradient 1/2 Im<chi_j|H_c|psi_j + psi_{j+1}>, (I - L_j) chi_j = lambda_{j+1}.

Several gradient steps per slice (Algorithm 1 step (c) with Eq. (gradStep) iterated ell
times on the slice problem max J_n[., phi^(k)], the intermediate states held fixed):
    u_n <- u_n + rho beta_n grad J_n[u_n, phi^(k)]          (ell times)
(the step is scaled by beta_n so that ell = 1 is the plain gradient step, Theorem 2), then
Algorithm 1 step (e): Err = sum_n tau sum_{j in slice n} || grad J_n[u^(k+1), phi^(k)]_j ||_2,
the Euclidean norm taken over the controls of step j; the loop runs while Err > eta.

Pins (tests/test_oracle_finite.py, tests/test_oracle_cn.py, tests/test_oracle_inner.py): closed-form spin rotations, unitarity,
reversibility, overlap invariance, central finite differences of J_tau,
scipy's Frechet derivative of expm, ISM == plain gradient iterates, Theorem 1
(value and argmax by an independent linear solve), Theorem 2 per slice,
assembled boundaries == sequential propagation, rotor Gauss-Legendre nodes,
free-rotor phases, slice-problem gradients and Err against central finite differences of
J_n, ell = 1 == plain method, N = 1 with ell steps == plain method with ell steps per
iteration.  No function here is parity-unpinned.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = [
    "slice_starts", "hamiltonian", "step_unitary", "step_unitaries", "hhat",
    "forward", "backward", "inner", "objective", "gradient", "plain_gradient_method",
    "assemble", "boundaries", "intermediate_states", "ism_slice_gradient",
    "ism_gradient", "ism_iterate", "theorem1_functional", "theorem1_argmax",
    "cn_generator", "step_unitary_cn", "step_unitaries_cn", "gradient_cn",
    "plain_gradient_method_cn", "ism_gradient_cn", "ism_iterate_cn",
    "subproblem_objective", "subproblem_gradient", "ism_iterate_inner",
]


def slice_starts(K: int, N: int) -> np.ndarray:
    """s_n = floor(n K / N), n = 0..N: a partition 0 = t_0 < ... < t_N = T of the
    time grid (Sec. 2; the paper allows any partition)."""
    if not (1 <= N <= K):
        raise ValueError("need 1 <= N <= K")
    return np.array([(n * K) // N for n in range(N + 1)], dtype=np.int64)


def hamiltonian(H0: np.ndarray, Hc: np.ndarray, uj: np.ndarray) -> np.ndarray:
    """H(u_j) = H0 + sum_c u_{j,c} H_c  (Eq. (dir) with the control on step j)."""
    H = np.array(H0, dtype=np.complex128, copy=True)
    for c in range(Hc.shape[0]):
        H = H + uj[c] * Hc[c]
    return H


def _eig(H: np.ndarray):
    Hh = 0.5 * (H + H.conj().T)
    w, V = np.linalg.eigh(Hh)
    return w, V


def step_unitary(H: np.ndarray, tau: float) -> np.ndarray:
    """U = exp(-i tau H), the exact exponential of the step's Hamiltonian (Eq. (dir) with a
    constant control on the step), by scipy's scaling-and-squaring Pade evaluation.

    The eigendecomposition form V diag(e^{-i tau w}) V^dagger is exact in exact arithmetic
    too, but its rounding is nearly the same from one step to the next (the step
    Hamiltonians differ only through the controls), so composed over a long trajectory it
    drifts coherently: 9.4e-13 on psi(T) of the 256 rotors at K = 20000, against 1.8e-14 for
    this evaluation, both measured against an extended-precision power series."""
    return sla.expm(-1j * tau * np.asarray(H, dtype=np.complex128))


def step_unitaries(H0, Hc, u, tau):
    """[U_0, ..., U_{K-1}] for controls u of shape (K, C)."""
    return [step_unitary(hamiltonian(H0, Hc, u[j]), tau) for j in range(u.shape[0])]


def _phi1(x: np.ndarray) -> np.ndarray:
    """(e^{ix} - 1)/(ix), evaluated as sin(x)/x + i 2 sin^2(x/2)/x, with its series near 0."""
    out = np.empty(x.shape, dtype=np.complex128)
    small = np.abs(x) < 1e-4
    xs = x[small]
    out[small] = (1 - xs ** 2 / 6 + xs ** 4 / 120) + 1j * (xs / 2 - xs ** 3 / 24)
    xl = x[~small]
    out[~small] = np.sin(xl) / xl + 1j * 2 * np.sin(xl / 2) ** 2 / xl
    return out


def hhat(H: np.ndarray, Hcs: np.ndarray, tau: float) -> np.ndarray:
    """Step-averaged control operators Hhat_c = (1/tau) int_0^tau e^{isH} H_c e^{-isH} ds.

    In the eigenbasis of H: (V^dagger Hhat V)_ab = (V^dagger H_c V)_ab phi1(tau (w_a - w_b)).
    Returns shape (C, d, d)."""
    w, V = _eig(H)
    Phi = _phi1(tau * (w[:, None] - w[None, :]))
    out = []
    for c in range(Hcs.shape[0]):
        A = V.conj().T @ Hcs[c] @ V
        out.append(V @ (A * Phi) @ V.conj().T)
    return np.stack(out)


def forward(Us, psi0):
    """psi_0 = psi0, psi_{j+1} = U_j psi_j; returns the list psi_0..psi_K (vectors or matrices)."""
    out = [np.array(psi0, dtype=np.complex128)]
    for U in Us:
        out.append(U @ out[-1])
    return out


def backward(Us, target):
    """lambda_K = psi_f, lambda_j = U_j^dagger lambda_{j+1}; returns lambda_0..lambda_K."""
    out = [np.array(target, dtype=np.complex128)]
    for U in reversed(Us):
        out.append(U.conj().T @ out[-1])
    return out[::-1]


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a|b>: sum conj(a) b for states, Tr(a^dagger b)/d for gates (matrices)."""
    if a.ndim == 1:
        return complex(np.vdot(a, b))
    return complex(np.trace(a.conj().T @ b)) / a.shape[0]


def objective(psiK, target, u, alpha, tau):
    """J_tau = Re<psi_K|psi_f> - tau/2 sum_j alpha_j sum_c u_{j,c}^2 and F = |<psi_K|psi_f>|^2."""
    z = inner(psiK, target)
    pen = 0.5 * tau * float(np.sum(alpha[:, None] * u ** 2))
    return z.real - pen, abs(z) ** 2


def gradient(H0, Hc, psi0, target, u, T, alpha):
    """Exact (1/tau) dJ_tau/du of the exponential step map, plus J and F at u.

    Returns (g[K,C], J, F, psi_K)."""
    K = u.shape[0]
    tau = T / K
    Us = step_unitaries(H0, Hc, u, tau)
    psis = forward(Us, psi0)
    lams = backward(Us, target)
    g = np.zeros_like(u)
    for j in range(K):
        Hh = hhat(hamiltonian(H0, Hc, u[j]), Hc, tau)
        for c in range(Hc.shape[0]):
            g[j, c] = inner(lams[j], Hh[c] @ psis[j]).imag - alpha[j] * u[j, c]
    J, F = objective(psis[-1], target, u, alpha, tau)
    return g, J, F, psis[-1]


def plain_gradient_method(H0, Hc, psi0, target, u0, T, alpha, rho, iters):
    """Constant-step gradient ascent u^{k+1} = u^k + rho g(u^k) (Eq. (gradStep)).

    Returns dict with the final u, and per-iteration J^(k), F^(k) (at u^k, before the
    update) and Err^(k) = tau sum |g^(k)| (the L1 size of the gradient, Algorithm 1 step (e))."""
    u = np.array(u0, dtype=np.float64, copy=True)
    tau = T / u.shape[0]
    Js, Fs, Errs = [], [], []
    for _ in range(iters):
        g, J, F, _ = gradient(H0, Hc, psi0, target, u, T, alpha)
        Js.append(J); Fs.append(F); Errs.append(tau * float(np.sum(np.abs(g))))
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs), "Err": np.array(Errs)}


# ----------------------------------------------------------------------------
# ISM
# ----------------------------------------------------------------------------

def assemble(Us, s):
    """Slice propagators M_n = U_{s_{n+1}-1} ... U_{s_n} (propagator assembling, Sec. 3)."""
    d = Us[0].shape[0]
    Ms = []
    for n in range(len(s) - 1):
        M = np.eye(d, dtype=np.complex128)
        for j in range(s[n], s[n + 1]):
            M = Us[j] @ M
        Ms.append(M)
    return Ms


def boundaries(Ms, psi0, target):
    """The 2N products of Sec. 3: Psi_0 = psi0, Psi_{n+1} = M_n Psi_n (forward) and
    Lambda_N = psi_f, Lambda_n = M_n^dagger Lambda_{n+1} (adjoint).
    Psi_n = psi(t_n) and Lambda_n = chi(t_n)."""
    N = len(Ms)
    Psi = [np.array(psi0, dtype=np.complex128)]
    for n in range(N):
        Psi.append(Ms[n] @ Psi[-1])
    Lam = [None] * (N + 1)
    Lam[N] = np.array(target, dtype=np.complex128)
    for n in range(N - 1, -1, -1):
        Lam[n] = Ms[n].conj().T @ Lam[n + 1]
    return Psi, Lam


def intermediate_states(Psi, Lam, s, K):
    """phi_n = (T - t_n)/T psi(t_n) + t_n/T chi(t_n)   (Eq. (cible)); t_n/T = s_n/K."""
    return [(1.0 - s[n] / K) * Psi[n] + (s[n] / K) * Lam[n] for n in range(len(s))]


def ism_slice_gradient(Us, Hhats, u, alpha, phi_n, phi_n1, sn, sn1, K):
    """Gradient of the slice problem n, scaled by beta_n (Theorem 2).

    psi^n from phi_n forward over steps sn..sn1-1 (Eq. (dirpara)); chi^n from phi_{n+1}
    backward (end condition of the Re-form of J_n, Sec. 2).  Returns
    beta_n [Im<chi^n_j|Hhat_{c,j}|psi^n_j> - alpha_{n,j} u_{j,c}] for j in [sn, sn1),
    with alpha_{n,j} = alpha_j / beta_n."""
    beta = K / (sn1 - sn)
    psi = [phi_n]
    for j in range(sn, sn1):
        psi.append(Us[j] @ psi[-1])
    chi = [None] * (sn1 - sn + 1)
    chi[-1] = phi_n1
    for j in range(sn1 - 1, sn - 1, -1):
        chi[j - sn] = Us[j].conj().T @ chi[j - sn + 1]
    C = u.shape[1]
    g = np.zeros((sn1 - sn, C))
    for j in range(sn, sn1):
        for c in range(C):
            ov = inner(chi[j - sn], Hhats[j][c] @ psi[j - sn]).imag
            g[j - sn, c] = beta * (ov - (alpha[j] / beta) * u[j, c])
    return g, psi[-1]


def ism_gradient(H0, Hc, psi0, target, u, T, alpha, N):
    """One ISM gradient evaluation: Algorithm 1 steps (a)-(c) with the boundaries by
    propagator assembling.  Returns (g[K,C], J, F, phi list, Psi, Lam)."""
    K = u.shape[0]
    tau = T / K
    s = slice_starts(K, N)
    Us = step_unitaries(H0, Hc, u, tau)
    Hhats = [hhat(hamiltonian(H0, Hc, u[j]), Hc, tau) for j in range(K)]
    Ms = assemble(Us, s)
    Psi, Lam = boundaries(Ms, psi0, target)
    phi = intermediate_states(Psi, Lam, s, K)
    g = np.zeros_like(u)
    for n in range(N):
        gn, _ = ism_slice_gradient(Us, Hhats, u, alpha, phi[n], phi[n + 1], s[n], s[n + 1], K)
        g[s[n]:s[n + 1]] = gn
    J, F = objective(Psi[-1], target, u, alpha, tau)
    return g, J, F, phi, Psi, Lam


def ism_iterate(H0, Hc, psi0, target, u0, T, alpha, rho, iters, N):
    """ISM (Algorithm 1) with one constant-step gradient step per slice and per iteration.

    Returns the same record as plain_gradient_method."""
    u = np.array(u0, dtype=np.float64, copy=True)
    tau = T / u.shape[0]
    Js, Fs, Errs = [], [], []
    for _ in range(iters):
        g, J, F, _, _, _ = ism_gradient(H0, Hc, psi0, target, u, T, alpha, N)
        Js.append(J); Fs.append(F); Errs.append(tau * float(np.sum(np.abs(g))))
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs), "Err": np.array(Errs)}


# ----------------------------------------------------------------------------
# Theorem 1
# ----------------------------------------------------------------------------

def theorem1_functional(Ms, phi, u, alpha, s, K, T):
    """J_par[u, phi] = sum_n beta_n J_n with J_n in its squared-distance form
    J_n = -1/2 ||M_n phi_n - phi_{n+1}||^2 - alpha_n/2 tau sum_{j in slice} |u_j|^2 (Sec. 2)."""
    tau = T / K
    tot = 0.0
    for n in range(len(Ms)):
        beta = K / (s[n + 1] - s[n])
        diff = Ms[n] @ phi[n] - phi[n + 1]
        dist2 = float(np.real(np.vdot(diff, diff)))
        pen = 0.5 * tau * float(np.sum((alpha[s[n]:s[n + 1]] / beta)[:, None] * u[s[n]:s[n + 1]] ** 2))
        tot += beta * (-0.5 * dist2 - pen)
    return tot


def theorem1_argmax(Ms, psi0, target, s, K):
    """Maximiser of J_par over the interior phi_1..phi_{N-1} (phi_0 = psi0, phi_N = psi_f
    fixed), by solving the stationarity conditions as one dense linear system:
      (beta_{n-1} + beta_n) phi_n - beta_{n-1} M_{n-1} phi_{n-1} - beta_n M_n^dagger phi_{n+1} = 0
    for n = 1..N-1 (uses M_n^dagger M_n = I).  Independent of Eq. (cible)."""
    N = len(Ms)
    d = Ms[0].shape[0]
    if N == 1:
        return [np.array(psi0), np.array(target)]
    beta = [K / (s[n + 1] - s[n]) for n in range(N)]
    A = np.zeros(((N - 1) * d, (N - 1) * d), dtype=np.complex128)
    b = np.zeros((N - 1) * d, dtype=np.complex128)
    for n in range(1, N):
        r = (n - 1) * d
        A[r:r + d, r:r + d] = (beta[n - 1] + beta[n]) * np.eye(d)
        if n - 1 >= 1:
            A[r:r + d, r - d:r] = -beta[n - 1] * Ms[n - 1]
        else:
            b[r:r + d] += beta[n - 1] * Ms[n - 1] @ psi0
        if n + 1 <= N - 1:
            A[r:r + d, r + d:r + 2 * d] = -beta[n] * Ms[n].conj().T
        else:
            b[r:r + d] += beta[n] * Ms[n].conj().T @ target
    x = np.linalg.solve(A, b)
    return [np.array(psi0)] + [x[(n - 1) * d:n * d] for n in range(1, N)] + [np.array(target)]


# ----------------------------------------------------------------------------
# Crank-Nicolson step map (Sec. 3: the paper's own scheme for finite dimension)
# ----------------------------------------------------------------------------

def cn_generator(H: np.ndarray, tau: float) -> np.ndarray:
    """L_j = (i tau / 2) H_j, so that the Crank-Nicolson step solves
    (I + L_j) psi_{j+1} = (I - L_j) psi_j  (Sec. 3, time discretisation)."""
    return 0.5j * tau * np.asarray(H, dtype=np.complex128)


def step_unitary_cn(H: np.ndarray, tau: float) -> np.ndarray:
    """U_j = (I + L_j)^{-1} (I - L_j): the Cayley transform of -i tau H_j, unitary for
    Hermitian H_j."""
    L = cn_generator(H, tau)
    I = np.eye(L.shape[0], dtype=np.complex128)
    return np.linalg.solve(I + L, I - L)


def step_unitaries_cn(H0, Hc, u, tau):
    return [step_unitary_cn(hamiltonian(H0, Hc, u[j]), tau) for j in range(u.shape[0])]


def _cn_step_gradient(H, Hc, lam_next, psi_j, psi_next, tau):
    """(1/tau) dJ/du_{j,c} of the Crank-Nicolson step, without the penalty (the discrete
    gradient of Sec. 3 read as in the design notes):
        chi_j solves (I - L_j) chi_j = lambda_{j+1},
        g_{j,c} = 1/2 Im <chi_j | H_c | psi_j + psi_{j+1}>.
    Derivation: U = (I+L)^{-1}(I-L) gives dU/du_c = -(i tau/2) (I+L)^{-1} H_c (I + U), and
    ((I+L)^{-1})^dagger = (I-L)^{-1}."""
    L = cn_generator(H, tau)
    I = np.eye(L.shape[0], dtype=np.complex128)
    chi = np.linalg.solve(I - L, lam_next)
    s = psi_j + psi_next
    return np.array([0.5 * inner(chi, Hc[c] @ s).imag for c in range(Hc.shape[0])])


def gradient_cn(H0, Hc, psi0, target, u, T, alpha):
    """Exact (1/tau) dJ_tau/du of the Crank-Nicolson step map, plus J and F at u.
    Returns (g[K,C], J, F, psi_K)."""
    K = u.shape[0]
    tau = T / K
    Us = step_unitaries_cn(H0, Hc, u, tau)
    psis = forward(Us, psi0)
    lams = backward(Us, target)
    g = np.zeros_like(u)
    for j in range(K):
        H = hamiltonian(H0, Hc, u[j])
        g[j] = _cn_step_gradient(H, Hc, lams[j + 1], psis[j], psis[j + 1], tau) - alpha[j] * u[j]
    J, F = objective(psis[-1], target, u, alpha, tau)
    return g, J, F, psis[-1]


def plain_gradient_method_cn(H0, Hc, psi0, target, u0, T, alpha, rho, iters):
    """Constant-step gradient ascent (Eq. (gradStep)) with the Crank-Nicolson map."""
    u = np.array(u0, dtype=np.float64, copy=True)
    tau = T / u.shape[0]
    Js, Fs, Errs = [], [], []
    for _ in range(iters):
        g, J, F, _ = gradient_cn(H0, Hc, psi0, target, u, T, alpha)
        Js.append(J); Fs.append(F); Errs.append(tau * float(np.sum(np.abs(g))))
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs), "Err": np.array(Errs)}


def ism_gradient_cn(H0, Hc, psi0, target, u, T, alpha, N):
    """ISM gradient (Algorithm 1 steps (a)-(c)) with the Crank-Nicolson map: propagator
    assembling, boundaries, intermediate states (Eq. (cible)); per slice the forward
    trajectory from phi_n, the adjoint from phi_{n+1} and
        beta_n [ 1/2 Im<chi^n_j|H_c|psi^n_j + psi^n_{j+1}> - alpha_{n,j} u_{j,c} ],
    chi^n_j solving (I - L_j) chi^n_j = lambda^n_{j+1}.  Returns (g, J, F, phi, Psi, Lam)."""
    K = u.shape[0]
    tau = T / K
    s = slice_starts(K, N)
    Us = step_unitaries_cn(H0, Hc, u, tau)
    Ms = assemble(Us, s)
    Psi, Lam = boundaries(Ms, psi0, target)
    phi = intermediate_states(Psi, Lam, s, K)
    g = np.zeros_like(u)
    for n in range(N):
        sn, sn1 = s[n], s[n + 1]
        beta = K / (sn1 - sn)
        psi = [phi[n]]
        for j in range(sn, sn1):
            psi.append(Us[j] @ psi[-1])
        lam = [None] * (sn1 - sn + 1)
        lam[-1] = phi[n + 1]
        for j in range(sn1 - 1, sn - 1, -1):
            lam[j - sn] = Us[j].conj().T @ lam[j - sn + 1]
        for j in range(sn, sn1):
            H = hamiltonian(H0, Hc, u[j])
            gj = _cn_step_gradient(H, Hc, lam[j - sn + 1], psi[j - sn], psi[j - sn + 1], tau)
            g[j] = beta * (gj - (alpha[j] / beta) * u[j])
    J, F = objective(Psi[-1], target, u, alpha, tau)
    return g, J, F, phi, Psi, Lam


def ism_iterate_cn(H0, Hc, psi0, target, u0, T, alpha, rho, iters, N):
    """ISM with one gradient step per slice (Algorithm 1), Crank-Nicolson map."""
    u = np.array(u0, dtype=np.float64, copy=True)
    tau = T / u.shape[0]
    Js, Fs, Errs = [], [], []
    for _ in range(iters):
        g, J, F, _, _, _ = ism_gradient_cn(H0, Hc, psi0, target, u, T, alpha, N)
        Js.append(J); Fs.append(F); Errs.append(tau * float(np.sum(np.abs(g))))
        u = u + rho * g
    return {"u": u, "J": np.array(Js), "F": np.array(Fs), "Err": np.array(Errs)}


# ----------------------------------------------------------------------------
# Several gradient steps per slice problem and the Err stopping rule (Algorithm 1)
# ----------------------------------------------------------------------------

def _slice_maps(H0, Hc, u, sn, sn1, tau, step):
    """Step maps of the steps sn..sn1-1 under the controls u (full (K, C) array), as a
    length-K list with the entries outside the slice left empty."""
    K = u.shape[0]
    Us = [None] * K
    if step == "cn":
        Us[sn:sn1] = step_unitaries_cn(H0, Hc, u[sn:sn1], tau)
    else:
        Us[sn:sn1] = step_unitaries(H0, Hc, u[sn:sn1], tau)
    return Us


def subproblem_objective(H0, Hc, u, alpha, phi_n, phi_n1, sn, sn1, T, step="exp"):
    """Slice functional in its Re-form (Sec. 2):
        J_n = Re<psi_n(t_{n+1})|phi_{n+1}> - alpha_n/2 tau sum_{j in slice} |u_j|^2,
    psi_n propagated from phi_n over steps sn..sn1-1 (Eq. (dirpara)), alpha_n = alpha/beta_n."""
    K = u.shape[0]
    tau = T / K
    beta = K / (sn1 - sn)
    Us = _slice_maps(H0, Hc, u, sn, sn1, tau, step)
    psi = phi_n
    for j in range(sn, sn1):
        psi = Us[j] @ psi
    pen = 0.5 * tau * float(np.sum((alpha[sn:sn1] / beta)[:, None] * u[sn:sn1] ** 2))
    return inner(psi, phi_n1).real - pen


def subproblem_gradient(H0, Hc, u, alpha, phi_n, phi_n1, sn, sn1, T, step="exp"):
    """beta_n grad J_n[u, phi] on the steps sn..sn1-1, with grad J_n = (1/tau) dJ_n/du_j
    (the exact discrete gradient of the slice functional for the chosen step map).
    Returns an (sn1 - sn, C) array."""
    K = u.shape[0]
    tau = T / K
    if step != "cn":
        Us = _slice_maps(H0, Hc, u, sn, sn1, tau, step)
        Hhats = [None] * K
        for j in range(sn, sn1):
            Hhats[j] = hhat(hamiltonian(H0, Hc, u[j]), Hc, tau)
        g, _ = ism_slice_gradient(Us, Hhats, u, alpha, phi_n, phi_n1, sn, sn1, K)
        return g
    beta = K / (sn1 - sn)
    Us = _slice_maps(H0, Hc, u, sn, sn1, tau, "cn")
    psi = [phi_n]
    for j in range(sn, sn1):
        psi.append(Us[j] @ psi[-1])
    lam = [None] * (sn1 - sn + 1)
    lam[-1] = phi_n1
    for j in range(sn1 - 1, sn - 1, -1):
        lam[j - sn] = Us[j].conj().T @ lam[j - sn + 1]
    g = np.zeros((sn1 - sn, u.shape[1]))
    for j in range(sn, sn1):
        H = hamiltonian(H0, Hc, u[j])
        gj = _cn_step_gradient(H, Hc, lam[j - sn + 1], psi[j - sn], psi[j - sn + 1], tau)
        g[j - sn] = beta * (gj - (alpha[j] / beta) * u[j])
    return g


def ism_iterate_inner(H0, Hc, psi0, target, u0, T, alpha, rho, iters, N, ell, eta=0.0,
                      step="exp"):
    """Algorithm 1 with step (c) = ell constant-step gradient steps on every slice problem.

    Iteration k: boundaries and intermediate states phi^(k) at u^(k) (steps (a)-(b), by
    propagator assembling); on each slice, ell steps u_n <- u_n + rho beta_n grad J_n[u_n,
    phi^(k)] (steps (c)-(d)); then Err^(k) = sum_n tau sum_j ||grad J_n[u^(k+1), phi^(k)]_j||
    (step (e)).  The loop stops after the iteration whose Err is <= eta (eta <= 0: never).
    Returns {"u", "J", "F", "Err", "iters"}: J^(k), F^(k) at u^(k) and Err^(k) for every
    iteration run, "iters" the number of iterations run."""
    u = np.array(u0, dtype=np.float64, copy=True)
    K = u.shape[0]
    tau = T / K
    s = slice_starts(K, N)
    maps = step_unitaries_cn if step == "cn" else step_unitaries
    Js, Fs, Errs = [], [], []
    for _ in range(iters):
        Ms = assemble(maps(H0, Hc, u, tau), s)
        Psi, Lam = boundaries(Ms, psi0, target)
        phi = intermediate_states(Psi, Lam, s, K)
        J, F = objective(Psi[-1], target, u, alpha, tau)
        Js.append(J); Fs.append(F)
        err = 0.0
        for n in range(N):
            sn, sn1 = s[n], s[n + 1]
            beta = K / (sn1 - sn)
            for _l in range(ell):
                g = subproblem_gradient(H0, Hc, u, alpha, phi[n], phi[n + 1], sn, sn1, T, step)
                u[sn:sn1] = u[sn:sn1] + rho * g
            g = subproblem_gradient(H0, Hc, u, alpha, phi[n], phi[n + 1], sn, sn1, T, step)
            err += tau * float(np.sum(np.sqrt(np.sum((g / beta) ** 2, axis=1))))
        Errs.append(err)
        if eta > 0 and err <= eta:
            break
    return {"u": u, "J": np.array(Js), "F": np.array(Fs), "Err": np.array(Errs),
            "iters": len(Errs)}
