"""Long-trajectory pins of the oracle's step maps (P3 extended to the benchmark's length).

Rounding that is nearly the same at every step adds up linearly over a trajectory instead
of as a random walk.  These pins run the rotor batch's own trajectories (d = 21, K = 20000,
tau H up to 0.25) through the oracle and compare psi(T) and lambda(0) with an
extended-precision evaluation of the same step maps (tests/_extended.py, unit roundoff
5.4e-20): the exponential of Eq. (dir) by its power series, and the Crank-Nicolson map of
Sec. 3 by tridiagonal elimination.  The bars are the FP64 parity bars' budget for the
oracle's own share: the GPU comparisons at this length are only as sharp as the oracle.

Measured when these pins were written (256 rotors): the oracle's exponential (scipy's
Pade scaling and squaring) within 1.8e-14, the eigendecomposition form of the same
exponential 9.4e-13 (coherent drift; see the guard below), the Crank-Nicolson map (LU
solve) within 2.4e-13 on instances 0-7.
"""
import numpy as np

import problems
from oracle import finite as O
import _extended as X


def _orc_ends(p, b, step):
    Us = (O.step_unitaries if step == "exp" else O.step_unitaries_cn)(p.H0_of(b), p.Hc, p.u0[b],
                                                                     p.T / p.K)
    return O.forward(Us, p.psi0)[-1], O.backward(Us, p.target)[0]


def test_exp_map_over_20000_steps():
    p = problems.rotor()
    idx = [0, 6]
    xf = X.trajectory_end(p, idx)
    xb = X.trajectory_end(p, idx, backward=True)
    for i, b in enumerate(idx):
        psiK, lam0 = _orc_ends(p, b, "exp")
        assert np.linalg.norm(psiK - xf[i]) <= 5e-14, np.linalg.norm(psiK - xf[i])
        assert np.linalg.norm(lam0 - xb[i]) <= 5e-14, np.linalg.norm(lam0 - xb[i])


def test_exp_map_eigendecomposition_form_drifts():
    """Guard: the eigendecomposition evaluation of the same exponentials as a step matrix
    V e^{-i tau w} V^dagger, the oracle's first form, misses the bar above on these
    trajectories (6.7e-13), so the pin can tell them apart.  The rounding of that matrix
    product is nearly the same at every step, since consecutive step Hamiltonians differ only
    through the controls."""
    p = problems.rotor()
    xf = X.trajectory_end(p, [0])[0]
    tau = p.T / p.K
    psi = np.array(p.psi0, dtype=complex)
    for j in range(p.K):
        H = O.hamiltonian(p.H0_of(0), p.Hc, p.u0[0, j])
        w, V = np.linalg.eigh(0.5 * (H + H.conj().T))
        U = (V * np.exp(-1j * tau * w)[None, :]) @ V.conj().T
        psi = U @ psi
    assert np.linalg.norm(psi - xf) > 2e-13


def test_cn_map_over_20000_steps():
    p = problems.rotor()
    idx = [1, 4]
    xf = X.trajectory_end(p, idx, step="cn")
    xb = X.trajectory_end(p, idx, backward=True, step="cn")
    for i, b in enumerate(idx):
        psiK, lam0 = _orc_ends(p, b, "cn")
        assert np.linalg.norm(psiK - xf[i]) <= 5e-13, np.linalg.norm(psiK - xf[i])
        assert np.linalg.norm(lam0 - xb[i]) <= 5e-13, np.linalg.norm(lam0 - xb[i])


def test_density_cn_map_over_1024_steps():
    """The five-spin density run (d = 32, tau = T/2^15) under the Crank-Nicolson map: the
    oracle's conjugation by U_j = I + D_j, D_j = -2 (I + L_j)^{-1} L_j, against the
    extended-precision evaluation over the first 1024 steps (measured 1.8e-15); and the guard:
    conjugating by the rounded U_j = (I + L_j)^{-1}(I - L_j) itself, whose entries near 1
    carry a rounding that repeats from step to step, drifts much further (6.4e-14 here,
    1.8e-12 at the full 2^15 steps)."""
    from oracle import density as D
    p = problems.spin5_density()
    Kc = 1024
    tau = p.T / p.K
    ref = X.density_cn_end(p, Kc)
    n0 = np.linalg.norm(p.psi0)
    Ds = [D._cn_difference(O.hamiltonian(p.H0, p.Hc, p.u0[0, j]), tau) for j in range(Kc)]
    got = D.forward_cn(Ds, p.psi0)[-1]
    err = np.linalg.norm(got - ref) / n0
    assert err <= 5e-15, err
    Us = [O.step_unitary_cn(O.hamiltonian(p.H0, p.Hc, p.u0[0, j]), tau) for j in range(Kc)]
    guard = np.linalg.norm(D.forward(Us, p.psi0)[-1] - ref) / n0
    assert guard > 3e-14, guard


def test_extended_reference_closed_forms():
    """The reference itself: with u = 0 every basis component only turns its phase,
    psi_r(T) = e^{-i B r(r+1) T} (P14), and the Crank-Nicolson phase is that of the Cayley
    factor (1 - i tau h/2)/(1 + i tau h/2) per step."""
    p = problems.rotor(batch=2, K=2000, T=1.0)
    p.u0[:] = 0.0
    rng = np.random.default_rng(5)
    v = rng.standard_normal(p.d) + 1j * rng.standard_normal(p.d)
    p.psi0 = v / np.linalg.norm(v)
    h = np.real(np.diag(p.H0[1])).astype(np.longdouble)
    tau = np.longdouble(p.T / p.K)            # K steps of the FP64 step length
    got = X.trajectory_end(p, [1])[0]
    assert np.max(np.abs(got - np.exp(-1j * h * tau * p.K) * p.psi0)) <= 1e-15
    cay = ((1 - 0.5j * tau * h) / (1 + 0.5j * tau * h)) ** p.K
    got = X.trajectory_end(p, [1], step="cn")[0]
    assert np.max(np.abs(got - cay * p.psi0)) <= 1e-15


def test_gpe_strang_over_2000_steps():
    """The condensate workload's first 2000 Strang steps (n = 4096, g = 10, tau = 1e-3):
    the oracle's psi against an all-extended-precision sweep, within 2e-14 (measured 2e-15
    here, 1.1e-14 over the full 10^4 steps).  Guard: the same sweep with FP64 numpy FFTs and
    FP64 kinetic factors drifts by more than 2e-13 (4e-12 measured; 1.9e-11 over 10^4 steps)."""
    from oracle import gpe as G
    p = problems.gpe()
    K = 2000
    x = X.gpe_psi_end(p, K)
    dx = p.L / p.n
    nrm = lambda f: float(np.sqrt(dx * np.sum(np.abs(f) ** 2)))
    psi, _ = G.strang_forward(p.psi0, p.u0[0, :K, 0], p.V0, p.V1, p.V2, p.g, p.L, p.T / p.K,
                              keep=False)
    assert nrm(psi - x) <= 2e-14, nrm(psi - x)
    _, k, _ = G.grid(p.n, p.L)
    half = np.exp(-1j * (p.T / p.K) * k ** 2 / 4)
    f = np.array(p.psi0, dtype=complex)
    tau = p.T / p.K
    for j in range(K):
        a = np.fft.ifft(half * np.fft.fft(f))
        b = np.exp(-1j * tau * (G.potential(p.V0, p.V1, p.V2, p.u0[0, j, 0]) + p.g * np.abs(a) ** 2)) * a
        f = np.fft.ifft(half * np.fft.fft(b))
    assert nrm(f - x) > 2e-13, nrm(f - x)


def test_gpe_plain_fp64_drift_full_size(monkeypatch):
    """The FP64 budget of the condensate workload at its full size (n = 4096, K = 10^4): the
    same method evaluated in plain FP64 (numpy's FFT, FP64 kinetic factors) drifts from the
    oracle by 1.9e-11 on psi(T) and 5.9e-10 (relative) on the gradient.  Rounding of a slowly
    varying state is nearly the same at every one of the 4 x 10^4 transforms, so it adds up
    linearly.  These measured drifts are the full-size FP64 bars of the GPU condensate test:
    the GPU's FP64 path must be at least as accurate as a plain FP64 evaluation."""
    import os
    from oracle import gpe as G
    p = problems.gpe()
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "gpe_n4096_k10000.npz"))

    def kinetic_fp64(f, tau, k, sign=-1):
        return np.fft.ifft(np.exp(sign * 1j * tau * k ** 2 / 4) * np.fft.fft(f))

    monkeypatch.setattr(G, "_kinetic", kinetic_fp64)
    g, J, F, psiK = G.adjoint_gradient(p.psi0, p.target, p.u0[0, :, 0], p.V0, p.V1, p.V2, p.g,
                                       p.L, p.T)
    dx = p.L / p.n
    e_psi = float(np.sqrt(dx * np.sum(np.abs(psiK - ref["psiT"]) ** 2)))
    e_g = float(np.linalg.norm(g - ref["g"]) / np.linalg.norm(ref["g"]))
    assert 1.5e-11 <= e_psi <= 2.5e-11, e_psi
    assert 4e-10 <= e_g <= 8e-10, e_g
