"""Extended-precision reference trajectories for the long-trajectory pins.

The arithmetic is x87 extended precision (numpy.longdouble, 64-bit significand, unit
roundoff 5.4e-20), so the rounding of a 20000-step trajectory stays near 1e-15 and the
result serves as the exact value against which the FP64 oracle's accumulated rounding is
measured.  Two step maps, both of the piecewise-constant Hamiltonian
H_j = diag(h0) + u_j Hc with Hc real, symmetric and tridiagonal (the rotor):

* exponential (Eq. (dir) with the control held on the step): exp(-i tau H_j) applied to the
  state by its power series, summed until a term falls below 1e-25;
* Crank-Nicolson (Sec. 3): (I + L_j) psi_{j+1} = (I - L_j) psi_j, L_j = (i tau/2) H_j,
  solved by tridiagonal elimination.

and the condensate's Strang splitting (Eq. (OS)) with extended-precision transforms.

Only tests import this module.
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble
CLD = np.clongdouble


def _coeffs(p, idx):
    d = p.d
    hd = np.stack([np.real(np.diag(p.H0_of(b))) for b in idx]).astype(LD)      # (B, d)
    C = np.real(p.Hc[0]).astype(LD)
    off = np.array([C[r, r + 1] for r in range(d - 1)], dtype=LD)              # (d-1,)
    if np.max(np.abs(np.real(p.Hc[0]) - np.diag(off, 1) - np.diag(off, -1))) != 0:
        raise ValueError("control operator must be real symmetric tridiagonal with zero diagonal")
    return hd, off, p.u0[idx, :, 0].astype(LD)


def _hx(hd, e, x):
    y = hd * x
    y[:, :-1] += e * x[:, 1:]
    y[:, 1:] += e * x[:, :-1]
    return y


def trajectory_end(p, idx, backward: bool = False, step: str = "exp") -> np.ndarray:
    """psi_K from psi0 (backward=False) or lambda_0 from the target (backward=True) for the
    instances idx, as complex128 (rounded once from the extended result)."""
    hd, off, u = _coeffs(p, idx)
    tau = LD(p.T / p.K)                 # the same FP64 step length both sides use
    x = np.zeros((len(idx), p.d), dtype=CLD)
    x[:] = np.asarray(p.target if backward else p.psi0).astype(CLD)
    sgn = LD(1) if backward else LD(-1)                 # exp(+/- i tau H)
    for j in (range(p.K - 1, -1, -1) if backward else range(p.K)):
        e = u[:, j][:, None] * off[None, :]
        if step == "exp":
            term = x.copy()
            acc = x.copy()
            for k in range(1, 60):
                term = _hx(hd, e, term) * (sgn * 1j * tau / LD(k))
                acc += term
                if np.max(np.abs(term)) < 1e-25:
                    break
            x = acc
        else:
            # forward: (I + a H) y = (I - a H) x with a = i tau/2; the adjoint step
            # U^dagger = (I - a H)^{-1} (I + a H) flips the sign of a
            a = (-sgn) * 1j * tau / 2
            rhs = x - a * _hx(hd, e, x)
            dg = 1 + a * hd
            of = a * e
            d = p.d
            cp = np.zeros((len(idx), d - 1), dtype=CLD)
            dp = np.zeros((len(idx), d), dtype=CLD)
            cp[:, 0] = of[:, 0] / dg[:, 0]
            dp[:, 0] = rhs[:, 0] / dg[:, 0]
            for r in range(1, d):
                den = dg[:, r] - of[:, r - 1] * cp[:, r - 1]
                if r < d - 1:
                    cp[:, r] = of[:, r] / den
                dp[:, r] = (rhs[:, r] - of[:, r - 1] * dp[:, r - 1]) / den
            y = np.empty_like(dp)
            y[:, -1] = dp[:, -1]
            for r in range(d - 2, -1, -1):
                y[:, r] = dp[:, r] - cp[:, r] * y[:, r + 1]
            x = y
    return x.astype(np.complex128)


def gpe_psi_end(p, K: int) -> np.ndarray:
    """psi_K of the condensate's Strang sweep (Eq. (OS)) over the first K steps of p's
    controls (instance 0), every operation in extended precision: the transforms by scipy's
    FFT on longdouble data, the kinetic factors e^{-i tau k^2/4} and the phases
    e^{-i tau (V + g|a|^2)} from the FP64 inputs (tau = T/K of p, the FP64 wavenumbers
    2 pi fftfreq(n, L/n), V0, V1, V2)."""
    import scipy.fft as sf
    n = p.n
    tau = LD(p.T / p.K)
    dx = p.L / n
    k = (2 * np.pi * np.fft.fftfreq(n, d=dx)).astype(LD)
    half = np.exp(-1j * tau * k * k / 4)
    V0, V1, V2 = p.V0.astype(LD), p.V1.astype(LD), LD(p.V2)
    u = p.u0[0, :K, 0].astype(LD)
    psi = np.asarray(p.psi0).astype(CLD)
    for j in range(K):
        a = sf.ifft(half * sf.fft(psi))
        V = V0 + u[j] * V1 + u[j] * u[j] * V2
        th = tau * (V + LD(p.g) * (a.real ** 2 + a.imag ** 2))
        psi = sf.ifft(half * sf.fft(np.exp(-1j * th) * a))
    return psi.astype(np.complex128)


def density_cn_end(p, K: int) -> np.ndarray:
    """rho_K of the Crank-Nicolson conjugation map over the first K steps of p's controls
    (instance 0): rho <- U rho U^dagger with U - I = 2 sum_{k>=1} (-L)^k, L = (i tau/2) H_j,
    the series summed to 11 terms (tau ||H|| / 2 ~ 1.5e-3 on the five-spin run, so the
    remainder is below 1e-30), every operation in extended precision (tau = T/K of p)."""
    H0 = np.asarray(p.H0).astype(CLD)
    Hc = np.asarray(p.Hc).astype(CLD)
    tau = LD(p.T) / LD(p.K)
    u = p.u0[0, :K].astype(LD)
    rho = np.asarray(p.psi0).astype(CLD)
    for j in range(K):
        H = H0.copy()
        for c in range(Hc.shape[0]):
            H = H + u[j, c] * Hc[c]
        L = (0.5j * tau) * H
        term = -L
        D = 2 * term
        for _ in range(10):
            term = -(term @ L)
            D = D + 2 * term
        Dh = D.conj().T
        rho = rho + (D @ rho + rho @ Dh) + D @ rho @ Dh
    return rho.astype(np.complex128)
