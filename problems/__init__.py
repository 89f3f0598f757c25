"""Seeded synthetic inputs for the ISM hot path.

This module only *generates problem data*: Hamiltonians, initial and target
states, initial controls.  It holds none of the method's arithmetic (no
propagation, no gradient, no ISM step), so both the FP64 oracle and the HIP
path can read the same inputs without sharing any computation.

Every generator takes an explicit seed and uses NumPy's PCG64
(``numpy.random.default_rng``).  Complex arrays are complex128, row-major.

Workloads (shapes follow the paper's three benchmarks, Sec. 4):

* ``spin2``       two coupled spin-1/2 (d=4), state transfer |00> -> |11>.
                  Stand-in for the coupled-spin benchmark (Sec. 4.A).
* ``rotor``       batch of rigid rotors (m=0, j=0..jmax), H = B j(j+1) - u cos(theta).
                  Stand-in for molecular orientation (Sec. 4.B); the target is the
                  top eigenvector of cos(theta) restricted to j <= 4, as in the paper.
* ``spin_chain_gate`` / ``spin_chain_state``  open Ising chain with per-spin x/y
                  controls; gate synthesis towards a Haar-random unitary, or state
                  transfer |0..0> -> |1..1>.
* ``spin5_density`` five coupled spin-1/2 in the density-matrix formalism with the
                  coupling topology of Sec. 4.A, I_x^(1) -> I_x^(5).
* ``gpe``         1-D Gross-Pitaevskii problem with a moving harmonic trap;
                  initial and target states are imaginary-time ground states
                  (Sec. 4.C uses ground states of the trap Hamiltonians as well).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "FiniteProblem", "GpeProblem", "pauli", "kron_chain", "haar_unitary",
    "spin2", "rotor", "rotor_cos_matrix", "rotor_target", "spin_chain_gate",
    "spin_chain_state", "spin5_density", "spin_operators", "gpe", "gpe_grid", "gpe_ground_state", "serving_trace",
    "slice_starts",
]


@dataclass
class FiniteProblem:
    """A finite-dimensional control problem i d/dt psi = (H0 + sum_c u_c Hc) psi.

    H0 has shape (batch, d, d) (one per instance) or (d, d) (shared);
    Hc has shape (C, d, d); psi0/target have shape (d,) for state transfer or
    (d, d) for gate synthesis (kind == "gate") and for density matrices (kind == "density");
    u0 has shape (batch, K, C).
    alpha is an array of shape (K,) (penalty weight per step, Eq. for J).
    """
    name: str
    H0: np.ndarray
    Hc: np.ndarray
    psi0: np.ndarray
    target: np.ndarray
    T: float
    K: int
    N: int
    u0: np.ndarray
    alpha: np.ndarray
    rho: float
    iters: int
    kind: str = "state"
    meta: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return self.Hc.shape[-1]

    @property
    def C(self) -> int:
        return self.Hc.shape[0]

    @property
    def batch(self) -> int:
        return self.u0.shape[0]

    def H0_of(self, b: int) -> np.ndarray:
        return self.H0[b] if self.H0.ndim == 3 else self.H0


@dataclass
class GpeProblem:
    """1-D GPE  i d/dt psi = (-1/2 d_xx + V(x,u) + g|psi|^2) psi on a periodic grid.

    V(x,u) = V0(x) + u V1(x) + u^2 V2 (here the moving trap (x-u)^2/2).
    """
    name: str
    n: int
    L: float
    g: float
    V0: np.ndarray
    V1: np.ndarray
    V2: float
    psi0: np.ndarray
    target: np.ndarray
    T: float
    K: int
    N: int
    u0: np.ndarray      # (batch, K, 1)
    rho: float
    iters: int
    meta: dict = field(default_factory=dict)

    @property
    def dx(self) -> float:
        return self.L / self.n

    @property
    def batch(self) -> int:
        return self.u0.shape[0]


def slice_starts(K: int, N: int) -> np.ndarray:
    """Slice start indices s_n = floor(n K / N), n = 0..N (uniform-as-possible partition)."""
    return np.array([(n * K) // N for n in range(N + 1)], dtype=np.int64)


# ----------------------------------------------------------------------------
# spin operators
# ----------------------------------------------------------------------------

def pauli() -> dict:
    sx = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    sy = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    sz = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    return {"x": sx, "y": sy, "z": sz, "i": np.eye(2, dtype=np.complex128)}


def kron_chain(ops) -> np.ndarray:
    out = np.array([[1.0 + 0j]])
    for o in ops:
        out = np.kron(out, o)
    return out


def embed(op: np.ndarray, site: int, n: int) -> np.ndarray:
    """Single-site operator acting on spin `site` of an n-spin register (site 0 = most significant)."""
    p = pauli()
    return kron_chain([op if k == site else p["i"] for k in range(n)])


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex Ginibre matrix with the phases of diag(R)
    divided out (Mezzadri, Notices AMS 54 (2007))."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


# ----------------------------------------------------------------------------
# coupled spins (stand-in for Sec. 4.A)
# ----------------------------------------------------------------------------

def spin2(seed: int = 1000, K: int = 1000, N: int = 8, T: float = 1.0,
          iters: int = 50, rho: float = 0.5) -> FiniteProblem:
    """Two coupled spin-1/2: H0 = (pi/2) sz(x)sz, controls on sx(x)I + I(x)sx and sy(x)I + I(x)sy.
    psi0 = |00>, target |11>, u0 = 0.1 + U(-0.01, 0.01) per (step, control), alpha = 0."""
    p = pauli()
    H0 = (math.pi / 2) * np.kron(p["z"], p["z"])
    Hx = np.kron(p["x"], p["i"]) + np.kron(p["i"], p["x"])
    Hy = np.kron(p["y"], p["i"]) + np.kron(p["i"], p["y"])
    psi0 = np.zeros(4, dtype=np.complex128); psi0[0] = 1
    tgt = np.zeros(4, dtype=np.complex128); tgt[3] = 1
    rng = np.random.default_rng(seed)
    u0 = 0.1 + rng.uniform(-0.01, 0.01, size=(1, K, 2))
    return FiniteProblem("spin2", H0, np.stack([Hx, Hy]), psi0, tgt, T, K, N, u0,
                         np.zeros(K), rho, iters)


# ----------------------------------------------------------------------------
# rigid rotor (stand-in for Sec. 4.B)
# ----------------------------------------------------------------------------

def rotor_cos_matrix(jmax: int) -> np.ndarray:
    """cos(theta) in the |j, m=0> basis, j = 0..jmax: tridiagonal with
    <j+1|cos|j> = (j+1)/sqrt((2j+1)(2j+3))."""
    d = jmax + 1
    C = np.zeros((d, d))
    for j in range(d - 1):
        v = (j + 1) / math.sqrt((2 * j + 1) * (2 * j + 3))
        C[j, j + 1] = C[j + 1, j] = v
    return C


def rotor_target(jmax: int, jcut: int = 4) -> np.ndarray:
    """Eigenvector of cos(theta) with the largest eigenvalue inside j <= jcut, embedded
    in the full basis, sign fixed so that its j=0 component is positive (Sec. 4.B)."""
    C = rotor_cos_matrix(jmax)[: jcut + 1, : jcut + 1]
    w, v = np.linalg.eigh(C)
    vec = v[:, -1]
    if vec[0] < 0:
        vec = -vec
    out = np.zeros(jmax + 1, dtype=np.complex128)
    out[: jcut + 1] = vec
    return out


def rotor(seed: int = 1001, batch: int = 256, jmax: int = 20, T: float = 10.0,
          K: int = 20000, N: int = 128, iters: int = 10, rho: float = 1.0) -> FiniteProblem:
    """Batch of rotors H_b = B_b j(j+1) - u cos(theta), B_b ~ U(0.8, 1.2);
    psi0 = |0,0>, target = rotor_target; u0 = 1.0 + U(-0.01, 0.01)."""
    rng = np.random.default_rng(seed)
    d = jmax + 1
    Bs = rng.uniform(0.8, 1.2, size=batch)
    D = np.diag([j * (j + 1) for j in range(d)]).astype(np.float64)
    H0 = np.stack([B * D for B in Bs]).astype(np.complex128)
    Hc = (-rotor_cos_matrix(jmax))[None].astype(np.complex128)
    psi0 = np.zeros(d, dtype=np.complex128); psi0[0] = 1
    tgt = rotor_target(jmax)
    u0 = 1.0 + rng.uniform(-0.01, 0.01, size=(batch, K, 1))
    return FiniteProblem("rotor", H0, Hc, psi0, tgt, T, K, N, u0, np.zeros(K), rho, iters,
                         meta={"B": Bs, "cos": rotor_cos_matrix(jmax)})


# ----------------------------------------------------------------------------
# Ising spin chain (gate synthesis / state transfer)
# ----------------------------------------------------------------------------

def _chain_ops(n: int, rng: np.random.Generator):
    p = pauli()
    J = rng.uniform(0.5, 1.5, size=n - 1)
    d = 2 ** n
    H0 = np.zeros((d, d), dtype=np.complex128)
    for i in range(n - 1):
        H0 += J[i] * embed(p["z"], i, n) @ embed(p["z"], i + 1, n)
    Hc = []
    for i in range(n):
        Hc.append(embed(p["x"], i, n))
        Hc.append(embed(p["y"], i, n))
    return H0, np.stack(Hc), J


def spin_chain_gate(seed: int = 1002, n: int = 8, T: float = 20.0, K: int = 2000,
                    N: int = 64, iters: int = 5, rho: float = 0.5) -> FiniteProblem:
    """Open Ising chain H0 = sum_i J_i sz_i sz_{i+1}, J_i ~ U(0.5,1.5), controls sx_i, sy_i;
    the propagated object is the d x d evolution operator from the identity towards a
    Haar-random unitary W; u0 ~ U(-0.5, 0.5)."""
    rng = np.random.default_rng(seed)
    H0, Hc, J = _chain_ops(n, rng)
    d = 2 ** n
    W = haar_unitary(d, rng)
    u0 = rng.uniform(-0.5, 0.5, size=(1, K, 2 * n))
    return FiniteProblem("spin_chain_gate", H0, Hc, np.eye(d, dtype=np.complex128), W,
                         T, K, N, u0, np.zeros(K), rho, iters, kind="gate", meta={"J": J})


def banded_gate(seed: int = 1006, d: int = 160, K: int = 6, N: int = 2,
                T: float = 0.06) -> FiniteProblem:
    """Gate synthesis with a dimension that is no power of two: H0 Hermitian with a random
    diagonal U(-1, 1) and nearest-neighbour couplings U(0.5, 1.5) e^{i phi}; control 0 a real
    symmetric coupling of i and i+1 (weights U(0.5, 1)), control 1 an imaginary antisymmetric
    coupling of i and i+3; identity towards a Haar-random W; u0 ~ U(-0.5, 0.5)."""
    rng = np.random.default_rng(seed)
    H0 = np.diag(rng.uniform(-1, 1, d)).astype(np.complex128)
    cpl = rng.uniform(0.5, 1.5, d - 1) * np.exp(1j * rng.uniform(0, 2 * np.pi, d - 1))
    H0 += np.diag(cpl, 1) + np.diag(cpl.conj(), -1)
    w0 = rng.uniform(0.5, 1.0, d - 1)
    w1 = rng.uniform(0.5, 1.0, d - 3)
    Hc = np.zeros((2, d, d), dtype=np.complex128)
    Hc[0] = np.diag(w0, 1) + np.diag(w0, -1)
    Hc[1] = 1j * (np.diag(w1, 3) - np.diag(w1, -3))
    W = haar_unitary(d, rng)
    u0 = rng.uniform(-0.5, 0.5, size=(1, K, 2))
    return FiniteProblem("banded_gate", H0, Hc, np.eye(d, dtype=np.complex128), W, T, K, N, u0,
                         np.zeros(K), 0.5, 5, kind="gate")


def spin_chain_state(seed: int, n: int, T: float, K: int, N: int, iters: int = 200,
                     rho: float = 0.5) -> FiniteProblem:
    """Chain state transfer |0..0> -> |1..1> (same Hamiltonian family as the gate problem)."""
    rng = np.random.default_rng(seed)
    H0, Hc, J = _chain_ops(n, rng)
    d = 2 ** n
    psi0 = np.zeros(d, dtype=np.complex128); psi0[0] = 1
    tgt = np.zeros(d, dtype=np.complex128); tgt[-1] = 1
    u0 = 0.1 + rng.uniform(-0.01, 0.01, size=(1, K, 2 * n))
    return FiniteProblem("spin_chain_state", H0, Hc, psi0, tgt, T, K, N, u0, np.zeros(K),
                         rho, iters, meta={"J": J})


# ----------------------------------------------------------------------------
# five coupled spins, density matrices (Sec. 4.A)
# ----------------------------------------------------------------------------

SPIN5_BONDS = ((0, 1), (0, 2), (1, 2), (1, 4), (2, 3))   # J12, J13, J23, J25, J34 (0-based)


def spin_operators(n: int):
    """I_x^(k), I_y^(k), I_z^(k) = sigma/2 on spin k of an n-spin register."""
    p = pauli()
    return ([0.5 * embed(p["x"], k, n) for k in range(n)],
            [0.5 * embed(p["y"], k, n) for k in range(n)],
            [0.5 * embed(p["z"], k, n) for k in range(n)])


def spin5_density(seed: int = 1005, K: int = 2 ** 15, N: int = 8, Jp: float = 140.0,
                  T: Optional[float] = None, u_amp: float = 100.0, iters: int = 5,
                  rho: float = 1e4) -> FiniteProblem:
    """Five coupled spins: H0 = 2 pi Jp sum_{bonds} I_z^(a) I_z^(b) over the bonds 1-2, 1-3,
    2-3, 2-5, 3-4; controls u_x^k I_x^(k) + u_y^k I_y^(k) in the order (x1, y1, ..., x5, y5);
    density matrices rho(0) = I_x^(1), rho_f = I_x^(5); alpha = 0; constant step 1e4.
    T defaults to 10/Jp (the printed T = Jp/10 is read as 10/Jp); the paper's step count is
    2^15.  u0: a constant field u_amp on the five x controls plus U(-u_amp/10, u_amp/10) on
    every control (rad per unit time), so that the transfer and the gradient start far from
    zero."""
    Ix, Iy, Iz = spin_operators(5)
    H0 = np.zeros((32, 32), dtype=np.complex128)
    for a, b in SPIN5_BONDS:
        H0 += 2 * math.pi * Jp * (Iz[a] @ Iz[b])
    Hc = []
    for k in range(5):
        Hc.append(Ix[k])
        Hc.append(Iy[k])
    T = 10.0 / Jp if T is None else T
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-0.1 * u_amp, 0.1 * u_amp, size=(1, K, 10))
    u0[:, :, 0::2] += u_amp
    return FiniteProblem("spin5_density", H0, np.stack(Hc), Ix[0], Ix[4], T, K, N, u0,
                         np.zeros(K), rho, iters, kind="density", meta={"Jp": Jp})


# ----------------------------------------------------------------------------
# Gross-Pitaevskii (stand-in for Sec. 4.C)
# ----------------------------------------------------------------------------

def gpe_grid(n: int, L: float):
    """Periodic grid x_m = -L/2 + m L/n (endpoint excluded) and angular wavenumbers."""
    dx = L / n
    x = -L / 2 + dx * np.arange(n)
    k = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    return x, k, dx


def gpe_ground_state(n: int, L: float, g: float, x0: float, dtau: float = 1e-3,
                     tol: float = 1e-13, max_steps: int = 200000) -> np.ndarray:
    """Ground state of -1/2 d_xx + (x-x0)^2/2 + g|psi|^2 by imaginary-time split-step
    relaxation, renormalised every step (norm dx sum |psi|^2 = 1), phase real-positive.
    Input preparation only."""
    x, k, dx = gpe_grid(n, L)
    psi = np.exp(-0.5 * (x - x0) ** 2).astype(np.complex128)
    psi /= math.sqrt(dx * np.sum(np.abs(psi) ** 2))
    half = np.exp(-dtau * k ** 2 / 4)
    V = 0.5 * (x - x0) ** 2
    for _ in range(max_steps):
        a = np.fft.ifft(half * np.fft.fft(psi))
        a = np.exp(-dtau * (V + g * np.abs(a) ** 2)) * a
        new = np.fft.ifft(half * np.fft.fft(a))
        new /= math.sqrt(dx * np.sum(np.abs(new) ** 2))
        if np.linalg.norm(new - psi) < tol:
            psi = new
            break
        psi = new
    ph = psi[np.argmax(np.abs(psi))]
    psi = psi * (abs(ph) / ph)
    return psi


_GS_CACHE: dict = {}


def gpe(seed: int = 1003, n: int = 4096, L: float = 40.0, g: float = 10.0, dt: float = 1e-3,
        K: int = 10000, N: int = 64, x_init: float = 0.0, x_target: float = 5.0,
        batch: int = 1, iters: int = 10, rho: float = 0.1, gs_tol: float = 1e-13) -> GpeProblem:
    """Moving harmonic trap V(x,u) = (x-u)^2/2 = x^2/2 - u x + u^2/2, control u = trap centre.
    psi0 / target: ground states at x_init / x_target; u0 = x_target t/T + U(-0.01, 0.01)."""
    x, _, _ = gpe_grid(n, L)
    key = (n, L, g, gs_tol)
    if key + (x_init,) not in _GS_CACHE:
        _GS_CACHE[key + (x_init,)] = gpe_ground_state(n, L, g, x_init, tol=gs_tol)
    if key + (x_target,) not in _GS_CACHE:
        _GS_CACHE[key + (x_target,)] = gpe_ground_state(n, L, g, x_target, tol=gs_tol)
    psi0 = _GS_CACHE[key + (x_init,)]
    tgt = _GS_CACHE[key + (x_target,)]
    T = dt * K
    rng = np.random.default_rng(seed)
    t = (np.arange(K) + 0.5) * dt
    u0 = (x_target * t / T)[None, :, None] + rng.uniform(-0.01, 0.01, size=(batch, K, 1))
    return GpeProblem("gpe", n, L, g, 0.5 * x ** 2, -x.copy(), 0.5, psi0, tgt, T, K, N,
                      u0, rho, iters)


# ----------------------------------------------------------------------------
# serving trace
# ----------------------------------------------------------------------------

SERVE_STANDARD_K = (1000, 2000, 5000, 10000, 20000)
SERVE_STANDARD_N = (16, 32, 64, 128)


def serving_trace(seed: int = 1004, n_req: int = 2000, rate: float = 200.0,
                  shapes: str = "continuous"):
    """Poisson arrivals (exponential gaps, mean 1/rate) of solve requests with a seeded
    type and size: spin chains d in {4,16,64,256}, rotors jmax in {10,20,40},
    GPE grids {1024, 4096}.  shapes = "continuous": N uniform in [16,128], K log-uniform in
    [1000, 20000]; "standard": N and K drawn from the standard shapes SERVE_STANDARD_N and
    SERVE_STANDARD_K (requests of one type, size and shape can share a batched launch)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        typ = ["spin", "rotor", "gpe"][rng.integers(0, 3)]
        if shapes == "standard":
            N = int(SERVE_STANDARD_N[rng.integers(0, len(SERVE_STANDARD_N))])
            K = int(SERVE_STANDARD_K[rng.integers(0, len(SERVE_STANDARD_K))])
        else:
            N = int(rng.integers(16, 129))
            K = int(round(math.exp(rng.uniform(math.log(1000), math.log(20000)))))
        K = max(K, N)
        if typ == "spin":
            size = int([4, 16, 64, 256][rng.integers(0, 4)])
        elif typ == "rotor":
            size = int([10, 20, 40][rng.integers(0, 3)])
        else:
            size = int([1024, 4096][rng.integers(0, 2)])
        out.append({"id": i, "arrival": t, "type": typ, "size": size, "N": N, "K": K,
                    "seed": int(rng.integers(0, 2 ** 31))})
    return out


# per-type settings of a served solve: final time, gradient step
SERVE_RHO = {"spin": 0.5, "rotor": 1.0, "gpe": 0.1}


def request_problem(req: dict):
    """The problem of one serving-trace request (batch 1): spin d=4 is the two-spin
    system, d >= 16 the open chain with log2(d) spins (|0..0> -> |1..1>), both with T=2;
    rotors with T=10 and the j<=4 target; GPE with dt=1e-3 (T = K dt) and the x0=5
    ground-state target."""
    typ, size, K, N, seed = req["type"], req["size"], req["K"], req["N"], req["seed"]
    if typ == "spin":
        if size == 4:
            return spin2(seed=seed, K=K, N=N, T=2.0)
        return spin_chain_state(seed, n=int(round(math.log2(size))), T=2.0, K=K, N=N)
    if typ == "rotor":
        return rotor(seed=seed, batch=1, jmax=size, T=10.0, K=K, N=N)
    return gpe(seed=seed, n=size, K=K, N=N)
