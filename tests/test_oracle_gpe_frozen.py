"""Pins of the frozen-density propagator assembling oracle (oracle/gpe_frozen.py; the reading
of Sec. 4.C's propagator assembling for the condensate).

  * the frozen forward step S_j and adjoint step R_j, evaluated at the exact trajectory's
    a_j, reproduce the exact Strang step and the exact adjoint step of oracle/gpe.py;
  * with the exact trajectory's a_j, the assembled boundaries equal the sequential sweeps';
  * M_n is unitary, and A_n is the transpose of the nonlinear slice map's linearisation in
    the real inner product Re<.|.> (checked against its central difference);
  * the lagged iteration differs from the plain gradient method along the way and reaches
    the same fixed point (both stationary to 1e-13, controls equal to 1e-12).
"""
import numpy as np

import problems
from oracle import gpe as G
from oracle import gpe_frozen as FZ


def _small(K=64, N=4, T=1.0, x_target=1.0):
    return problems.gpe(n=32, L=20.0, g=1.0, dt=T / K, K=K, N=N, x_target=x_target)


def _args(p):
    return (p.psi0, p.target, p.u0[0, :, 0], p.V0, p.V1, p.V2, p.g, p.L, p.T)


def test_frozen_steps_at_the_exact_trajectory_are_the_exact_steps():
    p = _small()
    u = p.u0[0, :, 0]
    tau = p.T / p.K
    _, k, dx = G.grid(p.n, p.L)
    _, rec = G.strang_forward(p.psi0, u, p.V0, p.V1, p.V2, p.g, p.L, tau)
    rng = np.random.default_rng(2)
    for j in (0, 17, p.K - 1):
        V = G.potential(p.V0, p.V1, p.V2, u[j])
        nxt = FZ.frozen_forward_step(rec["psi"][j], rec["a"][j], k, V, p.g, tau)
        assert np.max(np.abs(nxt - rec["psi"][j + 1])) <= 1e-15
        nu = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
        ref, _ = G._adjoint_steps(nu, rec, u, p.V1, p.V2, p.g, p.L, tau, j, j + 1, dx)
        got = FZ.frozen_adjoint_step(nu, rec["a"][j], k, V, p.g, tau)
        assert np.max(np.abs(got - ref)) <= 1e-14


def test_exact_densities_give_the_sequential_boundaries():
    p = _small()
    u = p.u0[0, :, 0]
    tau = p.T / p.K
    s = [(i * p.K) // p.N for i in range(p.N + 1)]
    _, rec = G.strang_forward(p.psi0, u, p.V0, p.V1, p.V2, p.g, p.L, tau)
    Ms = FZ.assemble_forward(rec["a"], u, p.V0, p.V1, p.V2, p.g, p.L, tau, s)
    As = FZ.assemble_adjoint(rec["a"], u, p.V0, p.V1, p.V2, p.g, p.L, tau, s)
    Psi, Lam = FZ.frozen_boundaries(Ms, As, p.psi0, p.target)
    _, _, _, psi_b, nu_b = G.ism_bec_gradient(*_args(p), p.N)
    for i in range(p.N + 1):
        assert np.linalg.norm(Psi[i] - psi_b[i]) <= 1e-12 * np.linalg.norm(psi_b[i])
        assert np.linalg.norm(Lam[i] - nu_b[i]) <= 1e-12 * np.linalg.norm(nu_b[i])


def test_forward_map_unitary_and_adjoint_map_its_linearised_transpose():
    p = _small()
    u = p.u0[0, :, 0]
    tau = p.T / p.K
    s = [(i * p.K) // p.N for i in range(p.N + 1)]
    _, rec = G.strang_forward(p.psi0, u, p.V0, p.V1, p.V2, p.g, p.L, tau)
    Ms = FZ.assemble_forward(rec["a"], u, p.V0, p.V1, p.V2, p.g, p.L, tau, s)
    As = FZ.assemble_adjoint(rec["a"], u, p.V0, p.V1, p.V2, p.g, p.L, tau, s)
    n = p.n
    i = 1
    assert np.max(np.abs(Ms[i].conj().T @ Ms[i] - np.eye(n))) <= 1e-12
    lo, hi = s[i], s[i + 1]
    psi_n = rec["psi"][lo]

    def slice_map(x):
        end, _ = G.strang_forward(x, u[lo:hi], p.V0, p.V1, p.V2, p.g, p.L, tau, keep=False)
        return end

    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        nu = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        eps = 1e-6
        Dd = (slice_map(psi_n + eps * d) - slice_map(psi_n - eps * d)) / (2 * eps)
        lhs = np.vdot(FZ.apply_adjoint_map(As[i], nu), d).real
        rhs = np.vdot(nu, Dd).real
        assert abs(lhs - rhs) <= 1e-7 * max(abs(rhs), 1.0)


def test_lagged_iteration_reaches_the_plain_fixed_point():
    p = _small()
    u0 = p.u0[0, :, 0]
    args = _args(p)
    pl20 = G.plain_gradient_method(*args, 0.5, 20)
    fz20 = FZ.ism_bec_frozen_iterate(*args, 0.5, 20, p.N)
    # the lagged boundaries change the iterates (the exact BEC variant would not)
    assert np.linalg.norm(pl20["u"] - fz20["u"]) > 1e-6 * np.linalg.norm(pl20["u"] - u0)
    pl = G.plain_gradient_method(*args, 0.5, 80)
    fz = FZ.ism_bec_frozen_iterate(*args, 0.5, 80, p.N)
    for u in (pl["u"], fz["u"]):
        g = G.adjoint_gradient(p.psi0, p.target, u, p.V0, p.V1, p.V2, p.g, p.L, p.T)[0]
        assert np.linalg.norm(g) <= 1e-11
    assert np.linalg.norm(pl["u"] - fz["u"]) <= 1e-12 * np.linalg.norm(pl["u"] - u0)
