"""Pins of the Newton slice solver oracle (oracle/newton.py; Sec. 4.B, one matrix-free
Newton step with GMRES per slice problem).

  * GMRES: with as many steps as unknowns it equals a direct solve (numpy.linalg.solve) of
    an explicit nonsymmetric system, and with fewer steps its residual is the smallest over
    the Krylov space (checked against a least-squares solve over an explicit Krylov basis);
  * the difference Jacobian of the slice gradient, assembled column by column on a small
    slice problem, is symmetric and equals the second differences of the slice functional
    J_n itself (subproblem_objective, a function of values only), scaled by beta_n / tau;
  * Newton's step converges quadratically near a maximum of a slice problem;
  * with N = 1 the slice problem is the whole problem: one iteration equals a Newton-GMRES
    step on the plain gradient of finite.gradient.
"""
import numpy as np
import pytest

import problems
from oracle import finite as O
from oracle import newton as NW


def test_gmres_full_dimension_is_a_direct_solve():
    rng = np.random.default_rng(1)
    n = 12
    A = rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n)
    x = NW.gmres(lambda v: A @ v, b, n)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-11


def test_gmres_minimises_the_residual_over_the_krylov_space():
    rng = np.random.default_rng(2)
    n, m = 20, 5
    A = rng.standard_normal((n, n)) + 3 * np.eye(n)
    b = rng.standard_normal(n)
    x = NW.gmres(lambda v: A @ v, b, m)
    Kr = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(m)], axis=1)
    Q, _ = np.linalg.qr(Kr)
    c = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
    best = Q @ c
    assert np.linalg.norm(A @ x - b) <= np.linalg.norm(A @ best - b) * (1 + 1e-9)
    assert np.linalg.norm(x - best) / np.linalg.norm(best) <= 1e-8


def _small_slice():
    p = problems.spin2(K=6, N=2, T=1.0, seed=4)
    u = p.u0[0] + 0.3 * np.random.default_rng(3).standard_normal(p.u0[0].shape)
    s = O.slice_starts(p.K, p.N)
    tau = p.T / p.K
    Psi, Lam = O.boundaries(O.assemble(O.step_unitaries(p.H0, p.Hc, u, tau), s), p.psi0, p.target)
    phi = O.intermediate_states(Psi, Lam, s, p.K)
    return p, u, s, phi


def test_difference_jacobian_is_the_hessian_of_the_slice_functional():
    p, u, s, phi = _small_slice()
    n, sn, sn1 = 0, s[0], s[1]
    shape = u[sn:sn1].shape
    beta = p.K / (sn1 - sn)
    tau = p.T / p.K

    def grad_fn(flat):
        w = np.array(u, copy=True)
        w[sn:sn1] = flat.reshape(shape)
        return O.subproblem_gradient(p.H0, p.Hc, w, p.alpha, phi[n], phi[n + 1], sn, sn1, p.T).ravel()

    def jn(flat):
        w = np.array(u, copy=True)
        w[sn:sn1] = flat.reshape(shape)
        return O.subproblem_objective(p.H0, p.Hc, w, p.alpha, phi[n], phi[n + 1], sn, sn1, p.T)

    un = u[sn:sn1].ravel()
    dim = un.size
    A = np.stack([NW.slice_hvp(grad_fn, un, e, 1e-5) for e in np.eye(dim)], axis=1)
    assert np.max(np.abs(A - A.T)) <= 1e-8 * np.max(np.abs(A))
    h = 1e-3
    Hs = np.zeros((dim, dim))
    E = np.eye(dim) * h
    for i in range(dim):
        for k in range(dim):
            Hs[i, k] = (jn(un + E[i] + E[k]) - jn(un + E[i] - E[k]) - jn(un - E[i] + E[k])
                        + jn(un - E[i] - E[k])) / (4 * h * h)
    Hs *= beta / tau
    assert np.max(np.abs(A - Hs)) <= 1e-5 * np.max(np.abs(Hs))


def test_newton_step_converges_quadratically_on_a_slice_problem():
    """Slice 0 of a two-spin problem, full-dimension GMRES (Newton up to the difference
    quotient): the gradient norm falls 6.5e-3, 7.6e-5, 3.1e-9, 1.6e-15 in its last steps,
    each below a constant times the square of the previous one (a linear rate with the
    ratio 7.6e-5 / 6.5e-3 would leave 9e-7 after the third)."""
    p, u, s, phi = _small_slice()
    n, sn, sn1 = 0, s[0], s[1]
    w = np.array(u, copy=True)
    norms = []
    for _ in range(8):
        g = O.subproblem_gradient(p.H0, p.Hc, w, p.alpha, phi[n], phi[n + 1], sn, sn1, p.T)
        norms.append(float(np.linalg.norm(g)))
        d = NW.newton_slice_step(p.H0, p.Hc, w, p.alpha, phi[n], phi[n + 1], sn, sn1, p.T,
                                 m=g.size, eps=1e-5)
        w[sn:sn1] += d
    assert norms[4] < 1e-2
    for k in (4, 5):
        assert norms[k + 1] <= 100 * norms[k] ** 2
    assert norms[6] <= 1e-7 and norms[7] <= 1e-12


def test_one_slice_is_a_newton_step_on_the_whole_problem():
    p = problems.spin2(K=40, N=1, T=2.0, seed=9)
    u0 = p.u0[0]
    r = NW.ism_newton_iterate(p.H0, p.Hc, p.psi0, p.target, u0, p.T, p.alpha, 1, 1, 6)

    def g_fn(flat):
        return O.gradient(p.H0, p.Hc, p.psi0, p.target, flat.reshape(u0.shape), p.T,
                          p.alpha)[0].ravel()

    g = g_fn(u0.ravel())
    d = NW.gmres(lambda v: NW.slice_hvp(g_fn, u0.ravel(), v, 1e-5), -g, 6)
    assert np.max(np.abs(r["u"] - (u0 + d.reshape(u0.shape)))) <= 1e-12


def test_newton_ism_converges_where_the_paper_says():
    """Sec. 4.B: the Newton slice solver fails for N = 1 and converges for larger N.  On the
    two-spin problem (T = 2) one slice stalls near J = 0, while eight slices reach
    F > 0.99 in six iterations."""
    p = problems.spin2(K=200, N=8, T=2.0)
    r8 = NW.ism_newton_iterate(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 6, 8, 10)
    r1 = NW.ism_newton_iterate(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha, 6, 1, 10)
    assert r8["F"][-1] > 0.99
    assert abs(r1["J"][-1]) < 1e-3
