"""torch.autograd wrapper: the backward pass is the library's adjoint, checked by central
finite differences (torch.autograd.gradcheck) and against the oracle gradient."""
import sys

import numpy as np
import pytest

import problems
from oracle import finite as O

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _handle(p, prec="fp64"):
    from paper_1603_01237_amd import _lib
    return _lib.from_problem(p, precision=prec, io_device=True, set_u=False)


def test_gradcheck_state_fp64():
    import torch
    from paper_1603_01237_amd.autograd import ISMObjective
    _say("case gradcheck state")
    p = problems.spin2(K=6, N=3)
    h = _handle(p)
    u = torch.tensor(p.u0, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: ISMObjective.apply(x, h), (u,), eps=1e-6,
                                    atol=1e-8, rtol=1e-6)
    h.close()


def test_gradcheck_gate_fp64():
    import torch
    from paper_1603_01237_amd.autograd import ISMObjective
    _say("case gradcheck gate")
    rng = np.random.default_rng(4)
    base = problems.spin2(K=12, N=3)
    W = problems.haar_unitary(4, rng)
    p = problems.FiniteProblem("g", base.H0, base.Hc, np.eye(4, dtype=complex), W, 1.0, 12, 3,
                               rng.uniform(-1, 1, (1, 12, 2)), np.zeros(12), 0.5, 1, kind="gate")
    h = _handle(p)
    u = torch.tensor(p.u0, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: ISMObjective.apply(x, h), (u,), eps=1e-6,
                                    atol=1e-8, rtol=1e-6)
    h.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-3)])
def test_backward_matches_oracle(prec, tol):
    import torch
    from paper_1603_01237_amd.autograd import ISMObjective
    _say("case backward", prec)
    p = problems.rotor(batch=2, K=60, N=6, T=0.5)
    h = _handle(p, prec)
    u = torch.tensor(p.u0, dtype=torch.float64, device="cuda", requires_grad=True)
    J = ISMObjective.apply(u, h)
    (J * torch.tensor([1.0, -2.0], dtype=torch.float64, device="cuda")).sum().backward()
    gu = u.grad.cpu().numpy()
    tau = p.T / p.K
    for b, w in ((0, 1.0), (1, -2.0)):
        gr, Jr, _, _ = O.gradient(p.H0[b], p.Hc, p.psi0, p.target, p.u0[b], p.T, p.alpha)
        assert abs(J[b].item() - Jr) <= max(tol, 1e-4 if prec == "fp32" else 0)
        rel = np.linalg.norm(gu[b] - w * tau * gr) / np.linalg.norm(w * tau * gr)
        assert rel <= tol, rel
    h.close()


def test_handle_reuse_between_forward_and_backward():
    import torch
    from paper_1603_01237_amd.autograd import ISMObjective
    _say("case reuse")
    p = problems.spin2(K=20, N=4)
    h = _handle(p)
    u1 = torch.tensor(p.u0, dtype=torch.float64, device="cuda", requires_grad=True)
    u2 = torch.tensor(p.u0 * 1.5, dtype=torch.float64, device="cuda", requires_grad=True)
    J1 = ISMObjective.apply(u1, h)
    J2 = ISMObjective.apply(u2, h)       # the handle now holds u2
    J1.sum().backward()                  # must use u1
    J2.sum().backward()
    tau = p.T / p.K
    g1, *_ = O.gradient(p.H0, p.Hc, p.psi0, p.target, p.u0[0], p.T, p.alpha)
    g2, *_ = O.gradient(p.H0, p.Hc, p.psi0, p.target, 1.5 * p.u0[0], p.T, p.alpha)
    assert np.max(np.abs(u1.grad.cpu().numpy()[0] - tau * g1)) <= 1e-12
    assert np.max(np.abs(u2.grad.cpu().numpy()[0] - tau * g2)) <= 1e-12
    h.close()


def test_module_with_optimizer_improves_objective():
    import torch
    from paper_1603_01237_amd.autograd import ISMControl
    _say("case optimizer")
    p = problems.spin2(K=100, N=5)
    h = _handle(p)
    m = ISMControl(h, p.u0)
    opt = torch.optim.Adam(m.parameters(), lr=0.05)
    J0 = m().item()
    for _ in range(20):
        opt.zero_grad()
        loss = -m().sum()
        loss.backward()
        opt.step()
    J1 = m().item()
    assert J1 > J0 + 0.05
    h.close()


def test_forward_backward_under_a_side_stream():
    """Forward and backward issued under a non-default torch stream: the handle's stream is
    ordered against it both ways, so J and the gradient equal those computed on the default
    stream, bitwise; gradcheck passes under the side stream as well.  The controls are
    produced by a torch kernel on the side stream right before the call, so an unordered
    read would see stale values."""
    import torch
    from paper_1603_01237_amd.autograd import ISMObjective
    _say("case side stream")
    p = problems.rotor(batch=2, K=60, N=6, T=0.5)
    h = _handle(p)
    base = torch.tensor(p.u0, dtype=torch.float64, device="cuda")
    u_ref = base.clone().requires_grad_(True)
    J_ref = ISMObjective.apply(u_ref, h)
    J_ref.sum().backward()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for _ in range(3):
            u = base.clone().requires_grad_(True)     # written on the side stream
            J = ISMObjective.apply(u, h)
            J.sum().backward()
            assert torch.equal(J, J_ref) and torch.equal(u.grad, u_ref.grad)
        assert torch.autograd.gradcheck(lambda x: ISMObjective.apply(x, h),
                                        (base.clone().requires_grad_(True),), eps=1e-6,
                                        atol=1e-8, rtol=1e-6)
    torch.cuda.synchronize()
    h.close()


def test_autograd_gate_synthesis_full_size():
    """The gate-synthesis configuration with autograd (8-spin chain, d = 256, 16 controls,
    K = 2000, N = 64): backward through ISMObjective checked by a central finite difference
    of the forward J along a random direction (FP64, relative 1e-6; the difference step
    1e-4 leaves a truncation near 1e-9 of the directional derivative), and the FP32 mixed
    backward against the FP64 one (relative 1e-3)."""
    import torch
    from paper_1603_01237_amd.autograd import ISMObjective
    _say("case autograd gate d256")
    p = problems.spin_chain_gate()
    grads = {}
    for prec in ("fp64", "fp32"):
        h = _handle(p, prec)
        u = torch.tensor(p.u0, dtype=torch.float64, device="cuda", requires_grad=True)
        J = ISMObjective.apply(u, h)
        J.sum().backward()
        grads[prec] = u.grad.detach().clone()
        if prec == "fp64":
            v = torch.tensor(np.random.default_rng(8).standard_normal(p.u0.shape),
                             dtype=torch.float64, device="cuda")
            v = v / torch.linalg.vector_norm(v)
            eps = 1e-4
            with torch.no_grad():
                Jp = ISMObjective.apply(u.detach() + eps * v, h)
                Jm = ISMObjective.apply(u.detach() - eps * v, h)
            fd = ((Jp - Jm) / (2 * eps)).sum().item()
            an = (grads[prec] * v).sum().item()
            _say("directional", an, fd, abs(an - fd) / abs(fd))
            assert abs(an - fd) <= 1e-6 * abs(fd)
        h.close()
    rel = (torch.linalg.vector_norm(grads["fp32"] - grads["fp64"]) /
           torch.linalg.vector_norm(grads["fp64"])).item()
    _say("fp32 vs fp64 backward", rel)
    assert rel <= 1e-3
