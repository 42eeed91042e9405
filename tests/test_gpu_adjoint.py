"""GPU adjoint gradients of final surface populations (FP64, 3D).

Checked against (i) the oracle's tangent-mode gradient (an independent
forward-mode computation with the block-matrix Frechet derivative),
(ii) central finite differences of the GPU forward path (h = 1e-5 eV on the
coupling constants), (iii) conservation of the norm (sum_s dP_s/dtheta = 0)
and (iv) independence of the checkpoint interval K.
"""
import sys

import numpy as np
import pytest

from paper_1903_04946_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_04946_amd import soprop
    soprop.lib()
    return torch


def base_model(n):
    """LVC model with theta = (lambda12 on mode 1, lambda13 on mode 2,
    lambda23 on mode 3); vtable holds V at theta = 0 and dvtables dV/dtheta
    (per eV)."""
    m = synth.lvc_3d(n=n, dv_params=True)
    theta0 = np.array([c[3] for c in m.meta["couplings"]])
    v0 = synth.lvc_vtable_theta(m, np.zeros(3))
    return m, theta0, v0


def make_plan(torch, m, v0, comp, order, dt):
    from paper_1903_04946_amd import soprop
    return soprop.Plan(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, v0, comp=comp, order=order, dt=dt,
                       dvtables=m.dvtables)


@pytest.mark.parametrize("comp,order,nsteps,K", [("triple_jump", 4, 3, 1), ("triple_jump", 4, 3, 2),
                                                 ("suzuki", 4, 2, 5), ("strang", 2, 6, 4)])
def test_adjoint_vs_oracle_tangent(torch_cuda, orc, comp, order, nsteps, K):
    torch = torch_cuda
    m, theta0, v0 = base_model(32)
    plan = make_plan(torch, m, v0, comp, order, 10.0)
    plan.set_params(theta0)
    psi0 = torch.from_numpy(m.psi0).cuda()
    ws = plan.adjoint_workspace(nsteps, K)
    w = np.array([0.2, -0.5, 1.0])
    pops = plan.adjoint_forward(psi0, nsteps, K, ws)
    grad = plan.adjoint_backward(nsteps, K, w, ws)
    P = orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, synth.lvc_vtable_theta(m, theta0))
    cid = {"strang": 0, "triple_jump": 1, "suzuki": 2}[comp]
    opops, ograd = orc.gradient(P, m.dvtables, m.psi0, orc.VTV, cid, order, 10.0, nsteps, w)
    print(f"[adjoint] gpu grad {grad} oracle {ograd}")
    np.testing.assert_allclose(pops, opops, rtol=0, atol=1e-12)
    assert np.max(np.abs(grad - ograd)) < 1e-10 * max(1.0, np.max(np.abs(ograd)))
    # the single call gives the same two sweeps
    pops1, grad1 = plan.adjoint(psi0, nsteps, K, w, ws)
    np.testing.assert_array_equal(pops1, pops)
    np.testing.assert_array_equal(grad1, grad)


def test_adjoint_norm_and_k_independence(torch_cuda):
    torch = torch_cuda
    m, theta0, v0 = base_model(64)
    plan = make_plan(torch, m, v0, "suzuki", 4, 10.0)
    plan.set_params(theta0)
    psi0 = torch.from_numpy(m.psi0).cuda()
    grads = []
    for K in (1, 3, 8):
        ws = plan.adjoint_workspace(8, K)
        plan.adjoint_forward(psi0, 8, K, ws)
        grads.append(plan.adjoint_backward(8, K, [0, 0, 1.0], ws))
    for g in grads[1:]:
        assert np.max(np.abs(g - grads[0])) < 1e-11 * max(1.0, np.max(np.abs(grads[0])))
    ws = plan.adjoint_workspace(8, 3)
    plan.adjoint_forward(psi0, 8, 3, ws)
    gn = plan.adjoint_backward(8, 3, [1.0, 1.0, 1.0], ws)
    assert np.max(np.abs(gn)) < 1e-11


def test_adjoint_vs_finite_differences_128(torch_cuda):
    """128^3 x 3, TJ-6, dt = 10: gradient of P_3 vs central differences with
    h = 1e-5 eV."""
    torch = torch_cuda
    m, theta0, v0 = base_model(128)
    nsteps, K = 6, 2
    plan = make_plan(torch, m, v0, "triple_jump", 6, 10.0)
    psi0 = torch.from_numpy(m.psi0).cuda()
    plan.set_params(theta0)
    ws = plan.adjoint_workspace(nsteps, K)
    plan.adjoint_forward(psi0, nsteps, K, ws)
    grad = plan.adjoint_backward(nsteps, K, [0, 0, 1.0], ws)
    h = 1e-5
    fd = np.zeros(3)
    for k in range(3):
        vals = []
        for sgn in (1, -1):
            th = theta0.copy()
            th[k] += sgn * h
            plan.set_params(th)
            vals.append(plan.adjoint_forward(psi0, nsteps, K, ws)[2])
        fd[k] = (vals[0] - vals[1]) / (2 * h)
    print(f"[adjoint 128^3] grad {grad} fd {fd}")
    assert np.max(np.abs(grad - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd)))


@pytest.mark.timeout(300)
def test_adjoint_config5_500_steps_k50(torch_cuda):
    """The full adjoint configuration at 128^3 x 3: TJ-6, dt = 10, 500 steps,
    checkpoints every K = 50 steps, so that ten reconstructions by time
    reversibility (Appendix A) each run 50 steps backwards before a stored
    state replaces the recomputed one.  Gradient of P_3 against central
    differences (h = 1e-5 eV) within 1e-6 relative, and the gradient of the
    total norm vanishes (sum_s dP_s/dtheta = 0)."""
    torch = torch_cuda
    m, theta0, v0 = base_model(128)
    nsteps, K = 500, 50
    plan = make_plan(torch, m, v0, "triple_jump", 6, 10.0)
    psi0 = torch.from_numpy(m.psi0).cuda()
    plan.set_params(theta0)
    ws = plan.adjoint_workspace(nsteps, K)
    pops = plan.adjoint_forward(psi0, nsteps, K, ws)
    grad = plan.adjoint_backward(nsteps, K, [0, 0, 1.0], ws)
    print(f"[adjoint 128^3 x 500] pops {pops}", flush=True)
    plan.adjoint_forward(psi0, nsteps, K, ws)
    gn = plan.adjoint_backward(nsteps, K, [1.0, 1.0, 1.0], ws)
    h = 1e-5
    fd = np.zeros(3)
    for k in range(3):
        vals = []
        for sgn in (1, -1):
            th = theta0.copy()
            th[k] += sgn * h
            plan.set_params(th)
            vals.append(plan.adjoint_forward(psi0, nsteps, K, ws)[2])
        fd[k] = (vals[0] - vals[1]) / (2 * h)
        print(f"[adjoint 128^3 x 500] theta_{k}: grad {grad[k]:.12e} fd {fd[k]:.12e}",
              flush=True)
    print(f"[adjoint 128^3 x 500] norm gradient {gn}")
    assert np.max(np.abs(gn)) < 1e-10 * max(1.0, np.max(np.abs(grad)))
    assert np.max(np.abs(grad - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd)))
    assert np.all(np.abs(fd) > 0)


def test_adjoint_256_bench_shape(torch_cuda):
    """256^3 x 3, TJ-6, dt = 10 (the largest adjoint configuration, at the
    bench's launch shape): gradient of P_3 vs central differences (h = 1e-5
    eV) and the conservation of the total norm (sum_s dP_s/dtheta = 0)."""
    torch = torch_cuda
    m, theta0, v0 = base_model(256)
    nsteps, K = 3, 2
    plan = make_plan(torch, m, v0, "triple_jump", 6, 10.0)
    psi0 = torch.from_numpy(m.psi0).cuda()
    plan.set_params(theta0)
    ws = plan.adjoint_workspace(nsteps, K)
    plan.adjoint_forward(psi0, nsteps, K, ws)
    grad = plan.adjoint_backward(nsteps, K, [0, 0, 1.0], ws)
    plan.adjoint_forward(psi0, nsteps, K, ws)
    gn = plan.adjoint_backward(nsteps, K, [1.0, 1.0, 1.0], ws)
    assert np.max(np.abs(gn)) < 1e-11
    h = 1e-5
    fd = np.zeros(3)
    for k in range(3):
        vals = []
        for sgn in (1, -1):
            th = theta0.copy()
            th[k] += sgn * h
            plan.set_params(th)
            vals.append(plan.adjoint_forward(psi0, nsteps, K, ws)[2])
        fd[k] = (vals[0] - vals[1]) / (2 * h)
    print(f"[adjoint 256^3] grad {grad} fd {fd}")
    assert np.max(np.abs(grad - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_populations_autograd(torch_cuda):
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    m, theta0, v0 = base_model(32)
    plan = make_plan(torch, m, v0, "triple_jump", 4, 10.0)
    psi0 = torch.from_numpy(m.psi0).cuda()
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    pops = soprop.PopulationsFn.apply(theta, plan, psi0, 3, 2)
    loss = pops[2] - 0.3 * pops[1]
    loss.backward()
    ws = plan.adjoint_workspace(3, 2)
    plan.set_params(theta0)
    plan.adjoint_forward(psi0, 3, 2, ws)
    ref = plan.adjoint_backward(3, 2, [0.0, -0.3, 1.0], ws)
    np.testing.assert_allclose(theta.grad.numpy(), ref, rtol=0, atol=1e-14)


def sub_model(n, surfaces):
    """The LVC model restricted to the given surfaces (the diabatic block of
    V and of dV/dtheta), with the initial packet moved onto the last of them
    and, for one surface, a parameter table of its own (D = q_3 on the
    diagonal), since the couplings have no diagonal part."""
    m, theta0, _ = base_model(n)
    full = synth.lvc_vtable_theta(m, theta0)
    idx = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    pairs = [(a, b) for i, a in enumerate(surfaces) for b in surfaces[i:]]
    rows = [idx[(min(a, b), max(a, b))] for a, b in pairs]
    vt = np.ascontiguousarray(full[rows])
    if len(surfaces) == 1:
        n2 = m.n[2]
        x = m.lo[2] + np.arange(n2) * ((m.hi[2] - m.lo[2]) / n2)
        q3 = np.broadcast_to(x[None, None, :], (m.n[0], m.n[1], n2)).ravel()
        dv = np.ascontiguousarray(0.01 * q3[None, None, :])
    else:
        dv = np.ascontiguousarray(m.dvtables[:, rows, :])
    psi0 = np.zeros((len(surfaces),) + m.psi0.shape[1:], dtype=np.complex128)
    psi0[-1] = m.psi0[2]
    return m, vt, dv, psi0


@pytest.mark.parametrize("surfaces", [(1, 2), (0, 2), (2,)])
def test_adjoint_fewer_surfaces_vs_oracle_tangent(torch_cuda, orc, surfaces):
    """Two surfaces (the compact eigen form's rotation angle) and one surface
    against the oracle's tangent-mode gradient."""
    from paper_1903_04946_amd import soprop
    torch = torch_cuda
    m, vt, dv, psi0 = sub_model(32, surfaces)
    S = len(surfaces)
    nsteps, K = 3, 2
    plan = soprop.Plan(m.n, m.lo, m.hi, S, m.inv_mass, vt, comp="triple_jump", order=4, dt=10.0,
                       dvtables=dv)
    ws = plan.adjoint_workspace(nsteps, K)
    w = np.array([0.3, -0.7][:S]) if S == 2 else np.array([1.0])
    pops, grad = plan.adjoint(torch.from_numpy(psi0).cuda(), nsteps, K, w, ws)
    P = orc.Problem(m.n, m.lo, m.hi, S, m.inv_mass, vt)
    opops, ograd = orc.gradient(P, dv, psi0, orc.VTV, 1, 4, 10.0, nsteps, w)
    print(f"[adjoint S={S}] gpu grad {grad} oracle {ograd}")
    np.testing.assert_allclose(pops, opops, rtol=0, atol=1e-12)
    assert np.max(np.abs(grad - ograd)) < 1e-10 * max(1.0, np.max(np.abs(ograd)))
    if S == 2:
        assert np.max(np.abs(ograd)) > 1e-6  # the couplings move population
