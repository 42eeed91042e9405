"""The allocation-free trapezoid entry point (sop_propagate_trapezoid_noalloc)
against the allocating one (sop_propagate_trapezoid), called through the C
ABI: the same kernel on the same inputs, so bitwise equal results and equal
iteration counts, on two calls in a row (the second with a smaller input, on
another plan), and a refusal, before any device work, of a workspace larger
than the static scratch."""
import ctypes
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


def states(m, count):
    x = m.axes()[0]
    return np.stack([m.psi0 * np.exp(1j * 0.5 * i * x) for i in range(count)])


def call(L, name, plan, psi, count, nsteps, tol=1e-13, max_iter=10000):
    it = ctypes.c_int64(-1)
    rc = getattr(L, name)(plan._h, ctypes.c_void_p(psi.data_ptr()), int(count), int(nsteps),
                          float(tol), int(max_iter), ctypes.byref(it))
    return rc, int(it.value)


def test_noalloc_equals_allocating_entry_point(torch_cuda):
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    L = soprop.lib()
    cases = [  # (grid, surfaces, scheme, order, count, steps): the second is smaller
        (1024, 2, "triple_jump", 4, 6, 2),
        (512, 1, "suzuki", 4, 2, 3),
    ]
    for n, S, comp, order, count, nsteps in cases:
        m = synth.random_small([n], S, seed=11 + n, lo=-8, hi=8, coupling=0.4)
        plan = soprop.Plan.from_model(m, comp=comp, order=order, dt=0.05 * (512 / n) ** 2)
        init = states(m, count)
        a = torch.from_numpy(init.copy()).cuda()
        b = torch.from_numpy(init.copy()).cuda()
        rc_a, it_a = call(L, "sop_propagate_trapezoid_noalloc", plan, a, count, nsteps)
        assert rc_a == 0, L.sop_last_error()
        rc_b, it_b = call(L, "sop_propagate_trapezoid", plan, b, count, nsteps)
        assert rc_b == 0, L.sop_last_error()
        torch.cuda.synchronize()
        print(f"[noalloc] n={n} S={S} {comp}-{order} count={count}: {it_a} iterations", flush=True)
        assert it_a == it_b and it_a >= count * nsteps
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        assert not np.array_equal(a.cpu().numpy(), init)
        plan.close()


def test_noalloc_refuses_more_than_its_scratch(torch_cuda):
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    L = soprop.lib()
    m = synth.random_small([8192], 2, seed=3, lo=-40, hi=40, coupling=0.4)
    plan = soprop.Plan.from_model(m, comp="strang", order=2, dt=0.05)
    count = 128  # 128 x 2 x 8192 x 16 B = 32 MiB of residuals alone
    init = states(m, count)
    psi = torch.from_numpy(init.copy()).cuda()
    rc, it = call(L, "sop_propagate_trapezoid_noalloc", plan, psi, count, 1)
    assert rc == 1  # SOP_ERR_INVALID
    assert b"static scratch" in L.sop_last_error()
    assert it == -1  # out-parameter untouched
    np.testing.assert_array_equal(psi.cpu().numpy(), init)
    plan.close()
