"""GPU parity of sop_interpolate (trigonometric interpolation between grids,
Appendix B) against the oracle's plain interpolation, and at the benchmark's
full size (128^3 -> 256^3, three surfaces, range and density each grown by
sqrt(2)) against the closed form of a band-limited state.

Tolerance: 1e-12 relative L2 (FP64), as for the propagation parity tests.
"""
import sys

import numpy as np
import pytest

from paper_1903_04946_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
R2 = 2.0**0.5


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


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def plan_for(m, dtype=None):
    from paper_1903_04946_amd import soprop
    kw = {} if dtype is None else {"dtype": dtype}
    return soprop.Plan.from_model(m, comp="strang", order=2, dt=0.01, **kw)


def gpu_interp(torch, ma, psi, mb):
    from paper_1903_04946_amd import soprop
    pa, pb = plan_for(ma), plan_for(mb)
    src = torch.from_numpy(np.ascontiguousarray(psi)).cuda()
    dst = torch.full(pb.shape, complex("nan"), dtype=torch.complex128).cuda()
    soprop.interpolate(pa, src, pb, dst)
    torch.cuda.synchronize()
    return dst.cpu().numpy()


def oracle_interp(orc, psi, ma, mb):
    return orc.interpolate(psi, ma.n, ma.lo, ma.hi, mb.n, mb.lo, mb.hi)


@pytest.mark.parametrize("na,La,nb,Lb", [(64, 5.0, 128, 5.0 * R2), (1024, 10.0, 512, 9.0),
                                         (256, 6.0, 256, 7.5)])
def test_1d_against_oracle(torch_cuda, orc, na, La, nb, Lb):
    torch = torch_cuda
    ma = synth.random_small([na], 2, seed=3, lo=-La, hi=La)
    mb = synth.random_small([nb], 2, seed=4, lo=-Lb, hi=Lb)
    for psi in (ma.psi0, synth.random_state(ma.psi0.shape, seed=9)):
        got = gpu_interp(torch, ma, psi, mb)
        ref = oracle_interp(orc, psi, ma, mb)
        err = rel_l2(got, ref)
        print(f"[interp 1d {na}->{nb}] rel L2 {err:.2e}")
        assert err < TOL


@pytest.mark.parametrize("na,La,nb,lob,hib", [(32, 7.0, 48, -7.0 * R2, 7.0 * R2),
                                              (64, 7.0, 32, -6.0, 6.5),
                                              (48, 7.0, 64, -8.3, 5.1)])
def test_3d_against_oracle(torch_cuda, orc, na, La, nb, lob, hib):
    torch = torch_cuda
    ma = synth.lvc_3d(n=na, lo=-La, hi=La)
    mb = synth.lvc_3d(n=nb, lo=lob, hi=hib)
    for psi in (ma.psi0, synth.random_state(ma.psi0.shape, seed=11)):
        got = gpu_interp(torch, ma, psi, mb)
        ref = oracle_interp(orc, psi, ma, mb)
        err = rel_l2(got, ref)
        print(f"[interp 3d {na}->{nb}] rel L2 {err:.2e}")
        assert err < TOL


def test_equal_grids_identity(torch_cuda):
    torch = torch_cuda
    m = synth.lvc_3d(n=64)
    psi = synth.random_state(m.psi0.shape, seed=2)
    got = gpu_interp(torch, m, psi, m)
    assert rel_l2(got, psi) < 1e-13


def _trig(x, lo, hi, modes):
    return sum(a * np.exp(2j * np.pi * k * (x - lo) / (hi - lo)) for k, a in modes)


def test_bench_shape_band_limited_closed_form(torch_cuda):
    """128^3 -> 256^3 on a box sqrt(2) wider per axis (three surfaces): a
    separable band-limited state is interpolated exactly at every point
    inside the source box, and is zero outside it."""
    torch = torch_cuda
    ma = synth.lvc_3d(n=128, lo=-7.0, hi=7.0)
    mb = synth.lvc_3d(n=256, lo=-7.0 * R2, hi=7.0 * R2)
    modes = [[(1, 1.0), (-5, 0.3j), (63, 0.1)], [(0, 0.5), (7, -0.2)],
             [(-2, 0.4 + 0.1j), (30, 0.6), (-63, 0.05j)]]
    fa = [_trig(ma.axes()[a], ma.lo[a], ma.hi[a], modes[a]) for a in range(3)]
    psi = np.stack([np.einsum("i,j,k->ijk", *fa) * (s + 1) for s in range(3)])
    got = gpu_interp(torch, ma, psi, mb)
    fb = []
    for a in range(3):
        x = mb.axes()[a]
        fb.append(np.where((x >= ma.lo[a]) & (x < ma.hi[a]), _trig(x, ma.lo[a], ma.hi[a], modes[a]), 0))
    ref = np.einsum("i,j,k->ijk", *fb)
    worst = 0.0
    for s in range(3):
        worst = max(worst, rel_l2(got[s], ref * (s + 1)))
    print(f"[interp 128->256 closed form] rel L2 {worst:.2e}")
    assert worst < TOL


def test_refusals(torch_cuda):
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    ma = synth.lvc_3d(n=32)
    mb = synth.lvc_3d(n=48)
    pa, pb = plan_for(ma), plan_for(mb)
    x = torch.zeros(pa.shape, dtype=torch.complex128).cuda()
    with pytest.raises(soprop.SopError):  # same buffer in and out
        soprop.interpolate(pa, x, pa, x)
    pc = plan_for(ma, dtype=torch.complex64)
    y = torch.zeros(pc.shape, dtype=torch.complex64).cuda()
    with pytest.raises(soprop.SopError):  # FP32 plans are not supported
        soprop.interpolate(pc, y, pb, torch.zeros(pb.shape, dtype=torch.complex128).cuda())
    m1 = synth.random_small([64], 2, seed=1)
    p1 = plan_for(m1)
    with pytest.raises(soprop.SopError):  # ndim differs
        soprop.interpolate(p1, torch.zeros(p1.shape, dtype=torch.complex128).cuda(), pb,
                           torch.zeros(pb.shape, dtype=torch.complex128).cuda())


def test_matrices_follow_the_source_grid(torch_cuda, orc):
    """One destination plan fed from two source grids in turn: the kept axis
    matrices are formed again whenever the source grid changes."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    m1 = synth.lvc_3d(n=32, lo=-7.0, hi=7.0)
    m2 = synth.lvc_3d(n=32, lo=-6.0, hi=6.5)
    mb = synth.lvc_3d(n=48, lo=-8.0, hi=8.0)
    p1, p2, pb = plan_for(m1), plan_for(m2), plan_for(mb)
    psi = synth.random_state(m1.psi0.shape, seed=4)
    src = torch.from_numpy(psi).cuda()
    dst = torch.empty(pb.shape, dtype=torch.complex128).cuda()
    for p, m in ((p1, m1), (p2, m2), (p1, m1), (p1, m1)):
        soprop.interpolate(p, src, pb, dst)
        got = dst.cpu().numpy()
        ref = oracle_interp(orc, psi, m, mb)
        err = rel_l2(got, ref)
        print(f"[interp source switch] rel L2 {err:.2e}")
        assert err < TOL
