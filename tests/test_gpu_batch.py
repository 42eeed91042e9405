"""GPU parity of batches (sop_batch_*): many independent plans of uneven grid
sizes, orders, dt and step counts in one graph launch.

Every member is compared with the FP64 oracle at 1e-12 relative L2 and with
its own single-plan run: 3D members (the work-queue launch and the lockstep
passes share the single-plan pass bodies) bitwise, 1D members bitwise when
the tuner keeps the single-plan schedule and to 1e-12 otherwise (same DFTs,
other radix order).
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1903_04946_amd import synth
from parity import assert_parity

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
SPLIT_ID = {"VTV": 0, "TVT": 1, "VT": 2, "TV": 3}
COMP_ID = {"strang": 0, "triple_jump": 1, "suzuki": 2}


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


# (kind, n, S, split, comp, order, dt, nsteps, packet offset)
MIX = [
    ("1d", 512, 2, "VTV", "strang", 2, 0.03, 7, -1.0),
    ("1d", 1024, 2, "VTV", "triple_jump", 4, 0.02, 5, 0.5),
    ("1d", 2048, 2, "VTV", "suzuki", 4, 0.05, 3, -2.5),
    ("1d", 4096, 2, "VTV", "triple_jump", 6, 0.01, 2, 1.5),
    ("1d", 8192, 2, "VTV", "suzuki", 6, 0.04, 1, -0.5),
    ("1d", 1024, 2, "TVT", "triple_jump", 4, 0.02, 4, 0.0),
    ("1d", 1024, 2, "VTV", "strang", 2, 0.011, 0, 2.0),      # zero steps
    ("1d", 256, 1, "VTV", "suzuki", 4, 0.02, 3, 0.0),        # one surface
    ("3d", 32, 3, "VTV", "triple_jump", 4, 10.0, 2, 0.0),
    ("3d", 32, 3, "VTV", "strang", 2, 7.0, 3, 0.7),
    ("3d", 32, 3, "VTV", "suzuki", 4, 4.0, 0, 0.0),           # zero steps
    ("3d", 48, 3, "VTV", "suzuki", 4, 12.0, 1, -0.4),
    ("3d", 48, 3, "VTV", "strang", 2, 5.0, 2, 0.3),
    ("3d", 32, 3, "TVT", "triple_jump", 4, 10.0, 2, 0.0),     # own executor
    ("3d", 64, 1, "VTV", "strang", 2, 0.05, 2, 0.0),          # one surface, 64^3
    ("3d", 32, 2, "VTV", "triple_jump", 4, 0.05, 3, 0.0),     # two surfaces
]


def member_model(kind, n, S, off):
    if kind == "1d":
        if S == 2:
            return synth.two_surface_1d(n=n, x0=-2.0 + off, p0=0.5 * off)
        return synth.random_small([n], 1, seed=n, lo=-8, hi=8)
    if S == 3:
        return synth.lvc_3d(n=n, q0=(off, -off, 0.5 * off), p0=(0.3, -0.2, off))
    return synth.random_small([n, n, n], S, seed=n + S, lo=-6, hi=6)


def build_members(torch, dtype, mix=MIX):
    from paper_1903_04946_amd import soprop
    models, plans, ns = [], [], []
    for kind, n, S, split, comp, order, dt, nsteps, off in mix:
        m = member_model(kind, n, S, off)
        models.append(m)
        plans.append(soprop.Plan.from_model(m, split=split, comp=comp, order=order, dt=dt,
                                            dtype=dtype))
        ns.append(nsteps)
    return models, plans, ns


def states(torch, models, dtype):
    return [torch.from_numpy(np.ascontiguousarray(m.psi0)).to(dtype).cuda() for m in models]


def single_runs(torch, plans, models, ns, dtype, reps=1):
    out = []
    for p, m, k in zip(plans, models, ns):
        psi = torch.from_numpy(np.ascontiguousarray(m.psi0)).to(dtype).cuda()
        for _ in range(reps):
            p.propagate(psi, k)
        out.append(psi)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in out]


def check_vs_single(batch, got, ref, tol):
    """3D members and untuned 1D members bitwise; other 1D members to tol."""
    d = batch.describe()
    exact = set()
    for g in d["groups"]:
        exact.update(g["members"])
    exact.update(d["solo"])
    for f in d["families"]:
        if f["variant"] == 0:
            exact.update(f["members"])
    for i, (a, b) in enumerate(zip(got, ref)):
        if i in exact:
            np.testing.assert_array_equal(a, b, err_msg=f"member {i}")
        else:
            assert rel_l2(a, b) < tol, f"member {i}: {rel_l2(a, b):.2e}"


def test_batch_fp64_matches_oracle_and_single_runs(torch_cuda, orc):
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    models, plans, ns = build_members(torch, torch.complex128)
    batch = soprop.Batch(plans)
    d = batch.describe()
    print("[batch] " + json.dumps(d))
    # grouping: every 1D member in a family, 3D VTV members on 32/48/64 in
    # lockstep groups, the 3D TVT member on its own executor
    assert sorted(i for f in d["families"] for i in f["members"]) == \
        [i for i, r in enumerate(MIX) if r[0] == "1d"]
    assert d["solo"] == [i for i, r in enumerate(MIX) if r[0] == "3d" and r[3] == "TVT"]
    psis = states(torch, models, torch.complex128)
    batch.propagate(psis, ns)
    batch.check()
    assert batch.describe()["graph"]
    assert not any(g["queue"] for g in batch.describe()["groups"])
    got = [x.cpu().numpy() for x in psis]
    for i, ((kind, n, S, split, comp, order, dt, k, off), m) in enumerate(zip(MIX, models)):
        if k == 0:
            np.testing.assert_array_equal(got[i], m.psi0.astype(got[i].dtype))
            continue
        P = orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, m.vtable, m.hbar)
        ref = orc.propagate(P, m.psi0, SPLIT_ID[split], COMP_ID[comp], order, dt, k)
        assert_parity(got[i], ref, FP64_TOL, f"batch member {i} {kind} n={n} S={S} {split} "
                      f"{comp}-{order} nsteps={k}")
    check_vs_single(batch, got, single_runs(torch, plans, models, ns, torch.complex128),
                    FP64_TOL)


def test_batch_graph_replays_and_eager_path(torch_cuda):
    """Replays of the captured graph (with eager work and synchronisations in
    between) equal the eager branches bitwise and the single-plan runs."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    models, plans, ns = build_members(torch, torch.complex128)
    bg = soprop.Batch(plans)
    be = soprop.Batch(plans)
    be.set_graphs(False)
    pg = states(torch, models, torch.complex128)
    pe = states(torch, models, torch.complex128)
    for rep in range(3):
        bg.propagate(pg, ns)
        torch.cuda.synchronize()
        be.propagate(pe, ns)
        torch.cuda.synchronize()
        _ = torch.ones(4096, device="cuda").sum()  # unrelated eager work
        for i in range(len(ns)):
            np.testing.assert_array_equal(pg[i].cpu().numpy(), pe[i].cpu().numpy(),
                                          err_msg=f"replay {rep} member {i}")
    assert bg.describe()["graph"] and not be.describe()["graph"]
    ref = single_runs(torch, plans, models, ns, torch.complex128, reps=3)
    check_vs_single(bg, [x.cpu().numpy() for x in pg], ref, FP64_TOL)


def test_batch_changed_steps_and_reverse_direction(torch_cuda):
    """New step counts rebuild the descriptors; direction -1 undoes +1."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    models, plans, ns = build_members(torch, torch.complex128)
    batch = soprop.Batch(plans)
    psis = states(torch, models, torch.complex128)
    ns2 = [k + 1 for k in ns]
    batch.propagate(psis, ns)
    batch.propagate(psis, ns2)
    batch.propagate(psis, [k for k in ns2], direction=-1)
    batch.propagate(psis, ns, direction=-1)
    torch.cuda.synchronize()
    for i, m in enumerate(models):
        assert rel_l2(psis[i].cpu().numpy(), m.psi0) < 1e-12, f"member {i}"


def test_batch_fp32(torch_cuda, orc):
    """FP32 members against the FP64 oracle: measured at most 8.1e-7 (per
    surface and element 7.7e-7); stated bounds 2e-6 and 4e-6."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    mix = [r for r in MIX if r[7] > 0 and r[3] == "VTV"]
    models, plans, ns = build_members(torch, torch.complex64, mix)
    batch = soprop.Batch(plans)
    psis = states(torch, models, torch.complex64)
    batch.propagate(psis, ns)
    torch.cuda.synchronize()
    for i, ((kind, n, S, split, comp, order, dt, k, off), m) in enumerate(zip(mix, models)):
        P = orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, m.vtable, m.hbar)
        ref = orc.propagate(P, m.psi0, SPLIT_ID[split], COMP_ID[comp], order, dt, k)
        assert_parity(psis[i].cpu().numpy().astype(np.complex128), ref, 2e-6,
                      f"batch fp32 member {i} {kind} n={n} {comp}-{order}", elem_tol=4e-6)


def test_batch_tuning_cache(torch_cuda, tmp_path):
    """Choices written to SOPROP_TUNE_CACHE are read back by the next batch."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    mix = [MIX[1], MIX[4], MIX[8], MIX[11]]
    models, plans, ns = build_members(torch, torch.complex128, mix)
    path = tmp_path / "tune.json"
    old = os.environ.get("SOPROP_TUNE_CACHE")
    os.environ["SOPROP_TUNE_CACHE"] = str(path)
    try:
        d1 = soprop.Batch(plans).describe()
        assert path.exists()
        cache = json.loads(path.read_text())
        assert "1d/n1024/s2/c128" in cache and "3d/n48/s3/c128/z" in cache
        d2 = soprop.Batch(plans).describe()
    finally:
        if old is None:
            del os.environ["SOPROP_TUNE_CACHE"]
        else:
            os.environ["SOPROP_TUNE_CACHE"] = old
    assert all(not f["from_cache"] for f in d1["families"] if f["tuned_ms"])
    assert all(f["from_cache"] for f in d2["families"] if f["n"] in (1024, 8192))
    assert all(g["from_cache"] for g in d2["groups"])
    for a, b in zip(d1["families"], d2["families"]):
        assert a["variant"] == b["variant"]
    for a, b in zip(d1["groups"], d2["groups"]):
        assert (a["z_cols"], a["y_cols"], a["x_rows"]) == (b["z_cols"], b["y_cols"], b["x_rows"])


def test_batch_every_variant_matches_oracle(torch_cuda, orc):
    """Each 1D schedule variant and each 3D tile variant, forced through the
    tuning cache, gives oracle parity."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    mix = [("1d", n, 2, "VTV", "triple_jump", 4, 0.02, 2, 0.3)
           for n in (512, 1024, 2048, 4096, 8192)]
    mix += [("3d", n, 3, "VTV", "suzuki", 4, 10.0, 1, 0.2) for n in (32, 48)]
    models, plans, ns = build_members(torch, torch.complex128, mix)
    refs = []
    for (kind, n, S, split, comp, order, dt, k, off), m in zip(mix, models):
        P = orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, m.vtable, m.hbar)
        refs.append(orc.propagate(P, m.psi0, SPLIT_ID[split], COMP_ID[comp], order, dt, k))
    path = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"sop_variants_{os.getpid()}.json")
    old = os.environ.get("SOPROP_TUNE_CACHE")
    os.environ["SOPROP_TUNE_CACHE"] = path
    try:
        for v in range(5):
            # variant 4 exists for two surfaces of 1024 points only
            entries = {}
            for n in (512, 1024, 2048, 4096, 8192):
                entries[f"1d/n{n}/s2/c128"] = str(min(v, 1) if n == 8192 else
                                                  (v if v < 4 or n == 1024 else 0))
            for n in (32, 48):
                entries[f"3d/n{n}/s3/c128/z"] = str(min(v, 1))
                entries[f"3d/n{n}/s3/c128/y"] = str(min(v, 2))
                entries[f"3d/n{n}/s3/c128/x"] = str(min(v, 2))
            with open(path, "w") as f:
                json.dump(entries, f)
            batch = soprop.Batch(plans)
            d = batch.describe()
            psis = states(torch, models, torch.complex128)
            batch.propagate(psis, ns)
            torch.cuda.synchronize()
            for i, ref in enumerate(refs):
                assert_parity(psis[i].cpu().numpy(), ref, FP64_TOL, f"variant {v} member {i}")
            batch.close()
    finally:
        if os.path.exists(path):
            os.remove(path)
        if old is None:
            del os.environ["SOPROP_TUNE_CACHE"]
        else:
            os.environ["SOPROP_TUNE_CACHE"] = old


def test_ensemble_manifest_bench_shape(torch_cuda, orc):
    """The 256-member ensemble the benchmark times (FP64): sampled members
    equal their single-plan runs, the cheapest 3D member and the most and
    least expensive 1D members match the oracle, every member keeps its
    norm."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    man = synth.batch_manifest()
    models = [synth.ensemble_model(e) for e in man]
    plans = [soprop.Plan.from_model(m, comp=e["scheme"], order=e["order"], dt=e["dt"])
             for e, m in zip(man, models)]
    ns = [e["nsteps"] for e in man]
    batch = soprop.Batch(plans)
    psis = states(torch, models, torch.complex128)
    batch.propagate(psis, ns)
    batch.check()
    d = batch.describe()
    print("[ensemble] " + json.dumps({k: v for k, v in d.items() if k != "families"}))
    # the most expensive member of each kind plus a spread of others
    cost = [e["nsteps"] * (e["order"] if e["order"] > 2 else 1) * np.prod(m.n)
            for e, m in zip(man, models)]
    pick = {int(np.argmax([c if e["kind"] == k else -1 for c, e in zip(cost, man)]))
            for k in ("1d", "3d")}
    pick.update(range(0, 256, 37))
    for i in sorted(pick):
        one = torch.from_numpy(models[i].psi0.copy()).cuda()
        plans[i].propagate(one, ns[i])
        a, b = psis[i].cpu().numpy(), one.cpu().numpy()
        if man[i]["kind"] == "3d":
            np.testing.assert_array_equal(a, b, err_msg=f"member {i}")
        else:
            assert rel_l2(a, b) < FP64_TOL, f"member {i}"
    for i, (p, x) in enumerate(zip(plans, psis)):
        assert abs(p.observables(x)["norm"] - 1.0) < 1e-10, f"member {i}"
    kinds = [e["kind"] for e in man]
    c1 = [c if k == "1d" else np.inf for c, k in zip(cost, kinds)]
    c3 = [c if k == "3d" else np.inf for c, k in zip(cost, kinds)]
    c1max = [c if k == "1d" else -1 for c, k in zip(cost, kinds)]
    for i in sorted({int(np.argmin(c3)), int(np.argmin(c1)), int(np.argmax(c1max))}):
        m, e = models[i], man[i]
        P = orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, m.vtable, m.hbar)
        ref = orc.propagate(P, m.psi0, SPLIT_ID["VTV"], COMP_ID[e["scheme"]], e["order"],
                            e["dt"], ns[i])
        assert_parity(psis[i].cpu().numpy(), ref, FP64_TOL,
                      f"ensemble member {i} {e['kind']} n={e['n']} {e['scheme']}-{e['order']} "
                      f"nsteps={ns[i]} vs oracle")


def test_batch_plane_pass_equals_three_passes(torch_cuda):
    """Lockstep groups with the fused xy plane pass and with three separate
    passes give bitwise the same states."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    mix = [r for r in MIX if r[0] == "3d" and r[3] == "VTV"]
    models, plans, ns = build_members(torch, torch.complex128, mix)
    a = soprop.Batch(plans)
    b = soprop.Batch(plans)
    a.set_queue(False)
    b.set_queue(False)
    b.set_plane_pass(False)
    assert all(g["plane"] for g in a.describe()["groups"])
    pa = states(torch, models, torch.complex128)
    pb = states(torch, models, torch.complex128)
    a.propagate(pa, ns)
    b.propagate(pb, ns)
    torch.cuda.synchronize()
    assert not any(g["plane"] for g in b.describe()["groups"])
    for i in range(len(ns)):
        np.testing.assert_array_equal(pa[i].cpu().numpy(), pb[i].cpu().numpy(), err_msg=f"{i}")


QUEUE_MIX = [
    ("3d", 32, 3, "VTV", "triple_jump", 4, 10.0, 3, 0.0),
    ("3d", 32, 3, "VTV", "strang", 2, 7.0, 5, 0.7),
    ("3d", 32, 3, "VTV", "suzuki", 4, 4.0, 0, 0.0),           # zero steps
    ("3d", 32, 3, "VTV", "suzuki", 6, 9.0, 1, -0.3),
    ("3d", 48, 3, "VTV", "suzuki", 4, 12.0, 2, -0.4),
    ("3d", 48, 3, "VTV", "strang", 2, 5.0, 7, 0.3),
    ("3d", 64, 3, "VTV", "triple_jump", 4, 10.0, 1, 0.2),
    ("3d", 64, 1, "VTV", "strang", 2, 0.05, 3, 0.0),
    ("3d", 32, 2, "VTV", "triple_jump", 4, 0.05, 2, 0.0),
    ("3d", 48, 1, "VTV", "triple_jump", 4, 0.05, 2, 0.0),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_queue_equals_lockstep(torch_cuda, dtype):
    """The work-queue launch of the 3D groups (one persistent launch per
    group, tiles ordered round by round) gives bitwise the states of the
    lockstep pass launches and of the single-plan runs, and its round table
    has the shape the step counts imply."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    models, plans, ns = build_members(torch, dt, QUEUE_MIX)
    q = soprop.Batch(plans)
    q.set_queue(True)
    lk = soprop.Batch(plans)
    pq = states(torch, models, dt)
    pl = states(torch, models, dt)
    q.propagate(pq, ns)
    q.check()
    lk.propagate(pl, ns)
    lk.check()
    d = q.describe()
    print("[queue] " + json.dumps(d["groups"]), flush=True)
    Ms = [p.info.M for p in plans]
    for g in d["groups"]:
        assert g["queue"]
        cyc = sorted((ns[i] * Ms[i] for i in g["members"]), reverse=True)
        assert g["rounds"] == (3 * cyc[0] + 1 if cyc[0] > 0 else 0)
    assert not any(g["queue"] for g in lk.describe()["groups"])
    ref = single_runs(torch, plans, models, ns, dt)
    for i in range(len(ns)):
        a = pq[i].cpu().numpy()
        np.testing.assert_array_equal(a, pl[i].cpu().numpy(), err_msg=f"member {i} vs lockstep")
        np.testing.assert_array_equal(a, ref[i], err_msg=f"member {i} vs single run")
    # a second call replays the captured graph
    q.propagate(pq, ns)
    q.check()
    ref2 = single_runs(torch, plans, models, ns, dt, reps=2)
    for i in range(len(ns)):
        np.testing.assert_array_equal(pq[i].cpu().numpy(), ref2[i], err_msg=f"replay {i}")


def test_batch_queue_spin_limit_reports(torch_cuda):
    """A poll limit of one makes the queue's first dependency wait run out:
    the launch leaves early, sop_batch_check reports it once, and the next
    launch with the default limit propagates correctly."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    mix = [r for r in QUEUE_MIX if r[7] > 0][:4]
    models, plans, ns = build_members(torch, torch.complex128, mix)
    b = soprop.Batch(plans)
    b.set_queue(True)
    b.set_queue_spin(1)
    psis = states(torch, models, torch.complex128)
    b.propagate(psis, ns)
    with pytest.raises(soprop.SopError, match="ran a wait out of polls"):
        b.check()
    b.check()  # reported once
    b.set_queue_spin(1 << 21)
    psis = states(torch, models, torch.complex128)
    b.propagate(psis, ns)
    b.check()
    ref = single_runs(torch, plans, models, ns, torch.complex128)
    for i in range(len(ns)):
        np.testing.assert_array_equal(psis[i].cpu().numpy(), ref[i], err_msg=f"member {i}")
    with pytest.raises(soprop.SopError):
        b.set_queue_spin(0)


@pytest.mark.timeout(600)
def test_ensemble_manifest_full_final_time(torch_cuda, orc):
    """The 256-member manifest with every member run to t_f = 10 a.u.
    (200 to 2000 steps of up to 125 substeps): the lockstep chains exceed
    the graph's launch budget, so this covers the batch's eager path too.
    Sampled members (the most expensive of each kind and a spread) equal
    their single-plan runs (3D bitwise, 1D to the FP64 bar); the cheapest 1D
    and 3D members match the oracle; every member keeps its norm."""
    torch = torch_cuda
    from paper_1903_04946_amd import soprop
    man = synth.batch_manifest(t_final=10.0)
    models = [synth.ensemble_model(e) for e in man]
    plans = [soprop.Plan.from_model(m, comp=e["scheme"], order=e["order"], dt=e["dt"])
             for e, m in zip(man, models)]
    ns = [e["nsteps"] for e in man]
    assert min(ns) >= 200 and max(ns) <= 2000
    batch = soprop.Batch(plans)
    psis = states(torch, models, torch.complex128)
    batch.propagate(psis, ns)
    batch.check()
    d = batch.describe()
    print("[ensemble t_f=10] " + json.dumps({k: v for k, v in d.items() if k != "families"}),
          flush=True)
    Ms = [p.info.M for p in plans]
    cost = [k * M * int(np.prod(m.n)) for k, M, m in zip(ns, Ms, models)]
    kinds = [e["kind"] for e in man]
    pick = {int(np.argmax([c if k == kk else -1 for c, k in zip(cost, kinds)]))
            for kk in ("1d", "3d")}
    pick.update(range(5, 256, 51))
    # the schedule variant each 1D family runs (0: the single plan's own)
    fam = {f["n"]: f["variant"] for f in d["families"]}
    for i in sorted(pick):
        one = torch.from_numpy(models[i].psi0.copy()).cuda()
        plans[i].propagate(one, ns[i])
        a, b = psis[i].cpu().numpy(), one.cpu().numpy()
        print(f"[ensemble t_f=10] member {i} {kinds[i]} n={man[i]['n']} "
              f"{man[i]['scheme']}-{man[i]['order']} nsteps={ns[i]} vs single run", flush=True)
        if kinds[i] == "3d" or fam[man[i]["n"]] == 0:
            np.testing.assert_array_equal(a, b, err_msg=f"member {i}")
        else:
            # a tuned family runs the member's transforms in another radix
            # order, with other rounded twiddles: each set of FP64 roots of
            # unity carries its own fixed rounding of the modulus, applied
            # at every transform, so the two runs drift apart in proportion
            # to the number of transforms (Sec. "Dynamic Fourier method":
            # the FFT's rounding floor; 4.0e-12 after 59,750 SF-8 substeps of
            # 512 points in radix 4 against radix 8), plus a random walk
            substeps = ns[i] * Ms[i]
            tol = max(FP64_TOL, 6e-15 * np.sqrt(substeps), 2e-16 * substeps)
            assert_parity(a, b, tol, f"member {i} ({man[i]['n']} points, variant "
                          f"{fam[man[i]['n']]}) vs its single run")
    for i, (p, x) in enumerate(zip(plans, psis)):
        assert abs(p.observables(x)["norm"] - 1.0) < 1e-10, f"member {i}"
    for kk in ("1d", "3d"):
        i = int(np.argmin([c if k == kk else np.inf for c, k in zip(cost, kinds)]))
        m, e = models[i], man[i]
        P = orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, m.vtable, m.hbar)
        ref = orc.propagate(P, m.psi0, SPLIT_ID["VTV"], COMP_ID[e["scheme"]], e["order"],
                            e["dt"], ns[i])
        assert_parity(psis[i].cpu().numpy(), ref, FP64_TOL,
                      f"ensemble t_f=10 member {i} {kk} n={e['n']} {e['scheme']}-{e['order']} "
                      f"nsteps={ns[i]} vs oracle")
    batch.close()
