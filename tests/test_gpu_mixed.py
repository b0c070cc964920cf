"""GPU tests of the mixed-degree path: integer bucketing (bit-exact offsets),
the persistent degree-bucketed launch against the oracle for every compiled
tile set, graph capture/replay against eager execution, and the full
262144-element mixed batch on a sample of elements."""
import numpy as np
import pytest

from gpu_util import flush, rel_errors, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp32": (2e-6, 2e-5), "fp64": (1e-12, 1e-12)}   # derivation: test_gpu_forward.py


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def nshp(p):
    return (p + 1) * (p + 1) * (p + 2) // 2


def mixed_batch(nx=6, ny=5, nz=3, seed=2, drop=1):
    from paper_1310_1194_amd import meshgen
    b = meshgen.make_batch(nx, ny, nz, amp=0.2, seed=seed, mixed=True)
    return b.subset(np.arange(b.ne - drop))


def unpack(A, b, offA, offb, pdeg, idx):
    out = []
    for e in idx:
        n = nshp(int(pdeg[e]))
        out.append((A[offA[e]:offA[e] + n * n].reshape(n, n), b[offb[e]:offb[e] + n]))
    return out


def check_against_oracle(batch, A, b, offA, offb, form, idx=None):
    import oracle
    idx = np.arange(batch.ne) if idx is None else idx
    got = unpack(A, b, offA, offb, batch.p, idx)
    worst = (0.0, 0.0)
    for d in range(1, 7):
        sel = [k for k, e in enumerate(idx) if batch.p[e] == d]
        if not sel:
            continue
        sub = batch.subset(idx[sel])
        Ar, br, _ = oracle.integrate(d, sub.coords, sub.D, sub.beta, sub.c, sub.f)
        gA, mA = rel_errors(np.stack([got[k][0] for k in sel]), Ar)
        gb, _ = rel_errors(np.stack([got[k][1] for k in sel]), br)
        flush(f"    p={d} ({len(sel)} el): A global {gA:.3e} max-elem {mA:.3e}  b {gb:.3e}")
        assert gA <= TOL[form][0] and mA <= TOL[form][1]
        assert gb <= TOL[form][0]      # b rides in the contraction: the form's tolerance
        worst = (max(worst[0], gA), max(worst[1], mA))
    return worst


@pytest.mark.parametrize("form", ["fp32", "fp64"])
def test_mixed_every_tile_set(torch_cuda, form):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = mixed_batch()
    X = to_dev(batch)
    pd = torch.from_numpy(batch.p).cuda()
    plan = F.MixedPlan(batch.ne + 10, form)
    offA, offb = plan.bucket(pd)
    n2 = np.array([nshp(int(p)) ** 2 for p in batch.p])
    n1 = np.array([nshp(int(p)) for p in batch.p])
    assert np.array_equal(offA.cpu().numpy(), np.concatenate([[0], np.cumsum(n2)]))
    assert np.array_equal(offb.cpu().numpy(), np.concatenate([[0], np.cumsum(n1)]))
    A, b = plan.alloc_outputs(offA, offb)
    for t in range(plan.tile_count):
        plan.tile = t
        A.fill_(float("nan"))
        b.fill_(float("nan"))
        flush(f"[mixed] form={form} tile set {t} ({plan.tile_describe(t)}) ne={batch.ne}")
        plan.integrate(*X, A, b, offA, offb)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(A).all()) and bool(torch.isfinite(b).all())
        check_against_oracle(batch, A.cpu().numpy(), b.cpu().numpy(), offA.cpu().numpy(), offb.cpu().numpy(), form)
    plan.close()


def test_mixed_matches_direct_launches(torch_cuda):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = mixed_batch(seed=9)
    X = to_dev(batch)
    plan = F.MixedPlan(batch.ne, "fp64")
    offA, offb = plan.bucket(torch.from_numpy(batch.p).cuda())
    A, b = plan.alloc_outputs(offA, offb)
    plan.integrate(*X, A, b, offA, offb)
    oA, ob = offA.cpu().numpy(), offb.cpu().numpy()
    Ah, bh = A.cpu().numpy(), b.cpu().numpy()
    for d in range(1, 7):
        idx = np.nonzero(batch.p == d)[0]
        sub = batch.subset(idx)
        Ad, bd = F.integrate_raw(*to_dev(sub), d, "fp64")
        got = unpack(Ah, bh, oA, ob, batch.p, idx)
        ref = Ad.cpu().numpy()
        for k in range(len(idx)):
            assert np.allclose(got[k][0], ref[k], rtol=1e-13, atol=1e-14 * np.abs(ref[k]).max())
    plan.close()


def test_invalid_degrees_flagged(torch_cuda):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = mixed_batch(nx=3, ny=3, nz=2, seed=4)
    p = batch.p.copy()
    p[3] = 0
    p[7] = 9
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan = F.MixedPlan(batch.ne, "fp32")
    offA, offb = plan.bucket(torch.from_numpy(p).cuda(), status=st)
    oA = offA.cpu().numpy()
    assert int(st.item()) & 2
    assert oA[4] == oA[3] and oA[8] == oA[7]
    A, b = plan.alloc_outputs(offA, offb)
    plan.integrate(*to_dev(batch), A, b, offA, offb)
    torch.cuda.synchronize()
    good = np.array([e for e in range(batch.ne) if e not in (3, 7)])
    batch.p = p
    check_against_oracle(batch, A.cpu().numpy(), b.cpu().numpy(), oA, offb.cpu().numpy(), "fp32", good)
    plan.close()


def test_graph_capture_replays(torch_cuda):
    """Capture bucketing + persistent launch once; every replay (with eager work
    and synchronisations in between) must equal the eager result bit for bit."""
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = mixed_batch(seed=21)
    X = to_dev(batch)
    pd = torch.from_numpy(batch.p).cuda()
    plan = F.MixedPlan(batch.ne, "fp32")
    offA, offb = plan.bucket(pd)
    A, b = plan.alloc_outputs(offA, offb)
    plan.integrate(*X, A, b, offA, offb)
    torch.cuda.synchronize()
    A0, b0 = A.clone(), b.clone()
    gA, gb = torch.empty_like(A), torch.empty_like(b)
    goA, gob = torch.empty_like(offA), torch.empty_like(offb)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.capture(*X, pd, gA, gb, goA, gob, status=st)
    for r in range(4):
        gA.fill_(float("nan"))
        goA.fill_(-1)
        plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(goA, offA) and torch.equal(gob, offb), r
        assert torch.equal(gA, A0) and torch.equal(gb, b0), r
        _ = (A0 * 2).sum().item()     # eager work between replays
    assert int(st.item()) == 0
    plan.close()


def test_full_mixed_batch_sampled(torch_cuda):
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    batch = meshgen.workload("mixed_262144")
    flush(f"[mixed-full] ne={batch.ne}")
    X = to_dev(batch)
    pd = torch.from_numpy(batch.p).cuda()
    plan = F.MixedPlan(batch.ne, "fp32")
    offA, offb = plan.bucket(pd)
    A, b = plan.alloc_outputs(offA, offb)
    ms = plan.autotune(*X, A, b, offA, offb, reps=1)
    flush(f"    autotuned tile set {plan.tile}: {ms:.2f} ms")
    plan.integrate(*X, A, b, offA, offb)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(batch.ne, 120, replace=False))
    oA, ob = offA.cpu().numpy(), offb.cpu().numpy()
    # gather only the sampled ranges from the device
    parts_A, parts_b, oA2, ob2 = [], [], [], []
    posA = posb = 0
    for e in idx:
        n = nshp(int(batch.p[e]))
        parts_A.append(A[oA[e]:oA[e] + n * n].cpu().numpy())
        parts_b.append(b[ob[e]:ob[e] + n].cpu().numpy())
        oA2.append(posA); ob2.append(posb)
        posA += n * n; posb += n
    sub = batch.subset(idx)
    check_against_oracle(sub, np.concatenate(parts_A), np.concatenate(parts_b), np.array(oA2), np.array(ob2), "fp32")
    plan.close()


def test_integrate_after_capture_needs_bucketing(torch_cuda):
    """Capturing enqueues nothing: before the first replay the plan holds no
    bucketing of the captured batch, so an eager integrate (or autotune) is
    refused on the host with INVALID_ARG and no kernel runs; after a replay
    the graph's bucketing is in place and the eager launch matches it."""
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd.native import FeintError
    torch = torch_cuda
    batch = mixed_batch(nx=3, ny=3, nz=2, seed=23)
    X = to_dev(batch)
    pd = torch.from_numpy(batch.p).cuda()
    n2 = np.array([nshp(int(p)) ** 2 for p in batch.p])
    n1 = np.array([nshp(int(p)) for p in batch.p])
    plan = F.MixedPlan(batch.ne, "fp64")
    offA = torch.zeros(batch.ne + 1, dtype=torch.int64, device="cuda")
    offb = torch.zeros_like(offA)
    A = torch.full((int(n2.sum()),), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((int(n1.sum()),), float("nan"), dtype=torch.float64, device="cuda")
    flush(f"[mixed] capture without replay, ne={batch.ne}")
    plan.capture(*X, pd, A, b, offA, offb)
    with pytest.raises(FeintError) as ei:
        plan.integrate(*X, A, b, offA, offb)
    assert ei.value.code == -1
    with pytest.raises(FeintError):
        plan.autotune(*X, A, b, offA, offb, reps=1)
    torch.cuda.synchronize()
    assert bool(torch.isnan(A).all())          # nothing ran
    plan.replay()
    torch.cuda.synchronize()
    A1 = A.clone()
    A.fill_(float("nan"))
    plan.integrate(*X, A, b, offA, offb)       # uses the graph's bucketing
    torch.cuda.synchronize()
    assert torch.equal(A, A1)
    check_against_oracle(batch, A.cpu().numpy(), b.cpu().numpy(), offA.cpu().numpy(), offb.cpu().numpy(), "fp64")
    plan.close()
