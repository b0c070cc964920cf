"""GPU parity on the symmetric prism rule (fully symmetric triangle rule of
degree 2p x (p+1) Gauss points in zeta, the point counts of the paper's
Table 3) against the oracle on its own, independently solved rule: every
degree, form and compiled variant, element constants and vertex fields,
mapped points in the specified point order, the det J flag, the full p = 4
workload on a sample of elements, and the adjoint.  Tolerances are those of
the collapsed-rule forward and adjoint tests."""
import numpy as np
import pytest

from gpu_util import flush, grad_errors, rel_errors, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (2e-6, 2e-5), "bf16x3": (1e-5, 5e-5), "fp16x3": (2e-6, 2e-5)}   # derivation: test_gpu_forward.py
SYM = "symmetric"


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def rule_batch(p, seed):
    """Several tiles' worth of elements with a ragged count; every mesh has
    interior vertices, so some prisms are distorted."""
    from paper_1310_1194_amd import meshgen
    dims = {1: (5, 3, 3), 2: (4, 3, 2), 3: (3, 3, 2), 4: (3, 2, 2), 5: (2, 2, 2), 6: (2, 2, 2), 7: (2, 2, 2)}[p]
    b = meshgen.make_batch(*dims, amp=0.2, seed=seed)
    return b.subset(np.arange(b.ne - 1))


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("p", range(1, 8))
def test_rule_parity_every_tile(torch_cuda, p, form):
    import oracle
    import paper_1310_1194_amd as F
    batch = rule_batch(p, 100 + p)
    Ar, br, _ = oracle.integrate(p, batch.coords, batch.D, batch.beta, batch.c, batch.f, rule=SYM)
    X = to_dev(batch)
    for tile in range(F.tile_count(p, form, rule=SYM)):
        F.tile_set(p, form, tile, rule=SYM)
        flush(f"[rule] p={p} form={form} tile={F.tile_describe(p, form, tile, rule=SYM)} ne={batch.ne}")
        A, b = F.integrate_raw(*X, p, form, rule=SYM)
        torch_cuda.cuda.synchronize()
        gA, mA = rel_errors(A.cpu().numpy(), Ar)
        gb, mb = rel_errors(b.cpu().numpy(), br)
        flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e} / {mb:.3e}")
        assert gA <= TOL[form][0] and mA <= TOL[form][1]
        assert gb <= TOL[form][0] and mb <= TOL[form][1]
    F.tile_set(p, form, 0, rule=SYM)


@pytest.mark.parametrize("form", ["fp64", "bf16x3"])
@pytest.mark.parametrize("p", [1, 3, 4, 7])
def test_rule_with_vertex_fields(torch_cuda, p, form):
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    batch = rule_batch(p, 110 + p)
    Dv, bv, cv, fv = meshgen.vertex_fields(batch.ne, 120 + p)
    Ar, br, _ = oracle.integrate_fields(p, batch.coords, Dv, bv, cv, fv, rule=SYM)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    flush(f"[rule-fields] p={p} form={form} ne={batch.ne}")
    A, b = F.integrate_fields_raw(t(batch.coords), t(Dv), t(bv), t(cv), t(fv), p, form, rule=SYM)
    torch.cuda.synchronize()
    gA, mA = rel_errors(A.cpu().numpy(), Ar)
    gb, mb = rel_errors(b.cpu().numpy(), br)
    flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e} / {mb:.3e}")
    assert gA <= TOL[form][0] and mA <= TOL[form][1]
    assert gb <= TOL[form][0] and mb <= TOL[form][1]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rule_mapped_points_and_status(torch_cuda, p):
    """xq in the rule's point order (q = k ntri + t) and the det J <= 0 flag,
    from every compiled variant."""
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = rule_batch(p, 130 + p)
    batch.coords[1] = batch.coords[1][[3, 4, 5, 0, 1, 2]]       # element 1 inverted
    Ar, br, flags, xr = oracle.integrate(p, batch.coords, batch.D, batch.beta, batch.c, batch.f,
                                         want_xq=True, rule=SYM)
    assert flags[1] == 1 and flags.sum() == 1
    X = to_dev(batch)
    for tile in range(F.tile_count(p, "fp64", rule=SYM)):
        F.tile_set(p, "fp64", tile, rule=SYM)
        flush(f"[rule xq/status] p={p} tile={F.tile_describe(p, 'fp64', tile, rule=SYM)}")
        xq = torch.full((batch.ne, F.nq(p, SYM), 3), float("nan"), dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        A, b = F.integrate_raw(*X, p, "fp64", xq=xq, status=st, rule=SYM)
        torch.cuda.synchronize()
        assert int(st.item()) & 1 == 1
        assert np.abs(xq.cpu().numpy() - xr).max() < 1e-15
        g, m = rel_errors(A.cpu().numpy(), Ar)
        assert g < 1e-12 and m < 1e-12
    F.tile_set(p, "fp64", 0, rule=SYM)


@pytest.mark.parametrize("form", ["fp64", "bf16x3"])
def test_rule_full_size_sampled(torch_cuda, form):
    """The p = 4 workload (131072 elements) on the symmetric rule, in the
    benchmark's launch configuration; the oracle checks a seeded sample."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    batch = meshgen.workload("p4_131072")
    flush(f"[rule-full] p4_131072 form={form} ne={batch.ne}")
    X = to_dev(batch)
    A, b = F.integrate_raw(*X, 4, form, rule=SYM)
    torch.cuda.synchronize()
    rng = np.random.default_rng(321)
    idx = np.unique(np.concatenate([np.sort(rng.choice(batch.ne, 96, replace=False)), [0, batch.ne - 1]]))
    sub = batch.subset(idx)
    Ar, br, _ = oracle.integrate(4, sub.coords, sub.D, sub.beta, sub.c, sub.f, rule=SYM)
    ti = torch.from_numpy(idx).cuda()
    gA, mA = rel_errors(A[ti].cpu().numpy(), Ar)
    gb, _ = rel_errors(b[ti].cpu().numpy(), br)
    flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e}")
    assert gA <= TOL[form][0] and mA <= TOL[form][1] and gb <= TOL[form][0]
    assert bool(torch.isfinite(A).all())


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("p", range(1, 8))
def test_rule_adjoint_parity(torch_cuda, p, form):
    """The adjoint on the symmetric rule, every compiled block shape, against
    the oracle's reverse-mode gradient on its own rule, globally and per
    element (the tolerances of the collapsed-rule adjoint tests)."""
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    tol = {"fp64": (1e-11, 1e-10), "fp32": (4e-6, 5e-5)}[form]
    batch = rule_batch(p, 140 + p)
    n = F.nshp(p)
    rng = np.random.default_rng(150 + p)
    G = rng.normal(size=(batch.ne, n, n))
    g = rng.normal(size=(batch.ne, n))
    if form == "fp32":      # the fp32 form sees the seeds rounded to FP32
        G = G.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    ref = oracle.adjoint(p, batch.coords, batch.D, batch.beta, batch.c, batch.f, G, g, rule=SYM)
    dt = torch.float64 if form == "fp64" else torch.float32
    X = to_dev(batch)
    Gd, gd = torch.from_numpy(G).cuda().to(dt), torch.from_numpy(g).cuda().to(dt)
    for tile in range(F.adjoint_tile_count(p, form)):
        F.adjoint_tile_set(p, form, tile)
        flush(f"[rule adjoint] p={p} form={form} block {F.adjoint_tile_describe(p, form, tile)} ne={batch.ne}")
        got = F.adjoint_raw(*X, Gd, gd, p, form, rule=SYM)
        torch.cuda.synchronize()
        for name, a, r in zip(("dcoords", "dD", "dbeta", "dc", "df"), got, ref[:5]):
            e, m = grad_errors(a.cpu().numpy(), r, floor=1e-2)
            flush(f"    {name}: global {e:.3e} max-elem {m:.3e}")
            assert e <= tol[0] and m <= tol[1], name
    F.adjoint_tile_set(p, form, 0)
