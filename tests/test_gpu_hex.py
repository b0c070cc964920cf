"""GPU parity of hexahedral elements (Table 1's tensor-product element)
against the oracle, through the C-ABI: every degree, form and compiled
variant, mapped points in the rule's point order, the det J flag, an empty
batch, and the full 64x64x16 hexahedral workload on a sample of elements.
Tolerances are those of the prism forward tests."""
import numpy as np
import pytest

from gpu_util import flush, rel_errors

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (1e-5, 1e-4)}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def hex_batch(p, seed):
    """Several tiles' worth of hexahedra with a ragged count; every mesh has
    interior vertices, so some elements are distorted."""
    from paper_1310_1194_amd import meshgen
    dims = {1: (5, 4, 3), 2: (4, 3, 3), 3: (3, 3, 2), 4: (3, 2, 2), 5: (2, 2, 2), 6: (2, 2, 2), 7: (2, 2, 2)}[p]
    b = meshgen.make_hex_batch(*dims, amp=0.2, seed=seed)
    return b.subset(np.arange(b.ne - 1))


def dev(torch, b):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t(b.coords), t(b.D), t(b.beta), t(b.c), t(b.f)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("p", range(1, 8))
def test_hex_parity_every_tile(torch_cuda, p, form):
    import oracle
    import paper_1310_1194_amd as F
    batch = hex_batch(p, 200 + p)
    Ar, br, _ = oracle.integrate_hex(p, batch.coords, batch.D, batch.beta, batch.c, batch.f)
    X = dev(torch_cuda, batch)
    for tile in range(F.hex_tile_count(p, form)):
        F.hex_tile_set(p, form, tile)
        flush(f"[hex] p={p} form={form} tile={F.hex_tile_describe(p, form, tile)} ne={batch.ne}")
        A, b = F.integrate_hex_raw(*X, p, form)
        torch_cuda.cuda.synchronize()
        gA, mA = rel_errors(A.cpu().numpy(), Ar)
        gb, mb = rel_errors(b.cpu().numpy(), br)
        flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e} / {mb:.3e}")
        assert gA <= TOL[form][0] and mA <= TOL[form][1]
        assert gb <= TOL[form][0] and mb <= TOL[form][1]
    F.hex_tile_set(p, form, 0)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_hex_mapped_points_and_status(torch_cuda, p):
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = hex_batch(p, 210 + p)
    batch.coords[1] = batch.coords[1][[4, 5, 6, 7, 0, 1, 2, 3]]      # element 1 inverted
    Ar, br, flags, xr = oracle.integrate_hex(p, batch.coords, batch.D, batch.beta, batch.c, batch.f, want_xq=True)
    assert flags[1] == 1 and flags.sum() == 1
    X = dev(torch, batch)
    for tile in range(F.hex_tile_count(p, "fp64")):
        F.hex_tile_set(p, "fp64", tile)
        flush(f"[hex xq/status] p={p} tile={F.hex_tile_describe(p, 'fp64', tile)}")
        xq = torch.full((batch.ne, (p + 1) ** 3, 3), float("nan"), dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        A, b = F.integrate_hex_raw(*X, p, "fp64", xq=xq, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) & 1 == 1
        assert np.abs(xq.cpu().numpy() - xr).max() < 1e-15
        g, m = rel_errors(A.cpu().numpy(), Ar)
        assert g < 1e-12 and m < 1e-12
    F.hex_tile_set(p, "fp64", 0)


def test_hex_empty_batch(torch_cuda):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    z = lambda *s: torch.empty(s, dtype=torch.float64, device="cuda")
    A, b = F.integrate_hex_raw(z(0, 8, 3), z(0, 3, 3), z(0, 3), z(0), z(0), 2, "fp64")
    assert A.shape == (0, 27, 27) and b.shape == (0, 27)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_hex_full_size_sampled(torch_cuda, form):
    """The 64x64x16 hexahedral mesh at p = 4 (65536 elements) in the benchmark's
    launch configuration; the oracle checks a seeded sample."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    batch = meshgen.workload("hex_p4_65536")
    flush(f"[hex-full] hex_p4_65536 form={form} ne={batch.ne}")
    X = dev(torch, batch)
    A, b = F.integrate_hex_raw(*X, 4, form)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([np.sort(rng.choice(batch.ne, 64, replace=False)), [0, batch.ne - 1]]))
    sub = batch.subset(idx)
    Ar, br, _ = oracle.integrate_hex(4, sub.coords, sub.D, sub.beta, sub.c, sub.f)
    ti = torch.from_numpy(idx).cuda()
    gA, mA = rel_errors(A[ti].cpu().numpy(), Ar)
    gb, _ = rel_errors(b[ti].cpu().numpy(), br)
    flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e}")
    assert gA <= TOL[form][0] and mA <= TOL[form][1] and gb <= TOL[form][0]
    assert bool(torch.isfinite(A).all())
