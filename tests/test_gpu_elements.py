"""GPU parity of the other element types of Table 1 -- hexahedra (tensor
product basis) and tetrahedra (complete basis) -- against the oracle, through
the C-ABI: every degree, form (FP64, FP32 and the split forms) and compiled
variant, mapped points in the
rule's point order, the det J flag, an empty batch, and the full p = 4
meshes on a sample of elements.  Tolerances are those of the prism forward
tests, except that the FP32 global tolerance grows with the length K = 4 nq
of the contraction's FP32 sums as 2 sqrt(K) 2^-24 once that exceeds 2e-6
(hexahedra at p = 7 contract K = 2048 terms point by point: measured 2.1e-6;
5.4e-6 allowed)."""
import numpy as np
import pytest

from gpu_util import flush, rel_errors

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (2e-6, 2e-5), "bf16x3": (1e-5, 5e-5), "fp16x3": (2e-6, 2e-5)}   # derivation: test_gpu_forward.py
NV = {"hex": 8, "tet": 4}


def fp32_global_tol(K):
    return max(TOL["fp32"][0], 2.0 * np.sqrt(K) * 2.0 ** -24)
INVERT = {"hex": [4, 5, 6, 7, 0, 1, 2, 3], "tet": [0, 2, 1, 3]}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def elem_batch(kind, p, seed):
    """Several tiles' worth of elements with a ragged count; every mesh has
    interior vertices, so some elements are distorted."""
    from paper_1310_1194_amd import meshgen
    if kind == "hex":
        dims = {1: (5, 4, 3), 2: (4, 3, 3), 3: (3, 3, 2), 4: (3, 2, 2), 5: (2, 2, 2), 6: (2, 2, 2), 7: (2, 2, 2)}[p]
        b = meshgen.make_hex_batch(*dims, amp=0.2, seed=seed)
    else:
        dims = {1: (4, 3, 3), 2: (3, 3, 2), 3: (3, 2, 2), 4: (2, 2, 2), 5: (2, 2, 2), 6: (2, 2, 2), 7: (2, 2, 2)}[p]
        b = meshgen.make_tet_batch(*dims, amp=0.2, seed=seed)
    return b.subset(np.arange(b.ne - 1))


def oracle_of(kind, p, b, **kw):
    import oracle
    fn = oracle.integrate_hex if kind == "hex" else oracle.integrate_tet
    return fn(p, b.coords, b.D, b.beta, b.c, b.f, **kw)


def dev(torch, b):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t(b.coords), t(b.D), t(b.beta), t(b.c), t(b.f)


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("p", range(1, 8))
@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_elem_parity_every_tile(torch_cuda, kind, p, form):
    import paper_1310_1194_amd as F
    batch = elem_batch(kind, p, 200 + p)
    Ar, br, _ = oracle_of(kind, p, batch)
    X = dev(torch_cuda, batch)
    for tile in range(F.elem_tile_count(kind, p, form)):
        F.elem_tile_set(kind, p, form, tile)
        flush(f"[{kind}] p={p} form={form} tile={F.elem_tile_describe(kind, p, form, tile)} ne={batch.ne}")
        A, b = F.integrate_elem_raw(kind, *X, p, form)
        torch_cuda.cuda.synchronize()
        gA, mA = rel_errors(A.cpu().numpy(), Ar)
        gb, mb = rel_errors(b.cpu().numpy(), br)
        flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e} / {mb:.3e}")
        tg = fp32_global_tol(4 * F.ELEMENTS[kind][2](p)) if form == "fp32" else TOL[form][0]
        assert gA <= tg and mA <= TOL[form][1]
        assert gb <= tg and mb <= TOL[form][1]
    F.elem_tile_set(kind, p, form, 0)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [3, 4, 7])
def test_tet_reference_gemm_full_waves(torch_cuda, p, form):
    """The reference-matrix kernels ("ref...") on 150 tetrahedra: two full
    waves of 64 elements (nine of 16) and a ragged tail, so that both the
    full-wave store path and the masked one run at every degree where the
    every-tile test has fewer elements than a wave."""
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    batch = meshgen.make_tet_batch(4, 4, 2, amp=0.2, seed=230 + p)
    batch = batch.subset(np.arange(150))
    Ar, br, _ = oracle_of("tet", p, batch)
    X = dev(torch_cuda, batch)
    ran = 0
    for tile in range(F.elem_tile_count("tet", p, form)):
        name = F.elem_tile_describe("tet", p, form, tile)
        if not name.startswith("ref"):
            continue
        F.elem_tile_set("tet", p, form, tile)
        flush(f"[tet ref] p={p} form={form} tile={name} ne={batch.ne}")
        A, b = F.integrate_elem_raw("tet", *X, p, form)
        torch_cuda.cuda.synchronize()
        gA, mA = rel_errors(A.cpu().numpy(), Ar)
        gb, mb = rel_errors(b.cpu().numpy(), br)
        flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e} / {mb:.3e}")
        tg = fp32_global_tol(4 * F.ELEMENTS["tet"][2](p)) if form == "fp32" else TOL[form][0]
        assert gA <= tg and mA <= TOL[form][1]
        assert gb <= tg and mb <= TOL[form][1]
        ran += 1
    F.elem_tile_set("tet", p, form, 0)
    assert ran >= 1


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_elem_mapped_points_and_status(torch_cuda, kind, p):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = elem_batch(kind, p, 210 + p)
    batch.coords[1] = batch.coords[1][INVERT[kind]]                 # element 1 inverted
    Ar, br, flags, xr = oracle_of(kind, p, batch, want_xq=True)
    assert flags[1] == 1 and flags.sum() == 1
    X = dev(torch, batch)
    nqe = F.ELEMENTS[kind][2](p)
    for tile in range(F.elem_tile_count(kind, p, "fp64")):
        F.elem_tile_set(kind, p, "fp64", tile)
        flush(f"[{kind} xq/status] p={p} tile={F.elem_tile_describe(kind, p, 'fp64', tile)}")
        xq = torch.full((batch.ne, nqe, 3), float("nan"), dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        A, b = F.integrate_elem_raw(kind, *X, p, "fp64", xq=xq, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) & 1 == 1
        assert np.abs(xq.cpu().numpy() - xr).max() < 1e-15
        g, m = rel_errors(A.cpu().numpy(), Ar)
        assert g < 1e-12 and m < 1e-12
    F.elem_tile_set(kind, p, "fp64", 0)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_elem_empty_batch(torch_cuda, kind):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    z = lambda *s: torch.empty(s, dtype=torch.float64, device="cuda")
    A, b = F.integrate_elem_raw(kind, z(0, NV[kind], 3), z(0, 3, 3), z(0, 3), z(0), z(0), 2, "fp64")
    n = F.ELEMENTS[kind][1](2)
    assert A.shape == (0, n, n) and b.shape == (0, n)


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("name,kind", [("hex_p4_65536", "hex"), ("tet_p4_393216", "tet")])
def test_elem_full_size_sampled(torch_cuda, name, kind, form):
    """The p = 4 meshes of the other element types on the 64x64x16 vertex grid,
    in the benchmark's launch configuration; the oracle checks a seeded sample."""
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    batch = meshgen.workload(name)
    flush(f"[{kind}-full] {name} form={form} ne={batch.ne}")
    X = dev(torch, batch)
    A, b = F.integrate_elem_raw(kind, *X, 4, form)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([np.sort(rng.choice(batch.ne, 64, replace=False)), [0, batch.ne - 1]]))
    sub = batch.subset(idx)
    Ar, br, _ = oracle_of(kind, 4, sub)
    ti = torch.from_numpy(idx).cuda()
    gA, mA = rel_errors(A[ti].cpu().numpy(), Ar)
    gb, _ = rel_errors(b[ti].cpu().numpy(), br)
    flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e}")
    assert gA <= TOL[form][0] and mA <= TOL[form][1] and gb <= TOL[form][0]
    assert bool(torch.isfinite(A).all())
