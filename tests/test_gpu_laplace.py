"""GPU parity of the Laplace-only kernels (the paper's own term, eq. (1), on its
quadrature: the symmetric rule with the N_I points of Table 3) against the
oracle's element loop with D = I and no convection, reaction or source, through
the C-ABI: every degree, form and compiled variant on a small ragged batch, the
mapped points and the det J flag, and the full p = 4 workload and the paper's
500 MB batch size at p = 7 on the autotuned variant (a sample of elements)."""
import numpy as np
import pytest

from gpu_util import flush, rel_errors

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (2e-6, 2e-5)}   # derivation: test_gpu_forward.py


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def lap_batch(p, seed):
    from paper_1310_1194_amd import meshgen
    dims = {1: (5, 3, 3), 2: (4, 3, 2), 3: (3, 3, 2), 4: (3, 2, 2), 5: (2, 2, 2), 6: (2, 2, 1), 7: (2, 1, 1)}[p]
    b = meshgen.make_batch(*dims, amp=0.2, seed=seed)
    return b.subset(np.arange(b.ne - 1))


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("p", range(1, 8))
def test_laplace_every_tile(torch_cuda, p, form):
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = lap_batch(p, 300 + p)
    Ar, flags = oracle.integrate_laplace(p, batch.coords)
    assert flags.sum() == 0
    X = dev(torch, batch.coords)
    for t in range(F.laplace_tile_count(p, form)):
        F.laplace_tile_set(p, form, t)
        flush(f"[laplace] p={p} form={form} tile={F.laplace_tile_describe(p, form, t)} ne={batch.ne}")
        A = F.integrate_laplace_raw(X, p, form)
        torch.cuda.synchronize()
        g, m = rel_errors(A.cpu().numpy(), Ar)
        flush(f"    A: global {g:.3e} max-elem {m:.3e}")
        assert g <= TOL[form][0] and m <= TOL[form][1]
    F.laplace_tile_set(p, form, 0)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_laplace_mapped_points_and_status(torch_cuda, p):
    """Mapped points in the symmetric rule's order and the det J <= 0 flag."""
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = lap_batch(p, 320)
    batch.coords[1] = batch.coords[1][[3, 4, 5, 0, 1, 2]]     # element 1 inverted
    n = F.nshp(p)
    D = np.repeat(np.eye(3)[None], batch.ne, axis=0)
    z3, z1 = np.zeros((batch.ne, 3)), np.zeros(batch.ne)
    Ar, _, flags, xr = oracle.integrate(p, batch.coords, D, z3, z1, z1, want_xq=True, rule="symmetric")
    assert flags[1] == 1
    X = dev(torch, batch.coords)
    nqs = F.nq(p, "symmetric")
    for t in range(F.laplace_tile_count(p, "fp64")):
        F.laplace_tile_set(p, "fp64", t)
        xq = torch.full((batch.ne, nqs, 3), float("nan"), dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        A = F.integrate_laplace_raw(X, p, "fp64", xq=xq, status=st)
        torch.cuda.synchronize()
        flush(f"[laplace xq/status] p={p} tile={F.laplace_tile_describe(p, 'fp64', t)}")
        assert int(st.item()) & 1 == 1
        assert np.abs(xq.cpu().numpy() - xr).max() < 1e-15
        g, m = rel_errors(A.cpu().numpy().reshape(batch.ne, n, n), Ar)
        assert g < 1e-12 and m < 1e-12
    F.laplace_tile_set(p, "fp64", 0)


def test_laplace_empty_batch(torch_cuda):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    A = F.integrate_laplace_raw(torch.empty((0, 6, 3), dtype=torch.float64, device="cuda"), 3, "fp32")
    assert A.shape == (0, 40, 40)


@pytest.mark.parametrize("case,form", [("p4_131072", "fp32"), ("p4_131072", "fp64"), ("paper_p7", "fp32")])
def test_laplace_full_size_sampled(torch_cuda, case, form):
    """Full-size batches on the autotuned variant: the p = 4 workload mesh, and at
    p = 7 the paper's batch size (element matrices of about 500 MB in single
    precision: 500e6 / (4 * 288^2) = 1507 elements of the p = 7 mesh)."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    if case == "p4_131072":
        p, batch = 4, meshgen.workload("p4_131072")
    else:
        p = 7
        full = meshgen.workload("p7_16384")
        batch = full.subset(np.arange(500_000_000 // (4 * F.nshp(7) ** 2)))
    flush(f"[laplace-full] {case} form={form} ne={batch.ne}")
    X = dev(torch, batch.coords)
    n = F.nshp(p)
    dt = torch.float64 if form == "fp64" else torch.float32
    A = torch.empty((batch.ne, n, n), dtype=dt, device="cuda")
    ms = F.laplace_autotune(X, p, form, A, reps=1)
    flush(f"    autotuned {F.laplace_tile_describe(p, form, F.laplace_tile_get(p, form))}: {ms:.3f} ms")
    A.fill_(float("nan"))
    F.integrate_laplace_raw(X, p, form, A=A)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([np.sort(rng.choice(batch.ne, 48 if p < 7 else 12, replace=False)),
                                    [0, batch.ne - 1]]))
    sub = batch.subset(idx)
    Ar, flags = oracle.integrate_laplace(p, sub.coords)
    g, m = rel_errors(A[torch.from_numpy(idx).cuda()].cpu().numpy(), Ar)
    flush(f"    A: global {g:.3e} max-elem {m:.3e} ({len(idx)} elements, {int(flags.sum())} with det J <= 0 somewhere)")
    assert g <= TOL[form][0] and m <= TOL[form][1]
    assert bool(torch.isfinite(A).all())
    F.laplace_tile_set(p, form, 0)
