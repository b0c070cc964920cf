"""GPU parity of the adjoint (gradients of sum_e <G_e,A_e> + <g_e,b_e>) against
the oracle's reverse-mode gradient and against central differences.

Tolerances (relative Frobenius error per gradient array):
  fp64  1e-11 (blocks of G summed with FP64 atomics for p >= 4 reorder sums);
  fp32  2e-5 (G, B and U = B G in FP32; S_q and the chain rule in FP64).
"""
import numpy as np
import pytest

from gpu_util import flush, small_batch, to_dev

pytestmark = pytest.mark.gpu

NAMES = ("dcoords", "dD", "dbeta", "dc", "df")
TOL = {"fp64": 1e-11, "fp32": 2e-5}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def rel(a, r):
    return float(np.linalg.norm(np.asarray(a) - r) / np.linalg.norm(r))


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("p", range(1, 8))
def test_adjoint_parity(torch_cuda, p, form):
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = small_batch(p, seed=40 + p)
    n = F.nshp(p)
    rng = np.random.default_rng(p)
    G = rng.normal(size=(batch.ne, n, n))
    g = rng.normal(size=(batch.ne, n))
    if form == "fp32":      # the fp32 form sees the seeds rounded to FP32
        G = G.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    ref = oracle.adjoint(p, batch.coords, batch.D, batch.beta, batch.c, batch.f, G, g)
    dt = torch.float64 if form == "fp64" else torch.float32
    X = to_dev(batch)
    Gd, gd = torch.from_numpy(G).cuda().to(dt), torch.from_numpy(g).cuda().to(dt)
    for tile in range(F.adjoint_tile_count(p, form)):
        F.adjoint_tile_set(p, form, tile)
        flush(f"[adjoint] p={p} form={form} block {F.adjoint_tile_describe(p, form, tile)} ne={batch.ne}")
        got = F.adjoint_raw(*X, Gd, gd, p, form)
        torch.cuda.synchronize()
        for name, a, r in zip(NAMES, got, ref[:5]):
            e = rel(a.cpu().numpy(), r)
            flush(f"    {name}: {e:.3e}")
            assert e <= TOL[form], name
    F.adjoint_tile_set(p, form, 0)


def test_adjoint_autotune(torch_cuda):
    """The autotuner times every block shape, keeps one, and the result of the
    kept shape is unchanged within the FP64 tolerance."""
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    p = 4
    batch = small_batch(p, seed=31)
    n = F.nshp(p)
    rng = np.random.default_rng(31)
    G = rng.normal(size=(batch.ne, n, n))
    g = rng.normal(size=(batch.ne, n))
    X = to_dev(batch)
    Gd, gd = torch.from_numpy(G).cuda(), torch.from_numpy(g).cuda()
    ms = F.adjoint_autotune(*X, Gd, gd, p, "fp64", reps=1)
    t = F.adjoint_tile_get(p, "fp64")
    flush(f"[adjoint-autotune] p={p}: block {F.adjoint_tile_describe(p, 'fp64', t)} {ms:.3f} ms")
    assert ms > 0 and 0 <= t < F.adjoint_tile_count(p, "fp64")
    got = F.adjoint_raw(*X, Gd, gd, p, "fp64")
    torch.cuda.synchronize()
    ref = oracle.adjoint(p, batch.coords, batch.D, batch.beta, batch.c, batch.f, G, g)
    for a, r in zip(got, ref[:5]):
        assert rel(a.cpu().numpy(), r) <= TOL["fp64"]
    F.adjoint_tile_set(p, "fp64", 0)


def test_autograd_function(torch_cuda):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = small_batch(1, seed=5).subset([0, 1])
    args = [t.clone().requires_grad_(True) for t in to_dev(batch)]

    def fn(*xs):
        A, b = F.integrate(*xs, 1, "fp64")
        return A, b

    assert torch.autograd.gradcheck(fn, args, eps=1e-6, atol=1e-8, rtol=1e-6)
    A, b = F.integrate(*args, 1, "fp64")
    (A.sum() + 2 * b.sum()).backward()
    assert all(a.grad is not None and torch.isfinite(a.grad).all() for a in args)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_adjoint_full_size_sampled(torch_cuda, form):
    """The p=3 adjoint workload (64x64x16 mesh, 131072 elements, G, g ~ N(0,1)):
    the 64 sampled elements against the oracle gradient and against central
    differences (h = 1e-6) of the GPU FP64 forward."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    p = 3
    batch = meshgen.workload("adj_p3_131072")
    G, g, sample = meshgen.adjoint_seeds(batch, p)
    dt = torch.float64 if form == "fp64" else torch.float32
    flush(f"[adjoint-full] form={form} ne={batch.ne}")
    X = to_dev(batch)
    Gd, gd = torch.from_numpy(G).cuda().to(dt), torch.from_numpy(g).cuda().to(dt)
    grads = F.adjoint_raw(*X, Gd, gd, p, form)
    torch.cuda.synchronize()
    sub = batch.subset(sample)
    Gs, gs = G[sample], g[sample]
    if form == "fp32":
        Gs = Gs.astype(np.float32).astype(np.float64)
        gs = gs.astype(np.float32).astype(np.float64)
    ref = oracle.adjoint(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, Gs, gs)
    si = torch.from_numpy(sample).cuda()
    for name, a, r in zip(NAMES, grads, ref[:5]):
        e = rel(a[si].cpu().numpy(), r)
        flush(f"    {name} vs oracle: {e:.3e}")
        assert e <= TOL[form]
    if form != "fp64":
        return
    # central differences of the GPU forward, all 32 inputs of the 64 elements
    h = 1e-6
    m = len(sample)
    flat = np.concatenate([sub.coords.reshape(m, 18), sub.D.reshape(m, 9), sub.beta, sub.c[:, None], sub.f[:, None]], 1)
    plus = np.repeat(flat[:, None, :], 32, 1) + h * np.eye(32)[None]
    minus = np.repeat(flat[:, None, :], 32, 1) - h * np.eye(32)[None]
    both = np.concatenate([plus, minus], 1).reshape(-1, 32)
    Xp = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in
          (both[:, :18].reshape(-1, 6, 3), both[:, 18:27].reshape(-1, 3, 3), both[:, 27:30], both[:, 30], both[:, 31])]
    A, b = F.integrate_raw(*Xp, p, "fp64")
    Ae = A.cpu().numpy().reshape(m, 64, -1)
    be = b.cpu().numpy().reshape(m, 64, -1)
    Le = np.einsum("mkij,mij->mk", Ae.reshape(m, 64, F.nshp(p), F.nshp(p)), Gs) + np.einsum("mki,mi->mk", be, gs)
    fd = (Le[:, :32] - Le[:, 32:]) / (2 * h)
    got = np.concatenate([grads[0][si].cpu().numpy().reshape(m, 18), grads[1][si].cpu().numpy().reshape(m, 9),
                          grads[2][si].cpu().numpy(), grads[3][si].cpu().numpy()[:, None],
                          grads[4][si].cpu().numpy()[:, None]], 1)
    err = np.linalg.norm(fd - got, axis=1) / np.linalg.norm(got, axis=1)
    flush(f"    central differences: max per-element rel err {err.max():.3e}")
    assert err.max() < 1e-6


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_adjoint_p7_full_size_sampled(torch_cuda, form):
    """The p=7 workload (32x32x8 mesh at +-0.3h, 16384 elements) with the same
    loss: G, g drawn on the device; the 64 sampled elements against the oracle."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    p = 7
    batch = meshgen.workload("p7_16384")
    dt = torch.float64 if form == "fp64" else torch.float32
    G, g, sample = meshgen.adjoint_seeds_device(batch, p, seed=4, dtype=dt)
    flush(f"[adjoint-p7] form={form} ne={batch.ne}")
    grads = F.adjoint_raw(*to_dev(batch), G, g, p, form)
    torch.cuda.synchronize()
    si = torch.from_numpy(sample).cuda()
    Gs = G[si].double().cpu().numpy()
    gs = g[si].double().cpu().numpy()
    del G, g
    sub = batch.subset(sample)
    ref = oracle.adjoint(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, Gs, gs)
    for name, a, r in zip(NAMES, grads, ref[:5]):
        e = rel(a[si].cpu().numpy(), r)
        flush(f"    {name} vs oracle: {e:.3e}")
        assert e <= TOL[form]
