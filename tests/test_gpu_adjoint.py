"""GPU parity of the adjoint (gradients of sum_e <G_e,A_e> + <g_e,b_e>) against
the oracle's reverse-mode gradient and against central differences.

Tolerances, per gradient array (dcoords, dD, dbeta, dc, df): the global
relative Frobenius error over the batch, and the maximum over elements of
the element's error relative to its own reference norm (floored at 1e-2 of
the batch's root-mean-square element norm, because dc and df are single sums
of terms of random sign that can cancel to near zero; `gpu_util.grad_errors`):
  fp64  1e-11 global, 1e-10 per element (partial gradients of the waves that
        share an element are summed with FP64 atomics, in varying order;
        measured <= 6e-15 global, 6e-13 per element);
  fp32  4e-6 global, 5e-5 per element (G, the tables and the products U, T
        accumulated in FP32 over K = n or 4 nij terms, u = 2^-24 times
        sqrt(K) times the cancellation ratio; S_q and the chain rule in FP64;
        measured <= 3.4e-7 global, 8e-6 per element).
The FP32 adjoint is also held against central differences (h = 1e-6) of the
FP64 forward on the sampled elements of the p = 3 workload: 1e-5 per element
(FP32 rounding of the contraction, ~1e-7, plus the differences' own
truncation and cancellation error, ~1e-8).
"""
import numpy as np
import pytest

from gpu_util import flush, grad_errors, small_batch, to_dev

pytestmark = pytest.mark.gpu

NAMES = ("dcoords", "dD", "dbeta", "dc", "df")
TOL = {"fp64": (1e-11, 1e-10), "fp32": (4e-6, 5e-5)}


def check_grads(got, ref, form, sel=None, tag=""):
    """Every gradient array against the oracle, globally and per element."""
    for name, a, r in zip(NAMES, got, ref[:5]):
        a = a[sel] if sel is not None else a
        g, m = grad_errors(a.cpu().numpy(), r, floor=1e-2)
        flush(f"    {name}{tag}: global {g:.3e} max-elem {m:.3e}")
        assert g <= TOL[form][0] and m <= TOL[form][1], name


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
        check_grads(got, ref, form)
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
    check_grads(got, ref, "fp64")
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
    """The p=3 adjoint workload (64x64x16 mesh, 131072 elements, G, g ~ N(0,1)),
    in the benchmark's launch configuration (block shape autotuned first): the
    64 sampled elements against the oracle gradient and, in both forms, against
    central differences (h = 1e-6) of the GPU FP64 forward."""
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
    ms = F.adjoint_autotune(*X, Gd, gd, p, form, reps=1)
    flush(f"    autotuned block {F.adjoint_tile_describe(p, form, F.adjoint_tile_get(p, form))}: {ms:.3f} ms")
    grads = F.adjoint_raw(*X, Gd, gd, p, form)
    torch.cuda.synchronize()
    sub = batch.subset(sample)
    Gs, gs = G[sample], g[sample]
    if form == "fp32":
        Gs = Gs.astype(np.float32).astype(np.float64)
        gs = gs.astype(np.float32).astype(np.float64)
    ref = oracle.adjoint(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, Gs, gs)
    si = torch.from_numpy(sample).cuda()
    check_grads(grads, ref, form, si, " vs oracle")
    # central differences of the GPU FP64 forward, all 32 inputs of the 64 elements
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
    # the FP32 adjoint saw G, g rounded to FP32: differentiate the same loss
    Le = np.einsum("mkij,mij->mk", Ae.reshape(m, 64, F.nshp(p), F.nshp(p)), Gs) + np.einsum("mki,mi->mk", be, gs)
    fd = (Le[:, :32] - Le[:, 32:]) / (2 * h)
    got = np.concatenate([grads[0][si].cpu().numpy().reshape(m, 18), grads[1][si].cpu().numpy().reshape(m, 9),
                          grads[2][si].cpu().numpy(), grads[3][si].cpu().numpy()[:, None],
                          grads[4][si].cpu().numpy()[:, None]], 1)
    err = np.linalg.norm(fd - got, axis=1) / np.linalg.norm(got, axis=1)
    flush(f"    central differences: max per-element rel err {err.max():.3e}")
    assert err.max() < (1e-6 if form == "fp64" else 1e-5)


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
    X = to_dev(batch)
    ms = F.adjoint_autotune(*X, G, g, p, form, reps=1)
    flush(f"    autotuned block {F.adjoint_tile_describe(p, form, F.adjoint_tile_get(p, form))}: {ms:.3f} ms")
    grads = F.adjoint_raw(*X, G, g, p, form)
    torch.cuda.synchronize()
    si = torch.from_numpy(sample).cuda()
    Gs = G[si].double().cpu().numpy()
    gs = g[si].double().cpu().numpy()
    del G, g
    sub = batch.subset(sample)
    ref = oracle.adjoint(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, Gs, gs)
    check_grads(grads, ref, form, si, " vs oracle")
