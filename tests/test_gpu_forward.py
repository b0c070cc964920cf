"""GPU parity of the forward integration against the FP64 oracle, through the C-ABI.

Tolerances (relative Frobenius error against the oracle, per result A and b,
global over the batch and maximum over single elements):
  fp64    1e-12 global and per element (the target of the method's FP64 form),
          per element raised to 16 u kappa_e where the element's det J is badly
          conditioned (kappa_e = max over points of |J e1||J e2||J e3| / |det J|;
          library and oracle form J by different formulas, and near a point
          where det J nearly vanishes the rounding of det J and of J^-1 grows
          with kappa_e: measured a few u kappa_e, e.g. 3.4e-12 on an inverted
          element of p7_16384 with kappa_e = 9.1e3);
  bf16x3  1e-5 global (the target of the split form); per element 5e-5: the
          split keeps 16 bits of each operand, so the neglected lo*lo product
          and the FP32 accumulation leave ~2^-17 relative per term, summed
          over K = 4 nq terms with cancellation (measured <= 4e-6 on A,
          6e-6 on b, at every degree and tile);
  fp32    2e-6 global, 2e-5 per element: W_q and the tables rounded to FP32
          (u = 2^-24) and FP32 sums of K terms give sqrt(K) u (sum |terms| /
          |entry|) per entry, i.e. 1e-6 to 1e-5 for the largest cancellation
          ratios of these meshes and a few 1e-7 in the Frobenius norm
          (measured <= 9e-7 global and per element);
  fp16x3  as fp32 (hi+lo fp16 keeps 22 bits of each operand, so the FP32
          accumulation dominates; measured <= 6e-7).
The load vector is formed by the same contraction as A (a spare padded
column of Y carries w det J f), so it carries the form's precision and is held
to the same tolerances as A; at p = 7 (no spare column) it is accumulated in
FP64 and is well inside them.
"""
import numpy as np
import pytest

from gpu_util import elem_errors, flush, fp64_elem_tol, oracle_of, rel_errors, small_batch, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (2e-6, 2e-5), "bf16x3": (1e-5, 5e-5), "fp16x3": (2e-6, 2e-5)}
BTOL = TOL


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def run_gpu(torch, batch, p, form, tile=None):
    import paper_1310_1194_amd as F
    if tile is not None:
        F.tile_set(p, form, tile)
    args = to_dev(batch)
    A, b = F.integrate_raw(*args, p, form)
    torch.cuda.synchronize()
    if tile is not None:
        F.tile_set(p, form, 0)
    return A.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("p", range(1, 8))
def test_forward_parity_every_tile(torch_cuda, p, form):
    import paper_1310_1194_amd as F
    batch = small_batch(p, seed=p)
    Ar, br, _ = oracle_of(batch, p)
    for tile in range(F.tile_count(p, form)):
        flush(f"[parity] p={p} form={form} tile={F.tile_describe(p, form, tile)} ne={batch.ne}")
        A, b = run_gpu(torch_cuda, batch, p, form, tile)
        gA, mA = rel_errors(A, Ar)
        gb, mb = rel_errors(b, br)
        flush(f"    A: global {gA:.3e} max-elem {mA:.3e}   b: global {gb:.3e} max-elem {mb:.3e}")
        assert gA <= TOL[form][0] and mA <= TOL[form][1]
        assert gb <= BTOL[form][0] and mb <= BTOL[form][1]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mapped_points_and_status(torch_cuda, p):
    """Mapped points and the det J <= 0 flag, from every compiled variant."""
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = small_batch(p, seed=11)
    batch.coords[1] = batch.coords[1][[3, 4, 5, 0, 1, 2]]     # element 1 inverted: det J < 0
    Ar, br, flags, xr = oracle.integrate(p, batch.coords, batch.D, batch.beta, batch.c, batch.f, want_xq=True)
    assert flags[1] == 1 and flags.sum() == 1
    args = to_dev(batch)
    for tile in range(F.tile_count(p, "fp64")):
        flush(f"[xq/status] p={p} tile={F.tile_describe(p, 'fp64', tile)}")
        F.tile_set(p, "fp64", tile)
        xq = torch.full((batch.ne, F.nq(p), 3), float("nan"), dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        A, b = F.integrate_raw(*args, p, "fp64", xq=xq, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) & 1 == 1
        assert np.abs(xq.cpu().numpy() - xr).max() < 1e-15
        # signed det J: the inverted element still matches the oracle
        g, m = rel_errors(A.cpu().numpy(), Ar)
        assert g < 1e-12 and m < 1e-12
        st.zero_()
        F.integrate_raw(*to_dev(small_batch(p, seed=12)), p, "fp64", status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
    F.tile_set(p, "fp64", 0)


def test_deterministic(torch_cuda):
    import paper_1310_1194_amd as F
    batch = small_batch(4, seed=3)
    args = to_dev(batch)
    for form in ("fp64", "bf16x3"):
        A1, b1 = F.integrate_raw(*args, 4, form)
        A2, b2 = F.integrate_raw(*args, 4, form)
        assert bool((A1 == A2).all()) and bool((b1 == b2).all())


def test_empty_batch(torch_cuda):
    import paper_1310_1194_amd as F
    torch = torch_cuda
    z = lambda *s: torch.empty(s, dtype=torch.float64, device="cuda")
    A, b = F.integrate_raw(z(0, 6, 3), z(0, 3, 3), z(0, 3), z(0), z(0), 2, "fp64")
    assert A.shape == (0, 18, 18) and b.shape == (0, 18)


@pytest.mark.parametrize("form", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("p", [4, 5, 7])
def test_split_forms_per_element_scale(torch_cuda, p, form):
    """The split forms on elements whose coefficients span eight orders of
    magnitude (D, beta, c scaled together by 10^u, u ~ U(-4, 4) per element)
    and whose source term spans another eight independently (f by 10^v,
    v ~ U(-6, 2)): every compiled tile against the oracle, per element.  The
    fp16 form's power-of-two scales are chosen per element (A and the load
    vector separately), so the relative error per element must stay at the
    unscaled batch's level."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd.meshgen import Batch
    b0 = small_batch(p, seed=11)
    rng = np.random.default_rng(1000 + p)
    sa = 10.0 ** rng.uniform(-4.0, 4.0, b0.ne)
    sf = 10.0 ** rng.uniform(-6.0, 2.0, b0.ne)
    batch = Batch(b0.coords, np.ascontiguousarray(b0.D * sa[:, None, None]),
                  np.ascontiguousarray(b0.beta * sa[:, None]), np.ascontiguousarray(b0.c * sa),
                  np.ascontiguousarray(b0.f * sf))
    Ar, br, _ = oracle_of(batch, p)
    X = to_dev(batch)
    for tile in range(F.tile_count(p, form)):
        F.tile_set(p, form, tile)
        flush(f"[scale] p={p} form={form} tile={F.tile_describe(p, form, tile)} ne={batch.ne}")
        A, b = F.integrate_raw(*X, p, form)
        torch_cuda.cuda.synchronize()
        eA = elem_errors(A.cpu().numpy(), Ar)
        eb = elem_errors(b.cpu().numpy(), br)
        flush(f"    max-elem A {eA.max():.3e}  b {eb.max():.3e}")
        assert eA.max() <= TOL[form][1] and eb.max() <= BTOL[form][1]
    F.tile_set(p, form, 0)


FULL = [("p1_4096", "fp64"), ("p1_524288", "fp64"), ("p1_524288", "fp32")] + \
    [(w, f) for w in ("p4_131072", "p7_16384") for f in ("fp64", "fp32", "bf16x3", "fp16x3")]


@pytest.mark.parametrize("name,form", FULL)
def test_full_size_sampled(torch_cuda, name, form):
    """Full-size workloads in the benchmark's launch configuration (the tile
    shape autotuned on the whole batch first, as the benchmark does); the
    oracle checks a seeded sample of elements, the first and the last one by
    one, and every output must be finite."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    p = meshgen.WORKLOADS[name]["p"]
    batch = meshgen.workload(name)
    flush(f"[full] {name} form={form} ne={batch.ne}")
    args = to_dev(batch)
    dt = torch.float64 if form == "fp64" else torch.float32
    n = F.nshp(p)
    A = torch.empty((batch.ne, n, n), dtype=dt, device="cuda")
    b = torch.empty((batch.ne, n), dtype=dt, device="cuda")
    ms = F.autotune(*args, p, form, A, b, reps=1)
    tile = F.tile_get(p, form)
    flush(f"    autotuned tile {F.tile_describe(p, form, tile)}: {ms:.3f} ms")
    A.fill_(float("nan"))
    b.fill_(float("nan"))
    F.integrate_raw(*args, p, form, A=A, b=b)
    torch.cuda.synchronize()
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(batch.ne, min(batch.ne, 96 if p < 7 else 24), replace=False))
    idx = np.unique(np.concatenate([idx, [0, batch.ne - 1]]))
    sub = batch.subset(idx)
    Ar, br, _ = oracle.integrate(p, sub.coords, sub.D, sub.beta, sub.c, sub.f)
    ti = torch.from_numpy(idx).cuda()
    gA, mA = rel_errors(A[ti].cpu().numpy(), Ar)
    gb, mb = rel_errors(b[ti].cpu().numpy(), br)
    flush(f"    A: global {gA:.3e} max-elem {mA:.3e}   b: global {gb:.3e} max-elem {mb:.3e}")
    assert gA <= TOL[form][0] and gb <= BTOL[form][0]
    if form == "fp64":
        tol = fp64_elem_tol(sub.coords, p)
        assert (elem_errors(A[ti].cpu().numpy(), Ar) <= tol).all()
        assert (elem_errors(b[ti].cpu().numpy(), br) <= tol).all()
    else:
        assert mA <= TOL[form][1] and mb <= BTOL[form][1]
    assert bool(torch.isfinite(A).all()) and bool(torch.isfinite(b).all())
    F.tile_set(p, form, 0)


def test_p7_fp64_error_tracks_det_condition(torch_cuda):
    """Every 16th element of p7_16384 (1024 elements, perturbed by 0.3 h, so
    some corners invert): the FP64 form against the oracle element by element,
    each within max(1e-12, 16 u kappa_e); the sample must reach the badly
    conditioned regime (some kappa_e > 1e3) for the check to mean anything."""
    import oracle
    import paper_1310_1194_amd as F
    from gpu_util import det_condition
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    p = 7
    batch = meshgen.workload("p7_16384")
    idx = np.arange(0, batch.ne, 16)
    flush(f"[p7 fp64 conditioning] every 16th of {batch.ne}")
    A, b = F.integrate_raw(*to_dev(batch), p, "fp64")
    torch.cuda.synchronize()
    sub = batch.subset(idx)
    Ar, br, _ = oracle.integrate(p, sub.coords, sub.D, sub.beta, sub.c, sub.f)
    ti = torch.from_numpy(idx).cuda()
    eA = elem_errors(A[ti].cpu().numpy(), Ar)
    eb = elem_errors(b[ti].cpu().numpy(), br)
    pts, _ = oracle.prism_rule(p, "collapsed")
    kap = det_condition(sub.coords, pts)
    tol = fp64_elem_tol(sub.coords, p)
    w = int(np.argmax(eA))
    flush(f"    worst element {idx[w]}: error {eA[w]:.3e}, kappa {kap[w]:.3e}, tolerance {tol[w]:.3e}")
    assert kap.max() > 1e3
    assert (eA <= tol).all() and (eb <= tol).all()
    gA, _ = rel_errors(A[ti].cpu().numpy(), Ar)
    assert gA <= 1e-12
