"""The allocation-free mixed-degree entry point (feint_integrate_mixed_noalloc)
against the plan-based one (feint_mixed_bucket + feint_integrate_mixed, the
same first tile set) through the C-ABI: offsets bit for bit, element matrices
and vectors identical, and both against the oracle; two calls in a row, the
second on a smaller batch, so that whatever the first call left in the
library's fixed scratch must not leak into the second."""
import ctypes

import numpy as np
import pytest

from gpu_util import flush, rel_errors, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp32": (2e-6, 2e-5), "fp64": (1e-12, 1e-12)}   # derivation: test_gpu_forward.py


def nshp(p):
    return (p + 1) * (p + 1) * (p + 2) // 2


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1310_1194_amd as F
    for d in range(1, 7):
        F.prepare(d)
    return torch


def batch_of(nx, ny, nz, seed):
    from paper_1310_1194_amd import meshgen
    b = meshgen.make_batch(nx, ny, nz, amp=0.2, seed=seed, mixed=True)
    return b.subset(np.arange(b.ne - 1))          # ragged count


def plan_result(torch, batch, form):
    import paper_1310_1194_amd as F
    X = to_dev(batch)
    pd = torch.from_numpy(batch.p).cuda()
    plan = F.MixedPlan(batch.ne, form)
    plan.tile = 0
    offA, offb = plan.bucket(pd)
    A, b = plan.alloc_outputs(offA, offb)
    plan.integrate(*X, A, b, offA, offb)
    torch.cuda.synchronize()
    out = (offA.cpu().numpy(), offb.cpu().numpy(), A.cpu().numpy(), b.cpu().numpy())
    plan.close()
    return out


def noalloc_result(torch, batch, form):
    import paper_1310_1194_amd as F
    X = to_dev(batch)
    pd = torch.from_numpy(batch.p).cuda()
    n = np.array([nshp(int(p)) for p in batch.p])
    dt = torch.float64 if form == "fp64" else torch.float32
    A = torch.full((int((n * n).sum()),), float("nan"), dtype=dt, device="cuda")
    b = torch.full((int(n.sum()),), float("nan"), dtype=dt, device="cuda")
    offA = torch.full((batch.ne + 1,), -1, dtype=torch.int64, device="cuda")
    offb = torch.full_like(offA, -1)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    F.integrate_mixed_noalloc(*X, pd, A, b, offA, offb, form=form, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return offA.cpu().numpy(), offb.cpu().numpy(), A.cpu().numpy(), b.cpu().numpy()


def check_oracle(batch, offA, offb, A, b, form):
    import oracle
    for d in range(1, 7):
        idx = np.nonzero(batch.p == d)[0]
        if len(idx) == 0:
            continue
        n = nshp(d)
        sub = batch.subset(idx)
        Ar, br, _ = oracle.integrate(d, sub.coords, sub.D, sub.beta, sub.c, sub.f)
        gA = np.stack([A[offA[e]:offA[e] + n * n].reshape(n, n) for e in idx])
        gb = np.stack([b[offb[e]:offb[e] + n] for e in idx])
        eA, mA = rel_errors(gA, Ar)
        eb, mb = rel_errors(gb, br)
        flush(f"    p={d} ({len(idx)} el): A {eA:.3e} / {mA:.3e}  b {eb:.3e} / {mb:.3e}")
        assert eA <= TOL[form][0] and mA <= TOL[form][1]
        assert eb <= TOL[form][0] and mb <= TOL[form][1]


@pytest.mark.parametrize("form", ["fp32", "fp64"])
def test_noalloc_matches_plan_two_calls(torch_cuda, form):
    torch = torch_cuda
    for k, dims in enumerate([(7, 6, 3), (3, 3, 2)]):         # second call: a smaller batch
        batch = batch_of(*dims, seed=60 + k)
        flush(f"[noalloc] form={form} call {k + 1}: ne={batch.ne}")
        ref = plan_result(torch, batch, form)
        got = noalloc_result(torch, batch, form)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert np.isfinite(got[2]).all() and np.isfinite(got[3]).all()
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])
        check_oracle(batch, *got, form)


def test_noalloc_rejects_oversized_batch(torch_cuda):
    """Beyond the fixed scratch: FEINT_ERR_TOO_LARGE from the host check,
    before any launch, with the reason in the last-error text."""
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd.native import Elements, lib
    torch = torch_cuda
    dummy = torch.zeros(64, dtype=torch.float64, device="cuda")
    ptr = ctypes.c_void_p(dummy.data_ptr())
    el = Elements(ptr, ptr, ptr, ptr, ptr, F.api.NOALLOC_MAX_NE + 1)
    code = lib().feint_integrate_mixed_noalloc(ctypes.byref(el), ptr, 1, ptr, ptr, ptr, ptr, None, None)
    assert code == -6
    assert b"exceed" in lib().feint_last_error()
    assert lib().feint_integrate_mixed_noalloc(ctypes.byref(el), ptr, 2, ptr, ptr, ptr, ptr, None, None) == -3
