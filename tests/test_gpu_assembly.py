"""GPU parity of the global assembly (colour by colour, no atomics) against the
oracle's plain assembly: the CSR pattern bit for bit, values and right-hand
side to the rounding of a reordered sum, a valid colouring, accumulation, and
sampled rows of a large mesh.

Tolerance: each global entry is a sum of at most a few dozen element
contributions added in colour order instead of element order, so
|gpu - oracle| <= 8 eps sum|contributions| (eps of the form's dtype)."""
import numpy as np
import pytest

from gpu_util import flush, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def abs_sums(dofs, ndof, A):
    """Per-entry sum of |contribution|, in the oracle's CSR order."""
    import oracle
    return oracle.assemble(dofs, ndof, np.abs(A), np.zeros(A.shape[:2]))[2]


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("p,dims", [(1, (4, 3, 3)), (2, (3, 3, 2)), (3, (3, 2, 2)), (4, (2, 2, 2))])
def test_assembly_parity(torch_cuda, p, dims, form):
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    batch = meshgen.make_batch(*dims, amp=0.2, seed=20 + p)
    dofs, ndof = meshgen.dof_map(*dims, p)
    flush(f"[assembly] p={p} dims={dims} form={form} ne={batch.ne} ndof={ndof}")
    A, b = F.integrate_raw(*to_dev(batch), p, form)
    plan = F.AsmPlan(dofs, ndof)
    vals, rhs = plan.assemble(A, b, form)
    row_ptr, col_idx = plan.pattern()
    torch.cuda.synchronize()
    An, bn = A.double().cpu().numpy(), b.double().cpu().numpy()
    r_rp, r_ci, r_v, r_rhs = oracle.assemble(dofs, ndof, An, bn)
    assert np.array_equal(row_ptr.cpu().numpy(), r_rp)
    assert np.array_equal(col_idx.cpu().numpy().astype(np.int64), r_ci)
    eps = np.finfo(np.float64 if form == "fp64" else np.float32).eps
    got = vals.double().cpu().numpy()
    bound = 8 * eps * abs_sums(dofs, ndof, An) + 1e-300
    err = np.abs(got - r_v)
    flush(f"    values: max |diff| / bound = {(err / bound).max():.3f}, nnz={plan.nnz}, colours={plan.ncolors}")
    assert np.all(err <= bound)
    rb = np.zeros(ndof)
    for e in range(batch.ne):
        rb[dofs[e]] += np.abs(bn[e])
    assert np.all(np.abs(rhs.double().cpu().numpy() - r_rhs) <= 8 * eps * rb + 1e-300)
    # colouring: no dof appears twice within a colour
    col = plan.colors()
    for c in range(plan.ncolors):
        d = dofs[col == c].ravel()
        assert len(np.unique(d)) == len(d)
    # accumulate: a second pass onto the first result doubles every entry
    # (the contributions are added one by one onto it, so to rounding)
    vals2, rhs2 = plan.assemble(A, b, form, values=vals.clone(), rhs=rhs.clone(), accumulate=True)
    torch.cuda.synchronize()
    assert np.all(np.abs(vals2.double().cpu().numpy() - 2 * got) <= 2 * bound + 2 * eps * np.abs(got))
    r1 = rhs.double().cpu().numpy()
    assert np.all(np.abs(rhs2.double().cpu().numpy() - 2 * r1) <= 16 * eps * rb + 2 * eps * np.abs(r1) + 1e-300)
    plan.close()


def test_end_to_end_fp64(torch_cuda):
    """Oracle element matrices assembled by the oracle vs GPU integration
    followed by GPU assembly: FP64, relative 1e-12 of the largest entry."""
    import oracle
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    p, dims = 3, (3, 3, 2)
    batch = meshgen.make_batch(*dims, amp=0.2, seed=31)
    dofs, ndof = meshgen.dof_map(*dims, p)
    Ar, br, _ = oracle.integrate(p, batch.coords, batch.D, batch.beta, batch.c, batch.f)
    _, _, r_v, r_rhs = oracle.assemble(dofs, ndof, Ar, br)
    A, b = F.integrate_raw(*to_dev(batch), p, "fp64")
    plan = F.AsmPlan(dofs, ndof)
    vals, rhs = plan.assemble(A, b, "fp64")
    torch.cuda.synchronize()
    assert np.abs(vals.cpu().numpy() - r_v).max() <= 1e-12 * np.abs(r_v).max()
    assert np.abs(rhs.cpu().numpy() - r_rhs).max() <= 1e-12 * np.abs(r_rhs).max()
    plan.close()


def test_large_mesh_sampled_rows(torch_cuda):
    """p = 4 on a 32x32x8 mesh (16384 prisms, FP32 element matrices): 64 sampled
    rows of the assembled matrix against the sum of the incident elements' rows."""
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import meshgen
    torch = torch_cuda
    p, dims = 4, (32, 32, 8)
    batch = meshgen.make_batch(*dims, amp=0.2, seed=9)
    dofs, ndof = meshgen.dof_map(*dims, p)
    flush(f"[assembly-large] ne={batch.ne} ndof={ndof}")
    A, b = F.integrate_raw(*to_dev(batch), p, "fp32")
    plan = F.AsmPlan(dofs, ndof)
    vals, rhs = plan.assemble(A, b, "fp32")
    row_ptr, col_idx = plan.pattern()
    torch.cuda.synchronize()
    rp, ci, v = row_ptr.cpu().numpy(), col_idx.cpu().numpy(), vals.double().cpu().numpy()
    rows = np.random.default_rng(0).choice(ndof, 64, replace=False)
    where = {}
    for e in range(batch.ne):
        for a, g in enumerate(dofs[e]):
            where.setdefault(int(g), []).append((e, a))
    for i in rows:
        inc = where[int(i)]
        es = torch.tensor([e for e, _ in inc], device="cuda")
        Ae = A[es].double().cpu().numpy()
        ref, mag = {}, {}
        for k, (e, a) in enumerate(inc):
            for bb, g in enumerate(dofs[e]):
                ref[int(g)] = ref.get(int(g), 0.0) + Ae[k, a, bb]
                mag[int(g)] = mag.get(int(g), 0.0) + abs(Ae[k, a, bb])
        got = dict(zip(ci[rp[i]:rp[i + 1]].tolist(), v[rp[i]:rp[i + 1]].tolist()))
        assert set(got) == set(ref)
        for g in ref:
            assert abs(got[g] - ref[g]) <= 8 * np.finfo(np.float32).eps * mag[g] + 1e-30
    plan.close()
