"""GPU parity of the integration with spatially varying coefficients (values
at the six vertices, evaluated at each point with the geometry shape
functions) against the oracle, for every degree, form and compiled variant.
Tolerances are those of the forward tests (the coefficients only change how
W_q is formed, in FP64, before the contraction)."""
import numpy as np
import pytest

from gpu_util import flush, rel_errors, small_batch

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (2e-6, 2e-5), "bf16x3": (1e-5, 5e-5), "fp16x3": (2e-6, 2e-5)}   # derivation: test_gpu_forward.py


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def vertex_fields(ne, seed):
    from paper_1310_1194_amd import meshgen
    return meshgen.vertex_fields(ne, seed)


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("p", range(1, 8))
def test_fields_parity_every_tile(torch_cuda, p, form):
    import oracle
    import paper_1310_1194_amd as F
    torch = torch_cuda
    batch = small_batch(p, seed=70 + p)
    Dv, bv, cv, fv = vertex_fields(batch.ne, 80 + p)
    Ar, br, _ = oracle.integrate_fields(p, batch.coords, Dv, bv, cv, fv)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    args = [t(batch.coords), t(Dv), t(bv), t(cv), t(fv)]
    for tile in range(F.tile_count(p, form)):
        F.tile_set(p, form, tile)
        flush(f"[fields] p={p} form={form} tile={F.tile_describe(p, form, tile)} ne={batch.ne}")
        A, b = F.integrate_fields_raw(*args, p, form)
        torch.cuda.synchronize()
        gA, mA = rel_errors(A.double().cpu().numpy(), Ar)
        gb, mb = rel_errors(b.double().cpu().numpy(), br)
        flush(f"    A: {gA:.3e} / {mA:.3e}   b: {gb:.3e} / {mb:.3e}")
        assert gA <= TOL[form][0] and mA <= TOL[form][1]
        assert gb <= TOL[form][0] and mb <= TOL[form][1]
    F.tile_set(p, form, 0)


def test_constant_fields_match_element_constants(torch_cuda):
    import paper_1310_1194_amd as F
    from gpu_util import to_dev
    torch = torch_cuda
    p = 3
    batch = small_batch(p, seed=91)
    rep = lambda a: torch.from_numpy(np.ascontiguousarray(np.repeat(a[:, None], 6, axis=1))).cuda()
    A0, b0 = F.integrate_raw(*to_dev(batch), p, "fp64")
    A1, b1 = F.integrate_fields_raw(torch.from_numpy(batch.coords).cuda(), rep(batch.D), rep(batch.beta),
                                    rep(batch.c), rep(batch.f), p, "fp64")
    torch.cuda.synchronize()
    assert float((A1 - A0).abs().max()) <= 1e-14 * float(A0.abs().max())
    assert float((b1 - b0).abs().max()) <= 1e-14 * float(b0.abs().max())
