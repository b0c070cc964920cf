"""Python entry points over libfeint (argument marshalling only).

torch supplies device memory and the current stream; every step of the
integration runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import native
import numpy as np

from .native import FORMS, RULES, Elements, FeintError, Fields, check, lib


def nshp(p: int) -> int:
    return (p + 1) * (p + 1) * (p + 2) // 2


def nq(p: int, rule: str = "collapsed") -> int:
    if rule == "collapsed":
        return (p + 1) ** 3
    return lib().feint_nq_rule(int(p), _rule(rule))


def _rule(rule: str) -> int:
    if rule not in RULES:
        raise ValueError(f"unknown rule {rule!r}")
    return RULES[rule]


def rule_points(p: int, rule: str = "collapsed"):
    """Host copy of a rule's points: numpy [nq, 4] = (xi1, xi2, zeta, w)."""
    n = nq(p, rule)
    out = np.zeros((n, 4))
    check("feint_rule_points", lib().feint_rule_points(int(p), _rule(rule), out.ctypes.data_as(ctypes.c_void_p), n))
    return out


def out_dtype(form: str) -> torch.dtype:
    return torch.float64 if form == "fp64" else torch.float32


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_input(name, t, shape_tail, ne):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != (ne, *shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {(ne, *shape_tail)}")


def elements(coords, D, beta, c, f) -> Elements:
    ne = coords.shape[0]
    _check_input("coords", coords, (6, 3), ne)
    _check_input("D", D, (3, 3), ne)
    _check_input("beta", beta, (3,), ne)
    _check_input("c", c, (), ne)
    _check_input("f", f, (), ne)
    return Elements(coords.data_ptr(), D.data_ptr(), beta.data_ptr(), c.data_ptr(), f.data_ptr(), ne)


def prepare(p: int, rule: str = "collapsed") -> None:
    if rule == "collapsed":
        check("feint_prepare", lib().feint_prepare(int(p)))
    else:
        check("feint_prepare_rule", lib().feint_prepare_rule(int(p), _rule(rule)))


def integrate_raw(coords, D, beta, c, f, p: int, form: str = "fp64", *, A=None, b=None,
                  xq=None, status=None, rule: str = "collapsed"):
    """Forward integration into (optionally preallocated) outputs; returns (A, b)."""
    if rule != "collapsed":
        return _integrate_rule(elements(coords, D, beta, c, f), None, coords, p, form, rule, A, b, xq, status)
    if form not in FORMS:
        raise ValueError(f"unknown form {form!r}")
    el = elements(coords, D, beta, c, f)
    ne, n = coords.shape[0], nshp(p)
    dt = out_dtype(form)
    if A is None:
        A = torch.empty((ne, n, n), dtype=dt, device=coords.device)
    if b is None:
        b = torch.empty((ne, n), dtype=dt, device=coords.device)
    if A.dtype != dt or b.dtype != dt or A.numel() != ne * n * n or b.numel() != ne * n:
        raise ValueError("output tensors have the wrong dtype or size")
    if xq is not None and (xq.dtype != torch.float64 or xq.numel() != ne * nq(p) * 3):
        raise ValueError("xq must be float64 with ne*nq*3 entries")
    if status is not None and (status.dtype != torch.int32 or status.numel() < 1):
        raise ValueError("status must be an int32 tensor")
    check("feint_integrate", lib().feint_integrate(ctypes.byref(el), int(p), FORMS[form], _ptr(A), _ptr(b),
                                                   _ptr(xq), _ptr(status), _stream()))
    return A, b


def fields(coords, Dv, betav, cv, fv) -> Fields:
    ne = coords.shape[0]
    for t, k in zip([coords, Dv, betav, cv, fv], [18, 54, 18, 6, 6]):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != ne * k:
            raise ValueError("vertex fields must be contiguous float64 of the documented shapes")
    return Fields(coords.data_ptr(), Dv.data_ptr(), betav.data_ptr(), cv.data_ptr(), fv.data_ptr(), ne)


def _integrate_rule(el, fl, coords, p, form, rule, A, b, xq, status):
    if form not in FORMS:
        raise ValueError(f"unknown form {form!r}")
    ne, n = coords.shape[0], nshp(p)
    dt = out_dtype(form)
    if A is None:
        A = torch.empty((ne, n, n), dtype=dt, device=coords.device)
    if b is None:
        b = torch.empty((ne, n), dtype=dt, device=coords.device)
    if A.dtype != dt or b.dtype != dt or A.numel() != ne * n * n or b.numel() != ne * n:
        raise ValueError("output tensors have the wrong dtype or size")
    if xq is not None and (xq.dtype != torch.float64 or xq.numel() != ne * nq(p, rule) * 3):
        raise ValueError("xq must be float64 with ne*nq*3 entries")
    if status is not None and (status.dtype != torch.int32 or status.numel() < 1):
        raise ValueError("status must be an int32 tensor")
    check("feint_integrate_rule",
          lib().feint_integrate_rule(ctypes.byref(el) if el is not None else None,
                                     ctypes.byref(fl) if fl is not None else None, int(p), FORMS[form],
                                     _rule(rule), _ptr(A), _ptr(b), _ptr(xq), _ptr(status), _stream()))
    return A, b


def integrate_fields_raw(coords, Dv, betav, cv, fv, p: int, form: str = "fp64", *, A=None, b=None,
                         xq=None, status=None, rule: str = "collapsed"):
    """Forward integration with coefficients given at the six vertices of every
    element (Dv [ne,6,3,3], betav [ne,6,3], cv [ne,6], fv [ne,6], FP64)."""
    if form not in FORMS:
        raise ValueError(f"unknown form {form!r}")
    ne, n = coords.shape[0], nshp(p)
    fl = fields(coords, Dv, betav, cv, fv)
    if rule != "collapsed":
        return _integrate_rule(None, fl, coords, p, form, rule, A, b, xq, status)
    dt = out_dtype(form)
    if A is None:
        A = torch.empty((ne, n, n), dtype=dt, device=coords.device)
    if b is None:
        b = torch.empty((ne, n), dtype=dt, device=coords.device)
    if A.dtype != dt or b.dtype != dt or A.numel() != ne * n * n or b.numel() != ne * n:
        raise ValueError("output tensors have the wrong dtype or size")
    check("feint_integrate_fields", lib().feint_integrate_fields(ctypes.byref(fl), int(p), FORMS[form], _ptr(A),
                                                                 _ptr(b), _ptr(xq), _ptr(status), _stream()))
    return A, b


# Other element types of Table 1: kind -> (vertices, shape functions, points, C-ABI prefix)
ELEMENTS = {
    "hex": (8, lambda p: (p + 1) ** 3, lambda p: (p + 1) ** 3, "hex"),
    "tet": (4, lambda p: (p + 1) * (p + 2) * (p + 3) // 6, lambda p: (p + 2) ** 3, "tet"),
}


def hex_nshp(p: int) -> int:
    return ELEMENTS["hex"][1](p)


def tet_nshp(p: int) -> int:
    return ELEMENTS["tet"][1](p)


def _elem_inputs(kind, coords, D, beta, c, f) -> Elements:
    ne = coords.shape[0]
    _check_input("coords", coords, (ELEMENTS[kind][0], 3), ne)
    _check_input("D", D, (3, 3), ne)
    _check_input("beta", beta, (3,), ne)
    _check_input("c", c, (), ne)
    _check_input("f", f, (), ne)
    return Elements(coords.data_ptr(), D.data_ptr(), beta.data_ptr(), c.data_ptr(), f.data_ptr(), ne)


def _fn(kind, name):
    return getattr(lib(), name.format(ELEMENTS[kind][3]))


def integrate_elem_raw(kind: str, coords, D, beta, c, f, p: int, form: str = "fp64", *, A=None, b=None, xq=None,
                       status=None):
    """Hexahedra ("hex", coords [ne,8,3]) or tetrahedra ("tet", coords [ne,4,3]):
    forward integration; returns (A, b)."""
    if form not in FORMS:
        raise ValueError(f"unknown form {form!r}")
    el = _elem_inputs(kind, coords, D, beta, c, f)
    ne, n, nqe = coords.shape[0], ELEMENTS[kind][1](p), ELEMENTS[kind][2](p)
    dt = out_dtype(form)
    if A is None:
        A = torch.empty((ne, n, n), dtype=dt, device=coords.device)
    if b is None:
        b = torch.empty((ne, n), dtype=dt, device=coords.device)
    if A.dtype != dt or b.dtype != dt or A.numel() != ne * n * n or b.numel() != ne * n:
        raise ValueError("output tensors have the wrong dtype or size")
    if xq is not None and (xq.dtype != torch.float64 or xq.numel() != ne * nqe * 3):
        raise ValueError("xq must be float64 with ne*nq*3 entries")
    name = f"feint_integrate_{ELEMENTS[kind][3]}"
    check(name, getattr(lib(), name)(ctypes.byref(el), int(p), FORMS[form], _ptr(A), _ptr(b), _ptr(xq),
                                     _ptr(status), _stream()))
    return A, b


def elem_tile_count(kind: str, p: int, form: str) -> int:
    return _fn(kind, "feint_{}_tile_count")(int(p), FORMS[form])


def elem_tile_get(kind: str, p: int, form: str) -> int:
    return _fn(kind, "feint_{}_tile_get")(int(p), FORMS[form])


def elem_tile_set(kind: str, p: int, form: str, tile: int) -> None:
    check(f"feint_{kind}_tile_set", _fn(kind, "feint_{}_tile_set")(int(p), FORMS[form], int(tile)))


def elem_tile_describe(kind: str, p: int, form: str, tile: int) -> str:
    buf = ctypes.create_string_buffer(32)
    check(f"feint_{kind}_tile_describe", _fn(kind, "feint_{}_tile_describe")(int(p), FORMS[form], int(tile), buf, 32))
    return buf.value.decode()


def elem_autotune(kind: str, coords, D, beta, c, f, p: int, form: str, A, b, reps: int = 2) -> float:
    el = _elem_inputs(kind, coords, D, beta, c, f)
    best = ctypes.c_double(0)
    check(f"feint_{kind}_autotune", _fn(kind, "feint_{}_autotune")(ctypes.byref(el), int(p), FORMS[form], _ptr(A),
                                                                    _ptr(b), int(reps), ctypes.byref(best), _stream()))
    return best.value


def integrate_hex_raw(coords, D, beta, c, f, p: int, form: str = "fp64", **kw):
    return integrate_elem_raw("hex", coords, D, beta, c, f, p, form, **kw)


def integrate_tet_raw(coords, D, beta, c, f, p: int, form: str = "fp64", **kw):
    return integrate_elem_raw("tet", coords, D, beta, c, f, p, form, **kw)


def hex_tile_count(p, form):
    return elem_tile_count("hex", p, form)


def hex_tile_get(p, form):
    return elem_tile_get("hex", p, form)


def hex_tile_set(p, form, tile):
    return elem_tile_set("hex", p, form, tile)


def hex_tile_describe(p, form, tile):
    return elem_tile_describe("hex", p, form, tile)


def hex_autotune(*a, **kw):
    return elem_autotune("hex", *a, **kw)


def _laplace_inputs(coords, p, form):
    if form not in ("fp64", "fp32"):
        raise ValueError("the Laplace kernels run in the fp64 and fp32 forms")
    ne = coords.shape[0]
    _check_input("coords", coords, (6, 3), ne)
    return ne, nshp(p)


def integrate_laplace_raw(coords, p: int, form: str = "fp32", *, A=None, xq=None, status=None):
    """The paper's own term: the Laplace stiffness matrix of prisms on its
    quadrature (the symmetric rule, N_I points), no coefficients, no load
    vector; returns A [ne, n, n]."""
    ne, n = _laplace_inputs(coords, p, form)
    dt = out_dtype(form)
    if A is None:
        A = torch.empty((ne, n, n), dtype=dt, device=coords.device)
    if A.dtype != dt or A.numel() != ne * n * n:
        raise ValueError("A has the wrong dtype or size")
    if xq is not None and (xq.dtype != torch.float64 or xq.numel() != ne * nq(p, "symmetric") * 3):
        raise ValueError("xq must be float64 with ne*nq*3 entries")
    if status is not None and (status.dtype != torch.int32 or status.numel() < 1):
        raise ValueError("status must be an int32 tensor")
    check("feint_integrate_laplace", lib().feint_integrate_laplace(_ptr(coords), ne, int(p), FORMS[form], _ptr(A),
                                                                   _ptr(xq), _ptr(status), _stream()))
    return A


def laplace_tile_count(p: int, form: str) -> int:
    return lib().feint_laplace_tile_count(int(p), FORMS[form])


def laplace_tile_get(p: int, form: str) -> int:
    return lib().feint_laplace_tile_get(int(p), FORMS[form])


def laplace_tile_set(p: int, form: str, tile: int) -> None:
    check("feint_laplace_tile_set", lib().feint_laplace_tile_set(int(p), FORMS[form], int(tile)))


def laplace_tile_describe(p: int, form: str, tile: int) -> str:
    buf = ctypes.create_string_buffer(32)
    check("feint_laplace_tile_describe", lib().feint_laplace_tile_describe(int(p), FORMS[form], int(tile), buf, 32))
    return buf.value.decode()


def laplace_autotune(coords, p: int, form: str, A, reps: int = 2) -> float:
    ne, _ = _laplace_inputs(coords, p, form)
    best = ctypes.c_double(0)
    check("feint_laplace_autotune", lib().feint_laplace_autotune(_ptr(coords), ne, int(p), FORMS[form], _ptr(A),
                                                                 int(reps), ctypes.byref(best), _stream()))
    return best.value


def adjoint_raw(coords, D, beta, c, f, G, g, p: int, form: str = "fp64", rule: str = "collapsed"):
    """Gradients of sum_e <G_e,A_e> + <g_e,b_e>: (dcoords, dD, dbeta, dc, df), FP64."""
    el = elements(coords, D, beta, c, f)
    ne, n = coords.shape[0], nshp(p)
    dt = out_dtype(form)
    G = G.contiguous().to(dt)
    g = g.contiguous().to(dt)
    if G.numel() != ne * n * n or g.numel() != ne * n:
        raise ValueError("G, g have the wrong size")
    outs = [torch.empty_like(t) for t in (coords, D, beta, c, f)]
    if rule == "collapsed":
        check("feint_integrate_adjoint",
              lib().feint_integrate_adjoint(ctypes.byref(el), int(p), FORMS[form], _ptr(G), _ptr(g),
                                            *[_ptr(o) for o in outs], _stream()))
    else:
        check("feint_integrate_adjoint_rule",
              lib().feint_integrate_adjoint_rule(ctypes.byref(el), int(p), FORMS[form], _rule(rule), _ptr(G),
                                                 _ptr(g), *[_ptr(o) for o in outs], _stream()))
    return tuple(outs)


class IntegrateFn(torch.autograd.Function):
    """(coords, D, beta, c, f) -> (A, b) with the hand-written adjoint as backward."""

    @staticmethod
    def forward(ctx, coords, D, beta, c, f, p, form):
        ctx.p, ctx.form = p, form
        ctx.save_for_backward(coords, D, beta, c, f)
        return integrate_raw(coords, D, beta, c, f, p, form)

    @staticmethod
    def backward(ctx, gA, gb):
        coords, D, beta, c, f = ctx.saved_tensors
        n = nshp(ctx.p)
        dt = out_dtype(ctx.form)
        if gA is None:
            gA = torch.zeros((coords.shape[0], n, n), dtype=dt, device=coords.device)
        if gb is None:
            gb = torch.zeros((coords.shape[0], n), dtype=dt, device=coords.device)
        grads = adjoint_raw(coords, D, beta, c, f, gA, gb, ctx.p, ctx.form)
        return (*grads, None, None)


def integrate(coords, D, beta, c, f, p: int, form: str = "fp64"):
    """Element matrices and load vectors; differentiable for the fp64 and fp32 forms."""
    if torch.is_grad_enabled() and any(t.requires_grad for t in (coords, D, beta, c, f)):
        return IntegrateFn.apply(coords, D, beta, c, f, p, form)
    return integrate_raw(coords, D, beta, c, f, p, form)


def tile_count(p: int, form: str, rule: str = "collapsed") -> int:
    if rule == "collapsed":
        return lib().feint_tile_count(int(p), FORMS[form])
    return lib().feint_rule_tile_count(int(p), FORMS[form], _rule(rule))


def tile_get(p: int, form: str, rule: str = "collapsed") -> int:
    if rule == "collapsed":
        return lib().feint_tile_get(int(p), FORMS[form])
    return lib().feint_rule_tile_get(int(p), FORMS[form], _rule(rule))


def tile_set(p: int, form: str, tile: int, rule: str = "collapsed") -> None:
    if rule == "collapsed":
        check("feint_tile_set", lib().feint_tile_set(int(p), FORMS[form], int(tile)))
    else:
        check("feint_rule_tile_set", lib().feint_rule_tile_set(int(p), FORMS[form], _rule(rule), int(tile)))


def tile_describe(p: int, form: str, tile: int, rule: str = "collapsed") -> str:
    buf = ctypes.create_string_buffer(32)
    if rule == "collapsed":
        check("feint_tile_describe", lib().feint_tile_describe(int(p), FORMS[form], int(tile), buf, 32))
    else:
        check("feint_rule_tile_describe",
              lib().feint_rule_tile_describe(int(p), FORMS[form], _rule(rule), int(tile), buf, 32))
    return buf.value.decode()


def autotune(coords, D, beta, c, f, p: int, form: str, A, b, reps: int = 3, rule: str = "collapsed") -> float:
    """Time every compiled tile shape on these buffers, keep the fastest; returns its ms."""
    el = elements(coords, D, beta, c, f)
    best = ctypes.c_double(0)
    if rule == "collapsed":
        check("feint_autotune", lib().feint_autotune(ctypes.byref(el), int(p), FORMS[form], _ptr(A), _ptr(b),
                                                     int(reps), ctypes.byref(best), _stream()))
    else:
        check("feint_autotune_rule",
              lib().feint_autotune_rule(ctypes.byref(el), None, int(p), FORMS[form], _rule(rule), _ptr(A), _ptr(b),
                                        int(reps), ctypes.byref(best), _stream()))
    return best.value


def autotune_fields(coords, Dv, betav, cv, fv, p: int, form: str, A, b, reps: int = 3,
                    rule: str = "collapsed") -> float:
    """autotune for the vertex-field entry point."""
    fl = fields(coords, Dv, betav, cv, fv)
    best = ctypes.c_double(0)
    check("feint_autotune_rule",
          lib().feint_autotune_rule(None, ctypes.byref(fl), int(p), FORMS[form], _rule(rule), _ptr(A), _ptr(b),
                                    int(reps), ctypes.byref(best), _stream()))
    return best.value


def adjoint_tile_count(p: int, form: str) -> int:
    return lib().feint_adjoint_tile_count(int(p), FORMS[form])


def adjoint_tile_get(p: int, form: str) -> int:
    return lib().feint_adjoint_tile_get(int(p), FORMS[form])


def adjoint_tile_set(p: int, form: str, tile: int) -> None:
    check("feint_adjoint_tile_set", lib().feint_adjoint_tile_set(int(p), FORMS[form], int(tile)))


def adjoint_tile_describe(p: int, form: str, tile: int) -> str:
    buf = ctypes.create_string_buffer(32)
    check("feint_adjoint_tile_describe",
          lib().feint_adjoint_tile_describe(int(p), FORMS[form], int(tile), buf, 32))
    return buf.value.decode()


def adjoint_autotune(coords, D, beta, c, f, G, g, p: int, form: str = "fp64", reps: int = 2) -> float:
    """Time every compiled adjoint block shape on these inputs, keep the fastest; returns its ms."""
    el = elements(coords, D, beta, c, f)
    ne, n = coords.shape[0], nshp(p)
    dt = out_dtype(form)
    G = G.contiguous().to(dt)
    g = g.contiguous().to(dt)
    if G.numel() != ne * n * n or g.numel() != ne * n:
        raise ValueError("G, g have the wrong size")
    outs = [torch.empty_like(t) for t in (coords, D, beta, c, f)]
    best = ctypes.c_double(0)
    check("feint_adjoint_autotune",
          lib().feint_adjoint_autotune(ctypes.byref(el), int(p), FORMS[form], _ptr(G), _ptr(g),
                                       *[_ptr(o) for o in outs], int(reps), ctypes.byref(best), _stream()))
    return best.value


NOALLOC_MAX_NE = 1048576     # FEINT_NOALLOC_MAX_NE


def integrate_mixed_noalloc(coords, D, beta, c, f, p, A, b, offA, offb, form: str = "fp32", status=None):
    """Mixed-degree integration through the library's allocation-free entry
    point (bucketing + persistent launch on the library's fixed scratch):
    every buffer is the caller's; the tables of degrees 1..6 must have been
    prepared (`prepare(d)`); at most NOALLOC_MAX_NE elements."""
    if form not in ("fp32", "fp64"):
        raise ValueError("mixed batches support the fp32 and fp64 forms")
    if p.dtype != torch.int8 or not p.is_contiguous() or p.numel() != coords.shape[0]:
        raise TypeError("p must be a contiguous int8 tensor with one entry per element")
    ne = coords.shape[0]
    if offA.dtype != torch.int64 or offb.dtype != torch.int64 or offA.numel() < ne + 1 or offb.numel() < ne + 1:
        raise ValueError("offA, offb must be int64 with ne + 1 entries")
    dt = out_dtype(form)
    if A.dtype != dt or b.dtype != dt:
        raise ValueError("A, b must have the form's dtype")
    el = elements(coords, D, beta, c, f)
    code = lib().feint_integrate_mixed_noalloc(ctypes.byref(el), _ptr(p), FORMS[form], _ptr(A), _ptr(b),
                                               _ptr(offA), _ptr(offb), _ptr(status), _stream())
    if code == -6:
        raise FeintError("feint_integrate_mixed_noalloc", code, lib().feint_last_error().decode())
    check("feint_integrate_mixed_noalloc", code)


class MixedPlan:
    """Mixed-degree batches (degrees 1..6) through one persistent,
    degree-bucketed launch; optionally captured once into a HIP graph."""

    def __init__(self, ne_max: int, form: str = "fp32"):
        if form not in ("fp32", "fp64"):
            raise ValueError("mixed batches support the fp32 and fp64 forms")
        self.form = form
        self.ne_max = int(ne_max)
        h = ctypes.c_void_p()
        check("feint_mixed_plan_create", lib().feint_mixed_plan_create(self.ne_max, FORMS[form], ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().feint_mixed_plan_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._captured = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bucket(self, p, status=None):
        """Degree bucketing of p (int8 device tensor); returns (offA, offb), int64 [ne+1]."""
        if p.dtype != torch.int8 or not p.is_cuda or not p.is_contiguous():
            raise TypeError("p must be a contiguous int8 CUDA tensor")
        ne = p.numel()
        offA = torch.empty(ne + 1, dtype=torch.int64, device=p.device)
        offb = torch.empty(ne + 1, dtype=torch.int64, device=p.device)
        check("feint_mixed_bucket", lib().feint_mixed_bucket(self._h, _ptr(p), ne, _ptr(offA), _ptr(offb),
                                                             _ptr(status), _stream()))
        return offA, offb

    def alloc_outputs(self, offA, offb):
        """Packed outputs sized from the totals in offA[-1], offb[-1] (synchronises)."""
        dt = out_dtype(self.form)
        nA, nb = int(offA[-1].item()), int(offb[-1].item())
        return (torch.empty(max(nA, 1), dtype=dt, device=offA.device),
                torch.empty(max(nb, 1), dtype=dt, device=offA.device))

    def integrate(self, coords, D, beta, c, f, A, b, offA, offb, status=None):
        el = elements(coords, D, beta, c, f)
        check("feint_integrate_mixed", lib().feint_integrate_mixed(self._h, ctypes.byref(el), _ptr(A), _ptr(b),
                                                                   _ptr(offA), _ptr(offb), _ptr(status), _stream()))

    def capture(self, coords, D, beta, c, f, p, A, b, offA, offb, status=None):
        """Capture bucketing + persistent launch for these buffers into a HIP graph.

        The graph holds raw device pointers, so the plan keeps references to
        every captured tensor until the next capture or close(): a replay
        never writes into memory the caching allocator has handed out again.
        """
        el = elements(coords, D, beta, c, f)
        self._captured = None
        check("feint_mixed_graph_capture",
              lib().feint_mixed_graph_capture(self._h, ctypes.byref(el), _ptr(p), _ptr(A), _ptr(b), _ptr(offA),
                                              _ptr(offb), _ptr(status), _stream()))
        self._captured = (coords, D, beta, c, f, p, A, b, offA, offb, status)

    def replay(self):
        check("feint_mixed_graph_launch", lib().feint_mixed_graph_launch(self._h, _stream()))

    def autotune(self, coords, D, beta, c, f, A, b, offA, offb, reps: int = 2) -> float:
        el = elements(coords, D, beta, c, f)
        best = ctypes.c_double(0)
        check("feint_mixed_autotune", lib().feint_mixed_autotune(self._h, ctypes.byref(el), _ptr(A), _ptr(b),
                                                                 _ptr(offA), _ptr(offb), int(reps),
                                                                 ctypes.byref(best), _stream()))
        return best.value

    @property
    def tile(self) -> int:
        return lib().feint_mixed_tile_get(self._h)

    @tile.setter
    def tile(self, t: int):
        check("feint_mixed_tile_set", lib().feint_mixed_tile_set(self._h, int(t)))

    @property
    def tile_count(self) -> int:
        return lib().feint_mixed_tile_count(self._h)

    def tile_describe(self, t: int) -> str:
        buf = ctypes.create_string_buffer(64)
        check("feint_mixed_tile_describe", lib().feint_mixed_tile_describe(self._h, int(t), buf, 64))
        return buf.value.decode()


class AsmPlan:
    """Global assembly (CSR) of one degree's element matrices: pattern,
    colouring and position map built once from a host dof map."""

    def __init__(self, dofs, ndof: int):
        import numpy as np
        d = np.ascontiguousarray(dofs, dtype=np.int32)
        ne, n = d.shape
        self._h = ctypes.c_void_p()
        check("feint_asm_plan_create", lib().feint_asm_plan_create(d.ctypes.data_as(ctypes.c_void_p), int(ne),
                                                                   int(n), int(ndof), ctypes.byref(self._h)))
        self.ne, self.n, self.ndof = int(ne), int(n), int(ndof)
        nnz = ctypes.c_int64(0)
        nc = ctypes.c_int(0)
        check("feint_asm_plan_info", lib().feint_asm_plan_info(self._h, ctypes.byref(nnz), ctypes.byref(nc)))
        self.nnz, self.ncolors = int(nnz.value), int(nc.value)

    def pattern(self):
        """(row_ptr int64 [ndof+1], col_idx int32 [nnz]) as device tensors."""
        row_ptr = torch.empty(self.ndof + 1, dtype=torch.int64, device="cuda")
        col_idx = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        check("feint_asm_plan_pattern", lib().feint_asm_plan_pattern(self._h, _ptr(row_ptr), _ptr(col_idx),
                                                                     _stream()))
        return row_ptr, col_idx

    def colors(self):
        import numpy as np
        out = np.empty(self.ne, dtype=np.int32)
        check("feint_asm_plan_colors", lib().feint_asm_plan_colors(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def assemble(self, A, b, form: str = "fp64", values=None, rhs=None, accumulate: bool = False):
        """values [nnz], rhs [ndof] in the dtype of A (allocated when not given)."""
        dt = out_dtype(form)
        if A.dtype != dt or b.dtype != dt or A.numel() != self.ne * self.n * self.n or b.numel() != self.ne * self.n:
            raise ValueError("A, b do not match the plan and form")
        A = A.contiguous(); b = b.contiguous()
        if values is None:
            values = torch.empty(self.nnz, dtype=dt, device=A.device)
        if rhs is None:
            rhs = torch.empty(self.ndof, dtype=dt, device=A.device)
        check("feint_assemble", lib().feint_assemble(self._h, FORMS[form], _ptr(A), _ptr(b), _ptr(values), _ptr(rhs),
                                                     1 if accumulate else 0, _stream()))
        return values, rhs

    def close(self):
        if self._h:
            lib().feint_asm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
