"""Seeded synthetic workloads: perturbed prism meshes, per-element coefficients,
mixed degrees and adjoint seeds.

This module only draws and arranges inputs.  It holds none of the integration
arithmetic (no quadrature, no basis, no Jacobian): it is shared by the GPU
path and by the CPU oracle used in the tests, so that both see bit-identical
inputs.

Mesh (the paper's geometrically bilinear prisms, Sec. 4): an ``nx x ny`` grid of
squares on [0,1]^2, each split along its (0,0)-(1,1) diagonal into two
counter-clockwise triangles, extruded over ``nz`` layers on [0,1].  Prism
vertices ``v0..v2`` are the bottom triangle and ``v3..v5`` the top one, with
``v(a+3)`` directly above ``v(a)``.  Every strictly interior grid vertex is
moved by an independent uniform offset in ``[-amp*h_d, +amp*h_d]`` per
direction ``d`` (``h = (1/nx, 1/ny, 1/nz)``), so the meshed domain stays the
unit cube.

Coefficients per element: ``D = L L^T + I`` with ``L_ij ~ N(0, 0.3)``,
``beta ~ N(0,1)^3``, ``c ~ U(0,1)``, ``f ~ U(-1,1)``.

Draw order from ``numpy.random.default_rng(seed)`` (PCG64):
  1. vertex offsets ``uniform(-1,1,(nvert,3))``
  2. ``L = normal(0,0.3,(ne,3,3))``
  3. ``beta = normal(0,1,(ne,3))``
  4. ``c = uniform(0,1,ne)``
  5. ``f = uniform(-1,1,ne)``
  6. (mixed batch only) ``p = integers(1,7,ne)`` then ``perm = permutation(ne)``
     applied to every per-element array
  7. (adjoint only, after the above) ``G = normal(0,1,(ne,n,n))``,
     ``g = normal(0,1,(ne,n))``, ``sample = choice(ne,64,replace=False)``
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


def nshp(p: int) -> int:
    """Number of prism shape functions, (p+1)^2 (p+2) / 2 (Table 1, prism row)."""
    return (p + 1) * (p + 1) * (p + 2) // 2


def nq(p: int) -> int:
    """Number of collapsed-Gauss quadrature points, (p+1)^3."""
    return (p + 1) ** 3


@dataclass
class Batch:
    """Element-major FP64 inputs for ``ne`` prisms (C-contiguous arrays)."""

    coords: np.ndarray          # [ne, 6, 3]
    D: np.ndarray               # [ne, 3, 3]
    beta: np.ndarray            # [ne, 3]
    c: np.ndarray               # [ne]
    f: np.ndarray               # [ne]
    p: Optional[np.ndarray] = None   # [ne] int8, mixed batches only
    meta: dict = field(default_factory=dict)

    @property
    def ne(self) -> int:
        return int(self.coords.shape[0])

    def subset(self, idx) -> "Batch":
        idx = np.asarray(idx)
        return Batch(
            np.ascontiguousarray(self.coords[idx]),
            np.ascontiguousarray(self.D[idx]),
            np.ascontiguousarray(self.beta[idx]),
            np.ascontiguousarray(self.c[idx]),
            np.ascontiguousarray(self.f[idx]),
            None if self.p is None else np.ascontiguousarray(self.p[idx]),
            dict(self.meta),
        )


def grid_vertices(nx: int, ny: int, nz: int, amp: float, u: np.ndarray) -> np.ndarray:
    """Perturbed grid vertex positions, id = (k*(ny+1)+j)*(nx+1)+i."""
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    i = i.ravel(); j = j.ravel(); k = k.ravel()
    xyz = np.stack([i / nx, j / ny, k / nz], axis=1).astype(np.float64)
    interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    off = u * (amp * h)
    off[~interior] = 0.0
    return xyz + off


def prism_connectivity(nx: int, ny: int, nz: int) -> np.ndarray:
    """[ne, 6] vertex ids; element id e = ((k*ny + j)*nx + i)*2 + s."""
    def vid(i, j, k):
        return (k * (ny + 1) + j) * (nx + 1) + i

    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k = k.ravel(); j = j.ravel(); i = i.ravel()
    v00 = lambda kk: vid(i, j, kk)
    v10 = lambda kk: vid(i + 1, j, kk)
    v11 = lambda kk: vid(i + 1, j + 1, kk)
    v01 = lambda kk: vid(i, j + 1, kk)
    t0 = [v00(k), v10(k), v11(k), v00(k + 1), v10(k + 1), v11(k + 1)]
    t1 = [v00(k), v11(k), v01(k), v00(k + 1), v11(k + 1), v01(k + 1)]
    conn = np.empty((nx * ny * nz, 2, 6), dtype=np.int64)
    conn[:, 0, :] = np.stack(t0, axis=1)
    conn[:, 1, :] = np.stack(t1, axis=1)
    return conn.reshape(-1, 6)


def make_batch(nx: int, ny: int, nz: int, amp: float = 0.2, seed: int = 0,
               mixed: bool = False, with_conn: bool = False) -> Batch:
    """Mesh + coefficients (draw steps 1-6)."""
    rng = np.random.default_rng(seed)
    nvert = (nx + 1) * (ny + 1) * (nz + 1)
    u = rng.uniform(-1.0, 1.0, (nvert, 3))
    verts = grid_vertices(nx, ny, nz, amp, u)
    conn = prism_connectivity(nx, ny, nz)
    ne = conn.shape[0]
    coords = np.ascontiguousarray(verts[conn])               # [ne, 6, 3]
    L = rng.normal(0.0, 0.3, (ne, 3, 3))
    D = np.einsum("eik,ejk->eij", L, L) + np.eye(3)[None]
    beta = rng.normal(0.0, 1.0, (ne, 3))
    c = rng.uniform(0.0, 1.0, ne)
    f = rng.uniform(-1.0, 1.0, ne)
    meta = dict(nx=nx, ny=ny, nz=nz, amp=amp, seed=seed)
    b = Batch(coords, np.ascontiguousarray(D), beta, c, f, None, meta)
    if with_conn:
        b.meta["conn"] = conn
        b.meta["verts"] = verts
    if mixed:
        pdeg = rng.integers(1, 7, ne).astype(np.int8)
        perm = rng.permutation(ne)
        b = Batch(np.ascontiguousarray(coords[perm]), np.ascontiguousarray(b.D[perm]),
                  np.ascontiguousarray(beta[perm]), np.ascontiguousarray(c[perm]),
                  np.ascontiguousarray(f[perm]), np.ascontiguousarray(pdeg[perm]), meta)
        b.meta["perm"] = perm
    b.meta["rng"] = rng
    return b


def hex_connectivity(nx: int, ny: int, nz: int) -> np.ndarray:
    """One hexahedron per grid cell, vertices v = i + 2j + 4k at the cell's
    corner (ix + i, iy + j, iz + k)."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    vid = lambda i, j, k: (k * (ny + 1) + j) * (nx + 1) + i
    corners = [vid(ix + (v & 1), iy + ((v >> 1) & 1), iz + ((v >> 2) & 1)) for v in range(8)]
    return np.stack(corners, axis=1)


def make_hex_batch(nx: int, ny: int, nz: int, amp: float = 0.2, seed: int = 0) -> Batch:
    """Hexahedral mesh of the perturbed vertex grid (one hexahedron per cell,
    coords [ne, 8, 3]) with the element-constant coefficient recipe."""
    rng = np.random.default_rng(seed)
    nvert = (nx + 1) * (ny + 1) * (nz + 1)
    u = rng.uniform(-1.0, 1.0, (nvert, 3))
    verts = grid_vertices(nx, ny, nz, amp, u)
    conn = hex_connectivity(nx, ny, nz)
    ne = conn.shape[0]
    coords = np.ascontiguousarray(verts[conn])               # [ne, 8, 3]
    L = rng.normal(0.0, 0.3, (ne, 3, 3))
    D = np.einsum("eik,ejk->eij", L, L) + np.eye(3)[None]
    beta = rng.normal(0.0, 1.0, (ne, 3))
    c = rng.uniform(0.0, 1.0, ne)
    f = rng.uniform(-1.0, 1.0, ne)
    return Batch(coords, np.ascontiguousarray(D), beta, c, f, None, dict(nx=nx, ny=ny, nz=nz, amp=amp, seed=seed,
                                                                         element="hexahedron"))


# The six tetrahedra of a cube cell around its main diagonal (corner 0 to
# corner 7, corners v = i + 2j + 4k), each listed with positive orientation.
_TETS_OF_CUBE = [(0, 1, 3, 7), (0, 3, 2, 7), (0, 2, 6, 7), (0, 6, 4, 7), (0, 4, 5, 7), (0, 5, 1, 7)]


def make_tet_batch(nx: int, ny: int, nz: int, amp: float = 0.2, seed: int = 0) -> Batch:
    """Tetrahedral mesh of the perturbed vertex grid (six tetrahedra per cell
    around the cell's main diagonal, coords [ne, 4, 3]) with the
    element-constant coefficient recipe."""
    rng = np.random.default_rng(seed)
    nvert = (nx + 1) * (ny + 1) * (nz + 1)
    u = rng.uniform(-1.0, 1.0, (nvert, 3))
    verts = grid_vertices(nx, ny, nz, amp, u)
    cells = hex_connectivity(nx, ny, nz)
    conn = np.concatenate([cells[:, list(t)] for t in _TETS_OF_CUBE], axis=0)
    ne = conn.shape[0]
    coords = np.ascontiguousarray(verts[conn])               # [ne, 4, 3]
    L = rng.normal(0.0, 0.3, (ne, 3, 3))
    D = np.einsum("eik,ejk->eij", L, L) + np.eye(3)[None]
    beta = rng.normal(0.0, 1.0, (ne, 3))
    c = rng.uniform(0.0, 1.0, ne)
    f = rng.uniform(-1.0, 1.0, ne)
    return Batch(coords, np.ascontiguousarray(D), beta, c, f, None, dict(nx=nx, ny=ny, nz=nz, amp=amp, seed=seed,
                                                                         element="tetrahedron"))


def vertex_fields(ne: int, seed: int):
    """Coefficients given at the six vertices of every element, drawn with the
    element-constant recipe per vertex: D = L L^T + I (L ~ N(0, 0.3^2)),
    beta ~ N(0, 1), c ~ U(0, 1), f ~ U(-1, 1).  Shapes [ne,6,3,3], [ne,6,3],
    [ne,6], [ne,6], FP64, contiguous."""
    rng = np.random.default_rng(seed)
    L = rng.normal(0.0, 0.3, (ne, 6, 3, 3))
    D = np.einsum("evik,evjk->evij", L, L) + np.eye(3)
    beta = rng.normal(0.0, 1.0, (ne, 6, 3))
    c = rng.uniform(0.0, 1.0, (ne, 6))
    f = rng.uniform(-1.0, 1.0, (ne, 6))
    return tuple(np.ascontiguousarray(a) for a in (D, beta, c, f))


def adjoint_seeds(batch: Batch, p: int, dtype=np.float64):
    """Draw step 7: G ~ N(0,1) [ne,n,n], g ~ N(0,1) [ne,n], 64 sampled ids."""
    rng = batch.meta["rng"]
    n = nshp(p)
    ne = batch.ne
    G = rng.normal(0.0, 1.0, (ne, n, n)).astype(dtype, copy=False)
    g = rng.normal(0.0, 1.0, (ne, n)).astype(dtype, copy=False)
    sample = np.sort(rng.choice(ne, min(64, ne), replace=False))
    return G, g, sample


def adjoint_seeds_device(batch: Batch, p: int, seed: int, dtype=None, device="cuda"):
    """Step 7 for batches whose G does not fit comfortably in host memory
    (16384 elements at p = 7: 10.9 GB in FP64): G ~ N(0,1) [ne,n,n] and
    g ~ N(0,1) [ne,n] drawn on the device from torch's generator seeded with
    `seed` (G first, then g), and 64 sampled ids from numpy's generator."""
    import torch
    dtype = dtype or torch.float64
    n = nshp(p)
    ne = batch.ne
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    G = torch.randn((ne, n, n), generator=gen, dtype=dtype, device=device)
    g = torch.randn((ne, n), generator=gen, dtype=dtype, device=device)
    sample = np.sort(np.random.default_rng(seed).choice(ne, min(64, ne), replace=False))
    return G, g, sample


def dof_map(nx: int, ny: int, nz: int, p: int):
    """Global numbering of the degree-p nodal degrees of freedom of the
    structured prism mesh (mesh topology only; no integration arithmetic).

    Local node a = k * ntri + t of an element sits at reference position
    (xi1, xi2) = (i/p, j/p) of the triangle lattice (t runs over j outer, i
    inner, i + j <= p) and at the k-th of the p+1 ascending Gauss-Lobatto
    nodes in zeta.  On the unperturbed grid those nodes are points of the
    lattice (I, J, K), I in [0, p nx], J in [0, p ny], K in [0, p nz]:
      triangle T0 = (v00, v10, v11):  I = p i + i' + j',  J = p j + j',
      triangle T1 = (v00, v11, v01):  I = p i + i',       J = p j + i' + j',
      K = p k + k'.
    Global id = (K (p ny + 1) + J) (p nx + 1) + I.  Returns (dofs [ne, n]
    int32, number of global degrees of freedom)."""
    tri = [(i, j) for j in range(p + 1) for i in range(p + 1 - j)]
    ntri = len(tri)
    n = ntri * (p + 1)
    NI, NJ, NK = p * nx + 1, p * ny + 1, p * nz + 1
    ndof = NI * NJ * NK
    assert ndof < 2 ** 31
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k = k.ravel(); j = j.ravel(); i = i.ravel()
    ti = np.array([t[0] for t in tri]); tj = np.array([t[1] for t in tri])
    kk = np.arange(p + 1)
    dofs = np.empty((nx * ny * nz, 2, n), dtype=np.int64)
    for s in range(2):
        if s == 0:
            I = p * i[:, None] + (ti + tj)[None, :]
            J = p * j[:, None] + tj[None, :]
        else:
            I = p * i[:, None] + ti[None, :]
            J = p * j[:, None] + (ti + tj)[None, :]
        K = p * k[:, None, None] + kk[None, :, None]                    # [e, k', 1]
        g = (K * NJ + J[:, None, :]) * NI + I[:, None, :]              # [e, k', t]
        dofs[:, s, :] = g.reshape(-1, n)
    return np.ascontiguousarray(dofs.reshape(-1, n).astype(np.int32)), int(ndof)


# The workloads of the paper-derived configurations (mesh sizes and amplitudes).
WORKLOADS = {
    "p1_4096":      dict(nx=16, ny=16, nz=8,  amp=0.2, seed=0, p=1),
    "p4_131072":    dict(nx=64, ny=64, nz=16, amp=0.2, seed=1, p=4),
    "mixed_262144": dict(nx=64, ny=64, nz=32, amp=0.2, seed=2, p=None),
    "adj_p3_131072": dict(nx=64, ny=64, nz=16, amp=0.2, seed=3, p=3),
    "p7_16384":     dict(nx=32, ny=32, nz=8,  amp=0.3, seed=4, p=7),
    # the p = 1 distributions at a size where HBM rather than launch latency bounds
    "p1_524288":    dict(nx=64, ny=64, nz=64, amp=0.2, seed=0, p=1),
    # hexahedra (one per cell) on the vertex grid of the p = 4 prism workload
    "hex_p4_65536": dict(nx=64, ny=64, nz=16, amp=0.2, seed=1, p=4, element="hexahedron"),
    # hexahedra at p = 5..7 (element matrices of 6.1, 7.7 and 4.3 GB in FP64)
    "hex_p5_16384": dict(nx=32, ny=32, nz=16, amp=0.2, seed=1, p=5, element="hexahedron"),
    "hex_p6_8192":  dict(nx=32, ny=16, nz=16, amp=0.2, seed=1, p=6, element="hexahedron"),
    "hex_p7_2048":  dict(nx=16, ny=16, nz=8,  amp=0.2, seed=1, p=7, element="hexahedron"),
    # tetrahedra (six per cell) on the vertex grid of the p = 4 prism workload
    "tet_p4_393216": dict(nx=64, ny=64, nz=16, amp=0.2, seed=1, p=4, element="tetrahedron"),
    "tet_p1_393216": dict(nx=64, ny=64, nz=16, amp=0.2, seed=1, p=1, element="tetrahedron"),
    "tet_p2_393216": dict(nx=64, ny=64, nz=16, amp=0.2, seed=1, p=2, element="tetrahedron"),
}


def workload(name: str) -> Batch:
    w = WORKLOADS[name]
    if w.get("element") == "hexahedron":
        return make_hex_batch(w["nx"], w["ny"], w["nz"], w["amp"], w["seed"])
    if w.get("element") == "tetrahedron":
        return make_tet_batch(w["nx"], w["ny"], w["nz"], w["amp"], w["seed"])
    return make_batch(w["nx"], w["ny"], w["nz"], w["amp"], w["seed"], mixed=w["p"] is None)
