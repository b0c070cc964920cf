"""Pins of the degree-of-freedom map and of the oracle's global assembly
(Sec. 2: element matrices summed through the element-to-global numbering),
checked against what the assembled operator must satisfy."""
import numpy as np
import pytest

import oracle
from paper_1310_1194_amd import meshgen


def dof_positions(batch, dofs, p):
    """Physical position of every element's local nodes (oracle geometry map);
    returns [ndof, 3] and the largest disagreement between elements sharing a dof."""
    nodes = oracle.nodes(p)
    ndof = int(dofs.max()) + 1
    pos = np.full((ndof, 3), np.nan)
    worst = 0.0
    for e in range(batch.ne):
        for a in range(nodes.shape[0]):
            x = oracle.geometry(batch.coords[e], nodes[a])[3]
            g = dofs[e, a]
            if np.isnan(pos[g, 0]):
                pos[g] = x
            else:
                worst = max(worst, float(np.abs(pos[g] - x).max()))
    return pos, worst


def dense(row_ptr, cols, vals, ndof):
    M = np.zeros((ndof, ndof))
    for i in range(ndof):
        M[i, cols[row_ptr[i]:row_ptr[i + 1]]] = vals[row_ptr[i]:row_ptr[i + 1]]
    return M


@pytest.mark.parametrize("p,dims", [(1, (3, 2, 2)), (2, (2, 2, 2)), (3, (2, 1, 1))])
def test_dof_map_is_the_node_lattice(p, dims):
    """Each global dof is one physical point: all elements that share it map
    their local node to the same position, and distinct dofs are distinct points."""
    batch = meshgen.make_batch(*dims, amp=0.2, seed=3)
    dofs, ndof = meshgen.dof_map(*dims, p)
    assert dofs.shape == (batch.ne, oracle.nshp(p))
    assert ndof == (p * dims[0] + 1) * (p * dims[1] + 1) * (p * dims[2] + 1)
    assert sorted(np.unique(dofs)) == list(range(ndof))          # every lattice node is used
    assert all(len(set(r)) == len(r) for r in dofs)
    pos, worst = dof_positions(batch, dofs, p)
    assert worst < 1e-14
    d = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=2) + np.eye(ndof)
    assert d.min() > 1e-6


def element_mats(batch, p, D=None, beta=None, c=None, f=None):
    ne = batch.ne
    D = batch.D if D is None else np.broadcast_to(D, (ne, 3, 3)).copy()
    beta = batch.beta if beta is None else np.broadcast_to(beta, (ne, 3)).copy()
    c = batch.c if c is None else np.full(ne, float(c))
    f = batch.f if f is None else np.full(ne, float(f))
    A, b, _ = oracle.integrate(p, batch.coords, D, beta, c, f)
    return A, b


def test_pattern_is_the_coupling_graph():
    p, dims = 2, (2, 2, 1)
    batch = meshgen.make_batch(*dims, amp=0.2, seed=5)
    dofs, ndof = meshgen.dof_map(*dims, p)
    A, b = element_mats(batch, p)
    row_ptr, cols, vals, rhs = oracle.assemble(dofs, ndof, A, b)
    pairs = {(int(i), int(j)) for r in dofs for i in r for j in r}
    got = {(i, int(cols[k])) for i in range(ndof) for k in range(row_ptr[i], row_ptr[i + 1])}
    assert got == pairs
    assert all(np.all(np.diff(cols[row_ptr[i]:row_ptr[i + 1]]) > 0) for i in range(ndof))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_assembled_operator_invariants(p):
    dims = (2, 2, 2) if p < 3 else (2, 1, 1)
    batch = meshgen.make_batch(*dims, amp=0.2, seed=7 + p)
    dofs, ndof = meshgen.dof_map(*dims, p)
    I3 = np.eye(3)
    # pure diffusion (D = I): symmetric, zero row sums, and K u = 0 on interior
    # rows for a linear u (the geometry functions lie in the element space, the
    # rule integrates these integrands exactly, and Laplace(u) = 0)
    K_e, _ = element_mats(batch, p, D=I3, beta=np.zeros(3), c=0.0, f=0.0)
    K = dense(*oracle.assemble(dofs, ndof, K_e, np.zeros((batch.ne, dofs.shape[1])))[:3], ndof)
    scale = np.abs(K).max()
    assert np.abs(K - K.T).max() < 1e-13 * scale
    assert np.abs(K.sum(axis=1)).max() < 1e-12 * scale
    pos, _ = dof_positions(batch, dofs, p)
    u = pos @ np.array([0.3, -1.1, 0.7]) + 0.25
    interior = np.all((pos > 1e-9) & (pos < 1 - 1e-9), axis=1)
    assert interior.any() or p < 2
    Ku = K @ u
    assert np.abs(Ku[interior]).max() < 1e-11 * scale * np.abs(u).max()
    assert np.abs(Ku[~interior]).max() > 1e-3 * scale * np.abs(u).max()   # the boundary flux is not zero
    # mass (c = 1): total = volume of the unit cube; load (f = 1): total = volume
    M_e, b_e = element_mats(batch, p, D=np.zeros((3, 3)), beta=np.zeros(3), c=1.0, f=1.0)
    row_ptr, cols, vals, rhs = oracle.assemble(dofs, ndof, M_e, b_e)
    assert abs(vals.sum() - 1.0) < 1e-13
    assert abs(rhs.sum() - 1.0) < 1e-13
    # general coefficients: sum of all entries equals the sum of the element sums
    A_e, b_e = element_mats(batch, p)
    row_ptr, cols, vals, rhs = oracle.assemble(dofs, ndof, A_e, b_e)
    assert abs(vals.sum() - A_e.sum()) < 1e-12 * np.abs(A_e).sum()
    assert abs(rhs.sum() - b_e.sum()) < 1e-12 * np.abs(b_e).sum()
