"""Helpers of the GPU parity tests: seeded inputs on the device, the oracle on the
host, and the relative-error metrics the tolerances are stated in."""
import sys

import numpy as np

import oracle
from paper_1310_1194_amd import meshgen


def flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(batch):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t(batch.coords), t(batch.D), t(batch.beta), t(batch.c), t(batch.f)


def rel_errors(got, ref):
    """(global relative Frobenius error, max over elements of the per-element one)."""
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    glob = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    per = np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    return float(glob), float(per.max())


def grad_errors(got, ref, floor=1e-3):
    """Errors of one gradient array, [ne, ...]: (global relative Frobenius
    error, max over elements of ||got_e - ref_e|| / d_e).  d_e is the element's
    own reference norm, floored at `floor` times the root-mean-square of those
    norms over the batch, so that an element whose gradient happens to be
    nearly zero (dc, df are single sums of random terms) is judged on the
    batch's scale rather than on its own."""
    ne = ref.shape[0]
    got = np.asarray(got, dtype=np.float64).reshape(ne, -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ne, -1)
    glob = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    nrm = np.linalg.norm(ref, axis=1)
    d = np.maximum(nrm, floor * np.sqrt(np.mean(nrm ** 2)))
    per = np.linalg.norm(got - ref, axis=1) / d
    return float(glob), float(per.max())


def oracle_of(batch, p):
    return oracle.integrate(p, batch.coords, batch.D, batch.beta, batch.c, batch.f)


def small_batch(p, seed=0, amp=0.2):
    """A few tiles' worth of elements, with a ragged count."""
    dims = {1: (5, 3, 3), 2: (4, 3, 2), 3: (3, 3, 2), 4: (3, 2, 2), 5: (2, 2, 2), 6: (2, 2, 1), 7: (2, 1, 1)}[p]
    b = meshgen.make_batch(*dims, amp=amp, seed=seed)
    keep = b.ne - 1 if b.ne > 2 else b.ne   # ragged: drop the last element
    return b.subset(np.arange(keep))
