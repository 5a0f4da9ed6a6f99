"""Sparse SPD inputs in CSR form (int32 row pointers and column indices).

The matrices are inputs to conjugate gradient; building them is not part of
the solver.  Column indices are sorted within each row.
"""
import numpy as np


def poisson_csr(side, ndim):
    """Standard (2*ndim+1)-point Laplacian on a ``side^ndim`` interior grid.

    Diagonal ``2*ndim``, off-diagonals ``-1``; the zero Dirichlet boundary is
    eliminated, so boundary rows simply have fewer entries.  Unknowns are
    numbered lexicographically with x fastest.  For side=128, ndim=3 this is the
    n=2,097,152, nnz=14,581,760 system of the CG benchmark.
    """
    side = int(side)
    n = side ** ndim
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for _ in range(ndim):
        coords.append(rem % side)
        rem //= side
    # neighbour offsets in ascending column order: -stride_{d-1} ... -1, 0, +1 ... +stride_{d-1}
    strides = [side ** d for d in range(ndim)]
    offs = [(-strides[d], d, -1) for d in reversed(range(ndim))] + [(0, None, 0)] + \
           [(strides[d], d, +1) for d in range(ndim)]
    cols_list, vals_list, valid_list = [], [], []
    for off, d, sgn in offs:
        if d is None:
            valid = np.ones(n, dtype=bool)
            val = float(2 * ndim)
        else:
            c = coords[d]
            valid = (c > 0) if sgn < 0 else (c < side - 1)
            val = -1.0
        cols_list.append(idx + off)
        vals_list.append(np.full(n, val))
        valid_list.append(valid)
    cols = np.stack(cols_list, axis=1)
    vals = np.stack(vals_list, axis=1)
    valid = np.stack(valid_list, axis=1)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[valid].astype(np.int32)
    values = vals[valid].astype(np.float64)
    return rowptr.astype(np.int32), colind, values


def poisson2d_csr_torch(side, device="cuda"):
    """``poisson_csr(side, 2)`` built with torch on ``device`` (same arrays).

    For large batches of inputs: building millions of rows on the host is
    slow, on the device it takes milliseconds.  Returns (rowptr int32,
    colind int32, values float64) tensors.
    """
    import torch
    side = int(side)
    n = side * side
    idx = torch.arange(n, device=device, dtype=torch.int64)
    ix, iy = idx % side, idx // side
    # neighbour slots in ascending column order: -side, -1, 0, +1, +side
    valid = torch.stack([iy > 0, ix > 0, torch.ones_like(ix, dtype=torch.bool), ix < side - 1, iy < side - 1], 1)
    offs = torch.tensor([-side, -1, 0, 1, side], device=device, dtype=torch.int64)
    cols = idx[:, None] + offs[None, :]
    vals = torch.tensor([-1.0, -1.0, 4.0, -1.0, -1.0], device=device, dtype=torch.float64).expand(n, 5)
    rowptr = torch.zeros(n + 1, device=device, dtype=torch.int64)
    rowptr[1:] = torch.cumsum(valid.sum(1), 0)
    return rowptr.to(torch.int32), cols[valid].to(torch.int32), vals[valid].contiguous()


def random_spd_csr(n, seed=0, median=12.0, sigma=1.0, max_degree=200):
    """Random symmetric, strictly diagonally dominant (hence SPD) matrix.

    Configuration model: each row draws an off-diagonal degree
    ``clip(round(LogNormal(ln median, sigma)), 1, max_degree)``; the stubs are
    shuffled and paired, self-pairs dropped and duplicate pairs merged by
    summing.  Each pair carries one N(0,1) value, mirrored to keep A symmetric.
    The diagonal is 1.1 times the absolute off-diagonal row sum (1.0 for a row
    left without off-diagonals).
    """
    rng = np.random.default_rng(seed)
    deg = np.clip(np.rint(rng.lognormal(np.log(median), sigma, n)), 1, max_degree).astype(np.int64)
    stubs = np.repeat(np.arange(n, dtype=np.int64), deg)
    if stubs.size % 2:
        stubs = stubs[:-1]
    rng.shuffle(stubs)
    a, b = stubs[0::2], stubs[1::2]
    v = rng.standard_normal(a.size)
    keep = a != b
    a, b, v = a[keep], b[keep], v[keep]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    vals = np.concatenate([v, v])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, vals = key[order], vals[order]
    ukey, start = np.unique(key, return_index=True)
    vsum = np.add.reduceat(vals, start)
    r = ukey // n
    c = ukey % n
    absrow = np.bincount(r, weights=np.abs(vsum), minlength=n)
    diag = 1.1 * absrow
    diag[absrow == 0] = 1.0
    # merge the diagonal in, keeping columns sorted within each row
    r_all = np.concatenate([r, np.arange(n, dtype=np.int64)])
    c_all = np.concatenate([c, np.arange(n, dtype=np.int64)])
    v_all = np.concatenate([vsum, diag])
    order = np.argsort(r_all * n + c_all, kind="stable")
    r_all, c_all, v_all = r_all[order], c_all[order], v_all[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r_all, minlength=n), out=rowptr[1:])
    return rowptr.astype(np.int32), c_all.astype(np.int32), v_all.astype(np.float64)


def rhs_uniform(n, seed=0, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, int(n))


def rhs_normal(n, seed=0):
    return np.random.default_rng(seed).standard_normal(int(n))


def lognormal_sides(count, lo=64, hi=1024, seed=0):
    """Side lengths ``round(exp(U[ln lo, ln hi]))`` for batched instances."""
    u = np.random.default_rng(seed).uniform(np.log(lo), np.log(hi), int(count))
    return np.rint(np.exp(u)).astype(np.int64)


def csr_to_dense(rowptr, colind, values, n):
    A = np.zeros((n, n))
    for i in range(n):
        for k in range(int(rowptr[i]), int(rowptr[i + 1])):
            A[i, int(colind[k])] += values[k]
    return A
