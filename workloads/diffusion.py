"""Variable-coefficient diffusion problems -div(k grad u) = f (inputs only).

k = exp(g) with g a stationary Gaussian random field of standard deviation
sigma and squared-exponential covariance exp(-r^2 / (2 ell^2)), drawn by
FFT synthesis on a periodic grid twice the size of the domain (so the
periodic wrap-around does not correlate opposite edges), scaled so that its
variance is sigma^2 in expectation.

The discretisation is the vertex-centred 5-point finite-volume scheme on an
N x N interior grid (h = 1) with zero Dirichlet values on the ring of nodes
around it: the transmissibility of the face between nodes a and b is the
harmonic mean 2 k_a k_b / (k_a + k_b), the diagonal holds the sum of the
node's four face transmissibilities and each interior neighbour gets -T.
With k = 1 everywhere this is the standard 5-point Laplacian (4, -1).
"""
import numpy as np


def grf_log_k(n, seed=0, sigma=1.0, ell=16.0):
    """g on the (n+2) x (n+2) nodes (interior plus the Dirichlet ring)."""
    m = n + 2
    M = 2 * m
    rng = np.random.default_rng(seed)
    d = np.minimum(np.arange(M), M - np.arange(M)).astype(np.float64)   # periodic distance
    cov = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * ell * ell))
    lam = np.maximum(np.fft.fft2(cov).real, 0.0)                       # covariance eigenvalues
    xi = rng.standard_normal((M, M))
    g = np.fft.ifft2(np.sqrt(lam) * np.fft.fft2(xi)).real                # E[g^2] = cov(0) = 1
    return sigma * g[:m, :m]


def diffusion_csr(k):
    """CSR (int32, int32, float64) of the FV matrix for node coefficients k
    ((n+2) x (n+2), ring included); unknowns are the n x n interior nodes,
    numbered row-major with x fastest; column indices sorted in each row."""
    k = np.asarray(k, dtype=np.float64)
    m = k.shape[0]
    n = m - 2
    kc = k[1:-1, 1:-1]

    def t(a, b):
        return 2.0 * a * b / (a + b)
    ts = t(kc, k[:-2, 1:-1])    # face to the node below (y - 1)
    tw = t(kc, k[1:-1, :-2])    # x - 1
    te = t(kc, k[1:-1, 2:])     # x + 1
    tn = t(kc, k[2:, 1:-1])     # y + 1
    diag = ts + tw + te + tn
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    idx = iy * n + ix
    cols = np.stack([idx - n, idx - 1, idx, idx + 1, idx + n], axis=-1)
    vals = np.stack([-ts, -tw, diag, -te, -tn], axis=-1)
    valid = np.stack([iy > 0, ix > 0, np.ones_like(ix, bool), ix < n - 1, iy < n - 1], axis=-1)
    counts = valid.reshape(-1, 5).sum(1)
    rowptr = np.zeros(n * n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return (rowptr.astype(np.int32), cols.reshape(-1, 5)[valid.reshape(-1, 5)].astype(np.int32),
            vals.reshape(-1, 5)[valid.reshape(-1, 5)].astype(np.float64))


def diffusion_problem(n, seed=0, sigma=1.0, ell=16.0):
    """(rowptr, colind, values, log_k interior n x n, f) for field `seed`."""
    g = grf_log_k(n, seed=seed, sigma=sigma, ell=ell)
    rp, ci, v = diffusion_csr(np.exp(g))
    f = np.random.default_rng(10_000_000 + seed).standard_normal(n * n)
    return rp, ci, v, g[1:-1, 1:-1].copy(), f


def grf_log_k_torch(n, seed=0, sigma=1.0, ell=16.0, device="cuda"):
    """grf_log_k on ``device`` with torch's generator (a different random
    stream than the numpy version: same law, same seeding discipline)."""
    import torch
    m = n + 2
    M = 2 * m
    gen = torch.Generator(device=device).manual_seed(int(seed))
    ar = torch.arange(M, device=device, dtype=torch.float64)
    d = torch.minimum(ar, M - ar)
    cov = torch.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * ell * ell))
    lam = torch.clamp(torch.fft.fft2(cov).real, min=0.0)
    xi = torch.randn((M, M), generator=gen, device=device, dtype=torch.float64)
    g = torch.fft.ifft2(torch.sqrt(lam) * torch.fft.fft2(xi)).real
    return sigma * g[:m, :m]


def diffusion_csr_torch(k):
    """diffusion_csr for a torch tensor k on any device (same arrays)."""
    import torch
    m = k.shape[0]
    n = m - 2
    kc = k[1:-1, 1:-1]

    def t(a, b):
        return 2.0 * a * b / (a + b)
    ts, tw, te, tn = t(kc, k[:-2, 1:-1]), t(kc, k[1:-1, :-2]), t(kc, k[1:-1, 2:]), t(kc, k[2:, 1:-1])
    diag = ts + tw + te + tn
    iy, ix = torch.meshgrid(torch.arange(n, device=k.device), torch.arange(n, device=k.device), indexing="ij")
    idx = iy * n + ix
    cols = torch.stack([idx - n, idx - 1, idx, idx + 1, idx + n], dim=-1).reshape(-1, 5)
    vals = torch.stack([-ts, -tw, diag, -te, -tn], dim=-1).reshape(-1, 5)
    valid = torch.stack([iy > 0, ix > 0, torch.ones_like(ix, dtype=torch.bool), ix < n - 1, iy < n - 1],
                        dim=-1).reshape(-1, 5)
    rowptr = torch.zeros(n * n + 1, dtype=torch.int64, device=k.device)
    rowptr[1:] = torch.cumsum(valid.sum(1), 0)
    return rowptr.to(torch.int32), cols[valid].to(torch.int32), vals[valid].contiguous()


def diffusion_problem_torch(n, seed=0, sigma=1.0, ell=16.0, device="cuda"):
    """(rowptr, colind, values, log_k [n, n], f) as torch tensors on ``device``."""
    import torch
    g = grf_log_k_torch(n, seed=seed, sigma=sigma, ell=ell, device=device)
    rp, ci, v = diffusion_csr_torch(torch.exp(g))
    gen = torch.Generator(device=device).manual_seed(10_000_000 + int(seed))
    f = torch.randn(n * n, generator=gen, device=device, dtype=torch.float64)
    return rp, ci, v, g[1:-1, 1:-1].contiguous(), f


def diffusion_planes(k):
    """The FV operator of diffusion_csr as five per-pixel planes [S, W, C, E, N]
    (numpy float64, [5, n, n]); zero where the neighbour is on the ring."""
    k = np.asarray(k, dtype=np.float64)
    kc = k[1:-1, 1:-1]

    def t(a, b):
        return 2.0 * a * b / (a + b)
    ts, tw, te, tn = t(kc, k[:-2, 1:-1]), t(kc, k[1:-1, :-2]), t(kc, k[1:-1, 2:]), t(kc, k[2:, 1:-1])
    c = ts + tw + te + tn
    s, w, e, nn = -ts.copy(), -tw.copy(), -te.copy(), -tn.copy()
    s[0, :] = 0.0
    w[:, 0] = 0.0
    e[:, -1] = 0.0
    nn[-1, :] = 0.0
    return np.stack([s, w, c, e, nn])


def diffusion_planes_torch(k):
    """diffusion_planes for a torch tensor k (same values)."""
    import torch
    kc = k[1:-1, 1:-1]

    def t(a, b):
        return 2.0 * a * b / (a + b)
    ts, tw, te, tn = t(kc, k[:-2, 1:-1]), t(kc, k[1:-1, :-2]), t(kc, k[1:-1, 2:]), t(kc, k[2:, 1:-1])
    c = ts + tw + te + tn
    s, w, e, nn = -ts.clone(), -tw.clone(), -te.clone(), -tn.clone()
    s[0, :] = 0.0
    w[:, 0] = 0.0
    e[:, -1] = 0.0
    nn[-1, :] = 0.0
    return torch.stack([s, w, c, e, nn])
