"""Seeded synthetic input matrices.

This module only builds inputs.  It holds none of IterativeCUR's arithmetic and is the
one module that both the HIP path's tests/benchmarks and the FP64 oracle consume.
Every generator is deterministic in its seed.  Small inputs are made with NumPy in FP64
and rounded once to FP32 (the precision the library reads); large ones can be made
directly on a torch device from the same NumPy-drawn random factors.

Workloads (shapes and spectra of the paper's test problems; the paper's own
SuiteSparse and MATLAB gallery matrices are not available and are stood in for by
these synthetic families):

* planted spectrum  A = P diag(sigma) Q^T with P, Q orthonormal (QR of Gaussians);
* exactly low rank  A = G1 G2^T with Gaussian factors (the paper's Low-Rank matrix,
  §5.1, at any size);
* RBF kernel        A_ij = exp(-||x_i - y_j||^2 / (2 h^2)), x_i, y_j ~ U[0,1]^3;
* batch of planted-spectrum matrices of uneven sizes and tolerances;
* sparse low rank plus noise (CSR): A = P Q + E with sparse Gaussian factors.
"""
import math

import numpy as np


def _rng(seed, stream):
    return np.random.default_rng([int(seed), int(stream)])


def orthonormal(rows, cols, seed, stream):
    """Q factor of the QR of a rows x cols standard Gaussian matrix (FP64)."""
    Z = _rng(seed, stream).standard_normal((rows, cols))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))[None, :]


def planted(m, n, sigma, seed):
    """A = P diag(sigma) Q^T (FP64), with len(sigma) = K <= min(m, n)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    K = sigma.size
    P = orthonormal(m, K, seed, 1)
    Q = orthonormal(n, K, seed, 2)
    return (P * sigma[None, :]) @ Q.T


def planted_geometric(m=2000, n=1500, decades_per=40.0, seed=0):
    """Planted spectrum sigma_i = 10^(-i/40), i = 0 .. min(m,n)-1; default size is the
    2000 x 1500 dense test matrix."""
    k = min(m, n)
    sigma = 10.0 ** (-np.arange(k) / decades_per)
    return planted(m, n, sigma, seed), sigma


def exact_lowrank(m, n, r, seed):
    """A = G1 G2^T with G1 (m x r), G2 (n x r) standard Gaussian (FP64)."""
    g = _rng(seed, 3)
    G1 = g.standard_normal((m, r))
    G2 = g.standard_normal((n, r))
    return G1 @ G2.T


def integer_spectrum(m, n, K, seed, emax=12, density=1.0):
    """A = sum_k 2^e_k p_k q_k^T with p_k, q_k in {-1, 0, 1} (zero with probability
    1 - density) and exponents e_k falling from emax to 0 over the K terms (FP64 holding
    integers).  A has exact rank <= K and a decaying spectrum; with |a_ij| < 2^(8 T) its
    entries are exact in T BF16 pieces, and its sketch with a +-1 operator is an exact
    integer in FP32 while partial sums stay below 2^24."""
    g = _rng(seed, 6)
    e = emax - (np.arange(K) * (emax + 1)) // K
    P = g.integers(-1, 2, (m, K)) * (g.random((m, K)) < density)
    Q = g.integers(-1, 2, (n, K)) * (g.random((n, K)) < density)
    return (P * (2.0 ** e)[None, :]) @ Q.T


def rbf_points(m, n, seed, dim=3):
    """Seeded point sets x (m x dim) and y (n x dim), uniform on [0,1]^dim."""
    g = _rng(seed, 4)
    return g.random((m, dim)), g.random((n, dim))


def rbf(m, n, seed, h=0.5):
    """RBF kernel matrix A_ij = exp(-||x_i - y_j||^2 / (2 h^2)) computed in FP64 with
    NumPy (coordinate-wise squared differences, summed in coordinate order)."""
    x, y = rbf_points(m, n, seed)
    d2 = np.zeros((m, n))
    for k in range(x.shape[1]):
        d2 += (x[:, k][:, None] - y[:, k][None, :]) ** 2
    return np.exp(-d2 / (2.0 * h * h))


def rbf_torch(m, n, seed, h=0.5, device="cuda", block=4096):
    """Same matrix as rbf(), built on a torch device in row blocks, returned as a
    contiguous FP32 tensor.  Values equal rbf()'s up to the last bit of the device's
    FP64 exp; tests that compare against the oracle copy this tensor to the host
    rather than regenerating it."""
    import torch
    x, y = rbf_points(m, n, seed)
    xt = torch.from_numpy(x).to(device)
    yt = torch.from_numpy(y).to(device)
    out = torch.empty((m, n), dtype=torch.float32, device=device)
    for r0 in range(0, m, block):
        r1 = min(m, r0 + block)
        d2 = torch.zeros((r1 - r0, n), dtype=torch.float64, device=device)
        for k in range(x.shape[1]):
            d2 += (xt[r0:r1, k][:, None] - yt[:, k][None, :]) ** 2
        out[r0:r1] = torch.exp(-d2 / (2.0 * h * h)).to(torch.float32)
    return out


def planted_torch(m, n, sigma, seed, device="cuda", noise=0.0, noise_seed=None):
    """A = P diag(sigma) Q^T (+ noise * N(0,1)) built on a torch device in FP64 and
    returned as FP32.  P, Q come from NumPy-drawn Gaussians (same streams as
    planted()) orthonormalised on the device."""
    import torch
    sigma = np.asarray(sigma, dtype=np.float64)
    K = sigma.size
    Zp = torch.from_numpy(_rng(seed, 1).standard_normal((m, K))).to(device)
    Zq = torch.from_numpy(_rng(seed, 2).standard_normal((n, K))).to(device)
    P, Rp = torch.linalg.qr(Zp)
    P = P * torch.sign(torch.diagonal(Rp))[None, :]
    del Zp, Rp
    Q, Rq = torch.linalg.qr(Zq)
    Q = Q * torch.sign(torch.diagonal(Rq))[None, :]
    del Zq, Rq
    s = torch.from_numpy(sigma).to(device)
    A = ((P * s[None, :]) @ Q.T).to(torch.float32)
    del P, Q
    if noise:
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed if noise_seed is None else noise_seed) + 7919)
        for r0 in range(0, m, 4096):
            r1 = min(m, r0 + 4096)
            E = torch.randn((r1 - r0, n), generator=gen, dtype=torch.float64, device=device)
            A[r0:r1] = (A[r0:r1].double() + noise * E).float()
    return A


def precision_form_sigma(K=4096):
    """sigma_i = (1 + i)^-2, truncated to K terms."""
    return (1.0 + np.arange(K)) ** -2.0


def precision_form_device(m=60000, n=40000, K=4096, seed=0, noise_rel=1e-9, device="cuda"):
    """The precision-form test matrix A = P diag((1+i)^-2) Q^T + E on the device, FP32:
    P (m x K), Q (n x K) orthonormal from device-drawn Gaussians (K = 4096 terms; the tail
    beyond them is about 2e-6 relative), E Gaussian scaled so that ||E||_F = noise_rel
    ||P diag Q^T||_F (a literal 1e-9 N(0,1) per entry would exceed a 1e-5 tolerance at
    this size)."""
    import torch
    A = planted_device(m, n, precision_form_sigma(K), seed, device=device)
    if noise_rel:
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed) * 2 + 7919)
        scale = noise_rel * float(np.sqrt(np.sum(precision_form_sigma(K) ** 2))) / np.sqrt(float(m) * n)
        for r0 in range(0, m, 4096):
            r1 = min(m, r0 + 4096)
            E = torch.randn((r1 - r0, n), generator=gen, dtype=torch.float64, device=device)
            A[r0:r1] = (A[r0:r1].double() + scale * E).float()
            del E
    return A


def low_rank_device(m=30000, n=30000, r=2000, seed=0, device="cuda"):
    """The rank-adaptive Low-Rank matrix of the paper's first experiment (§5.1):
    A = G1 G2^T with G1 (m x r) and G2 (n x r) standard Gaussian, drawn by the device's
    own generator (seeded).  The paper's matrix is exactly rank r in FP64; stored in FP32
    a product of unrounded Gaussians would carry a full-rank rounding term of about 2^-24
    of its entries, which the cross amplifies past a 1e-6 tolerance at this size.  So the
    Gaussians are rounded to multiples of 1/8 (each entry's law stays N(0,1) to within that
    grid): every product entry is then a multiple of 1/64 below 2^18 in magnitude, exact in
    FP32, and A is exactly rank r as stored."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 2 + 104729)
    G1 = torch.round(8.0 * torch.randn((m, r), generator=gen, dtype=torch.float64, device=device)) / 8.0
    G2 = torch.round(8.0 * torch.randn((n, r), generator=gen, dtype=torch.float64, device=device)) / 8.0
    A = torch.empty((m, n), dtype=torch.float32, device=device)
    for r0 in range(0, m, 4096):
        r1 = min(m, r0 + 4096)
        A[r0:r1] = (G1[r0:r1] @ G2.T).float()
    del G1, G2
    return A


def batch_specs(count=512, seed=0, m_range=(500, 8000), r0_range=(10.0, 400.0),
                logtol_range=(-6.0, -2.0)):
    """Per-matrix (m, n, r0, tol, K) for the uneven batch: m, n uniform integers,
    r0 uniform, tol log-uniform, sigma_i = exp(-i / r0) truncated at
    K = min(m, n, ceil(23 r0)) terms (sigma_K < 1e-10)."""
    g = _rng(seed, 5)
    specs = []
    for _ in range(count):
        m = int(g.integers(m_range[0], m_range[1] + 1))
        n = int(g.integers(m_range[0], m_range[1] + 1))
        r0 = float(g.uniform(*r0_range))
        tol = float(10.0 ** g.uniform(*logtol_range))
        K = int(min(m, n, math.ceil(23.0 * r0)))
        specs.append({"m": m, "n": n, "r0": r0, "tol": tol, "K": K})
    return specs


def batch_sigma(r0, K):
    return np.exp(-np.arange(K) / r0)


def planted_device(m, n, sigma, seed, device="cuda"):
    """A = P diag(sigma) Q^T with P, Q orthonormal from the QR of Gaussians drawn by the
    device's own generator (seeded), computed in FP64 on the device, returned as FP32.
    For large batches, where drawing the Gaussians on the host would dominate."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 2 + 1)
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    K = s.numel()
    P, Rp = torch.linalg.qr(torch.randn((m, K), generator=gen, dtype=torch.float64, device=device))
    P = P * torch.sign(torch.diagonal(Rp))[None, :]
    del Rp
    Q, Rq = torch.linalg.qr(torch.randn((n, K), generator=gen, dtype=torch.float64, device=device))
    Q = Q * torch.sign(torch.diagonal(Rq))[None, :]
    del Rq
    A = ((P * s[None, :]) @ Q.T).to(torch.float32)
    return A


def _sparse_rows(rows, cols, per_row, g, scale=1.0):
    """rows x cols CSR (scipy, FP64) with `per_row` distinct random columns per row and
    N(0, scale^2) values."""
    import scipy.sparse as sp
    per_row = min(per_row, cols)
    idx = np.argsort(g.random((rows, cols)), axis=1)[:, :per_row] if cols <= 4096 else \
        np.stack([g.choice(cols, per_row, replace=False) for _ in range(rows)])
    data = scale * g.standard_normal((rows, per_row))
    indptr = np.arange(0, rows * per_row + 1, per_row, dtype=np.int64)
    return sp.csr_matrix((data.ravel(), idx.ravel(), indptr), shape=(rows, cols))


def sparse_lowrank(m, n, r=300, p_per_row=5, q_per_row=100, noise_per_row=20, noise=1e-8, seed=0, decay=0.0):
    """A = P Q + E as a canonical scipy CSR matrix (FP64): P (m x r) with p_per_row
    Gaussian entries per row, Q (r x n) with q_per_row per row, E with noise_per_row
    entries of size `noise` per row (duplicates summed).  True rank r (the sparse
    low-rank-plus-noise workload, default shape scaled by the caller).  decay > 0 scales
    row k of Q by 10^(-k decay), giving a decaying spectrum."""
    import scipy.sparse as sp
    g = _rng(seed, 6)
    P = _sparse_rows(m, r, p_per_row, g)
    Q = _sparse_rows(r, n, q_per_row, g)
    if decay:
        Q = sp.diags(10.0 ** (-decay * np.arange(r))) @ Q
    E = _sparse_rows(m, n, noise_per_row, g, scale=noise)
    A = (P @ Q + E).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def csr_to_f32(A):
    """(rowptr int64, colind int32, vals float32) of a scipy CSR matrix, plus the FP64
    dense copy of the rounded values (for the oracle; small matrices only)."""
    A = A.tocsr()
    A.sort_indices()
    rowptr = A.indptr.astype(np.int64)
    colind = A.indices.astype(np.int32)
    vals = A.data.astype(np.float32)
    return rowptr, colind, vals


def csr_dense64(rowptr, colind, vals, shape):
    import scipy.sparse as sp
    return sp.csr_matrix((vals.astype(np.float64), colind, rowptr), shape=shape).toarray()


def to_f32(A):
    """Round an FP64 array once to FP32 (the values the library reads) and return both
    the FP32 array and its exact FP64 copy (the values the oracle reads)."""
    A32 = np.ascontiguousarray(np.asarray(A, dtype=np.float64).astype(np.float32))
    return A32, A32.astype(np.float64)
