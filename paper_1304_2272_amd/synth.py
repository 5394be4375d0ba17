"""Seeded synthetic inputs for the mixed-model GWAS GLS problem (Eq. 1).

This module draws inputs only: it contains none of the method's arithmetic
(no factorisation, no triangular solve, no normal equations).  Both the CPU
oracle and the GPU library consume what it produces.

Recipe (the shapes and distributions of the problem statement of Section 1,
with the kinship-style covariance used in the mixed model):

* k = 2000 background markers with allele frequencies f_j ~ U(0.05, 0.5);
  Z (n x k) has Binomial(2, f_j) entries, each column standardised with its
  empirical mean and standard deviation (ddof = 0; monomorphic columns are
  redrawn).
* Phi = Z Z^T / k and M = sigma^2 (h^2 Phi + (1 - h^2) I), SPD.
* X_L = [1, N(0,1) covariates] (n x (p-1)); beta ~ N(0, 1) ((p-1) x t).
* e ~ N(0, M) per trait column, drawn as
  sigma sqrt(h^2/k) Z g + sigma sqrt(1-h^2) eps with g ~ N(0, I_k),
  eps ~ N(0, I_n): its covariance is exactly M, and no factor of M is needed.
* y = X_L beta + e (n x t).
* SNP dosages x_ji ~ Binomial(2, f_i) with f_i ~ U(0.05, 0.5) drawn per SNP.
  Dosages are produced in fixed chunks of CHUNK columns, each chunk from its
  own child stream, so any column range is reproducible whatever the block
  partition used to read it.

Layouts: X_R is returned SNP-major, shape (cols, n), C-contiguous, which is the
column-major n x cols matrix whose column i is SNP i.
"""

from __future__ import annotations

import numpy as np

CHUNK = 1024          # columns per reproducible dosage chunk
K_BACKGROUND = 2000   # markers behind Phi

# child-stream indices of SeedSequence(seed)
_S_FZ, _S_Z, _S_XL, _S_BETA, _S_G, _S_EPS, _S_XR = range(7)


def _child(seed: int, *key: int) -> np.random.Generator:
    ss = np.random.SeedSequence(seed, spawn_key=tuple(key))
    return np.random.Generator(np.random.PCG64(ss))


def _dosages_from_uniform(u, f):
    """Binomial(2, f) from one uniform: 0 if u < (1-f)^2, 2 if u >= 1-f^2, else 1."""
    lo = (1.0 - f) ** 2
    hi = 1.0 - f * f
    return (u >= lo).astype(np.int8) + (u >= hi).astype(np.int8)


def background_genotypes(n: int, seed: int, k: int = K_BACKGROUND) -> np.ndarray:
    """Column-standardised background genotype matrix Z (n x k, float64)."""
    f = _child(seed, _S_FZ).uniform(0.05, 0.5, size=k)
    rng = _child(seed, _S_Z)
    Z = _dosages_from_uniform(rng.random((n, k)), f[None, :]).astype(np.float64)
    for _ in range(100):
        sd = Z.std(axis=0)
        bad = np.flatnonzero(sd == 0.0)
        if bad.size == 0:
            break
        Z[:, bad] = _dosages_from_uniform(rng.random((n, bad.size)), f[None, bad])
    Z -= Z.mean(axis=0)
    Z /= Z.std(axis=0)
    return Z


def covariance(Z: np.ndarray, h2: float = 0.5, sigma2: float = 1.0, device=None):
    """M = sigma^2 (h^2 Z Z^T / k + (1 - h^2) I).

    With ``device`` given (a torch device string) the n x n product is formed
    there in float64 and a torch tensor is returned; otherwise numpy on the host.
    """
    n, k = Z.shape
    if device is None:
        M = (sigma2 * h2 / k) * (Z @ Z.T)
        M[np.diag_indices(n)] += sigma2 * (1.0 - h2)
        return M
    import torch
    Zt = torch.from_numpy(Z).to(device)
    M = torch.mm(Zt, Zt.t().contiguous())
    M.mul_(sigma2 * h2 / k)
    M.diagonal().add_(sigma2 * (1.0 - h2))
    del Zt
    return M


def cohorts(count: int, seed: int, n_lo: int = 2000, n_hi: int = 30000, h2_lo: float = 0.2,
            h2_hi: float = 0.8):
    """Sizes and heritabilities of ``count`` cohorts: n_c ~ U{n_lo..n_hi},
    h2_c ~ U(h2_lo, h2_hi); cohort c draws its inputs from seed (seed, c)."""
    rng = _child(seed, 8)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    h2 = rng.uniform(h2_lo, h2_hi, size=count)
    return [dict(n=int(ns[c]), h2=float(h2[c]), seed=int(seed * 1000 + c)) for c in range(count)]


def make_problem(n: int, p: int, seed: int, t: int = 1, h2: float = 0.5,
                 sigma2: float = 1.0, k: int = K_BACKGROUND, device=None,
                 noise: bool = True):
    """Draw (M, X_L, Y) for one cohort.

    Returns a dict with M (n x n), XL (n x (p-1)), Y (n x t), beta
    ((p-1) x t) and the recipe parameters.  ``noise=False`` gives the
    noise-free y = X_L beta used by planted-coefficient checks.
    """
    if p < 2:
        raise ValueError("p >= 2")
    Z = background_genotypes(n, seed, k)
    M = covariance(Z, h2, sigma2, device)
    XL = np.empty((n, p - 1))
    XL[:, 0] = 1.0
    if p > 2:
        XL[:, 1:] = _child(seed, _S_XL).standard_normal((n, p - 2))
    beta = _child(seed, _S_BETA).standard_normal((p - 1, t))
    Y = XL @ beta
    if noise:
        g = _child(seed, _S_G).standard_normal((k, t))
        eps = _child(seed, _S_EPS).standard_normal((n, t))
        Y = Y + np.sqrt(sigma2 * h2 / k) * (Z @ g) + np.sqrt(sigma2 * (1.0 - h2)) * eps
    return {"M": M, "XL": XL, "Y": Y, "beta": beta, "n": n, "p": p, "t": t,
            "h2": h2, "sigma2": sigma2, "k": k, "seed": seed}


def banded_problem(n: int, p: int, seed: int, w: int, t: int = 1, h2: float = 0.5, sigma2: float = 1.0,
                   cover: int = 8, noise: bool = True, device=None):
    """A cohort whose relatives sit next to each other: M of half-bandwidth w.

    Local markers stand in for shared haplotypes: marker j is carried by a
    window of w + 1 consecutive individuals starting at a_j (windows evenly
    spaced so that each individual is in about ``cover`` of them), with
    Binomial(2, f_j) genotypes, f_j ~ U(0.05, 0.5), standardised within the
    window (monomorphic draws redrawn) and scaled by 1/sqrt(cover).  With Z
    the n x K matrix of these columns, Phi = Z Z^T has Phi(i, i') = 0 for
    |i - i'| > w and M = sigma^2 (h^2 Phi + (1 - h^2) I) is SPD.  e ~ N(0, M)
    is drawn as sigma (sqrt(h^2) Z g + sqrt(1 - h^2) eps).  Returns M in lower
    band storage, an (n, w + 1) array with M_band[j, d] = M(j + d, j), beside
    X_L, Y and beta as :func:`make_problem` draws them.  With ``device`` (a
    torch device string) the band is accumulated there, in the same order
    and float64 operations, and returned as a numpy array.
    """
    if not 1 <= w < n:
        raise ValueError("1 <= w < n")
    L = w + 1
    K = max(1, -(-cover * n // L))
    starts = np.linspace(0, n - L, K).round().astype(np.int64)
    f = _child(seed, 10).uniform(0.05, 0.5, size=K)
    rng = _child(seed, 11)
    g = _child(seed, _S_G).standard_normal((K, t))
    e = np.zeros((n, t))
    zs = []
    for j in range(K):
        z = _dosages_from_uniform(rng.random(L), f[j]).astype(np.float64)
        while z.std() == 0.0:
            z = _dosages_from_uniform(rng.random(L), f[j]).astype(np.float64)
        z = (z - z.mean()) / z.std() / np.sqrt(cover)
        zs.append(z)
        e[starts[j]:starts[j] + L] += np.outer(z, g[j])
    # column r of marker j's window gets z[r + d] z[r] at band offset d
    if device is None:
        band = np.zeros((n, L))
        pad = np.zeros((L + L, L))
        for j in range(K):
            pad[:L] = np.outer(zs[j], zs[j])
            band[starts[j]:starts[j] + L] += np.lib.stride_tricks.as_strided(pad, shape=(L, L),
                                                                             strides=((L + 1) * 8, L * 8))
    else:
        import torch
        bt = torch.zeros((n, L), dtype=torch.float64, device=device)
        pt = torch.zeros((L + L, L), dtype=torch.float64, device=device)
        for j in range(K):
            zt = torch.from_numpy(zs[j]).to(device)
            pt[:L] = torch.outer(zt, zt)
            bt[starts[j]:starts[j] + L] += torch.as_strided(pt, (L, L), (L + 1, L))
        band = bt.cpu().numpy()
        del bt, pt
    # entries past the matrix (row j + d >= n) stay zero
    band *= sigma2 * h2
    band[:, 0] += sigma2 * (1.0 - h2)
    for d in range(1, L):
        band[n - d:, d] = 0.0
    XL = np.empty((n, p - 1))
    XL[:, 0] = 1.0
    if p > 2:
        XL[:, 1:] = _child(seed, _S_XL).standard_normal((n, p - 2))
    beta = _child(seed, _S_BETA).standard_normal((p - 1, t))
    Y = XL @ beta
    if noise:
        eps = _child(seed, _S_EPS).standard_normal((n, t))
        Y = Y + np.sqrt(sigma2 * h2) * e + np.sqrt(sigma2 * (1.0 - h2)) * eps
    return {"M_band": band, "XL": XL, "Y": Y, "beta": beta, "n": n, "p": p, "t": t, "w": w,
            "h2": h2, "sigma2": sigma2, "seed": seed}


def band_to_dense(M_band: np.ndarray) -> np.ndarray:
    """The symmetric n x n matrix of lower band storage (n, w + 1)."""
    n, L = M_band.shape
    M = np.zeros((n, n))
    for d in range(L):
        idx = np.arange(n - d)
        M[idx + d, idx] = M_band[:n - d, d]
        M[idx, idx + d] = M_band[:n - d, d]
    return M


def snp_chunk(n: int, seed: int, chunk: int, dtype=np.float64, cohort=None) -> np.ndarray:
    """Dosage chunk ``chunk`` (CHUNK SNPs), SNP-major (CHUNK, n).

    With ``cohort`` set, the allele frequencies of the chunk's positions are
    the shared ones and the dosages are that cohort's own draw.
    """
    rng = _child(seed, _S_XR, chunk)
    f = rng.uniform(0.05, 0.5, size=CHUNK)
    if cohort is not None:
        rng = _child(seed, _S_XR, chunk, 2 + cohort)
    u = rng.random((CHUNK, n))
    return _dosages_from_uniform(u, f[:, None]).astype(dtype, copy=False)


def snp_block(n: int, seed: int, start: int, cols: int, dtype=np.float64, cohort=None) -> np.ndarray:
    """SNPs [start, start+cols) as a SNP-major (cols, n) array of ``dtype``."""
    out = np.empty((cols, n), dtype=dtype)
    c0 = start // CHUNK
    c1 = (start + cols + CHUNK - 1) // CHUNK
    for c in range(c0, c1):
        blk = snp_chunk(n, seed, c, dtype, cohort)
        lo = max(start, c * CHUNK)
        hi = min(start + cols, (c + 1) * CHUNK)
        out[lo - start:hi - start] = blk[lo - c * CHUNK:hi - c * CHUNK]
    return out


def imputed_block(n: int, seed: int, start: int, cols: int) -> np.ndarray:
    """Non-integer dosages in [0, 2] as imputation gives them (expected
    allele counts): the hard calls of :func:`snp_block` plus N(0, 0.2^2)
    noise, clipped to [0, 2]; SNP-major (cols, n) float64."""
    x = snp_block(n, seed, start, cols, dtype=np.float64)
    noise = _child(seed, _S_XR, 1 << 20, start).normal(0.0, 0.2, size=x.shape)
    return np.clip(x + noise, 0.0, 2.0)


def snp_block_device(n: int, seed: int, start: int, cols: int, device, dtype=None, cohort=None):
    """Device-side dosages for large runs, SNP-major (cols, n) torch tensor.

    Same distribution as :func:`snp_block`, drawn with torch's generator on
    ``device`` (seeded per chunk from the same seed sequence), so values
    differ from the host stream.  Default dtype int8.
    """
    import torch
    dtype = torch.int8 if dtype is None else dtype
    out = torch.empty((cols, n), dtype=dtype, device=device)
    c0 = start // CHUNK
    c1 = (start + cols + CHUNK - 1) // CHUNK
    g = torch.Generator(device=device)
    for c in range(c0, c1):
        st = np.random.SeedSequence(seed, spawn_key=(_S_XR, c, 1)).generate_state(2, np.uint64)
        g.manual_seed(int(st[0] & np.uint64(0x7FFFFFFFFFFFFFFF)))
        f = torch.rand(CHUNK, 1, generator=g, device=device, dtype=torch.float64) * 0.45 + 0.05
        if cohort is not None:   # shared positions and frequencies, the cohort's own dosages
            st = np.random.SeedSequence(seed, spawn_key=(_S_XR, c, 2 + cohort)).generate_state(2, np.uint64)
            g.manual_seed(int(st[0] & np.uint64(0x7FFFFFFFFFFFFFFF)))
        lo = max(start, c * CHUNK)
        hi = min(start + cols, (c + 1) * CHUNK)
        u = torch.rand(CHUNK, n, generator=g, device=device, dtype=torch.float32)[lo - c * CHUNK:hi - c * CHUNK]
        fr = f[lo - c * CHUNK:hi - c * CHUNK].float()
        d = (u >= (1.0 - fr) ** 2).to(dtype) + (u >= 1.0 - fr * fr).to(dtype)
        out[lo - start:hi - start] = d
    return out


# --- Workloads -------------------------------------------------------------

WORKLOADS = {
    # plain FP64, every SNP checked against the oracle
    "n1000_p4": dict(n=1000, p=4, m=10_000, x_dtype="f64", host_block=10_000),
    # plain FP64, X_R streamed in 5,000-SNP host blocks
    "n20000_p4": dict(n=20_000, p=4, m=500_000, x_dtype="f64", host_block=5_000),
    # precision leg, int8 dosages
    "n50000_p8": dict(n=50_000, p=8, m=1_000_000, x_dtype="i8", host_block=50_000),
    # differentiation workload
    "n10000_p4": dict(n=10_000, p=4, m=100_000, x_dtype="f64", host_block=10_000),
}

