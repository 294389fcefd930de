"""Seeded synthetic inputs for the approximate product.

This module holds no arithmetic of the approximation method itself: it only
draws test matrices.  Both the oracle-side tests and the GPU path are fed from
here, so that the two sides see bit-identical operands.

Generators follow the paper's appendix on matrix generation (Haar-distributed
singular vectors, Alg. C.1): a Gaussian matrix is QR-factored and the columns
of Q are multiplied by the signs of diag(R) (a zero sign counts as +1), which
gives a Haar-distributed orthogonal factor.  The spectral-decay laws are the
ones named for the workloads: exp(-i/20) with i = 0..n-1 (the Type-1 style
index base of the appendix) and power laws i**-alpha with i = 1..n.

Seeds: numpy PCG64 with ``seed = 42 + 100*config + 10*operand + stream``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def seed_of(config: int, operand: int, stream: int = 0) -> int:
    return 42 + 100 * config + 10 * operand + stream


def rng_of(config: int, operand: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_of(config, operand, stream)))


# ---------------------------------------------------------------------------
# Haar factors (Alg. C.1)
# ---------------------------------------------------------------------------
def _sign_fixed_q(M, qr):
    Q, R = qr(M)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def haar_columns(rows: int, cols: int, rng: np.random.Generator, device=None):
    """rows x cols matrix with orthonormal, Haar-distributed columns (cols <= rows).

    The Gaussian draw and the QR run on the host in float64 (the sign fix
    makes Q unique); with ``device`` set (a torch device string) the factor is
    then copied there as a float64 tensor.  No device linear-algebra library
    runs in the generator, so profiled processes see only the library's own
    kernels and plain copies and products.
    """
    M = rng.standard_normal((rows, cols))
    Q = _sign_fixed_q(M, np.linalg.qr)
    if device is None:
        return Q
    import torch
    return torch.from_numpy(np.ascontiguousarray(Q)).to(device=device, dtype=torch.float64)


def spectral_matrix(m: int, n: int, sigma: np.ndarray, rng: np.random.Generator,
                    device=None):
    """Q1 diag(sigma) Q2^T with Haar Q1 (m x r), Q2 (n x r), r = len(sigma)."""
    r = len(sigma)
    Q1 = haar_columns(m, r, rng, device)
    Q2 = haar_columns(n, r, rng, device)
    if device is None:
        return (Q1 * sigma[None, :]) @ Q2.T
    import torch
    s = torch.from_numpy(np.asarray(sigma, dtype=np.float64)).to(Q1.device)
    return (Q1 * s.unsqueeze(0)) @ Q2.T


def decay_exp(n: int, scale: float = 20.0) -> np.ndarray:
    return np.exp(-np.arange(n, dtype=np.float64) / scale)


def decay_power(n: int, alpha: float) -> np.ndarray:
    return np.arange(1, n + 1, dtype=np.float64) ** (-alpha)


# ---------------------------------------------------------------------------
# Structured classes used for the circulant path
# ---------------------------------------------------------------------------
def toeplitz_uniform(n: int, rng: np.random.Generator) -> np.ndarray:
    """Toeplitz matrix from 2n-1 U(0,1) values: T[i,j] = v[i-j+n-1]."""
    v = rng.random(2 * n - 1)
    i = np.arange(n)
    return v[(i[:, None] - i[None, :]) + n - 1]


def planted_circulant(n: int, modes, rng: np.random.Generator, noise: float = 0.0,
                      device=None, profiles=None):
    """A = sum_k R_k D^k over the given frequency set with random real data.

    Built entrywise in the spatial domain, with no FFT: for each mode k a
    random complex cycle profile c_k is drawn and A[p,q] += Re(c_k[(p-q)%n] w^{kq})
    for the class {k, n-k} together, so A is real and its circulant content
    sits on the planted classes only.  ``noise`` adds i.i.d. N(0, noise^2).
    With ``device`` the same draws are combined by torch on that device
    (float64); ``profiles`` (a list) receives the drawn c_k.
    """
    cs = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for _ in modes]
    if profiles is not None:
        profiles.extend(cs)
    if device is None:
        A = np.zeros((n, n))
        p = np.arange(n)[:, None]
        q = np.arange(n)[None, :]
        for k, c in zip(modes, cs):
            term = c[(p - q) % n] * np.exp(2j * np.pi * k * q / n)
            A += term.real
        if noise:
            A += noise * rng.standard_normal((n, n))
        return A
    import torch
    idx = torch.arange(n, device=device)
    diff = (idx[:, None] - idx[None, :]) % n
    A = torch.zeros((n, n), dtype=torch.float64, device=device)
    for k, c in zip(modes, cs):
        ct = torch.from_numpy(c).to(device)
        ph = torch.exp(2j * np.pi * ((k * idx) % n).to(torch.float64) / n)
        A += (ct[diff] * ph[None, :]).real
    del diff
    if noise:
        A += noise * torch.from_numpy(rng.standard_normal((n, n))).to(device)
    return A


def real_circulant_lists(n: int, S, rng: np.random.Generator) -> np.ndarray:
    """Random eigenvalue lists (len(S) x n, complex) of a real truncated
    circulant decomposition on the closed frequency set S: the member n-k of
    a pair gets L_{n-k}[p] = conj(L_k[-p]); the self-paired 0 and n/2 are
    made to satisfy it themselves."""
    S = [int(k) for k in S]
    pos = {k: t for t, k in enumerate(S)}
    L = np.zeros((len(S), n), dtype=np.complex128)
    neg = (-np.arange(n)) % n
    done = set()
    for k in S:
        if k in done:
            continue
        kk = (n - k) % n
        if kk not in pos:
            raise ValueError("frequency set is not closed under k -> n-k")
        v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        if kk == k:
            v = 0.5 * (v + np.conj(v[neg]))
            L[pos[k]] = v
        else:
            L[pos[k]] = v
            L[pos[kk]] = np.conj(v[neg])
        done.update((k, kk))
    return L


def sparse_overlay(m: int, n: int, frac: float, scale: float,
                   rng: np.random.Generator):
    """round(frac*m*n) distinct uniform positions with Laplace(0, scale) values.

    Returns (flat_positions, values); positions are sorted ascending.
    """
    nnz = int(round(frac * m * n))
    pos = np.sort(rng.choice(m * n, size=nnz, replace=False))
    vals = rng.laplace(0.0, scale, size=nnz)
    return pos, vals


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
@dataclass
class Pair:
    A: np.ndarray
    B: np.ndarray
    name: str


def workload_exp_decay(n: int = 256) -> Pair:
    """n=256 square float64, sigma_i = exp(-i/20), plus 1e-3 N(0,1) noise."""
    out = []
    for operand in (0, 1):
        rng = rng_of(1, operand)
        M = spectral_matrix(n, n, decay_exp(n), rng)
        M = M + 1e-3 * rng.standard_normal((n, n))
        out.append(M)
    return Pair(out[0], out[1], f"haar-exp20-noise n={n}")


def workload_power_decay(n: int = 4096, device=None, with_sparse: bool = False,
                frac: float = 0.01, lap_scale: float = 10.0) -> Pair:
    """Square Haar operands with sigma_i = i^-1.5; optional 1% Laplace overlay."""
    out = []
    for operand in (0, 1):
        rng = rng_of(2, operand)
        M = spectral_matrix(n, n, decay_power(n, 1.5), rng, device)
        if with_sparse:
            pos, vals = sparse_overlay(n, n, frac, lap_scale, rng_of(2, operand, 1))
            if device is None:
                M = M.copy()
                M.reshape(-1)[pos] += vals
            else:
                import torch
                flat = M.reshape(-1)
                flat[torch.from_numpy(pos).to(M.device)] += torch.from_numpy(vals).to(M.device)
        out.append(M)
    tag = "haar-pow1.5" + (f"+sparse{frac:g}" if with_sparse else "")
    return Pair(out[0], out[1], f"{tag} n={n}")


def workload_lowrank_sparse(n: int = 16384, rank: int = 1024, frac: float = 0.005, lap_scale: float = 20.0,
                device=None) -> Pair:
    """Square operands S + R: R = Q1 diag(i^-1.5, i = 1..rank) Q2^T with thin
    Haar factors (the energy beyond rank 1024 of the full law is ~4e-7 of the
    total), S = round(frac n^2) Laplace(0, lap_scale) entries at uniform
    positions."""
    out = []
    for operand in (0, 1):
        rng = rng_of(5, operand)
        M = spectral_matrix(n, n, decay_power(rank, 1.5), rng, device)
        pos, vals = sparse_overlay(n, n, frac, lap_scale, rng_of(5, operand, 1))
        if device is None:
            M = M.copy()
            M.reshape(-1)[pos] += vals
        else:
            import torch
            flat = M.reshape(-1)
            flat[torch.from_numpy(pos).to(M.device)] += torch.from_numpy(vals).to(M.device)
        out.append(M)
    return Pair(out[0], out[1], f"haar-pow1.5-r{rank}+sparse{frac:g}-laplace{lap_scale:g} n={n}")


def sinusoid_rows(m: int, n: int, rng: np.random.Generator, modes: int = 11, noise: float = 0.05) -> np.ndarray:
    """Rows that are sums of `modes` cosines (frequency f = 1..modes with
    N(0,1)/f amplitudes and random phases) plus N(0, noise^2): a few dominant
    frequencies per row, the structure Fourier-domain sparsification keeps."""
    t = np.arange(n)
    A = noise * rng.standard_normal((m, n))
    for f in range(1, modes + 1):
        amp = rng.standard_normal((m, 1)) / f
        A += amp * np.cos(2 * np.pi * f * t[None, :] / n + rng.random((m, 1)) * 6)
    return A


# ---------------------------------------------------------------------------
# Synthetic classes of the paper's result tables (App. "randomly generated
# matrices with a given distribution of singular values", Sec. 4.1)
# ---------------------------------------------------------------------------
def type1_matrix(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar Q1 diag(exp(-i/10)) Q2^T, i = 0..n-1."""
    return spectral_matrix(n, n, decay_exp(n, 10.0), rng)


def type3_matrix(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar Q1 diag((n - i)/n) Q2^T, i = 0..n-1 (linear decay)."""
    return spectral_matrix(n, n, (n - np.arange(n, dtype=np.float64)) / n, rng)


def type2_matrix(n: int, rng: np.random.Generator) -> np.ndarray:
    """A Type-1 matrix T plus full-rank noise 0.5 ||T||_F / ||U||_F U, U ~ U(0,1)."""
    T = type1_matrix(n, rng)
    U = rng.random((n, n))
    return T + (0.5 * np.linalg.norm(T) / np.linalg.norm(U)) * U


def general_uniform(n: int, rng: np.random.Generator) -> np.ndarray:
    """'General' matrix of the result figures: i.i.d. U(0,1) entries."""
    return rng.random((n, n))


def symmetric_uniform(n: int, rng: np.random.Generator) -> np.ndarray:
    """Random symmetric matrix (U + U^T) / 2, U with i.i.d. U(0,1) entries."""
    U = rng.random((n, n))
    return 0.5 * (U + U.T)


def hankel_uniform(n: int, rng: np.random.Generator) -> np.ndarray:
    """Hankel matrix from 2n-1 U(0,1) values: H[i,j] = v[i+j]."""
    v = rng.random(2 * n - 1)
    i = np.arange(n)
    return v[i[:, None] + i[None, :]]


def kappa_matrix(n: int) -> np.ndarray:
    """Symmetric sign-oscillating matrix exp(-|i - j|/2) sin(i + 1), the sine
    taken at the larger of the two indices (the lower triangle's row)."""
    i = np.arange(n)
    big = np.maximum(i[:, None], i[None, :])
    return np.exp(-0.5 * np.abs(i[:, None] - i[None, :])) * np.sin(big + 1.0)


def workload_toeplitz(n: int) -> Pair:
    A = toeplitz_uniform(n, rng_of(9, 0))
    B = toeplitz_uniform(n, rng_of(9, 1))
    return Pair(A, B, f"toeplitz-U01 n={n}")


def gaussian(rows: int, cols: int, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal((rows, cols))


def log2_int(n: int) -> int:
    k = int(round(math.log2(n)))
    if 1 << k != n:
        raise ValueError(f"{n} is not a power of two")
    return k
