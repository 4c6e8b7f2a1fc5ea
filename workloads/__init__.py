"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no part of the RSVD arithmetic: it only builds test
matrices A = U diag(s) V^T with Haar-distributed orthonormal factors and a
prescribed spectrum s, and describes the five workloads.

The paper's compression inputs are reshaped two-site tensors from TEBD and
TTN sweeps (Sec. III.A): square (chi d) x (chi d) matrices for the TEBD block
update, up to chi^2 x chi^2 for the TTN update, block-diagonal with a few
symmetry sectors, and singular values that decay like a power law near
criticality or exponentially away from it (Sec. IV, singular-value decay
discussion).  No such matrices ship with the paper, so they are replaced by
synthetic matrices with those shapes and spectra.

Seeds: matrix b of workload c uses seed 1000*c + b for A and 2000*c + b for
the Gaussian test matrix; cotangents use 3000*c + b.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def haar_frame(rng: np.random.Generator, m: int, r: int) -> np.ndarray:
    """m x r matrix with orthonormal columns, Haar distributed (thin QR of a
    Gaussian with the sign of diag(R) absorbed, Mezzadri 2007)."""
    g = rng.standard_normal((m, r))
    q, rr = np.linalg.qr(g)
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return q * d


def haar_unitary_frame(rng: np.random.Generator, m: int, r: int) -> np.ndarray:
    """m x r complex matrix with orthonormal columns, Haar distributed (thin QR
    of a circular complex Gaussian with the phases of diag(R) absorbed)."""
    g = (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))) / math.sqrt(2.0)
    q, rr = np.linalg.qr(g)
    d = np.diag(rr)
    d = np.where(d == 0, 1.0, d / np.where(d == 0, 1.0, np.abs(d)))
    return q * d


def make_complex_matrix(m: int, n: int, s: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(s) V^H with Haar unitary frames, complex128."""
    rng = np.random.default_rng(seed)
    U = haar_unitary_frame(rng, m, len(s))
    V = haar_unitary_frame(rng, n, len(s))
    return (U * s) @ V.conj().T


def make_matrix(m: int, n: int, s: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(s) V^T, U (m x r), V (n x r), r = len(s) <= min(m, n), FP64."""
    rng = np.random.default_rng(seed)
    r = len(s)
    U = haar_frame(rng, m, r)
    V = haar_frame(rng, n, r)
    return (U * s) @ V.T


# --------------------------------------------------------------------------
# Spectra (1-based index i = 1..min(m, n), no normalisation: sigma_1 = s_1)
# --------------------------------------------------------------------------
def spectrum_exp(r: int, alpha: float) -> np.ndarray:
    i = np.arange(1, r + 1, dtype=np.float64)
    return np.exp(-alpha * i)


def spectrum_power(r: int, gamma: float) -> np.ndarray:
    i = np.arange(1, r + 1, dtype=np.float64)
    return i ** (-gamma)


def spectrum_noisy_power(r: int, gamma: float, rel_noise: float, seed: int) -> np.ndarray:
    """|i^-gamma (1 + rel_noise xi_i)| sorted descending (xi standard normal)."""
    rng = np.random.default_rng(seed)
    i = np.arange(1, r + 1, dtype=np.float64)
    s = np.abs(i ** (-gamma) * (1.0 + rel_noise * rng.standard_normal(r)))
    return np.sort(s)[::-1].copy()


def spectrum_power_with_pairs(r: int, gamma: float, pairs=(8, 40, 100),
                              rel_gap: float = 1e-6) -> np.ndarray:
    """i^-gamma with s_{i+1} := s_i (1 - rel_gap) at the 1-based positions in pairs."""
    s = spectrum_power(r, gamma)
    for i in pairs:
        if i < r:
            s[i] = s[i - 1] * (1.0 - rel_gap)
    return s


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class Problem:
    m: int
    n: int
    k: int
    p: int
    q: int
    seed: int          # Gaussian test-matrix seed
    a_seed: int        # test-matrix seed
    spectrum: np.ndarray
    delta: float = 0.0

    @property
    def l(self) -> int:
        kk = min(self.k, self.m, self.n)
        return min(kk + self.p, self.m, self.n)

    def matrix(self) -> np.ndarray:
        return make_matrix(self.m, self.n, self.spectrum, self.a_seed)

    def gemm_flops(self) -> float:
        """Algorithmic GEMM work of one factorisation: 2(q+1) passes over A in
        the range finder, one for B = Q^T A, i.e. 2 m n l (2q + 2), plus the
        back-projection 2 m l k."""
        l = self.l
        kk = min(self.k, self.m, self.n)
        return 2.0 * self.m * self.n * l * (2 * self.q + 2) + 2.0 * self.m * l * kk


@dataclass
class Workload:
    name: str
    description: str
    problems: list = field(default_factory=list)
    storage: str = "f64"          # storage dtype of A
    precisions: tuple = ("f64",)  # sketch/power precisions exercised


def _round_half_up(x: float) -> int:
    return int(math.floor(x + 0.5))


def c1() -> Workload:
    s = spectrum_exp(128, 0.08)
    return Workload("C1", "one FP64 128x128, s_i = exp(-0.08 i), k=64 p=10 q=2",
                    [Problem(128, 128, 64, 10, 2, 2001, 1001, s)], "f64", ("f64",))


def c2(batch: int = 32) -> Workload:
    s = spectrum_power(512, 1.5)
    probs = [Problem(512, 512, 256, 16, 2, 2000 * 2 + b, 1000 * 2 + b, s)
             for b in range(batch)]
    return Workload("C2", f"{batch} x 512x512, s_i = i^-1.5, k=256 p=16 q=2", probs,
                    "f64", ("f64", "f32"))


def c3(batch: int = 16) -> Workload:
    probs = [Problem(1024, 1024, 64, 16, 3, 2000 * 3 + b, 1000 * 3 + b,
                     spectrum_noisy_power(1024, 1.2, 0.05, 5000 * 3 + b))
             for b in range(batch)]
    return Workload("C3", f"{batch} x 1024x1024, s_i = |i^-1.2 (1+0.05 xi)|, k=64 p=16 q=3",
                    probs, "f32", ("bf16",))


def c4_sizes(count: int = 512):
    rng = np.random.default_rng(4)
    m = rng.integers(32, 2048, size=count, endpoint=True)
    n = rng.integers(32, 2048, size=count, endpoint=True)
    alpha = rng.uniform(0.005, 0.1, size=count)
    return m, n, alpha


def c4(count: int = 512) -> Workload:
    m, n, alpha = c4_sizes(512)
    probs = []
    for b in range(count):
        mm, nn = int(m[b]), int(n[b])
        r = min(mm, nn)
        k = max(8, 8 * _round_half_up(r / 32.0))
        probs.append(Problem(mm, nn, k, 16, 2, 2000 * 4 + b, 1000 * 4 + b,
                             spectrum_exp(r, float(alpha[b])), delta=1e-10))
    return Workload("C4", f"{count} uneven m,n in [32,2048], s_i = exp(-alpha i), "
                    "k = min(m,n)/4 rounded to 8, p=16 q=2, delta=1e-10", probs,
                    "f32", ("f32",))


def c5(batch: int = 64) -> Workload:
    s = spectrum_power_with_pairs(1024, 1.5)
    probs = [Problem(1024, 1024, 128, 16, 2, 2000 * 5 + b, 1000 * 5 + b, s)
             for b in range(batch)]
    return Workload("C5", f"{batch} x 1024x1024, s_i = i^-1.5 with 3 pairs (gap 1e-6), "
                    "k=128 p=16 q=2", probs, "f32", ("f32",))


def tebd_product(batch: int = 64, chi: int = 100, K: int = 2, d: int = 5) -> Workload:
    """TEBD product update (Sec. III): a (chi K) x (chi d) matrix compressed to
    rank chi (ratio 1/min(K, d)); power-law spectrum s_i = i^-2."""
    m, n = chi * K, chi * d
    s = spectrum_power(min(m, n), 2.0)
    probs = [Problem(m, n, chi, 10, 2, 2000 * 6 + b, 1000 * 6 + b, s) for b in range(batch)]
    return Workload("TEBD-P", f"{batch} x {m}x{n} (chi={chi}, K={K}, d={d}), s_i = i^-2, k={chi} p=10 q=2",
                    probs, "f64", ("f64",))


def tebd_block(batch: int = 32, chi: int = 100, d: int = 5) -> Workload:
    """TEBD block update (Sec. III): a (chi d) x (chi d) matrix compressed to
    rank chi (ratio 1/d); power-law spectrum s_i = i^-2."""
    m = chi * d
    s = spectrum_power(m, 2.0)
    probs = [Problem(m, m, chi, 10, 2, 2000 * 7 + b, 1000 * 7 + b, s) for b in range(batch)]
    return Workload("TEBD-B", f"{batch} x {m}x{m} (chi={chi}, d={d}), s_i = i^-2, k={chi} p=10 q=2",
                    probs, "f64", ("f64",))


def c4_matrix_device(m: int, n: int, s: np.ndarray, seed: int, torch, device="cuda"):
    """Seeded m x n FP32 matrix with exact singular values s, built on the
    device (the Haar construction of the 512 uneven matrices up to 2048^2
    would take minutes on the host): diag(s) mixed by three Householder
    reflections on each side, in FP64, then rounded to FP32.  torch is the
    caller's torch module (this module does not import it)."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    A = torch.zeros((m, n), dtype=torch.float64, device=device)
    r = len(s)
    A[torch.arange(r), torch.arange(r)] = torch.from_numpy(np.ascontiguousarray(s)).to(device)
    for _ in range(3):
        u = torch.randn(m, generator=g, dtype=torch.float64, device=device)
        u /= u.norm()
        A -= 2.0 * torch.outer(u, u @ A)
        v = torch.randn(n, generator=g, dtype=torch.float64, device=device)
        v /= v.norm()
        A -= 2.0 * torch.outer(A @ v, v)
    return A.float().contiguous()


def cotangents(m: int, n: int, k: int, seed: int):
    """Seeded Gaussian cotangents (dU m x k, dS k, dVT k x n) for the adjoint."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((m, k)), rng.standard_normal(k),
            rng.standard_normal((k, n)))
