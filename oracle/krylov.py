"""Block-Krylov variant of the randomized SVD, named in the paper's outlook
(Sec. V) as a modified power scheme with faster convergence (Musco and
Musco 2015): instead of keeping only the last power-iteration basis, the
small SVD is taken over the whole block Krylov space
span{A Omega, (A A^T) A Omega, ..., (A A^T)^q A Omega}.

TEST INFRASTRUCTURE ONLY: imported by tests/.  The GPU library never imports
this module.

Steps (FP64, the same Omega, QR and Jacobi as the oracle's Alg. RSVD):
1. Omega = the n x l Gaussian of the seed, l = min(k + p, m, n);
2. Q_0 = orth(A Omega); for j = 1..q: Z = orth(A^T Q_{j-1}), Q_j = orth(A Z),
   so that span Q_j = span (A A^T)^j A Omega;
3. K = [Q_0, Q_1, ..., Q_q], its first L = min(l (q + 1), m, n) columns, and
   Q = orth(K) (m x L);
4. B = Q^T A, one-sided Jacobi on the columns of B^T, U = Q U~;
5. the truncation rule and discarded weight of the RSVD (w = ||A||_F^2 minus
   the kept sum of sigma^2, compensated), canonical signs.
With q = 0 this is the RSVD itself.
"""
import numpy as np

from . import gaussian, hqr, jacobi_cols


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def _ksum(vals):
    s = 0.0
    c = 0.0
    for v in vals:
        t = s + v
        c += (s - t) + v if abs(s) >= abs(v) else (v - t) + s
        s = t
    return s + c


def block_krylov_rsvd(A, k, p, q, seed, delta=0.0):
    A = np.array(A, dtype=np.float64)
    m, n = A.shape
    kk = min(k, m, n)
    l = min(kk + p, m, n)
    Qj, _ = hqr(A @ gaussian(seed, n, l))
    blocks = [Qj]
    for _ in range(q):
        Z, _ = hqr(A.T @ Qj)
        Qj, _ = hqr(A @ Z)
        blocks.append(Qj)
    L = min(l * (q + 1), m, n)
    Q, _ = hqr(np.concatenate(blocks, axis=1)[:, :L])
    B = Q.T @ A
    G, J, status, sweeps = jacobi_cols(B.T)  # B^T J = V~ Sigma, so B = J Sigma V~^T
    sig = np.linalg.norm(G, axis=0)
    order = sorted(range(L), key=lambda j: -sig[j])
    sig = sig[order]
    Ufull = (Q @ J)[:, order]
    Vt = np.array([G[:, j] / s if s > 0 else np.zeros(n) for j, s in zip(order, sig)])
    a2 = _ksum((A * A).ravel())
    k_kept = kk
    if a2 == 0.0:
        k_kept = 0
    elif delta > 0.0:
        for kp in range(1, kk + 1):
            if max(0.0, a2 - _ksum(sig[:kp] ** 2)) <= delta * a2:
                k_kept = kp
                break
    w = max(0.0, a2 - _ksum(sig[:k_kept] ** 2)) if a2 > 0.0 else 0.0
    U = np.zeros((m, kk))
    S = np.zeros(kk)
    VT = np.zeros((kk, n))
    for j in range(k_kept):
        u = Ufull[:, j]
        sgn = 1.0 if u[int(np.argmax(np.abs(u)))] >= 0 else -1.0  # first index of the largest |u|
        U[:, j] = sgn * u
        VT[j] = sgn * Vt[j]
        S[j] = sig[j]
    return Result(U=U, S=S, VT=VT, w=w, k_kept=k_kept, status=status, sweeps=sweeps, L=L)
