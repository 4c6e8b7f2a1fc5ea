"""Single-view variant of the randomized SVD, named in the paper's outlook
(Sec. V; Tropp, Yurtsever, Udell and Cevher): A is read once, by two
sketches taken together, and never revisited.

TEST INFRASTRUCTURE ONLY: imported by tests/.  The GPU library never imports
this module.

Steps (FP64, the oracle's Gaussian, QR and Jacobi):
1. range test matrix Omega = the n x l Gaussian of the seed, l = min(k + p, m, n);
   co-range test matrix Psi (s x m), s = min(2 l + 1, m), the transposed m x s
   Gaussian of the seed with its top bit flipped (a different Philox key, so
   Psi and Omega are independent);
2. the one pass over A: Y = A Omega (m x l) and W = Psi A (s x n);
3. Q = orth(Y);
4. X = (Psi Q)^+ W, by a QR of Psi Q (s x l) and a triangular solve, so that
   Q X approximates A without touching A again;
5. one-sided Jacobi on the columns of X^T, U = Q U~, sort, canonical signs;
6. the discarded weight is the true squared error ||A - U S V^T||_F^2 of the
   kept triplets (Q X is not a projection of A, so the RSVD identity
   ||A||^2 - sum sigma^2 does not hold here); with delta > 0, k_kept is the
   smallest k' whose error is at most delta ||A||_F^2, at most k.
"""
import numpy as np

from . import gaussian, hqr, jacobi_cols


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def single_view_rsvd(A, k, p, seed, delta=0.0):
    A = np.array(A, dtype=np.float64)
    m, n = A.shape
    kk = min(k, m, n)
    l = min(kk + p, m, n)
    s = min(2 * l + 1, m)
    Omega = gaussian(seed, n, l)
    Psi = gaussian(seed ^ (1 << 63), m, s).T
    Y = A @ Omega
    W = Psi @ A
    Q, _ = hqr(Y)
    Q2, R2 = hqr(Psi @ Q)
    X = np.linalg.solve(R2, Q2.T @ W)  # R2 is l x l upper triangular
    G, J, status, sweeps = jacobi_cols(X.T)  # X^T J = V~ Sigma, X = J Sigma V~^T
    sig = np.linalg.norm(G, axis=0)
    order = sorted(range(l), key=lambda j: -sig[j])
    sig = sig[order]
    Ufull = (Q @ J)[:, order]
    Vt = np.array([G[:, j] / v if v > 0 else np.zeros(n) for j, v in zip(order, sig)])
    for j in range(l):  # canonical signs: the largest |u_j| entry (first on ties) positive
        if Ufull[int(np.argmax(np.abs(Ufull[:, j]))), j] < 0:
            Ufull[:, j] *= -1.0
            Vt[j] *= -1.0

    def err(kp):
        return float(np.sum((A - (Ufull[:, :kp] * sig[:kp]) @ Vt[:kp]) ** 2))

    a2 = float(np.sum(A * A))
    k_kept = kk
    if a2 == 0.0:
        k_kept = 0
    elif delta > 0.0:
        for kp in range(1, kk + 1):
            if err(kp) <= delta * a2:
                k_kept = kp
                break
    U = np.zeros((m, kk))
    S = np.zeros(kk)
    VT = np.zeros((kk, n))
    U[:, :k_kept] = Ufull[:, :k_kept]
    S[:k_kept] = sig[:k_kept]
    VT[:k_kept] = Vt[:k_kept]
    return Result(U=U, S=S, VT=VT, w=err(k_kept) if a2 > 0.0 else 0.0, k_kept=k_kept, status=status,
                  sweeps=sweeps, Q=Q, QX=Q @ X, l=l, s=s, Omega=Omega, Psi=Psi)
