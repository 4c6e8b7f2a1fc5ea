"""Complex-valued oracle: Alg. RSVD (Sec. II.B) and the full-SVD truncation
(Alg. TSVD, Sec. II.A) for complex matrices, as the paper's simulations use
complex double arithmetic (Sec. IV).  Plain numpy complex128, one problem at
a time, written for reading, not speed.

TEST INFRASTRUCTURE ONLY: imported by tests/.  The GPU library never imports
this module.

Conventions, as in the real oracle with Hermitian transposes:
- A is m x n; k is clamped to min(m, n); l = min(k + p, m, n).
- The Gaussian test matrix is circular: Omega(i, j) = (r cos t + i r sin t) / sqrt(2)
  from the Box-Muller pair of the Philox4x32-10 words of counter (i, j, 1, 0)
  under key (seed mod 2^32, seed >> 32); u1 = 1 - (w0:w1 >> 11) 2^-53 and
  u2 = (w2:w3 >> 11) 2^-53, r = sqrt(-2 ln u1), t = 2 pi u2.  The third
  counter word keeps these draws apart from the real generator's, whose
  counters have third word 0.
- Orthonormal factors come from Householder QR with diag(R) real and >= 0.
- The small SVD is one-sided Jacobi on the columns of G = B^H; a column pair
  is first brought to a real inner product by a unit phase, then rotated as in
  the real method, so B = J Sigma Vt with J the accumulated unitary.
- Outputs: S descending, VT = V^H; the largest-modulus entry of each column of
  U (lowest index on ties) is made real and positive, the matching row of VT
  taking the conjugate phase.
- w is ||A||_F^2 minus the kept sum of sigma^2 (compensated sums); with
  delta > 0, k_kept is the smallest k' with w(k') <= delta ||A||_F^2, at most k.
"""
import math

import numpy as np

from . import philox4x32_10

OK, ERR_NONFINITE, ERR_NOCONV = 0, -4, -5


def _uniforms(words):
    w0, w1, w2, w3 = (int(x) for x in words)
    u1 = 1.0 - (((w0 << 32) | w1) >> 11) * 2.0 ** -53
    u2 = (((w2 << 32) | w3) >> 11) * 2.0 ** -53
    return u1, u2


def cgaussian(seed, n, l):
    """n x l circular complex Gaussian test matrix (E|w|^2 = 1)."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    om = np.empty((n, l), dtype=np.complex128)
    for i in range(n):
        for j in range(l):
            u1, u2 = _uniforms(philox4x32_10((i, j, 1, 0), key))
            r = math.sqrt(-2.0 * math.log(u1))
            t = 2.0 * math.pi * u2
            om[i, j] = complex(r * math.cos(t), r * math.sin(t)) / math.sqrt(2.0)
    return om


def chqr(Y):
    """Thin Householder QR of the m x l matrix Y (m >= l): Q (m x l) with
    orthonormal columns and R (l x l) upper triangular, diag(R) real >= 0."""
    Y = np.array(Y, dtype=np.complex128)
    m, l = Y.shape
    R = Y.copy()
    vs = []
    for j in range(l):
        x = R[j:, j].copy()
        nx = np.linalg.norm(x)
        if nx == 0.0:
            vs.append(None)
            continue
        ph = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        v = x.copy()
        v[0] += ph * nx  # reflect x onto -ph ||x|| e_1 (no cancellation)
        v /= np.linalg.norm(v)
        R[j:, j:] -= 2.0 * np.outer(v, v.conj() @ R[j:, j:])
        vs.append(v)
    Q = np.zeros((m, l), dtype=np.complex128)
    Q[:l, :l] = np.eye(l)
    for j in reversed(range(l)):
        if vs[j] is not None:
            v = vs[j]
            Q[j:, :] -= 2.0 * np.outer(v, v.conj() @ Q[j:, :])
    R = np.triu(R[:l, :])
    # unit phases so that diag(R) is real and non-negative
    d = np.array([R[i, i] / abs(R[i, i]) if R[i, i] != 0 else 1.0 for i in range(l)])
    return Q * d, d.conj()[:, None] * R


def cjacobi_cols(G, max_sweeps=60):
    """One-sided Jacobi on the columns of the r x c complex matrix G, cyclic by
    rows.  Returns (G J, J, status, sweeps) with J unitary and the columns of
    G J mutually orthogonal."""
    G = np.array(G, dtype=np.complex128)
    r, c = G.shape
    J = np.eye(c, dtype=np.complex128)
    tol = max(r, c) * 2.0 ** -53
    for sweep in range(1, max_sweeps + 1):
        rotated = False
        for i in range(c - 1):
            for j in range(i + 1, c):
                a = np.vdot(G[:, i], G[:, i]).real
                b = np.vdot(G[:, j], G[:, j]).real
                g = np.vdot(G[:, i], G[:, j])  # g_i^H g_j
                ag = abs(g)
                if ag <= tol * math.sqrt(a * b) or ag == 0.0:
                    continue
                rotated = True
                e = g / ag  # column j times conj(e) makes the inner product real
                zeta = (b - a) / (2.0 * ag)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                cs = 1.0 / math.sqrt(1.0 + t * t)
                sn = cs * t
                for M in (G, J):
                    x = M[:, i].copy()
                    y = M[:, j] * e.conjugate()
                    M[:, i] = cs * x - sn * y
                    M[:, j] = sn * x + cs * y
        if not rotated:
            return G, J, OK, sweep
    return G, J, ERR_NOCONV, max_sweeps


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def _neumaier(vals):
    s = 0.0
    comp = 0.0
    for v in vals:
        t = s + v
        comp += (s - t) + v if abs(s) >= abs(v) else (v - t) + s
        s = t
    return s + comp


def _finish(A, Ufull, sig, Vt_full, k, delta, tail_direct):
    """Sort, truncation rule, discarded weight and canonical phases."""
    m, n = A.shape
    order = sorted(range(len(sig)), key=lambda j: -sig[j])  # stable: ties keep index order
    sig = np.array([sig[j] for j in order])
    Ufull = Ufull[:, order]
    Vt_full = Vt_full[order, :]
    a2 = _neumaier((np.abs(A) ** 2).ravel())

    def weight(kp):
        if tail_direct:
            return max(0.0, _neumaier(sig[kp:] ** 2))
        return max(0.0, a2 - _neumaier(sig[:kp] ** 2))

    kk = min(k, m, n)
    k_kept = kk
    if a2 == 0.0:
        k_kept = 0
    elif delta > 0.0:
        for kp in range(1, kk + 1):
            if weight(kp) <= delta * a2:
                k_kept = kp
                break
    w = weight(k_kept) if a2 > 0.0 else 0.0
    U = np.zeros((m, kk), dtype=np.complex128)
    S = np.zeros(kk)
    VT = np.zeros((kk, n), dtype=np.complex128)
    for j in range(k_kept):
        u = Ufull[:, j]
        big = int(np.argmax(np.abs(u)))  # first index of the largest modulus
        ph = u[big] / abs(u[big]) if u[big] != 0 else 1.0
        U[:, j] = u * np.conj(ph)
        VT[j, :] = Vt_full[j, :] * ph
        S[j] = sig[j]
    return U, S, VT, w, k_kept


def crsvd(A, k, p, q, seed, delta=0.0):
    """Alg. RSVD on a complex A: sketch, q power iterations with a QR after
    every product with A and with A^H, B = Q^H A, Jacobi SVD of B, U = Q U~."""
    A = np.array(A, dtype=np.complex128)
    m, n = A.shape
    if not np.all(np.isfinite(A)):
        return Result(status=ERR_NONFINITE)
    kk = min(k, m, n)
    l = min(kk + p, m, n)
    Q, _ = chqr(A @ cgaussian(seed, n, l))
    for _ in range(q):
        Z, _ = chqr(A.conj().T @ Q)
        Q, _ = chqr(A @ Z)
    B = Q.conj().T @ A  # l x n
    G, J, st, sweeps = cjacobi_cols(B.conj().T)  # G = B^H J = V~ Sigma
    sig = np.linalg.norm(G, axis=0)
    Vt = np.zeros((l, n), dtype=np.complex128)
    for j in range(l):
        if sig[j] > 0.0:
            Vt[j, :] = (G[:, j] / sig[j]).conj()
    U, S, VT, w, k_kept = _finish(A, Q @ J, sig, Vt, k, delta, tail_direct=False)
    return Result(U=U, S=S, VT=VT, w=w, k_kept=k_kept, status=st, sweeps=sweeps, l=l, Q=Q)


def cfullsvd(A, k, delta=0.0):
    """Alg. TSVD on a complex A: Jacobi on the columns of A^H (m <= n) or of A
    (m > n), then the same truncation with the tail sum as discarded weight."""
    A = np.array(A, dtype=np.complex128)
    m, n = A.shape
    if not np.all(np.isfinite(A)):
        return Result(status=ERR_NONFINITE)
    if m <= n:
        G, J, st, sweeps = cjacobi_cols(A.conj().T)  # A^H J = V Sigma, A = J Sigma V^H
        sig = np.linalg.norm(G, axis=0)
        Ufull = J
        Vt = np.array([(G[:, j] / sig[j]).conj() if sig[j] > 0 else np.zeros(n) for j in range(m)])
    else:
        G, J, st, sweeps = cjacobi_cols(A)  # A J = U Sigma, A = U Sigma J^H
        sig = np.linalg.norm(G, axis=0)
        Ufull = np.stack([G[:, j] / sig[j] if sig[j] > 0 else np.zeros(m) for j in range(n)], axis=1)
        Vt = J.conj().T
    U, S, VT, w, k_kept = _finish(A, Ufull, sig, Vt, k, delta, tail_direct=True)
    return Result(U=U, S=S, VT=VT, w=w, k_kept=k_kept, status=st, sweeps=sweeps)
