"""Python API over librsvd.  PyTorch provides device memory and streams only;
every step of the factorisation runs in the library's HIP kernels.

Alg. RSVD and Alg. TSVD refer to Sec. II.B and Sec. II.A of Kohn et al.,
"Probabilistic low-rank factorization accelerates tensor network simulations
of critical quantum many-body ground states".
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_DT = {torch.float64: L.RSVD_F64, torch.float32: L.RSVD_F32, torch.complex128: L.RSVD_F64}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_matrix(A):
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise ValueError("A must be a 2-D torch tensor")
    if A.device.type != "cuda":
        raise ValueError("A must be on a GPU device")
    if A.dtype not in (torch.float64, torch.float32):
        raise ValueError("A must be float64 or float32 (complex matrices go through a Plan)")
    if A.stride(1) != 1:
        A = A.contiguous()
    return A


def _outputs(m, n, k, dtype, device):
    kk = min(k, m, n)
    U = torch.empty((m, kk), dtype=dtype, device=device)
    S = torch.empty((kk,), dtype=torch.float64 if dtype == torch.complex128 else dtype, device=device)
    VT = torch.empty((kk, n), dtype=dtype, device=device)
    return U, S, VT


def rsvd_truncate(A, k, p=10, q=2, seed=0, delta=0.0, prec="f64"):
    """Rank-k randomized truncated SVD (Alg. RSVD).  Returns (U, S, VT, w, k_kept)
    with w the discarded squared Frobenius weight (FP64 tensor of shape [1]) and
    k_kept an int64 tensor of shape [1]; U/S/VT beyond k_kept are zero."""
    A = _check_matrix(A)
    m, n = A.shape
    U, S, VT = _outputs(m, n, k, A.dtype, A.device)
    w = torch.empty(1, dtype=torch.float64, device=A.device)
    kk = torch.empty(1, dtype=torch.int64, device=A.device)
    L.check(L.lib().rsvd_truncate(A.data_ptr(), _DT[A.dtype], m, n, A.stride(0), k, p, q,
                                  ctypes.c_uint64(seed), float(delta), L.PREC[prec], U.data_ptr(),
                                  U.shape[1], S.data_ptr(), VT.data_ptr(), n, w.data_ptr(),
                                  kk.data_ptr(), _stream()))
    return U, S, VT, w, kk


def rsvd_truncate_noalloc(A, k, p=10, q=2, seed=0, delta=0.0, prec="f64", out=None):
    """rsvd_truncate without device allocation inside the library
    (rsvd_truncate_noalloc): the call runs asynchronously on the current
    stream in the library's static scratch array.  out: optional
    (U, S, VT, w, k_kept, info) tensors to write into (needed under graph
    capture, where this wrapper must not allocate either).  Returns
    (U, S, VT, w, k_kept, info) without synchronising; info (int32 [1])
    receives the factorisation's status."""
    A = _check_matrix(A)
    m, n = A.shape
    if out is None:
        U, S, VT = _outputs(m, n, k, A.dtype, A.device)
        w = torch.empty(1, dtype=torch.float64, device=A.device)
        kk = torch.empty(1, dtype=torch.int64, device=A.device)
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    else:
        U, S, VT, w, kk, info = out
    L.check(L.lib().rsvd_truncate_noalloc(A.data_ptr(), _DT[A.dtype], m, n, A.stride(0), k, p, q,
                                          ctypes.c_uint64(seed), float(delta), L.PREC[prec], U.data_ptr(),
                                          U.stride(0), S.data_ptr(), VT.data_ptr(), VT.stride(0), w.data_ptr(),
                                          kk.data_ptr(), info.data_ptr(), _stream()))
    return U, S, VT, w, kk, info


def rsvd_truncate_adaptive(A, k0, k_max, delta, p=10, q=2, seed=0, prec="f64"):
    """Fixed-error truncation (rsvd_truncate_adaptive): rank k0, 2 k0, ... up to
    k_max until the delta cut binds.  Returns (U, S, VT, w, k_kept, attempts)
    with outputs sized for min(k_max, m, n)."""
    A = _check_matrix(A)
    m, n = A.shape
    U, S, VT = _outputs(m, n, k_max, A.dtype, A.device)
    w = torch.empty(1, dtype=torch.float64, device=A.device)
    kk = torch.empty(1, dtype=torch.int64, device=A.device)
    att = ctypes.c_int(0)
    L.check(L.lib().rsvd_truncate_adaptive(A.data_ptr(), _DT[A.dtype], m, n, A.stride(0), k0, k_max, p, q,
                                           ctypes.c_uint64(seed), float(delta), L.PREC[prec], U.data_ptr(),
                                           U.shape[1], S.data_ptr(), VT.data_ptr(), n, w.data_ptr(),
                                           kk.data_ptr(), ctypes.byref(att), _stream()))
    return U, S, VT, w, kk, att.value


def fullsvd_truncate(A, k, delta=0.0):
    """Truncation by the full SVD (Alg. TSVD), block one-sided Jacobi in FP64."""
    A = _check_matrix(A)
    m, n = A.shape
    U, S, VT = _outputs(m, n, k, A.dtype, A.device)
    w = torch.empty(1, dtype=torch.float64, device=A.device)
    kk = torch.empty(1, dtype=torch.int64, device=A.device)
    L.check(L.lib().fullsvd_truncate(A.data_ptr(), _DT[A.dtype], m, n, A.stride(0), k, float(delta),
                                     U.data_ptr(), U.shape[1], S.data_ptr(), VT.data_ptr(), n,
                                     w.data_ptr(), kk.data_ptr(), _stream()))
    return U, S, VT, w, kk


def gaussian(seed, n, l, device="cuda"):
    """The n x l Gaussian test matrix (FP64) the RSVD draws for this seed."""
    out = torch.empty((n, l), dtype=torch.float64, device=device)
    L.check(L.lib().rsvd_gaussian(ctypes.c_uint64(seed), n, l, out.data_ptr(), _stream()))
    return out


def philox4x32_10(words):
    """Device Philox4x32-10: words is a (count x 6) array of uint32 counter and
    key words; returns the (count x 4) output words as a numpy uint32 array."""
    import numpy as np
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint32)).view(np.int32)
    inp = torch.from_numpy(w).cuda()
    out = torch.empty((inp.shape[0], 4), dtype=torch.int32, device=inp.device)
    L.check(L.lib().rsvd_philox4x32_10(inp.data_ptr(), out.data_ptr(), inp.shape[0], _stream()))
    torch.cuda.current_stream().synchronize()
    return out.cpu().numpy().view(np.uint32)


class Plan:
    """A batch of independent truncations of arbitrary sizes run together.

    problems: list of dicts with keys m, n, k and (RSVD) p, q, seed, and
    optionally delta.  Outputs are allocated once by the plan and reused by
    every execute, so repeated executes on the same inputs upload nothing.
    dtype torch.complex128 makes a complex plan (RSVD_PLAN_COMPLEX): A, U, VT
    complex, S real.
    """

    def __init__(self, problems, dtype=torch.float64, prec="f64", fullsvd=False, graph=True,
                 save=False, refine=True, tune=False, round_launches=False, block_krylov=False, blocked_qr=False,
                 single_view=False, fp64_final=False, device="cuda"):
        self.dtype = dtype
        self.device = torch.device(device)
        self.fullsvd = fullsvd
        self.problems = [dict(pr) for pr in problems]
        n = len(self.problems)
        arr = (L.RsvdProblem * n)()
        for i, pr in enumerate(self.problems):
            arr[i].m = pr["m"]
            arr[i].n = pr["n"]
            arr[i].lda = pr.get("lda", pr["n"])
            arr[i].k = pr["k"]
            arr[i].p = pr.get("p", 0)
            arr[i].q = pr.get("q", 0)
            arr[i].seed = pr.get("seed", 0)
            arr[i].delta_trunc = pr.get("delta", 0.0)
            arr[i].ldu = 0
            arr[i].ldvt = 0
        flags = (L.PLAN_FULLSVD if fullsvd else 0) | (L.PLAN_GRAPH if graph else 0) | \
                (L.PLAN_SAVE if save else 0) | (0 if refine else L.PLAN_NO_REFINE) | \
                (L.PLAN_TUNE if tune else 0) | (L.PLAN_ROUND_LAUNCHES if round_launches else 0) | \
                (L.PLAN_BLOCK_KRYLOV if block_krylov else 0) | (L.PLAN_BLOCKED_QR if blocked_qr else 0) | \
                (L.PLAN_SINGLE_VIEW if single_view else 0) | (L.PLAN_FP64_FINAL if fp64_final else 0) | \
                (L.PLAN_COMPLEX if dtype == torch.complex128 else 0)
        h = ctypes.c_void_p()
        L.check(L.lib().rsvd_plan_create(arr, n, _DT[dtype], L.PREC[prec], flags, ctypes.byref(h)))
        self._h = h
        self.outputs = [_outputs(pr["m"], pr["n"], pr["k"], dtype, self.device) for pr in self.problems]
        self.w = torch.empty(n, dtype=torch.float64, device=self.device)
        self.k_kept = torch.empty(n, dtype=torch.int64, device=self.device)
        self.info = torch.empty(n, dtype=torch.int32, device=self.device)
        self._ptrs = (L.ptr_array([o[0].data_ptr() for o in self.outputs]),
                      L.ptr_array([o[1].data_ptr() for o in self.outputs]),
                      L.ptr_array([o[2].data_ptr() for o in self.outputs]))
        self._keep = None

    def tiles(self):
        """(rows, cols) of the workgroup tile of each tunable forward product, in launch order."""
        count = ctypes.c_int64()
        L.check(L.lib().rsvd_plan_tiles(self._h, None, 0, ctypes.byref(count)))
        buf = (ctypes.c_int32 * max(2 * count.value, 1))()
        L.check(L.lib().rsvd_plan_tiles(self._h, buf, count.value, ctypes.byref(count)))
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(count.value)]

    def set_tiles(self, tiles):
        """Fixes the tile of each tunable forward product (a list as returned by tiles())."""
        buf = (ctypes.c_int32 * max(2 * len(tiles), 1))(*[v for t in tiles for v in t])
        L.check(L.lib().rsvd_plan_set_tiles(self._h, buf, len(tiles)))

    @property
    def workspace_bytes(self):
        return int(L.lib().rsvd_plan_workspace_bytes(self._h))

    def execute(self, As):
        """Runs every problem on the current stream; As: list of device tensors.
        Returns (outputs, w, k_kept, info) without synchronising."""
        if len(As) != len(self.problems):
            raise ValueError("one input matrix per problem")
        for A, pr in zip(As, self.problems):
            if A.shape != (pr["m"], pr["n"]) or A.dtype != self.dtype or A.device.type != "cuda":
                raise ValueError("input matrix does not match its problem")
            if A.stride(1) != 1 or A.stride(0) != pr.get("lda", pr["n"]):
                raise ValueError("input matrix must be row-major with the plan's lda")
        aptr = L.ptr_array([A.data_ptr() for A in As])
        self._keep = As
        L.check(L.lib().rsvd_plan_execute(self._h, aptr, self._ptrs[0], self._ptrs[1], self._ptrs[2],
                                          self.w.data_ptr(), self.k_kept.data_ptr(),
                                          self.info.data_ptr(), _stream()))
        return self.outputs, self.w, self.k_kept, self.info

    def profile(self, As):
        """One execute without the graph, with HIP events around every launch.
        Returns {phase: (ms, launches, algorithmic_flops)}.  Blocking."""
        for A, pr in zip(As, self.problems):
            if A.shape != (pr["m"], pr["n"]) or A.dtype != self.dtype:
                raise ValueError("input matrix does not match its problem")
        nc = len(L.PHASES)
        ms = (ctypes.c_double * nc)()
        nl = (ctypes.c_int64 * nc)()
        fl = (ctypes.c_double * nc)()
        aptr = L.ptr_array([A.data_ptr() for A in As])
        L.check(L.lib().rsvd_plan_profile(self._h, aptr, self._ptrs[0], self._ptrs[1], self._ptrs[2],
                                          self.w.data_ptr(), self.k_kept.data_ptr(), self.info.data_ptr(),
                                          ms, nl, fl, nc, _stream()))
        return {name: (ms[i], int(nl[i]), fl[i]) for i, name in enumerate(L.PHASES)}

    def postselect(self, chi):
        """Sector post-selection (rsvd_plan_postselect): keep the chi largest
        singular values over all problems of the last execute, in place.
        Returns chi_s, a device int64 tensor with the number kept per problem."""
        chi_s = torch.empty(len(self.problems), dtype=torch.int64, device=self.device)
        L.check(L.lib().rsvd_plan_postselect(self._h, int(chi), chi_s.data_ptr(), _stream()))
        return chi_s

    def _cotangent_ptrs(self, dU, dS, dVT, dA):
        n = len(self.problems)
        if not (len(dU) == len(dS) == len(dVT) == n):
            raise ValueError("one cotangent triple per problem")
        for i, pr in enumerate(self.problems):
            U, S, VT = self.outputs[i]
            for g, ref in ((dU[i], U), (dS[i], S), (dVT[i], VT)):
                if g.shape != ref.shape or g.dtype != self.dtype or g.device.type != "cuda" or \
                        not g.is_contiguous():
                    raise ValueError("cotangent does not match its output (shape, dtype, contiguity)")
        if dA is None:
            dA = [torch.empty((pr["m"], pr.get("lda", pr["n"])), dtype=self.dtype, device=self.device)
                  [:, :pr["n"]] for pr in self.problems]
        if len(dA) != n:
            raise ValueError("one gradient buffer per problem")
        for g, pr in zip(dA, self.problems):
            if g.shape != (pr["m"], pr["n"]) or g.dtype != self.dtype or g.device.type != "cuda" or \
                    g.stride(1) != 1 or g.stride(0) != pr.get("lda", pr["n"]):
                raise ValueError("dA must be row-major m x n with the plan's lda and dtype")
        keep = (dU, dS, dVT, dA)
        ptrs = tuple(L.ptr_array([t.data_ptr() for t in group]) for group in keep)
        return ptrs, keep, dA

    def backward(self, dU, dS, dVT, broadening=0.0, dA=None):
        """Gradient over every A of <dU, U> + <dS, S> + <dVT, VT> for the most
        recent execute (plan created with save=True).  Cotangents: lists of
        contiguous tensors shaped like the outputs.  Returns the list of dA
        (allocated unless given), without synchronising."""
        ptrs, keep, dA = self._cotangent_ptrs(dU, dS, dVT, dA)
        self._keep_bw = keep
        L.check(L.lib().rsvd_plan_backward(self._h, *ptrs, float(broadening), _stream()))
        return dA

    def profile_backward(self, dU, dS, dVT, broadening=0.0, dA=None):
        """The reverse pass without the graph, with HIP events around every
        launch.  Returns {phase: (ms, launches, algorithmic_flops)}.  Blocking."""
        ptrs, keep, dA = self._cotangent_ptrs(dU, dS, dVT, dA)
        nc = len(L.PHASES)
        ms = (ctypes.c_double * nc)()
        nl = (ctypes.c_int64 * nc)()
        fl = (ctypes.c_double * nc)()
        L.check(L.lib().rsvd_plan_profile_backward(self._h, *ptrs, float(broadening), ms, nl, fl, nc,
                                                   _stream()))
        return {name: (ms[i], int(nl[i]), fl[i]) for i, name in enumerate(L.PHASES)}

    def close(self):
        if getattr(self, "_h", None):
            L.lib().rsvd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RSVDFunction(torch.autograd.Function):
    """Differentiable batched RSVD: forward runs a saving plan over the given
    matrices, backward calls the library's hand-written adjoint with the
    Gaussian test matrices held fixed (they depend on the seeds only).

    apply(spec, *As) -> (U_0, S_0, VT_0, U_1, S_1, VT_1, ...), where spec is a
    dict with keys k, p, q, seeds (one per matrix), delta, prec, broadening.
    """

    @staticmethod
    def forward(ctx, spec, *As):
        As = [_check_matrix(A) for A in As]
        dtype = As[0].dtype
        seeds = spec["seeds"]
        probs = [dict(m=A.shape[0], n=A.shape[1], lda=A.stride(0), k=spec["k"], p=spec.get("p", 10),
                      q=spec.get("q", 2), seed=int(seeds[i]), delta=spec.get("delta", 0.0))
                 for i, A in enumerate(As)]
        plan = Plan(probs, dtype, spec.get("prec", "f64"), graph=False, save=True, device=As[0].device)
        plan.execute(As)
        ctx.plan = plan
        ctx.broadening = float(spec.get("broadening", 0.0))
        ctx.shapes = [(A.shape, A.stride(0)) for A in As]
        outs = []
        for U, S, VT in plan.outputs:  # owned by this call's plan, never overwritten
            outs += [U, S, VT]
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        plan = ctx.plan
        nb = len(plan.problems)
        dU, dS, dVT = [], [], []
        for i in range(nb):
            for lst, g, ref in ((dU, grads[3 * i], plan.outputs[i][0]), (dS, grads[3 * i + 1], plan.outputs[i][1]),
                                (dVT, grads[3 * i + 2], plan.outputs[i][2])):
                lst.append(torch.zeros_like(ref) if g is None else g.to(ref.dtype).contiguous())
        dA = [torch.empty((shape[0], ld), dtype=plan.dtype, device=plan.device)[:, :shape[1]]
              for shape, ld in ctx.shapes]
        plan.backward(dU, dS, dVT, ctx.broadening, dA=dA)
        ctx.plan = None
        return (None,) + tuple(dA)


def rsvd(A, k, p=10, q=2, seed=0, delta=0.0, prec="f64", broadening=0.0):
    """Differentiable rank-k RSVD of one matrix: returns (U, S, VT)."""
    return RSVDFunction.apply(dict(k=k, p=p, q=q, seeds=[seed], delta=delta, prec=prec,
                                   broadening=broadening), A)


def rsvd_batch(As, k, p=10, q=2, seeds=None, delta=0.0, prec="f64", broadening=0.0):
    """Differentiable RSVD of a list of matrices (uniform k, p, q) in one plan:
    returns a list of (U, S, VT) triples."""
    seeds = list(range(len(As))) if seeds is None else list(seeds)
    out = RSVDFunction.apply(dict(k=k, p=p, q=q, seeds=seeds, delta=delta, prec=prec,
                                  broadening=broadening), *As)
    return [tuple(out[3 * i:3 * i + 3]) for i in range(len(As))]
