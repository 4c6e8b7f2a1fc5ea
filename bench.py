"""Benchmark: rank-k RSVDs per second on one MI355X.

Workload (the headline line): the TEBD-shaped critical-spectrum batch, 32
matrices 512 x 512 with s_i = i^-1.5 and Haar factors, k = 256, p = 16,
q = 2, FP64, solved as one batched plan (one HIP-graph launch per step).
Inputs are resident in HBM before timing starts.  A step is one RSVD of
every matrix of the batch.

Also reported, each in its own field: the same-GPU full-SVD truncation
(block one-sided Jacobi) and the plain FP64 one-at-a-time RSVD on the same
batch at their truncation errors, the power-step count that brings the RSVD
to within 1% of the optimal truncation error, the batch in FP32, the single
128 x 128 factorisation (latency), the 512-problem uneven batch, the TEBD
shapes, sector post-selection, the adaptive rank, the differentiation
workload (64 FP32 matrices 1024 x 1024, forward + adjoint), the
mixed-precision workload (16 x 1024^2) with singular-value and projector
errors against the FP64 CPU oracle, copy bandwidths (HBM and the last-level
cache), and the CPU FP64 oracle on the whole headline batch.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f64|f32|bf16]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the full-SVD and one-at-a-time legs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the post-selection, adaptive-rank, equal-error, FP32, C1, C4 and bandwidth legs "
                         "(only the C2 plan runs)")
    ap.add_argument("--c1-reps", type=int, default=300)
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the shape heuristic's GEMM tiles instead of tuning them on the first execute")
    ap.add_argument("--no-diff", action="store_true", help="skip the forward + adjoint leg")
    ap.add_argument("--diff-batch", type=int, default=64)
    ap.add_argument("--diff-steps", type=int, default=5)
    ap.add_argument("--only", choices=["c4"], default=None,
                    help="run one leg alone and print its JSON (for profiling that leg's kernels)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


# Algorithmic work of the small SVD of one headline-batch matrix (B = Q^T A,
# 272 x 512, one-sided Jacobi, about 8 sweeps), FLOPs.
SMALL_SVD_FLOPS_C2 = 1.77e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(mats, probs, sample):
    """The FP64 oracle (untuned), one problem per thread over the host cores
    this process may run on, on the first `sample` matrices of the batch."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    idx = list(range(min(sample, len(mats))))
    threads = max(1, min(cores, len(idx)))
    oracle.lib()

    def one(i):
        pr = probs[i]
        return oracle.rsvd(mats[i], pr.k, pr.p, pr.q, pr.seed).status

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        st = list(ex.map(one, idx))
    dt = time.perf_counter() - t0
    assert all(s == 0 for s in st)
    return {"value": len(idx) / dt, "unit": "RSVDs/s", "cores": threads, "host_cores": cores, "threads": threads,
            "kind": "oracle",
            "sample": f"{len(idx)} of the {len(mats)} matrices (512x512, k=256 p=16 q=2), FP64 C oracle, "
                      f"one matrix per thread on {threads} threads ({cores} host cores available), {dt:.1f} s wall"}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the FETCH_SIZE/WRITE_SIZE passes
    summarised under profiles/, or None when no pass was taken or the kernel's
    source changed since (the summary records the source's SHA-1)."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic_bytes_per_launch "):
                continue
            f = dict(kv.split("=", 1) for kv in line.split()[1:])
            if f.get("kernel") != kernel or f.get("workload") != workload:
                continue
            src = os.path.join(ROOT, f["source"])
            if os.path.exists(src) and hashlib.sha1(open(src, "rb").read()).hexdigest() == f["sha1"]:
                return float(f["bytes"])
    return None


def gen_matrices(probs, dtype):
    """Seeded test matrices, generated on the host in parallel (numpy releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(lambda pr: pr.matrix().astype(dtype), probs))


def diff_leg(args, P, torch, wl):
    """Differentiation workload: 64 FP32 matrices 1024 x 1024, s_i = i^-1.5 with
    three near-degenerate pairs, k = 128, p = 16, q = 2, FP32 sketch products;
    one step = forward of the whole batch plus the hand-written adjoint for
    seeded Gaussian cotangents (both HIP-graph launches)."""
    import numpy as np
    W = wl.c5(args.diff_batch)
    probs = W.problems
    log(f"[bench] differentiation leg: generating {len(probs)} matrices 1024x1024")
    mats = gen_matrices(probs, np.float32)
    As = [torch.from_numpy(A).cuda() for A in mats]
    plist = [dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs]
    plan = P.Plan(plist, torch.float32, "f32", graph=True, save=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(1234)
    dU = [torch.randn((pr.m, pr.k), generator=g, device="cuda") for pr in probs]
    dS = [torch.randn((pr.k,), generator=g, device="cuda") for pr in probs]
    dVT = [torch.randn((pr.k, pr.n), generator=g, device="cuda") for pr in probs]
    dA = [torch.empty((pr.m, pr.n), device="cuda") for pr in probs]
    for _ in range(2):
        plan.execute(As)
        plan.backward(dU, dS, dVT, 0.0, dA=dA)
    torch.cuda.synchronize()
    steps = args.diff_steps
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(As)
    torch.cuda.synchronize()
    fms = (time.perf_counter() - t0) / steps * 1e3
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(As)
        plan.backward(dU, dS, dVT, 0.0, dA=dA)
    torch.cuda.synchronize()
    tms = (time.perf_counter() - t0) / steps * 1e3
    info = plan.info.cpu().numpy()
    finite = all(bool(torch.isfinite(x).all()) for x in dA)
    bprof = plan.profile_backward(dU, dS, dVT, 0.0, dA=dA)
    bw_gemm_ms, bw_gemm_n, bw_gemm_fl = bprof["bw_gemm"]
    fprof = plan.profile(As)
    fwd_fl = sum(v[2] for k, v in fprof.items() if k in ("sketch", "gram", "project", "backproj"))
    plan.close()
    # the same forward from a plan that saves nothing for an adjoint: its small
    # SVD runs on the triangular factor of B (n = 7.1 l here)
    fplan = P.Plan(plist, torch.float32, "f32", graph=True)
    fplan.execute(As)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fplan.execute(As)
    torch.cuda.synchronize()
    nsms = (time.perf_counter() - t0) / steps * 1e3
    ns_ok = bool(np.all(fplan.info.cpu().numpy() == 0))
    fplan.close()
    return {
        "workload": f"C5: {len(probs)} x 1024x1024 FP32, s_i=i^-1.5 with 3 pairs (gap 1e-6), "
                    "k=128 p=16 q=2, FP32 sketch products, adjoint products FP64",
        "forward_ms": fms,
        "forward_nosave_ms": nsms,
        "forward_nosave_per_s": len(probs) / (nsms / 1e3),
        "forward_backward_ms": tms,
        "backward_ms": tms - fms,
        "forward_backward_per_s": len(probs) / (tms / 1e3),
        "status_ok": bool(np.all(info == 0)) and finite and ns_ok,
        "bw_phases_ms": {k: round(v[0], 4) for k, v in bprof.items() if v[1] > 0},
        "fw_phases_ms": {k: round(v[0], 4) for k, v in fprof.items() if v[1] > 0},
        "bw_gemm_flops": bw_gemm_fl,
        "fw_gemm_flops": fwd_fl,
        "bw_gemm_tflops": bw_gemm_fl / (bw_gemm_ms * 1e-3) / 1e12 if bw_gemm_ms else None,
        "bw_gemm_frac_of_fp64_peak": (bw_gemm_fl / (bw_gemm_ms * 1e-3) / 1e12) / 78.6 if bw_gemm_ms else None,
    }


def precision_leg(args, P, torch, wl):
    """Mixed precision on the TTN-shaped batch: 16 matrices 1024 x 1024 stored
    in FP32, s_i = |i^-1.2 (1 + 0.05 xi)|, k = 64, p = 16, q = 3.  The same
    batch runs with BF16 and with FP32 sketch and power-iteration products
    (FP64 Cholesky QR, FP64 projection B = Q^T A, FP64 small SVD) and fully in
    FP64 (the FP32 values upcast), and the two mixed forms again with their last
    power step in FP64 (RSVD_PLAN_FP64_FINAL).  Reports the step times, the GEMM work
    rate, the truncation error against the optimum and each mixed form's
    singular values against the FP64 path's, relative to sigma_1."""
    import numpy as np
    W = wl.c3(16)
    probs = W.problems
    log(f"[bench] precision leg: generating {len(probs)} matrices 1024x1024")
    mats = gen_matrices(probs, np.float32)
    A32 = [torch.from_numpy(A).cuda() for A in mats]
    A64 = [A.double() for A in A32]
    plist = [dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs]
    gemm_flops = sum(pr.gemm_flops() for pr in probs)
    # the optimal discarded weight of each input: the stored FP32 values' own tail
    tails = [float(np.sum(np.linalg.svd(A.astype(np.float64), compute_uv=False)[pr.k:] ** 2))
             for A, pr in zip(mats[:2], probs[:2])]
    out = {"workload": f"C3: {len(probs)} x 1024x1024 FP32 storage, s_i=|i^-1.2 (1+0.05 xi)|, k=64 p=16 q=3"}
    sig = {}
    ref0 = mats[0].astype(np.float64)
    forms = (("bf16", "bf16", torch.float32, A32, False), ("f32", "f32", torch.float32, A32, False),
             ("f64", "f64", torch.float64, A64, False), ("bf16_fp64_final", "bf16", torch.float32, A32, True),
             ("f32_fp64_final", "f32", torch.float32, A32, True))
    for key, prec_, dtype, As, f64f in forms:
        prec = key
        plan = P.Plan(plist, dtype, prec_, graph=True, fp64_final=f64f)
        plan.execute(As)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.diff_steps):
            plan.execute(As)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.diff_steps * 1e3
        w = plan.w.cpu().numpy()
        ok = bool(np.all(plan.info.cpu().numpy() == 0))
        sig[prec] = [o[1].double().cpu().numpy() for o in plan.outputs]
        out[prec] = {"ms": ms, "per_s": len(probs) / (ms / 1e3),
                     "gemm_tflops": gemm_flops / (ms * 1e-3) / 1e12, "status_ok": ok,
                     "eps_F_over_delta_EY": [float(np.sqrt(w[b] / tails[b])) for b in range(len(tails))]}
        U, S, VT = (t.double().cpu().numpy() for t in plan.outputs[0])
        out[prec]["vs_oracle_problem0"] = vs_oracle(ref0, probs[0], U, S, VT)
        # the sketch and power products read A (in the sketch precision) once each:
        # achieved bytes per second of those passes, against HBM and the cache
        prof = plan.profile(As)
        sk_ms = prof["sketch"][0]
        nbytes = sum(sketch_bytes(pr, prec_, f64f, 8 if dtype == torch.float64 else 4) for pr in probs)
        out[prec]["sketch_ms"] = sk_ms
        out[prec]["sketch_bytes"] = nbytes
        out[prec]["sketch_GBs"] = nbytes / (sk_ms * 1e-3) / 1e9 if sk_ms and nbytes else None
        out[prec]["sketch_frac_of_hbm"] = out[prec]["sketch_GBs"] / 8000.0 if out[prec]["sketch_GBs"] else None
        plan.close()
    for prec in ("bf16", "f32", "bf16_fp64_final", "f32_fp64_final"):
        out[prec]["max_dsigma_over_s1_vs_f64"] = max(
            float(np.max(np.abs(a - b)) / b[0]) for a, b in zip(sig[prec], sig["f64"]))
        out[prec]["speedup_vs_f64"] = out["f64"]["ms"] / out[prec]["ms"]
    return out


def sketch_bytes(pr, prec, fp64_final=False, storage=4):
    """Algorithmic bytes of the 2q + 1 sketch and power products of one
    problem: each reads A once (sketch precision: 2, 4 or 8 bytes), reads its
    l-column operand (Omega in the sketch precision, the FP64 bases after)
    and writes its l-column product (FP32 in the mixed modes, else FP64).
    With the last power step in FP64 (products 2q - 1 and 2q), those two read
    A in its storage type (`storage` bytes) and write FP64 products."""
    ea = {"bf16": 2, "f32": 4, "f64": 8}[prec]
    ey = 8 if prec == "f64" else 4
    m, n, l = pr.m, pr.n, pr.l
    total = 0
    for s in range(2 * pr.q + 1):
        rows_in, rows_out = (n, m) if s % 2 == 0 else (m, n)
        f64 = fp64_final and s >= 2 * pr.q - 1
        total += (m * n * (storage if f64 else ea) + rows_in * l * (ea if s == 0 else 8)
                  + rows_out * l * (8 if f64 else ey))
    return total


def timed(torch, fn, steps, warmup=1):
    """Mean wall time (ms) of fn over `steps` calls after `warmup`, bracketed by synchronisation."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def vs_oracle(A64, pr, U, S, VT):
    """Singular-value and projector errors of one GPU factorisation against
    the FP64 CPU oracle on the same input and the same Gaussian test matrix:
    max |d sigma_i| / sigma_1, max |d sigma_i| / sigma_i, the same over the
    leading quarter of the kept values, and the sines of the largest
    principal angles between the kept left and right singular subspaces."""
    import numpy as np

    import oracle
    ref = oracle.rsvd(A64, pr.k, pr.p, pr.q, pr.seed, pr.delta)
    k = min(int(np.count_nonzero(S)), ref.k_kept)
    d = np.abs(S[:k] - ref.S[:k])
    q4 = max(1, k // 4)

    def sin_theta(X, Y):  # ||(I - Y Y^T) X||_2 for orthonormal columns
        return float(np.linalg.norm(X - Y @ (Y.T @ X), 2))

    return {"k": k, "max_dsigma_over_s1": float(np.max(d) / ref.S[0]),
            "max_dsigma_over_si": float(np.max(d / ref.S[:k])),
            "max_dsigma_over_s1_leading_quarter": float(np.max(d[:q4]) / ref.S[0]),
            "argmax_i": int(np.argmax(d)),
            "sin_theta_U": sin_theta(U[:, :k], ref.U[:, :k]), "sin_theta_V": sin_theta(VT[:k].T, ref.VT[:k].T)}


def c1_leg(P, torch, wl, reps):
    """The single 128 x 128 FP64 factorisation (k = 64, p = 10, q = 2):
    latency per factorisation, median over `reps` calls, of a one-problem
    plan's graph launch, of the blocking one-shot call, of the
    allocation-free call, and of the same-GPU full-SVD truncation."""
    import numpy as np
    pr = wl.c1().problems[0]
    A = torch.from_numpy(pr.matrix()).cuda()
    plan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed)], torch.float64, "f64", graph=True)
    fplan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k)], torch.float64, "f64", fullsvd=True, graph=True)

    def median_us(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1) * 1e3)
        return float(np.median(t))

    out = {"workload": "C1: one 128x128 FP64, s_i=exp(-0.08 i), k=64 p=10 q=2"}
    out["rsvd_plan_graph_us"] = median_us(lambda: plan.execute([A]))
    out["rsvd_one_shot_us"] = median_us(lambda: P.rsvd_truncate(A, pr.k, pr.p, pr.q, pr.seed))
    out["rsvd_noalloc_us"] = median_us(lambda: P.rsvd_truncate_noalloc(A, pr.k, pr.p, pr.q, pr.seed))
    out["fullsvd_plan_graph_us"] = median_us(lambda: fplan.execute([A]))
    out["speedup_vs_fullsvd"] = out["fullsvd_plan_graph_us"] / out["rsvd_plan_graph_us"]
    _, w, _, info = plan.execute([A])
    _, fw, _, finfo = fplan.execute([A])
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and int(finfo.item()) == 0
    out["eps_F_over_delta_EY_rsvd"] = float(np.sqrt(w.item() / fw.item()))
    out["reps"] = reps
    plan.close()
    fplan.close()
    return out


def qsweep_leg(P, torch, probs, As, w_full, q_max=6):
    """The power-step count that brings the RSVD of the headline batch to
    eps_F / delta_EY <= 1.01 (the optimum is the full SVD's discarded
    weight), with the step time at each q."""
    import numpy as np
    out = {}
    for q in range(probs[0].q + 1, q_max + 1):
        plan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=q, seed=pr.seed) for pr in probs], torch.float64,
                      "f64", graph=True)
        ms = timed(torch, lambda: plan.execute(As), 5)
        _, w, _, info = plan.execute(As)
        torch.cuda.synchronize()
        ratio = float(np.mean(np.sqrt(w.cpu().numpy() / w_full)))
        ok = bool(np.all(info.cpu().numpy() == 0))
        plan.close()
        out[f"q{q}"] = {"ms_per_step": ms, "per_s": len(probs) / (ms / 1e3), "eps_F_over_delta_EY": ratio,
                        "status_ok": ok}
        if ratio <= 1.01:
            out["q_for_1pct"] = q
            break
    return out


def c2_f32_leg(P, torch, probs, mats, w_full, sig64, steps):
    """The headline batch stored in FP32 with FP32 sketch and power products
    (FP64 Cholesky QR, FP64 B = Q^T A, FP64 small SVD), and its full-SVD
    truncation from the same FP32 values."""
    import numpy as np
    A32 = [torch.from_numpy(A.astype(np.float32)).cuda() for A in mats]
    plist = [dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs]
    plan = P.Plan(plist, torch.float32, "f32", graph=True)
    ms = timed(torch, lambda: plan.execute(A32), steps, 3)
    outs, w, _, info = plan.execute(A32)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    s32 = [o[1].double().cpu().numpy() for o in outs]
    fplan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k) for pr in probs], torch.float32, "f64", fullsvd=True)
    fms = timed(torch, lambda: fplan.execute(A32), 2)
    fplan.close()
    res = {"workload": "C2 in FP32: 32 x 512x512 stored FP32, FP32 sketch/power products",
           "ms_per_step": ms, "per_s": len(probs) / (ms / 1e3),
           "gemm_tflops": sum(pr.gemm_flops() for pr in probs) / (ms * 1e-3) / 1e12,
           "fullsvd_ms_per_step": fms, "speedup_vs_fullsvd": fms / ms,
           "eps_F_over_delta_EY": float(np.mean(np.sqrt(w.cpu().numpy() / w_full))),
           "max_dsigma_over_s1_vs_gpu_f64": max(float(np.max(np.abs(a - b)) / b[0]) for a, b in zip(s32, sig64))}
    U, S, VT = (t.double().cpu().numpy() for t in outs[0])
    res["vs_oracle_problem0"] = vs_oracle(A32[0].double().cpu().numpy(), probs[0], U, S, VT)
    plan.close()
    return res


def c4_leg(P, torch, wl, steps, subset_every=16, extras=True):
    """The uneven batch of symmetry sectors: 512 problems, m, n uniform in
    [32, 2048], s_i = exp(-alpha i), k = min(m, n)/4 rounded to 8, p = 16,
    q = 2, delta_trunc = 1e-10, stored FP32 with FP32 sketch products; one
    plan, one graph launch.  On every `subset_every`-th problem: the same
    problems as one batched plan, one at a time in FP64 (rsvd_truncate per
    matrix), and by the full-SVD truncation."""
    import numpy as np
    W = wl.c4(512)
    probs = W.problems
    log(f"[bench] C4 leg: generating {len(probs)} matrices on the device")
    As = [wl.c4_matrix_device(pr.m, pr.n, pr.spectrum, 9000 + b, torch) for b, pr in enumerate(probs)]
    torch.cuda.synchronize()
    plist = [dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed, delta=pr.delta) for pr in probs]
    plan = P.Plan(plist, torch.float32, "f32", graph=True)
    ms = timed(torch, lambda: plan.execute(As), steps)
    _, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    w, kk, info = w.cpu().numpy(), kk.cpu().numpy(), info.cpu().numpy()
    # optimal discarded weight at the kept rank, from the exact spectrum
    opt = np.array([np.sum(pr.spectrum[int(kk[b]):] ** 2) for b, pr in enumerate(probs)])
    tot = np.array([np.sum(pr.spectrum ** 2) for pr in probs])
    ratio = np.sqrt(np.maximum(w, 0) / np.maximum(opt, 1e-300 * tot))
    gemm = sum(pr.gemm_flops() for pr in probs)
    prof = plan.profile(As)
    plan.close()
    res = {"workload": "C4: 512 uneven problems, m,n in [32,2048], s_i=exp(-alpha i), k=min(m,n)/4, p=16 q=2, "
                       "delta=1e-10, FP32 storage and sketch products",
           "ms_per_step": ms, "per_s": len(probs) / (ms / 1e3), "gemm_tflops": gemm / (ms * 1e-3) / 1e12,
           "gemm_flops": gemm, "status_ok": bool(np.all(info == 0)),
           "cut_binds": int(np.sum(kk < np.array([min(pr.k, pr.m, pr.n) for pr in probs]))),
           "eps_F_over_delta_EY_median": float(np.median(ratio[opt > 1e-13 * tot])),
           "eps_F_over_delta_EY_max": float(np.max(ratio[opt > 1e-13 * tot])),
           "phases_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1] > 0}}
    if not extras:  # the batch plan alone (profiling)
        del As
        torch.cuda.empty_cache()
        return res
    # the tile autotuner on the uneven batch: the first execute of a tuned plan
    # times every tile of each tunable product on these inputs, then the plan
    # is timed like the untuned one
    tplan = P.Plan(plist, torch.float32, "f32", graph=True, tune=True)
    heur = tplan.tiles()
    t0 = time.perf_counter()
    tplan.execute(As)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    tms = timed(torch, lambda: tplan.execute(As), steps)
    tuned = tplan.tiles()
    tplan.close()
    res["tuned"] = {"ms_per_step": tms, "speedup_vs_heuristic": ms / tms, "tuning_execute_s": tune_s,
                    "products": len(tuned), "changed": int(sum(a != b for a, b in zip(tuned, heur))),
                    "tiles": [f"{a}x{b}" for a, b in tuned], "heuristic": [f"{a}x{b}" for a, b in heur]}
    sub = list(range(0, len(probs), subset_every))
    Ssub = [As[b] for b in sub]
    splan = P.Plan([plist[b] for b in sub], torch.float32, "f32", graph=True)
    sms = timed(torch, lambda: splan.execute(Ssub), steps)
    splan.close()

    def one_at_a_time():
        for b in sub:
            pr = probs[b]
            P.rsvd_truncate(As[b], pr.k, pr.p, pr.q, pr.seed, pr.delta, "f64")
    oms = timed(torch, one_at_a_time, 1)
    # the full SVD costs O(m n min(m, n)) per sweep: only the subset's problems with min(m, n) <= 640
    small = [b for b in sub if min(probs[b].m, probs[b].n) <= 640]
    Ssmall = [As[b] for b in small]
    fplan = P.Plan([dict(m=probs[b].m, n=probs[b].n, k=probs[b].k, delta=probs[b].delta) for b in small],
                   torch.float32, "f64", fullsvd=True)
    fms = timed(torch, lambda: fplan.execute(Ssmall), 1)
    fplan.close()
    rplan = P.Plan([plist[b] for b in small], torch.float32, "f32", graph=True)
    rms = timed(torch, lambda: rplan.execute(Ssmall), steps)
    rplan.close()
    res["subset"] = {"problems": len(sub), "every": subset_every, "batched_f32_ms": sms,
                     "one_at_a_time_f64_ms": oms, "speedup_vs_one_at_a_time_f64": oms / sms,
                     "fullsvd_problems": len(small), "fullsvd_min_mn_max": 640, "fullsvd_ms": fms,
                     "batched_f32_ms_same_problems": rms, "speedup_vs_fullsvd": fms / rms}
    del As
    torch.cuda.empty_cache()
    return res


def krylov_leg(P, torch, wl, steps):
    """The outlook's variants against the RSVD (same k, p, seed): step time and
    eps_F / delta_EY (delta_EY from the exact spectrum the inputs are built
    with) on the TTN-shaped batch (16 x 1024^2, BF16 sketch products) and the
    headline batch (32 x 512^2 FP64).
    * block-Krylov at equal passes over A (same q): L = (k + p)(q + 1) = 320 on
      the first batch; on the second L = min(272 x 3, 512) = 512 spans the
      whole row space and the projection is exact;
    * single view (Y = A Omega and W = Psi A, no power steps; one more product
      with A for its true error) against the RSVD without power steps (q = 0,
      two passes over A: Y and B)."""
    import numpy as np
    out = {}
    for name, W, dtype, prec in (("C3_bf16", wl.c3(16), torch.float32, "bf16"), ("C2_f64", wl.c2(32), torch.float64, "f64")):
        probs = W.problems
        log(f"[bench] block-Krylov leg: {name}")
        As = [torch.from_numpy(A).to(dtype).cuda() for A in gen_matrices(probs, np.float64)]
        plist = [dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs]
        opt = np.array([np.sum(pr.spectrum[pr.k:] ** 2) for pr in probs])
        res = {"L": min(probs[0].l * (probs[0].q + 1), probs[0].m, probs[0].n), "q": probs[0].q}
        plist0 = [dict(pr, q=0) for pr in plist]
        for key, pl, kw in (("rsvd", plist, {}), ("krylov", plist, dict(block_krylov=True)),
                            ("rsvd_q0", plist0, {}), ("single_view", plist0, dict(single_view=True))):
            plan = P.Plan(pl, dtype, prec, graph=True, **kw)
            ms = timed(torch, lambda: plan.execute(As), steps)
            _, w, _, info = plan.execute(As)
            torch.cuda.synchronize()
            res[key] = {"ms_per_step": ms, "per_s": len(probs) / (ms / 1e3),
                        "eps_F_over_delta_EY": float(np.mean(np.sqrt(w.cpu().numpy() / opt))),
                        "status_ok": bool(np.all(info.cpu().numpy() == 0))}
            plan.close()
        out[name] = res
        del As
    return out


def complex_leg(P, torch, wl, steps):
    """The headline shape in complex double (the paper's simulations are
    complex): 32 x 512^2, A = U diag(i^-1.5) V^H with Haar unitary U, V,
    k = 256, p = 16, q = 2, one complex plan (the real embedding, 1024^2 and
    rank 512, on the device), one graph launch per step; eps_F / delta_EY
    from the exact spectrum."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    probs = wl.c2(32).problems
    log("[bench] complex leg: generating 32 complex matrices 512x512")
    with ThreadPoolExecutor(8) as ex:
        mats = list(ex.map(lambda pr: wl.make_complex_matrix(pr.m, pr.n, pr.spectrum, pr.a_seed), probs))
    As = [torch.from_numpy(A).cuda() for A in mats]
    plist = [dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs]
    plan = P.Plan(plist, torch.complex128, "f64", graph=True)
    ms = timed(torch, lambda: plan.execute(As), steps)
    _, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    plan.close()
    opt = np.array([np.sum(pr.spectrum[pr.k:] ** 2) for pr in probs])
    w = w.cpu().numpy()
    out = {"workload": "C2 shape in complex double: 32 x 512x512, s_i=i^-1.5, k=256 p=16 q=2",
           "ms_per_step": ms, "per_s": len(probs) / (ms / 1e3),
           "eps_F_over_delta_EY": float(np.mean(np.sqrt(w / opt))),
           "status_ok": bool(np.all(info.cpu().numpy() == 0))}
    del As
    torch.cuda.empty_cache()
    return out


def bandwidth_leg(torch):
    """Device-to-device copy rates (read + write bytes per second): a 32 MiB
    buffer, which the 256 MB last-level cache holds, and 4 GiB, which it does
    not."""
    out = {}
    for name, nbytes in (("copy_32MiB_GBs", 32 << 20), ("copy_4GiB_GBs", 4 << 30)):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        reps = 50 if nbytes < (1 << 30) else 5
        ms = timed(torch, lambda: dst.copy_(src), reps, 3)
        out[name] = 2 * nbytes / (ms * 1e-3) / 1e9
        del src, dst
    torch.cuda.empty_cache()
    return out



def tebd_leg(P, torch, wl):
    """The TEBD compression shapes (Sec. III): 64 product updates (200 x 500,
    ratio 1/2) and 32 block updates (500 x 500, ratio 1/5) at chi = 100, FP64,
    each batch one graph launch, against the same-GPU full-SVD truncation."""
    import numpy as np
    out = {}
    for name, W in (("product_200x500", wl.tebd_product(64)), ("block_500x500", wl.tebd_block(32))):
        log(f"[bench] TEBD leg: {name}")
        probs = W.problems
        As = [torch.from_numpy(pr.matrix()).cuda() for pr in probs]
        plan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs],
                      torch.float64, "f64", graph=True)
        fplan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k) for pr in probs], torch.float64, "f64", fullsvd=True)
        res = {}
        for key, pl, steps in (("rsvd", plan, 10), ("fullsvd", fplan, 3)):
            pl.execute(As)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                pl.execute(As)
            torch.cuda.synchronize()
            res[key] = (time.perf_counter() - t0) / steps * 1e3
            _, w, _, info = pl.execute(As)
            torch.cuda.synchronize()
            assert np.all(info.cpu().numpy() == 0)
            res[key + "_w"] = w.cpu().numpy()
        out[name] = {"batch": len(probs), "rsvd_per_s": len(probs) / (res["rsvd"] / 1e3), "rsvd_ms": res["rsvd"],
                     "fullsvd_per_s": len(probs) / (res["fullsvd"] / 1e3), "speedup_vs_fullsvd": res["fullsvd"] / res["rsvd"],
                     "eps_F_over_delta_EY_rsvd": float(np.mean(np.sqrt(res["rsvd_w"] / res["fullsvd_w"])))}
        plan.close()
        fplan.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is "
                                   "design-only (independent problems would be split by flop count)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1710_01463_amd as P
    import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_mib:
        # a plain copy kernel of known size, for scaling FETCH_SIZE / WRITE_SIZE counters
        n = args.copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}))
        return
    if args.only == "c4":
        print(json.dumps(c4_leg(P, torch, wl, args.steps, extras=False)))
        return
    W = wl.c2(args.batch)
    probs = W.problems
    log(f"[bench] generating {len(probs)} matrices {probs[0].m}x{probs[0].n}")
    mats = gen_matrices(probs, np.float64)
    dtype = torch.float64 if args.prec == "f64" else torch.float32
    As = [torch.from_numpy(A).to(dtype).cuda() for A in mats]
    plist = [dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs]
    plan = P.Plan(plist, dtype, args.prec, graph=True, tune=not args.no_tune)
    heuristic_tiles = plan.tiles()
    if not args.no_tune:
        t0 = time.perf_counter()
        plan.execute(As)  # times every tile of each forward product, then executes
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t0
        log(f"[bench] tuning execute {tune_s:.2f} s, tiles {plan.tiles()}")

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        plan.execute(As)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute(As)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    value = len(probs) / (ms / 1e3)
    gemm_flops = sum(pr.gemm_flops() for pr in probs)
    outs, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    w_rsvd = w.cpu().numpy()
    assert np.all(info == 0), f"non-zero status {info}"
    sig64 = [o[1].double().cpu().numpy() for o in outs]  # before post-selection truncates the outputs

    result = {
        "metric": "rank-k RSVDs/sec (batched, one graph launch per step)",
        "value": value,
        "unit": "RSVDs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32+f64", "bf16": "bf16+f64"}[args.prec],
        "data": "synthetic: A = U diag(i^-1.5) V^T, Haar U, V (seeded)",
        "config": {"workload": f"C2: {len(probs)} x 512x512, s_i=i^-1.5, k=256 p=16 q=2, "
                               f"sketch/power arithmetic {args.prec}",
                   "batch": len(probs), "m": 512, "n": 512, "k": 256, "p": 16, "q": 2},
        "gemm_tflops": gemm_flops / (ms / 1e3) / 1e12,
    }
    if not args.no_tune:
        # the same batch with the shape heuristic's tiles, timed the same way
        hplan = P.Plan(plist, dtype, args.prec, graph=True)
        for _ in range(max(args.warmup, 1)):
            hplan.execute(As)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            hplan.execute(As)
        torch.cuda.synchronize()
        hms = (time.perf_counter() - t0) / args.steps * 1e3
        hplan.close()
        result["tiles"] = {"tuned": [f"{a}x{b}" for a, b in plan.tiles()],
                           "heuristic": [f"{a}x{b}" for a, b in heuristic_tiles],
                           "tuning_execute_s": round(tune_s, 3), "heuristic_ms_per_step": hms}

    # per-phase breakdown (eager launches, HIP events on the plan's stream) and
    # the roofline of the dominant kernel, priced at the method's algorithmic work
    prof = plan.profile(As)
    result["phases_ms"] = {k: round(v[0], 4) for k, v in prof.items() if v[1] > 0}
    dom = max(prof, key=lambda k: prof[k][0])
    ms_dom, n_dom, fl_dom = prof[dom]
    kernel_of = {"jacobi": "jacobi_round_kernel", "sketch": "gemm_kernel", "gram": "gemm_kernel",
                 "project": "gemm_kernel", "backproj": "gemm_kernel", "chol": "chol_rl_kernel",
                 "trsm": "trsm_kernel"}
    if dom == "jacobi":
        # algorithmic work of the small SVD of one 272 x 512 B (one-sided Jacobi,
        # about 8 sweeps): 1.77 GFLOP per matrix; one step processes the batch's
        # matrices over n_dom launches
        alg = len(probs) * SMALL_SVD_FLOPS_C2
        peak = 78.6  # FP64 MFMA: the Grams and rotations run on FP64 MFMA
    else:
        alg = fl_dom
        peak = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6}["f64" if dom != "sketch" else args.prec]
    avg_s = ms_dom / n_dom * 1e-3 if n_dom else 0.0
    achieved = (alg / n_dom) / avg_s / 1e12 if n_dom and ms_dom else 0.0
    traffic = measured_traffic(kernel_of.get(dom, dom), "C2") if args.prec == "f64" else None
    result["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                          "frac": achieved / peak, "traffic": traffic,
                          "kernel": kernel_of.get(dom, dom), "phase": dom,
                          "avg_launch_us": avg_s * 1e6 if n_dom else None,
                          "launches_per_step": n_dom,
                          "algorithmic_flops_per_launch": alg / n_dom if n_dom else None,
                          "executed_flops_per_launch": fl_dom / n_dom if n_dom else None,
                          "hbm_GBs": traffic / avg_s / 1e9 if traffic and avg_s else None,
                          "hbm_frac": traffic / avg_s / 8e12 if traffic and avg_s else None}

    # sector post-selection over the batch's outputs (the 32 problems as one
    # sector group, half of the 32 x 256 values kept); each timed call follows
    # a fresh execute, since the call truncates the outputs in place
    chi_ps = sum(pr.k for pr in probs) // 2
    ps_ms = []
    for _ in range(0 if args.no_extra else 5):
        plan.execute(As)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        chi_s = plan.postselect(chi_ps)
        e1.record()
        torch.cuda.synchronize()
        ps_ms.append(e0.elapsed_time(e1))
    if ps_ms:
        assert int(chi_s.sum()) == chi_ps
        result["postselect"] = {"sectors": len(probs), "candidates": int(sum(pr.k for pr in probs)), "chi": chi_ps,
                                "us": float(np.median(ps_ms)) * 1e3}

    # fixed-error truncation with an adaptive rank on one C2 matrix: rank 32,
    # 64, 128, ... until the 1e-4 relative discarded-weight cut binds (the first
    # call builds the plan of every rank tried; the second is timed)
    if args.prec == "f64" and not args.no_extra:
        ad = dict(k0=32, k_max=512, delta=1e-4, p=16, q=2, seed=probs[0].seed)
        P.rsvd_truncate_adaptive(As[0], ad["k0"], ad["k_max"], ad["delta"], ad["p"], ad["q"], seed=ad["seed"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, ad_w, ad_kk, ad_att = P.rsvd_truncate_adaptive(As[0], ad["k0"], ad["k_max"], ad["delta"], ad["p"],
                                                                ad["q"], seed=ad["seed"])
        torch.cuda.synchronize()
        ad.update(matrix="C2 problem 0 (512x512)", attempts=ad_att, k_kept=int(ad_kk.item()),
                  ms=(time.perf_counter() - t0) * 1e3)
        result["adaptive"] = ad

    w_full = None
    if not args.no_compare:
        # same-GPU full-SVD truncation on the same batch (FP64 Jacobi)
        log("[bench] full-SVD leg")
        fplan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k) for pr in probs], dtype, "f64", fullsvd=True)
        fms = timed(torch, lambda: fplan.execute(As), max(1, min(3, args.steps)))
        _, fw, fkk, finfo = fplan.execute(As)
        torch.cuda.synchronize()
        w_full = fw.cpu().numpy()
        fplan.close()
        # plain FP64 RSVD, one problem per call
        log("[bench] one-at-a-time leg")
        A64 = [torch.from_numpy(A).cuda() for A in mats]

        def one_at_a_time():
            for A, pr in zip(A64, probs):
                P.rsvd_truncate(A, pr.k, pr.p, pr.q, pr.seed)
        oms = timed(torch, one_at_a_time, 1)
        # equal truncation error: eps_F / delta_EY from the exact discarded weights
        eps_ratio = float(np.mean(np.sqrt(w_rsvd / w_full)))
        result["compare"] = {
            "fullsvd_per_s": len(probs) / (fms / 1e3),
            "fullsvd_ms_per_step": fms,
            "speedup_vs_fullsvd": fms / ms,
            "one_at_a_time_f64_per_s": len(probs) / (oms / 1e3),
            "speedup_vs_one_at_a_time_f64": oms / ms,
            "eps_F_over_delta_EY_rsvd": eps_ratio,
            "eps_F_over_delta_EY_fullsvd": 1.0,
        }
        if args.prec == "f64" and not args.no_extra:
            log("[bench] equal-error leg")
            result["equal_error"] = qsweep_leg(P, torch, probs, As, w_full)
            result["equal_error"]["fullsvd_ms_per_step"] = fms
            log("[bench] C2 FP32 leg")
            result["c2_f32"] = c2_f32_leg(P, torch, probs, mats, w_full, sig64, args.steps)

    if not args.no_extra:
        log("[bench] C1 leg")
        result["c1"] = c1_leg(P, torch, wl, args.c1_reps)
        result["c4"] = c4_leg(P, torch, wl, 3)
        result["variants"] = krylov_leg(P, torch, wl, 5)
        result["complex"] = complex_leg(P, torch, wl, 3)
        result["bandwidth"] = bandwidth_leg(torch)

    if not args.no_compare and args.prec == "f64":
        result["tebd"] = tebd_leg(P, torch, wl)

    if not args.no_diff:
        result["differentiation"] = diff_leg(args, P, torch, wl)

    if not args.no_diff:
        try:
            result["precision"] = precision_leg(args, P, torch, wl)
        except Exception as e:  # reported, never fatal to the main line
            result["precision"] = {"error": repr(e)}

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle leg")
        result["cpu_baseline"] = cpu_baseline(mats, probs, args.cpu_sample)

    print(json.dumps(result))


if __name__ == "__main__":
    main()
