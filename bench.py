"""Benchmark: FP64 tile Cholesky of the n=65536, nb=1024 Matern covariance
(nu=1.5, range=0.1, nugget=1e-6) on one MI355X, plus the mixed-precision
versus FP64 time-to-solution on the n=131072, nb=1024 Matern workload
(nu=0.5, range=0.03, nugget=1e-4, target accuracy 1e-9, 16 right-hand sides,
refined to 1e-9 relative residual).

One step = factorization (panel GEMM/SYRK, POTRF, TRSM under the static
left-looking schedule) + log-determinant + solve with 16 right-hand sides,
with the matrix already resident in HBM (generated on the GPU before the
timed region; the factor goes to separate storage so the input survives).
The metric counts n^3/3 flops per step.

Prints one JSON line. `roofline` is the dominant kernel (the panel GEMM)
timed with HIP events on the library's compute stream: algorithmic flops of
all its launches / summed launch time, against the FP64 matrix peak.
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload
(the leading 4096 x 4096 principal block, same tile size). `mxp_vs_fp64`,
`loglik_grad` and `ooc_vs_in_core` are the mixed-precision, likelihood-gradient
and out-of-core legs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
# HBM bytes per bulk panel-GEMM launch from the calibrated FETCH_SIZE and
# WRITE_SIZE counter passes (profiles/panel_update_fp64_counters_n65536_nb1024.md),
# valid for the kernel sources they were taken with.
PANEL_TRAFFIC = {"bytes_per_launch": 2.9906e+10,
                 "sources_sha256": "23aee1e0c1c85c6c8e4b675a14c4b2c183956712798071f07f1af3739e45cf35"}


def panel_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in ("gemm_f64.hip", "gemm_f64.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2410_09819_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return PANEL_TRAFFIC["bytes_per_launch"] if h.hexdigest() == PANEL_TRAFFIC["sources_sha256"] else None
METRIC = "Cholesky TFLOP/s (n^3/3) + % peak, MxP vs FP64 at stated backward error"


_CPU_SAMPLE = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
import seeded_inputs as si
w = json.loads(sys.argv[2]); ns = int(sys.argv[3]); threads = int(sys.argv[4])
pts = si.points(w["n"], seed=w["seed"])[:ns]
A = oracle.matern_matrix(pts, w["sigma2"], w["range"], w["nu"], w["nugget"])
t0 = time.perf_counter()
_, info = oracle.tile_cholesky(A, w["nb"], threads=threads)
print(json.dumps({"seconds": time.perf_counter() - t0, "info": int(info)}))
"""


def host_cpu():
    """CPU model, sockets and physical cores of the host (lscpu), and the
    CPUs this process may run on."""
    import subprocess
    info = {"model": None, "sockets": None, "physical_cores": None,
            "cpus_allowed": len(os.sched_getaffinity(0))}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        kv = {}
        for line in txt.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "0") or 0)
        per = int(kv.get("Core(s) per socket", "0") or 0)
        info["sockets"] = sockets or None
        info["physical_cores"] = sockets * per or None
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(w, ns=4096):
    """The CPU oracle (OpenMP over the tiles of a column) on a bounded sample
    of the same workload, in a child process with one thread per allowed
    CPU (the OMP_NUM_THREADS share when it is set), bound one per core."""
    import subprocess
    cpu = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or cpu["cpus_allowed"]
    threads = max(1, min(threads, cpu["cpus_allowed"]))
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OMP_PLACES="cores", OMP_PROC_BIND="close")
    r = subprocess.run([sys.executable, "-c", _CPU_SAMPLE, ROOT, json.dumps(w), str(ns), str(threads)],
                       env=env, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError("cpu baseline failed:\n" + r.stderr[-2000:])
    res = json.loads(r.stdout.strip().splitlines()[-1])
    assert res["info"] == 0
    dt = res["seconds"]
    return {"value": ns ** 3 / 3.0 / dt / 1e12, "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu["model"], "sockets": cpu["sockets"],
            "physical_cores_host": cpu["physical_cores"], "cpus_allowed": cpu["cpus_allowed"],
            "binding": "OMP_PLACES=cores OMP_PROC_BIND=close",
            "sample": "leading %dx%d principal block of the same matrix, nb=%d, factorization only "
                      "(%.1f s)" % (ns, ns, w["nb"], dt)}


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# Dense peaks of the arithmetic each class's updates execute (TFLOP/s): the
# FP32 class runs as three FP16 MFMA products per binary32 product.
CLASS_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 2500.0 / 3.0, "fp16": 2500.0, "bf16": 2500.0,
                     "fp8": 5000.0}
CLASS_NAMES = ("fp64", "fp32", "fp16", "bf16", "fp8")


def map_roofline(n, class_flops, factor_ms):
    """Map-weighted roofline of a mixed factorization: t* = sum_p F_p / peak_p
    over the update flops F_p executed in each class, plus the POTRF / TRSM
    remainder of n^3/3 at the FP64 peak; frac = t* / measured time."""
    upd = sum(class_flops)
    t_star = (n ** 3 / 3.0 - upd) / (CLASS_PEAK_TFLOPS["fp64"] * 1e12)
    for name, f in zip(CLASS_NAMES, class_flops):
        t_star += f / (CLASS_PEAK_TFLOPS[name] * 1e12)
    return {"t_star_s": t_star, "factor_s": factor_ms * 1e-3, "frac": t_star / (factor_ms * 1e-3),
            "class_peaks_tflops": CLASS_PEAK_TFLOPS}


def _tiles_t_times(T, n, nb, G, diag=True):
    """U_j = sum_{i >= j} T_ij^T G_i over the packed lower tiles T (tile (i, j)
    column-major); diag=False leaves out the diagonal tiles."""
    import torch
    Nt, nb2, p = n // nb, nb * nb, G.shape[1]
    out = torch.zeros_like(G)
    t = 0
    for j in range(Nt):
        cnt = Nt - j
        col = T[t * nb2:(t + cnt) * nb2].view(cnt, nb, nb)  # col[s] = T_{j+s, j}^T
        s0 = 0 if diag else 1
        if cnt > s0:
            Gs = G[(j + s0) * nb:].view(cnt - s0, nb, p)
            out[j * nb:(j + 1) * nb] += torch.matmul(col[s0:], Gs).sum(0)
        t += cnt
    return out


def _tiles_times(T, n, nb, U):
    """V_i = sum_{j <= i} T_ij U_j over the packed lower tiles T (diagonal
    tiles used as stored, in full)."""
    import torch
    Nt, nb2, p = n // nb, nb * nb, U.shape[1]
    out = torch.zeros_like(U)
    t = 0
    for j in range(Nt):
        cnt = Nt - j
        col = T[t * nb2:(t + cnt) * nb2].view(cnt, nb, nb)
        Ut = U[j * nb:(j + 1) * nb].t().contiguous().unsqueeze(0).expand(cnt, p, nb).contiguous()
        prod = torch.matmul(Ut, col)  # U_j^T T_ij^T = (T_ij U_j)^T
        out[j * nb:] += prod.transpose(1, 2).reshape(cnt * nb, p)
        t += cnt
    return out


def probe_backward_error(A, L64, n, nb, nprobe=32, seed=97):
    """||(A - L L^T) G||_F / ||A G||_F for nprobe seeded N(0,1) columns G.
    A: packed lower tiles of the symmetric matrix (diagonal tiles in full);
    L64: packed lower binary64 tiles of the factor, strict upper parts of
    the diagonal tiles zero. A check outside the timed region, in torch
    binary64 products over the tile columns."""
    import torch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    G = torch.randn(n, nprobe, generator=gen, dtype=torch.float64).to(A.device)
    AG = _tiles_times(A, n, nb, G) + _tiles_t_times(A, n, nb, G, diag=False)
    LLG = _tiles_times(L64, n, nb, _tiles_t_times(L64, n, nb, G))
    return float(torch.linalg.norm(AG - LLG) / torch.linalg.norm(AG))


def mxp_comparison(tc, si, dev, n=None, eps=None, extra_eps=(1e-7, 1e-6), repeats=2, warmup=1,
                   probes=True):
    """Time-to-solution at n=131072: FP64 = factorization + 16-RHS solve;
    mixed precision = tile norms already known from generation, precision
    map + factorization + refined 16-RHS solve to 1e-9. Same matrix, same
    right-hand sides, matrix resident in HBM. Each variant runs `warmup`
    untimed times and `repeats` timed times (the reported time is their
    mean). After the timed runs, the probe backward error of the variant's
    factor is measured outside the timed region. eps overrides the map's
    target accuracy (default: the mxp workload's 1e-9); the refinement
    target stays 1e-9. extra_eps: further maps, timed the same way and
    refined to the same 1e-9 residual (reported separately)."""
    import numpy as np
    import torch
    w = dict(si.WORKLOADS["mxp"])
    if eps:
        w["eps"] = eps
    n, nb, nrhs = n or w["n"], w["nb"], w["nrhs"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = torch.from_numpy(si.points(n, seed=w["seed"])).to(dev)
    ctx = tc.Context(n, nb, nrhs=nrhs)
    A, tf, fro = tc.matern_tiles(ctx, pts, theta, nb)
    tf_h = tf.cpu().numpy()
    B0 = torch.from_numpy(np.ascontiguousarray(
        si.standard_normal((n, nrhs), seed=si.rhs_seed(w["seed"])).T)).to(dev)
    B = torch.empty_like(B0)
    Nt = n // nb
    flops = n ** 3 / 3.0
    out = {"workload": "mxp tile Cholesky, n=%d nb=%d, Matern nu=%g range=%g nugget=%g, target %g, "
                       "%d RHS refined to 1e-9" % (n, nb, w["nu"], w["range"], w["nugget"], w["eps"], nrhs),
           "timing": "%d untimed + %d timed runs per variant, mean of the timed" % (warmup, repeats),
           "probe_backward_error": "||(A - L L^T) G||_F / ||A G||_F, 32 seeded N(0,1) probe columns, "
                                   "factor upcast to binary64, outside the timed region"}

    def runs(once):
        """warmup + repeats calls of once() -> (mean seconds, times, last result)"""
        for _ in range(warmup):
            r = once()
            r[0].close()
            del r
        ts, last = [], None
        for i in range(repeats):
            if last is not None:
                last[0].close()
                last = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            last = once()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sum(ts) / len(ts), ts, last

    # FP64 path
    storage = torch.empty(tc.factor_bytes(n, nb) // 8, dtype=torch.float64, device=dev)

    def fp64_once():
        F = tc.factorize(ctx, A, n, nb, storage=storage)
        B.copy_(B0)
        tc.solve(ctx, F, B)
        return (F,)

    t_fp64, ts, (F,) = runs(fp64_once)
    ms_f64 = F.stats.ms_total
    progress("mxp comparison: FP64 factor + solve %s s" % ["%.2f" % t for t in ts])
    if probes:
        tc.export(ctx, F, out=storage)  # in place: zero strict upper parts
        out["fp64_probe_backward_error"] = probe_backward_error(A, storage, n, nb)
    F.close()
    del storage, F
    torch.cuda.empty_cache()
    out.update({"fp64_time_to_solution_s": t_fp64, "fp64_times_s": ts, "fp64_factor_ms": ms_f64,
                "fp64_tflops": flops / (ms_f64 * 1e-3) / 1e12})

    def mixed(e2, fp64_update, label):
        """map at e2 + factorization + refined solve to 1e-9, timed"""
        holder = {}

        def once():
            holder.pop("storage", None)
            cm = tc.precision_map(Nt, tf_h, fro, e2)
            holder["storage"] = storage = torch.empty(
                tc.factor_bytes(n, nb, cm, fp64_update) // 8, dtype=torch.float64, device=dev)
            F = tc.factorize(ctx, A, n, nb, cmap=cm, storage=storage, fp64_update=fp64_update)
            B.copy_(B0)
            st = tc.solve_refine(ctx, F, A, B, max_iter=30, tol=1e-9)
            return F, st

        t2, ts, (F, st) = runs(once)
        progress("mxp comparison: %s, refined to 1e-9: %s s" % (label, ["%.2f" % t for t in ts]))
        cf = list(F.stats.class_flops)
        r = {"map_eps": e2, "fp64_update": "fp64" if fp64_update == tc.FP64 else "fp32",
             "mxp_time_to_solution_s": t2, "mxp_times_s": ts, "mxp_factor_ms": F.stats.ms_total,
             "mxp_tflops_fp64_equivalent": flops / (F.stats.ms_total * 1e-3) / 1e12,
             "speedup_time_to_solution": t_fp64 / t2, "ir_iterations": st["iterations"],
             "ir_rel_residual": st["rel_residual"], "converged": st["converged"],
             "ir_ms": st["ms_total"],
             "class_tiles": dict(zip(CLASS_NAMES, list(F.stats.class_tiles))),
             "class_flop_share": dict(zip(CLASS_NAMES, [c / max(sum(cf), 1.0) for c in cf])),
             "map_roofline": map_roofline(n, cf, F.stats.ms_total)}
        if probes:
            L64 = torch.empty_like(A)
            tc.export(ctx, F, out=L64)
            r["probe_backward_error"] = probe_backward_error(A, L64, n, nb)
            del L64
        F.close()
        del F
        holder.clear()
        torch.cuda.empty_cache()
        return r

    # the paper's four-precision scheme: binary64 updates into FP64 tiles
    out.update(mixed(w["eps"], tc.FP64, "mixed map, binary64 updates into FP64 tiles"))
    out["roofline_frac"] = out["map_roofline"]["frac"]
    # the same map with the updates into its FP64 tiles (diagonal SYRK
    # included) in the FP32 class's arithmetic: binary64 arithmetic only in
    # POTRF, TRSM and the refinement residuals
    out["fp32_updates_same_map"] = mixed(w["eps"], tc.FP32, "same map, FP32 updates into FP64 tiles")
    # the same refined-solve target (1e-9) reached from looser maps
    out["looser_maps_same_residual_target"] = [mixed(e2, tc.FP64, "map at %g" % e2)
                                               for e2 in extra_eps]
    del A
    torch.cuda.empty_cache()
    return out


def grad_leg(tc, si, dev):
    """Log-likelihood and its gradient at n=32768, nb=512 (4000 base points
    translated, nu=1/2): forward = covariance tiles + factorization +
    log-likelihood seed; backward = reverse sweep + contraction with the
    covariance derivatives. The data y = L(theta0) z is made before timing."""
    import numpy as np
    import torch
    w = si.WORKLOADS["grad"]
    n, nb, nu = w["n"], w["nb"], w["nu"]
    pts = si.translated_points(n, w["base_points"], seed=w["seed"])
    locs = torch.from_numpy(pts).to(dev)
    ctx = tc.Context(n, nb, timed=True)
    A0, _, _ = tc.matern_tiles(ctx, locs, (w["sigma2"], w["range"], nu, w["nugget"]), nb,
                               norms=False)
    F0 = tc.factorize(ctx, A0, n, nb, inplace=True)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    # y = L z by tiles: input synthesis, outside the timed region
    z = torch.from_numpy(np.asarray(si.standard_normal(n, seed=si.rhs_seed(w["seed"])))).to(dev)
    Nt = n // nb
    y.zero_()
    for j in range(Nt):
        for i in range(j, Nt):
            t = tc.tile_offset(Nt, i, j)
            Lij = A0[t * nb * nb:(t + 1) * nb * nb].view(nb, nb).t()
            if i == j:
                Lij = torch.tril(Lij)
            y[i * nb:(i + 1) * nb] += Lij @ z[j * nb:(j + 1) * nb]
    F0.close()
    del A0
    torch.cuda.empty_cache()
    th = w["theta_eval"]
    full = (th[0], th[1], nu, th[2])
    Lbar = torch.empty(tc.num_tiles(n, nb) * nb * nb, dtype=torch.float64, device=dev)
    A = torch.empty_like(Lbar)
    # scratch of the full and the memory-short reverse sweep, for binary64
    # and for mixed-precision factors
    scr = {(m, sh): torch.empty((tc.adjoint_min_bytes if sh else tc.adjoint_bytes)(n, nb, m),
                                dtype=torch.uint8, device=dev)
           for m in (False, True) for sh in (False, True)}
    mixed_tiles = {}

    def once(mixed=False, short=False):
        if mixed:  # the FP32-mixed variant: {FP64, FP32} map at 1e-9 per evaluation
            _, tf, fro = tc.matern_tiles(ctx, locs, full, nb, out=A, norms=True)
            cm = tc.precision_map(n // nb, tf.cpu().numpy(), fro, 1e-9,
                                  allowed=(tc.FP64, tc.FP32))
            mixed_tiles.update(fp64=int(np.count_nonzero(cm == tc.FP64)),
                               fp32=int(np.count_nonzero(cm == tc.FP32)))
            F = tc.factorize(ctx, A, n, nb, cmap=cm)
        else:
            tc.matern_tiles(ctx, locs, full, nb, out=A, norms=False)
            F = tc.factorize(ctx, A, n, nb, inplace=True)
        ll = tc.loglik_seed(ctx, F, y, Lbar)
        st = tc.factor_adjoint(ctx, F, Lbar, scratch=scr[(mixed, short)])
        g = tc.matern_grad(ctx, locs, full, nb, Lbar)
        F.close()
        return ll, g, st

    def timed(mixed=False, short=False, reps=3):
        once(mixed, short)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ll, g, st = once(mixed, short)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, ll, g, st

    dt, ll, g, st = timed()
    fwd = n ** 3 / 3.0
    out = {"workload": "loglik + gradient, n=%d nb=%d, Matern nu=%g, 4000 base points translated, "
                       "theta=(%g, %g, %g)" % (n, nb, nu, th[0], th[1], th[2]),
           "s_per_eval": dt, "loglik": ll, "grad": [float(v) for v in g],
           "reverse_sweep_ms": st.ms_total, "reverse_sweep_flops": st.flops_total,
           "reverse_sweep_tflops": st.flops_total / (st.ms_total * 1e-3) / 1e12,
           "reverse_panel_tflops": (st.gemm_flops / (st.ms_gemm * 1e-3) / 1e12
                                    if st.ms_gemm > 0 else None),
           "forward_plus_reverse_tflops": (fwd + st.flops_total) / dt / 1e12,
           "scratch_bytes": tc.adjoint_bytes(n, nb)}
    # memory-short reverse sweep (no transposed copy of Abar): same gradient
    dts, lls, gs, sts = timed(short=True, reps=2)
    out["memory_short"] = {
        "s_per_eval": dts, "reverse_sweep_ms": sts.ms_total,
        "reverse_panel_tflops": (sts.gemm_flops / (sts.ms_gemm * 1e-3) / 1e12
                                 if sts.ms_gemm > 0 else None),
        "scratch_bytes": tc.adjoint_min_bytes(n, nb),
        "grad_equal_to_full_form": bool(np.array_equal(gs, g))}
    # FP32-mixed variant, full and memory-short sweeps
    dtm, llm, gm, stm = timed(mixed=True, reps=2)
    dtms, _, gms, stms = timed(mixed=True, short=True, reps=2)
    out["fp32_mixed"] = {
        "map": "{FP64, FP32} at target 1e-9 (Section IV-C)", "tiles": dict(mixed_tiles),
        "s_per_eval": dtm, "loglik": llm, "grad": [float(v) for v in gm],
        "grad_max_rel_diff_vs_fp64": float(np.max(np.abs(gm - g) / np.abs(g))),
        "reverse_sweep_ms": stm.ms_total, "scratch_bytes": tc.adjoint_bytes(n, nb, True),
        "memory_short": {"s_per_eval": dtms, "reverse_sweep_ms": stms.ms_total,
                         "scratch_bytes": tc.adjoint_min_bytes(n, nb, True),
                         "grad_equal_to_full_form": bool(np.array_equal(gms, gm))}}
    del A, Lbar, scr
    torch.cuda.empty_cache()
    return out


def ooc_leg(tc, si, dev, n=122880, nb=2048, caches_gib=(40, 16)):
    """Out-of-core FP64 factorization from pinned host memory against the
    in-core factorization of the same matrix. The ooc workload's parameters
    (nu=1, range=0.05, nugget=1e-4) at n=122880, nb=2048: 57.2 GiB of packed
    lower tiles in one pinned host buffer (the largest size whose pinned
    allocation succeeds on the test machines). Two HBM tile caches: 40 GiB
    holds the peak working set (~29 GiB: every tile crosses the link once
    each way) and 16 GiB does not (operand tiles are evicted and reloaded).
    Each run starts from a fresh copy of A in the pinned buffer (in place)."""
    import numpy as np
    import torch
    w = si.WORKLOADS["ooc"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = torch.from_numpy(si.points(n, seed=w["seed"])).to(dev)
    ctx = tc.Context(n, nb, timed=True)
    A, _, _ = tc.matern_tiles(ctx, pts, theta, nb, norms=False)
    Ah = torch.empty(A.numel(), dtype=torch.float64, pin_memory=True)
    storage = torch.empty_like(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = tc.factorize(ctx, A, n, nb, storage=storage)
    torch.cuda.synchronize()
    t_in = time.perf_counter() - t0
    F.close()
    flops = n ** 3 / 3.0
    Nt = n // nb
    nb2 = nb * nb
    out = {"workload": "ooc FP64 tile Cholesky, n=%d nb=%d, Matern nu=%g range=%g nugget=%g, "
                       "pinned host tiles" % (n, nb, theta[2], theta[1], theta[3]),
           "in_core_s": t_in, "in_core_tflops": flops / t_in / 1e12, "runs": []}
    for gib in caches_gib:
        Ah.copy_(A)
        cache = torch.empty(gib << 30, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = tc.factorize_ooc(ctx, Ah, n, nb, cache)
        t_ooc = time.perf_counter() - t0
        del cache
        torch.cuda.empty_cache()
        # sampled agreement with the in-core factor
        worst = 0.0
        for (i, j) in [(0, 0), (Nt - 1, 0), (Nt // 2, Nt // 3), (Nt - 1, Nt - 2), (Nt - 1, Nt - 1)]:
            t = tc.tile_offset(Nt, i, j)
            a = storage[t * nb2:(t + 1) * nb2].view(nb, nb).t().cpu().numpy()
            b = Ah[t * nb2:(t + 1) * nb2].view(nb, nb).t().numpy()
            if i == j:
                a, b = np.tril(a), np.tril(b)
            worst = max(worst, float(np.abs(a - b).max() / np.abs(a).max()))
        out["runs"].append({
            "cache_gib": gib, "cache_slots": st["cache_slots"], "ooc_s": t_ooc,
            "ooc_tflops": flops / t_ooc / 1e12, "ooc_over_in_core": t_ooc / t_in,
            "bytes_h2d": st["bytes_h2d"], "bytes_d2h": st["bytes_d2h"],
            "h2d_gbps": st["bytes_h2d"] / t_ooc / 1e9, "d2h_gbps": st["bytes_d2h"] / t_ooc / 1e9,
            "tiles_reloaded": st["tiles_reloaded"], "evictions": st["evictions"],
            "chunks": st["chunks"], "max_rel_diff_sampled_tiles": worst})
    del A, storage, Ah
    torch.cuda.empty_cache()
    torch._C._host_emptyCache()
    return out


IMAGE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2, 4: 1}


def decode_image_tile(img, cm, nb, t):
    """Tile t (binary64, column-major nb x nb) of an out-of-core mixed
    factor's host image: tiles in their classes on 256-byte boundaries,
    then one int32 scale exponent per tile."""
    import numpy as np
    nb2 = nb * nb
    sizes = [(nb2 * IMAGE_BYTES[int(c)] + 255) // 256 * 256 for c in cm]
    off = sum(sizes[:t])
    end = sum(sizes)
    raw = img.numpy()
    e = int(raw[end:end + 4 * len(cm)].view(np.int32)[t])
    c = int(cm[t])
    b = raw[off:off + nb2 * IMAGE_BYTES[c]]
    if c == 0:
        v = b.view(np.float64)
    elif c == 1:
        v = b.view(np.float32).astype(np.float64)
    elif c == 2:
        v = b.view(np.float16).astype(np.float64)
    elif c == 3:
        v = (b.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        ex, m = (b >> 3) & 15, (b & 7).astype(np.float64)
        v = np.where(ex == 0, m * 2.0 ** -9, (1 + m / 8) * np.ldexp(1.0, ex.astype(np.int64) - 7))
        v = np.where(b & 0x80, -v, v)
    return np.ldexp(v, e).reshape(nb, nb).T


def ooc_mixed_leg(tc, si, dev, n=90112, nb=2048, eps=1e-9, caches_gib=(40, 20)):
    """Out-of-core mixed-precision factorization against the in-core mixed
    factorization of the same matrix and map. The ooc workload's parameters
    (nu=1, range=0.05, nugget=1e-4) at n=90112, nb=2048, target 1e-9: A in
    one exact-size pinned host buffer (30.9 GiB, binary64), the factor image
    (tiles in their classes) in another; together they stay below the ~64
    GiB of pinned host memory the test machines grant one process. Two HBM
    caches: 40 GiB holds the peak working set of tile bundles, 20 GiB does
    not (the minimum at this size is 15.1 GiB)."""
    import numpy as np
    import torch
    w = si.WORKLOADS["ooc"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = torch.from_numpy(si.points(n, seed=w["seed"])).to(dev)
    ctx = tc.Context(n, nb, timed=True)
    A, norms, fro = tc.matern_tiles(ctx, pts, theta, nb, norms=True)
    Nt = n // nb
    cm = tc.precision_map(Nt, norms.cpu().numpy(), fro, eps)
    storage = torch.empty(tc.factor_bytes(n, nb, cm) // 8, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = tc.factorize(ctx, A, n, nb, cmap=cm, storage=storage)
    torch.cuda.synchronize()
    t_in = time.perf_counter() - t0
    progress("ooc mixed: in-core mixed factorization %.2f s" % t_in)
    samples = [(Nt - 1, 0), (Nt // 2, Nt // 3), (Nt - 1, Nt - 2), (Nt // 3, Nt // 3 - 1), (Nt - 1, Nt - 1)]
    nb2 = nb * nb
    L64 = torch.empty_like(A)
    tc.export(ctx, F, out=L64)
    ref = {ij: L64[tc.tile_offset(Nt, *ij) * nb2:(tc.tile_offset(Nt, *ij) + 1) * nb2].view(nb, nb).t().cpu().numpy()
           for ij in samples}
    F.close()
    del F, storage, L64
    # the same map with the updates into FP64 tiles in FP32-class arithmetic
    storage = torch.empty(tc.factor_bytes(n, nb, cm, tc.FP32) // 8, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = tc.factorize(ctx, A, n, nb, cmap=cm, storage=storage, fp64_update=tc.FP32)
    torch.cuda.synchronize()
    t_in32 = time.perf_counter() - t0
    progress("ooc mixed: in-core, FP32-class updates %.2f s" % t_in32)
    F.close()
    del F, storage
    torch.cuda.empty_cache()
    flops = n ** 3 / 3.0
    cls_bytes = {c: int(np.sum(cm == c)) * nb2 * IMAGE_BYTES[c] for c in IMAGE_BYTES}
    out = {"workload": "ooc mixed-precision tile Cholesky, n=%d nb=%d, Matern nu=%g range=%g "
                       "nugget=%g, target %g, pinned host tiles" % (n, nb, theta[2], theta[1], theta[3], eps),
           "class_tiles": {k: int(np.sum(cm == c)) for k, c in (("fp64", 0), ("fp32", 1), ("fp16", 2),
                                                              ("bf16", 3), ("fp8", 4))},
           "factor_host_bytes": sum(cls_bytes.values()), "factor_fp64_bytes": len(cm) * nb2 * 8,
           "in_core_s": t_in, "in_core_tflops_fp64_equivalent": flops / t_in / 1e12, "runs": []}
    torch._C._host_emptyCache()  # pinned blocks torch keeps cached from earlier legs
    Abuf = tc.PinnedBuffer(A.numel() * 8)
    Ah = Abuf.view(torch.float64)
    Ah.copy_(A)
    del A
    torch.cuda.empty_cache()
    Ibuf = tc.PinnedBuffer(tc.ooc_mixed_host_bytes(n, nb, cm))
    img = Ibuf.tensor
    for gib in caches_gib:
        cache = torch.empty(gib << 30, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = tc.factorize_ooc_mixed(ctx, Ah, n, nb, cm, cache, L_host=img)
        t_ooc = time.perf_counter() - t0
        del cache
        torch.cuda.empty_cache()
        progress("ooc mixed: %d GiB cache %.2f s" % (gib, t_ooc))
        worst = 0.0
        for ij in samples:
            a = ref[ij]
            b = decode_image_tile(img, cm, nb, tc.tile_offset(Nt, *ij))
            if ij[0] == ij[1]:
                a, b = np.tril(a), np.tril(b)
            worst = max(worst, float(np.abs(a - b).max() / np.abs(a).max()))
        out["runs"].append({
            "cache_gib": gib, "cache_slots": st["cache_slots"], "ooc_s": t_ooc,
            "ooc_tflops_fp64_equivalent": flops / t_ooc / 1e12, "ooc_over_in_core": t_ooc / t_in,
            "bytes_h2d": st["bytes_h2d"], "bytes_d2h": st["bytes_d2h"],
            "h2d_gbps": st["bytes_h2d"] / t_ooc / 1e9, "d2h_gbps": st["bytes_d2h"] / t_ooc / 1e9,
            "tiles_reloaded": st["tiles_reloaded"], "evictions": st["evictions"],
            "chunks": st["chunks"], "max_rel_diff_sampled_tiles_vs_in_core": worst})
    # FP32-class updates into FP64 tiles, largest cache
    gib = max(caches_gib)
    cache = torch.empty(gib << 30, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, _ = tc.factorize_ooc_mixed(ctx, Ah, n, nb, cm, cache, L_host=img, fp64_update=tc.FP32)
    t_ooc = time.perf_counter() - t0
    del cache
    torch.cuda.empty_cache()
    progress("ooc mixed: FP32-class updates, %d GiB cache %.2f s" % (gib, t_ooc))
    out["fp32_updates"] = {
        "in_core_s": t_in32, "cache_gib": gib, "cache_slots": st["cache_slots"], "ooc_s": t_ooc,
        "ooc_tflops_fp64_equivalent": flops / t_ooc / 1e12, "ooc_over_in_core": t_ooc / t_in32,
        "bytes_h2d": st["bytes_h2d"], "bytes_d2h": st["bytes_d2h"],
        "h2d_gbps": st["bytes_h2d"] / t_ooc / 1e9, "tiles_reloaded": st["tiles_reloaded"]}
    del Ah, img
    Abuf.close()
    Ibuf.close()
    return out


def kl_sweep(tc, si, dev, ns=(32768, 65536), nb=1024, betas=(0.02627, 0.078809, 0.210158),
             eps_list=(1e-5, 1e-6, 1e-7, 1e-8), nugget=1e-4, seed=3):
    """The paper's mixed-precision study (Section V): for the Matern fields
    theta = (1, beta, 1/2) at the three correlation levels and the target
    accuracies of its figures, the KL divergence of Eq. 3 at y = 0,
    D = l_0 - l_a = (log|Sigma_a| - log|Sigma_0|) / 2, with Sigma_0 factored
    in FP64 and Sigma_a in mixed precision, and the factorization rates
    (FP64-equivalent TFLOP/s, n^3/3 over the factorization time), for the
    updates into FP64 tiles in binary64 and in FP32-class arithmetic. A
    nugget of 1e-4 is added on the diagonal (the map is computed from the
    tile norms of the same matrix)."""
    import numpy as np
    import torch
    out = {"workload": "Matern nu=1/2 sigma2=1 nugget=%g, nb=%d, Z-ordered seeded points (seed %d)" % (nugget, nb, seed),
           "rows": []}
    for n in ns:
        Nt = n // nb
        pts = torch.from_numpy(si.points(n, seed=seed)).to(dev)
        ctx = tc.Context(n, nb)
        for beta in betas:
            A, tf, fro = tc.matern_tiles(ctx, pts, (1.0, beta, 0.5, nugget), nb)
            tf_h = tf.cpu().numpy()
            storage = torch.empty(tc.factor_bytes(n, nb) // 8, dtype=torch.float64, device=dev)
            F = tc.factorize(ctx, A, n, nb, storage=storage)
            ld0, ms0 = tc.logdet(ctx, F), F.stats.ms_total
            F.close()
            del storage, F
            torch.cuda.empty_cache()
            for eps in eps_list:
                cm = tc.precision_map(Nt, tf_h, fro, eps)
                storage = torch.empty(tc.factor_bytes(n, nb, cm) // 8, dtype=torch.float64, device=dev)
                row = {"n": n, "beta": beta, "eps": eps, "fp64_factor_ms": ms0,
                       "fp64_tflops": n ** 3 / 3.0 / ms0 / 1e9}
                try:
                    F = tc.factorize(ctx, A, n, nb, cmap=cm, storage=storage)
                    ld = tc.logdet(ctx, F)
                    ms = F.stats.ms_total
                    cf = list(F.stats.class_flops)
                    tot = sum(cf)
                    row.update({"kl": 0.5 * (ld - ld0), "mxp_factor_ms": ms,
                                "mxp_tflops_fp64_equivalent": n ** 3 / 3.0 / ms / 1e9,
                                "speedup_factor": ms0 / ms,
                                "flop_share": {k: cf[i] / tot for i, k in enumerate(("fp64", "fp32", "fp16", "bf16", "fp8"))}})
                    F.close()
                    del F
                except tc.NotPositiveDefinite as e:
                    row.update({"kl": None, "breakdown_column": e.info})
                del storage
                torch.cuda.empty_cache()
                # the same map with FP32-class updates into its FP64 tiles
                storage = torch.empty(tc.factor_bytes(n, nb, cm, tc.FP32) // 8, dtype=torch.float64,
                                      device=dev)
                try:
                    F = tc.factorize(ctx, A, n, nb, cmap=cm, storage=storage, fp64_update=tc.FP32)
                    ld = tc.logdet(ctx, F)
                    ms = F.stats.ms_total
                    row.update({"kl_fp32_updates": 0.5 * (ld - ld0), "fp32_updates_factor_ms": ms,
                                "fp32_updates_tflops_fp64_equivalent": n ** 3 / 3.0 / ms / 1e9,
                                "fp32_updates_speedup_factor": ms0 / ms})
                    F.close()
                    del F
                except tc.NotPositiveDefinite as e:
                    row.update({"kl_fp32_updates": None, "fp32_updates_breakdown_column": e.info})
                del storage
                torch.cuda.empty_cache()
                out["rows"].append(row)
                progress("kl sweep: n=%d beta=%g eps=%g kl=%s kl(FP32 updates)=%s" % (
                    n, beta, eps, row.get("kl"), row.get("kl_fp32_updates")))
            del A, tf
            torch.cuda.empty_cache()
    return out


def ooc_ablation(tc, si, dev, n=81920, nb=2048, cache_gib=40, small_gib=8):
    """The paper's comparison of out-of-core strategies (Section IV-B) on
    one MI355X, FP64, the ooc workload's parameters at n=81920, nb=2048, a
    40 GiB tile cache (holds the working set): the full schedule
    (asynchronous copies, resident accumulator V1, operand reuse V2,
    diagonal tile kept through the TRSMs V3), without V3 (the diagonal
    factor written back after POTRF and reloaded for each TRSM), without
    operand reuse across columns (V1 only), with every copy on the compute
    stream (no overlap), and the combinations; against the in-core
    factorization. Then, with an
    8 GiB cache (below the ~13 GiB peak working set), next-use eviction
    against least-recently-used eviction."""
    import torch
    w = si.WORKLOADS["ooc"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = torch.from_numpy(si.points(n, seed=w["seed"])).to(dev)
    ctx = tc.Context(n, nb)
    A, _, _ = tc.matern_tiles(ctx, pts, theta, nb, norms=False)
    storage = torch.empty_like(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = tc.factorize(ctx, A, n, nb, storage=storage)
    torch.cuda.synchronize()
    t_in = time.perf_counter() - t0
    F.close()
    del storage
    flops = n ** 3 / 3.0
    out = {"workload": "ooc FP64 tile Cholesky, n=%d nb=%d, Matern nu=%g range=%g nugget=%g"
                       % (n, nb, theta[2], theta[1], theta[3]),
           "in_core_s": t_in, "in_core_tflops": flops / t_in / 1e12, "variants": []}
    torch._C._host_emptyCache()
    Abuf = tc.PinnedBuffer(A.numel() * 8)
    Ah = Abuf.view(torch.float64)
    cache = torch.empty(cache_gib << 30, dtype=torch.uint8, device=dev)
    small = cache[:small_gib << 30]
    for name, sync, no_reuse, lru, no_v3, cbuf in (
            ("async, V1+V2+V3 (default)", False, False, False, False, cache),
            ("async, V1+V2 (no V3: diagonal tile reloaded per TRSM)", False, False, False, True, cache),
            ("async, V1 (no operand reuse)", False, True, False, False, cache),
            ("sync, V1+V2+V3", True, False, False, False, cache),
            ("sync, V1+V2 (no V3)", True, False, False, True, cache),
            ("sync, V1 (no operand reuse)", True, True, False, False, cache),
            ("%d GiB cache, next-use eviction (default)" % small_gib, False, False, False, False, small),
            ("%d GiB cache, LRU eviction" % small_gib, False, False, True, False, small)):
        Ah.copy_(A)
        c2 = tc.Context(n, nb, ooc_sync=sync, ooc_no_reuse=no_reuse, ooc_lru=lru, ooc_no_v3=no_v3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = tc.factorize_ooc(c2, Ah, n, nb, cbuf)
        t = time.perf_counter() - t0
        c2.close()
        progress("ooc ablation: %s %.2f s" % (name, t))
        out["variants"].append({"variant": name, "cache_gib": cbuf.numel() >> 30,
                                "cache_slots": st["cache_slots"], "ooc_s": t, "tflops": flops / t / 1e12,
                                "ooc_over_in_core": t / t_in, "bytes_h2d": st["bytes_h2d"],
                                "bytes_d2h": st["bytes_d2h"], "tiles_reloaded": st["tiles_reloaded"],
                                "evictions": st["evictions"], "h2d_gbps": st["bytes_h2d"] / t / 1e9})
    del cache, small, A, Ah
    torch.cuda.empty_cache()
    Abuf.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mxp", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-grad", action="store_true", help="skip the likelihood-gradient leg")
    ap.add_argument("--mxp-only", action="store_true",
                    help="only the mixed-precision comparison (for profiling)")
    ap.add_argument("--grad-only", action="store_true",
                    help="only the likelihood-gradient leg (for profiling)")
    ap.add_argument("--no-ooc", action="store_true", help="skip the out-of-core leg")
    ap.add_argument("--mxp-n", type=int, default=0,
                    help="order of the mixed-precision comparison (default: the mxp workload's)")
    ap.add_argument("--mxp-eps", type=float, default=0.0,
                    help="target accuracy of the comparison's precision map (default: the mxp "
                         "workload's 1e-9; the refinement target stays 1e-9)")
    ap.add_argument("--mxp-repeats", type=int, default=2,
                    help="timed runs per variant of the mixed-precision comparison")
    ap.add_argument("--mxp-warmup", type=int, default=1,
                    help="untimed runs per variant of the mixed-precision comparison")
    ap.add_argument("--pmc-copy-gib", type=int, default=0,
                    help="before the steps, copy this many GiB device to device (the calibration "
                         "copy for HBM byte counters)")
    ap.add_argument("--ooc-only", action="store_true", help="only the out-of-core leg")
    ap.add_argument("--ooc-mixed-only", action="store_true",
                    help="only the out-of-core mixed-precision leg")
    ap.add_argument("--no-ooc-mixed", action="store_true",
                    help="skip the out-of-core mixed-precision leg")
    ap.add_argument("--kl-sweep", action="store_true",
                    help="only the KL-divergence / rate sweep over beta and the target accuracy")
    ap.add_argument("--ooc-ablation", action="store_true",
                    help="only the comparison of out-of-core strategies (sync/async, V1/V2/V3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the tile Cholesky here runs on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2410_09819_amd as tc
    import seeded_inputs as si

    if not os.path.exists(tc.LIB_PATH):
        from paper_2410_09819_amd import build
        build.build()
    dev = torch.device("cuda", 0)
    if (args.mxp_only or args.grad_only or args.ooc_only or args.ooc_mixed_only or args.kl_sweep
            or args.ooc_ablation):
        if args.kl_sweep:
            res = kl_sweep(tc, si, dev)
        elif args.ooc_ablation:
            res = ooc_ablation(tc, si, dev)
        elif args.mxp_only:
            res = mxp_comparison(tc, si, dev, args.mxp_n or None, args.mxp_eps or None,
                                 extra_eps=(), repeats=args.mxp_repeats, warmup=args.mxp_warmup)
        elif args.grad_only:
            res = grad_leg(tc, si, dev)
        elif args.ooc_only:
            res = ooc_leg(tc, si, dev)
        else:
            res = ooc_mixed_leg(tc, si, dev)
        print(json.dumps(res), flush=True)
        return
    w = si.WORKLOADS[args.workload]
    n, nb = w["n"], w["nb"]
    nrhs = 16
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = torch.from_numpy(si.points(n, seed=w["seed"])).to(dev)
    ctx = tc.Context(n, nb, timed=True)
    A, _, _ = tc.matern_tiles(ctx, pts, theta, nb, norms=False)
    storage = torch.empty(tc.factor_bytes(n, nb) // 8, dtype=torch.float64, device=dev)
    B0 = torch.from_numpy(np.ascontiguousarray(
        si.standard_normal((n, nrhs), seed=si.rhs_seed(w["seed"])).T)).to(dev)
    B = torch.empty_like(B0)

    def step():
        F = tc.factorize(ctx, A, n, nb, storage=storage)
        ld = tc.logdet(ctx, F)
        B.copy_(B0)
        tc.solve(ctx, F, B)
        return F, ld

    if args.pmc_copy_gib > 0:
        src = torch.ones(args.pmc_copy_gib << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gemm_ms = gemm_flops = 0.0
    gemm_launches = 0
    fact_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        F, ld = step()
        st = F.stats
        gemm_ms += st.ms_gemm
        gemm_flops += st.gemm_flops
        gemm_launches += st.gemm_launches
        fact_ms += st.ms_total
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    flops = n ** 3 / 3.0
    value = flops / (ms_per_step * 1e-3) / 1e12
    achieved = gemm_flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fp64 tile Cholesky, n=%d nb=%d, Matern nu=%g range=%g nugget=%g, "
                               "factor + logdet + %d-RHS solve" % (n, nb, w["nu"], w["range"],
                                                                   w["nugget"], nrhs),
                   "n": n, "nb": nb, "nrhs": nrhs, "precision": "fp64"},
        "pct_fp64_peak": 100.0 * value / FP64_PEAK_TFLOPS,
        "ms_factor": fact_ms / args.steps,
        "factor_tflops": flops / (fact_ms / args.steps * 1e-3) / 1e12,
        "logdet": ld,
        "roofline": {
            "kernel": "panel_update_kernel<false> (FP64 MFMA panel GEMM+SYRK, bulk of each column)",
            "bound": "mfma",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": (achieved / FP64_PEAK_TFLOPS) if achieved else None,
            "traffic": panel_traffic(),
            "traffic_unit": "HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
            "launches_per_step": gemm_launches / args.steps,
            "avg_launch_ms": gemm_ms / max(gemm_launches, 1),
            "flops_per_launch": gemm_flops / max(gemm_launches, 1),
        },
        "cpu_baseline": None,
    }
    tc.export(ctx, F, out=storage)  # the factor in place, strict upper parts zero
    out["backward_error"] = {
        "probe": probe_backward_error(A, storage, n, nb), "bound": 1e-12,
        "definition": "||(A - L L^T) G||_F / ||A G||_F, 32 seeded N(0,1) probe columns, "
                      "last timed step's factor, outside the timed region"}
    F.close()
    del storage, A, F
    torch.cuda.empty_cache()
    out["mxp_vs_fp64"] = None if args.no_mxp else mxp_comparison(tc, si, dev)
    out["loglik_grad"] = None if args.no_grad else grad_leg(tc, si, dev)
    out["ooc_vs_in_core"] = None if args.no_ooc else ooc_leg(tc, si, dev)
    out["ooc_mixed_vs_in_core"] = None if args.no_ooc_mixed else ooc_mixed_leg(tc, si, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
