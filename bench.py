"""Benchmark of the MI355X PIPECG library.

Main line (the JSON ``value``): PIPECG iterations per second on the 3-D
7-point Poisson problem on a 128^3 grid (N = 2,097,152, nnz = 14,581,760),
Jacobi preconditioner, x* uniform in [-1, 1] (seed 1), b = A x*, x0 = 0,
FP64.  One step = one PIPECG iteration (fused vector updates + Jacobi + dot
products, then SpMV with the reduction and scalar recurrences); the timed
region is one ppcg_solve of exactly ``--steps`` fixed iterations, inputs
resident in device memory, bracketed by device synchronisation.

Beside it: effective HBM bandwidth from the algorithmic byte model, the
roofline of the dominant kernel (average launch time from HIP events inside
the library), the FP64 CPU oracle timed on a bounded sample of the same
workload, and extra legs for the other workloads (64^2 latency case, mixed
precision on the 27-point 160^3 problem, the 256-system batch, serving).
"""

import argparse
import hashlib
import statistics
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "PPCG iters/sec + effective HBM GB/s (% of peak); solves/sec, p50/p99 latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank space removed, so a
    comment edit does not invalidate the stored counter figures."""
    h = hashlib.sha256()
    for f in ("ppcg_kernels.hpp", "ppcg_internal.hpp", "ppcg_fused.hpp"):
        with open(os.path.join(ROOT, "paper_2105_06176_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    e = d.get(f"{kernel}|{workload}")
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def sync():
    import torch

    torch.cuda.synchronize()


# The 128^3 storage the autotuner picks in plain runs, pinned so that the
# counter runs (kernels serialized, where timing-based choices can flip)
# measure the kernels timed here: SELL, 16-bit column offsets, the one-byte
# table of the matrix's distinct values, and the single-launch iteration.
C2_FLAGS_NAMES = ("FLAG_SELL_COL16", "FLAG_SELL_VALUE_TABLE", "FLAG_ITER_FUSED")


def survey_bytes_per_iter(n, nnz, fused):
    """The byte model of one PIPECG iteration before any reformulation: CSR
    matrix (8-byte values, 4-byte columns, 4-byte row pointers) and 22 FP64
    vector streams (two launches: the update reads n z q s p x r u w m dinv and
    writes z q s p x r u w m, the SpMV reads m and writes n), or 20 when one
    launch keeps n in registers."""
    return 12.0 * nnz + 4.0 * (n + 1) + 8.0 * (20 if fused else 22) * n


def leg_c2(args, torch, ppcg, wl, oracle):
    A = wl.poisson3d(128)
    b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1))
    bd = torch.as_tensor(b).cuda()
    flags = 0
    for name in C2_FLAGS_NAMES:
        flags |= getattr(ppcg, name)
    K = args.steps
    S = ppcg.Solver(A, fixed_iters=K, spmv_format="sell", flags=flags)
    mi = S.matrix_info()
    fused = mi["iter_launches"] == 1
    log(f"128^3: format={mi['format']} sigma={mi['sell_sigma']} stored={mi['nnz_stored']} "
        f"col_bytes={mi['col_index_bytes']} value_bytes={mi['value_bytes']} launches/iter={mi['iter_launches']} "
        f"setup={mi['setup_ms']:.1f}ms")
    x = torch.empty_like(bd)
    # warm-up: W iterations as solves of the timed length, so the timed solve
    # replays graphs captured here (no capture inside the timed region)
    for _ in range(max(1, math.ceil(args.warmup / K))):
        S.solve(bd, out=x)
    sync()
    t0 = time.perf_counter()
    _, info = S.solve(bd, out=x)
    sync()
    dt = time.perf_counter() - t0
    assert info["iters"] == K, info
    ips = K / dt
    gbs = mi["bytes_per_iter"] * ips / 1e9
    log(f"128^3 fixed {K}: {dt * 1e3:.2f} ms, {ips:.0f} it/s, {gbs:.0f} GB/s")

    # steady state: the difference of two solve lengths cancels the per-solve
    # initialisation (2-3 SpMVs), the final true residual and the host polls
    def best_time(k, reps=3):
        S.set_options(fixed_iters=k)
        S.solve(bd, out=x)
        ts = []
        for _ in range(reps):
            sync()
            t = time.perf_counter()
            _, inf = S.solve(bd, out=x)
            sync()
            ts.append(time.perf_counter() - t)
            assert inf["iters"] == k, inf  # no early stop (breakdown past convergence)
        return min(ts)

    k1, k2 = 20, 520
    t1, t2 = best_time(k1), best_time(k2)
    steady = (t2 - t1) / (k2 - k1)
    overhead = t1 - k1 * steady
    sb = survey_bytes_per_iter(A.n, A.nnz, fused)
    steady_res = {"us_per_iter": round(steady * 1e6, 3), "iters_per_s": round(1 / steady, 1),
                  "effective_gbs": round(mi["bytes_per_iter"] / steady / 1e9, 1),
                  "pct_peak_hbm": round(100 * mi["bytes_per_iter"] / steady / 1e9 / PEAK_HBM_GBS, 2),
                  "effective_gbs_survey_bytes": round(sb / steady / 1e9, 1),
                  "per_solve_init_finalize_ms": round(overhead * 1e3, 4),
                  "method": f"(t({k2}) - t({k1})) / {k2 - k1}, best of 3 solves each"}
    log(f"128^3 steady: {steady_res}")
    # kernel durations (HIP events attached to each launch on the library's stream)
    ms_a, ms_b = S.time_kernels(bd, iters=100)
    if fused:
        kname, bytes_dom, ms_dom = "k_fused", mi["bytes_per_iter"], ms_a
        other = {}
    else:
        dom = "vma" if ms_a >= ms_b else "spmv"
        bytes_dom = mi["bytes_vma"] if dom == "vma" else mi["bytes_spmv"]
        ms_dom = ms_a if dom == "vma" else ms_b
        kname = "k_vma<double>" if dom == "vma" else "k_spmv<double,MODE_ITER>"
        ms_o = ms_b if dom == "vma" else ms_a
        other = {"other_kernel_us": round(ms_o * 1e3, 3),
                 "other_kernel_gbs": round((mi["bytes_spmv"] if dom == "vma" else mi["bytes_vma"]) /
                                           (ms_o * 1e-3) / 1e9, 1)}
    log(f"kernel avg: {kname} {ms_dom * 1e3:.2f} us")
    achieved = bytes_dom / (ms_dom * 1e-3) / 1e9
    traffic = measured_traffic(kname, "poisson3d_128")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "traffic_source": "profiles/traffic.json (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE of this kernel "
                              "source)" if traffic else None,
            "kernel": kname, "bytes_per_launch": bytes_dom, "avg_launch_us": round(ms_dom * 1e3, 3), **other}
    if fused:
        # The same kernel on the byte-heavy storage (8-byte values, 32-bit
        # columns; slower, more bytes): the fraction of the HBM peak the
        # iteration reaches when bytes rather than latency bound it.
        F = ppcg.Solver(A, fixed_iters=K, spmv_format="sell",
                        flags=ppcg.FLAG_SELL_COL32 | ppcg.FLAG_SELL_FULL_VALUES | ppcg.FLAG_ITER_FUSED)
        mf = F.matrix_info()
        msf, _ = F.time_kernels(bd, iters=100)
        F.close()
        af = mf["bytes_per_iter"] / (msf * 1e-3) / 1e9
        roof["same_kernel_8byte_values_32bit_columns"] = {
            "bytes_per_launch": mf["bytes_per_iter"], "avg_launch_us": round(msf * 1e3, 3),
            "achieved": round(af, 1), "frac": round(af / PEAK_HBM_GBS, 4)}
        log(f"k_fused with 8-byte values: {msf * 1e3:.2f} us, {af:.0f} GB/s")
        # ... and on the chunks' shared offset lists (no column stream)
        F = ppcg.Solver(A, fixed_iters=K, spmv_format="sell", flags=ppcg.FLAG_SELL_SHARED_OFFSETS |
                        ppcg.FLAG_SELL_VALUE_TABLE | ppcg.FLAG_ITER_FUSED)
        mf = F.matrix_info()
        msf, _ = F.time_kernels(bd, iters=100)
        F.close()
        af = mf["bytes_per_iter"] / (msf * 1e-3) / 1e9
        roof["same_kernel_shared_offset_lists"] = {
            "bytes_per_launch": mf["bytes_per_iter"], "avg_launch_us": round(msf * 1e3, 3),
            "achieved": round(af, 1), "frac": round(af / PEAK_HBM_GBS, 4)}
        log(f"k_fused on shared offset lists: {msf * 1e3:.2f} us, {af:.0f} GB/s")
    # tolerance run (after the fixed iterations; untimed in the main value)
    S.set_options(tol=1e-10, max_iter=10000)
    S.solve(bd)
    sync()
    t0 = time.perf_counter()
    xt, it = S.solve(bd)
    sync()
    ttol = time.perf_counter() - t0
    tol_run = {"iters": it["iters"], "status": it["status"], "rel_resid_true": it["rel_resid_true"],
               "time_s": round(ttol, 4), "restarts": it["restarts"]}
    log(f"128^3 to 1e-10: {it['iters']} iters, true rel resid {it['rel_resid_true']:.2e}, {ttol * 1e3:.1f} ms")
    res = {"ips": ips, "dt": dt, "gbs": gbs, "mi": mi, "roofline": roof, "tol_run": tol_run, "steady": steady_res,
           "bytes_survey": sb, "fused": fused}
    if args.cpu_baseline:
        k = args.cpu_iters
        t0 = time.perf_counter()
        ref = oracle.pipecg(A, b, fixed_iters=k)
        tc = time.perf_counter() - t0
        ncpu, model = cpu_info()
        # the paper's CPU baseline: PIPECG with OpenMP and merged loops, on
        # the host's cores (at most 16: the GPU's share of the host)
        th = min(oracle.omp_default_threads(), 16)
        ko = 5 * k
        t0 = time.perf_counter()
        xo, sto, ito = oracle.pipecg_openmp(A, b, fixed_iters=ko, threads=th)
        to = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(k / tc, 3), "unit": "iters/s", "cores": 1, "kind": "oracle",
                               "sample": f"FP64 C oracle (single thread), PIPECG {k} fixed iterations of the "
                                         f"128^3 7-point problem incl. its initialisation, {tc:.1f} s",
                               "host_cpus": ncpu, "host_cpu_model": model,
                               "openmp": {"value": round(ito / to, 3), "unit": "iters/s", "cores": th,
                                          "kind": "PIPECG-OpenMP (the paper's CPU baseline: merged update loops)",
                                          "sample": f"{ito} fixed iterations of the same problem incl. its "
                                                    f"initialisation, {to:.1f} s, {th} threads"}}
        # parity of the timed configuration on the same sample
        S.set_options(fixed_iters=k)
        xg, _ = S.solve(bd)
        res["parity_x_k"] = {"k": k, "rel_diff_vs_oracle": float(np.linalg.norm(xg.cpu().numpy() - ref.x) /
                                                                  np.linalg.norm(ref.x))}
        log(f"oracle {k} iters: {tc:.1f}s ({k / tc:.2f} it/s); OpenMP {th} threads {ito / to:.1f} it/s; "
            f"GPU/oracle x_{k} rel diff {res['parity_x_k']['rel_diff_vs_oracle']:.2e}")
    S.close()
    return res


def leg_c1(torch, ppcg, wl, oracle):
    A = wl.poisson2d(64)
    b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1))
    bd = torch.as_tensor(b).cuda()
    S = ppcg.Solver(A, tol=1e-8)
    S.solve(bd)
    ts = []
    for _ in range(7):
        sync()
        t0 = time.perf_counter()
        _, info = S.solve(bd)
        sync()
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    ref = oracle.pipecg(A, b, tol=1e-8)
    t0 = time.perf_counter()
    oracle.pipecg(A, b, tol=1e-8)
    tc = time.perf_counter() - t0
    return {"workload": "2D 5-point Poisson 64^2, tol 1e-8", "iters": info["iters"], "oracle_iters": ref.iters,
            "time_to_solution_ms": round(t * 1e3, 3), "us_per_iter": round(t / info["iters"] * 1e6, 2),
            "solves_per_s": round(1 / t, 1), "rel_resid_true": info["rel_resid_true"],
            "oracle_time_ms": round(tc * 1e3, 2)}


def leg_c3(torch, ppcg, wl):
    t0 = time.perf_counter()
    A = wl.stencil27_lognormal(160, seed=0, shift=1e-3)
    b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1))
    log(f"27-pt 160^3 generated: nnz={A.nnz} in {time.perf_counter() - t0:.1f}s")
    bd = torch.as_tensor(b).cuda()
    out = {"workload": "3D 27-point lognormal 160^3 (N=4096000), shift 1e-3, tol 1e-10", "nnz": A.nnz}
    xs = {}
    # "mixed": FP32 vectors and values (always iterated with Algorithm 1)
    variants = [("fp64", {}), ("mixed_values", {"precision": "mixed_values"}), ("mixed", {"precision": "mixed"}),
                ("pcg_fp64", {"method": "pcg"}), ("pcg_mixed_values", {"method": "pcg", "precision": "mixed_values"})]
    for label, kw in variants:
        S = ppcg.Solver(A, tol=1e-10, max_iter=20000, spmv_format="sell", **kw)
        S.solve(bd)  # warm-up (graph capture, FP32 copy)
        sync()
        t0 = time.perf_counter()
        x, info = S.solve(bd)
        sync()
        t = time.perf_counter() - t0
        xs[label] = x.cpu().numpy()
        out[label] = {"status": info["status"], "method": ["pipecg", "pcg"][info["method"]],
                      "iters": info["iters"], "outer": info["outer_iters"],
                      "restarts": info["restarts"], "rel_resid_true": info["rel_resid_true"],
                      "time_s": round(t, 4), "solves_per_s": round(1 / t, 3)}
        log(f"27-pt {label}: {info}")
        S.close()
    for label, _ in variants[1:]:
        out[label]["solution_rel_diff_vs_fp64"] = float(np.linalg.norm(xs[label] - xs["fp64"]) /
                                                        np.linalg.norm(xs["fp64"]))
        out[label]["speedup_vs_fp64"] = round(out["fp64"]["time_s"] / out[label]["time_s"], 3)
    # against the FP64 oracle's own solve to 1e-10 (sampled entries written by
    # tests/golden/make_c3_p125_reference.py from the oracle alone)
    gold = os.path.join(ROOT, "tests", "golden", "c3_stencil27_160_tol.txt")
    if os.path.exists(gold):
        idx, ref = [], []
        with open(gold) as f:
            for line in f:
                p = line.split()
                if len(p) == 3 and p[0] == "x_tol":
                    idx.append(int(p[1]))
                    ref.append(float(p[2]))
        idx, ref = np.array(idx), np.array(ref)
        for label, _ in variants:
            out[label]["sampled_rel_diff_vs_oracle_solution"] = float(np.linalg.norm(xs[label][idx] - ref) /
                                                                      np.linalg.norm(ref))
        out["oracle_solution"] = {"source": "tests/golden/c3_stencil27_160_tol.txt (oracle PIPECG to 1e-10, "
                                            f"{len(idx)} sampled entries)",
                                  "note": "any x with true relative residual <= 1e-10 is a correct result; "
                                          "two such solutions differ by up to about kappa * 1e-10"}
    return out


def leg_pcg(torch, ppcg, wl, iters=500):
    """Algorithm 1 (classic PCG) beside Algorithm 2 (PIPECG) on the 128^3
    7-point problem: fixed-iteration rate, kernel durations against their
    byte models, and the solve to 1e-10."""
    A = wl.poisson3d(128)
    b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1))
    bd = torch.as_tensor(b).cuda()
    out = {"workload": "3D 7-point Poisson 128^3, FP64, fixed iterations and tol 1e-10"}
    # PIPECG in the autotuned storage and form, and forced to two launches
    # per iteration (the form whose update and SpMV kernels compare with PCG's)
    for label, method, flags in (("pcg", "pcg", 0), ("pipecg", "pipecg", 0),
                                 ("pipecg_two_launch", "pipecg", ppcg.FLAG_ITER_TWO_LAUNCH)):
        S = ppcg.Solver(A, fixed_iters=20, method=method, flags=flags)
        x = torch.empty_like(bd)
        S.solve(bd, out=x)
        S.set_options(fixed_iters=iters, method=method)
        sync()
        t0 = time.perf_counter()
        _, info = S.solve(bd, out=x)
        sync()
        dt = time.perf_counter() - t0
        assert info["iters"] == iters, info
        mi = S.matrix_info()
        ms_a, ms_b = S.time_kernels(bd, iters=100)
        S.set_options(tol=1e-10, max_iter=10000, method=method)
        S.solve(bd)
        sync()
        t0 = time.perf_counter()
        _, it = S.solve(bd)
        sync()
        ttol = time.perf_counter() - t0
        rec = {"iters_per_s": round(iters / dt, 1), "us_per_iter": round(dt / iters * 1e6, 2),
               "bytes_per_iter": mi["bytes_per_iter"], "launches_per_iter": mi["iter_launches"],
               "value_bytes": mi["value_bytes"], "col_index_bytes": mi["col_index_bytes"],
               "effective_gbs": round(mi["bytes_per_iter"] * iters / dt / 1e9, 1)}
        if method == "pipecg" and mi["iter_launches"] == 1:
            rec.update({"iteration_kernel_us": round(ms_a * 1e3, 2),
                        "iteration_kernel_gbs": round(mi["bytes_per_iter"] / (ms_a * 1e-3) / 1e9, 1)})
        else:
            rec.update({"update_kernel_us": round(ms_a * 1e3, 2),
                        "update_kernel_gbs": round(mi["bytes_vma"] / (ms_a * 1e-3) / 1e9, 1),
                        "spmv_kernel_us": round(ms_b * 1e3, 2),
                        "spmv_kernel_gbs": round(mi["bytes_spmv"] / (ms_b * 1e-3) / 1e9, 1)})
        rec.update({"tol_iters": it["iters"], "tol_status": it["status"],
                    "tol_rel_resid_true": it["rel_resid_true"], "tol_time_s": round(ttol, 4)})
        out[label] = rec
        log(f"{label}: {out[label]}")
        S.close()
    out["pipecg_over_pcg_time_per_iter"] = round(out["pipecg"]["us_per_iter"] / out["pcg"]["us_per_iter"], 3)
    return out


def leg_shard(torch, ppcg, wl, parts=8):
    """2-D decomposition (Section IV-C) of the 128^3 7-point matrix into
    equal-speed row slabs: one slab's SpMV part 1 (local columns), halo
    gather and part 2 (remote columns) on this GPU, beside the unsplit SpMV."""
    A = wl.poisson3d(128)
    x = wl.xstar_uniform(A.n, 1)
    xg = torch.as_tensor(x).cuda()
    b = ppcg.split_rows(A.rp, [1.0] * parts)
    k = parts // 2 - 1  # an interior slab: two halo planes
    lo, hi = b[k], b[k + 1]
    S = ppcg.Shard(A, lo, hi)
    info = S.info()
    xl = xg[lo:hi].contiguous()
    xh = torch.empty(max(info["halo"], 1), dtype=torch.float64, device="cuda")
    y = torch.empty(hi - lo, dtype=torch.float64, device="cuda")
    S.time(xg, xl, xh, y, iters=5)
    ms1, msg, ms2 = S.time(xg, xl, xh, y, iters=100)
    # two launches per iteration, so that the SpMV is a kernel of its own
    full = ppcg.Solver(A, spmv_format="sell", flags=ppcg.FLAG_ITER_TWO_LAUNCH)
    _, ms_spmv = full.time_kernels(xg, iters=50)
    full.close()
    S.close()
    link = 153e9  # bytes/s of one xGMI link (per direction), the exchange a real split would make
    out = {"workload": f"3D 7-point Poisson 128^3 split into {parts} equal row slabs; slab {k}",
           "rows": hi - lo, "nnz_local": info["nnz_local"], "nnz_remote": info["nnz_remote"],
           "halo": info["halo"], "halo_bytes": info["halo_bytes"],
           "part1_us": round(ms1 * 1e3, 2), "part1_gbs": round(info["bytes_part1"] / (ms1 * 1e-3) / 1e9, 1),
           "gather_us": round(msg * 1e3, 2), "part2_us": round(ms2 * 1e3, 2),
           "unsplit_spmv_us_whole_matrix": round(ms_spmv * 1e3, 2),
           "unsplit_spmv_us_per_slab": round(ms_spmv * 1e3 / parts, 2),
           "halo_transfer_us_one_xgmi_link": round(info["halo_bytes"] / link * 1e6, 2)}
    return out


def leg_hybrid(torch, ppcg, wl, iters=200, threads=8):
    """Host cores + GPU together (Section IV) on the 128^3 7-point problem:
    Hybrid-PIPECG-3 with the performance model's split and forced splits,
    Hybrid-PIPECG-1 and -2 (task parallel, every row on the GPU), and, on a
    32^3 problem where the paper found the task-parallel schemes best, all
    three beside the GPU-only solver."""

    def run(A, b, label, dst, **kw):
        H = ppcg.Hybrid(A, host_threads=threads, fixed_iters=20, **kw)
        H.solve(b)
        H.close()
        H = ppcg.Hybrid(A, host_threads=threads, fixed_iters=iters, **kw)
        t0 = time.perf_counter()
        x, info = H.solve(b)
        dt = time.perf_counter() - t0
        hi = H.info()
        dst[label] = {"iters_per_s": round(iters / dt, 1), "us_per_iter": round(dt / iters * 1e6, 1),
                      "scheme": hi["scheme"], "n_cpu": hi["n_cpu"], "n_gpu": hi["n_gpu"],
                      "t_cpu_spmv_ms": round(hi["t_cpu_spmv_ms"], 3), "t_gpu_spmv_ms": round(hi["t_gpu_spmv_ms"], 4),
                      "copy_bytes_per_iter": hi["copy_bytes_per_iter"]}
        log(f"hybrid {label}: {dst[label]}")
        H.close()

    A = wl.poisson3d(128)
    b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1))
    out = {"workload": f"3D 7-point Poisson 128^3 (and 32^3), FP64, {iters} fixed iterations, {threads} host threads"}
    for label, share in (("model", -1.0), ("share_0.02", 0.02), ("share_0", 0.0)):
        run(A, b, label, out, cpu_share=share)
    for scheme in (1, 2):
        run(A, b, f"scheme{scheme}", out, scheme=scheme)
    A = wl.poisson3d(32)
    b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1))
    small = {}
    for scheme in (1, 2, 3):
        run(A, b, f"scheme{scheme}", small, scheme=scheme)
    S = ppcg.Solver(A, fixed_iters=iters)
    bd = torch.as_tensor(b).cuda()
    S.solve(bd)
    sync()
    t0 = time.perf_counter()
    S.solve(bd)
    sync()
    dt = time.perf_counter() - t0
    small["gpu_engine"] = {"iters_per_s": round(iters / dt, 1), "us_per_iter": round(dt / iters * 1e6, 1)}
    S.close()
    out["poisson3d_32"] = small
    return out


def leg_c4(torch, ppcg, wl, count=256):
    spec = wl.batch_c4(seed=0, count=count)
    t0 = time.perf_counter()
    mats = [wl.shifted(wl.poisson2d(side), sh) for side, sh in spec]
    bs = [torch.as_tensor(wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1000 + i))).cuda()
          for i, A in enumerate(mats)]
    log(f"batch generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    solvers = [ppcg.Solver(A, tol=1e-10, spmv_format="sell") for A in mats]
    setup = time.perf_counter() - t0
    # sequential solo solves (warm: graph capture per handle excluded by a first pass)
    for S, b in zip(solvers, bs):
        S.solve(b)
    sync()
    t0 = time.perf_counter()
    seq_iters = 0
    for S, b in zip(solvers, bs):
        _, info = S.solve(b)
        seq_iters += info["iters"]
    sync()
    t_seq = time.perf_counter() - t0
    ppcg.solve_batch(solvers, bs)  # warm-up
    # three timed batches: the median is reported, the best beside it
    tb = []
    for _ in range(3):
        sync()
        t0 = time.perf_counter()
        xs, infos = ppcg.solve_batch(solvers, bs)
        sync()
        tb.append(time.perf_counter() - t0)
    t_batch = statistics.median(tb)
    ok = sum(1 for i in infos if i["status"] == 0 and i["rel_resid_true"] <= 1e-10)
    bytes_total = sum(S.matrix_info()["bytes_per_iter"] * i["iters"] for S, i in zip(solvers, infos))
    for S in solvers:
        S.close()
    return {"workload": f"{count} shifted 2D 5-point Poisson systems, side U[32,512], shift U[0,0.5), tol 1e-10",
            "sum_n": int(sum(A.n for A in mats)), "sum_nnz": int(sum(A.nnz for A in mats)),
            "batched_solves_per_s": round(count / t_batch, 2), "batched_solves_per_s_best_of_3": round(count / min(tb), 2),
            "sequential_solves_per_s": round(count / t_seq, 2),
            "batch_speedup": round(t_seq / t_batch, 3), "batch_time_s": round(t_batch, 4),
            "sequential_time_s": round(t_seq, 4), "converged": ok, "total_iters": int(sum(i["iters"] for i in infos)),
            "algorithmic_gbs": round(bytes_total / t_batch / 1e9, 1), "setup_s": round(setup, 2)}


def leg_p125(torch, ppcg, wl, side=165):
    """The paper's 125-point Poisson matrices (Table 2: 4.5M rows at side 165)
    under its protocol (Section VI): x* = 1/sqrt(N), b = A x*, absolute
    tolerance 1e-5 on sqrt((u,u)), at most 10000 iterations."""
    t0 = time.perf_counter()
    A = wl.poisson125(side)
    b = wl.rhs_from_solution(A, wl.xstar_paper(A.n))
    gen_s = time.perf_counter() - t0
    log(f"125-pt side {side}: N={A.n} nnz={A.nnz} generated in {gen_s:.1f}s")
    bd = torch.as_tensor(b).cuda()
    out = {"workload": f"125-point Poisson side {side} (Table 2), paper protocol: x*=1/sqrt(N), "
                       "absolute tol 1e-5 on sqrt((u,u)), maxit 10000", "n": A.n, "nnz": A.nnz}
    del b
    # FP64 with the autotuned storage (a one-byte value table when timed
    # faster), FP64 with the 8-byte values forced, FP32 values
    for label, prec, flags in (("fp64", "fp64", 0), ("fp64_full_values", "fp64", ppcg.FLAG_SELL_FULL_VALUES),
                               ("mixed_values", "mixed_values", 0)):
        S = ppcg.Solver(A, tol=1e-5, stop="abs", max_iter=10000, precision=prec, flags=flags)
        mi = S.matrix_info()
        S.solve(bd)
        sync()
        t0 = time.perf_counter()
        _, info = S.solve(bd)
        sync()
        t = time.perf_counter() - t0
        out[label] = {"status": info["status"], "iters": info["iters"], "time_s": round(t, 4),
                      "ms_per_iter": round(t / max(info["iters"], 1) * 1e3, 4),
                      "algorithmic_gbs": round(mi["bytes_per_iter"] * info["iters"] / t / 1e9, 1),
                      "precond_norm": info["precond_norm"], "rel_resid_true": info["rel_resid_true"],
                      "spmv_format": mi["format"], "lanes_per_row": mi["lanes_per_row"],
                      "sell_sigma": mi["sell_sigma"], "iter_launches": mi["iter_launches"],
                      "col_index_bytes": mi["col_index_bytes"], "value_bytes": mi["value_bytes"],
                      "distinct_values": mi["distinct_values"], "setup_ms": round(mi["setup_ms"], 1)}
        log(f"125-pt {label}: {out[label]}")
        S.close()
    return out


def leg_rspd(torch, ppcg, wl, oracle, iters=20, shapes=("rspd_4.1M", "offshore", "serena")):
    """Random sparse SPD matrices (uniform random columns, values U[-1,0),
    diagonally dominant by 1e-2): N = 4.1M at ~17 entries per row, and
    stand-ins with the N and nnz/N of Table 1's offshore and Serena matrices
    (Section VI-A; the matrices themselves are not used).  These systems
    converge to 1e-10 in about 25 iterations and pipelined CG breaks down
    near 40, so the rate is taken over 20 fixed iterations (checked to have
    run), beside the solve to 1e-10.  With the autotuned storage and
    iteration form: algorithmic GB/s, the SpMV's fraction of the HBM peak,
    and the full-size SpMV against the oracle bit for bit."""
    cases = {"rspd_4.1M": (4_096_000, 8, 0), "offshore": (259_789, 8, 1), "serena": (1_391_349, 23, 2),
             "queen": (4_147_110, 39, 3)}
    out = {"workload": f"random SPD (R14 generator), PIPECG FP64, {iters} fixed iterations, autotuned storage"}
    for name in shapes:
        n, draws, seed = cases[name]
        t0 = time.perf_counter()
        A = wl.random_spd(n, seed=seed, draws=draws)
        gen_s = time.perf_counter() - t0
        b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 1))
        bd = torch.as_tensor(b).cuda()
        S = ppcg.Solver(A, fixed_iters=iters)
        mi = S.matrix_info()
        x = torch.empty_like(bd)
        S.solve(bd, out=x)
        sync()
        t0 = time.perf_counter()
        _, info = S.solve(bd, out=x)
        sync()
        dt = time.perf_counter() - t0
        assert info["status"] == ppcg.OK and info["iters"] == iters, info
        S.set_options(tol=1e-10)
        S.solve(bd, out=x)
        sync()
        t0 = time.perf_counter()
        _, it = S.solve(bd, out=x)
        sync()
        ttol = time.perf_counter() - t0
        S.set_options(fixed_iters=iters)
        # the SpMV alone (two-launch kernels on the same storage) and the
        # iteration's kernels as the handle runs them
        xs = wl.xstar_uniform(A.n, 5)
        exact = bool(np.array_equal(S.spmv(torch.as_tensor(xs).cuda()).cpu().numpy(), oracle.spmv(A, xs)))
        T = ppcg.Solver(A, flags=ppcg.FLAG_ITER_TWO_LAUNCH)
        ms_vma, ms_spmv = T.time_kernels(bd, iters=30)
        mt = T.matrix_info()
        T.close()
        ms_a, _ = S.time_kernels(bd, iters=30)
        spmv_gbs = mt["bytes_spmv"] / (ms_spmv * 1e-3) / 1e9
        out[name] = {"n": A.n, "nnz": A.nnz, "nnz_per_row": round(A.nnz / A.n, 2), "generated_s": round(gen_s, 1),
                     "iters_per_s": round(iters / dt, 1), "us_per_iter": round(dt / iters * 1e6, 2),
                     "bytes_per_iter": mi["bytes_per_iter"],
                     "effective_gbs": round(mi["bytes_per_iter"] * iters / dt / 1e9, 1),
                     "launches_per_iter": mi["iter_launches"], "spmv_format": mi["format"],
                     "sell_sigma": mi["sell_sigma"], "lanes_per_row": mi["lanes_per_row"],
                     "nnz_stored": mi["nnz_stored"], "col_index_bytes": mi["col_index_bytes"],
                     "setup_ms": round(mi["setup_ms"], 1),
                     "spmv_kernel_us": round(ms_spmv * 1e3, 2), "spmv_kernel_gbs": round(spmv_gbs, 1),
                     "spmv_frac_of_peak": round(spmv_gbs / PEAK_HBM_GBS, 4),
                     "update_kernel_us": round(ms_vma * 1e3, 2),
                     "iteration_kernel_us": round(ms_a * 1e3, 2) if mi["iter_launches"] == 1 else None,
                     "spmv_bitwise_vs_oracle": exact,
                     "tol_1e-10": {"iters": it["iters"], "status": it["status"], "time_ms": round(ttol * 1e3, 3),
                                   "rel_resid_true": it["rel_resid_true"], "restarts": it["restarts"]}}
        log(f"random SPD {name}: {out[name]}")
        S.close()
        del A, b, bd, x
    return out


def _serve_requests(wl, n_req, seed=0, pool=0):
    """n_req requests; with pool > 0, drawn uniformly from pool distinct ones
    (same kind, size and tolerance distribution, far less host memory)."""
    if pool and pool < n_req:
        base = _serve_requests(wl, pool, seed)
        pick = np.random.default_rng(seed + 1).integers(pool, size=n_req)
        return [base[k] for k in pick]
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        kind = rng.choice(3, p=[0.4, 0.3, 0.3])
        N = float(np.exp(rng.uniform(math.log(1e3), math.log(4e6))))
        tol = float(rng.choice([1e-6, 1e-8, 1e-10]))
        if kind == 0:
            A = wl.poisson2d(max(8, int(round(math.sqrt(N)))))
        elif kind == 1:
            A = wl.poisson3d(max(4, int(round(N ** (1 / 3)))))
        else:
            A = wl.random_spd(max(64, int(N)), seed=int(rng.integers(1 << 30)))
        b = wl.rhs_from_solution(A, wl.xstar_uniform(A.n, 2000 + i))
        reqs.append((A, b, tol, "auto"))  # the server picks FP64 or FP32 values per request
    return reqs


def _run_server(ppcg, reqs, arrivals, depth=None):
    """Serve reqs arriving at the given times; returns the total time and the
    latencies.  depth (a dict), when given, receives the mean and largest
    queued and active counts seen after the steps."""
    srv = ppcg.Server(borrow=True)  # requests reference the generated arrays (no host copy)
    t0 = time.perf_counter()
    i = 0
    pending = {}
    lat = []
    qs, acts = [], []
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and arrivals[i] <= now:
            A, b, tol, prec = reqs[i]
            pending[srv.submit(A, b, tol, prec)] = arrivals[i]
            i += 1
        if pending:
            active, queued = srv.step()
            qs.append(queued)
            acts.append(active)
            # poll only when some request finished and is not yet fetched
            if len(pending) > active + queued:
                for rid in list(pending):
                    r = srv.poll(rid)
                    if r is not None:
                        lat.append(time.perf_counter() - t0 - pending.pop(rid))
        elif i < len(reqs):
            time.sleep(max(0.0, min(0.01, arrivals[i] - now)))
    total = time.perf_counter() - t0
    srv.close()
    if depth is not None and qs:
        depth.update({"queue_mean": round(float(np.mean(qs)), 1), "queue_max": int(max(qs)),
                      "active_mean": round(float(np.mean(acts)), 1), "active_max": int(max(acts))})
    return total, np.array(lat)


def leg_c5(ppcg, wl, n_req, loads=(0.5, 0.8, 1.0, 1.2), pool=0):
    """Serving: Poisson arrivals of n_req requests (drawn from `pool`
    distinct ones when pool > 0) at each load, as fractions of the measured
    saturation rate.  The per-precision and sequential comparisons run over
    the distinct requests."""
    t0 = time.perf_counter()
    reqs = _serve_requests(wl, n_req, pool=pool)
    log(f"serving: {n_req} requests ({pool or n_req} distinct) generated in {time.perf_counter() - t0:.1f}s")
    # warm-up over the stream's distinct requests: every variant below then
    # finds the SpMV autotuner's choices cached for its matrix signatures
    uniq = list({id(r[0]): r for r in reqs}.values())
    _run_server(ppcg, uniq, np.zeros(len(uniq)))
    sat_depth = {}
    total, lat = _run_server(ppcg, reqs, np.zeros(n_req), sat_depth)  # saturation: all at t = 0
    sat = n_req / total
    log(f"serving at saturation: {sat:.2f} solves/s, {sat_depth}")
    nu = len(uniq)
    total_u, _ = _run_server(ppcg, uniq, np.zeros(nu))
    # the distinct requests with every one in plain FP64, and with FP32 values
    total64, _ = _run_server(ppcg, [(A, b, tol, "fp64") for A, b, tol, _ in uniq], np.zeros(nu))
    log(f"serving, every request in FP64: {nu / total64:.2f} solves/s")
    total32, _ = _run_server(ppcg, [(A, b, tol, "mixed_values") for A, b, tol, _ in uniq], np.zeros(nu))
    log(f"serving, every request with FP32 values: {nu / total32:.2f} solves/s")
    # plain FP64 PPCG one request after another (a solver per request)
    t0 = time.perf_counter()
    import torch

    for A, b, tol, _ in uniq:
        S = ppcg.Solver(A, tol=tol, vec_mem="host")
        S.solve(torch.as_tensor(b), out=torch.empty(A.n, dtype=torch.float64))
        S.close()
    t_seq = time.perf_counter() - t0
    log(f"sequential FP64 solves: {nu / t_seq:.2f} solves/s")
    out = {"workload": f"{n_req} requests ({nu} distinct): 40% 2D 5-pt, 30% 3D 7-pt, 30% random SPD, "
                       "N log-uniform [1e3,4e6], "
                       "tol {1e-6,1e-8,1e-10}; precision chosen by the server (FP32 classic PCG with FP64 "
                       "reliable updates for >= 262144 rows, FP32 values with FP64 reliable updates "
                       "for >= 65536 rows, else FP64)",
           "saturation_solves_per_s": round(sat, 2),
           "distinct_requests": nu,
           "distinct_saturation_solves_per_s": round(nu / total_u, 2),
           "distinct_saturation_solves_per_s_all_fp64": round(nu / total64, 2),
           "distinct_saturation_solves_per_s_all_fp32_values": round(nu / total32, 2),
           "distinct_sequential_fp64_solves_per_s": round(nu / t_seq, 2),
           "served_over_sequential_fp64": round(t_seq / total_u, 3), "saturation_depth": sat_depth}
    rng = np.random.default_rng(0)
    for frac in loads:
        lam = frac * sat
        arr = np.cumsum(rng.exponential(1 / lam, size=n_req))
        depth = {}
        total, lat = _run_server(ppcg, reqs, arr, depth)
        out[f"load_{frac}"] = {"rate_per_s": round(lam, 2), "solves_per_s": round(n_req / total, 2),
                               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2), **depth}
        log(f"serving at {frac} x saturation: {out[f'load_{frac}']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--legs", default="c1,c3,c4,c5,p125,rspd,pcg,shard,hybrid",
                    help="extra legs: c1,c3,c4,c5,p125,rspd,rspd_queen,pcg,shard,hybrid or none")
    ap.add_argument("--serve-requests", type=int, default=800)
    ap.add_argument("--serve-pool", type=int, default=200,
                    help="draw the serving requests from this many distinct ones (0: all distinct)")
    ap.add_argument("--serve-loads", default="0.5,0.8,1.0,1.2",
                    help="arrival rates as fractions of the measured saturation rate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of 256 MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this library runs on one GPU; multi-GPU runs are not supported "
              "(only the per-unit row split and shard SpMV exist, measured by the 'shard' leg).", file=sys.stderr)
        sys.exit(2)
    import torch

    import oracle
    import workloads as wl
    from paper_2105_06176_amd import ppcg

    ppcg.lib()
    torch.cuda.set_device(0)
    log(f"device: {torch.cuda.get_device_name(0)}")
    copy_gbs = None
    if args.copy_calibration:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        sync()
        t0 = time.perf_counter()
        for _ in range(10):
            c.copy_(a)
        sync()
        copy_gbs = 2 * a.numel() * 8 * 10 / (time.perf_counter() - t0) / 1e9
        log(f"copy calibration: 256 MiB copies at {copy_gbs:.0f} GB/s")
        del a, c
    c2 = leg_c2(args, torch, ppcg, wl, oracle)
    legs = {}
    wanted = [x for x in args.legs.split(",") if x and x != "none"]
    for name in wanted:
        t0 = time.perf_counter()
        try:
            if name == "c1":
                legs[name] = leg_c1(torch, ppcg, wl, oracle)
            elif name == "c3":
                legs[name] = leg_c3(torch, ppcg, wl)
            elif name == "pcg":
                legs[name] = leg_pcg(torch, ppcg, wl)
            elif name == "shard":
                legs[name] = leg_shard(torch, ppcg, wl)
            elif name == "hybrid":
                legs[name] = leg_hybrid(torch, ppcg, wl)
            elif name == "c4":
                legs[name] = leg_c4(torch, ppcg, wl)
            elif name == "c5":
                legs[name] = leg_c5(ppcg, wl, args.serve_requests,
                                    tuple(float(v) for v in args.serve_loads.split(",") if v), args.serve_pool)
            elif name == "p125":
                legs[name] = leg_p125(torch, ppcg, wl)
            elif name == "rspd":
                legs[name] = leg_rspd(torch, ppcg, wl, oracle)
            elif name == "rspd_queen":
                legs[name] = leg_rspd(torch, ppcg, wl, oracle, shapes=("queen",))
        except Exception as e:  # a failing extra leg must not hide the main line
            legs[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"leg {name} done in {time.perf_counter() - t0:.1f}s: {legs[name]}")
    mi = c2["mi"]
    line = {
        "metric": METRIC, "value": round(c2["ips"], 2), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(c2["dt"] / args.steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "PIPECG, 3D 7-point Poisson 128^3 (N=2097152, nnz=14581760), Jacobi, "
                               "x*~U[-1,1] seed 1, b=A x*, x0=0, one solve of --steps fixed iterations, FP64",
                   "n": mi["n"], "nnz": mi["nnz"], "spmv_format": mi["format"], "sell_sigma": mi["sell_sigma"],
                   "nnz_stored": mi["nnz_stored"], "col_index_bytes": mi["col_index_bytes"],
                   "value_bytes": mi["value_bytes"], "launches_per_iter": mi["iter_launches"],
                   "bytes_per_iter": mi["bytes_per_iter"], "bytes_per_iter_survey_model": c2["bytes_survey"]},
        "effective_gbs": round(c2["gbs"], 1), "pct_peak_hbm": round(100 * c2["gbs"] / PEAK_HBM_GBS, 2),
        "effective_gbs_survey_bytes": round(c2["bytes_survey"] * c2["ips"] / 1e9, 1),
        "steady_state": c2["steady"], "roofline": c2["roofline"], "tol_1e-10": c2["tol_run"],
    }
    if copy_gbs is not None:
        line["copy_256MiB_gbs"] = round(copy_gbs, 1)
    if "cpu_baseline" in c2:
        line["cpu_baseline"] = c2["cpu_baseline"]
        line["parity_x_k"] = c2["parity_x_k"]
    line["legs"] = legs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
