#!/usr/bin/env python3
"""Benchmark of the mixed Burton-Miller hot path on one MI355X.

One step is one pass of the whole path over one batch of synthetic input:
bm_assemble (Nystrom matrix of the mixed system) -> bm_block_lu (Schur complement
U33 = -[M31 M32][M13; M23] and LU of U33, Theorem thm:LU) -> bm_rhs_plane_wave ->
bm_solve (8 right-hand sides, Corollary lem:for_ssm_RHS) -> bm_far_field (64 angles).
Inputs (geometry, angles) are resident in HBM before the timed region starts.

value = complete solves per second (one solve = the 8-right-hand-side system,
assembled, factored and solved, with its far field).  The ordinary 2N x 2N
formulation runs through the same kernels (same LU) as the comparator.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6   # MI355X dense FP64 matrix
PEAK_FP64_VECTOR_TFLOPS = 78.6  # MI355X FP64 vector
PEAK_HBM_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2512_14193_amd", "csrc")
# rocprofv3 FETCH_SIZE / WRITE_SIZE records (profiles/*.json): the file, the
# source text of the kernel it was measured on (file, first line starting with the
# start marker up to the end marker; None: the whole file), and the factorisation
# mode it was taken in
TRAFFIC = {
    "schur_gemm": ("schur_zgemm_star2048_traffic.json",
                   (("bm_zgemm.hip", None, "// Persistent form of the deep product"),), False),
    "panel": ("panel_star2048_traffic.json",
              (("bm_getrf.hip", "// 1. panel factorisation", "// 2. row interchanges outside the panel"),
               ("bm_internal.h", None, None)), True),
}


def kernel_hash(sources):
    h = hashlib.sha256()
    for name, start, end in sources:
        with open(os.path.join(CSRC, name), "rb") as f:
            text = f.read()
        a = text.index(start.encode()) if start else 0
        b = text.index(end.encode(), a) if end else len(text)
        h.update(text[a:b])
    return h.hexdigest()[:16]


def traffic_record(which, workload, lu_overlap):
    """HBM bytes per launch of a kernel from rocprofv3 counters, if they were taken
    on the current kernel sources, this workload and this factorisation mode; else
    None."""
    fname, sources, overlap = TRAFFIC[which]
    if overlap != lu_overlap:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_hash(sources) or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def run_formulation(form, w, steps, warmup, precision="fp64", tol=1e-12, lu_overlap=True):
    import torch
    from paper_2512_14193_amd import binding as B

    N = w.boundary.n_nodes
    R = len(w.theta_inc)
    dev = torch.device("cuda")
    geo = [torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
           for a in (w.boundary.x, w.boundary.dx, w.boundary.ddx, w.boundary.d3x)]
    theta_inc = torch.as_tensor(w.theta_inc, dtype=torch.float64, device=dev)
    theta_obs = torch.as_tensor(w.theta_obs, dtype=torch.float64, device=dev)
    P = B.Problem(N, form)
    if precision != "fp64":
        P.set_precision(precision, tol=tol, max_iter=10)
    if form == "mixed" and not lu_overlap:
        P.set_lu_overlap(False)  # the whole Schur product first, then the LU
    Bm = B.fortran_empty(P.rows, R)
    X = B.fortran_empty(P.rows, R)
    F = B.fortran_empty(len(w.theta_obs), R)

    def step():
        P.assemble_device(geo, w.physics)
        P.block_lu(sync=False)
        P.rhs_plane_wave(theta_inc, Bm)
        P.solve(Bm, X)
        P.far_field(X, theta_obs, F)

    for _ in range(warmup):
        step()
    P.sync()
    torch.cuda.synchronize()
    P.set_profiling(True)
    P.phase_times()  # reset the per-phase accumulators
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        if s == steps - 1:
            P.set_profiling(2)  # the last timed step also times each panel kernel
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, cnt = P.phase_times()
    refine = P.refine_stats()
    overlap_enabled, segments = P.lu_overlap_info() if form == "mixed" else (False, 0)
    P.set_profiling(False)
    P.sync()  # raises if a kernel reported a device-side error
    # pivot check on a fresh assembly (the ordinary matrix is factored in place)
    P.assemble_device(geo, w.physics)
    info = P.block_lu(sync=True)
    if info != 0:
        raise RuntimeError(f"{form}: singular factor, info = {info}")
    phases = {name: (ms[i] / cnt[i] if cnt[i] else None)
              for i, name in enumerate(["assemble", "schur_gemm", "lu", "solve", "far_field"])}
    # per panel launch, over the panels of the last timed step (the latest 64 when
    # a step has more: the last 64 panels, the shortest, at N = 8192)
    phases["panel_kernel_avg"] = ms[5] / cnt[5] if cnt[5] else None
    # the factorisation: U33 formed beside the LU (segments > 0: the "lu" phase is
    # the whole factorisation and "schur_gemm" the product's span inside it), or
    # formed first (the two phases add up)
    if segments > 0:
        phases["factor"] = phases["lu"]
    else:
        phases["factor"] = (phases["schur_gemm"] or 0.0) + (phases["lu"] or 0.0)
    out = {"seconds": t1 - t0, "phase_ms": phases, "X": X.cpu().numpy(), "F": F.cpu().numpy(),
           "refine_iterations": refine[0], "rel_residual": refine[1], "panel_launches_timed": cnt[5],
           "lu_overlap": {"enabled": overlap_enabled, "segments": segments}}
    P.close()
    return out


def mixed_precision_section(name, steps, warmup, tol):
    """FP64 block LU against the mixed-precision one (split-FP16 matrix-core Schur
    complement into a complex64 U33, its LU in complex64, FP64 refinement) on the
    same workload, both end to end, at the refinement target `tol` and at the tests'
    1e-12; the plain FP64 LU of the ordinary 2N x 2N system on the same boundary as
    the second reference.  Executed matrix-core rates: FP64 Gauss 3M executes 12 N^3
    flops; the split-FP16 product 48 N^3 (four real products of 2 N^3 multiply-adds,
    three FP16 terms each), the packing and line-maxima passes included in its time."""
    import numpy as np
    from paper_2512_14193_amd import inputs as I
    w = I.workload(name)
    N = w.boundary.n_nodes
    res = {}
    for key, prec, t in (("fp64", "fp64", tol), ("mixed", "mixed", tol), ("mixed_tol_1e-12", "mixed", 1e-12)):
        r = run_formulation("mixed", w, steps, warmup, precision=prec, tol=t)
        ph = r["phase_ms"]
        res[key] = {"solves_per_s": steps / r["seconds"], "ms_per_step": 1e3 * r["seconds"] / steps,
                    "phase_ms": ph, "refine_tol": t if prec == "mixed" else None,
                    "schur_tflops": 16.0 * N ** 3 / (ph["schur_gemm"] * 1e-3) / 1e12,
                    "schur_executed_mfma_tflops": (48.0 if prec == "mixed" and N >= 256 else 12.0) * N ** 3
                    / (ph["schur_gemm"] * 1e-3) / 1e12,
                    "schur_kernel": ("zgemm_kernel<true, true> (FP64 Gauss 3M)" if prec == "fp64" else
                                     "z16_gemm_kernel (split FP16, v_mfma_f32_32x32x16_f16)" if N >= 256 else
                                     "zgemm32_kernel (FP32 Gauss 3M)"),
                    "refine_iterations": r["refine_iterations"], "rel_residual": r["rel_residual"], "X": r["X"]}
    Xf = res["fp64"]["X"]
    rel = lambda a, b: float(np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)))  # noqa: E731
    diffs = {k: rel(res[k].pop("X"), Xf) for k in ("mixed", "mixed_tol_1e-12")}
    res["fp64"].pop("X")
    o = run_formulation("ordinary", w, steps, warmup)
    ordinary = {"solves_per_s": steps / o["seconds"], "ms_per_step": 1e3 * o["seconds"] / steps,
                "phase_ms": o["phase_ms"]}
    return {"workload": name, "unknowns": 3 * N, "steps": steps, "refine_tol": tol,
            "fp64": res["fp64"], "mixed": res["mixed"], "mixed_tol_1e-12": res["mixed_tol_1e-12"],
            "ordinary_fp64": ordinary,
            "speedup_mixed_over_fp64_block_lu": res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"],
            "speedup_mixed_tol_1e-12_over_fp64_block_lu":
                res["mixed_tol_1e-12"]["solves_per_s"] / res["fp64"]["solves_per_s"],
            "speedup_mixed_over_ordinary_fp64_lu": res["mixed"]["solves_per_s"] / ordinary["solves_per_s"],
            "rel_diff_mixed_vs_fp64": diffs["mixed"], "rel_diff_mixed_tol_1e-12_vs_fp64": diffs["mixed_tol_1e-12"],
            "rel_diff_uq_ordinary_vs_fp64_mixed_form": rel(o["X"], Xf[:2 * N])}


def fds_section(steps, warmup, n_nodes=65536):
    """The proxy-compressed fast direct solver (Sec. 4.2) on the ellipse of semi-axes
    10 and 1 with k0 = 50, k1 = 75 (eps1 = 2.25), N = 65536 nodes (196,608 unknowns,
    beyond a dense factorisation: its four blocks alone would need 275 GB), leaf
    cells of 256 nodes, 128 proxy points at least, rank tolerance 1e-10, eight
    seeded plane waves.  One step = compression and factorisation + 8-RHS solve +
    far field; the solve alone is timed as well (factors reused)."""
    import numpy as np
    import torch
    from paper_2512_14193_amd import binding as B
    from paper_2512_14193_amd import inputs as I
    bnd = I.ellipse(n_nodes, 10.0, 1.0)
    ph = I.Physics.from_wavenumbers(50.0, 75.0)
    dev = torch.device("cuda")
    geo = [torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous() for a in (bnd.x, bnd.dx, bnd.ddx, bnd.d3x)]
    th = torch.as_tensor(I.plane_wave_angles(8, 5), device=dev)
    tho = torch.as_tensor(I.observation_angles(64), device=dev)
    f = B.FDS(n_nodes, leaf=256, n_proxy=128, tol=1e-10)
    Bm = B.fortran_empty(3 * n_nodes, 8)
    X = B.fortran_empty(3 * n_nodes, 8)
    F = B.fortran_empty(64, 8)

    def step():
        f.factor(geo, ph)
        f.rhs_plane_wave(th, Bm)
        f.solve(Bm, X)
        f.far_field(X, tho, F)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ts0 = time.perf_counter()
    for _ in range(steps):
        f.solve(Bm, X)
    torch.cuda.synchronize()
    ts1 = time.perf_counter()
    info = f.info()
    f.close()
    Xn = X.cpu().numpy()
    return {"workload": f"ellipse semi-axes 10 and 1, N = {n_nodes} ({3 * n_nodes} unknowns), k0 = 50, k1 = 75, "
                        "one-point zeta-corrected quadrature, 8 plane waves",
            "leaf": 256, "n_proxy_min": 128, "rank_tol": 1e-10, "steps": steps,
            "solves_per_s": steps / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps,
            "solve_only_ms": 1e3 * (ts1 - ts0) / steps, "levels": info["levels"],
            "skeletons_per_level": info["skeletons_sum"], "skeletons_max_per_cell": info["skeletons_max"],
            "root_order": info["root_n"], "device_bytes": info["device_bytes"],
            "dense_blocks_bytes_would_be": 64 * n_nodes * n_nodes, "solution_finite": bool(np.isfinite(Xn).all())}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, X_gpu=None, F_gpu=None):
    """The oracle as it stands on the host cores: explicit 3N x 3N matrix, dense
    partial-pivot LU, 8-RHS solve and far field for the same workload; with the
    GPU's solution and far field of the same workload, their error against it."""
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    O.lib()  # build/load outside the timed region
    t0 = time.perf_counter()
    A = O.build_mixed(w.boundary, w.physics)
    Bm = O.rhs_plane_wave(w.boundary, w.physics, w.theta_inc)
    X = O.zgesv(A, Bm)
    N = w.boundary.n_nodes
    F = O.far_field(w.boundary, w.physics, X[:N], X[N:2 * N], w.theta_obs)
    t = time.perf_counter() - t0
    out = {"value": 1.0 / t, "unit": "solves/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"one full pass of {w.name} (assembly of the explicit {3 * N}x{3 * N} matrix, "
                     f"dense LU, {len(w.theta_inc)}-RHS solve, far field) on the host; {t:.1f} s"}
    rel = lambda a, b: float(np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)))  # noqa: E731
    if X_gpu is not None:
        out["gpu_vs_oracle_rel_err_solution"] = rel(X_gpu, X)
    if F_gpu is not None:
        out["gpu_vs_oracle_rel_err_far_field"] = rel(F_gpu, F)
    return out


def serving_section(rate, graph_max_n, max_inflight, lanes, concurrent_max_n, batch_max=2):
    """The served contour sweep (256 requests on 8 circles |k - c| = 0.5, stars
    with N in {512, ..., 4096}, 16 probing right-hand sides each) through the
    request server: closed-loop capacity (all requests queued at once, with and
    without graph replay for small N) and open-loop latency under Poisson
    arrivals at `rate` requests per second."""
    import numpy as np
    import torch
    from paper_2512_14193_amd import binding as B
    from paper_2512_14193_amd import inputs as I

    sw = I.serving_workload(rate=rate)
    dev = torch.device("cuda")
    geos = {}
    for c, n in enumerate(sw.sizes):
        bnd = I.star(int(n))
        geos[c] = [torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
                   for a in (bnd.x, bnd.dx, bnd.ddx, bnd.d3x)]
    Bs = [B.fortran(torch.as_tensor(I.probing_rhs(3 * r.n_nodes, sw.n_rhs, r.rhs_seed)).to(dev))
          for r in sw.requests]
    Xs = [B.fortran_empty(3 * r.n_nodes, sw.n_rhs) for r in sw.requests]
    torch.cuda.synchronize()

    def server_submit(server, r):
        return server.submit(geos[r.contour], r.physics, Bs[r.index], Xs[r.index])

    def run(server, open_loop):
        tickets = []
        t0 = time.perf_counter()
        for r in sw.requests:
            if open_loop:
                dt = t0 + r.arrival - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            tickets.append(server_submit(server, r))
        res = [server.wait(t) for t in tickets]
        bad = [x["status"] for x in res if x["status"] != 0]
        if bad:
            raise RuntimeError(f"served requests failed: {bad[:5]}")
        return res

    def warm(server, lanes=1):
        """Create the handles (on every lane) and capture the graphs before timing."""
        per_n = {}
        for r in sw.requests:
            per_n.setdefault(r.n_nodes, [])
            if len(per_n[r.n_nodes]) < lanes:
                per_n[r.n_nodes].append(r)
        for rs in per_n.values():
            for t in [server.submit(geos[r.contour], r.physics, Bs[r.index], Xs[r.index]) for r in rs]:
                server.wait(t)

    def summary(res):
        lat = np.array([x["t_done"] - x["t_submit"] for x in res]) * 1e3
        span = max(x["t_done"] for x in res) - min(x["t_submit"] for x in res)
        by_n = {}
        for x in res:
            by_n.setdefault(x["n"], []).append(x)
        return {"throughput_req_per_s": len(res) / span, "makespan_s": span,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                               "p99": float(np.percentile(lat, 99)), "max": float(lat.max()),
                               "mean": float(lat.mean())},
                "by_n": {str(n): {"requests": len(v),
                                  "device_ms_mean": float(np.mean([x["device_ms"] for x in v])),
                                  "latency_ms_p50": float(np.percentile([1e3 * (x["t_done"] - x["t_submit"])
                                                                         for x in v], 50))}
                         for n, v in sorted(by_n.items())}}

    out = {"workload": "contour sweep: 8 circles |k-c|=0.5 (c ~ U[2,20]) x 32 nodes = 256 requests, "
                       "star r=1+0.3cos5t with N ~ {512,1024,2048,4096}, k1 = 1.5 k0, 16 probing RHS, "
                       "Poisson arrivals",
           "sizes_per_contour": [int(n) for n in sw.sizes], "requests": len(sw.requests), "nrhs": sw.n_rhs,
           "rate_req_per_s": rate, "max_inflight_per_lane": max_inflight, "graph_max_n": graph_max_n,
           "lanes": lanes, "concurrent_max_n": concurrent_max_n, "batch_max": batch_max}
    srv = B.Server(max_inflight=max_inflight, graph_max_n=0, lanes=1)
    warm(srv)
    out["closed_loop_one_lane_eager"] = summary(run(srv, False))
    srv.close()
    if batch_max > 1:  # the same server factoring one request at a time
        srv = B.Server(max_inflight=max_inflight, graph_max_n=graph_max_n, lanes=lanes,
                       concurrent_max_n=concurrent_max_n)
        warm(srv, lanes)
        out["closed_loop_unbatched"] = summary(run(srv, False))
        srv.close()
    srv = B.Server(max_inflight=max_inflight, graph_max_n=graph_max_n, lanes=lanes,
                   concurrent_max_n=concurrent_max_n, batch_max=batch_max)
    warm(srv, lanes)
    closed = run(srv, False)
    out["batched_requests"] = int(sum(x["batched"] > 1 for x in closed))
    out["closed_loop"] = summary(closed)
    out["capacity_req_per_s"] = out["closed_loop"]["throughput_req_per_s"]
    sample = [0, 1, 2, 3, len(Xs) - 1]
    before = [Xs[i].clone() for i in sample]
    out["open_loop"] = summary(run(srv, True))
    torch.cuda.synchronize()
    out["bitwise_repeatable"] = all(torch.equal(Xs[i], b) for i, b in zip(sample, before))
    out["server_stats"] = srv.stats()
    srv.close()
    # the same sweep in mixed precision (split-FP16 Schur complement, complex64 LU,
    # refinement decided on the device: 2 passes, target 1e-10; same-N requests
    # factored together as above), against the FP64 served solutions
    fp64 = [x.clone() for x in Xs]
    srv = B.Server(max_inflight=max_inflight, graph_max_n=graph_max_n, lanes=lanes,
                   concurrent_max_n=concurrent_max_n, precision="mixed", refine_steps=2, refine_tol=1e-10,
                   batch_max=batch_max)
    warm(srv, lanes)
    tickets = []
    for r in sw.requests:
        tickets.append(server_submit(srv, r))
    res = [srv.wait(t) for t in tickets]
    ok = [x for x in res if x["status"] == 0]
    torch.cuda.synchronize()
    rel = [float((torch.linalg.norm(Xs[i] - fp64[i], dim=0) / torch.linalg.norm(fp64[i], dim=0)).max())
           for i, x in enumerate(res) if x["status"] == 0]
    out["closed_loop_mixed"] = dict(summary(ok), refine_steps=2, refine_tol=1e-10,
                                    not_converged=len(res) - len(ok),
                                    max_rel_diff_vs_fp64=max(rel) if rel else None)
    srv.close()
    return out


# Table tb:ssm_eigenvalues: the first "Mixed" row of each eigenvalue and its time
# on 2x EPYC 9654 (order-31 zeta-corrected quadrature, N = 4000)
SSM_PRINTED = {2: (0.42948496520839791 - 1.2813737976521153j, 98.895),
               3: (1.3080120322683002 - 1.6817888047453846j, 114.206)}


def ssm_section(n_nodes, per_side, quadrature="zeta31"):
    """Sakurai-Sugiura eigenvalues of the mixed equation on the disk of radius
    0.5 (eps0 = 1, eps1 = 4) in squares of side 0.1 around the two printed
    eigenvalues, L = M = 4 (Table tb:ssm_parameters), through the request server,
    on the order-31 zeta-corrected rule of that table by default."""
    import mpmath as mp
    import numpy as np
    from paper_2512_14193_amd import binding as B
    from paper_2512_14193_amd import inputs as I
    from paper_2512_14193_amd import ssm

    bnd = I.disk(n_nodes, 0.5)
    srv = B.Server(lanes=4, quadrature=quadrature)
    ssm.eigenvalues(bnd, 1.0, 4.0, SSM_PRINTED[2][0], per_side=1, server=srv)  # handle creation, untimed
    out = {"boundary": f"disk a=0.5, N={n_nodes}", "eps0": 1.0, "eps1": 4.0, "contour": "square, side 0.1",
           "nodes_per_side": per_side, "contour_quadrature": "Gauss-Legendre per side",
           "boundary_quadrature": {"zeta31": "zeta-corrected trapezoid, order 31", "kress": "Kress log-split",
                                   "zeta": "zeta-corrected trapezoid, one point"}[quadrature],
           "n_rhs": 4, "n_moments": 4, "results": []}
    mp.mp.dps = 40
    for order, (z0, paper_s) in SSM_PRINTED.items():
        res = ssm.eigenvalues(bnd, 1.0, 4.0, z0, side=0.1, per_side=per_side, server=srv)
        zero = complex(mp.findroot(lambda z: mp.hankel1(order, z), mp.mpc(z0.real, z0.imag)))
        out["results"].append({
            "hankel_order": order, "eigenvalues": [[v.real, v.imag] for v in res.eigenvalues],
            "rank": res.rank, "singular_values_rel": [float(v) for v in res.singular_values[:6] / res.singular_values[0]],
            "solves": res.n_solves, "seconds": res.seconds, "device_ms": res.device_ms,
            "max_abs_err_vs_hankel_zero": float(np.max(np.abs(res.eigenvalues - zero))) if len(res.eigenvalues)
            else None,
            "printed_value_abs_err_vs_hankel_zero": abs(z0 - zero),
            "paper_seconds_2x_epyc_9654": paper_s})
    srv.close()
    return out


def calibrate_copy(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="star2048")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-lu-overlap", action="store_true",
                    help="form the whole Schur complement before the LU (no segments beside the panels)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP64 vs mixed-precision comparison")
    ap.add_argument("--mixed-workload", default="star8192")
    ap.add_argument("--mixed-steps", type=int, default=3)
    ap.add_argument("--mixed-tol", type=float, default=1e-10,
                    help="relative residual target of the refinement in the mixed-precision comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the served contour sweep")
    ap.add_argument("--serving-rate", type=float, default=50.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--serving-graph-max-n", type=int, default=1024)
    ap.add_argument("--serving-inflight", type=int, default=4)
    ap.add_argument("--serving-lanes", type=int, default=4)
    ap.add_argument("--serving-concurrent-max-n", type=int, default=2048)
    ap.add_argument("--serving-batch-max", type=int, default=2,
                    help="queued FP64 requests of one N factored together (1: one at a time)")
    ap.add_argument("--no-ssm", action="store_true", help="skip the Sakurai-Sugiura eigenvalue section")
    ap.add_argument("--no-fds", action="store_true", help="skip the fast direct solver section (N = 65536)")
    ap.add_argument("--fds-steps", type=int, default=3)
    ap.add_argument("--ssm-n", type=int, default=4000)
    ap.add_argument("--ssm-per-side", type=int, default=48)
    ap.add_argument("--ssm-quadrature", default="zeta31", choices=["zeta31", "kress", "zeta"])
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (traffic-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path "
              "(independent solves would go one per GPU; one large factorisation would need a "
              "2-D block-cyclic LU); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import numpy as np
    from paper_2512_14193_amd import inputs as I

    w = I.workload(args.workload)
    N = w.boundary.n_nodes
    R = len(w.theta_inc)
    mixed = run_formulation("mixed", w, args.steps, args.warmup, lu_overlap=not args.no_lu_overlap)
    sec = mixed["seconds"]
    value = args.steps / sec
    ph = mixed["phase_ms"]
    # Algorithmic work: the Schur complement (m = n = N, k = 2N) is 8 m n k =
    # 16 N^3 real flops, the LU of U33 8/3 N^3.  The Schur kernel uses Gauss's
    # three-multiplication form and executes 12 N^3 real flops on the matrix
    # cores; that executed rate is reported beside the algorithmic one (the
    # hardware utilisation itself comes from the rocprof MFMA counters).
    flops_schur = 16.0 * N ** 3
    flops_schur_mfma = 12.0 * N ** 3
    flops_lu = 8.0 / 3.0 * N ** 3
    t_schur = ph["schur_gemm"] * 1e-3
    schur_tflops = flops_schur / t_schur / 1e12
    t_factor = ph["factor"] * 1e-3
    factor_tflops = (flops_schur + flops_lu) / t_factor / 1e12
    overlap = mixed["lu_overlap"]["segments"] > 0
    traffic = {k: traffic_record(k, w.name, overlap) for k in TRAFFIC}
    # The panel factorisation kernel: mean algorithmic flops of the step's panels
    # (LU of an R x 64 panel: sum_c 8 (R - c - 1)(63 - c) for the rank-1 updates and
    # 6 (R - c - 1) for the scaling, R = N - 64 i) over its mean launch duration.
    nb = 64
    panel_rows = [N - nb * i for i in range((N + nb - 1) // nb)]
    panel_flops = [sum(8.0 * max(R - c - 1, 0) * max(min(nb, R) - c - 1, 0) + 6.0 * max(R - c - 1, 0)
                       for c in range(min(nb, R))) for R in panel_rows]
    timed = panel_flops[-mixed["panel_launches_timed"]:]  # the panels the events covered
    panel_flops_mean = sum(timed) / len(timed)
    t_panel = ph["panel_kernel_avg"] * 1e-3
    panel_step_ms = ph["panel_kernel_avg"] * len(panel_rows)
    kern = {
        "panel": {"kernel": "panel_kernel<1, fused|plain> (one 64-column panel of the LU of U33; 64 dependent "
                            "pivot steps, one cross-workgroup exchange each; the fused form first applies the "
                            "previous panel's update to its columns)",
                  "bound": "alu", "achieved": panel_flops_mean / t_panel / 1e12, "peak": PEAK_FP64_VECTOR_TFLOPS,
                  "unit": "TFLOP/s", "frac": panel_flops_mean / t_panel / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
                  "traffic": traffic["panel"], "avg_launch_ms": ph["panel_kernel_avg"],
                  "launches_per_step": len(panel_rows),
                  "ms_per_step": panel_step_ms, "flops_per_launch_mean": panel_flops_mean,
                  "launches_timed": mixed["panel_launches_timed"]},
        "schur_gemm": {"kernel": ("zgemm_persist_kernel segments beside the LU (Schur complement, m=n=N, k=2N; "
                                  "16 N^3 algorithmic flops; time = the product's span, overlapped with the panels)")
                       if overlap else
                       "zgemm_kernel<true,true> (Schur complement, m=n=N, k=2N; 16 N^3 algorithmic flops)",
                       "bound": "mfma", "achieved": schur_tflops, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                       "frac": schur_tflops / PEAK_FP64_MFMA_TFLOPS, "traffic": traffic["schur_gemm"],
                       "avg_launch_ms": ph["schur_gemm"],
                       "launches_per_step": mixed["lu_overlap"]["segments"] if overlap else 1,
                       "ms_per_step": ph["schur_gemm"], "overlapped_with_lu": overlap},
    }
    # (the product's span overlaps the panels: it is not on the step's critical path)
    dominant = max(kern, key=lambda k: 0.0 if kern[k].get("overlapped_with_lu") else kern[k]["ms_per_step"])
    roofline = dict(kern[dominant])
    roofline["dominant_by_time_per_step"] = True
    roofline["other_kernels"] = {k: v for k, v in kern.items() if k != dominant}
    rec = {
        "metric": "block-LU solves/s (mixed Burton-Miller, assemble + factor + 8-RHS solve + far field)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "boundary": w.boundary.name, "n_nodes": N, "unknowns": 3 * N,
                   "k0": w.physics.k0.real, "k1": w.physics.k1.real, "eps1": w.physics.eps1, "nrhs": R,
                   "far_field_angles": len(w.theta_obs), "quadrature": "Kress log-split"},
        "roofline": roofline,
        "schur_executed_mfma_tflops": flops_schur_mfma / t_schur / 1e12,
        "phase_ms": ph,
        "factor_tflops": factor_tflops,
        "factor_mfma_frac": factor_tflops / PEAK_FP64_MFMA_TFLOPS,
        "lu_phase_tflops": None if overlap else flops_lu / (ph["lu"] * 1e-3) / 1e12,
        "lu_overlap": mixed["lu_overlap"],
        "rhs_solves_per_s": value * R,
    }
    if not args.no_comparator:
        ordi = run_formulation("ordinary", w, args.steps, args.warmup)
        v_ord = args.steps / ordi["seconds"]
        Xm, Xo = mixed["X"], ordi["X"]
        diff = float(np.max(np.linalg.norm(Xm[:2 * N] - Xo, axis=0) / np.linalg.norm(Xo, axis=0)))
        rec["comparator"] = {"formulation": "ordinary 2N x 2N Burton-Miller, same kernels",
                             "value": v_ord, "ms_per_step": 1e3 * ordi["seconds"] / args.steps,
                             "phase_ms": ordi["phase_ms"], "speedup_mixed_over_ordinary": value / v_ord,
                             "rel_diff_uq_mixed_vs_ordinary": diff,
                             "paper_context": "1.38-1.44x on 2x EPYC 9654 (CPU, zeta-corrected quadrature, disk)"}
    if not args.no_mixed:
        rec["mixed_precision"] = mixed_precision_section(args.mixed_workload, args.mixed_steps, 1, args.mixed_tol)
    if not args.no_serving:
        rec["serving"] = serving_section(args.serving_rate, args.serving_graph_max_n, args.serving_inflight,
                                         args.serving_lanes, args.serving_concurrent_max_n,
                                         args.serving_batch_max)
    if not args.no_ssm:
        rec["ssm"] = ssm_section(args.ssm_n, args.ssm_per_side, args.ssm_quadrature)
    if not args.no_fds:
        rec["fast_direct_solver"] = fds_section(args.fds_steps, 1)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, mixed["X"], mixed["F"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
