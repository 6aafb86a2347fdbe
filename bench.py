"""Benchmark of the MI355X hot path on the k = 10 periodic workload.

One step = the whole hot path on one batch: fill the 33 distinct mode blocks
of the body (N = 200, M = 240, P = 64, q = 400), factor them (QR + Jacobi
truncation at 1e-10), then solve 8 seeded incident waves (per-wave Q fill
and factorisation, batched GMRES to 1e-10 with the 3x3 neighbour sums,
recovery of the Bragg amplitudes and of the field at cell test points).

Prints one JSON line.  `value` is incident-wave solves per second of the
whole step (operator build included); the fill+QR FP64 rate, solve-only
throughput and latency percentiles are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_FP64 = 78.6      # TFLOP/s, MI355X FP64 vector and matrix (dense)
PEAK_HBM = 8000.0     # GB/s


def qr_flops(M: int, N: int) -> float:
    """Householder QR of a complex M x N block: 8 M N^2 - 8 N^3 / 3 real flops."""
    return 8.0 * M * N * N - 8.0 * N ** 3 / 3.0


def fill_flops(bodies) -> float:
    """Algorithmic FP64 work of the modal fill, per (collocation, source)
    pair: q/2 + 1 kernel samples (about 20 flops each, the reciprocal square
    root and the sine-cosine counted as one flop each) and the cosine sums of
    the P/2 + 1 distinct modes, 4 flops per (sample, mode) (a real weight
    times a complex sample)."""
    return float(sum(b.M * b.N * (b.q // 2 + 1) * (20 + 4 * (b.P // 2 + 1)) for b in bodies))


def nsum_pairs(pr: W.Problem) -> float:
    """Kernel evaluations of one A_else action: 8 images x (P M) targets x (P N) sources."""
    b = pr.body
    return 8.0 * (b.P * b.M) * (b.P * b.N)


def measured_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary
    (rocprofv3 --pmc, scaled by the same counters of a 2 GiB copy), or None
    if the kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_1506_05083_amd", "csrc", kernel_source)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("source_sha256") != digest:
        return None
    return float(kv["traffic_bytes_per_launch"])


def run_gpu(pr: W.Problem, steps: int, warmup: int):
    import torch
    import paper_1506_05083_amd as mfs

    b, lat = pr.body, pr.lattice
    ctx = mfs.create(0)
    geom = mfs.polar_geometry(b.shape.a, b.shape.eps, b.shape.j, b.M, b.N, b.tau, b.colloc)
    L = mfs.lattice(lat.ex, lat.ey, lat.z0, lat.p, lat.N0, lat.M1)
    waves = [(w.theta, w.phi) for w in pr.waves]

    def step():
        ts = time.perf_counter()
        op = mfs.build_operator(ctx, [mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, geom)])
        op.factor_modes(1e-10)
        t0 = time.perf_counter()
        res, tm = mfs.solve_incident(ctx, op, L, waves, tol=pr.gmres_tol, maxit=pr.maxit,
                                     targets=pr.targets, q_field=pr.q_field, timing=True)
        t1 = time.perf_counter()
        return op.timing(), res, tm, t1 - t0, t1 - ts

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t_start = time.perf_counter()
    for _ in range(steps):
        recs.append(step())
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    return t_total, recs


def run_batch_build(count: int):
    """Batched-build configuration: `count` seeded obstacles of uneven size
    (N 100..600, M = 1.2 N, P 32..160, k 5..30) filled in one persistent
    launch and factored (QR + truncation) in batched chunks.  Reports the
    fill + QR FP64 rate over the distinct blocks (8 M N^2 - 8 N^3 / 3 flops
    each) and the truncation time."""
    import torch
    import paper_1506_05083_amd as mfs

    bodies = W.batch_obstacles(count)
    ctx = mfs.create(0)
    specs = []
    for b in bodies:
        g = mfs.polar_geometry(b.shape.a, b.shape.eps, b.shape.j, b.M, b.N, b.tau, b.colloc)
        specs.append(mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, g))
    torch.cuda.synchronize()
    nblk = sum(b.P // 2 + 1 for b in bodies)
    print(f"[batch] filling {count} obstacles ({nblk} distinct blocks)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    op = mfs.build_operator(ctx, specs)
    t1 = time.perf_counter()
    print(f"[batch] filled in {t1 - t0:.2f} s; factoring", file=sys.stderr, flush=True)
    ranks = op.factor_modes(1e-10)
    t2 = time.perf_counter()
    print(f"[batch] factored in {t2 - t1:.2f} s", file=sys.stderr, flush=True)
    tm = op.timing()
    flops = sum((b.P // 2 + 1) * qr_flops(b.M, b.N) for b in bodies)
    gbytes = sum((b.P // 2 + 1) * ((b.M + 15) // 16 * 16) * b.N * 16 for b in bodies) / 1e9
    fflops = fill_flops(bodies)
    del op
    # the same build with the truncation as a complete orthogonal
    # decomposition (MFS_OPINV=cod; the library then forms no singular values)
    os.environ["MFS_OPINV"] = "cod"
    try:
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        op = mfs.build_operator(ctx, specs)
        t4 = time.perf_counter()
        op.factor_modes(1e-10)
        t5 = time.perf_counter()
        tmc = op.timing()
        del op
    finally:
        del os.environ["MFS_OPINV"]
    # the builds' idle blocks (about 35 GB each) go back to the device before
    # the next measurement
    torch.cuda.synchronize()
    mfs.release_cached_memory(0)
    print(f"[batch] complete orthogonal decomposition: factored in {t5 - t4:.2f} s", file=sys.stderr, flush=True)
    return {"obstacles": count, "distinct_blocks": nblk, "blocks_GB": gbytes, "qr_flops": flops,
            "fill_ms": tm["fill"], "qr_ms": tm["qr"], "trunc_ms": tm["svd"],
            "fill_qr_tflops": flops / ((tm["fill"] + tm["qr"]) * 1e-3) / 1e12,
            "qr_tflops": flops / (tm["qr"] * 1e-3) / 1e12,
            "fill_roofline": {"bound": "alu", "kernel": "fill_batch_kernel (all bodies, one persistent launch)",
                              "achieved": fflops / (tm["fill"] * 1e-3) / 1e12, "peak": PEAK_FP64,
                              "unit": "TFLOP/s", "frac": fflops / (tm["fill"] * 1e-3) / 1e12 / PEAK_FP64,
                              "flops": fflops,
                              "flops_counted": "per (m, j) pair: (q/2+1) kernel samples at 20 flops (rsqrt and "
                                               "sincos as one each) + 4 (q/2+1)(P/2+1) for the cosine sums"},
            "build_wall_s": t1 - t0, "factor_wall_s": t2 - t1,
            "cod": {"trunc_ms": tmc["svd"], "qr_ms": tmc["qr"], "factor_wall_s": t5 - t4},
            "mean_rank_fraction":
                float(np.mean([r / b.N for b, r in zip([bb for bb in bodies for _ in range(bb.P // 2 + 1)],
                                                       ranks)])),
            "workload": "seeded obstacles (seed 3): a U[0.2,0.4], eps U[0,0.15], j U{2..5}, N U{100..600}, "
                        "P U{32,64,96,128,160}, k U[5,30], M = ceil(1.2N), tau = 0.1"}


def run_large(nwaves: int, transmission: bool):
    """Large configuration (cups at k = 2 pi 13, N = 450, M = 540, P = 144),
    or its transmission variant (km = 1.5 k): operator build and
    factorisation, then nwaves incidences in one batched solve (near sums on
    the fly: the stored form would need 645 GB)."""
    import torch
    import paper_1506_05083_amd as mfs

    pr = (W.cup_periodic_large_transmission if transmission else W.cup_periodic_large)(nwaves)
    b, lat = pr.body, pr.lattice
    ctx = mfs.create(0)
    if transmission:
        g = mfs.transmission_geometry(b.shape, b.M, b.N, b.tau, b.colloc)
    else:
        g = mfs.body_geometry(b.shape, b.M, b.N, b.tau, b.colloc)
    print(f"[large] {pr.name}: {nwaves} incidences", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = mfs.build_operator(ctx, [mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, g, km=pr.km)])
    op.factor_modes(1e-10)
    t1 = time.perf_counter()
    L = mfs.lattice(lat.ex, lat.ey, lat.z0, lat.p, lat.N0, lat.M1)
    res, tm = mfs.solve_incident(ctx, op, L, [(w.theta, w.phi) for w in pr.waves], tol=pr.gmres_tol,
                                 maxit=pr.maxit, targets=pr.targets, q_field=pr.q_field, timing=True)
    t2 = time.perf_counter()
    ot = op.timing()
    return {"workload": pr.name, "incidences": nwaves, "build_factor_s": t1 - t0, "solve_s": t2 - t1,
            "solves_per_s": nwaves / (t2 - t0), "fill_ms": ot["fill"], "qr_ms": ot["qr"], "trunc_ms": ot["svd"],
            "periodizer_ms": tm["periodizer"], "gmres_ms": tm["gmres"], "jacobi_ms": tm["jacobi_ms"],
            "nsum_avg_ms": tm["nsum_avg"], "gmres_iters": [r.iters for r in res],
            "eps_flux_max": max(r.eps_flux for r in res), "q_cols": max(r.nq_cols for r in res)}


def run_serving(pr: W.Problem, nreq: int, nplain: int, slots: int):
    """Serving configuration: requests of the seeded stream against the
    resident factored k = 10 operator.  Plain baseline: the first nplain
    requests as one-at-a-time solves (mfs_solve_incident with one wave).
    Served: all nreq submitted at once to a server with `slots` slots
    (saturated throughput X_sat), then the same requests as a Poisson stream
    at 0.8 X_sat (latency = completion - submission, measured by the server)."""
    import torch
    import paper_1506_05083_amd as mfs

    b, lat = pr.body, pr.lattice
    ctx = mfs.create(0)
    geom = mfs.polar_geometry(b.shape.a, b.shape.eps, b.shape.j, b.M, b.N, b.tau, b.colloc)
    L = mfs.lattice(lat.ex, lat.ey, lat.z0, lat.p, lat.N0, lat.M1)
    op = mfs.build_operator(ctx, [mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, geom)])
    op.factor_modes(1e-10)
    waves, gaps = W.serving_stream(nreq)
    kw = dict(tol=pr.gmres_tol, maxit=pr.maxit, targets=pr.targets, q_field=pr.q_field)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_iters = []
    for w in waves[:nplain]:
        r = mfs.solve_incident(ctx, op, L, [(w.theta, w.phi)], **kw)[0]
        plain_iters.append(r.iters)
    t_plain = time.perf_counter() - t0
    srv = mfs.Server(ctx, op, L, slots=slots, admit_batch=min(8, slots), hbm_budget=200 << 30, **kw)

    def drain(tickets, submit_at=None):
        """Submit (at the given times, if any) and collect; returns wall time, latencies, results."""
        t_start = time.perf_counter()
        out, lat_ms = {}, {}
        todo = list(range(len(waves))) if submit_at is not None else []
        live = dict(tickets)
        while todo or live:
            now = time.perf_counter() - t_start
            while todo and submit_at[todo[0]] <= now:
                i = todo.pop(0)
                live[i] = srv.submit(waves[i].theta, waves[i].phi)
            for i in list(live):
                r = srv.poll(live[i])
                if r is not None:
                    out[i], lat_ms[i] = r[0], r[1]
                    assert r[2], f"request {i} did not converge"
                    del live[i]
            time.sleep(0.0005)
        return time.perf_counter() - t_start, lat_ms, out

    t_sat, lat_sat, res_sat = drain({i: srv.submit(w.theta, w.phi) for i, w in enumerate(waves)})
    x_sat = nreq / t_sat
    rate = 0.8 * x_sat
    arrivals = np.cumsum(gaps) / rate
    t_poi, lat_poi, res_poi = drain({}, submit_at=arrivals)
    srv.close()
    lp = np.array([lat_poi[i] for i in range(nreq)])
    ls = np.array([lat_sat[i] for i in range(nreq)])
    same = max(float(np.max(np.abs(res_sat[i].a - res_poi[i].a)) / np.max(np.abs(res_poi[i].a)))
               for i in range(nreq))
    return {
        "requests": nreq, "slots": slots, "plain_requests": nplain,
        "plain_solves_per_s": nplain / t_plain,
        "served_saturated_solves_per_s": x_sat,
        "speedup_vs_plain": x_sat / (nplain / t_plain),
        "saturated_latency_p50_ms": float(np.percentile(ls, 50)),
        "saturated_latency_p99_ms": float(np.percentile(ls, 99)),
        "poisson_rate_per_s": rate,
        "poisson_solves_per_s": nreq / t_poi,
        "poisson_latency_p50_ms": float(np.percentile(lp, 50)),
        "poisson_latency_p99_ms": float(np.percentile(lp, 99)),
        "max_amplitude_diff_saturated_vs_poisson": same,
        "gmres_iters_mean": float(np.mean([r.iters for r in res_poi.values()])),
        "stream": "seeded request stream (directions seed 4, exponential gaps seed 40), first "
                  f"{nreq} of the serving configuration's 10,000",
    }


def cpu_baseline(pr: W.Problem, iters: int):
    """The oracle, as it stands, on a bounded sample of the same workload
    (10-30 s of CPU work), scaled to incident-wave solves per second with
    the operator build amortised over the batch of waves, like `value`:
      - one-body fill and per-mode SVDs of the body, in full;
      - for one wave, in full: the Q fill (q_matrix) and its equilibrated
        truncated SVD (equilibrated_pinv_factors);
      - for one wave, extrapolated: the oracle's A_else point matrix on 4 of
        its P target rings (linear in rings), the C point matrix on 1/8 of
        the T-wall rows (scaled to all 42 image-evaluations of the 12 wall
        groups), and two matrix-vector products with a matrix of A_else's
        size (1/8 of its rows, scaled) times the GPU's GMRES iteration
        count `iters`."""
    import oracle.geometry as og
    import oracle.onebody as ob
    import oracle.periodic as op_

    b, lat = pr.body, pr.lattice
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    g = og.build_geometry(b)
    A = ob.modal_blocks(b, g)
    pinv = ob.ModalPinv(A)
    t_build = time.perf_counter() - t0

    ps = op_.PeriodicSolver.__new__(op_.PeriodicSolver)
    ps.body, ps.lat, ps.geom, ps.A, ps.k, ps.P, ps.pinv, ps.cut = b, lat, g, A, b.k, b.P, pinv, 1e-10
    ps.walls = op_.wall_nodes(lat)
    ps.Xs, ps.Ns = og.surface_points(g, b.P)
    ps.Ysrc = og.source_ring_points(g, b.P)
    w = pr.waves[0]
    kv = W.wave_vector(b.k, w)
    ps.kv = kv
    ps.alpha = np.exp(1j * kv[0] * lat.ex)
    ps.beta = np.exp(1j * kv[1] * lat.ey)
    ps.orders = op_.rb_orders(b.k, kv, lat)
    Y = ps.Ysrc.reshape(-1, 3)
    # A_else: RINGS angle rings of targets out of P, one at a time
    RINGS = 4
    t1 = time.perf_counter()
    for ring in range(RINGS):
        X = ps.Xs[ring:ring + 1].reshape(-1, 3)
        Nn = ps.Ns[ring:ring + 1].reshape(-1, 3)
        for _, wgt, shift in op_.image_list(lat, ps.alpha, ps.beta, op_.ELSE8):
            _ = wgt * op_.kernel.dG_dnx(b.k, X[:, None, :], Nn[:, None, :], Y[None, :, :] + shift)
    t_aelse = (time.perf_counter() - t1) * b.P / RINGS
    # C: 1/8 of the T wall, 9 images with gradients
    nT = ps.walls.T.shape[0]
    sub = ps.walls.T[: max(1, nT // 8)]
    t1 = time.perf_counter()
    op_.near_matrices(b.k, Y, sub, op_.image_list(lat, ps.alpha, ps.beta, op_.NEAR9))
    t_c = (time.perf_counter() - t1) * 8 * (42.0 / 9.0)
    # Q: the whole fill and the whole equilibrated truncated SVD
    t1 = time.perf_counter()
    Q = ps.q_matrix()
    t_qfill = time.perf_counter() - t1
    t1 = time.perf_counter()
    op_.equilibrated_pinv_factors(Q, 1e-10)
    t_qsvd = time.perf_counter() - t1
    K = np.ones((b.P * b.M // 8, b.P * b.N), dtype=np.complex128)
    v = np.ones(b.P * b.N, dtype=np.complex128)
    t1 = time.perf_counter()
    for _ in range(2):
        K @ v
    t_mv = (time.perf_counter() - t1) / 2 * 8
    t_wave = t_aelse + t_c + t_qfill + t_qsvd + iters * t_mv
    nw = len(pr.waves)
    t_step = t_build + nw * t_wave
    sample_s = time.perf_counter() - t0
    return {
        "value": nw / t_step, "unit": "solves/s", "cores": cores, "kind": "oracle",
        "sample": (f"oracle (numpy/scipy, {cores} threads) on the same workload: one-body fill + per-mode "
                   f"SVDs in full ({t_build:.1f} s); per wave, extrapolated from fractions: A_else "
                   f"assembly {t_aelse:.0f} s ({RINGS}/{b.P} of rows), C {t_c:.0f} s (1/8 of a wall); in full: "
                   f"Q fill {t_qfill:.1f} s, Q SVD {t_qsvd:.1f} s ({Q.shape[0]} x {Q.shape[1]}); {iters} GMRES "
                   f"products {iters * t_mv:.1f} s; {sample_s:.0f} s of CPU work measured"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-obstacles", type=int, default=256,
                    help="obstacles of the batched-build measurement (0 skips it)")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the serving measurement (0 skips it)")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 2 GiB device to device (the reference for the HBM byte counters)")
    ap.add_argument("--only", choices=["batch", "large", "large-transmission", "serve"],
                    help="run one other configuration's measurement alone and print its JSON line")
    ap.add_argument("--large-waves", type=int, default=8,
                    help="incidences of the large-cup measurement (0 skips it)")
    args = ap.parse_args()
    # stage lines from the library on stderr (the large configuration's
    # factorisation runs for minutes; its Jacobi sweeps and GMRES iterations
    # report as they finish)
    os.environ.setdefault("MFS_PROGRESS", "1")
    if args.only == "batch":
        print(json.dumps(run_batch_build(args.batch_obstacles)))
        return
    if args.only == "serve":
        print(json.dumps(run_serving(W.periodic_k10(1), args.serve_requests, min(8, args.serve_requests),
                                     args.serve_slots)))
        return
    if args.only in ("large", "large-transmission"):
        print(json.dumps(run_large(args.large_waves, args.only == "large-transmission")))
        return
    if args.copy_probe:
        import torch
        n = 1 << 28                        # 2 GiB of float64 read, 2 GiB written
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the work shards by "
              "incident wave, each GPU solving its own batch with no communication", file=sys.stderr)
        sys.exit(2)

    pr = W.periodic_k10(8)
    b = pr.body
    t_total, recs = run_gpu(pr, args.steps, args.warmup)
    K = args.steps
    nw = len(pr.waves)
    ms_step = 1e3 * t_total / K
    nd = b.P // 2 + 1
    flops = nd * qr_flops(b.M, b.N)
    fill_ms = np.array([r[0]["fill"] for r in recs])
    qr_ms = np.array([r[0]["qr"] for r in recs])
    svd_ms = np.array([r[0]["svd"] for r in recs])
    solve_ms = np.array([1e3 * r[3] for r in recs])
    tms = [r[2] for r in recs]
    res = recs[-1][1]
    nsum_avg = float(np.mean([t["nsum_avg"] for t in tms]))
    pairs = nsum_pairs(pr)                # one batched launch serves all waves
    pairs_per_s = pairs / (nsum_avg * 1e-3)
    near_bytes = float(np.median([t["near_bytes"] for t in tms]))
    near_alg = float(np.median([t["near_alg_bytes"] for t in tms]))
    near_modes = sorted({int(t["near_mode"]) for t in tms})
    nsum_share = float(np.median([t["nsum_avg"] * t["nsum_launches"] for t in tms])) / ms_step
    if near_bytes > 0:
        # stored near field: every launch streams the kernel values the
        # method needs once (the padding of the last 64-target tile of each
        # group is not counted; strengths and outputs are under 0.1%)
        gbs = near_alg / (nsum_avg * 1e-3) / 1e9
        traffic = measured_traffic("nsum.hip", "nsum_dense_periodic_k10_traffic.txt")
        roof_nsum = {"bound": "hbm", "kernel": "nsum_dense_mirror_mfma_kernel<8> (A_else surface sums and C wall "
                                               "sums from the mirror-paired stored near field on the matrix cores; "
                                               "all waves, mean over launches)",
                     "achieved": gbs, "peak": PEAK_HBM, "unit": "GB/s", "frac": gbs / PEAK_HBM,
                     "traffic": traffic, "traffic_unit": "bytes per launch",
                     "launch_ms": nsum_avg, "bytes_per_launch": near_alg,
                     "stored_bytes_per_launch": near_bytes,
                     "fill_ms": float(np.median([t["near_fill_ms"] for t in tms])), "share_of_step": nsum_share}
    else:
        # algorithmic FP64 work of one (target, source, image) pair: distance and
        # R^2 (8), 1/R and R (2), kR (1), sincos (2), kernel assembly (10), and one
        # complex multiply-accumulate (8) per incident wave of the batch
        flops_pair = 8 + 2 + 1 + 2 + 10 + 8 * nw
        nsum_tflops = pairs_per_s * flops_pair / 1e12
        roof_nsum = {"bound": "alu", "kernel": "nsum_kernel<8> (A_else surface sum, all waves)",
                     "achieved": nsum_tflops, "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": nsum_tflops / PEAK_FP64, "traffic": None,
                     "launch_ms": nsum_avg, "pairs_per_launch": pairs, "flops_per_pair": flops_pair,
                     "share_of_step": nsum_share}
    # the periodizer's blocked QR of the 8 waves' Q (one batch): FP64 rate of
    # its kernels against the FP64 peak (its trailing update is a dense
    # contraction, 8 m n^2 - 8 n^3 / 3 flops per matrix)
    q_qr_ms = float(np.median([t["q_qr_ms"] for t in tms]))
    q_qr_fl = float(np.median([t["q_qr_flops"] for t in tms]))
    roof_qr = {"bound": "alu", "kernel": "bqr_* blocked Householder QR of the periodizer Q (8 waves, one batch)",
               "achieved": q_qr_fl / (q_qr_ms * 1e-3) / 1e12, "peak": PEAK_FP64, "unit": "TFLOP/s",
               "frac": q_qr_fl / (q_qr_ms * 1e-3) / 1e12 / PEAK_FP64, "traffic": None, "launch_ms": q_qr_ms,
               "flops_per_launch": q_qr_fl, "share_of_step": q_qr_ms / ms_step,
               "post_qr_ms": float(np.median([t["q_post_ms"] for t in tms])),
               "jacobi_ms": float(np.median([t["jacobi_ms"] for t in tms]))}
    # the dominant single kernel: the stored-near-field sum when it is used
    if near_bytes > 0 or roof_nsum["share_of_step"] >= roof_qr["share_of_step"]:
        roofline, other = roof_nsum, roof_qr
    else:
        roofline, other = roof_qr, roof_nsum
    line = {
        "metric": "FP64 modal fill+QR TFLOP/s; incident-wave solves/s, p50/p99 @1e-10 rel err",
        "value": nw * K / t_total,
        "unit": "solves/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"periodic_k10: unit lattice, k=10, r=0.3(1+0.1cos3t), N={b.N}, M={b.M}, "
                               f"P={b.P}, q={b.q}, tau={b.tau}, z0={pr.lattice.z0}, p={pr.lattice.p}, "
                               f"N0={pr.lattice.N0:g}, M1={pr.lattice.M1}, {nw} seeded incidences, "
                               f"GMRES {pr.gmres_tol:g}"},
        "fill_qr_tflops": flops / ((np.median(fill_ms) + np.median(qr_ms)) * 1e-3) / 1e12,
        "fill_ms": float(np.median(fill_ms)), "qr_ms": float(np.median(qr_ms)),
        "trunc_ms": float(np.median(svd_ms)),
        "solve_ms": float(np.median(solve_ms)),
        "solve_only_solves_per_s": nw / (np.median(solve_ms) * 1e-3),
        "batch_solve_ms_p50": float(np.percentile(solve_ms, 50)),
        "batch_solve_ms_p99": float(np.percentile(solve_ms, 99)),
        "step_ms_max": float(max(1e3 * r[4] for r in recs)),
        "near_field": {0: "on the fly (budget 0)", 1: "stored", 2: "on the fly (did not fit)",
                       3: "low-rank image blocks (did not fit)"}[near_modes[-1]],
        "stage_ms": {k: float(np.median([t[k] for t in tms])) for k in ("rhs", "periodizer", "gmres", "recover")},
        "gmres_iters": [r.iters for r in res],
        "eps_flux_max": float(max(r.eps_flux for r in res)),
        "roofline": roofline,
        "roofline_other": other,
    }
    if args.batch_obstacles > 0:
        line["batch_build"] = run_batch_build(args.batch_obstacles)
    if args.serve_requests > 0:
        sv = run_serving(W.periodic_k10(1), args.serve_requests, min(8, args.serve_requests), args.serve_slots)
        line["serving"] = sv
        # the metric's p50/p99: request latency (completion - arrival) of the
        # Poisson stream at 0.8 of the saturated served rate
        line["latency_p50_ms"] = sv["poisson_latency_p50_ms"]
        line["latency_p99_ms"] = sv["poisson_latency_p99_ms"]
        line["latency_source"] = (f"serving: {sv['requests']} requests of the seeded stream, Poisson arrivals at "
                                  f"{sv['poisson_rate_per_s']:.1f}/s (0.8 of the saturated served rate)")
    if args.large_waves > 0:
        line["large"] = run_large(args.large_waves, False)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pr, int(round(np.mean([r.iters for r in res]))))
    print(json.dumps(line))


if __name__ == "__main__":
    main()
