"""Benchmark: batched symmetric-stair PCG (build + solve) on one MI355X.

One step = the whole hot path over one batch: build S and Phi^-1 from the
per-knot blocks (FP64) and solve every problem with FP32 PCG inside FP64
iterative refinement to relative residual 1e-6.  Inputs are resident in HBM
before the timed region starts.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--pc sym|add|bj]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the solve kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for a
# plain copy of known size (2.0 and 1.0), keyed by the workload/settings and by
# a hash of the kernel's sources: a changed kernel reports null.
# the scaled solve's device code and the host code that sets its launch and stopping parameters
SOLVE_SOURCES = ("pcg3.hip", "ssp_fused.h", "ssp_device.h", "ssp_host.h", "host.hip")
MEASURED_TRAFFIC = {
    # (workload, pc, precision, kernel): (sources sha256[:16], HBM bytes of one solve): rocprofv3 FETCH_SIZE x 2.0
    # + WRITE_SIZE x 1.0 (KiB, the factors a plain 1 GiB copy reads), summed over the three k_pcg3 instances (nx 6,
    # 14, 26) of one solve at 256 threads / 48 336 B
    ("batch4096_ragged", "sym", "fp32_refine64", 0):
        ("7832a2dd28d9765a", ((8431864.3125 + 2908337.1875 + 148507.75) * 2.0
                              + (2916113.21875 + 1499994.59375 + 41748.65625) * 1.0) * 1024),
}

# The KKT step's HBM bytes per call, the same counters and factors, summed
# over the kernels of the three state sizes (nx 26, 14, 6): (sources
# sha256[:16], right-hand side bytes, recovery bytes)
KKT_SOURCES = ("kkt.hip", "ssp_host.h", "host.hip")
MEASURED_KKT_TRAFFIC = {
    "batch4096_ragged": ("f647674a887fd787",
                         ((1431882.47 + 443152.46 + 90428.95) * 2.0 + (38557.83 + 21607.56 + 9358.26) * 1.0) * 1024,
                         ((1521470.02 + 464100.26 + 92836.45) * 2.0 + (65205.94 + 34264.34 + 14283.5) * 1.0) * 1024),
}


def solve_sources_hash(sources=SOLVE_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2309_06427_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(b, iters, outer, pc: str, precision: str, kernel: int = 0, onchip=None) -> np.ndarray:
    """Bytes the solve must stream per problem in the library's storage format:
    every stored block element each pass reads, once per pass, plus gamma in
    and lambda out once.  D_k and D_k^-1 are symmetric and stored packed
    (nx(nx+1)/2 elements), L_k full (nx^2); L_0 and Phi^-1[0][-1] do not
    exist and are not counted.

    fused kernel (2): each inner solve makes iters + 1 passes over D, L and
    D^-1; explicit kernel (1): iters passes over S (D, L) and Phi^-1 (D^-1,
    explicit sub-diagonal blocks M_k, full) plus one initial Phi^-1 pass.
    Every FP64 residual reads D and L in FP64 (or FP32 hi + FP32 lo); a zero
    start needs no residual before its first inner solve (the fused kernel),
    so there are `outer` residual sweeps, `outer + 1` for the explicit one.
    cooperative kernel (3): the blocks are read once into LDS and stay there;
    each FP64 residual reads only the FP32 lo parts (none under FP64 storage).
    scaled kernel (4): see scaled_bytes (blocks and vectors); this returns
    their sum.
    """
    if kernel == 4:
        blk, vec = scaled_bytes(b, iters, outer, precision, onchip)
        return blk + vec
    N = b.N.astype(np.float64)
    nx = b.nx.astype(np.float64)
    nn = nx * nx
    npk = nx * (nx + 1) / 2
    e = 8.0 if precision == "fp64" else 4.0
    it = iters.astype(np.float64)
    st = outer.astype(np.float64)
    if kernel == 3:
        lo = 0.0 if precision == "fp64" else 4.0
        return e * (N * 2 * npk + (N - 1) * nn) + lo * st * (N * npk + (N - 1) * nn) + 16.0 * N * nx
    if kernel == 2:
        inner = e * (N * 2 * npk + (N - 1) * nn) * (it + st)
        sweeps = st
    else:
        nbS = N * npk + (N - 1) * nn
        nbP = N * npk if pc == "bj" else N * npk + (N - 1) * nn
        inner = e * (it * (nbS + nbP) + st * nbP)
        sweeps = st + 1
    return inner + 8.0 * sweeps * (N * npk + (N - 1) * nn) + 16.0 * N * nx


def onchip_mask(b, pc: str, precision: str, mapping) -> np.ndarray:
    """Problems whose six recurrence vectors the scaled solve keeps in LDS,
    by the library's own rule for the scaled mapping (threads, lds_bytes)."""
    from paper_2309_06427_amd import solver
    hor = {int(x): solver.scaled_onchip_horizon(int(x), pc, precision, mapping[0], mapping[1])
           for x in np.unique(b.nx)}
    return np.array([int(b.N[i]) <= hor[int(b.nx[i])] for i in range(b.P)], dtype=bool)


def scaled_bytes(b, iters, outer, precision: str, onchip=None):
    """Bytes the scaled solve must move per problem, split into block bytes
    and vector bytes.  Per PCG pass (iters + outer passes: one initial pass
    per inner solve) it streams Oh_k (N - 1 blocks of nx^2 in the storage
    type); the update pass reads and writes the six recurrence vectors
    (12 e bytes per row), the initial pass reads the FP64 scaled residual and
    writes x, r, u, w (8 + 4 e).  Each outer step reads Z_k twice (N full
    blocks, the forward and back transform), forms the true residual from D
    (packed) and L in FP64 (hi + lo, or FP64) except for a zero start's first
    step, and moves FP64 vectors: residual 24 B per row (lambda, gamma in,
    r out), transforms 16 + 8 + e + 16 B per row (r in, rh out; x in, lambda
    read and written).  Once per solve: gamma read for its norm and lambda
    zeroed (16 B per row).  Problems in `onchip` keep the six recurrence
    vectors in LDS: no vector bytes per update pass, the initial pass reads
    only the FP64 residual and the back transform does not read x."""
    N = b.N.astype(np.float64)
    nx = b.nx.astype(np.float64)
    nn = nx * nx
    npk = nx * (nx + 1) / 2
    e = 8.0 if precision == "fp64" else 4.0
    it = iters.astype(np.float64)
    st = outer.astype(np.float64)
    rows = N * nx
    passes = it + st
    sweeps = np.maximum(st - 1, 0)  # zero start: the first outer step takes gamma as its residual
    blk = e * (N - 1) * nn * passes + 2 * e * N * nn * st + 8.0 * (N * npk + (N - 1) * nn) * sweeps
    ve = np.where(onchip, 0.0, e) if onchip is not None else e  # storage-type vector bytes per element in HBM
    vec = (rows * (12 * ve * it + (8 + 4 * ve) * st) + rows * (24.0 * sweeps + (40.0 + ve) * st) + 16.0 * rows)
    return blk, vec


def kkt_bytes(b):
    """Bytes the two KKT calls must move per problem, all FP64: each knot
    block they read once (Q_k^-1 on N knots; A_k, B_k and R_k^-1 on the
    N - 1 knots that have a successor) and each vector element once.
    Right-hand side: q, c in, r of N - 1 knots in, gamma out.  Recovery:
    q, lambda in, r of N - 1 knots in, dx and du out."""
    N = b.N.astype(np.float64)
    nx = b.nx.astype(np.float64)
    nu = b.nu.astype(np.float64)
    blocks = 8.0 * (N * nx * nx + (N - 1) * (nx * nx + nx * nu + nu * nu))
    rhs = blocks + 8.0 * (3 * N * nx + (N - 1) * nu)
    rec = blocks + 8.0 * (3 * N * nx + (N - 1) * nu + N * nu)
    return rhs, rec


def load_nets(b, warm: str) -> list:
    """Trained warm-start networks for the state sizes in the batch."""
    from paper_2309_06427_amd.train_warmstart import weights_path
    from paper_2309_06427_amd.warmstart import WarmStartNet
    nets = []
    for nx in sorted(set(int(x) for x in b.nx)):
        path = weights_path(nx)
        if os.path.exists(path):
            nets.append(WarmStartNet.load(path))
        elif warm == "learned":
            raise SystemExit(f"bench.py: no trained warm-start weights for nx={nx} ({path})")
    return nets


def cpu_baseline(b, pc, precision, tol, sample: int, sample1: int = 64) -> dict:
    """The oracle (build + the same PCG) on the host: all cores on the first
    `sample` problems and one core on the first `sample1`, each the best of
    three runs of at least 1 s; the build alone is timed the same way."""
    import oracle

    def best_rate(fn, count):
        fn()  # warm-up (and compiles the oracle if needed)
        best = 0.0
        for _ in range(3):
            done, t0 = 0, time.perf_counter()
            while True:
                fn()
                done += count
                el = time.perf_counter() - t0
                if el >= 1.0:
                    break
            best = max(best, done / el)
        return best

    sub = b.subset(range(min(sample, b.P)))
    sub1 = b.subset(range(min(sample1, b.P)))
    cores = oracle.get_threads()
    full = best_rate(lambda: oracle.solve_batch(sub, pc, precision, tol=tol), sub.P)
    build = best_rate(lambda: oracle.build_batch(sub, pc), sub.P)
    oracle.set_threads(1)
    try:
        full1 = best_rate(lambda: oracle.solve_batch(sub1, pc, precision, tol=tol), sub1.P)
        build1 = best_rate(lambda: oracle.build_batch(sub1, pc), sub1.P)
    finally:
        oracle.set_threads(cores)
    return {"value": round(full, 2), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"first {sub.P} problems of the batch, build + {precision} PCG to {tol:g}, OpenMP over "
                      f"problems, best of 3 runs of >= 1 s; one core: first {sub1.P} problems",
            "build_only_per_s": round(build, 2),
            "one_core": {"value": round(full1, 2), "build_only_per_s": round(build1, 2),
                         "build_ms_per_problem": round(1e3 / build1, 4),
                         "solve_ms_per_problem": round(1e3 / full1 - 1e3 / build1, 4)}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch4096_ragged")
    ap.add_argument("--pc", default="sym", choices=["sym", "add", "bj", "jacobi", "poly2", "poly3"])
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "fp32", "fp32_refine64"])
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--lds", type=int, default=0)
    ap.add_argument("--kernel", type=int, default=0, help="0 automatic (fused; cooperative for one long problem), 1 explicit two sweeps, 2 fused, "
                         "3 cooperative")
    ap.add_argument("--keep-inverses", action="store_true",
                    help="builds of the timed step also store Q^-1, R^-1 for the KKT step (the step does not use them)")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the per-preconditioner runs and the KKT step timing")
    ap.add_argument("--warm", default="auto", choices=["auto", "zero", "learned"],
                    help="learned: also run the step with the trained warm-start networks "
                         "(auto: when their weights are present); the analytic start runs unless zero")
    ap.add_argument("--mapping", default="",
                    help="fixed mapping instead of autotuning: per state size nx:threads:lds,... for the "
                         "fused solve, or scaled:threads:lds for the scaled solve")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default mapping instead of timing candidates per state size first")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="time eager launches only (default: also replay the step as a HIP graph)")
    ap.add_argument("--stream-calib", type=int, default=0, metavar="MIB",
                    help="print the read / write / copy rates of plain device kernels on MIB-sized buffers")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration "
                         "and measured copy bandwidth), print one JSON line and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "problems are independent and would shard across GPUs by problem, "
              "which is not implemented here", file=sys.stderr)
        return 2

    import torch

    from paper_2309_06427_amd import inputs, solver

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.stream_calib:
        # practical streaming rates of plain device kernels: read (sum), write (fill), copy
        n = args.stream_calib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        out = {}
        from paper_2309_06427_amd import _lib

        lib = _lib.load()

        def own_copy():
            _lib.check(lib.ssp_copy_bytes(x.data_ptr(), y.data_ptr(), n * 4,
                                          torch.cuda.current_stream().cuda_stream), "ssp_copy_bytes")

        for name, fn, moved in (("read", lambda: x.sum(), n * 4), ("write", lambda: y.fill_(1.0), n * 4),
                                ("copy", lambda: y.copy_(x), 2 * n * 4), ("own_copy", own_copy, 2 * n * 4)):
            for _ in range(3):
                fn()
            best = float("inf")
            for _ in range(10):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1))
            out[name + "_GBps"] = round(moved / best / 1e6, 1)
        print(json.dumps({"stream_bytes": n * 4, **out}), flush=True)
        return 0
    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": reps + 3,
                          "ms": ms, "GBps_read_plus_write": 2 * n * 4 / ms / 1e6}), flush=True)
        return 0
    w = inputs.WORKLOADS[args.workload]
    precision = args.precision or w.get("precision", "fp32_refine64")
    tol = w["tol"]
    t0 = time.perf_counter()
    b = inputs.make(args.workload)
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {args.workload}: {b.P} problems in {gen_s:.1f} s", file=sys.stderr, flush=True)

    db = solver.DeviceBatch(b)
    db.solver.set_keep_inverses(args.keep_inverses)
    if args.threads or args.kernel:
        db.solver.set_mapping(args.threads or 128, args.lds, args.kernel)
    stream = torch.cuda.current_stream()
    mapping = None
    if args.mapping:
        # a fixed per-state-size mapping, "nx:threads:lds,..." (e.g. from an earlier autotune)
        db.build(args.pc, precision)
        for item in args.mapping.split(","):
            if item.startswith("scaled:"):
                t_, l_ = (int(v) for v in item.split(":")[1:])
                db.solver.set_scaled_mapping(t_, l_)
                continue
            nx_, t_, l_ = (int(v) for v in item.split(":"))
            db.solver.set_group_mapping(nx_, t_, l_)
        mapping = db.solver.mapping()
    elif args.autotune and not (args.threads or args.lds or args.kernel):
        db.build(args.pc, precision)
        mapping = db.autotune(tol)
        print(f"[bench] autotuned mapping (nx, threads, lds, ms): {mapping}", file=sys.stderr, flush=True)
    else:
        mapping = db.solver.mapping()
    nets = load_nets(b, args.warm) if args.warm != "zero" else []
    # analytic start: lambda0 = alpha Phi^-1 gamma with the energy-optimal
    # alpha, which is the first PCG iterate from zero (one capped solve)
    modes = ["plain"] + (["analytic"] if args.warm != "zero" else []) + (["learned"] if nets else [])

    def step(mode, ev=None):
        if ev:
            ev[0].record(stream)
        db.build(args.pc, precision)
        if ev:
            ev[1].record(stream)
        if mode == "learned":
            db.lam.zero_()
            for net in nets:
                net.predict(db)
            if ev:
                ev[2].record(stream)
            db.solve(tol, warm_in_place=True, fallback=True)
        elif mode == "analytic":
            db.solve(tol, max_iter=1)
            if ev:
                ev[2].record(stream)
            db.solve(tol, warm_in_place=True, fallback=True)
        else:
            if ev:
                ev[2].record(stream)
            db.solve(tol)
        if ev:
            ev[3].record(stream)

    runs = {}
    for mode in modes:
        for _ in range(args.warmup):
            step(mode)
        torch.cuda.synchronize()
        # eager steps with per-phase events
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.steps):
            step(mode, ev[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        ph = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])] for e in ev])
        res = db.results()
        run = dict(wall=wall, build_ms=ph[:, 0], predict_ms=ph[:, 1], solve_ms=ph[:, 2], res=res)
        if args.graph:
            # the same step captured once into a HIP graph and replayed
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            with torch.cuda.stream(side):
                step(mode)  # allocations and lazily built lists happen outside the capture
            stream.wait_stream(side)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                step(mode)
            g.replay()
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            for k in range(args.steps):
                g.replay()
            torch.cuda.synchronize()
            run["graph_wall"] = time.perf_counter() - t_start
            gres = db.results()
            run["graph_matches_eager"] = bool(np.array_equal(gres["lam"], res["lam"]) and
                                              np.array_equal(gres["iters"], res["iters"]))
            del g
        runs[mode] = run
        print(f"[bench] {mode}: {args.steps} steps eager {wall:.3f} s"
              + (f", graph {run['graph_wall']:.3f} s" if args.graph else ""), file=sys.stderr, flush=True)

    plain = runs["plain"]
    res = plain["res"]
    # headline: the faster of the two ways to run the step (both are reported)
    def step_wall(r):
        return r.get("graph_wall", r["wall"])
    head_mode = min(runs, key=lambda m: step_wall(runs[m]))
    head = runs[head_mode]
    head_wall = step_wall(head)
    ok = bool(all(((r["res"]["status"] & ~24) == 0).all() and r["res"]["relres"].max() <= tol
                  for r in runs.values()))
    if args.graph:
        ok = ok and all(r["graph_matches_eager"] for r in runs.values())
    kern, coop_w, coop_g = db.solver.solve_kernel()  # the kernel the solves ran: 1 explicit, 2 fused, 3 cooperative
    oc = onchip_mask(b, args.pc, precision, db.solver.scaled_mapping()) if kern == 4 else None
    bytes_solve = float(algorithmic_bytes(b, res["iters"], res["outer"], args.pc, precision, kern, oc).sum())
    split = None
    if kern == 4:
        bb, vb = scaled_bytes(b, res["iters"], res["outer"], precision, oc)
        split = {"block_bytes": float(bb.sum()), "vector_bytes": float(vb.sum()),
                 "problems_with_vectors_in_lds": int(oc.sum())}
    rec = MEASURED_TRAFFIC.get((args.workload, args.pc, precision, args.kernel))
    traffic = rec[1] if rec and rec[0] == solve_sources_hash() else None
    solve_avg_s = float(plain["solve_ms"].mean()) / 1e3
    achieved = bytes_solve / solve_avg_s / 1e9
    value = b.P * args.steps / head_wall

    def timed(fn, reps):
        """Mean HIP-event time of fn() on the stream, ms, after one untimed call."""
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    compare = None
    if not args.no_compare:
        # every preconditioner on the same batch and precision: build and
        # solve timed apart, the solve's algorithmic bytes for the kernel it ran
        compare = {}
        for pc in ("jacobi", "bj", "add", "sym", "poly3"):
            build_ms = timed(lambda: db.build(pc, precision), 3)
            solve_ms = timed(lambda: db.solve(tol), 3)
            r = db.results()
            pk = db.solver.solve_kernel()[0]
            oc = onchip_mask(b, pc, precision, db.solver.scaled_mapping()) if pk == 4 else None
            by = float(algorithmic_bytes(b, r["iters"], r["outer"], pc, precision, pk, oc).sum())
            compare[pc] = {"iters_mean": round(float(r["iters"].mean()), 3),
                           "outer_mean": round(float(r["outer"].mean()), 3),
                           "max_relres": float(r["relres"].max()),
                           "pc_fallbacks": int(((r["status"] & 16) != 0).sum()),
                           "kernel": {1: "explicit", 2: "fused", 3: "cooperative", 4: "scaled"}[pk],
                           "build_ms": round(build_ms, 4),
                           "solve_ms": round(solve_ms, 4),
                           "solves_per_s": round(b.P / ((build_ms + solve_ms) / 1e3), 2),
                           "solve_algorithmic_bytes": by,
                           "solve_GBps": round(by / solve_ms / 1e6, 2),
                           "solve_frac": round(by / solve_ms / 1e6 / HBM_PEAK_GBS, 4)}

    kkt = None
    if not args.no_compare:
        # the KKT step around the solve (right-hand side, then recovery) on
        # the same batch after a build with the headline preconditioner;
        # gamma is restored afterwards
        gamma0 = db.gamma.clone()
        db.solver.set_keep_inverses(True)  # the KKT calls read Q^-1, R^-1 of the build
        kbuild_ms = timed(lambda: db.build(args.pc, precision), 3)
        gen = torch.Generator(device="cpu").manual_seed(11)
        nu_rows = int((b.N.astype(np.int64) * b.nu).sum())
        q = torch.randn(int(b.off_v[-1]), dtype=torch.float64, generator=gen).cuda()
        c = torch.randn(int(b.off_v[-1]), dtype=torch.float64, generator=gen).cuda()
        r = torch.randn(max(nu_rows, 1), dtype=torch.float64, generator=gen).cuda()
        rhs_ms = timed(lambda: db.kkt_rhs(q, r, c), 10)
        db.solve(tol)
        dx = torch.empty_like(db.gamma)
        du = torch.empty(max(nu_rows, 1), dtype=torch.float64, device=dx.device)
        rec_ms = timed(lambda: db.solver.kkt_recover(db.A, db.B, q, r, db.lam, dx, du), 10)
        rb, cb = (float(x.sum()) for x in kkt_bytes(b))
        krec = MEASURED_KKT_TRAFFIC.get(args.workload)
        kt = krec[1:] if krec and krec[0] == solve_sources_hash(KKT_SOURCES) else (None, None)
        kkt = {"build_ms_keeping_inverses": round(kbuild_ms, 4),
               "rhs_ms": round(rhs_ms, 4), "recover_ms": round(rec_ms, 4),
               "rhs_algorithmic_bytes": rb, "recover_algorithmic_bytes": cb,
               "rhs_GBps": round(rb / rhs_ms / 1e6, 2), "recover_GBps": round(cb / rec_ms / 1e6, 2),
               "rhs_frac": round(rb / rhs_ms / 1e6 / HBM_PEAK_GBS, 4),
               "recover_frac": round(cb / rec_ms / 1e6 / HBM_PEAK_GBS, 4),
               "rhs_traffic": kt[0], "recover_traffic": kt[1]}
        db.gamma.copy_(gamma0)
        db.solver.set_keep_inverses(args.keep_inverses)
        del gamma0, q, c, r, dx, du

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(b, args.pc, precision, tol, args.cpu_sample)

    def summary(r):
        d = {"solves_per_s": round(b.P * args.steps / r.get("graph_wall", r["wall"]), 2),
             "ms_per_step_eager": round(r["wall"] * 1e3 / args.steps, 4),
             "build_ms": round(float(r["build_ms"].mean()), 4),
             "predict_ms": round(float(r["predict_ms"].mean()), 4),
             "solve_ms": round(float(r["solve_ms"].mean()), 4),
             "iters_mean": round(float(r["res"]["iters"].mean()), 3),
             "outer_mean": round(float(r["res"]["outer"].mean()), 3),
             "max_relres": float(r["res"]["relres"].max()),
             "iters_p50": float(np.percentile(r["res"]["iters"], 50)),
             "iters_p99": float(np.percentile(r["res"]["iters"], 99)),
             "fallbacks": int(((r["res"]["status"] & 8) != 0).sum()),
             "pc_fallbacks": int(((r["res"]["status"] & 16) != 0).sum())}
        if "graph_wall" in r:
            d["ms_per_step_graph"] = round(r["graph_wall"] * 1e3 / args.steps, 4)
            d["graph_matches_eager"] = r["graph_matches_eager"]
        return d

    out = {
        "metric": "PCG solves/sec & HBM GB/s at rel-res 1e-6, sym-stair, batched+learned vs plain",
        "value": round(value, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head_wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "problems": b.P,
            "knots_total": int(b.N.sum()),
            "preconditioner": args.pc,
            "precision": precision,
            "tol": tol,
            "warm_start": {"learned": "learned (per-knot network, zero fallback)",
                           "analytic": "analytic (alpha Phi^-1 gamma, zero fallback)"}.get(head_mode, "zero"),
            "kernel": {1: "explicit", 2: "fused", 3: "cooperative", 4: "scaled"}[kern],
            "mapping": ({"own_knots_per_workgroup": coop_w, "workgroups": coop_g} if kern == 3 else
                        dict(zip(("threads", "lds_bytes", "persistent_workgroups"), db.solver.scaled_mapping()[:3]))
                        if kern == 4 else
                        [{"nx": m[0], "threads": m[1], "lds_bytes": m[2]} for m in mapping] if mapping else None),
            "timing": "hipGraph replay of the whole step" if args.graph else "eager launches",
            "step": ("build (FP64 assembly) + network inference + solve" if head_mode == "learned"
                     else "build (FP64 assembly) + analytic start + solve" if head_mode == "analytic"
                     else "build (FP64 assembly) + solve"),
        },
        "valid": ok,
        "detail": {
            "plain": summary(plain),
            "learned": summary(runs["learned"]) if "learned" in runs else None,
            "analytic": summary(runs["analytic"]) if "analytic" in runs else None,
            "solve_only_solves_per_s": round(b.P / solve_avg_s, 2),
            "solve_algorithmic_bytes": bytes_solve,
            "solve_bytes_split": split,
            "compare": compare,
            "kkt": kkt,
        },
        "roofline": {
            "kernel": {1: "k_pcg", 2: "k_pcg2", 3: "k_coop", 4: "k_pcg3"}[kern],
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            **({"note": "latency-bound: blocks stay in LDS, one grid-wide sum per PCG iteration"}
               if kern == 3 else
               {"note": "one persistent instance per state size, run concurrently; achieved and traffic cover "
                        "all of them over the solve phase"} if kern == 4 else {}),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    # free the library handles before interpreter shutdown
    for net in nets:
        net.close()
    db.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
