"""Benchmark: coarse solves/s to relative residual 1e-8 on one MI355X.

Workload: the synthetic 8^4 coarse operator with N_tv = 24 (196,608 unknowns,
clover-Wilson type, m0 from the limiting spectral disk with min Re / max|.| =
1e-4), seeded right-hand sides.
A step is one complete coarse solve of a fresh right-hand side with the
method's solver: polynomial preconditioning (d Leja-ordered harmonic Ritz
values) + GCRO-DR deflation/recycling (k vectors), reduced-precision inner
solve inside an FP64 flexible-GMRES outer loop; the FP64 true residual of
every solve is checked.  Plain FP64 GMRES(30) is run on the same operator and
right-hand sides for comparison (capped: on this operator it can stagnate).
The roofline entry is the kernel that streams the stored blocks in the method's
applies (on the odd-even reduced system, the A_e - D_eo kernel), timed live in
the timed solves with HIP events on the library's launch stream.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coarse solves/s to rel.res 1e-8 (plain FP64 vs poly+defl mixed); D_c GB/s"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=16)
    p.add_argument("--warmup", type=int, default=2,
                   help="untimed solves before the timed ones; two complete the recycle "
                        "space's u = 10 refreshes (the setup phase), so the timed solves "
                        "see it frozen")
    p.add_argument("--workload", default="c2")
    p.add_argument("--tol", type=float, default=1e-8)
    p.add_argument("--inner", default="f16s", choices=["f32", "f16s"])
    p.add_argument("--d", type=int, default=32)
    p.add_argument("--k", type=int, default=96)
    p.add_argument("--schur", type=int, default=1, choices=[0, 1],
                   help="solve the odd-even reduced system (1) or the full lattice (0)")
    p.add_argument("--full-steps", type=int, default=4,
                   help="timed solves of the same method on the full lattice, for comparison")
    p.add_argument("--m", type=int, default=30, help="new Arnoldi vectors per cycle")
    p.add_argument("--ortho", type=int, default=1, choices=[0, 1],
                   help="Arnoldi: 0 Gram-Schmidt twice, 1 single-sync (one reduction per step)")
    p.add_argument("--ss-steps", type=int, default=4,
                   help="timed solves of the same method with the other --ortho choice")
    p.add_argument("--inner-tol", type=float, default=1e-1)
    p.add_argument("--plain-steps", type=int, default=1)
    p.add_argument("--plain-max-cycles", type=int, default=400,
                   help="restart cycles of the plain GMRES(30) comparison (it may stagnate)")
    p.add_argument("--apply-reps", type=int, default=50)
    p.add_argument("--multi-rhs", type=int, default=64,
                   help="right-hand sides of the multi-RHS (MFMA) apply measurement (0: skip)")
    p.add_argument("--profile-every", type=int, default=8,
                   help="time one in this many launches of the apply's block kernel (0: off)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--summarize-trace", default=None, metavar="CSV",
                   help="only summarise a rocprofv3 kernel_trace.csv: per-kernel launches and "
                        "mean duration over launches longer than --min-us (launches that did work)")
    p.add_argument("--min-us", type=float, default=8.0)
    p.add_argument("--copy-probe", type=int, default=0, metavar="MiB",
                   help="only run a plain elementwise copy of this many MiB (read + write), "
                        "the reference for scaling HBM byte counters")
    return p.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def apply_bytes(V, n, prec):
    """Algorithmic bytes of one D_c apply: the 5 stored blocks per site (plus
    their FP16 scales), one read of the input and one write of the output."""
    sb = {"f64": 16, "f32": 8, "f16s": 4}[prec]
    sv = 16 if prec == "f64" else 8
    extra = 5 * 4 if prec == "f16s" else 0
    return V * (5 * n * n * sb + 2 * n * sv + extra)


def stage1_bytes(V, n, prec):
    """Algorithmic bytes of the apply's block kernel: the stored blocks (and
    scales) plus one read of the input vector; its per-coupling partial
    products are an intermediate of this design, not counted."""
    sb = {"f64": 16, "f32": 8, "f16s": 4}[prec]
    sv = 16 if prec == "f64" else 8
    extra = 5 * 4 if prec == "f16s" else 0
    return V * (5 * n * n * sb + n * sv + extra)


# HBM traffic of one launch of the roofline kernel on the 8^4, N_tv = 24
# workload with FP16 blocks (kernel 2: the reduced operator's A_e - D_eo
# kernel): rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (KiB per dispatch,
# median over the 3439 launches that did work, almost all later chain steps),
# each scaled by the ratio of true bytes to counter reading for a plain 1 GiB
# elementwise copy (--copy-probe 1024: FETCH_SIZE 524300 KiB for 1 GiB read,
# WRITE_SIZE 1048576 KiB for 1 GiB written).  Valid only for the apply source
# it was taken on.
TRAFFIC = {"workload": "c2", "prec": "f16s", "kernel": 2,
           "fetch_kib": 85536.4375, "fetch_scale": 1048576.0 / 524300.0,
           "write_kib": 1536.0, "write_scale": 1048576.0 / 1048576.0,
           "apply_source_sha256": "5c0bd7055b182519b7fa68ec2d705e971feff8dffbdb3ffb1659f6be9aa48858"}


def apply_source_digest():
    """sha256 of the apply section (block and gather kernels) of the HIP source."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_2205_09104_amd", "csrc", "kernels.hip")).read()
    a = re.search(r"^// -+ apply$", src, re.M).start()
    b = re.search(r"^// -+ block Jacobi$", src, re.M).start()
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def reduced_block_bytes(V, n, prec):
    """Block bytes of one launch of either kernel of the reduced operator: per
    row (V/2 of them) nine blocks and their FP16 scales -- the A_o^{-1} D_oe
    kernel reads the 8 hop blocks of an odd site and its self-block inverse,
    the A_e - D_eo kernel the 8 hop blocks of an even site and its self block."""
    sb = {"f64": 16, "f32": 8, "f16s": 4}[prec]
    extra = 9 * 4 if prec == "f16s" else 0
    return (V // 2) * (9 * n * n * sb + extra)


def reduced_vec_bytes(V, n, prec):
    """Bytes of one vector pass over the V/2 rows of a compressed vector."""
    return (V // 2) * n * (16 if prec == "f64" else 8)


def reduced_apply_bytes(V, n, prec):
    """Algorithmic bytes of one apply of the reduced operator: both kernels'
    blocks, one read of the input and one write of the output (the odd-row
    temporary between the kernels is this design's)."""
    return 2 * reduced_block_bytes(V, n, prec) + 2 * reduced_vec_bytes(V, n, prec)


def measured_traffic(workload, prec, kernel):
    t = TRAFFIC
    if (workload != t["workload"] or prec != t["prec"] or kernel != t["kernel"]
            or apply_source_digest() != t["apply_source_sha256"]):
        return None, None
    fetch = t["fetch_kib"] * 1024 * t["fetch_scale"]
    write = t["write_kib"] * 1024 * t["write_scale"]
    return fetch + write, {"fetch_bytes": fetch, "write_bytes": write,
                           "fetch_scale": t["fetch_scale"], "write_scale": t["write_scale"]}


def main():
    a = parse()
    if a.summarize_trace:
        summarize_trace(a.summarize_trace, a.min_us)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is a design only)"}))
        sys.exit(2)
    import torch

    if a.copy_probe:
        copy_probe(a.copy_probe)
        return

    import synth
    from paper_2205_09104_amd import CoarseOp, Opts

    torch.cuda.set_device(0)
    w = synth.WORKLOADS[a.workload]
    V, n = w.V, w.n
    log(f"workload {w.name}: dims {w.dims} n {n} N {w.N} m0 {w.m0():.6f}")
    t0 = time.time()
    A, B = synth.operator(w, device="cuda")
    op = CoarseOp(A, B, w.dims, mu=w.mu, store=("f64", "f32", "f16s"))
    del A, B
    torch.cuda.synchronize()
    log(f"operator built in {time.time() - t0:.1f}s")
    # the library launches on torch's current stream (the HIP null stream here)
    stream = torch.cuda.current_stream()
    # HIP events on one in a.profile_every launches of the apply's block kernel
    op.profile_apply(a.profile_every)

    kern = 2 if a.schur else 0     # the roofline kernel: D_eo stage, or the full block kernel

    def prof_totals(kernel=None):
        kk = kern if kernel is None else kernel
        return {p: (op.profile_apply_read(p, kernel=kk),
                    op.profile_apply_read(p, include_noops=True, kernel=kk))
                for p in ("f64", "f32", "f16s")}

    # ------------------------------------------------ back-to-back apply rates
    def apply_rate(prec):
        x = synth.rhs(w.dims, w.n_tv, 999, device="cuda")
        x = x if prec == "f64" else x.to(torch.complex64)
        out = torch.empty_like(x)
        for _ in range(3):
            op.apply(x, prec=prec, out=out)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(a.apply_reps):
            op.apply(x, prec=prec, out=out)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / a.apply_reps
        return ms, apply_bytes(V, n, prec) / (ms * 1e-3) / 1e9

    rates = {p: apply_rate(p) for p in ("f64", "f32", "f16s")}
    for p, (ms, gbs) in rates.items():
        log(f"apply {p} (both stages, back to back): {ms * 1e3:.1f} us, {gbs:.0f} GB/s algorithmic")

    def reduced_rate(prec):
        x = synth.rhs(w.dims, w.n_tv, 998, device="cuda")[: V // 2]
        x = x if prec == "f64" else x.to(torch.complex64)
        out = torch.empty_like(x)
        for _ in range(3):
            op.apply_reduced(x, prec=prec, out=out)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(a.apply_reps):
            op.apply_reduced(x, prec=prec, out=out)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / a.apply_reps
        return ms, reduced_apply_bytes(V, n, prec) / (ms * 1e-3) / 1e9

    rrates = {}
    if a.schur:
        rrates = {p: reduced_rate(p) for p in ("f64", "f32", "f16s")}
        for p, (ms, gbs) in rrates.items():
            log(f"reduced apply {p} (both kernels, back to back): {ms * 1e3:.1f} us, "
                f"{gbs:.0f} GB/s algorithmic")

    # ------------------------------------------------ multi-RHS (MFMA) apply
    multi = {}
    if a.multi_rhs > 0:
        R = a.multi_rhs
        flops = 72.0 * V * n * n * R           # complex n x n times n x R per coupling, 9 couplings
        for p, peak in (("f64", 78.6), ("f32", 157.3), ("f16s", 157.3)):
            X = torch.stack([synth.rhs(w.dims, w.n_tv, 500 + r, device="cuda") for r in range(R)])
            X = X if p == "f64" else X.to(torch.complex64)
            Y = torch.empty_like(X)
            for _ in range(2):
                op.apply_multi(X, prec=p, out=Y)
            times = []
            for _ in range(5):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                op.apply_multi(X, prec=p, out=Y)
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = sorted(times)[2]
            tf = flops / (ms * 1e-3) / 1e12
            multi[p] = {"n_rhs": R, "ms": ms, "TFLOP/s": tf, "peak": peak, "frac": tf / peak,
                        "mfma": "f64 16x16x4" if p == "f64" else "f32 16x16x4"}
            log(f"multi-RHS apply {p} R={R}: {ms:.3f} ms, {tf:.1f} TFLOP/s ({100 * tf / peak:.1f}% of {peak})")
            del X, Y

    # ------------------------------------------------ method solve (timed)
    opts = Opts(m=a.m + a.k, k=a.k, d=a.d, u=10, prec=a.inner, outer=1, m_outer=10,
                max_outer=50, inner_tol=a.inner_tol, seed=1, max_cycles=100000, schur=a.schur,
                ortho=a.ortho)

    def one_solve(r, o):
        b = synth.rhs(w.dims, w.n_tv, r, device="cuda")
        x, st, rc = op.solve(b, a.tol, o)
        return x, st[0], rc

    setup_ms = 0.0
    for r in range(a.warmup):
        x, st, rc = one_solve(r, opts)
        setup_ms += st["t_setup_ms"]
        log(f"warmup solve {r}: rc {rc} relres {st['rel_res_true']:.2e} iters {st['iters']} "
            f"matvecs {st['matvecs']} setup {st['t_setup_ms']:.0f} ms")
    rhs = [synth.rhs(w.dims, w.n_tv, r, device="cuda") for r in range(a.warmup, a.warmup + a.steps)]
    torch.cuda.synchronize()
    pre = prof_totals()
    pre_oe = prof_totals(1)
    pre_pass = {p: (op.profile_apply_passes(p, kern), op.profile_apply_passes(p, 1))
                for p in ("f64", "f32", "f16s")}
    t0 = time.perf_counter()
    stats = []
    for b in rhs:
        x, st, rc = op.solve(b, a.tol, opts)
        stats.append(st[0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    x_last = x
    post = prof_totals()
    post_oe = prof_totals(1)
    # timed-region block-kernel launches that did work: (count, ms) per
    # precision, and their vector passes
    prof = {p: (post[p][0][0] - pre[p][0][0], post[p][0][1] - pre[p][0][1]) for p in post}
    prof_oe = {p: (post_oe[p][0][0] - pre_oe[p][0][0], post_oe[p][0][1] - pre_oe[p][0][1])
               for p in post_oe}
    passes = {p: op.profile_apply_passes(p, kern) - pre_pass[p][0] for p in pre_pass}
    passes_oe = {p: op.profile_apply_passes(p, 1) - pre_pass[p][1] for p in pre_pass}
    for i, st in enumerate(stats):
        log(f"timed solve {i}: status {st['status']} relres {st['rel_res_true']:.2e} "
            f"iters {st['iters']} matvecs {st['matvecs']} outer {st['outer_iters']} "
            f"{st['t_solve_ms']:.0f} ms")
    ok = all(s["status"] == 0 and s["rel_res_true"] <= a.tol for s in stats)
    value = a.steps / dt if ok else 0.0

    # ------------------------------------------------ same method, full lattice
    full_cmp = None
    if a.schur and a.full_steps > 0:
        fo = Opts(m=a.m + a.k, k=a.k, d=a.d, u=10, prec=a.inner, outer=1, m_outer=10,
                  max_outer=50, inner_tol=a.inner_tol, seed=1, max_cycles=100000, schur=0)
        for r in range(a.warmup):              # setup: polynomial and recycle space
            one_solve(r, fo)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fst = [one_solve(r, fo)[1] for r in range(a.warmup, a.warmup + a.full_steps)]
        torch.cuda.synchronize()
        fdt = time.perf_counter() - t1
        full_cmp = {"solves_per_s": a.full_steps / fdt, "steps": a.full_steps,
                    "matvecs_per_solve": [s["matvecs"] for s in fst],
                    "converged": all(s["status"] == 0 for s in fst)}
        log(f"same method on the full lattice: {a.full_steps / fdt:.2f} solves/s")

    # ------------------------------------------------ same method, single-sync Arnoldi
    ss_cmp = None
    if a.ss_steps > 0:
        so = Opts(m=a.m + a.k, k=a.k, d=a.d, u=10, prec=a.inner, outer=1, m_outer=10,
                  max_outer=50, inner_tol=a.inner_tol, seed=1, max_cycles=100000,
                  schur=a.schur, ortho=1 - a.ortho)
        for r in range(a.warmup):
            one_solve(r, so)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sst = [one_solve(r, so)[1] for r in range(a.warmup, a.warmup + a.ss_steps)]
        torch.cuda.synchronize()
        sdt = time.perf_counter() - t1
        ss_cmp = {"ortho": 1 - a.ortho, "solves_per_s": a.ss_steps / sdt, "steps": a.ss_steps,
                  "matvecs_per_solve": [s["matvecs"] for s in sst],
                  "iters_per_solve": [s["iters"] for s in sst],
                  "converged": all(s["status"] == 0 for s in sst)}
        log(f"same method with ortho={1 - a.ortho}: {a.ss_steps / sdt:.2f} solves/s")

    # ------------------------------------------------ FP64 comparisons (one RHS each)
    # GMRES(30) plain, with the polynomial preconditioner (d = 4, 8, 16), and
    # with polynomial + deflation; each capped near 12000 matvecs since the
    # plain and polynomial-only variants can stagnate on this operator.
    comp = {}
    if a.plain_steps > 0:
        cases = [("gmres30", Opts(m=30, prec="f64", max_cycles=a.plain_max_cycles))]
        for d in (4, 8, 16):
            cases.append((f"gmres30_poly_d{d}",
                          Opts(m=30, d=d, prec="f64", seed=1,
                               max_cycles=max(1, 12000 // (30 * d)))))
        cases.append(("gmres_poly_d16_defl_k32",
                      Opts(m=62, k=32, d=16, prec="f64", seed=1, max_cycles=400)))
        r = a.warmup
        for name, o in cases:
            if o.k > 0:
                one_solve(r + 1, o)           # setup solve: builds the recycle space
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, st, rc = one_solve(r, o)
            torch.cuda.synchronize()
            pdt = time.perf_counter() - t1
            conv = st["status"] == 0
            comp[name] = {"solves_per_s": (1.0 / pdt) if conv else 0.0, "converged": conv,
                          "iters": st["iters"], "matvecs": st["matvecs"],
                          "rel_res_true": st["rel_res_true"], "ms": 1e3 * pdt}
            log(f"fp64 {name}: status {st['status']} relres {st['rel_res_true']:.2e} "
                f"iters {st['iters']} matvecs {st['matvecs']} {1e3 * pdt:.0f} ms")
    plain = comp.get("gmres30", {"solves_per_s": None})

    # forward error of the last timed solve against an FP64 solve to 1e-12
    # (polynomial + deflation, FP64 throughout), outside the timed region
    ref_opts = Opts(m=62, k=32, d=16, prec="f64", seed=1, max_cycles=2000)
    xr, sr, _ = op.solve(rhs[-1], 1e-12, ref_opts)
    err_vs_fp64 = float(torch.linalg.vector_norm(x_last - xr) / torch.linalg.vector_norm(xr))
    log(f"forward error of the last solve vs FP64 (rel.res {sr[0]['rel_res_true']:.1e}): "
        f"{err_vs_fp64:.2e}")

    whole = prof_totals()     # the whole run so far, for comparison with a kernel tracer
    op.profile_apply(0)

    # ------------------------------------------------ CPU oracle baseline
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(w, a, stats, x_check=(x_last, rhs[-1]))

    inner = a.inner
    launches, tot_ms = prof[inner]
    avg_us = 1e3 * tot_ms / max(launches, 1)
    if a.schur:
        # per launch: the nine blocks per row, plus the vector passes of its
        # epilogue (2 to 5; summed over the timed launches by the library)
        s1b = (launches * reduced_block_bytes(V, n, inner) +
               passes[inner] * reduced_vec_bytes(V, n, inner)) / max(launches, 1)
    else:
        s1b = stage1_bytes(V, n, inner)
    achieved = s1b / (avg_us * 1e-6) / 1e9 if launches else None
    traffic, traffic_detail = measured_traffic(w.name, inner, kern)
    kname = (f"k_reduced_eo ({inner} blocks; A_e x_e - D_eo t_o with the chain epilogue)"
             if a.schur else f"k_apply_blocks ({inner} blocks)")
    oe = None
    if a.schur:
        l1, m1 = prof_oe[inner]
        if l1:
            b1 = (l1 * reduced_block_bytes(V, n, inner) +
                  passes_oe[inner] * reduced_vec_bytes(V, n, inner)) / l1
            oe = {"kernel": f"k_reduced_oe ({inner} blocks; t_o = A_o^-1 D_oe x_e)",
                  "timed_launches": l1, "avg_us": 1e3 * m1 / l1, "bytes_per_launch": b1,
                  "GB/s": b1 / (1e-3 * m1 / l1) / 1e9}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{inner} blocks, f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {'x'.join(map(str, w.dims))} lattice, N_tv={w.n_tv} "
                               f"({w.N} unknowns), mu={w.mu}, m0={w.m0():.6f}",
                   "solver": f"{'odd-even reduced system; ' if a.schur else ''}FGMRES(10) fp64 "
                             f"outer; inner {inner} GCRO-DR(m={a.m + a.k},k={a.k}) + poly "
                             f"d={a.d}, inner_tol={a.inner_tol}"
                             f"{', single-sync Arnoldi' if a.ortho else ''}",
                   "tol": a.tol, "parallelism": "single GPU"},
        "setup_ms": setup_ms,
        "iters_per_solve": [s["iters"] for s in stats],
        "matvecs_per_solve": [s["matvecs"] for s in stats],
        "rel_res_true": [s["rel_res_true"] for s in stats],
        "err_vs_fp64_last_solve": err_vs_fp64,
        "plain_fp64_gmres30": plain,
        "same_method_full_lattice": full_cmp,
        "same_method_other_ortho": ss_cmp,
        "fp64_comparison": comp,
        "apply_back_to_back": {p: {"us": r[0] * 1e3, "GB/s": r[1]} for p, r in rates.items()},
        "reduced_apply_back_to_back": {p: {"us": r[0] * 1e3, "GB/s": r[1]}
                                       for p, r in rrates.items()},
        "multi_rhs_apply": multi,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                     "traffic_detail": traffic_detail,
                     "kernel": f"{kname}, timed in the solves",
                     "traffic_GBs": (traffic / (avg_us * 1e-6) / 1e9) if (traffic and launches) else None,
                     "timed_launches": launches, "sampling": f"1 in {a.profile_every}",
                     "avg_us": avg_us, "bytes_per_launch": s1b,
                     "other_reduced_kernel": oe,
                     "f64_block_kernel": {"launches": prof["f64"][0],
                                          "avg_us": 1e3 * prof["f64"][1] / max(prof["f64"][0], 1)},
                     "whole_run_all_launches": {
                         p: {"timed_launches": whole[p][1][0],
                             "avg_us": 1e3 * whole[p][1][1] / max(whole[p][1][0], 1)}
                         for p in whole}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def summarize_trace(path, min_us):
    """Per kernel of a rocprofv3 kernel trace: all launches and their mean
    duration, and the same over launches longer than min_us (a finished
    Arnoldi cycle turns its remaining launches into near-empty ones)."""
    import csv
    import statistics
    d = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
            d.setdefault(name[:90], []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    rows = sorted(d.items(), key=lambda kv: -sum(kv[1]))[:20]
    print(f"{'kernel':90s} {'launches':>9s} {'mean_us':>8s} {'work':>9s} {'mean_us':>8s} {'median':>8s}")
    for k, v in rows:
        w = [x for x in v if x > min_us]
        print(f"{k:90s} {len(v):9d} {statistics.mean(v):8.2f} {len(w):9d} "
              f"{(statistics.mean(w) if w else 0):8.2f} {(statistics.median(w) if w else 0):8.2f}")


def copy_probe(mib):
    """y = 1.0 * x over mib MiB of float32, 5 launches: each reads and writes
    exactly mib MiB of HBM-resident data."""
    import torch
    torch.cuda.set_device(0)
    x = torch.ones(mib * (1 << 18), dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_MiB": mib, "launches": 5}), flush=True)


def cpu_baseline(w, a, stats, x_check=None):
    """The FP64 oracle on the host.  Sample: oracle D_c applies for about
    a.cpu_seconds; the oracle's solves/s is bounded above by one over (time per
    apply x matvecs the GPU method needed per solve), its orthogonalisation and
    setup not counted.  Also checks the last GPU solution's FP64 residual with
    the oracle apply."""
    import numpy as np

    import synth
    from oracle import operator as dop
    A, B = synth.operator(w)
    oop = dop.build(w.dims, A.numpy(), B.numpy(), w.mu)
    del A, B
    v = synth.rhs(w.dims, w.n_tv, 0).numpy()
    dop.apply(oop, v)
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < a.cpu_seconds:
        dop.apply(oop, v)
        reps += 1
    per_apply = (time.perf_counter() - t0) / reps
    mv = float(np.mean([s["matvecs"] for s in stats]))
    try:
        from threadpoolctl import threadpool_info
        blas = [{k: i.get(k) for k in ("internal_api", "num_threads")} for i in threadpool_info()]
    except Exception:  # noqa: BLE001
        blas = None
    out = {"value": 1.0 / (per_apply * mv), "unit": "solves/s", "cores": 1, "kind": "oracle",
           "host_cpus": os.cpu_count(), "blas_pools": blas,
           "sample": f"{reps} FP64 oracle D_c applies ({per_apply:.3f} s each, numpy einsum, one "
                     f"thread) x {mv:.0f} matvecs per solve of the GPU method; an upper bound "
                     f"(orthogonalisation and setup not counted)"}
    if x_check is not None:
        x, b = (t.cpu().numpy() for t in x_check)
        r = b - dop.apply(oop, x)
        out["oracle_relres_last_solve"] = float(np.linalg.norm(r) / np.linalg.norm(b))
    return out


if __name__ == "__main__":
    main()
