"""Benchmark: coarse solves/s to relative residual 1e-8 on one MI355X.

Workload (default): the synthetic 16^3 x 32 twisted-mass coarse operator with
N_tv = 24 (6,291,456 unknowns, mu = 1e-3, m0 from the limiting spectral disk
with min Re / max|.| = 1e-4), seeded Gaussian right-hand sides.
A step is one complete coarse solve of a fresh right-hand side with the
paper's coarsest-level method on the odd-even reduced system: left block
Jacobi with B = D_ee, polynomial preconditioning (d Leja-ordered harmonic Ritz
values of B^{-1} S) and GCRO-DR deflation / recycling (k vectors), as a
reduced-precision (FP16-stored blocks, FP32 arithmetic) inner solve inside an
FP64 flexible-GMRES outer loop; the FP64 true residual of every solve is
checked.  Plain FP64 GMRES(30) runs on the same operator and right-hand side
for comparison (capped by wall time: on this operator it stagnates).  The
roofline entry is the kernel that streams the stored blocks in the method's
applies (the A_e - D_eo kernel, here with the even inverses of block Jacobi),
timed live in the timed solves with HIP events on the library's launch stream.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2]
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
    p.add_argument("--warmup", type=int, default=3,
                   help="untimed solves before the timed ones; the first builds the polynomial "
                        "and the recycle space, the first two complete its u = 10 refreshes "
                        "(the setup phase), so the timed solves see it frozen")
    p.add_argument("--workload", default="c3")
    p.add_argument("--tol", type=float, default=1e-8)
    p.add_argument("--inner", default="f16s", choices=["f64", "f32", "f16s"])
    p.add_argument("--d", type=int, default=96)
    p.add_argument("--k", type=int, default=384)
    p.add_argument("--bj", type=int, default=1, choices=[0, 1],
                   help="left block Jacobi (B = D_ee on the reduced system)")
    p.add_argument("--u", type=int, default=30, help="recycle-space refreshes before freezing")
    p.add_argument("--schur", type=int, default=1, choices=[0, 1],
                   help="solve the odd-even reduced system (1) or the full lattice (0)")
    p.add_argument("--full-steps", type=int, default=-1,
                   help="timed solves of the same method on the full lattice, for comparison "
                        "(-1: 4 on lattices up to 8^4, else 0)")
    p.add_argument("--m", type=int, default=30, help="new Arnoldi vectors per cycle")
    p.add_argument("--ortho", type=int, default=1, choices=[0, 1],
                   help="Arnoldi: 0 Gram-Schmidt twice, 1 single-sync (one reduction per step)")
    p.add_argument("--ss-steps", type=int, default=-1,
                   help="timed solves of the same method with the other --ortho choice "
                        "(-1: 4 on lattices up to 8^4, else 0)")
    p.add_argument("--bj-steps", type=int, default=-1,
                   help="timed solves of the same method with the other --bj choice "
                        "(-1: 4 on lattices up to 8^4, else 0)")
    p.add_argument("--c1-steps", type=int, default=40,
                   help="solves of the 4^4 workload (launch-bound) with and without the "
                        "Arnoldi cycles replayed as HIP graphs (0: skip)")
    p.add_argument("--c2-steps", type=int, default=16,
                   help="timed solves of the same method on the 8^4 workload after the "
                        "headline (0: skip)")
    p.add_argument("--inner-tol", type=float, default=5e-2)
    p.add_argument("--reduced-kernels", type=int, default=0, choices=[0, 1],
                   help="reduced operator: 0 the single-read kernel pair where it applies, "
                        "1 the two-kernel form")
    p.add_argument("--plain-steps", type=int, default=1)
    p.add_argument("--plain-seconds", type=float, default=15.0,
                   help="wall-time cap of each FP64 comparison solve (they can stagnate); "
                        "reported as not converged with the residual reached")
    p.add_argument("--apply-reps", type=int, default=50)
    p.add_argument("--multi-rhs", type=int, default=64,
                   help="right-hand sides of the multi-RHS (MFMA) apply measurement (0: skip)")
    p.add_argument("--profile-every", type=int, default=8,
                   help="time one in this many launches of the apply's block kernel (0: off)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--ref-tol", type=float, default=1e-11,
                   help="tolerance of the reference solve for the forward error (same method, "
                        "its FP64 outer loop carried further)")
    p.add_argument("--summarize-trace", default=None, metavar="CSV",
                   help="only summarise a rocprofv3 kernel_trace.csv: per-kernel launches and "
                        "mean duration over launches longer than --min-us (launches that did work)")
    p.add_argument("--min-us", type=float, default=8.0)
    p.add_argument("--kernel-probe", type=int, default=0, metavar="CHAINS",
                   help="only build the workload's operator and its polynomial and run this "
                        "many polynomial chains q(A~) v of the method's reduced operator (the "
                        "solves' A_o^-1 D_oe and A_e - D_eo launches, chain epilogues), for "
                        "kernel traces and hardware counters")
    p.add_argument("--multi-probe", type=int, default=0, metavar="REPS",
                   help="only build the workload's operator and run this many multi-RHS (MFMA) "
                        "applies of --multi-rhs right-hand sides in --inner precision, for "
                        "kernel traces and hardware counters")
    p.add_argument("--mixed-probe", type=int, default=0, metavar="BATCHES",
                   help="only run this many solves of the launch-bound mixed batch (4^4, 6x4^3, "
                        "6^2x4^2; eager) with --batch-launches, for kernel traces")
    p.add_argument("--batch-launches", type=int, default=1, choices=[0, 1],
                   help="lockstep batches: 1 batched Gram-Schmidt and chain launches, 0 per column")
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


# HBM traffic of one launch of the roofline kernel on the 16^3 x 32,
# N_tv = 24 twisted-mass workload with FP16 blocks (kernel 1 of the
# single-read form: k_reduced_scatter, every launch of the solves' reduced
# applies): rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (KiB per
# dispatch, median over 116 launches) of
# `dc_kernel_probe chain 16 16 16 32 24 f16s 3 0.001`, each scaled by the
# ratio of true bytes to counter reading for 1 GiB device copies
# (`dc_kernel_probe copy 1024`: FETCH_SIZE 524299.5 KiB for 1 GiB read,
# WRITE_SIZE 1048576 KiB for 1 GiB written).  Valid only for the apply
# source it was taken on.
TRAFFIC = {"workload": "c3", "prec": "f16s", "kernel": 1,
           "fetch_kib": 2696996.0, "fetch_scale": 1048576.0 / 524299.5,
           "write_kib": 196610.1875, "write_scale": 1048576.0 / 1048576.0,
           "apply_source_sha256": "43cc144ec0a389f60a8a257000baef54b081f700817b708daa8b6647d7a5af35"}


def apply_source_digest():
    """sha256 of the apply section (block and gather kernels) of the HIP source."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_2205_09104_amd", "csrc", "kernels.hip")).read()
    a = re.search(r"^// -+ apply$", src, re.M).start()
    b = re.search(r"^// -+ block Jacobi$", src, re.M).start()
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def reduced_block_bytes(V, n, prec, blocks=9):
    """Block bytes of one launch of a reduced-operator kernel that reads
    `blocks` blocks (and their FP16 scales) per row, V/2 rows: nine for either
    kernel of the two-kernel form (the A_o^{-1} D_oe kernel reads the 8 hop
    blocks of an odd site and its self-block inverse, the A_e - D_eo kernel the
    8 hop blocks of an even site and its self block or inverse) and for the
    single-read form's scatter kernel (the 8 hop blocks of an odd site, each
    used in both directions, and its inverse); one for its gather kernel (the
    even site's self block or inverse)."""
    sb = {"f64": 16, "f32": 8, "f16s": 4}[prec]
    extra = blocks * 4 if prec == "f16s" else 0
    return (V // 2) * (blocks * n * n * sb + extra)


def reduced_vec_bytes(V, n, prec):
    """Bytes of one vector pass over the V/2 rows of a compressed vector."""
    return (V // 2) * n * (16 if prec == "f64" else 8)


def reduced_apply_bytes(V, n, prec):
    """Algorithmic bytes of one apply of the reduced operator: every stored
    block read once (per even/odd site pair the 8 hop blocks joining them to
    their neighbours and the two self blocks or inverses: ten), one read of the
    input and one write of the output.  Intermediate vectors between kernels
    are a design's own and not counted."""
    return reduced_block_bytes(V, n, prec, blocks=10) + 2 * reduced_vec_bytes(V, n, prec)


def single_read(prec, n):
    """Whether the library's reduced applies take the single-read kernel pair
    (its default for FP32 / FP16 blocks with n a multiple of 8, n <= 64)."""
    return prec != "f64" and n % 8 == 0 and 8 <= n <= 64


def measured_traffic(workload, prec, kernel):
    t = TRAFFIC
    if (workload != t["workload"] or prec != t["prec"] or kernel != t["kernel"]
            or apply_source_digest() != t["apply_source_sha256"]):
        return None, None
    fetch = t["fetch_kib"] * 1024 * t["fetch_scale"]
    write = t["write_kib"] * 1024 * t["write_scale"]
    return fetch + write, {"fetch_bytes": fetch, "write_bytes": write,
                           "fetch_scale": t["fetch_scale"], "write_scale": t["write_scale"]}


def m0_reading(w):
    """How m0 was set for the workload (synth/m0.json): the calibration method,
    the target ratio min Re eig / max |eig|, and where available the ratio the
    Ritz values of a long Arnoldi run on the 8^4 lattice of the same family
    give (an estimate: the leftmost Ritz pair is not converged)."""
    import synth
    tab = synth.load_m0_table()
    e = tab.get(w.name, {})
    out = {"method": e.get("method"), "rho_target": e.get("rho_target")}
    if "rho_achieved" in e:
        out["rho_achieved"] = e["rho_achieved"]
    ref = e if "rho_ritz" in e else tab.get("c2", {})
    if "rho_ritz" in ref:
        out["rho_ritz_estimate"] = {k: ref[k] for k in ("rho_ritz", "ritz_min_re", "ritz_max_abs",
                                                        "ritz_steps", "ritz_left_residual")}
        out["rho_ritz_estimate"]["lattice"] = "8^4 (c2)" if ref is not e else w.name
    return out


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
    if a.mixed_probe:
        mixed_probe(a)
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
    if a.kernel_probe:
        kernel_probe(op, w, a)
        return
    if a.multi_probe:
        multi_probe(op, w, a)
        return
    # HIP events on one in a.profile_every launches of the apply's block kernel
    op.profile_apply(a.profile_every)

    import paper_2205_09104_amd as dc
    dc.set_reduced_kernels(a.reduced_kernels)
    single = a.schur and a.reduced_kernels == 0 and single_read(a.inner, n)
    # the roofline kernel: the single-read scatter kernel (slot 1), the D_eo
    # kernel of the two-kernel form (slot 2), or the full-lattice block kernel
    kern = (1 if single else 2) if a.schur else 0
    other = 3 - kern if a.schur else None

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
    small = w.V <= 4096
    full_steps = a.full_steps if a.full_steps >= 0 else (4 if small else 0)
    ss_steps = a.ss_steps if a.ss_steps >= 0 else (4 if small else 0)
    bj_steps = a.bj_steps if a.bj_steps >= 0 else (4 if small else 0)

    def method_opts(**kw):
        base = dict(m=a.m + a.k, k=a.k, d=a.d, u=a.u, prec=a.inner, outer=1, m_outer=10,
                    max_outer=50, inner_tol=a.inner_tol, seed=1, max_cycles=100000,
                    schur=a.schur, ortho=a.ortho, block_jacobi=a.bj)
        base.update(kw)
        return Opts(**base)

    opts = method_opts()

    def one_solve(r, o, tol=None):
        b = synth.rhs(w.dims, w.n_tv, r, device="cuda")
        x, st, rc = op.solve(b, a.tol if tol is None else tol, o)
        return x, st[0], rc

    def timed_solves(o, first, count, label):
        """count solves of fresh right-hand sides first.. after setup, timed."""
        rr = [synth.rhs(w.dims, w.n_tv, r, device="cuda") for r in range(first, first + count)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = []
        for i, b in enumerate(rr):
            x, st, rc = op.solve(b, a.tol, o)
            out.append(st[0])
            log(f"{label} solve {i}: status {st[0]['status']} relres "
                f"{st[0]['rel_res_true']:.2e} matvecs {st[0]['matvecs']} "
                f"{st[0]['t_solve_ms']:.0f} ms")
        torch.cuda.synchronize()
        return out, time.perf_counter() - t1

    setup_ms = 0.0
    for r in range(a.warmup):
        x, st, rc = one_solve(r, opts)
        setup_ms += st["t_setup_ms"]
        log(f"warmup solve {r}: rc {rc} relres {st['rel_res_true']:.2e} iters {st['iters']} "
            f"matvecs {st['matvecs']} setup {st['t_setup_ms']:.0f} ms, "
            f"{st['t_solve_ms']:.0f} ms")
    rhs = [synth.rhs(w.dims, w.n_tv, r, device="cuda") for r in range(a.warmup, a.warmup + a.steps)]
    torch.cuda.synchronize()
    pre = prof_totals()
    pre_oe = prof_totals(other) if a.schur else None
    pre_pass = {p: (op.profile_apply_passes(p, kern),
                    op.profile_apply_passes(p, other) if a.schur else 0)
                for p in ("f64", "f32", "f16s")}
    t0 = time.perf_counter()
    stats = []
    for i, b in enumerate(rhs):
        x, st, rc = op.solve(b, a.tol, opts)
        stats.append(st[0])
        log(f"timed solve {i}: status {st[0]['status']} relres {st[0]['rel_res_true']:.2e} "
            f"matvecs {st[0]['matvecs']} {st[0]['t_solve_ms']:.0f} ms")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    x_last = x
    post = prof_totals()
    post_oe = prof_totals(other) if a.schur else None
    # timed-region block-kernel launches that did work: (count, ms) per
    # precision, and their vector passes
    prof = {p: (post[p][0][0] - pre[p][0][0], post[p][0][1] - pre[p][0][1]) for p in post}
    prof_oe = ({p: (post_oe[p][0][0] - pre_oe[p][0][0], post_oe[p][0][1] - pre_oe[p][0][1])
                for p in post_oe} if a.schur else {})
    passes = {p: op.profile_apply_passes(p, kern) - pre_pass[p][0] for p in pre_pass}
    passes_oe = ({p: op.profile_apply_passes(p, other) - pre_pass[p][1] for p in pre_pass}
                 if a.schur else {})
    ok = all(s["status"] == 0 and s["rel_res_true"] <= a.tol for s in stats)
    value = a.steps / dt if ok else 0.0
    log(f"method: {value:.3f} solves/s ({1e3 * dt / a.steps:.0f} ms per solve)")

    def comparison(o, steps, label):
        for r in range(a.warmup):             # its own setup: polynomial, recycle space
            one_solve(r, o)
        st, sdt = timed_solves(o, a.warmup, steps, label)
        res = {"solves_per_s": steps / sdt, "steps": steps,
               "matvecs_per_solve": [s["matvecs"] for s in st],
               "iters_per_solve": [s["iters"] for s in st],
               "converged": all(s["status"] == 0 for s in st)}
        log(f"{label}: {steps / sdt:.3f} solves/s")
        return res

    # ------------------------------------------------ same method without / with block Jacobi
    bj_cmp = None
    if bj_steps > 0 and a.schur:
        bj_cmp = comparison(method_opts(block_jacobi=1 - a.bj), bj_steps,
                            f"same method, block_jacobi={1 - a.bj}")
        bj_cmp["block_jacobi"] = 1 - a.bj

    # ------------------------------------------------ same method, full lattice
    full_cmp = None
    if a.schur and full_steps > 0:
        full_cmp = comparison(method_opts(schur=0, ortho=0, block_jacobi=0), full_steps,
                              "same method on the full lattice (no block Jacobi)")

    # ------------------------------------------------ same method, other Arnoldi
    ss_cmp = None
    if ss_steps > 0:
        ss_cmp = comparison(method_opts(ortho=1 - a.ortho), ss_steps,
                            f"same method, ortho={1 - a.ortho}")
        ss_cmp["ortho"] = 1 - a.ortho

    # ------------------------------------------------ FP64 comparisons (one RHS each)
    # Plain GMRES(30) (and on small lattices with the polynomial, d = 4, 8,
    # 16, and polynomial + deflation), each capped by wall time: the plain and
    # polynomial-only variants stagnate on these operators.
    comp = {}
    if a.plain_steps > 0:
        cases = [("gmres30", Opts(m=30, prec="f64"))]
        if small:
            for d in (4, 8, 16):
                cases.append((f"gmres30_poly_d{d}", Opts(m=30, d=d, prec="f64", seed=1)))
            cases.append(("gmres_poly_d16_defl_k32", Opts(m=62, k=32, d=16, prec="f64", seed=1)))
        r = a.warmup
        for name, o in cases:
            if o.k > 0:
                o.max_cycles = 400
                one_solve(r + 1, o)           # setup solve: builds the recycle space
            # time two cycles, then cap the cycle count by the wall-time budget
            o.max_cycles = 2
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            one_solve(r, o)
            torch.cuda.synchronize()
            per_cycle = (time.perf_counter() - t1) / 2
            o.max_cycles = max(2, int(a.plain_seconds / max(per_cycle, 1e-6)))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, st, rc = one_solve(r, o)
            torch.cuda.synchronize()
            pdt = time.perf_counter() - t1
            conv = st["status"] == 0
            comp[name] = {"solves_per_s": (1.0 / pdt) if conv else 0.0, "converged": conv,
                          "cycles_cap": o.max_cycles, "iters": st["iters"],
                          "matvecs": st["matvecs"], "rel_res_true": st["rel_res_true"],
                          "ms": 1e3 * pdt}
            log(f"fp64 {name}: status {st['status']} relres {st['rel_res_true']:.2e} "
                f"iters {st['iters']} matvecs {st['matvecs']} {1e3 * pdt:.0f} ms")
    plain = comp.get("gmres30", {"solves_per_s": None})

    # forward error of the last timed solve against a reference: the same
    # method carried to a.ref_tol (its FP64 outer loop makes the reference an
    # FP64-accurate solution), outside the timed region
    xr, sr, _ = op.solve(rhs[-1], a.ref_tol, opts)
    err_vs_fp64 = float(torch.linalg.vector_norm(x_last - xr) / torch.linalg.vector_norm(xr))
    log(f"forward error of the last solve vs the reference (rel.res {sr[0]['rel_res_true']:.1e}): "
        f"{err_vs_fp64:.2e}")
    del xr

    whole = prof_totals()     # the whole run so far, for comparison with a kernel tracer
    op.profile_apply(0)

    # ------------------------------------------------ CPU oracle baseline
    cpu = None
    if not a.no_cpu:
        r_last = (rhs[-1] - op.apply(x_last)).cpu().numpy()
        cpu = cpu_baseline(w, a, stats, x_check=(x_last.cpu().numpy(), rhs[-1].cpu().numpy(),
                                                 r_last))

    # ------------------------------------------------ the 4^4 workload: eager vs graph replay
    c1res = mixres = None
    if a.c1_steps > 0 and w.name != "c1":
        c1res = c1_graphs(a)
        try:
            mixres = mixed_graphs(a)
        except Exception as e:   # an extra key: reported, never fatal to the line
            mixres = {"error": f"{type(e).__name__}: {e}"}
            log(f"mixed batch graph replay failed: {e}")

    # ------------------------------------------------ the same method on the 8^4 workload
    c2res = None
    if a.c2_steps > 0 and w.name != "c2":
        op.close()
        del op
        torch.cuda.empty_cache()
        w2 = synth.WORKLOADS["c2"]
        A2, B2 = synth.operator(w2, device="cuda")
        op2 = CoarseOp(A2, B2, w2.dims, mu=w2.mu, store=("f64", "f32", "f16s"))
        del A2, B2
        # the same method with at most 10 recycle refreshes, which the warm-up
        # solves complete (this lattice's solves take one or two cycles each),
        # and a polynomial of degree at most 32: on this smaller lattice a
        # degree-64 polynomial needs about twice the matvecs
        opts2 = method_opts(u=min(a.u, 10), d=min(a.d, 32))
        for r in range(a.warmup):
            op2.solve(synth.rhs(w2.dims, w2.n_tv, r, device="cuda"), a.tol, opts2)
        rr = [synth.rhs(w2.dims, w2.n_tv, r, device="cuda")
              for r in range(a.warmup, a.warmup + a.c2_steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st2 = [op2.solve(b, a.tol, opts2)[1][0] for b in rr]
        torch.cuda.synchronize()
        c2dt = time.perf_counter() - t1
        conv2 = all(s["status"] == 0 for s in st2)
        c2res = {"workload": f"c2: {'x'.join(map(str, w2.dims))} lattice, N_tv={w2.n_tv} "
                             f"({w2.N} unknowns), mu={w2.mu}, m0={w2.m0():.6f}",
                 "u": opts2.u, "d": opts2.d,
                 "solves_per_s": (a.c2_steps / c2dt) if conv2 else 0.0, "steps": a.c2_steps,
                 "ms_per_step": 1e3 * c2dt / a.c2_steps,
                 "matvecs_per_solve": [s["matvecs"] for s in st2],
                 "rel_res_true_max": max(s["rel_res_true"] for s in st2), "converged": conv2}
        log(f"same method on c2: {a.c2_steps / c2dt:.2f} solves/s")
        op2.close()

    inner = a.inner
    launches, tot_ms = prof[inner]
    avg_us = 1e3 * tot_ms / max(launches, 1)
    if a.schur:
        # per launch: the nine blocks per row, plus its vector passes (summed
        # over the timed launches by the library: the scatter kernel x_e and its
        # eight partial vectors; the D_eo kernel 2 to 5 with its epilogue)
        s1b = (launches * reduced_block_bytes(V, n, inner) +
               passes[inner] * reduced_vec_bytes(V, n, inner)) / max(launches, 1)
    else:
        s1b = stage1_bytes(V, n, inner)
    achieved = s1b / (avg_us * 1e-6) / 1e9 if launches else None
    traffic, traffic_detail = measured_traffic(w.name, inner, kern)
    if single:
        kname = (f"k_reduced_scatter ({inner} blocks; per odd row t_o = A_o^-1 D_oe x_e and, "
                 f"from the same read of each hop block, the eight D_eo products of t_o)")
    elif a.schur and a.bj:
        kname = (f"k_reduced_eo ({inner} blocks; x_e - A_e^-1 D_eo t_o with the chain "
                 f"epilogue)")
    elif a.schur:
        kname = f"k_reduced_eo ({inner} blocks; A_e x_e - D_eo t_o with the chain epilogue)"
    else:
        kname = f"k_apply_blocks ({inner} blocks)"
    oe = None
    if a.schur:
        l1, m1 = prof_oe[inner]
        if l1:
            b1 = (l1 * reduced_block_bytes(V, n, inner, blocks=1 if single else 9) +
                  passes_oe[inner] * reduced_vec_bytes(V, n, inner)) / l1
            oname = (f"k_reduced_gather ({inner} blocks; the eight partial vectors summed per "
                     f"even row, A_e^-1 and the chain epilogue)" if single else
                     f"k_reduced_oe ({inner} blocks; t_o = A_o^-1 D_oe x_e)")
            oe = {"kernel": oname,
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
                   "solver": f"{'odd-even reduced system; ' if a.schur else ''}"
                             f"{'left block Jacobi B = D_ee; ' if a.bj and a.schur else ''}"
                             f"FGMRES(10) fp64 outer; inner {inner} GCRO-DR(m={a.m + a.k},"
                             f"k={a.k}, u={a.u}) + poly d={a.d}, inner_tol={a.inner_tol}"
                             f"{', single-sync Arnoldi' if a.ortho else ''}",
                   "tol": a.tol, "parallelism": "single GPU",
                   "m0_reading": m0_reading(w)},
        "setup_ms": setup_ms,
        "iters_per_solve": [s["iters"] for s in stats],
        "matvecs_per_solve": [s["matvecs"] for s in stats],
        "rel_res_true": [s["rel_res_true"] for s in stats],
        "err_vs_fp64_last_solve": err_vs_fp64,
        "plain_fp64_gmres30": plain,
        "same_method_full_lattice": full_cmp,
        "same_method_other_ortho": ss_cmp,
        "same_method_other_block_jacobi": bj_cmp,
        "c2_same_method": c2res,
        "c1_graph_replay": c1res,
        "mixed_batch_graph_replay": mixres,
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


def c1_graphs(a):
    """The 4^4, N_tv = 8 workload (4,096 unknowns, launch-bound): solves/s to
    1e-10 with eager launches and with every Arnoldi cycle replayed as one
    captured HIP graph, for plain FP64 GMRES(30) and for the method (reduced
    system, block Jacobi, polynomial d = 4, GCRO-DR(38, 8), FP64)."""
    import torch

    import synth
    from paper_2205_09104_amd import CoarseOp, Opts
    w = synth.WORKLOADS["c1"]
    A, B = synth.operator(w, device="cuda")
    out = {"workload": f"c1: {'x'.join(map(str, w.dims))} lattice, N_tv={w.n_tv} "
                       f"({w.N} unknowns), mu={w.mu}, m0={w.m0():.6f}", "tol": 1e-10}
    cases = {"gmres30_fp64": dict(m=30, prec="f64"),
             "method_fp64": dict(m=38, k=8, d=4, u=10, prec="f64", seed=1, schur=1,
                                 block_jacobi=1, ortho=1)}
    for name, kw in cases.items():
        res = {}
        for graphs in (0, 1):
            op = CoarseOp(A, B, w.dims, mu=w.mu)
            o = Opts(**kw, graphs=graphs)
            for r in range(3):
                op.solve(synth.rhs(w.dims, w.n_tv, r, device="cuda"), 1e-10, o)
            rr = [synth.rhs(w.dims, w.n_tv, r, device="cuda") for r in range(3, 3 + a.c1_steps)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = [op.solve(b, 1e-10, o)[1][0] for b in rr]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res["graphs" if graphs else "eager"] = {
                "solves_per_s": a.c1_steps / dt if all(s["status"] == 0 for s in st) else 0.0,
                "ms_per_solve": 1e3 * dt / a.c1_steps,
                "iters_per_solve": float(sum(s["iters"] for s in st)) / len(st),
                "graph_stats": list(op.graph_stats())}
            op.close()
        res["speedup"] = (res["graphs"]["solves_per_s"] / res["eager"]["solves_per_s"]
                          if res["eager"]["solves_per_s"] else None)
        log(f"c1 {name}: eager {res['eager']['solves_per_s']:.1f}, graphs "
            f"{res['graphs']['solves_per_s']:.1f} solves/s")
        out[name] = res
    return out


def mixed_graphs(a):
    """A launch-bound mixed batch (4^4, 6x4^3 and 6^2x4^2 lattices of the 4^4
    workload's family, N_tv = 8, two right-hand sides each, FP64, polynomial
    d = 4, GMRES(20) in lockstep, tolerance 1e-10): batches/s with the
    Gram-Schmidt and chain launches per column / per operator, batched (one
    launch for all columns), and batched with each lockstep cycle's steps
    replayed as one HIP graph."""
    import torch

    from paper_2205_09104_amd import CoarseOp, Opts
    dims_list, w, ops, bs, tols = mixed_batch()
    out = {"lattices": ["x".join(map(str, d)) for d in dims_list], "n_tv": w.n_tv,
           "rhs_per_lattice": 2, "tol": 1e-10}
    import paper_2205_09104_amd as dc
    # per_column: the Gram-Schmidt passes and chain steps launched per column
    # and per operator; eager / graphs: batched launches (the default)
    try:
        for name, graphs, batched in (("per_column", 0, 0), ("eager", 0, 1), ("graphs", 1, 1)):
            dc.set_batch_launches(batched)
            o = Opts(m=20, d=4, seed=3, graphs=graphs)
            CoarseOp.solve_multi(ops, bs, tols, o)       # polynomial, tile choice, recordings
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = [CoarseOp.solve_multi(ops, bs, tols, o) for _ in range(a.c1_steps)]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ok = all(rc == 0 for _, _, rc in sts)
            out[name] = {"batches_per_s": a.c1_steps / dt if ok else 0.0,
                         "ms_per_batch": 1e3 * dt / a.c1_steps,
                         "graph_stats": list(ops[0].graph_stats())}
    finally:
        dc.set_batch_launches(1)
    out["speedup"] = (out["graphs"]["batches_per_s"] / out["eager"]["batches_per_s"]
                      if out["eager"]["batches_per_s"] else None)
    log(f"mixed batch: per-column launches {out['per_column']['batches_per_s']:.1f}, batched "
        f"eager {out['eager']['batches_per_s']:.1f}, graphs {out['graphs']['batches_per_s']:.1f} "
        f"batches/s")
    for op in ops:
        op.close()
    return out


def mixed_batch(device="cuda"):
    """The launch-bound mixed batch: operators, right-hand sides, tolerances."""
    import torch

    import synth
    from paper_2205_09104_amd import CoarseOp
    w = synth.WORKLOADS["c1"]
    dims_list = [(4, 4, 4, 4), (6, 4, 4, 4), (6, 6, 4, 4)]
    ops, bs = [], []
    for i, dims in enumerate(dims_list):
        A = synth.self_blocks(dims, w.n_tv, w.m0(), w.seed, device=device)
        B = synth.hop_blocks(dims, w.n_tv, w.seed, device=device)
        ops.append(CoarseOp(A, B, dims))
        bs.append(torch.stack([synth.rhs(dims, w.n_tv, 10 * i + r, device=device) for r in range(2)]))
    return dims_list, w, ops, bs, [[1e-10, 1e-10]] * len(ops)


def mixed_probe(a):
    """a.mixed_probe eager solves of the mixed batch with a.batch_launches (after
    one untimed solve), printing batches/s and the lockstep step counts."""
    import torch

    import paper_2205_09104_amd as dc
    from paper_2205_09104_amd import CoarseOp, Opts
    _, _, ops, bs, tols = mixed_batch()
    dc.set_batch_launches(a.batch_launches)
    o = Opts(m=20, d=4, seed=3)
    CoarseOp.solve_multi(ops, bs, tols, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.mixed_probe):
        _, st, rc = CoarseOp.solve_multi(ops, bs, tols, o)
        assert rc == 0
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = [max(s["iters"] for s in sg) for sg in st]
    log(f"mixed probe, batch launches {a.batch_launches}: {a.mixed_probe / dt:.1f} batches/s, "
        f"lockstep steps per operator {steps}")
    for op in ops:
        op.close()


def multi_probe(op, w, a):
    """a.multi_probe multi-RHS applies of a.multi_rhs right-hand sides (blocks
    and vectors of --inner precision; FP64 with --inner f64)."""
    import torch

    import synth
    R = a.multi_rhs
    X = torch.stack([synth.rhs(w.dims, w.n_tv, 500 + r, device="cuda") for r in range(R)])
    if a.inner != "f64":
        X = X.to(torch.complex64)
    Y = torch.empty_like(X)
    op.apply_multi(X, prec=a.inner, out=Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.multi_probe):
        op.apply_multi(X, prec=a.inner, out=Y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.multi_probe
    tf = 72.0 * w.V * w.n * w.n * R / dt / 1e12
    print(json.dumps({"multi_probe": w.name, "n_rhs": R, "prec": a.inner,
                      "reps": a.multi_probe, "ms": 1e3 * dt, "TFLOP/s": tf}), flush=True)


def kernel_probe(op, w, a):
    """a.kernel_probe polynomial chains of the method's operator (reduced,
    block Jacobi per --bj, blocks of --inner precision, degree --d): each
    chain is d - 1 applies, i.e. d - 1 launches of each reduced kernel with the
    first / later chain-step epilogues."""
    import torch

    import synth
    from paper_2205_09104_amd import Opts
    o = Opts(d=a.d, prec=a.inner, seed=1, schur=a.schur, block_jacobi=a.bj)
    th = op.poly_setup(o)
    rows = w.V // 2 if a.schur else w.V
    x = synth.rhs(w.dims, w.n_tv, 0, device="cuda")[:rows].to(torch.complex64).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.kernel_probe):
        op.poly_apply(x, o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"kernel_probe": w.name, "chains": a.kernel_probe, "d": len(th),
                      "applies": a.kernel_probe * (len(th) - 1), "ms": 1e3 * dt}), flush=True)


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
    """The FP64 oracle on the host, timed on a bounded sample: the oracle's
    single-site stencil (self block and 8 hop blocks times the site's and its
    neighbours' vectors, dop.apply_site) over sampled sites for about
    a.cpu_seconds.  One apply of the reduced operator costs at least V such
    site stencils (V/2 even rows of 9 block products, V/2 odd rows of 8 plus
    the inverse), so the oracle's solves/s is bounded above by
    1 / (V x time per site x matvecs per solve of the GPU method): an
    extrapolation that leaves out orthogonalisation, inverses and setup.
    Also re-derives the last GPU solution's FP64 residual at sampled sites
    with the oracle's stencil."""
    import numpy as np

    import synth
    from oracle import operator as dop
    from oracle.lattice import neighbours
    fwd, bwd = neighbours(w.dims)
    m0 = w.m0()
    rng = np.random.default_rng(7)
    sites = rng.choice(w.V, size=min(w.V, 64), replace=False)

    def blocks(s):
        A = synth.self_blocks(w.dims, w.n_tv, m0, w.seed, sites=[int(s)]).numpy()[0]
        B = synth.hop_blocks(w.dims, w.n_tv, w.seed, sites=[int(s)]).numpy()[0]
        Bb = synth.hop_blocks(w.dims, w.n_tv, w.seed, sites=bwd[:, s].tolist()).numpy()
        return A, B, np.stack([Bb[m, m] for m in range(4)])

    blk = [blocks(s) for s in sites]
    n = w.n
    psi = rng.standard_normal((9, n)) + 1j * rng.standard_normal((9, n))
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < a.cpu_seconds:
        A, B, Bb = blk[reps % len(blk)]
        dop.apply_site(A, B, Bb, psi[0], psi[1:5], psi[5:9], w.mu)
        reps += 1
    per_site = (time.perf_counter() - t0) / reps
    mv = float(np.mean([s["matvecs"] for s in stats]))
    try:
        from threadpoolctl import threadpool_info
        blas = [{k: i.get(k) for k in ("internal_api", "num_threads")} for i in threadpool_info()]
    except Exception:  # noqa: BLE001
        blas = None
    out = {"value": 1.0 / (w.V * per_site * mv), "unit": "solves/s", "cores": 1, "kind": "oracle",
           "extrapolated": True, "host_cpus": os.cpu_count(), "blas_pools": blas,
           "sample": f"{reps} oracle site stencils (numpy, one thread; {1e6 * per_site:.1f} us "
                     f"each) over {len(sites)} sampled sites, x {w.V} sites per apply of the "
                     f"reduced operator x {mv:.0f} matvecs per solve of the GPU method: an "
                     f"upper bound (orthogonalisation, inverses and setup not counted)"}
    if x_check is not None:
        x, b, r_gpu = x_check
        worst = 0.0
        for s, (A, B, Bb) in zip(sites[:16], blk[:16]):
            Dx = dop.apply_site(A, B, Bb, x[s], x[fwd[:, s]], x[bwd[:, s]], w.mu)
            worst = max(worst, float(np.abs((b[s] - Dx) - r_gpu[s]).max()))
        out["residual_rows_checked"] = 16
        out["residual_rows_max_abs_diff"] = worst / float(np.abs(b).max())
    return out


if __name__ == "__main__":
    main()
