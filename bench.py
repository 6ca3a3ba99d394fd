"""Benchmark: time-to-solution at 1e-10 of MSPCG against plain FP64 CG on one GPU,
plus dslash_eo bandwidth against the HBM roofline.

One step = one full MSPCG solve (Algorithm 1, FP64 outer, low-precision batched
block CG as preconditioner) of the normal equation from x = 0 to a true relative
residual of 1e-10, on a seeded synthetic gauge field and source that are
resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1811_08488_amd import mspcg as M  # noqa: E402
from paper_1811_08488_amd import synth  # noqa: E402
from paper_1811_08488_amd.workloads import WORKLOADS  # noqa: E402

METRIC = "time-to-solution @1e-10 MSPCG vs plain CG (s); dslash GB/s & % HBM roofline"
HBM_PEAK_GBS = 8000.0
PREC = {"f32": M.F32, "f16": M.F16, "bf16": M.BF16, "f64": M.F64}
BYTES = {M.F64: (8, 0), M.F32: (4, 0), M.F16: (2, 4), M.BF16: (2, 4)}


def dslash_bytes_per_site(prec, Ls, nrhs):
    """Algorithmic bytes per 5D output site: in + out spinor (+ norms) + links shared over Ls and rhs."""
    w, n = BYTES[prec]
    return 2 * (24 * w + n) + 144 * w / (Ls * nrhs)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_problem(w, torch):
    eps = w.eps if w.eps is not None else synth.tuned_eps()
    t0 = time.time()
    log(f"[bench] {w.name}: generating links ({w.V} sites)")
    U = synth.gauge_field(w.L, eps, w.gauge_seed)
    log(f"[bench] links generated in {time.time() - t0:.1f}s (eps={eps:.4f})")
    A = M.Action(w.L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c, t_bc=-1)
    h = M.Handle(A, U)
    # the source phi[rhs][lex][s][spin][colour], streamed into the two parities
    # (cb = lex >> 1) of device fields in their storage layout
    t0 = time.time()
    fields = {p: h.field(M.F64, w.nrhs, p) for p in (0, 1)}
    views = {p: fields[p].data.view(w.nrhs, A.V // 2, 12, w.Ls, 2) for p in (0, 1)}
    for r, cb0, ev, od in synth.source_cb_chunks(w.L, w.Ls, w.nrhs, w.source_seed):
        for p, part in ((0, ev), (1, od)):
            lay = M.to_device_layout(part[None]).reshape(len(part), 12, w.Ls, 2)
            views[p][r, cb0:cb0 + len(part)] = torch.from_numpy(lay).to(fields[p].data.device)
    log(f"[bench] source generated in {time.time() - t0:.1f}s")
    b = h.field(M.F64, w.nrhs, 0)
    h.prepare_rhs(b, fields[0], fields[1])
    torch.cuda.synchronize()
    del fields, views
    torch.cuda.empty_cache()
    return h, A, U, eps, b


def time_dslash(h, A, w, prec, reps=50, warm=5):
    """Average duration of one dslash_eo launch: HIP events on the stream the
    kernel is launched on, bracketing `reps` back-to-back launches."""
    import torch

    stream = torch.cuda.Stream()
    fin = h.field(prec, w.nrhs, 1)
    fout = h.field(prec, w.nrhs, 0)
    with torch.cuda.stream(stream):
        src = h.upload(synth.cb_field(w.L, w.Ls, w.nrhs, 99), 1, M.F64)
        h.convert(fin, src, stream=stream)
        for _ in range(warm):
            h.dslash_eo(fout, fin, 0, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            h.dslash_eo(fout, fin, 0, stream=stream)
        e1.record(stream)
        stream.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nsites5 = (A.V // 2) * w.Ls * w.nrhs
    bytes_ = dslash_bytes_per_site(prec, w.Ls, w.nrhs) * nsites5
    return {"ms": ms, "bytes": bytes_, "gbs": bytes_ / (ms * 1e-3) / 1e9}


def time_m5inv(h, A, w, prec, reps=50, warm=5):
    """Average duration of one m5inv launch (HIP events on the launch stream)."""
    import torch

    stream = torch.cuda.Stream()
    fin = h.field(prec, w.nrhs, 1)
    fout = h.field(prec, w.nrhs, 1)
    with torch.cuda.stream(stream):
        src = h.upload(synth.cb_field(w.L, w.Ls, w.nrhs, 98), 1, M.F64)
        h.convert(fin, src, stream=stream)
        for _ in range(warm):
            h.m5inv(fout, fin, 0, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            h.m5inv(fout, fin, 0, stream=stream)
        e1.record(stream)
        stream.synchronize()
    ms = e0.elapsed_time(e1) / reps
    w_, n = BYTES[prec]
    bytes_ = 2 * (24 * w_ + n) * (A.V // 2) * w.Ls * w.nrhs
    flops = 2 * 2 * 12 * w.Ls * w.Ls * (A.V // 2) * w.nrhs  # two chiralities, 12 columns each, Ls x Ls multiply-adds
    return {"us": ms * 1e3, "GB/s": bytes_ / (ms * 1e-3) / 1e9, "frac_hbm": bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "TFLOP/s": flops / (ms * 1e-3) / 1e12}


def kernel_source_hash():
    """SHA-256 of the HIP sources the hop kernel is compiled from."""
    import hashlib

    hsh = hashlib.sha256()
    for f in ("kernels.hip", "common.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1811_08488_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def measured_traffic(workload, prec_name):
    """HBM bytes per dslash_eo launch from the committed hardware-counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when there is none for this workload or the kernel source changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hop_kernel_dslash_eo_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    v = kv.get(f"traffic_bytes_per_launch_{prec_name}")
    return None if v is None else float(v)


def cpu_baseline(w, U, outer_iters, n_inner, nblk, max_sites5=12_000_000):
    """Oracle (FP64 C++/OpenMP) time per application of A, projected to the
    oracle's own MSPCG solve at the GPU's outer iteration count.  Where the
    lattice is too large for the host (more than max_sites5 5D sites per
    parity and right-hand side), the sample is the first Lt' time slices
    (periodic in t'), one right-hand side, scaled by volume and nrhs."""
    import oracle as O

    Lt = w.L[3]
    lt = Lt
    while (w.V // Lt) * lt // 2 * w.Ls > max_sites5 and lt > 2 and (lt // 2) % 2 == 0:
        lt //= 2
    L = (w.L[0], w.L[1], w.L[2], lt)
    Usub = U.reshape(Lt, -1, 4, 3, 3)[:lt].reshape(-1, 4, 3, 3)
    oa = O.Action(L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c)
    x = synth.cb_field(L, w.Ls, 1, 5)[0]
    t0 = time.time()
    n = 0
    while n < 1 or (time.time() - t0 < 10.0 and n < 10):
        O.mdagm(oa, Usub, x)
        n += 1
    t_sample = (time.time() - t0) / n
    scale = (Lt / lt) * w.nrhs
    t_A = t_sample * scale
    nb = int(np.prod(nblk)) if nblk else 0
    # the oracle's preconditioner applies its literal A_s (one full-lattice A per block)
    a_per_outer = 1 + n_inner * nb
    a_total = outer_iters * a_per_outer + 2
    where = "the full lattice" if lt == Lt else f"the first {lt} of {Lt} time slices"
    return {
        "value": t_A * a_total,
        "unit": "s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": f"{n} applications of A = D_PC^+ D_PC on {where}, one right-hand side ({t_sample:.2f} s each), "
                  f"scaled x{scale:g} to the workload and projected to the {a_total} applications of the "
                  f"oracle's MSPCG at the GPU's {outer_iters} outer iterations",
    }


def kernels_only(w, torch):
    """dslash_eo in each storage precision, then a plain copy (F64 -> F64 conversion, which reads and
    writes exactly one field) used to calibrate the HBM byte counters."""
    eps = w.eps if w.eps is not None else synth.tuned_eps()
    U = synth.gauge_field(w.L, eps, w.gauge_seed)
    A = M.Action(w.L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c, t_bc=-1)
    h = M.Handle(A, U)
    src = h.upload(synth.cb_field(w.L, w.Ls, w.nrhs, 99), 1, M.F64)
    for p in (M.F64, M.F32, M.F16):
        fin, fout = h.field(p, w.nrhs, 1), h.field(p, w.nrhs, 0)
        h.convert(fin, src)
        for _ in range(10):
            h.dslash_eo(fout, fin, 0)
    for p in (M.F64, M.F32):  # M_5^{-1}: the dense fifth-dimension contraction on the matrix cores
        fin, fout = h.field(p, w.nrhs, 1), h.field(p, w.nrhs, 1)
        h.convert(fin, src)
        for _ in range(10):
            h.m5inv(fout, fin, 0)
    dst = h.field(M.F64, w.nrhs, 1)
    for _ in range(10):
        h.convert(dst, src)
    torch.cuda.synchronize()
    field_bytes = (A.V // 2) * w.Ls * w.nrhs * 24 * 8
    print(json.dumps({"kernels_only": w.name, "copy_bytes_read": field_bytes, "copy_bytes_written": field_bytes}),
          flush=True)


def study(w, torch, ks=(3, 4, 6, 8, 12, 18), inner_prec=None, snake_modes=(0, 1), inner_tols=(0.0,), sweeps=(1,),
          max_iter=20000, reps=2):
    """Inner-iteration sweep with and without the snake terms (Sec. 2.3, Sec. 3):
    outer iterations and time-to-solution for each k, plain CG for reference.
    inner_tols > 0 add runs with precision-based inner stopping (k the maximum),
    the alternative to a fixed k that Sec. 3 sets aside; sweeps > 1 add runs
    with several multisplitting sweeps per preconditioner application (Sec. 2.1)."""
    h, A, U, eps, b = build_problem(w, torch)
    x = h.field(M.F64, w.nrhs, 0)
    prec = PREC[inner_prec or w.inner_prec]
    rows = []
    x.data.zero_()
    st = h.cg_solve(x, b, tol=w.tol, max_iter=50000, reliable=w.reliable)
    rows.append({"solver": "cg", "outer_iters": st["outer_iters"], "seconds": st["seconds"],
                 "true_rel_resid": st["true_rel_resid"]})
    log(f"[study] plain CG: {st['outer_iters']} iterations, {st['seconds']:.3f}s")
    for no_snake in snake_modes:
        for nsw in sweeps:
            for itol in inner_tols:
                for k in ks:
                    for rep in range(reps):  # the first solve of a shape tunes and captures
                        x.data.zero_()
                        st = h.mspcg_solve(x, b, w.nblk, k, prec, tol=w.tol, max_iter=max_iter,
                                           reliable=w.reliable, no_snake=no_snake, inner_tol=itol, n_sweeps=nsw)
                    rows.append({"solver": "mspcg", "k": k, "snake_terms": not no_snake, "inner_tol": itol,
                                 "sweeps": nsw, "status": st["status"], "outer_iters": st["outer_iters"],
                                 "seconds": st["seconds"], "true_rel_resid": st["true_rel_resid"]})
                    log(f"[study] k={k} snake={not no_snake} inner_tol={itol:g} sweeps={nsw}: "
                        f"{st['outer_iters']} outer, {st['seconds']:.3f}s")
    print(json.dumps({"study": "inner iterations and snake terms", "workload": w.name,
                      "inner_prec": inner_prec or w.inner_prec, "blocks": list(w.nblk), "tol": w.tol, "rows": rows}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mobius_16x16x16x32_ls16")
    ap.add_argument("--inner-prec", default=None)
    ap.add_argument("--n-inner", type=int, default=None)
    ap.add_argument("--cg-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--study", action="store_true",
                    help="sweep the inner iterations k with and without the snake terms instead of the benchmark")
    ap.add_argument("--study-k", default="3,4,6,8,12,18", help="inner iteration counts of the study")
    ap.add_argument("--study-snake-only", action="store_true", help="study: skip the runs without snake terms")
    ap.add_argument("--study-sweeps", default="1", help="study: multisplitting sweeps per preconditioner application")
    ap.add_argument("--study-max-iter", type=int, default=20000, help="study: outer iteration limit of each solve")
    ap.add_argument("--study-no-snake-only", action="store_true", help="study: only the runs without snake terms")
    ap.add_argument("--study-reps", type=int, default=2,
                    help="study: solves per setting (the last is reported; the first also tunes and captures)")
    ap.add_argument("--study-inner-tol", default="0",
                    help="study: inner stopping tolerances (0 = fixed k; > 0: precision-based stopping, k the maximum)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch dslash_eo (F64/F32/F16) and a plain F64 copy of the same size, 10 times each "
                         "(the workload for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (sharding the "
              "lattice over GPUs, with halo exchange for the outer operator, is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    # the solvers report progress every 50 outer iterations (long solves on the large lattices)
    os.environ.setdefault("MSPCG_VERBOSE", "50")
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    w = WORKLOADS[args.workload]
    inner_prec = PREC[args.inner_prec or w.inner_prec]
    k = args.n_inner if args.n_inner is not None else w.n_inner
    nblk = w.nblk
    if args.kernels_only:
        kernels_only(w, torch)
        return
    if args.study:
        study(w, torch, ks=tuple(int(v) for v in args.study_k.split(",")), inner_prec=args.inner_prec,
              snake_modes=(0,) if args.study_snake_only else (1,) if args.study_no_snake_only else (0, 1),
              inner_tols=tuple(float(v) for v in args.study_inner_tol.split(",")),
              sweeps=tuple(int(v) for v in args.study_sweeps.split(",")), max_iter=args.study_max_iter,
              reps=max(1, args.study_reps))
        return
    h, A, U, eps, b = build_problem(w, torch)
    x = h.field(M.F64, w.nrhs, 0)

    def mspcg_step():
        x.data.zero_()
        return h.mspcg_solve(x, b, nblk, k, inner_prec, tol=w.tol, max_iter=20000, reliable=w.reliable)

    def cg_step():
        x.data.zero_()
        return h.cg_solve(x, b, tol=w.tol, max_iter=50000, reliable=w.reliable)

    for i in range(args.warmup):
        log(f"[bench] warmup mspcg {i} (tunes launch shapes, captures the preconditioner)")
        st = mspcg_step()
        log(f"[bench] warmup mspcg {i}: {st['outer_iters']} outer, {st['seconds']:.3f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(mspcg_step())
        log(f"[bench] step {i}: {stats[-1]['outer_iters']} outer, {stats[-1]['seconds']:.3f}s")
    torch.cuda.synchronize()
    t_ms = (time.perf_counter() - t0) / args.steps

    cg_stats, t_cg = None, None
    if args.cg_steps > 0:
        cg_step()  # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.cg_steps):
            cg_stats = cg_step()
            log(f"[bench] plain CG {i}: {cg_stats['outer_iters']} iterations, {cg_stats['seconds']:.3f}s")
        torch.cuda.synchronize()
        t_cg = (time.perf_counter() - t1) / args.cg_steps

    dsl = {p: time_dslash(h, A, w, PREC[p]) for p in ("f64", "f32", "f16")}
    for p, d in dsl.items():
        log(f"[bench] dslash_eo {p}: {d['ms'] * 1e3:.1f} us, {d['gbs']:.0f} GB/s")
    m5 = {p: time_m5inv(h, A, w, PREC[p]) for p in ("f64", "f32")}
    for p, d in m5.items():
        log(f"[bench] m5inv {p}: {d['us']:.1f} us, {d['GB/s']:.0f} GB/s")
    main_k = dsl["f64"]
    out = {
        "metric": METRIC,
        "value": t_ms,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_ms * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+" + {M.F32: "f32", M.F16: "f16", M.BF16: "bf16", M.F64: "f64"}[inner_prec],
        "data": "synthetic",
        "config": {
            "workload": w.name, "lattice": list(w.L), "Ls": w.Ls, "nrhs": w.nrhs, "mobius_b_c": [w.b, w.c],
            "M5": w.M5, "mf": w.mf, "blocks": list(nblk), "n_inner": k, "tol": w.tol, "reliable": w.reliable,
            "gauge_eps": round(eps, 5),
        },
        "mspcg": {"seconds": t_ms, "outer_iters": stats[-1]["outer_iters"], "inner_iters": stats[-1]["inner_iters"],
                  "true_rel_resid": stats[-1]["true_rel_resid"]},
        "plain_cg": None if cg_stats is None else {
            "seconds": t_cg, "iters": cg_stats["outer_iters"], "true_rel_resid": cg_stats["true_rel_resid"]},
        "mspcg_speedup_vs_cg": None if t_cg is None else t_cg / t_ms,
        "dslash_eo": {p: {"us": d["ms"] * 1e3, "GB/s": d["gbs"], "frac_hbm": d["gbs"] / HBM_PEAK_GBS}
                      for p, d in dsl.items()},
        "m5inv": m5,
        "roofline": {"bound": "hbm", "achieved": main_k["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": main_k["gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(w.name, "f64"),
                     "algorithmic_bytes": main_k["bytes"], "avg_launch_us": main_k["ms"] * 1e3,
                     "kernel": "hop_kernel<double> (dslash_eo, FP64)"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, U, stats[-1]["outer_iters"], k, nblk)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
