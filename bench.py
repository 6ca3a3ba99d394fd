"""Benchmark: time-to-solution at 1e-10 of MSPCG against plain FP64 CG on one GPU,
plus the bandwidth of the operator kernels against the HBM roofline.

One step = one full MSPCG solve (Algorithm 1, FP64 outer, low-precision batched
block CG as preconditioner) of the normal equation from x = 0 to a true relative
residual of 1e-10, on a seeded synthetic gauge field and source that are
resident in HBM before timing starts.

The default workload is Moebius 24^3x64 x Ls=24 (2x2x2x4 blocks of 12^3x16,
8 inner FP16 iterations): far larger than the 256 MB last-level cache, and
the default run (one warm-up and three timed solves, plain CG, one more
MSPCG solve at 4 inner iterations, the kernel timings and the CPU baseline)
takes about four minutes.  The largest one-GPU workload (48^3x96 x 12) takes
about 40 s per solve; run it with --workload mobius_48x48x48x96_ls12 and
--steps 1.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
    python bench.py --workload NAME --oracle-check    # full FP64 CPU oracle solve next to the GPU's

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
# Vector ALU ceiling: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane
# instructions per second, at 4 flops per instruction for the two-term dot
# products (v_dot2_f32_f16) and packed operations the FP16 hop is built from
VALU_PEAK_TFLOPS = 157.3
# flops per 5D output site of a hop: the Wilson hop 1320 (8 directions x (12
# for the spin projection + 2 x 66 for the link times two colour vectors) + 7 x 24
# for the accumulation) plus 72 for the fifth-dimension epilogue terms
HOP_FLOPS_PER_SITE5 = 1392
PREC = {"f32": M.F32, "f16": M.F16, "bf16": M.BF16, "f64": M.F64}
BYTES = {M.F64: (8, 0), M.F32: (4, 0), M.F16: (2, 4), M.BF16: (2, 4)}
PNAME = {v: k for k, v in PREC.items()}
DEFAULT_WORKLOAD = "mobius_24x24x24x64_ls24"


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

    torch.cuda.synchronize()  # (nothing else may run beside the timed launches)
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

    torch.cuda.synchronize()
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
    # the recurrence along s: three multiply-adds and one multiply per real value
    flops = 7 * 24 * w.Ls * (A.V // 2) * w.nrhs
    return {"us": ms * 1e3, "GB/s": bytes_ / (ms * 1e-3) / 1e9, "frac_hbm": bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "TFLOP/s": flops / (ms * 1e-3) / 1e12}


def kernel_source_hash():
    """SHA-256 of the HIP sources the kernels are compiled from."""
    import hashlib

    hsh = hashlib.sha256()
    for f in ("kernels.hip", "common.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1811_08488_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def measured_traffic(workload, label):
    """HBM bytes per launch of kernel `label` (e.g. dslash_eo_f64, block_hop1_f16)
    from the committed hardware-counter summary of the workload (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy's readings), or None when there is none
    or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
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
    v = kv.get(f"traffic_bytes_per_launch_{label}")
    return None if v is None else float(v)


def block_hop_bytes(prec, Ls, nrhs, n_in, n_out, n_extra):
    """Algorithmic bytes of one launch of a block hop: every input and output
    5D site of its domains once (with the F16/BF16 norms), the links of every
    output 4D site once (8 x 18 reals), and n_extra more 4D sites' worth of
    spinors for the operands read on the blocks' own sites (hop 2: M_5 p;
    hop 4: M_5^+ y and the block residual r, which it updates in place:
    r -= alpha A_s p; its output is r)."""
    w, n = BYTES[prec]
    site5 = (24 * w + n) * Ls * nrhs
    return (n_in + n_out + n_extra) * site5 + n_out * 144 * w


def time_block_hops(h, w, prec, nblk, reps=20, warm=3):
    """Average duration of each of the four block-hop launches of an inner
    iteration (HIP events on the stream they are launched on), with its
    algorithmic bytes and fraction of the HBM roofline."""
    import torch

    n_be = h.block_hop(nblk, prec, w.nrhs, 1, 0)[0]  # hop 1 reads the blocks' own even sites
    torch.cuda.synchronize()  # (nothing else may run beside the timed launches)
    stream = torch.cuda.Stream()
    out = {}
    for hop in (1, 2, 3, 4):
        with torch.cuda.stream(stream):
            h.block_hop(nblk, prec, w.nrhs, hop, warm, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            n_in, n_out = h.block_hop(nblk, prec, w.nrhs, hop, reps, stream=stream)
            e1.record(stream)
            stream.synchronize()
        ms = e0.elapsed_time(e1) / reps
        by = block_hop_bytes(prec, w.Ls, w.nrhs, n_in, n_out, {1: 0, 2: 1, 3: 0, 4: 2}[hop] * n_be)
        fl = HOP_FLOPS_PER_SITE5 * n_out * w.Ls * w.nrhs
        out[hop] = {"us": ms * 1e3, "bytes": by, "GB/s": by / (ms * 1e-3) / 1e9,
                    "frac_hbm": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "flops": fl,
                    "TFLOP/s": fl / (ms * 1e-3) / 1e12, "frac_valu": fl / (ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS,
                    "sites_in": n_in, "sites_out": n_out}
    return out


def host_description():
    """nproc (CPUs this process may use) and the CPU model."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return ncpu, model


def sample_box(L, Ls, max_sites5):
    """A sub-lattice of L (extents halved, t first, then z, y, x, each kept even
    and >= 2) whose 5D sites per parity are at most max_sites5."""
    box = list(L)
    while (np.prod(box) // 2) * Ls > max_sites5:
        for mu in (3, 2, 1, 0):
            if box[mu] >= 4 and (box[mu] // 2) % 2 == 0:
                box[mu] //= 2
                break
        else:
            break
    return tuple(box)


def time_oracle_A(w, box, threads, reps=5):
    """Median seconds of `reps` oracle applications of A = D_PC^+ D_PC on a
    periodic `box` with `threads` OpenMP threads."""
    import oracle as O

    O.set_num_threads(threads)
    U = synth.gauge_field(box, 0.43, 5)
    oa = O.Action(box, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c)
    x = synth.cb_field(box, w.Ls, 1, 6)[0]
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        O.mdagm(oa, U, x)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def cpu_baseline(w, cg_iters, reliable):
    """The FP64 CPU oracle on the host: measured time per application of A
    (median of 5, all cores and one core, on sub-lattice samples of the
    workload with its Ls), scaled to the workload's volume and right-hand
    sides, and projected to plain CG: A applications at the GPU's plain-CG
    iteration count (one per iteration, the initial and final true residuals
    and the reliable updates).  The vector updates, about 3% of the oracle's
    flops, are left out: a projection, labelled as such."""
    import oracle as O

    ncpu, model = host_description()
    threads = O.num_threads()
    sites_full = (w.V // 2) * w.Ls
    box_all = sample_box(w.L, w.Ls, 2_500_000)
    box_one = sample_box(w.L, w.Ls, 250_000)
    t_all = time_oracle_A(w, box_all, threads)
    t_one = time_oracle_A(w, box_one, 1)
    O.set_num_threads(threads)
    per_all = t_all * sites_full / ((np.prod(box_all) // 2) * w.Ls) * w.nrhs
    per_one = t_one * sites_full / ((np.prod(box_one) // 2) * w.Ls) * w.nrhs
    a_total = cg_iters + 2 + (cg_iters // reliable if reliable else 0)
    return {
        "value": per_all * a_total,
        "unit": "s",
        "cores": threads,
        "kind": "oracle",
        "projection": True,
        "sample": f"oracle A = D_PC^+ D_PC, median of 5 applications on a {'x'.join(map(str, box_all))} x Ls={w.Ls} "
                  f"box with {threads} threads ({t_all:.3f} s) and on a {'x'.join(map(str, box_one))} box with 1 "
                  f"thread ({t_one:.3f} s), scaled by volume x nrhs to {per_all:.2f} s ({threads} threads) and "
                  f"{per_one:.1f} s (1 thread) per A on the workload, times the {a_total} A applications of plain "
                  f"CG at the GPU's {cg_iters} iterations (projection)",
        "s_per_A_all_cores": per_all,
        "s_per_A_one_core": per_one,
        "host_nproc": ncpu,
        "host_cpu": model,
    }


def oracle_residual(w, U, h, x, b):
    """||b - A x|| / ||b|| of a GPU solution, A applied by the FP64 CPU oracle."""
    import oracle as O

    oa = O.Action(w.L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c)
    xs, bs = h.download(x), h.download(b)
    out = []
    for r in range(w.nrhs):
        res = bs[r] - O.mdagm(oa, U, xs[r])
        out.append(float(np.linalg.norm(res) / np.linalg.norm(bs[r])))
    return out


def kernels_only(w, torch, inner_prec, nblk, k):
    """The workload of the hardware-counter runs: 10 launches each of
    dslash_eo (F64, F32, F16, BF16), m5inv (F64, F32), the four block hops of
    the inner iteration (inner precision, after one preconditioner call fills
    the block vectors), then 10 plain copies (F64 -> F64 conversion, which reads
    and writes exactly one field) that calibrate the HBM byte counters."""
    eps = w.eps if w.eps is not None else synth.tuned_eps()
    U = synth.gauge_field(w.L, eps, w.gauge_seed)
    A = M.Action(w.L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c, t_bc=-1)
    h = M.Handle(A, U)
    src = h.upload(synth.cb_field(w.L, w.Ls, w.nrhs, 99), 1, M.F64)
    for p in (M.F64, M.F32, M.F16, M.BF16):
        fin, fout = h.field(p, w.nrhs, 1), h.field(p, w.nrhs, 0)
        h.convert(fin, src)
        for _ in range(10):
            h.dslash_eo(fout, fin, 0)
        del fin, fout
    for p in (M.F64, M.F32):  # M_5^{-1}: the recurrence along the fifth dimension
        fin, fout = h.field(p, w.nrhs, 1), h.field(p, w.nrhs, 1)
        h.convert(fin, src)
        for _ in range(10):
            h.m5inv(fout, fin, 0)
        del fin, fout
    if nblk is not None:
        r = h.upload(synth.cb_field(w.L, w.Ls, w.nrhs, 97), 0, M.F64)
        z = h.field(M.F64, w.nrhs, 0)
        h.local_block_cg(z, r, nblk, k, inner_prec)
        del r, z
        torch.cuda.synchronize()
        for hop in (1, 2, 3, 4):  # (as the solve launches them: the fused dot product on the second)
            h.block_hop(nblk, inner_prec, w.nrhs, hop, 10)
    dst = h.field(M.F64, w.nrhs, 1)
    for _ in range(10):
        h.convert(dst, src)
    torch.cuda.synchronize()
    field_bytes = (A.V // 2) * w.Ls * w.nrhs * 24 * 8
    print(json.dumps({"kernels_only": w.name, "copy_bytes_read": field_bytes, "copy_bytes_written": field_bytes}),
          flush=True)


def oracle_check(w, torch, inner_prec, nblk, k):
    """The GPU's MSPCG and plain-CG solutions against a full FP64 CPU oracle
    solve (plain CG from x = 0 to the same tolerance): relative error of each,
    their true residuals recomputed by the oracle, and the oracle's measured
    time-to-solution.  Long: the oracle runs for minutes on the larger lattices
    (a progress line every 30 s)."""
    import threading

    import oracle as O

    h, A, U, eps, b = build_problem(w, torch)
    xm, xc = h.field(M.F64, w.nrhs, 0), h.field(M.F64, w.nrhs, 0)
    h.mspcg_solve(xm, b, nblk, k, inner_prec, tol=w.tol, max_iter=20000, reliable=w.reliable)  # tunes, captures
    xm.data.zero_()
    stm = h.mspcg_solve(xm, b, nblk, k, inner_prec, tol=w.tol, max_iter=20000, reliable=w.reliable)
    stc = h.cg_solve(xc, b, tol=w.tol, max_iter=50000, reliable=w.reliable)
    log(f"[oracle-check] GPU: MSPCG {stm['outer_iters']} outer {stm['seconds']:.2f}s, "
        f"CG {stc['outer_iters']} {stc['seconds']:.2f}s")
    bs, xms, xcs = h.download(b), h.download(xm), h.download(xc)
    oa = O.Action(w.L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c)
    rows = []
    for r in range(w.nrhs):
        done = threading.Event()
        t0 = time.perf_counter()

        def progress():
            while not done.wait(30.0):
                log(f"[oracle-check] oracle CG on rhs {r} running, {time.perf_counter() - t0:.0f}s")

        th = threading.Thread(target=progress, daemon=True)
        th.start()
        xo, st_o = O.solve(oa, U, bs[r], tol=w.tol, maxiter=50000, reliable=w.reliable)
        done.set()
        th.join()
        t_o = time.perf_counter() - t0
        log(f"[oracle-check] oracle CG rhs {r}: {st_o.iters} iterations, {t_o:.1f}s")

        def rel(a, c):
            return float(np.linalg.norm(a - c) / np.linalg.norm(c))

        res = {}
        for name, xs in (("mspcg", xms[r]), ("cg", xcs[r])):
            res[name] = float(np.linalg.norm(bs[r] - O.mdagm(oa, U, xs)) / np.linalg.norm(bs[r]))
        rows.append({"rhs": r, "oracle_cg_iters": st_o.iters, "oracle_cg_seconds": t_o,
                     "oracle_cg_true_rel_resid": st_o.true_rel_resid,
                     "mspcg_rel_error_vs_oracle": rel(xms[r], xo), "cg_rel_error_vs_oracle": rel(xcs[r], xo),
                     "mspcg_true_rel_resid_oracle": res["mspcg"], "cg_true_rel_resid_oracle": res["cg"]})
    ncpu, model = host_description()
    print(json.dumps({"oracle_check": w.name, "oracle_threads": O.num_threads(), "host_nproc": ncpu,
                      "host_cpu": model, "gpu_mspcg": {"outer_iters": stm["outer_iters"], "seconds": stm["seconds"]},
                      "gpu_cg": {"iters": stc["outer_iters"], "seconds": stc["seconds"]}, "rows": rows}),
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
                    first = None
                    for rep in range(reps):  # the first solve of a shape tunes and captures
                        x.data.zero_()
                        st = h.mspcg_solve(x, b, w.nblk, k, prec, tol=w.tol, max_iter=max_iter,
                                           reliable=w.reliable, no_snake=no_snake, inner_tol=itol, n_sweeps=nsw)
                        first = st["seconds"] if first is None else first
                    rows.append({"solver": "mspcg", "k": k, "snake_terms": not no_snake, "inner_tol": itol,
                                 "sweeps": nsw, "status": st["status"], "outer_iters": st["outer_iters"],
                                 "inner_iters": st["inner_iters"], "seconds": st["seconds"],
                                 "first_solve_seconds": first, "tuning_and_capture_s": first - st["seconds"],
                                 "vs_cg": rows[0]["seconds"] / st["seconds"],
                                 "true_rel_resid": st["true_rel_resid"]})
                    log(f"[study] k={k} snake={not no_snake} inner_tol={itol:g} sweeps={nsw}: "
                        f"{st['outer_iters']} outer, {st['seconds']:.3f}s (first solve {first:.3f}s), "
                        f"{rows[0]['seconds'] / st['seconds']:.3f}x plain CG")
    print(json.dumps({"study": "inner iterations and snake terms", "workload": w.name,
                      "inner_prec": inner_prec or w.inner_prec, "blocks": list(w.nblk), "tol": w.tol, "rows": rows}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--inner-prec", default=None)
    ap.add_argument("--n-inner", type=int, default=None)
    ap.add_argument("--cg-steps", type=int, default=1)
    ap.add_argument("--extra-k", type=int, default=4,
                    help="one more MSPCG solve (warm, then timed) with this many inner iterations, reported beside "
                         "the configured one (4: the fastest of the inner-iteration study on 24^3x64x24); 0: none")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-residual", action="store_true",
                    help="skip the oracle's recomputation of the MSPCG solution's true residual")
    ap.add_argument("--oracle-check", action="store_true",
                    help="full FP64 CPU oracle CG solve next to the GPU's solves (relative errors; minutes)")
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
                    help="only launch the operator kernels (dslash_eo, m5inv, block hops) and a plain F64 copy, "
                         "10 times each (the workload for hardware-counter runs)")
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
        kernels_only(w, torch, inner_prec, nblk, k)
        return
    if args.oracle_check:
        oracle_check(w, torch, inner_prec, nblk, k)
        return
    if args.study:
        study(w, torch, ks=tuple(int(v) for v in args.study_k.split(",")), inner_prec=args.inner_prec,
              snake_modes=(0,) if args.study_snake_only else (1,) if args.study_no_snake_only else (0, 1),
              inner_tols=tuple(float(v) for v in args.study_inner_tol.split(",")),
              sweeps=tuple(int(v) for v in args.study_sweeps.split(",")), max_iter=args.study_max_iter,
              reps=max(1, args.study_reps))
        return
    if nblk is None:
        print(f"bench.py times MSPCG: workload {w.name} has no blocking", file=sys.stderr)
        sys.exit(2)
    h, A, U, eps, b = build_problem(w, torch)
    x = h.field(M.F64, w.nrhs, 0)

    def mspcg_step(timing=0):
        x.data.zero_()
        return h.mspcg_solve(x, b, nblk, k, inner_prec, tol=w.tol, max_iter=20000, reliable=w.reliable,
                             timing=timing)

    first_s, split = None, None
    for i in range(args.warmup):
        log(f"[bench] warmup mspcg {i}" + (" (tunes launch shapes, captures the preconditioner)" if i == 0 else ""))
        timing = 1 if (i == args.warmup - 1 and i > 0) else 0
        st = mspcg_step(timing)
        if i == 0:
            first_s = st["seconds"]
        if timing:
            split = st
        log(f"[bench] warmup mspcg {i}: {st['outer_iters']} outer, {st['seconds']:.3f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(mspcg_step())
        log(f"[bench] step {i}: {stats[-1]['outer_iters']} outer, {stats[-1]['seconds']:.3f}s")
    torch.cuda.synchronize()
    t_ms = (time.perf_counter() - t0) / args.steps
    if split is None:  # fewer than two warm-up solves: one more, untimed, for the time split
        split = mspcg_step(1)
    resid_oracle = None
    if not args.no_oracle_residual:
        t1 = time.perf_counter()
        resid_oracle = oracle_residual(w, U, h, x, b)
        log(f"[bench] oracle true residual of the MSPCG solution {resid_oracle} ({time.perf_counter() - t1:.1f}s)")

    cg_stats, t_cg, cg_split = None, None, None
    if args.cg_steps > 0:
        x.data.zero_()
        cg_split = h.cg_solve(x, b, tol=w.tol, max_iter=50000, reliable=w.reliable, timing=1)  # warm, untimed
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.cg_steps):
            x.data.zero_()
            cg_stats = h.cg_solve(x, b, tol=w.tol, max_iter=50000, reliable=w.reliable)
            log(f"[bench] plain CG {i}: {cg_stats['outer_iters']} iterations, {cg_stats['seconds']:.3f}s")
        torch.cuda.synchronize()
        t_cg = (time.perf_counter() - t1) / args.cg_steps

    extra = None
    if args.extra_k > 0 and args.extra_k != k:
        for rep in range(2):  # (the first tunes and captures the new graph)
            x.data.zero_()
            st_e = h.mspcg_solve(x, b, nblk, args.extra_k, inner_prec, tol=w.tol, max_iter=20000,
                                 reliable=w.reliable)
        extra = {"n_inner": args.extra_k, "seconds": st_e["seconds"], "outer_iters": st_e["outer_iters"],
                 "inner_iters": st_e["inner_iters"], "true_rel_resid": st_e["true_rel_resid"],
                 "speedup_vs_cg": None if t_cg is None else t_cg / st_e["seconds"]}
        log(f"[bench] MSPCG with k={args.extra_k}: {st_e['outer_iters']} outer, {st_e['seconds']:.3f}s")

    dsl = {p: time_dslash(h, A, w, PREC[p]) for p in ("f64", "f32", "f16", "bf16")}
    for p, d in dsl.items():
        log(f"[bench] dslash_eo {p}: {d['ms'] * 1e3:.1f} us, {d['gbs']:.0f} GB/s")
    m5 = {p: time_m5inv(h, A, w, PREC[p]) for p in ("f64", "f32")}
    for p, d in m5.items():
        log(f"[bench] m5inv {p}: {d['us']:.1f} us, {d['GB/s']:.0f} GB/s")
    bh = time_block_hops(h, w, inner_prec, nblk)
    pn = PNAME[inner_prec]
    for hop, d in bh.items():
        log(f"[bench] block hop {hop} {pn}: {d['us']:.1f} us, {d['GB/s']:.0f} GB/s ({d['frac_hbm']:.2f})")
    # the dominant kernel of the timed step: the block hop with the largest time per inner
    # iteration (k launches per outer iteration each, against one per outer iteration for
    # each FP64 hop of the outer operator)
    dom = max(bh, key=lambda hop: bh[hop]["us"])
    d = bh[dom]
    outer = stats[-1]["outer_iters"]
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
        "dtype": "f64+" + pn,
        "data": "synthetic",
        "config": {
            "workload": w.name, "lattice": list(w.L), "Ls": w.Ls, "nrhs": w.nrhs, "mobius_b_c": [w.b, w.c],
            "M5": w.M5, "mf": w.mf, "blocks": list(nblk), "n_inner": k, "inner_prec": pn, "tol": w.tol,
            "reliable": w.reliable, "gauge_eps": round(eps, 5),
        },
        "mspcg": {"seconds": t_ms, "outer_iters": outer, "inner_iters": stats[-1]["inner_iters"],
                  "true_rel_resid": stats[-1]["true_rel_resid"], "true_rel_resid_oracle": resid_oracle,
                  "first_solve_s_with_tuning_and_capture": first_s,
                  "time_split_s": {"outer_operator": split["t_outer_op"], "preconditioner": split["t_precond"],
                                   "outer_blas": split["t_blas"], "solve": split["seconds"]}},
        "plain_cg": None if cg_stats is None else {
            "seconds": t_cg, "iters": cg_stats["outer_iters"], "true_rel_resid": cg_stats["true_rel_resid"],
            "time_split_s": {"outer_operator": cg_split["t_outer_op"], "outer_blas": cg_split["t_blas"]}},
        "mspcg_speedup_vs_cg": None if t_cg is None else t_cg / t_ms,
        "mspcg_other_k": extra,
        "dslash_eo": {p: {"us": v["ms"] * 1e3, "GB/s": v["gbs"], "frac_hbm": v["gbs"] / HBM_PEAK_GBS,
                          "traffic": measured_traffic(w.name, f"dslash_eo_{p}")} for p, v in dsl.items()},
        "m5inv": m5,
        "block_hops": {f"hop{hop}_{pn}": {**v, "traffic": measured_traffic(w.name, f"block_hop{hop}_{pn}")}
                       for hop, v in bh.items()},
        # the FP16 block hops are bound by vector-instruction issue (hardware
        # counters: VALU busy about 3/4 of the launch, HBM about half), so the
        # roofline is the vector ALU's; the HBM figures are kept beside it
        "roofline": {"bound": "alu", "achieved": d["TFLOP/s"], "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": d["frac_valu"], "traffic": measured_traffic(w.name, f"block_hop{dom}_{pn}"),
                     "algorithmic_flops": d["flops"], "algorithmic_bytes": d["bytes"], "hbm_GB/s": d["GB/s"],
                     "hbm_frac": d["frac_hbm"], "avg_launch_us": d["us"],
                     "kernel": f"hop_kernel<{pn}> block hop {dom} of the inner iteration "
                               f"({k * (outer + 1)} launches per solve)"},
    }
    if not args.no_cpu_baseline and cg_stats is not None:
        out["cpu_baseline"] = cpu_baseline(w, cg_stats["outer_iters"], w.reliable)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
