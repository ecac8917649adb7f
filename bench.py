"""Benchmark: hybrid VSIE matrix-vector products per second and GMRES time-to-1e-6 at 2 mm.

Workload: 96x112x128 voxels at 2 mm (head-like phantom, seed 0), eight conformal loops on a
120 mm cylinder (near, pFFT), open tube shield r = 340 mm, L = 1.2 m, ~20k triangles (far:
dense block + ACA + TT). One step is one application of the full operator of eq. (15) in
FP64 to one right-hand side already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-solve] [--no-cpu-baseline]

Prints one JSON line. Runs on one GPU only.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def stage_bytes(info, s):
    """Algorithmic HBM bytes of one launch of each matvec stage (FP64: 16 B per complex value)."""
    c = 16
    ne1, ne2, ne3 = info["n_ext"]
    P1, P2, P3 = info["fft"]
    n1, n2, n3 = info["n"]
    nv = n1 * n2 * n3
    Ne = ne1 * ne2 * ne3
    SO = (P1 // 2 + 1) * (P2 // 2 + 1) * (P3 // 2 + 1)
    mf, mn = info["m_far"], info["m_near"]
    # body currents couple only at tissue voxels (chi != 0); the kernels that take them read x_b
    # inside each x row's tissue run only, and the TT update of y_b touches tissue voxels only
    nt = info["n_tissue"]
    b = {
        # the grid build is fused into the first pass: it reads the body currents at tissue voxels
        # (and, per grid voxel, one 4-byte projection-row index) and writes the x-transformed rows
        "fft_x_fwd": c * (3 * nt + 3 * ne3 * ne2 * P1) + 4 * Ne,
        "fft_y_fwd": c * (3 * ne3 * ne2 * P1 + 3 * ne3 * P2 * P1),
        "fft_z_conv": c * (2 * 3 * ne3 * P2 * P1 + 6 * SO),
        "fft_y_inv": c * (3 * ne3 * P2 * P1 + 3 * ne3 * ne2 * P1),
        "fft_x_inv": c * (3 * ne3 * ne2 * P1 + 3 * Ne),
        # x_b read and y_b written everywhere (identity rows in air); the x-pass output and dv/chi
        # read at tissue voxels only; one mask byte per voxel
        "body_out": c * (2 * 3 * nv + 3 * nt + nt) + nv,
        "pfft_gather": mn * 375 * (8 + c),
        # unique entries of the complex-symmetric far block plus x; the packed-tile partial sums
        # are charged to the reduction kernel
        "gemv_far": c * (mf * (mf + 1) // 2 + mf),
        "gemv_far_reduce": c * (((mf + 127) // 128) * mf + mf),
        "precorrect": info["precorr_nnz"] * (c + 4 + c),
        "aca": 2 * c * (mf + mn) * info["aca_rank"],
    }
    r = info["tt_rank"]
    # tt_pre, per component: x_b at tissue voxels and each of the four cores once (G4 serves the
    # forward and the transpose products in one pass), plus x_f read and y_f updated once;
    # tt_post, per component: the first two cores and the read-modify-write of y_b at tissue voxels
    b["tt_pre"] = sum(c * (nt + n1 * r[a][0] + r[a][0] * n2 * r[a][1] + r[a][1] * n3 * r[a][2] + r[a][2] * mf)
                      for a in range(3)) + c * 3 * mf
    b["tt_post"] = sum(c * (2 * nt + n1 * r[a][0] + r[a][0] * n2 * r[a][1]) for a in range(3))
    return b.get(s)


KERNEL_OF_STAGE = {   # stages that are a single kernel launch, and that kernel's name
    "fft_x_fwd": "k_fft2", "fft_y_fwd": "k_fft2", "fft_z_conv": "k_zconv4",
    "fft_y_inv": "k_fft2", "fft_x_inv": "k_fft2", "body_out": "k_body_out", "pfft_gather": "k_pfft_gather",
    "gemv_far": "k_symv_tiles", "gemv_far_reduce": "k_symv_reduce", "precorrect": "k_csr_add",
}


def kernel_source_sha(kernel):
    """sha256 over the kernel's own source, its launcher(s) and the compile-time constants of the
    shared kernel header (tile sizes and layouts): the traffic figure is void once any of them
    changes."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2206_12409_amd", "csrc")
    text = open(os.path.join(csrc, "kernels.hip")).read()
    parts = []
    for key in ("void %s(" % kernel, "void launch_%s" % kernel.replace("k_", "", 1)):
        at = text.find(key)
        while at >= 0:
            brace, semi = text.find("{", at), text.find(";", at)
            if 0 <= brace < semi:   # a definition, not a declaration or instantiation
                start = text.rfind("\ntemplate", 0, at)
                start = start if start >= 0 else at
                end = text.find("\n}\n", at)
                parts.append(text[start:end])
            at = text.find(key, at + len(key))
    parts += [ln for ln in open(os.path.join(csrc, "kernels.h")) if ln.startswith("constexpr")]
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was taken on the
    kernel as it is now; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_2mm.txt" % kernel)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_sha(kernel) or "traffic_bytes" not in kv:
        return None
    return float(kv["traffic_bytes"])


def _pmc_rows(db, counter):
    import re
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                       (counter,)).fetchall()
    con.close()
    return [(re.sub(r"\(.*", "", n), float(v)) for n, v in rows]


def write_traffic(kernel, fetch_db, write_db, commands):
    """profiles/traffic_<kernel>_2mm.txt from a FETCH_SIZE run and a WRITE_SIZE run (KiB per
    dispatch), each scaled by what the counter reads for the calibration copy (512 MiB read,
    1 GiB written, float32 -> float64)."""
    copy_read, copy_written = float(1 << 29), float(1 << 30)
    out = {}
    for name, db, ref in (("fetch", fetch_db, copy_read), ("write", write_db, copy_written)):
        counter = "FETCH_SIZE" if name == "fetch" else "WRITE_SIZE"
        rows = _pmc_rows(db, counter)
        # the instantiation the product runs (the most dispatches; setup runs the others briefly)
        names = [n for n, v in rows if (kernel + "<double") in n]
        main_name = max(set(names), key=names.count) if names else None
        kv = [v for n, v in rows if n == main_name]
        cv = [v for n, v in rows if "direct_copy" in n and v * 1024 > 0.25 * ref]
        if not kv or not cv:
            raise SystemExit("no %s dispatches of %s or of the calibration copy in %s" % (counter, kernel, db))
        k_kib = sum(kv) / len(kv)
        c_kib = sum(cv) / len(cv)
        factor = ref / (c_kib * 1024)
        out[name] = (k_kib, len(kv), c_kib, factor, k_kib * 1024 * factor)
    traffic = out["fetch"][4] + out["write"][4]
    path = os.path.join(ROOT, "profiles", "traffic_%s_2mm.txt" % kernel)
    with open(path, "w") as f:
        f.write("# HBM traffic per launch of %s<double> on the 2 mm workload (MI355X)\n" % kernel)
        for c in commands:
            f.write("# command: %s\n" % c)
        for name in ("fetch", "write"):
            k_kib, n, c_kib, factor, b = out[name]
            f.write("# %s: kernel %.1f KiB/dispatch (%d dispatches), calibration copy %.1f KiB for %d B "
                    "-> factor %.4f -> %.4e B\n" % (name.upper(), k_kib, n, c_kib,
                                                     copy_read if name == "fetch" else copy_written, factor, b))
        f.write("kernel=%s\n" % kernel)
        f.write("fetch_bytes=%.6e\n" % out["fetch"][4])
        f.write("write_bytes=%.6e\n" % out["write"][4])
        f.write("traffic_bytes=%.6e\n" % traffic)
        f.write("source_sha256=%s\n" % kernel_source_sha(kernel))
    print(open(path).read())


def write_pmc_summary(kernel, db, out_name, commands):
    """profiles/<out_name>.txt: mean counter values per dispatch of `kernel` (each instantiation)
    from a rocprofv3 --pmc database, with the matrix-core rate derived from the MFMA op counters
    (512 flops per counted op) and the kernel's duration."""
    import re
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value, duration from counters_collection").fetchall()
    con.close()
    agg = {}
    for n, c, v, d in rows:
        name = re.sub(r"\(.*", "", n)
        if kernel not in name:
            continue
        a = agg.setdefault(name, {})
        a.setdefault(c, []).append(float(v))
        a.setdefault("_dur", []).append(float(d))
    peaks = {"double": 78.6, "float": 157.3}
    path = os.path.join(ROOT, "profiles", out_name + ".txt")
    with open(path, "w") as f:
        f.write("# rocprofv3 counters per dispatch (MI355X, 2 mm workload)\n")
        for c in commands:
            f.write("# command: %s\n" % c)
        for name, a in sorted(agg.items()):
            dur = sum(a["_dur"]) / len(a["_dur"])
            ndisp = max(len(v) for c, v in a.items() if c != "_dur")
            f.write("%s: %d dispatches, mean duration %.1f us\n" % (name, ndisp, dur / 1e3))
            for c, vals in sorted(a.items()):
                if c != "_dur":
                    f.write("  %-32s %.6g\n" % (c, sum(vals) / len(vals)))
            for prec, key in (("double", "SQ_INSTS_VALU_MFMA_MOPS_F64"), ("float", "SQ_INSTS_VALU_MFMA_MOPS_F32")):
                if prec in name and key in a:
                    flops = 512 * sum(a[key]) / len(a[key])
                    rate = flops / (dur * 1e-9) / 1e12
                    f.write("  matrix-core flops per dispatch %.4g -> %.2f TFLOP/s = %.3f of the %.1f TFLOP/s "
                            "dense peak\n" % (flops, rate, rate / peaks[prec], peaks[prec]))
    print(open(path).read())


def write_trace_summary(stats_csv, out_name, command, top=25):
    """profiles/<out_name>.txt: the top kernels of a rocprofv3 --kernel-trace --stats run."""
    import csv
    import re
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    path = os.path.join(ROOT, "profiles", out_name + ".txt")
    with open(path, "w") as f:
        f.write("# rocprofv3 kernel statistics (MI355X)\n# command: %s\n" % command)
        f.write("%-64s %7s %11s %11s %7s\n" % ("kernel", "calls", "total_ms", "avg_us", "pct"))
        for r in rows[:top]:
            name = re.sub(r"\(.*", "", r["Name"])[:64]
            f.write("%-64s %7s %11.3f %11.2f %7.2f\n" % (name, r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                        float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    print(open(path).read())


def copy_calibration():
    """A plain device copy of known size for scaling the FETCH_SIZE and WRITE_SIZE counters to
    bytes: float32 -> float64 conversion of 2^27 elements (512 MiB read, 1 GiB written), so the
    read and written byte counts differ and each counter can be matched to its side."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
    dst = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copy calibration: 3 x (%d B read, %d B written)" % (src.numel() * 4, dst.numel() * 8),
          file=sys.stderr, flush=True)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count()


def cpu_baseline(budget_s=6.0, solve=False):
    """The oracle on the host cores, on the small configuration of the same method (16^3 voxels at
    5 mm: sphere, 60 mm loop with one port, closed 2000-triangle shield): dense assembly of the full
    system of eq. (11) (O_direct, every block by direct quadrature), then its O(N^2) product timed
    for `budget_s`; optionally the dense LU solve of the port. The product rate in complex
    multiply-adds per second is what the oracle's dense product would run at on the 2 mm system."""
    from oracle import system
    import vsie_synth as synth
    p = synth.tiny_case()
    d = system.discretize(p)
    t0 = time.perf_counter()
    S, _ = system.assemble_direct(d)
    assemble_s = time.perf_counter() - t0
    x = synth.complex_normal(d.N, 3)
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        S.matvec(x)
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    out = dict(macs_per_s=S.Z.shape[0] * S.Z.shape[1] / dt, n_coupled=S.Z.shape[0], n_total=d.N, reps=reps,
               product_s=dt, assemble_s=assemble_s)
    if solve:
        t0 = time.perf_counter()
        S.solve(system.port_rhs(d, 0))
        out["lu_solve_s"] = time.perf_counter() - t0
    return out


def other_precisions(op, x, y, args):
    """complex64 product rate and error, and the FP64 rate with the far-block chain on a second
    stream (checked to give the identical result)."""
    import torch
    x32 = x.to(torch.complex64)
    y32 = torch.empty_like(x32)
    for _ in range(args.warmup):
        op.matvec(x32, out=y32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n32 = max(10, args.steps // 2)
    for _ in range(n32):
        op.matvec(x32, out=y32)
    torch.cuda.synchronize()
    value32 = n32 / (time.perf_counter() - t0)
    err32 = float(torch.linalg.norm(y32.to(torch.complex128) - y) / torch.linalg.norm(y))
    print("fp32: %.1f matvec/s, rel err vs fp64 %.2e" % (value32, err32), file=sys.stderr, flush=True)
    # complex64 stage times (the paper's three named parts in complex64)
    op.profile(True)
    for _ in range(20):
        op.matvec(x32, out=y32)
    st32 = {k: v[0] / v[1] for k, v in op.profile_read().items()}
    op.profile(False)
    tp = ["build_grid", "fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv", "body_out", "pfft_gather",
          "precorrect", "tt_pre", "tt_post"]
    t32 = sum(st32.get(k, 0) for k in tp)
    print("fp32 stage ms: %s" % json.dumps({k: round(v, 4) for k, v in st32.items()}), file=sys.stderr, flush=True)
    value32 = dict(value=value32, three_parts_ms=round(t32, 4), three_parts_per_s=round(1e3 / t32, 1) if t32 else None)

    # the same product with the far-block chain on a second stream
    op.set_concurrency(True)
    yc = torch.empty_like(x)
    for _ in range(args.warmup):
        op.matvec(x, out=yc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.matvec(x, out=yc)
    torch.cuda.synchronize()
    value_conc = args.steps / (time.perf_counter() - t0)
    same = bool(torch.equal(yc, y))
    op.set_concurrency(False)
    print("fp64 concurrent far block: %.1f matvec/s (identical result: %s)" % (value_conc, same), file=sys.stderr,
          flush=True)

    # the same product replayed from a captured HIP graph (one submission per product)
    yg = torch.empty_like(x)
    for _ in range(args.warmup):
        op.matvec_graph(x, yg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.matvec_graph(x, yg)
    torch.cuda.synchronize()
    graph = dict(value=round(args.steps / (time.perf_counter() - t0), 3), unit="matvec/s",
                 identical_result=bool(torch.equal(yg, y)))
    print("fp64 graph-replayed product: %s" % graph, file=sys.stderr, flush=True)

    return value32, err32, value_conc, same, graph


def learned_solve(pkg, synth, op, X_plain, args):
    """The learned preconditioner at 2 mm: training pairs from the preconditioned plain solves of
    every port of other seeded phantoms (same grid), training on the GPU, then flexible GMRES on
    the workload's eliminated system with the network, against the plain preconditioned solve."""
    import torch
    t0 = time.perf_counter()
    net = pkg.Net(seed=1, pair_capacity=args.learn_pairs)
    for seed in range(100, 100 + args.learn_phantoms):
        opt = pkg.Operator(synth.two_mm_case(seed))
        n = net.collect(opt, range(opt.n_ports), restart=args.restart, max_iter=args.max_iter, tol=1e-6)
        opt.close()
        del opt
        torch.cuda.synchronize()
        print("learned: phantom %d, %d pairs held" % (seed, n), file=sys.stderr, flush=True)
    collect_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses = [net.train(1, lr=args.learn_lr, seed=e) for e in range(args.learn_epochs)]
    train_s = time.perf_counter() - t0
    net.attach(op)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, st = op.solve_ports(range(op.n_ports), tol=1e-6, restart=args.restart, max_iter=args.max_iter,
                           method=pkg.vsie.VSIE_SCHUR_LEARNED, allow_noconv=True)
    wall = time.perf_counter() - t0
    conv = [s_["rel_residual"] <= 1e-6 for s_ in st]
    # the plain method judges the result: distance from its solution, and the residual under the
    # full operator of eq. (15) applied by vsie_matvec
    diff = float(torch.linalg.norm(X - X_plain) / torch.linalg.norm(X_plain))
    B = torch.stack([op.rhs(pt) for pt in range(op.n_ports)])
    res = float(max(torch.linalg.norm(B[i] - op.matvec(X[i].contiguous())) / torch.linalg.norm(B[i])
                    for i in range(op.n_ports)))
    its = [s_["iterations"] for s_ in st]
    return dict(method="far currents eliminated, flexible GMRES with the base preconditioner plus the trained "
                       "network's body correction (bf16 MFMA convolutions)",
                train_phantoms=list(range(100, 100 + args.learn_phantoms)), pairs=net.info()["n_pairs"],
                epochs=args.learn_epochs, lr=args.learn_lr, loss_first_epoch=losses[0], loss_last_epoch=losses[-1],
                collect_seconds=round(collect_s, 2), train_seconds=round(train_s, 2),
                seconds_total=round(wall, 3), converged_ports=int(sum(conv)), mean_iterations=float(np.mean(its)),
                max_rel_residual=float(max(s_["rel_residual"] for s_ in st)), full_operator_residual=res,
                rel_diff_vs_plain=diff,
                ms_per_iteration=round(1e3 * sum(s_["seconds"] for s_ in st) / max(1, sum(its)), 3),
                time_to_1e6_mean_s=(round(float(np.mean([s_["seconds"] for s_ in st])), 4) if all(conv) else None))


def one_mm(args):
    """The 1 mm configuration (192x224x256 voxels, 32 channels, 40k-triangle shield): setup, the
    FP64 and complex64 products with their stage times, the elimination, and the preconditioned
    eliminated solve of the first ports. Prints one JSON line (an extra workload, not the 2 mm
    headline)."""
    import torch

    import paper_2206_12409_amd as pkg
    import vsie_synth as synth
    torch.cuda.set_device(0)
    problem = synth.one_mm_case()
    t0 = time.perf_counter()
    op = pkg.Operator(problem)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = op.info()
    info["n"] = tuple(int(v) for v in problem.grid.n)
    print("1 mm setup %.1f s: %s" % (setup_s, json.dumps(info)), file=sys.stderr, flush=True)
    x = torch.from_numpy(synth.complex_normal(op.N, 1234)).cuda()
    y = torch.empty_like(x)
    out = {"workload": "hybrid VSIE 1 mm: 192x224x256 head-like phantom (seed 7), 32-loop array %d near RWG, "
                       "open shield %d far RWG, 297.2 MHz" % (op.m_near, op.m_far),
           "n_unknowns": op.N, "setup_seconds": round(setup_s, 1), "info": info}
    for name, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        xx = x.to(dt)
        yy = torch.empty_like(xx)
        for _ in range(args.warmup):
            op.matvec(xx, out=yy)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.matvec(xx, out=yy)
        torch.cuda.synchronize()
        rate = args.steps / (time.perf_counter() - t0)
        op.profile(True)
        for _ in range(5):
            op.matvec(xx, out=yy)
        st = {k: round(v[0] / v[1], 4) for k, v in op.profile_read().items()}
        op.profile(False)
        out[name] = {"matvec_per_s": round(rate, 2), "ms": round(1e3 / rate, 3), "stages_ms": st}
        print("1 mm %s: %.2f matvec/s %s" % (name, rate, json.dumps(st)), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sinfo = op.schur_setup(precond=True)
    torch.cuda.synchronize()
    schur_s = time.perf_counter() - t0
    ports = list(range(min(args.one_mm_ports, op.n_ports)))
    t0 = time.perf_counter()
    X, sts = op.solve_ports(ports, tol=1e-6, restart=args.restart, max_iter=args.max_iter, method=2,
                            allow_noconv=True)
    wall = time.perf_counter() - t0
    its = [s_["iterations"] for s_ in sts]
    res = float(max(torch.linalg.norm(op.rhs(pt) - op.matvec(X[i].contiguous())) / torch.linalg.norm(op.rhs(pt))
                    for i, pt in enumerate(ports)))
    out["solve"] = dict(method="far currents eliminated, right-preconditioned GMRES", ports=ports,
                        schur_setup_seconds=round(schur_s, 1), n_proxy=sinfo["n_proxy"],
                        seconds_total=round(wall, 2), mean_iterations=float(np.mean(its)),
                        converged_ports=int(sum(s_["rel_residual"] <= 1e-6 for s_ in sts)),
                        max_rel_residual=float(max(s_["rel_residual"] for s_ in sts)), full_operator_residual=res,
                        time_to_1e6_mean_s=round(float(np.mean([s_["seconds"] for s_ in sts])), 3))
    print(json.dumps({"one_mm": out}), flush=True)


def uneven_phantoms(args):
    """Six head-like phantoms of uneven grids inside one shield (vsie_synth.uneven_phantom_set): the
    first operator assembles the dense far block, the others share it (vsie_create_shared); the
    products of all six run from one captured graph (FP64 and complex64); then every port of every
    phantom is solved with the elimination of the far currents, complex64 inner cycles and FP64
    flexible GMRES to 1e-6. Prints one JSON line (an extra workload, not the 2 mm headline)."""
    import torch

    import paper_2206_12409_amd as pkg
    import vsie_synth as synth
    torch.cuda.set_device(0)
    problems = synth.uneven_phantom_set()
    ops, setup = [], []
    for i, pr in enumerate(problems):
        t0 = time.perf_counter()
        ops.append(pkg.Operator(pr, share_far_with=ops[0] if ops else None))
        torch.cuda.synchronize()
        setup.append(round(time.perf_counter() - t0, 1))
        print("phantom %s: setup %.1f s, N %d, ports %d" % (pr.name, setup[-1], ops[-1].N, ops[-1].n_ports),
              file=sys.stderr, flush=True)
    out = {"workload": "six head-like phantoms at 2 mm (48^3 to 112x128x144), 8 to 32 channels each, one shared "
                       "open shield (%d far RWG)" % ops[0].m_far,
           "phantoms": [dict(grid=list(pr.grid.n), n_unknowns=op.N, ports=op.n_ports, setup_seconds=st)
                        for pr, op, st in zip(problems, ops, setup)]}
    for name, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        xs = [torch.from_numpy(synth.complex_normal(op.N, 500 + i)).cuda().to(dt) for i, op in enumerate(ops)]
        ys = [torch.empty_like(x) for x in xs]
        for op, x, y in zip(ops, xs, ys):
            op.matvec(x, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for op, x, y in zip(ops, xs, ys):
                op.matvec(x, out=y)
        torch.cuda.synchronize()
        eager = args.steps / (time.perf_counter() - t0)
        ref = [y.clone() for y in ys]
        G = pkg.ProductGraph(ops, xs, ys)
        G.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            G.launch()
        torch.cuda.synchronize()
        graph = args.steps / (time.perf_counter() - t0)
        same = all(bool(torch.equal(a, b)) for a, b in zip(ys, ref))
        G.close()
        out[name] = dict(batches_per_s_graph=round(graph, 2), batches_per_s_eager=round(eager, 2),
                         products_per_s_graph=round(6 * graph, 1), identical_result=same)
        print("%s: six products per graph launch %.2f/s (eager %.2f/s, identical %s)" % (name, graph, eager, same),
              file=sys.stderr, flush=True)
    solves = []
    for k, (pr, op) in enumerate(zip(problems, ops)):
        t0 = time.perf_counter()
        op.schur_setup(precond=True)
        torch.cuda.synchronize()
        s_setup = time.perf_counter() - t0
        ports = list(range(op.n_ports))
        t0 = time.perf_counter()
        X, sts = op.solve_ports(ports, tol=1e-6, restart=args.restart, max_iter=args.max_iter, method=3,
                                allow_noconv=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        b0 = op.rhs(0)
        res0 = float(torch.linalg.norm(b0 - op.matvec(X[0].contiguous())) / torch.linalg.norm(b0))
        solves.append(dict(grid=list(pr.grid.n), ports=len(ports), schur_setup_seconds=round(s_setup, 2),
                           seconds_total=round(wall, 2), seconds_per_port=round(wall / len(ports), 3),
                           converged=int(sum(s_["rel_residual"] <= 1e-6 for s_ in sts)),
                           mean_inner_iterations=float(np.mean([s_["iterations"] for s_ in sts])),
                           port0_full_operator_residual=res0))
        print("phantom %s: %s" % (pr.name, json.dumps(solves[-1])), file=sys.stderr, flush=True)
        del X
        op.close()   # frees its elimination before the next phantom's (the shared block stays)
    out["solve"] = dict(method="far currents eliminated, FP64 flexible GMRES with complex64 inner GMRES cycles",
                        phantoms=solves, ports_total=sum(s_["ports"] for s_ in solves),
                        seconds_total=round(sum(s_["seconds_total"] for s_ in solves), 2))
    print(json.dumps({"uneven_phantoms": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solve", action="store_true", help="also time the oracle's dense LU solve (small case)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner training and solve")
    ap.add_argument("--one-mm", action="store_true", help="run the 1 mm configuration instead (extra workload)")
    ap.add_argument("--one-mm-ports", type=int, default=4, help="ports solved at 1 mm")
    ap.add_argument("--uneven-phantoms", action="store_true",
                    help="run the six-phantom batch in one shield instead (extra workload)")
    ap.add_argument("--learn-phantoms", type=int, default=2, help="seeded training phantoms (seeds 100, 101, ...)")
    ap.add_argument("--learn-pairs", type=int, default=2048)
    ap.add_argument("--learn-epochs", type=int, default=3)
    ap.add_argument("--learn-lr", type=float, default=3e-4)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--max-iter", type=int, default=1000, help="iterations of the preconditioned solve")
    ap.add_argument("--plain-max-iter", type=int, default=500, help="iterations of plain GMRES and mixed IR")
    ap.add_argument("--only-fp64", action="store_true", help="skip the complex64 and concurrent-product runs")
    ap.add_argument("--solve-only", action="store_true",
                    help="set up, then only the preconditioned far-eliminated solve of every port (for profiling)")
    ap.add_argument("--calib-copy", action="store_true", help="run the copy used to scale HBM counters")
    ap.add_argument("--write-traffic", nargs=3, metavar=("KERNEL", "FETCH_DB", "WRITE_DB"),
                    help="write profiles/traffic_<KERNEL>_2mm.txt from two rocprofv3 --pmc databases")
    ap.add_argument("--write-trace", nargs=2, metavar=("STATS_CSV", "NAME"),
                    help="write profiles/NAME.txt from a rocprofv3 --kernel-trace --stats CSV")
    ap.add_argument("--write-pmc", nargs=3, metavar=("KERNEL", "DB", "NAME"),
                    help="write profiles/NAME.txt with the counters of KERNEL from a rocprofv3 --pmc database")
    ap.add_argument("--command", action="append", default=[], help="command line recorded in the summary")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.write_traffic[2], args.command)
        return
    if args.write_pmc:
        write_pmc_summary(args.write_pmc[0], args.write_pmc[1], args.write_pmc[2], args.command)
        return
    if args.write_trace:
        write_trace_summary(args.write_trace[0], args.write_trace[1], " ; ".join(args.command))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the path has no multi-GPU mode); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.one_mm:
        one_mm(args)
        return
    if args.uneven_phantoms:
        uneven_phantoms(args)
        return
    import torch

    import paper_2206_12409_amd as pkg
    import vsie_synth as synth

    torch.cuda.set_device(0)
    problem = synth.two_mm_case()
    t0 = time.perf_counter()
    op = pkg.Operator(problem)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = op.info()
    info["n"] = tuple(int(v) for v in problem.grid.n)
    print("setup %.1f s: %s" % (setup_s, json.dumps(info)), file=sys.stderr, flush=True)

    if args.solve_only:
        B = torch.stack([op.rhs(pt) for pt in range(op.n_ports)])
        sinfo = op.schur_setup(precond=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, sts = op.solve(B, tol=1e-6, restart=args.restart, max_iter=args.max_iter, method=2, allow_noconv=True)
        wall = time.perf_counter() - t0
        print(json.dumps({"solve_only": dict(ports=op.n_ports, seconds=round(wall, 3), n_proxy=sinfo["n_proxy"],
                                             iterations=[s_["iterations"] for s_ in sts],
                                             converged=all(s_["rel_residual"] <= 1e-6 for s_ in sts))}), flush=True)
        return
    if args.calib_copy:
        copy_calibration()
    x = torch.from_numpy(synth.complex_normal(op.N, 1234)).cuda()
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        op.matvec(x, out=y)
    torch.cuda.synchronize()
    # per-stage times (every stage, HIP events on the stage's stream) over a profiling pass
    op.profile(True)
    for _ in range(20):
        op.matvec(x, out=y)
    stages = op.profile_read()
    op.profile(False)
    pre = {k: v[0] / v[1] for k, v in stages.items()}
    dom = max((k for k in pre if k in KERNEL_OF_STAGE), key=pre.get)
    # timed region: K products; events only around the dominant kernel, read back afterwards
    torch.cuda.synchronize()
    op.profile(True, stages=[dom])
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.matvec(x, out=y)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dom_timed = op.profile_read()[dom]
    op.profile(False)
    value = args.steps / el
    print("fp64: %.1f matvec/s (%.3f ms)" % (value, 1e3 * el / args.steps), file=sys.stderr, flush=True)

    value32 = err32 = value_conc = same = graph = None
    batched = None
    if not args.only_fp64:
        value32, err32, value_conc, same, graph = other_precisions(op, x, y, args)
        # eight right-hand sides per call: the far block is read once for all of them (groups of up to 16)
        X8 = torch.stack([torch.from_numpy(synth.complex_normal(op.N, 2000 + s)) for s in range(8)]).cuda()
        Y8 = torch.empty_like(X8)
        for _ in range(2):
            op.matvec(X8, out=Y8)
        torch.cuda.synchronize()
        nb = max(5, args.steps // 8)
        t0 = time.perf_counter()
        for _ in range(nb):
            op.matvec(X8, out=Y8)
        torch.cuda.synchronize()
        batched = dict(nrhs=8, value=round(8 * nb / (time.perf_counter() - t0), 3), unit="RHS matvec/s",
                       dtype="c128")
        print("fp64 batched: %s" % batched, file=sys.stderr, flush=True)

    per_stage = pre
    print("stage ms: %s" % json.dumps({k: round(v, 4) for k, v in per_stage.items()}), file=sys.stderr, flush=True)
    rl = {}
    for k, ms in per_stage.items():
        b = stage_bytes(info, k)
        if b:
            rl[k] = dict(ms=round(ms, 4), gbs=round(b / (ms * 1e-3) / 1e9, 1))
    db = stage_bytes(info, dom)
    dom_ms = dom_timed[0] / dom_timed[1]
    achieved = db / (dom_ms * 1e-3) / 1e9
    conv_ms = sum(per_stage.get(k, 0) for k in ("build_grid", "fft_x_fwd", "fft_y_fwd", "fft_z_conv",
                                                   "fft_y_inv", "fft_x_inv", "body_out"))
    conv_b = sum(stage_bytes(info, k) or 0 for k in ("build_grid", "fft_x_fwd", "fft_y_fwd", "fft_z_conv",
                                                  "fft_y_inv", "fft_x_inv", "body_out"))
    print("stages: %s" % json.dumps(rl), file=sys.stderr, flush=True)

    solve = {}
    if not args.no_solve:
        B = torch.stack([op.rhs(pt) for pt in range(op.n_ports)])
        # far currents eliminated, reduced system right-preconditioned (block diagonal), GMRES(restart)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sinfo = op.schur_setup(precond=True)
        schur_setup_s = time.perf_counter() - t0
        for _ in range(3):
            op.schur_matvec(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            op.schur_matvec(x)
        torch.cuda.synchronize()
        red_ms = (time.perf_counter() - t0) / 20 * 1e3
        t0 = time.perf_counter()
        Xs, sts = op.solve(B, tol=1e-6, restart=args.restart, max_iter=args.max_iter, method=2, allow_noconv=True)
        wall = time.perf_counter() - t0
        its = [s_["iterations"] for s_ in sts]
        conv = [s_["rel_residual"] <= 1e-6 for s_ in sts]
        solve["schur_precond"] = dict(
            method="far currents eliminated (Schur complement through the ACA/TT factors), GMRES on the reduced "
                   "system right-preconditioned by its near-block inverse and the body diagonal",
            restart=args.restart, max_iter=args.max_iter, ports=op.n_ports, setup_seconds=round(schur_setup_s, 3),
            n_proxy=sinfo["n_proxy"], reduced_matvec_ms=round(red_ms, 4), seconds_total=round(wall, 3),
            converged_ports=int(sum(conv)), mean_iterations=float(np.mean(its)),
            max_rel_residual=float(max(s_["rel_residual"] for s_ in sts)),
            ms_per_iteration=round(1e3 * sum(s_["seconds"] for s_ in sts) / max(1, sum(its)), 3),
            gram_schmidt_second_passes=int(sum(s_["gs_second_passes"] for s_ in sts)),
            time_to_1e6_mean_s=(round(float(np.mean([s_["seconds"] for s_ in sts])), 4) if all(conv) else None))
        print("schur_precond: %s" % solve["schur_precond"], file=sys.stderr, flush=True)
        # the same with complex64 inner cycles under FP64 flexible GMRES
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xm, stm = op.solve(B, tol=1e-6, restart=args.restart, max_iter=args.max_iter, method=3, allow_noconv=True)
        wall = time.perf_counter() - t0
        convm = [s_["rel_residual"] <= 1e-6 for s_ in stm]
        solve["schur_precond_mixed"] = dict(
            method="as schur_precond, solved by FP64 flexible GMRES with complex64 inner GMRES cycles",
            seconds_total=round(wall, 3), converged_ports=int(sum(convm)),
            mean_inner_iterations=float(np.mean([s_["iterations"] for s_ in stm])),
            mean_fp64_steps=float(np.mean([s_["refinements"] for s_ in stm])),
            max_rel_residual=float(max(s_["rel_residual"] for s_ in stm)),
            rel_diff_vs_fp64=float(torch.linalg.norm(Xm - Xs) / torch.linalg.norm(Xs)),
            time_to_1e6_mean_s=(round(float(np.mean([s_["seconds"] for s_ in stm])), 4) if all(convm) else None))
        print("schur_precond_mixed: %s" % solve["schur_precond_mixed"], file=sys.stderr, flush=True)
        if not args.no_learned:
            solve["learned"] = learned_solve(pkg, synth, op, Xs, args)
            print("learned: %s" % solve["learned"], file=sys.stderr, flush=True)
        # plain FP64 GMRES(restart) on the full system (Sec. IV-C uses restart 50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, sts = op.solve(B, tol=1e-6, restart=args.restart, max_iter=args.plain_max_iter, allow_noconv=True)
        wall = time.perf_counter() - t0
        its = [s_["iterations"] for s_ in sts]
        conv = [s_["rel_residual"] <= 1e-6 for s_ in sts]
        solve["gmres64"] = dict(
            restart=args.restart, max_iter=args.plain_max_iter, ports=op.n_ports, seconds_total=round(wall, 3),
            converged_ports=int(sum(conv)), mean_iterations=float(np.mean(its)),
            max_rel_residual=float(max(s_["rel_residual"] for s_ in sts)),
            ms_per_iteration=round(1e3 * sum(s_["seconds"] for s_ in sts) / max(1, sum(its)), 3),
            time_to_1e6_mean_s=(round(float(np.mean([s_["seconds"] for s_ in sts])), 3) if all(conv) else None))
        print("gmres64: %s" % solve["gmres64"], file=sys.stderr, flush=True)
        xm, sm = op.solve(B[0], tol=1e-6, restart=args.restart, max_iter=args.plain_max_iter, method=1,
                          inner_tol=1e-3, allow_noconv=True)
        diff = float(torch.linalg.norm(xm - Xs[0]) / torch.linalg.norm(Xs[0]))
        solve["ir_mixed_port0"] = dict(seconds=round(sm[0]["seconds"], 3), inner_iterations=sm[0]["iterations"],
                                       fp64_steps=sm[0]["refinements"], rel_residual=sm[0]["rel_residual"],
                                       converged=sm[0]["rel_residual"] <= 1e-6, rel_diff_vs_schur=diff)
        print("ir_mixed: %s" % solve["ir_mixed_port0"], file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cb = cpu_baseline(solve=args.cpu_solve)
        n_red = op.m_far + op.m_near + 3 * info["n_tissue"]
        cpu = dict(value=cb["macs_per_s"] / float(n_red) ** 2, unit="matvec/s", cores=blas_threads(), kind="oracle",
                   sample="the oracle's dense O(N^2) product of the fully assembled system (eq. (11)) of the 16^3 "
                          "5 mm configuration (sphere, loop, closed 2000-triangle shield; %d coupled of %d "
                          "unknowns), %d products in %.1f s after a %.1f s assembly, scaled by (%d / %d)^2 to the "
                          "2 mm workload's coupled unknowns" % (cb["n_coupled"], cb["n_total"], cb["reps"],
                                                               cb["reps"] * cb["product_s"], cb["assemble_s"],
                                                               n_red, cb["n_coupled"]),
                   small_config=dict(product_s=round(cb["product_s"], 5), assemble_s=round(cb["assemble_s"], 2),
                                     lu_solve_s=round(cb["lu_solve_s"], 2) if "lu_solve_s" in cb else None))

    # the paper's three named parts: volume convolution, pFFT (projection, gather, precorrection)
    # and the TT coupling, as stage sums
    tp = ["build_grid", "fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv", "body_out", "pfft_gather",
          "precorrect", "tt_pre", "tt_post"]
    t_ms = sum(per_stage.get(k, 0) for k in tp)
    t_b = sum(stage_bytes(info, k) or 0 for k in tp)
    three = {"ms": round(t_ms, 4), "matvec_per_s": round(1e3 / t_ms, 1) if t_ms else None, "bytes": t_b,
             "gbs": round(t_b / (t_ms * 1e-3) / 1e9, 1) if t_ms else None,
             "frac": round(t_b / (t_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4) if t_ms else None}
    # the whole product of eq. (15): every stage's algorithmic bytes over the measured product time
    all_b = sum(stage_bytes(info, k) or 0 for k in per_stage)
    product_rl = {"bytes": all_b, "ms": round(1e3 / value, 4),
                  "gbs": round(all_b * value / 1e9, 1), "frac": round(all_b * value / 1e9 / PEAK_HBM_GBS, 4)}

    out = {
        "metric": "VSIE matvec/s + GMRES time-to-1e-6 at 2 mm VIR, plain vs learned-precond",
        "value": round(value, 3),
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 / value, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "hybrid VSIE 2 mm: 96x112x128 head-like phantom (seed 0), 8-loop array "
                               "%d near RWG, open shield %d far RWG, 297.2 MHz, single RHS"
                               % (op.m_near, op.m_far),
                   "n_unknowns": op.N, "n_ext": list(info["n_ext"]), "fft": list(info["fft"]),
                   "tt_rank": info["tt_rank"], "aca_rank": info["aca_rank"]},
        "roofline": {"bound": "hbm", "stage": dom, "kernel": KERNEL_OF_STAGE[dom], "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(KERNEL_OF_STAGE[dom]), "traffic_unit": "bytes per launch",
                     "bytes_per_launch": db, "avg_ms": round(dom_ms, 4),
                     "timing": "HIP events around every launch of the kernel in the timed products"},
        "volume_conv": {"ms": round(conv_ms, 4), "bytes": conv_b,
                        "gbs": round(conv_b / (conv_ms * 1e-3) / 1e9, 1) if conv_ms else None},
        "stages": rl,
        "three_parts": three,
        "roofline_product": product_rl,
        "c64": {"value": round(value32["value"], 3) if value32 else None, "unit": "matvec/s", "rel_err_vs_c128": err32,
                "three_parts_ms": value32["three_parts_ms"] if value32 else None,
                "three_parts_per_s": value32["three_parts_per_s"] if value32 else None},
        "concurrent_far_block": {"value": round(value_conc, 3) if value_conc else None, "unit": "matvec/s",
                                 "identical_result": same},
        "graph_product": graph,
        "zpass_autotune": {k: op.zpass_tuning(complex64=(k == "c64")) for k in ("c128", "c64")},
        "batched_rhs": batched,
        "solve": solve,
        "setup_seconds": round(setup_s, 2),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
