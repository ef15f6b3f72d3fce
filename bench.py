#!/usr/bin/env python3
"""SpMV benchmark on one MI355X: prints one JSON line.

One step = one product y = A x (Section 1) on the resident R-MAT scale-24 matrix, FP64 values and
int32 indices, in the headline format (CSBR: compressed sparse blocks over frequency-ranked
columns); the matrix and x are in HBM before the timed region.  --warmup untimed products, then
--steps timed ones (the paper's protocol takes the minimum of 550, Section 5.2).
value = 2 nnz / (mean time of a step), GFLOP/s.

roofline: the headline product's kernels (summed average durations from the library's HIP-event
profiler on the launch stream) against the algorithmic bytes
  B = 12 nnz + 8 n_touched + 8 m + the format's tables (block pointers, units, column order),
and the 8 TB/s HBM peak; traffic = bytes measured by rocprofv3 counters for the same kernels.

Beside the step: every format's conversion (minimum and median of --convert-reps) with its
algorithmic fraction, its steady-state product (--spmv-reps) with its roofline, break-even
counts against row-split CRS, the relabelled matrix, reduced precision, several right-hand
sides, batches, the serving loop, and the oracle on the host (cpu_baseline).
"""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
METRIC = "SpMV GFLOP/s + % HBM roofline (R-MAT s24); served p99 latency at req/s"
FMTS = ("rowsplit", "merge", "csbh", "csb", "bcohc", "bcohch", "csbr")
HEADLINE = "csbr"
WORKLOADS = {
    "rmat24": "R-MAT scale 24 (m = n = 16,777,216), edge factor 16 (268,435,456 raw entries), "
              "(a,b,c,d) = (0.57,0.19,0.19,0.05), repeats summed, FP64 values and x U(-1,1), "
              "int32 indices, seed 0",
    "chunglu": "Chung-Lu power law, gamma 2.1, n = 10,000,000, 200,000,000 raw entries, repeats "
               "summed, FP64 values and x U(-1,1), int32 indices, seed 0",
    "rmat24p": "R-MAT scale 24 as rmat24 under a random relabelling of rows and of columns "
               "(seeded permutations, streams 3 with seeds 1 and 2)",
    "rmat14": "R-MAT scale 14 (m = n = 16,384), edge factor 16, (a,b,c,d) = "
              "(0.57,0.19,0.19,0.05), FP64 values and x U(-1,1), seed 0",
}


KERNEL_SOURCES = ("k_spmv.hip", "k_spmv_crs.hip", "k_spmm.hip", "k_convert.hip", "k_hot.hip",
                  "k_partition.hip", "k_bcoh.hip", "spx_internal.h", "dev_merge.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src):
    """C++ source without its comments and with runs of white space made one blank: what the
    compiler sees, so that an edit of a comment does not mark measurements of the code stale."""
    out, i, n = [], 0, len(src)
    while i < n:
        ch = src[i]
        if ch in "\"'":  # string or character literal, copied whole
            j = i + 1
            while j < n and src[j] != ch:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(ch)
            i += 1
    return " ".join("".join(out).split())


def src_hash(*names):
    """Hash of the kernel sources' code (comments and layout left out)."""
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2502_19284_amd", "csrc", n), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def spmv_bytes(fmt, m, nnz, n_touched, A, val_bytes=8, vec_bytes=8):
    """Algorithmic bytes of one product (matrix read once, x touched columns once, y once)."""
    b = (4 + val_bytes) * nnz + vec_bytes * (n_touched + m)
    if fmt in ("rowsplit", "merge"):
        b += 4 * (m + 1)
    if fmt == "merge":
        b += 8 * (A.parts + 1) + 12 * A.parts  # tile starts, carry rows and values
    if fmt == "rowsplit":
        b += 4 * (A.parts + 1)
    if fmt in ("csbh", "csb"):
        beta = 1 << A.log2_beta
        nbr = (m + beta - 1) // beta
        nbc = (A.shape[1] + beta - 1) // beta
        b += 4 * (nbr * nbc + 1) + 16 * A.parts
    if fmt in ("bcohc", "bcohch"):
        nb = A.export("blk_coord").numel()
        b += 8 * (nb + 1) + 8 * (A.parts + 1)  # block pointers and coordinates, partition table
    if fmt == "csbr":
        # block pointers, unit table, column of each column rank, rank of each row (the ranked
        # copies of x and y are not counted: x is counted once, as read, and y once, as written)
        b += 4 * A.export("blk_ptr").numel() + 16 * A.parts + 4 * A.export("col_order").numel()
        b += 4 * m
    return b


def convert_bytes(E, nnz, m, fmt, A):
    """Algorithmic bytes of a conversion: the triplets read once (16 B each), the stored entries
    written once (12 B each) and the offsets / block pointers written."""
    b = 16 * E + 12 * nnz
    if fmt in ("rowsplit", "merge"):
        b += 4 * (m + 1)
    else:
        b += 4 * A.export("blk_ptr").numel()
    return b


def kernel_bytes(name, E, nnz, m, split_keys, split_levels):
    """Algorithmic bytes per launch of conversion kernels (None when not modelled).

    The sort's segmented split levels move different numbers of keys (every key at the top
    levels, only those of still-large segments below); split_keys / split_levels is their mean
    per launch.  A CRS or CSB conversion's first level reads the triplets instead (msd_*0_csr,
    msd_*0_csb)."""
    per_level = split_keys / split_levels if split_levels else 0
    if name in ("msd_scatter0_csr", "msd_scatter0_csb"):
        # row + col + value read, key + value written
        return 32 * E
    if name in ("msd_count0_csr", "msd_count0_csb"):
        return 8 * E
    if name == "msd_scatter":
        # read 8-byte key + 8-byte value, write both
        return 32 * per_level
    if name == "msd_count":
        return 8 * per_level
    if name == "msd_local":
        # every key and value read once and written once
        return 32 * E
    if name == "rsort_downsweep":
        return 32 * E
    if name == "rsort_upsweep":
        return 8 * E
    if name == "keys":
        return 16 * E
    if name in ("gather", "dedup_gather"):
        # sorted keys and values read once, column (packed index) and value written
        return 16 * E + 12 * nnz
    return None


def copy_probe(torch, nbytes=2 << 30, reps=20):
    """Plain device-to-device copy (torch) as the achievable-bandwidth reference: GB/s counting
    read + write."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    best = 1e30
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2 * nbytes / (best * 1e-3) / 1e9


def host_cpu():
    """Host CPU as lscpu reports it: model, sockets, cores per socket, threads per core."""
    import subprocess
    info = {"logical_cpus": os.cpu_count()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except Exception:
        return info
    keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
            "Thread(s) per core": "threads_per_core", "CPU(s)": "logical_cpus",
            "NUMA node(s)": "numa_nodes"}
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        k, v = k.strip(), v.strip()
        if k in keys:
            info[keys[k]] = int(v) if v.isdigit() else v
    if isinstance(info.get("sockets"), int) and isinstance(info.get("cores_per_socket"), int):
        info["physical_cores"] = info["sockets"] * info["cores_per_socket"]
    return info


def precision_errors(w, samples):
    """Row-scaled error |y - y_ref| / sum_k |a_ik x_k| of reduced-precision results on sampled rows
    against the FP64 oracle (its accurate Algorithm 1 restricted to those rows)."""
    import numpy as np

    from oracle import spmv as ref
    rows = samples["rows"]
    _, _, yr, sc = ref.rows_reference(w["m"], w["n"], w["row"], w["col"], w["val"], w["x"], rows)
    out = {}
    nz = sc > 0
    for name, y in samples["results"].items():
        e = np.abs(y - yr)[nz] / sc[nz]
        out[name] = {"max": float(e.max()), "median": float(np.median(e)), "rows": int(nz.sum())}
    return out


def gather_probe(spx, torch, reps=10):
    """Random 8-byte loads (library probe kernel): 2^28 loads from a 4 MiB window (inside one
    XCD's L2: the L2 request rate) and from a 128 MiB window (every load misses: the 128-byte
    line-fill rate that bounds a product's x gathers).  Rates in G loads/s, best of reps."""
    x = torch.rand(1 << 24, dtype=torch.float64, device="cuda")
    out = None
    res = {}
    n = 1 << 28
    for name, window in (("l2_window_4MiB", 1 << 19), ("hbm_window_128MiB", 1 << 24)):
        best = 1e30
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            out = spx.probe_gather(x, window, n, out)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        res[name + "_Gloads_s"] = round(n / (best * 1e-3) / 1e9, 1)
    res["line_fill_GB_s"] = round(res["hbm_window_128MiB_Gloads_s"] * 128, 1)
    del x, out
    return res


def cpu_baseline(w, budget_s=12.0):
    """The oracle on the benchmarked GPU's host cores, on a bounded sample of the same matrix (the
    rows whose index hashes into 1/8 of the range): Algorithm 1 as printed (sequential, one core) -- the
    reported value -- and, beside it, the oracle's ParCRS (Section 5.1: rows in dynamic chunks of
    512 over all host threads) and its triplet -> CRS conversion of the sample.  Only the
    products (and the conversion, separately) are timed."""
    import numpy as np

    from oracle import spmv as ref
    m, n = w["m"], w["n"]
    rows = np.arange(m, dtype=np.uint64)
    keep = ((rows * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)) < np.uint64(1 << 29)
    sel = keep[w["row"]]
    r = w["row"][sel]
    local = (np.cumsum(keep) - 1)[r].astype(np.int32)
    nrows = int(keep.sum())
    t0 = time.perf_counter()
    rp, c, v = ref.crs(nrows, n, local, w["col"][sel], w["val"][sel])
    conv_s = time.perf_counter() - t0
    nnz = int(rp[-1])

    def timed(fn, budget, cap):
        times = []
        t_start = time.perf_counter()
        while True:
            t1 = time.perf_counter()
            fn()
            times.append(time.perf_counter() - t1)
            if time.perf_counter() - t_start > budget or len(times) >= cap:
                return times
    times = timed(lambda: ref.alg1(rp, c, v, w["x"]), budget_s, 50)
    threads = ref.parcrs(rp, c, v, w["x"])[1]
    ptimes = timed(lambda: ref.parcrs(rp, c, v, w["x"]), budget_s / 3, 200)
    best, pbest = min(times), min(ptimes)
    # the bytes model of the GPU products, on the sample: CRS arrays, touched x, y
    touched = int(np.count_nonzero(np.bincount(c, minlength=n)))
    B = 12 * nnz + 4 * (nrows + 1) + 8 * (touched + nrows)
    Bc = 16 * int(sel.sum()) + 12 * nnz + 4 * (nrows + 1)  # triplets read, CRS written
    return {"value": round(2 * nnz / best / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
            "gb_s": round(B / best / 1e9, 3), "bytes_model": B,
            "kind": "oracle", "host": host_cpu(),
            "sample": "oracle Algorithm 1 (sequential, plain FP64) on the %d rows (1/8 of the "
                      "rows, chosen by a multiplicative hash of the row index) holding %d of "
                      "the workload's stored entries; minimum of %d runs, %.1f s of timed CPU work"
                      % (nrows, nnz, len(times), sum(times)),
            "ms_min": round(best * 1e3, 3), "ms_median": round(statistics.median(times) * 1e3, 3),
            "parcrs": {"value": round(2 * nnz / pbest / 1e9, 4), "unit": "GFLOP/s",
                       "gb_s": round(B / pbest / 1e9, 3),
                       "threads": threads, "ms_min": round(pbest * 1e3, 3),
                       "ms_median": round(statistics.median(ptimes) * 1e3, 3),
                       "runs": len(ptimes)},
            "crs_conversion_ms": round(conv_s * 1e3, 1),
            "crs_conversion_gb_s": round(Bc / conv_s / 1e9, 3)}


def time_products(spx, torch, A, x, y, reps):
    """reps products of a resident matrix after 10 warm-up ones: per-call event times (ms) and
    the library's per-kernel statistics over the timed calls."""
    for _ in range(10):
        A.spmv(x, out=y)
    torch.cuda.synchronize()
    spx.profile_enable(True)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        A.spmv(x, out=y)
        e1.record()
        times.append((e0, e1))
    torch.cuda.synchronize()
    ks = spx.profile_collect()
    spx.profile_enable(False)
    return [a.elapsed_time(b) for a, b in times], ks


def product_kernels(ks):
    """The kernels of one product (each launched once per product) and their summed average and
    minimum durations: the bytes model covers the whole product, so it is set against the time
    of all its kernels."""
    names = sorted(ks, key=lambda k: -ks[k]["avg_ms"])
    return ("+".join(names), sum(ks[k]["avg_ms"] for k in names),
            sum(ks[k]["min_ms"] for k in names))


def precision_leg(spx, torch, args, row_d, col_d, val_d, x_d, m, n, n_touched, copy_gbs, rows):
    """FP32 and bfloat16 stored values (FP32 x, y) in the CRS formats and CSBR: steady-state
    product and its roofline; the results on the sampled rows are kept for the error against the
    FP64 oracle (computed in the host leg, where the oracle runs)."""
    x32 = x_d.float()
    y32 = torch.empty(m, dtype=torch.float32, device="cuda")
    rows_d = torch.from_numpy(rows).cuda()
    out, results = {}, {}
    for vt, vb in (("f32", 4), ("bf16", 2)):
        for f in ("rowsplit", "merge", "csbr"):
            A = spx.convert(row_d, col_d, val_d, (m, n), f, value_type=vt)
            ms, ks = time_products(spx, torch, A, x32, y32, args.spmv_reps)
            results["%s_%s" % (f, vt)] = y32[rows_d].double().cpu().numpy()
            kname, kavg, _ = product_kernels(ks)
            B = spmv_bytes(f, m, A.nnz, n_touched, A, val_bytes=vb, vec_bytes=4)
            ach = B / (kavg * 1e-3) / 1e9
            out["%s_%s" % (f, vt)] = {
                "ms_min": round(min(ms), 4), "ms_median": round(statistics.median(ms), 4),
                "gflops_median_time": round(2 * A.nnz / (statistics.median(ms) * 1e-3) / 1e9, 1),
                "kernels": {k: round(v["avg_ms"], 4) for k, v in ks.items()},
                "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(ach / HBM_PEAK_GBS, 4),
                             "frac_of_copy": round(ach / copy_gbs, 4), "bytes_per_launch": int(B),
                             "avg_ms": round(kavg, 4)},
                "scaled_error_vs_fp64_oracle": None,
                "convert_ms": round(A.convert_ms, 3),
            }
            log("spmv %-8s %-4s median %.4f ms  %.1f GFLOP/s  %.1f%% of HBM peak"
                % (f, vt, statistics.median(ms), out["%s_%s" % (f, vt)]["gflops_median_time"],
                   100 * ach / HBM_PEAK_GBS))
            A.close()
    return out, {"rows": rows, "results": results}


def spmm_leg(spx, torch, np, synth, args):
    """Y = A X with k right-hand sides: Chung-Lu matrix (gamma 2.1, n = 10^7, 2*10^8 raw entries)
    stored in FP32, FP32 column-major X and Y, merge-path CRS; per k the product time (10 warm-up,
    --spmm-reps timed), GFLOP/s = 2 nnz k / t, and the bytes model
      B = 8 nnz + 4 (m+1) + 4 k (n_touched + m) + merge tables
    against all of the product's kernels (X staging, hot rows, tiles, carries)."""
    t0 = time.perf_counter()
    w = synth.workload("chunglu", seed=0)
    m, n = w["m"], w["n"]
    log("generated chunglu: m=%d n=%d raw=%d in %.1f s" % (m, n, len(w["row"]),
                                                          time.perf_counter() - t0))
    n_touched = int(np.count_nonzero(np.bincount(w["col"], minlength=n)))
    dev = lambda a, t: torch.from_numpy(a).to("cuda", dtype=t)
    A = spx.convert(dev(w["row"], torch.int32), dev(w["col"], torch.int32),
                    dev(w["val"], torch.float64), (m, n), "merge", value_type="f32")
    del w
    torch.cuda.empty_cache()
    gen = torch.Generator(device="cuda")
    out = {"workload": WORKLOADS["chunglu"] + "; values stored FP32, X uniform(-1,1) FP32, "
                       "column-major X and Y", "format": "merge", "nnz": A.nnz,
           "n_touched_columns": n_touched, "convert_ms": round(A.convert_ms, 3), "k": {}}
    for k in [int(v) for v in args.spmm_ks.split(",") if v]:
        gen.manual_seed(k)
        X = (torch.rand((k, n), generator=gen, device="cuda", dtype=torch.float32) * 2 - 1).t()
        Y = torch.empty((k, m), dtype=torch.float32, device="cuda").t()
        for _ in range(10):
            A.spmm(X, out=Y)
        torch.cuda.synchronize()
        spx.profile_enable(True)
        ev = []
        for _ in range(args.spmm_reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            A.spmm(X, out=Y)
            e1.record()
            ev.append((e0, e1))
        torch.cuda.synchronize()
        ks = spx.profile_collect()
        spx.profile_enable(False)
        ms = [a.elapsed_time(b) for a, b in ev]
        kname, kavg, _ = product_kernels(ks)
        B = 8 * A.nnz + 4 * (m + 1) + 4 * k * (n_touched + m) + 12 * (A.parts + 1) + 8 * k * A.parts
        ach = B / (kavg * 1e-3) / 1e9
        med = statistics.median(ms)
        out["k"][str(k)] = {
            "ms_min": round(min(ms), 4), "ms_median": round(med, 4),
            "gflops_median_time": round(2 * A.nnz * k / (med * 1e-3) / 1e9, 1),
            "kernels": {kk: round(v["avg_ms"], 4) for kk, v in ks.items()},
            "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": int(B),
                         "avg_ms": round(kavg, 4)}}
        log("spmm k=%2d median %.4f ms  %.1f GFLOP/s  %.1f%% of HBM peak  %s"
            % (k, med, out["k"][str(k)]["gflops_median_time"], 100 * ach / HBM_PEAK_GBS,
               out["k"][str(k)]["kernels"]))
        del X, Y
    A.close()
    torch.cuda.empty_cache()
    return out


def batch_matrices(synth, np, count):
    """count uneven matrices: rows log-uniform in [1e3, 1e6], average degree log-uniform in
    [4, 64], even i Chung-Lu (gamma 2.1), odd i Erdos-Renyi; FP32 values uniform(-1,1)."""
    rng = np.random.default_rng(512)
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(1e3), np.log(1e6))))
        deg = float(np.exp(rng.uniform(np.log(4), np.log(64))))
        E = int(n * deg)
        if i % 2:
            row, col = synth.uniform(n, n, E, seed=3000 + i)
        else:
            row, col = synth.chunglu(n, E, 2.1, seed=3000 + i)
        yield n, n, row, col, synth.values(E, seed=3000 + i)


def batch_leg(spx, torch, np, synth, args):
    """Products of --batch-count uneven matrices (merge-path CRS, FP32): one launch per matrix
    (eager, and captured in a graph) against the batch's single persistent launch (eager, and in
    a graph), with autotuned plans and with one fixed plan for all."""
    t0 = time.perf_counter()
    hs, xs, ys = [], [], []
    nnz = 0
    bytes_model = 0
    for m, n, row, col, val in batch_matrices(synth, np, args.batch_count):
        n_touched = int(np.count_nonzero(np.bincount(col, minlength=n)))
        d = [torch.from_numpy(a).to("cuda") for a in (row, col, val)]
        A = spx.convert(d[0], d[1], d[2], (m, n), "merge", value_type="f32")
        del d
        hs.append(A)
        xs.append(torch.rand(n, device="cuda") * 2 - 1)
        ys.append(torch.empty(m, device="cuda"))
        nnz += A.nnz
        bytes_model += 8 * A.nnz + 4 * (m + 1) + 4 * (n_touched + m)
    log("batch: %d matrices, %d stored entries, converted in %.1f s"
        % (len(hs), nnz, time.perf_counter() - t0))

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    def per_matrix():
        for A, x, y in zip(hs, xs, ys):
            A.spmv(x, out=y)

    def graphed(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return g

    out = {"matrices": "%d uneven: rows log-uniform in [1e3, 1e6], average degree log-uniform "
                       "in [4, 64], alternately Chung-Lu (gamma 2.1) and Erdos-Renyi; FP32 values"
                       % len(hs), "nnz": nnz, "bytes_model": bytes_model}
    res = {}
    res["per_matrix_eager_ms"] = timed(per_matrix)
    g1 = graphed(per_matrix)
    res["per_matrix_graph_ms"] = timed(g1.replay)
    del g1
    t1 = time.perf_counter()
    B = spx.Batch(hs)
    out["autotune_s"] = round(time.perf_counter() - t1, 2)
    out["plans"] = {p: B.plans.count(p) for p in sorted(set(B.plans))}
    B.bind(xs, ys)
    out["launch"] = B.info()
    res["batch_eager_ms"] = timed(B.spmv)
    g2 = graphed(B.spmv)
    res["batch_graph_ms"] = timed(g2.replay)
    del g2
    B.close()
    for plan in ("merge4", "merge8", "merge16"):
        Bf = spx.Batch(hs, [plan] * len(hs))
        Bf.bind(xs, ys)
        res["batch_fixed_%s_ms" % plan] = timed(Bf.spmv)
        Bf.close()
    for k, v in res.items():
        out[k] = round(v, 4)
    out["best_fixed_plan_ms"] = round(min(v for k, v in res.items()
                                          if k.startswith("batch_fixed_")), 4)
    best = min(res["batch_eager_ms"], res["batch_graph_ms"])
    out["gflops_batch"] = round(2 * nnz / (best * 1e-3) / 1e9, 1)
    out["gflops_per_matrix_eager"] = round(2 * nnz / (res["per_matrix_eager_ms"] * 1e-3) / 1e9, 1)
    ach = bytes_model / (best * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": "batch_spmv", "achieved": round(ach, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                       "bytes_per_launch": int(bytes_model)}
    log("batch: per-matrix eager %.3f ms, per-matrix graph %.3f ms, one launch %.3f ms "
        "(graph %.3f ms), best single plan for all %.3f ms; plans %s"
        % (res["per_matrix_eager_ms"], res["per_matrix_graph_ms"], res["batch_eager_ms"],
           res["batch_graph_ms"], out["best_fixed_plan_ms"], out["plans"]))
    for A in hs:
        A.close()
    del xs, ys
    torch.cuda.empty_cache()
    return out


SERVE_MATRICES = (
    "64 resident matrices, FP32 values uniform(-1,1), merge-path CRS: 56 R-MAT "
    "(a,b,c,d) = (0.57,0.19,0.19,0.05) with scale 16 + i mod 7 and edge factor 8/16/32 by "
    "(i div 7) mod 3, seed 1000 + i; 8 Erdos-Renyi with n = 2^(16 + j mod 5), average degree 8, "
    "seed 2000 + j")


def serve_matrices(synth, np):
    """The serving workload's matrices as (m, n, row, col, val) generators."""
    for i in range(56):
        scale, ef = 16 + i % 7, (8, 16, 32)[(i // 7) % 3]
        row, col = synth.rmat(scale, ef, seed=1000 + i)
        yield (1 << scale, 1 << scale, row, col, synth.values(len(row), seed=1000 + i))
    for j in range(8):
        n = 1 << (16 + j % 5)
        row, col = synth.uniform(n, n, 8 * n, seed=2000 + j)
        yield (n, n, row, col, synth.values(len(row), seed=2000 + j))


def serving_leg(spx, torch, np, synth, args):
    """Open-loop serving: Poisson arrivals at each rate for --serve-seconds, matrix chosen by a
    Zipf(1) popularity over a seeded permutation of the 64 matrices, half SpMV and half PageRank
    steps (damping 0.85).  The same schedule is replayed against the coalescing server (4 slots,
    batches of up to 32) and the plain path (one request per launch, arrival order).  Latency is
    submit -> completion seen by the scheduler; throughput is completed requests / wall time."""
    t0 = time.perf_counter()
    srv = {"coalesced": spx.Server(slots=4, max_batch=32), "plain": spx.Server(coalesce=False)}
    ids = {k: [] for k in srv}
    shapes = []
    for m, n, row, col, val in serve_matrices(synth, np):
        d = [torch.from_numpy(a).to("cuda") for a in (row, col, val)]
        for k, S in srv.items():
            mid, _ = S.add_matrix(d[0], d[1], d[2], (m, n), "merge", value_type="f32")
            ids[k].append(mid)
        shapes.append((m, n))
        del d
    log("serving: 64 matrices admitted in %.1f s" % (time.perf_counter() - t0))
    st0 = srv["coalesced"].stats()
    rng = np.random.default_rng(0)
    perm = rng.permutation(64)
    pop = 1.0 / np.arange(1, 65)
    pop = pop / pop.sum()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    xs = [torch.rand(n, generator=gen, device="cuda") * 2 - 1 for (m, n) in shapes]
    ring = 64
    ys = [[torch.empty(m, device="cuda") for _ in range(ring)] for (m, n) in shapes]
    out = {"matrices": SERVE_MATRICES, "bytes_resident": st0["bytes_resident"],
           "popularity": "Zipf(1) over a seeded permutation", "mix": "50% SpMV, 50% PageRank step",
           "rates": {}}

    def schedule(rate, seconds, seed):
        r = np.random.default_rng(seed)
        cnt = max(1, int(rate * seconds))
        arr = np.cumsum(r.exponential(1e6 / rate, cnt))
        which = perm[r.choice(64, cnt, p=pop)]
        kind = r.integers(0, 2, cnt)
        return arr, which, kind

    def reqs_for(S, key, which, kind):
        cnt = [0] * 64
        rq = []
        for w, kd in zip(which, kind):
            y = ys[w][cnt[w] % ring]
            cnt[w] += 1
            rq.append(S.request(ids[key][w], xs[w], y, "pagerank" if kd else "spmv", 0.85))
        return rq

    # warm-up: every batch width and both paths
    arr, which, kind = schedule(20000.0, 0.2, 99)
    for key, S in srv.items():
        S.replay(reqs_for(S, key, which, kind), arr)
    for rate in [float(v) for v in args.serve_rates.split(",") if v]:
        arr, which, kind = schedule(rate, args.serve_seconds, int(rate))
        row = {}
        for key, S in srv.items():
            b0 = S.stats()["batches"]
            lat, wall = S.replay(reqs_for(S, key, which, kind), arr)
            nb = S.stats()["batches"] - b0
            row[key] = {"requests": len(lat), "p50_us": round(float(np.percentile(lat, 50)), 1),
                        "p99_us": round(float(np.percentile(lat, 99)), 1),
                        "mean_us": round(float(lat.mean()), 1),
                        "throughput_req_s": round(len(lat) / (wall * 1e-6), 1),
                        "batches": nb, "mean_batch": round(len(lat) / max(nb, 1), 2)}
        log("serve %6.0f req/s: coalesced p50 %.0f us p99 %.0f us (%.0f req/s, batch %.1f) | "
            "plain p50 %.0f us p99 %.0f us (%.0f req/s)"
            % (rate, row["coalesced"]["p50_us"], row["coalesced"]["p99_us"],
               row["coalesced"]["throughput_req_s"], row["coalesced"]["mean_batch"],
               row["plain"]["p50_us"], row["plain"]["p99_us"], row["plain"]["throughput_req_s"]))
        out["rates"][str(int(rate))] = row
    for S in srv.values():
        S.close()
    del xs, ys
    torch.cuda.empty_cache()
    return out


def _short(name):
    name = name.split("(")[0].replace("void ", "")
    return name.split("<")[0] + ("<csbh>" if "<true>" in name or "KeyCsbh" in name else "")


def summarize_rocprof(prof_dir, label):
    """Markdown summary of rocprofv3 output in prof_dir and the traffic table for bench.py.

    prof_dir/trace: --kernel-trace --stats run; prof_dir/fetch: --pmc TCC_EA0_RDREQ_32B
    TCC_EA0_RDREQ_64B TCC_EA0_RDREQ_128B TCC_EA0_RDREQ; prof_dir/write: --pmc TCC_EA0_WRREQ
    TCC_EA0_WRREQ_64B; optionally prof_dir/l2: --pmc TCC_REQ TCC_HIT TCC_MISS.  Bytes read
    through the L2 = 32 / 64 / 128 x the requests of each size; bytes written = 32 x (WRREQ -
    WRREQ_64B) + 64 x WRREQ_64B.  Both are calibrated on the 2 GiB device copy of the copy
    probe (2 GiB read and 2 GiB written)."""
    import csv
    import collections
    lines = []
    stats = os.path.join(prof_dir, "trace", label + "_kernel_stats.csv")
    rows = list(csv.DictReader(open(stats)))
    lines.append("| kernel | calls | avg ms | min ms | max ms | share |")
    lines.append("|---|---|---|---|---|---|")
    for r in rows[:30]:
        lines.append("| `%s` | %s | %.4f | %.4f | %.4f | %.1f%% |" % (
            r["Name"].split("(")[0].replace("void ", "")[:70], r["Calls"],
            float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6,
            float(r["Percentage"])))
    per = {}
    for c in ("fetch", "write"):
        disp = collections.defaultdict(lambda: collections.defaultdict(float))
        names = {}
        for r in csv.DictReader(open(os.path.join(prof_dir, c, label + "_counter_collection.csv"))):
            d = int(r["Dispatch_Id"])
            disp[d][r["Counter_Name"]] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
        per[c] = {}
        for d, v in disp.items():
            if c == "fetch":
                b = 32 * v["TCC_EA0_RDREQ_32B"] + 64 * v["TCC_EA0_RDREQ_64B"] + \
                    128 * v["TCC_EA0_RDREQ_128B"]
            else:
                b = 32 * (v["TCC_EA0_WRREQ"] - v["TCC_EA0_WRREQ_64B"]) + 64 * v["TCC_EA0_WRREQ_64B"]
            per[c][d] = (names[d], b)
    gib2 = float(2 << 30)
    fac = {}
    for c in ("fetch", "write"):
        copies = [b for (nm, b) in per[c].values() if nm.startswith("__amd_rocclr_copyBuffer")]
        fac[c] = gib2 / max(copies) if copies else 1.0
    lines.append("")
    lines.append("Calibration on the 2 GiB device copy of the copy probe: bytes read x %.4f, "
                 "bytes written x %.4f." % (fac["fetch"], fac["write"]))
    lines.append("")
    lines.append("| kernel | dispatches | read GB/dispatch | written GB/dispatch | total GB/dispatch |")
    lines.append("|---|---|---|---|---|")
    agg = collections.defaultdict(lambda: [[], []])
    for i, c in enumerate(("fetch", "write")):
        for nm, b in per[c].values():
            agg[_short(nm)][i].append(b * fac[c])
    traffic = {}
    for k, (fv, wv) in sorted(agg.items(), key=lambda kv: -sum(kv[1][0]) / max(len(kv[1][0]), 1)):
        fa = sum(fv) / max(len(fv), 1)
        wa = sum(wv) / max(len(wv), 1)
        traffic[k] = fa + wa
        if fa + wa > 1e7:
            lines.append("| `%s` | %d | %.3f | %.3f | %.3f |" % (k[:60], len(fv), fa / 1e9, wa / 1e9,
                                                               (fa + wa) / 1e9))
    l2dir = os.path.join(prof_dir, "l2", label + "_counter_collection.csv")
    if os.path.exists(l2dir):
        # L2 requests and hits per dispatch (TCC_REQ, TCC_HIT summed over the channels) beside
        # the 128-byte lines fetched from memory: the two rates that bound a gather (about 261 G
        # requests/s and 56 G lines/s on this chip)
        disp = collections.defaultdict(lambda: collections.defaultdict(float))
        names = {}
        for r in csv.DictReader(open(l2dir)):
            d = int(r["Dispatch_Id"])
            disp[d][r["Counter_Name"]] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
        l2 = collections.defaultdict(list)
        for d, v in disp.items():
            l2[_short(names[d])].append((v.get("TCC_REQ", 0.0), v.get("TCC_HIT", 0.0)))
        lines.append("")
        lines.append("L2 requests and hits per dispatch (`--pmc TCC_REQ TCC_HIT TCC_MISS`), with the "
                     "128-byte lines read from memory (read bytes above / 128):")
        lines.append("")
        lines.append("| kernel | L2 requests (M) | hits (M) | hit rate | lines read (M) |")
        lines.append("|---|---|---|---|---|")
        for k, vs in sorted(l2.items(), key=lambda kv: -sum(a for a, _ in kv[1]) / len(kv[1])):
            req = sum(a for a, _ in vs) / len(vs)
            hit = sum(b for _, b in vs) / len(vs)
            if req < 1e6:
                continue
            fv = agg[k][0] if k in agg else []
            rd = sum(fv) / max(len(fv), 1) / 128
            lines.append("| `%s` | %.1f | %.1f | %.3f | %.1f |" % (k[:60], req / 1e6, hit / 1e6,
                                                                hit / max(req, 1), rd / 1e6))
    return "\n".join(lines), {"kernel_src": src_hash(*KERNEL_SOURCES),
                              "traffic_bytes_per_launch": traffic}


PIPE_COUNTERS = ("TA_TA_BUSY_sum", "TD_TD_BUSY_sum", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU",
                 "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD")


def summarize_pipe(prof_dir, label, cus=256, xcds=8):
    """Markdown table of the vector memory pipeline counters of one `--pmc` pass (PIPE_COUNTERS)
    per product kernel: the texture address (TA) and texture data (TD) units' busy cycles as a
    share of each CU's active cycles (TA / TD busy summed over the `cus` CUs, GRBM_GUI_ACTIVE
    summed over the `xcds` XCDs), and the VALU, LDS and vector-memory read instructions issued
    per dispatch (wave instructions, millions)."""
    import csv
    import collections
    disp = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for r in csv.DictReader(open(os.path.join(prof_dir, label + "_counter_collection.csv"))):
        d = int(r["Dispatch_Id"])
        disp[d][r["Counter_Name"]] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    agg = collections.defaultdict(list)
    for d, v in disp.items():
        agg[_short(names[d])].append(v)
    lines = ["| kernel | dispatches | TA busy | TD busy | VALU (M) | LDS (M) | VMEM reads (M) |",
             "|---|---|---|---|---|---|---|"]
    for k in sorted(agg):
        if not k.startswith("k_spmv") and not k.startswith("k_csbr"):
            continue
        vs = agg[k]
        mean = lambda c: sum(v[c] for v in vs) / len(vs)
        cyc = mean("GRBM_GUI_ACTIVE") / xcds
        if cyc <= 0:
            continue
        lines.append("| `%s` | %d | %.0f%% | %.0f%% | %.1f | %.1f | %.1f |" % (
            k[:60], len(vs), 100 * mean("TA_TA_BUSY_sum") / cus / cyc,
            100 * mean("TD_TD_BUSY_sum") / cus / cyc, mean("SQ_INSTS_VALU") / 1e6,
            mean("SQ_INSTS_LDS") / 1e6, mean("SQ_INSTS_VMEM_RD") / 1e6))
    return "\n".join(lines)


ALIASES = {"hot_gather": "k_hot_gather_t"}


def load_traffic(kernels):
    """Measured bytes per launch (reads + writes through the L2, from rocprofv3 counters) summed
    over `kernels`, if the table in profiles/ was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic_rmat24.json")
    if not os.path.exists(p):
        return None
    t = json.load(open(p))
    if t.get("kernel_src") != src_hash(*KERNEL_SOURCES):
        return None
    tb = t["traffic_bytes_per_launch"]
    tot = 0
    for k in kernels:
        k = ALIASES.get(k, k)
        v = tb.get(k) if k in tb else tb.get("k_" + k)
        if v is None:
            return None
        tot += v
    return int(tot)


def line_model(name):
    """Modelled 128-byte lines of x per product (16 doubles per line) on a workload, on the CPU:
    the floor each layout's order sets, used to choose the layouts (no GPU, no oracle).

    * CRS: distinct x lines among every 64 consecutive entries (one wave's gathers).
    * CSBH (beta = 2^13): distinct (block, x line) pairs - each block's lines fetched once - and
      the lines if blocks with at least T entries staged their whole 512-line x window in LDS.
    * CSBR: lines of the columns beyond the 2^18 most frequent ranks, counted once per (panel,
      line) - the frequent ones stay in L2 - for rows as given or ranked by count, columns
      ranked by count alone or by (count, first panel, last panel); and the lines the ranked
      copy of x gathers (distinct x lines among 64 consecutive ranks)."""
    import numpy as np

    import synth
    w = synth.workload(name, seed=0)
    m, n = w["m"], w["n"]
    key = np.unique((w["row"].astype(np.int64) << 32) | w["col"].astype(np.int64))
    del w
    r, c = key >> 32, key & 0xFFFFFFFF
    del key
    out = {"workload": name, "nnz": int(len(r))}
    out["crs_wave_lines_M"] = round(len(np.unique(((np.arange(len(r)) >> 6) << 32) |
                                                  (c >> 4))) / 1e6, 1)
    k = 13
    nbc = (n + (1 << k) - 1) >> k
    blk = (r >> k) * nbc + (c >> k)
    cnt_b = np.bincount(blk)
    pairs = np.unique((blk << 9) | ((c & ((1 << k) - 1)) >> 4))
    lines_b = np.bincount(pairs >> 9, minlength=len(cnt_b))
    out["csbh_block_lines_M"] = round(len(pairs) / 1e6, 1)
    out["csbh_staged"] = {}
    for T in (512, 2048, 8192):
        d = cnt_b >= T
        out["csbh_staged"][T] = {"entries_pct": round(100 * cnt_b[d].sum() / len(r), 1),
                                 "lines_gathered_M": round(lines_b[d].sum() / 1e6, 2),
                                 "lines_staged_M": round(int(d.sum()) * 512 / 1e6, 2)}
    del blk, pairs
    cnt = np.bincount(c, minlength=n)
    rcnt = np.bincount(r, minlength=m)
    order = np.lexsort((np.arange(m), -rcnt))
    ranked_rows = np.empty(m, np.int64)
    ranked_rows[order] = np.arange(m)
    H, PB = 1 << 18, 14
    out["csbr"] = {}
    for rows_name, rowmap in (("rows as given", None), ("rows ranked", ranked_rows)):
        panel = (r if rowmap is None else rowmap[r]) >> PB
        first = np.full(n, 1 << 40, np.int64)
        last = np.full(n, -1, np.int64)
        np.minimum.at(first, c, panel)
        np.maximum.at(last, c, panel)
        for cols_name, keys in (("count", (np.arange(n), -cnt)),
                                ("count, first, last", (np.arange(n), last, first, -cnt))):
            oc = np.lexsort(keys)
            rank = np.empty(n, np.int64)
            rank[oc] = np.arange(n)
            rk = rank[c]
            cold = rk >= H
            cold_lines = len(np.unique((panel[cold] << 32) | (rk[cold] >> 4)))
            nr = int((cnt > 0).sum())
            xr_lines = len(np.unique(((np.arange(nr) >> 6) << 32) | (oc[:nr] >> 4)))
            out["csbr"]["%s; columns by %s" % (rows_name, cols_name)] = {
                "cold_lines_M": round(cold_lines / 1e6, 1), "x_r_gather_lines_M":
                round(xr_lines / 1e6, 1)}
    return out


def timed_products(spx, torch, A, x, y, reps):
    """Steady-state product of a resident matrix: times, per-kernel statistics and the roofline
    of all the product's kernels against the bytes model."""
    ms, ks = time_products(spx, torch, A, x, y, reps)
    kname, kavg, kmin = product_kernels(ks)
    return ms, ks, kname, kavg, kmin


def product_record(f, A, ms, ks, kname, kavg, kmin, B, copy_gbs):
    ach = B / (kavg * 1e-3) / 1e9
    return {
        "ms_min": round(min(ms), 4), "ms_median": round(statistics.median(ms), 4),
        "runs": len(ms),
        "gflops_min_time": round(2 * A.nnz / (min(ms) * 1e-3) / 1e9, 1),
        "gflops_median_time": round(2 * A.nnz / (statistics.median(ms) * 1e-3) / 1e9, 1),
        "kernels": {k: round(v["avg_ms"], 4) for k, v in ks.items()},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "frac_of_copy": round(ach / copy_gbs, 4), "bytes_per_launch": int(B),
                     "avg_ms": round(kavg, 4), "min_ms": round(kmin, 4),
                     "traffic": load_traffic(kname.split("+"))},
        "parts": A.parts, "log2_beta": A.log2_beta,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--summarize-rocprof", metavar="DIR",
                    help="print a markdown summary of rocprofv3 CSV output in DIR and write "
                         "profiles/traffic_rmat24.json, then exit")
    ap.add_argument("--summarize-pipe", metavar="DIR",
                    help="print the pipeline counter table of a --pmc run (PIPE_COUNTERS) in DIR")
    ap.add_argument("--line-model", metavar="WORKLOAD",
                    help="print the modelled x lines per product of each layout on WORKLOAD "
                         "(CPU only, minutes; about 20 GB of host memory at scale 24), then exit")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=550, help="timed products of the step")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--headline", default=HEADLINE, help="format of the timed step")
    ap.add_argument("--spmv-reps", type=int, default=550)
    ap.add_argument("--convert-reps", type=int, default=25)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--formats", default=",".join(FMTS))
    ap.add_argument("--relabelled", type=int, default=1,
                    help="also time the headline and merge-path products on the relabelled matrix")
    ap.add_argument("--precision", type=int, default=1,
                    help="also time the FP32 / bfloat16 forms of the CRS formats")
    ap.add_argument("--spmm", type=int, default=1,
                    help="also time Y = A X with k right-hand sides on the Chung-Lu matrix")
    ap.add_argument("--spmm-ks", default="1,4,8,16,32")
    ap.add_argument("--spmm-reps", type=int, default=20)
    ap.add_argument("--batch", type=int, default=1,
                    help="also time 512 uneven matrices in one persistent launch")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--serve", type=int, default=1,
                    help="also run the serving loop over 64 resident matrices")
    ap.add_argument("--serve-rates", default="1000,5000,10000,20000,50000")
    ap.add_argument("--serve-seconds", type=float, default=0.5)
    args = ap.parse_args()
    if args.summarize_rocprof:
        md, tj = summarize_rocprof(args.summarize_rocprof, "rmat24")
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        with open(os.path.join(ROOT, "profiles", "traffic_rmat24.json"), "w") as f:
            json.dump(tj, f, indent=1, sort_keys=True)
        print(md)
        return
    if args.summarize_pipe:
        print(summarize_pipe(args.summarize_pipe, "rmat24"))
        return
    if args.line_model:
        print(json.dumps(line_model(args.line_model), indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the multi-GPU "
              "sharding is described, not run)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    fmts = [f for f in args.formats.split(",") if f]
    if args.headline not in fmts:
        fmts.append(args.headline)

    import numpy as np
    import torch

    import paper_2502_19284_amd as spx
    import synth
    if not os.path.exists(spx.LIB_PATH):
        from paper_2502_19284_amd import build as spx_build
        spx_build.build()
    spx.load()
    torch.cuda.set_device(0)
    spx.use_torch_allocator(True)

    t0 = time.perf_counter()
    w = synth.workload(args.workload, seed=0)
    m, n, E = w["m"], w["n"], len(w["row"])
    log("generated %s: m=%d n=%d raw=%d in %.1f s" % (args.workload, m, n, E,
                                                       time.perf_counter() - t0))
    counts = np.bincount(w["row"], minlength=m)
    n_touched = int(np.count_nonzero(np.bincount(w["col"], minlength=n)))
    rng = np.random.default_rng(1)
    sample_rows = np.unique(np.concatenate([rng.integers(0, m, 2000), np.argsort(counts)[-12:],
                                            [0, m - 1]])).astype(np.int64)
    dev = lambda a, t: torch.from_numpy(a).to("cuda", dtype=t)
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()  # the caller's upload of the triplets (pageable host memory)
    row_d, col_d = dev(w["row"], torch.int32), dev(w["col"], torch.int32)
    val_d = dev(w["val"], torch.float64)
    torch.cuda.synchronize()
    up_ms = (time.perf_counter() - t0) * 1e3
    up_bytes = E * (4 + 4 + 8)
    upload = {"bytes": up_bytes, "ms": round(up_ms, 2),
              "GB_s": round(up_bytes / (up_ms * 1e-3) / 1e9, 1),
              "what": "row, col (int32) and val (FP64) of the raw triplets, host numpy (pageable) "
                      "to device, before any conversion; not part of convert ms"}
    log("triplet upload %.1f ms (%.1f GB/s)" % (up_ms, upload["GB_s"]))
    x_d = dev(w["x"], torch.float64)
    y_d = torch.empty(m, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    copy_gbs = copy_probe(torch)
    gprobe = gather_probe(spx, torch)
    log("copy probe %.0f GB/s; gather probe %s" % (copy_gbs, gprobe))

    # ---------------------------------------------------------------- the step
    A = spx.convert(row_d, col_d, val_d, (m, n), args.headline)
    nnz = A.nnz
    for _ in range(args.warmup):
        A.spmv(x_d, out=y_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        A.spmv(x_d, out=y_d)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_per_step = t_steps / args.steps * 1e3
    value = 2.0 * nnz / (ms_per_step * 1e-3) / 1e9
    log("step: %d products (%s) in %.3f s, %.4f ms per product, %.1f GFLOP/s"
        % (args.steps, args.headline, t_steps, ms_per_step, value))
    ms, ks, kname, kavg, kmin = timed_products(spx, torch, A, x_d, y_d, args.spmv_reps)
    B = spmv_bytes(args.headline, m, nnz, n_touched, A)
    head = product_record(args.headline, A, ms, ks, kname, kavg, kmin, B, copy_gbs)
    dom = max(ks.items(), key=lambda kv: kv[1]["avg_ms"])
    roofline = dict(head["roofline"])
    roofline.update({"launches_per_step": len(ks), "dominant_kernel": dom[0],
                     "dominant_share": round(dom[1]["avg_ms"] / kavg, 3),
                     "bytes_model": "12 nnz + 8 n_touched + 8 m + format tables"})
    A.close()

    # ---------------------------------------------------------------- every format
    conv_ms = {}
    spmv = {}
    conv_rec = {}
    for f in fmts:
        conv_ms[f] = []
        A = None
        for r in range(max(1, args.convert_reps)):
            if A is not None:
                A.close()
            A = spx.convert(row_d, col_d, val_d, (m, n), f)
            conv_ms[f].append(A.convert_ms)
        Bc = convert_bytes(E, A.nnz, m, f, A)
        sort_b = 32 * (A.sort_split_keys + E)
        tmin = min(conv_ms[f])
        conv_rec[f] = {"ms_min": round(tmin, 3), "ms_median": round(statistics.median(conv_ms[f]), 3),
                       "runs": len(conv_ms[f]),
                       "algorithmic_bytes": int(Bc),
                       "algorithmic_frac": round(Bc / (tmin * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "sort_pass_bytes_model": int(sort_b),
                       "sort_pass_frac": round(sort_b / (tmin * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "sort_levels": A.sort_levels, "sort_split_keys": A.sort_split_keys}
        ms, ks, kname, kavg, kmin = timed_products(spx, torch, A, x_d, y_d, args.spmv_reps)
        spmv[f] = product_record(f, A, ms, ks, kname, kavg, kmin,
                                 spmv_bytes(f, m, A.nnz, n_touched, A), copy_gbs)
        log("%-8s convert %.2f ms (%.1f%% of HBM peak on its algorithmic bytes); spmv median "
            "%.4f ms  %.1f GFLOP/s  %.1f%% of HBM peak"
            % (f, tmin, 100 * conv_rec[f]["algorithmic_frac"], spmv[f]["ms_median"],
               spmv[f]["gflops_median_time"], 100 * spmv[f]["roofline"]["frac"]))
        A.close()
    be = {}
    if "rowsplit" in fmts:
        ref_conv = conv_rec["rowsplit"]["ms_min"]
        ref_spmv = spmv["rowsplit"]["ms_min"]
        for f in fmts:
            conv_rec[f]["in_rowsplit_products"] = round(conv_rec[f]["ms_min"] / ref_spmv, 1)
            if f != "rowsplit":
                N = spx.break_even(conv_rec[f]["ms_min"], ref_conv, ref_spmv, spmv[f]["ms_min"])
                be[f] = None if math.isinf(N) else round(N, 1)

    prec, prec_samples = (None, None)
    if args.precision:
        prec, prec_samples = precision_leg(spx, torch, args, row_d, col_d, val_d, x_d, m, n,
                                           n_touched, copy_gbs, sample_rows)
    del row_d, col_d, val_d, x_d, y_d
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- relabelled matrix
    relab = None
    if args.relabelled and args.workload == "rmat24":
        t0 = time.perf_counter()
        wp = synth.workload("rmat24p", seed=0)
        log("generated rmat24p in %.1f s" % (time.perf_counter() - t0))
        np_touched = int(np.count_nonzero(np.bincount(wp["col"], minlength=n)))
        rd, cd = dev(wp["row"], torch.int32), dev(wp["col"], torch.int32)
        vd, xd = dev(wp["val"], torch.float64), dev(wp["x"], torch.float64)
        del wp
        yd = torch.empty(m, dtype=torch.float64, device="cuda")
        relab = {"workload": WORKLOADS["rmat24p"], "formats": {}}
        for f in sorted({args.headline, "merge"}):
            A = spx.convert(rd, cd, vd, (m, n), f)
            ms, ks, kname, kavg, kmin = timed_products(spx, torch, A, xd, yd, args.spmv_reps)
            rec = product_record(f, A, ms, ks, kname, kavg, kmin,
                                 spmv_bytes(f, m, A.nnz, np_touched, A), copy_gbs)
            rec["convert_ms"] = round(A.convert_ms, 3)
            relab["formats"][f] = rec
            log("relabelled %-8s spmv median %.4f ms  %.1f GFLOP/s  %.1f%% of HBM peak"
                % (f, rec["ms_median"], rec["gflops_median_time"], 100 * rec["roofline"]["frac"]))
            A.close()
        del rd, cd, vd, xd, yd
        torch.cuda.empty_cache()

    mm = spmm_leg(spx, torch, np, synth, args) if args.spmm else None
    bt = batch_leg(spx, torch, np, synth, args) if args.batch else None
    served = serving_leg(spx, torch, np, synth, args) if args.serve else None

    best = max(fmts, key=lambda f: spmv[f]["gflops_median_time"])
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "m": m, "n": n, "raw_entries": E,
                   "nnz": nnz, "n_touched_columns": n_touched, "format": args.headline,
                   "step": "one y = A x on the resident matrix (matrix, x and y in HBM)",
                   "residency": "the matrix (%.1f GB) is larger than the 256 MiB MALL and streams "
                                "from HBM in every product; x (%d MB) and its ranked copy fit the "
                                "MALL and may stay there between products"
                                % (12 * nnz / 1e9, round(8 * n / 1e6))},
        "roofline": roofline,
        "spmv_steady": {"best_format": best, "gflops": spmv[best]["gflops_median_time"],
                        "hbm_frac": spmv[best]["roofline"]["frac"]},
        "spmv": spmv, "convert": conv_rec, "triplet_upload": upload,
        "break_even_vs_rowsplit": be,
        "relabelled": relab,
        "reduced_precision": prec,
        "spmm": mm,
        "batch": bt,
        "serving": served,
        "copy_probe_gbs": round(copy_gbs, 1),
        "gather_probe": gprobe,
        "kernel_src": src_hash(*KERNEL_SOURCES),
    }
    if args.cpu_baseline:
        torch.cuda.empty_cache()
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(w)
        if prec_samples is not None:
            errs = precision_errors(w, prec_samples)
            for k, e in errs.items():
                prec[k]["scaled_error_vs_fp64_oracle"] = e
                log("%s: error vs FP64 oracle on %d sampled rows: max %.3g median %.3g"
                    % (k, e["rows"], e["max"], e["median"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
