"""Benchmark: SpGEMM GFLOP/s on the irregular power-law squaring workload.

One step = the whole hot path on one MI355X: analyze (upper bounds, scan,
binning, C~ sizing) + compute (per-bin insert kernels, long-row segments and
column ranges, row pointers, allocation of C, copy into C) + plan release,
inputs already resident in HBM.  Prints one JSON line.  The roofline entry is
for the dominant kernel, timed with HIP events that the library records on
its stream during the timed steps; its algorithmic bytes are computed on the
host from the same segment / range plan the library uses.  The batched
(512 banded problems) and differentiable (forward + backward) forms are
reported beside the plain path.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
METRIC = "SpGEMM GFLOP/s and % HBM roofline; batched/backward vs plain on 1 MI355X"
WORKLOAD = ("irregular C=A*A, A 200000x200000 CSR, power-law row degrees "
            "(exponent 2.1, mean 16, cap 20000), uniform distinct columns, FP64 U[-1,1]")

# long rows (Algorithm 3 group 5): the library's plans.  Merge method
# (default when B has more columns than a dense window): one-wavefront
# segments and column ranges; column windows: pieces of 2^shift columns.
LONG_MIN = 512
WAVE_TILE = 1024
MAX_SEGS = 512
RANGE_TARGET = WAVE_TILE // 4
MIN_SHIFT, MAX_SHIFT = 4, 30
WIN_SEG, WIN_TARGET, WIN_DIRECT = 512, 512, 1024
WIN_BITMAP_LOG, WIN_SPLIT, WIN_MAX_PIECES = 18, 16384, 1024


def dense_cols(s):
    """Columns of the dense window: with at most this many columns in B the
    library takes column windows for long rows by default."""
    return 2048 if s == 8 else 4096


def win_plan(u, n, s):
    """(mode, items, shift, segments) of a long row, as the library plans it:
    'DS' direct sparse, 'DD' direct dense, 'PT' partitioned, None."""
    dl = 11 if s == 8 else 12
    if n <= (1 << dl):
        return "DD", -(-u // WIN_SPLIT), 0, 0
    if u <= WIN_DIRECT:
        return "DS", 1, 0, 0
    w = n * WIN_TARGET // u
    sh = min(int(math.floor(math.log2(w))) if w >= 1 else 0, WIN_BITMAP_LOG)
    R = -(-n // (1 << sh))
    while R > WIN_MAX_PIECES and sh < WIN_BITMAP_LOG:
        sh += 1
        R = -(-n // (1 << sh))
    if R > WIN_MAX_PIECES:
        return None, 0, 0, 0
    return "PT", R, sh, -(-u // WIN_SEG)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ext", action="store_true",
                    help="skip the batched and differentiable forms")
    ap.add_argument("--n", type=int, default=200000, help="rows (default: the full workload)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 4 device-to-device copies of MIB MiB (the calibration "
                         "kernel for the HBM byte counters) and exit")
    ap.add_argument("--batch-one-shot", action="store_true",
                    help="only run the one-shot batched product of the 512 banded problems "
                         "(1 warm-up, 3 timed; the command its kernel profile comes from)")
    ap.add_argument("--diff-backward", action="store_true",
                    help="only run the backward of the differentiable workload (plan and "
                         "forward once, then 1 warm-up and 3 timed backward calls; the command "
                         "its kernel profile comes from)")
    ap.add_argument("--diff-forward", action="store_true",
                    help="only run the forward product of the differentiable workload "
                         "(2 warm-up, 3 timed; the command its kernel profiles come from)")
    return ap.parse_args()


def copy_probe(mib):
    """A plain copy kernel of known size: FETCH_SIZE / WRITE_SIZE of this
    launch against 2 x its bytes give the counters' scale."""
    import torch
    x = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    for _ in range(4):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": mib << 20, "copy_probe_bytes_written": mib << 20,
                      "launches": 4}), flush=True)


# files the long-row kernels of each method are compiled from: counter
# figures stay valid only while these are unchanged
_CSRC = "paper_1504_05022_amd/csrc/"
KERNEL_SOURCES = {
    "merge": (_CSRC + "long.hip", _CSRC + "common.hpp", _CSRC + "internal.hpp", _CSRC + "radix.hpp"),
    "window": (_CSRC + "window.hip", _CSRC + "common.hpp", _CSRC + "internal.hpp"),
}


def source_sha1(method):
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[method]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def counters_file(kernel):
    """Committed HBM counter summary of a kernel on this workload."""
    return os.path.join(ROOT, "profiles", "%s_irregular_AxA_200k_hbm_counters.md" % kernel.split()[0])


def measured_traffic(kernel, method):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (two rocprofv3 passes, calibrated on a plain copy), or None when there is
    none for this kernel or its sources changed since it was taken."""
    try:
        kv = {}
        for line in open(counters_file(kernel)):
            if ":" in line and not line.startswith(("#", "|", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("source_sha1") != source_sha1(method) or not kernel.startswith(kv["traffic_kernel"]):
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def compulsory_bytes(A, nnz_c, s=8):
    """sum over distinct inputs [4(rows+1) + nnz(4+s)] + 4(m+1) + nnz(C)(4+s)."""
    return 4 * (A.rows + 1) + A.nnz * (4 + s) + 4 * (A.rows + 1) + nnz_c * (4 + s)


def ranges_to_index(starts, lens):
    """Concatenation of arange(starts[k], starts[k] + lens[k])."""
    lens = np.asarray(lens, np.int64)
    tot = int(lens.sum())
    if tot == 0:
        return np.zeros(0, np.int64)
    off = np.repeat(np.asarray(starts, np.int64) - (np.cumsum(lens) - lens), lens)
    return off + np.arange(tot, dtype=np.int64)


def merge_kernel_bytes(A, B, crp, cci, s):
    """Algorithmic bytes of the first passes of the two one-wavefront
    long-row kernels of the merge method.

    Segment kernel (first pass: the 512-product segments of rows longer
    than 1024 products), per segment: its A entries (P, column, value, B's
    row pointer: 16 + s bytes each), the gathered B entries (4 + s each) and
    the segment's products plus its range starts, which it writes.
    Range kernel (its first pass, 512-entry wavefront sorts), per column
    range of a split row: its entries (4 + s each, only if it holds at most
    512 of them; larger ranges go on to the next pass), its result and piece
    record; per split row, the range-start table once (4 bytes per range
    boundary and segment: a range reads the row of its own start and of the
    next range's start, so each row is counted once)."""
    arp = A.row_ptr.astype(np.int64)
    brp = B.row_ptr.astype(np.int64)
    deg = np.diff(arp)
    bdeg = np.diff(brp)
    n = B.cols
    rows_of = np.repeat(np.arange(A.rows), deg)
    w = bdeg[A.col_idx]
    u = np.bincount(rows_of, weights=w, minlength=A.rows).astype(np.int64)
    seg_bytes = 0
    rng_bytes = 0
    for i in np.nonzero(u > LONG_MIN)[0]:
        ui = int(u[i])
        e0, e1 = int(arp[i]), int(arp[i + 1])
        lens = w[e0:e1]
        starts = np.cumsum(lens) - lens
        ends = starts + lens
        if ui <= WAVE_TILE:
            continue  # one-item row: the second (1024-product) pass
        segp = max(WAVE_TILE // 2, -(-ui // MAX_SEGS))
        if segp > WAVE_TILE // 2:
            continue  # segments too long for the first pass
        nseg = -(-ui // segp)
        wdt = -(-(n * RANGE_TARGET) // ui)
        shift = min(max(int(math.ceil(math.log2(max(wdt, 1)))), MIN_SHIFT), MAX_SHIFT)
        npiece = -(-n // (1 << shift))
        p0 = np.arange(nseg, dtype=np.int64) * segp
        p1 = np.minimum(p0 + segp, ui)
        d_seg = np.searchsorted(starts, p1, "left") - np.searchsorted(ends, p0, "right")
        seg_bytes += int(d_seg.sum()) * (16 + s) + 2 * ui * (4 + s) + nseg * ((npiece + 1) * 4 + 128)
        js = A.col_idx[e0:e1]
        cols = B.col_idx[ranges_to_index(brp[js], bdeg[js])]
        E = np.bincount(cols >> shift, minlength=npiece)
        r = np.bincount(cci[int(crp[i]):int(crp[i + 1])] >> shift, minlength=npiece)
        small = E <= WAVE_TILE // 2  # the first (512-entry) wavefront pass
        rng_bytes += (npiece + 1) * nseg * 4 + int((E[small] + r[small]).sum()) * (4 + s) + npiece * 64
    return seg_bytes, rng_bytes


def window_kernel_bytes(A, B, crp, s):
    """Algorithmic bytes of one launch of each window-method kernel.

    Per A entry of a long row read by a kernel: column, value, two entries of
    the product scan P and two of B's row pointers (16 + s bytes; the
    symbolic kernel skips the value).  Per product: the B entry it gathers
    (4 + s; the symbolic kernel reads the column only), or the partial entry
    (key 4 + s) for partitioned rows.  Partition kernel: reads the row's A
    entries and B entries, writes the partials (4 + s per product) and the
    piece-start table (2 bytes per segment and piece boundary).  Symbolic
    kernel: columns only, plus the table (two entries per segment and piece)
    and an 8-byte count per item.  Numeric kernel: A and B entries (direct
    rows) or partials and table (partitioned rows), and the output entries
    written into C (4 + s each) -- the compulsory output of the long rows."""
    arp = A.row_ptr.astype(np.int64)
    brp = B.row_ptr.astype(np.int64)
    deg = np.diff(arp)
    bdeg = np.diff(brp)
    n = B.cols
    rows_of = np.repeat(np.arange(A.rows), deg)
    u = np.bincount(rows_of, weights=bdeg[A.col_idx], minlength=A.rows).astype(np.int64)
    cnnz = np.diff(crp.astype(np.int64))
    part = sym = num = 0
    for i in np.nonzero(u > LONG_MIN)[0]:
        ui, di, ci = int(u[i]), int(deg[i]), int(cnnz[i])
        mode, R, sh, nseg = win_plan(ui, n, s)
        if mode == "PT":
            part += di * (16 + s) + ui * (4 + s) + ui * (4 + s) + 2 * nseg * (R + 1)
            sym += ui * 4 + 4 * nseg * R + 8 * R
            num += ui * (4 + s) + 4 * nseg * R + ci * (4 + s)
        elif mode is not None:
            sym += di * 16 + ui * 4 + 8 * R
            num += di * (16 + s) + ui * (4 + s) + ci * (4 + s)
    return part, sym, num


def row_upper_bounds(A, B):
    """u_i = sum over the entries a_ij of nnz(b_j*) (Algorithm 2), on the host."""
    deg = np.diff(A.row_ptr.astype(np.int64))
    bdeg = np.diff(B.row_ptr.astype(np.int64))
    return np.bincount(np.repeat(np.arange(A.rows), deg), weights=bdeg[A.col_idx],
                       minlength=A.rows).astype(np.int64)


def memory_accounting(u, crp, info, s, long_min=LONG_MIN):
    """Temporary storage of one product under the three allocation schemes
    the paper compares (precise nnz(c_i); hybrid: the Algorithm 3 sizes plus
    2x growth of a long row's 256-entry slot until its result fits; upper
    bound u_i), in MB of (column, value) entries, next to the device memory
    this implementation's plan held after the product (spgemm_info)."""
    cn = np.diff(crp.astype(np.int64))
    grow = cn[u > long_min]
    cap = np.where(grow > 256, 256 * 2.0 ** np.ceil(np.log2(np.maximum(grow, 1) / 256.0)), 0)
    mb = (4 + s) / 1e6
    precise = int(cn.sum())
    hybrid = int(info.nnz_tilde) + int(cap.sum())
    upper = int(info.nnz_hat)
    return {"precise_MB": round(precise * mb, 1), "hybrid_MB": round(hybrid * mb, 1),
            "upper_bound_MB": round(upper * mb, 1),
            "hybrid_over_precise": round(hybrid / max(precise, 1), 3),
            "upper_over_precise": round(upper / max(precise, 1), 3),
            "this_implementation_scratch_MB": round(int(info.bytes_scratch) / 1e6, 1)}


def memory_table(torch, S, L):
    """Memory of the three allocation schemes and of this implementation for
    workloads 1, 3 (both products of R(AP)), 4 (summed over its problems) and
    5; workload 2 is reported with the headline."""
    def one(A, B):
        dA, dB = L.CsrMatrix.from_host(A), L.CsrMatrix.from_host(B)
        plan = L.Plan(dA, dB)
        C = plan.compute()
        torch.cuda.synchronize()
        crp = C.row_ptr.cpu().numpy()
        info = plan.info
        plan.close()
        del C, dA, dB
        return memory_accounting(row_upper_bounds(A, B), crp, info, A.val.dtype.itemsize)

    def add(rows):
        keys = ("precise_MB", "hybrid_MB", "upper_bound_MB", "this_implementation_scratch_MB")
        t = {k: round(sum(r[k] for r in rows), 1) for k in keys}
        t["hybrid_over_precise"] = round(t["hybrid_MB"] / max(t["precise_MB"], 1e-9), 3)
        t["upper_over_precise"] = round(t["upper_bound_MB"] / max(t["precise_MB"], 1e-9), 3)
        return t

    out = {}
    A1, _ = S.config1()
    out["workload1_AxA_2000"] = one(A1, A1)
    A3, P3, R3 = S.config3()
    AP = S.Csr(*gpu_product(torch, L, A3, P3))
    out["workload3_AxP"] = one(A3, P3)
    out["workload3_Rx(AP)"] = one(R3, AP)
    out["workload4_512_problems"] = add([one(a, b) for a, b in S.config4()])
    A5, B5 = S.config5()
    out["workload5_AxB"] = one(A5, B5)
    return out


def gpu_product(torch, L, A, B):
    """A*B on the GPU (this library), as a host CSR tuple."""
    C = L.spgemm(L.CsrMatrix.from_host(A), L.CsrMatrix.from_host(B))
    return C.to_host()


def extensions(args, torch, S, L):
    """Batched (workload 4) and differentiable (workload 5) forms against the
    plain path on the same GPU, and both orders of the multigrid Galerkin
    products."""
    out = {}
    reps = 5
    # ---- batched: 512 banded problems, mixed binary32 / binary64
    try:
        probs = S.config4()
        dev = [(L.CsrMatrix.from_host(a), L.CsrMatrix.from_host(b)) for a, b in probs]
        del probs
        torch.cuda.synchronize()
        b = L.Batch(dev)
        st = b.stats.as_dict()
        b.run(views=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.run(views=False)
        torch.cuda.synchronize()
        bms = (time.perf_counter() - t0) * 1e3 / reps
        b.close()
        # one-shot form: every stage inside the call (analysis, C~, ESC,
        # compaction, output allocation), nothing kept between calls
        outs, ost = L.batch_multiply(dev, return_stats=True)
        del outs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            outs = L.batch_multiply(dev)
            del outs
        torch.cuda.synchronize()
        oms = (time.perf_counter() - t0) * 1e3 / 3
        ost = ost.as_dict()
        # the same problems one plain call after another
        for a_, b_ in dev[:8]:
            L.spgemm(a_, b_)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a_, b_ in dev:
            C = L.spgemm(a_, b_)
            del C
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3
        # ... and with plans analyzed beforehand (only compute() timed), the
        # fair comparison with a batch whose structure was set up at create
        plans = [L.Plan(a_, b_) for a_, b_ in dev]
        for pl in plans[:8]:
            pl.compute()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pl in plans:
            C = pl.compute()
            del C
        torch.cuda.synchronize()
        cms = (time.perf_counter() - t0) * 1e3
        for pl in plans:
            pl.close()
        del plans, dev
        out["batched"] = {
            "workload": "512 banded problems, n log-uniform in [1024, 65536], 4-32 nnz/row "
                        "in a 5% band, FP64 even / FP32 odd",
            "ms_per_run": round(bms, 3), "gflops": round(st["flops"] / (bms * 1e-3) / 1e9, 2),
            "plain_sequential_ms": round(pms, 3),
            "plain_compute_reused_plans_ms": round(cms, 3),
            "speedup_vs_compute_reused_plans": round(cms / bms, 3),
            "plain_gflops": round(st["flops"] / (pms * 1e-3) / 1e9, 2),
            "speedup_vs_plain": round(pms / bms, 3), "flops": st["flops"], "nnz_c": st["nnz_c"],
            "fallback": st["fallback"], "bin_edges": st["bin_edges"], "shapes": st["shapes"],
            "tune_ms": [round(x, 3) for x in st["tune_ms"]],
            "one_shot_ms": round(oms, 3),
            "one_shot_speedup_vs_plain": round(pms / oms, 3),
            "one_shot_scratch_gb": round(ost["bytes_scratch"] / 1e9, 3),
            "one_shot_items": ost["items"]}
    except Exception as e:  # reported, not fatal to the headline number
        out["batched"] = {"error": repr(e)[:300]}
    torch.cuda.empty_cache()
    # ---- differentiable: A 500000^2 power law x B 500000x4096, binary32
    try:
        A, B = S.config5()
        dA, dB = L.CsrMatrix.from_host(A), L.CsrMatrix.from_host(B)
        del A, B
        plan = L.Plan(dA, dB)
        C = plan.compute()
        dc = torch.randn(C.nnz, dtype=torch.float32, device="cuda")
        plan.backward(C, dc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            C = L.spgemm(dA, dB)
        torch.cuda.synchronize()
        fms = (time.perf_counter() - t0) * 1e3 / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.backward(C, dc)
        torch.cuda.synchronize()
        bwms = (time.perf_counter() - t0) * 1e3 / reps
        fl = int(plan.info.flops)
        plan.close()
        # per-stage breakdown of the forward (every stage timer on)
        _, finfo = L.spgemm(dA, dB, return_info=True, timing=1)
        fstages = {k: round(float(v), 4) for k, v in zip(L.STAGES, finfo.stage_ms) if v > 0}
        out["backward"] = {
            "workload": "A 500000^2 power law (2.2, mean 20) x B 500000x4096 (32/row), FP32 N(0,1)",
            "forward_ms": round(fms, 3), "forward_gflops": round(fl / (fms * 1e-3) / 1e9, 2),
            "forward_stage_ms": fstages,
            "backward_ms": round(bwms, 3),
            "backward_gflops": round(2 * fl / (bwms * 1e-3) / 1e9, 2),
            "backward_over_forward": round(bwms / fms, 3), "flops_forward": fl}
    except Exception as e:
        out["backward"] = {"error": repr(e)[:300]}
    torch.cuda.empty_cache()
    # ---- merge-algorithm microbenchmark (five algorithms, three entry types)
    try:
        out["merge"] = merge_microbench(torch, L)
    except Exception as e:
        out["merge"] = {"error": repr(e)[:300]}
    torch.cuda.empty_cache()
    # ---- Galerkin products R*A*P of the multigrid experiment, both orders
    try:
        out["galerkin"] = galerkin_orders(torch, S, L, reps)
    except Exception as e:
        out["galerkin"] = {"error": repr(e)[:300]}
    torch.cuda.empty_cache()
    # ---- memory of the allocation schemes (Section 4), workloads 1, 3, 4, 5
    try:
        out["memory_workloads"] = memory_table(torch, S, L)
    except Exception as e:
        out["memory_workloads"] = {"error": repr(e)[:300]}
    return out


def merge_microbench(torch, L, total_log2=25, reps=3):
    """Merging 2^25 entries as pairs of sorted runs of length l = 2^4..2^13
    with each of the five algorithms, for 32-bit keys alone and with 32- or
    64-bit values: the best rate (Gentries/s, inputs and outputs in HBM) over
    work-group sizes 64..1024 and the size that gave it, and the fastest
    algorithm per (entry type, l)."""
    total = 1 << total_log2
    gen = torch.Generator(device="cuda")
    gen.manual_seed(150405022)
    keys0 = torch.randint(0, 1 << 31, (total,), dtype=torch.int32, device="cuda", generator=gen)
    res = {}
    for vb, name in ((0, "key32"), (4, "key32_val32"), (8, "key32_val64")):
        vals = None if vb == 0 else torch.arange(total, dtype=torch.int32 if vb == 4 else torch.int64,
                                                   device="cuda")
        per = {}
        for lg in range(4, 14):
            l = 1 << lg
            keys = keys0.view(-1, l).sort(dim=1).values.reshape(-1).contiguous()
            row = {}
            for alg in L.MERGE_ALGORITHMS:
                best = None
                for nt in (64, 128, 256, 512, 1024):
                    tile = max(2 * l, 2 * nt)
                    if alg == "merge_path" and tile // nt > 32:
                        continue
                    if tile * (4 + vb) * (2 if alg == "ranking" else 1) > 160 * 1024:
                        continue
                    L.merge_pairs(keys, vals, l, alg, nt)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        L.merge_pairs(keys, vals, l, alg, nt)
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    if best is None or ms < best[0]:
                        best = (ms, nt)
                if best is not None:
                    row[alg] = {"gentries_s": round(total / (best[0] * 1e-3) / 1e9, 2),
                                "threads": best[1]}
            if row:
                row["fastest"] = max(row, key=lambda a: row[a]["gentries_s"])
            else:
                row["fastest"] = None  # no tile of 2l entries fits in LDS
            per["l=2^%d" % lg] = row
            del keys
        res[name] = per
        del vals
    return res


def tiny_rows_ablation(torch, L, dA, nrows, reps=5):
    """Bin group 3 (rows of 2..32 products) of the headline workload: the
    wavefront ESC against the paper's heap method (one thread per row, one
    kernel per exact size), stage time from the library's event timers and
    whole-step time."""
    tiny = 1 << L.STAGES.index("tiny")
    res = {"rows": nrows}
    for key, heap in (("wavefront_esc", 0), ("heap_method", 1)):
        stage = 0.0
        L.spgemm(dA, dA, tiny_heap=heap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            C, info = L.spgemm(dA, dA, return_info=True, timing=1, timing_mask=tiny, tiny_heap=heap)
            stage += float(info.stage_ms[L.STAGES.index("tiny")])
            del C
        torch.cuda.synchronize()
        res[key] = {"stage_ms": round(stage / reps, 4),
                    "step_ms": round((time.perf_counter() - t0) * 1e3 / reps, 4)}
    res["heap_over_esc"] = round(res["heap_method"]["stage_ms"] /
                                 max(res["wavefront_esc"]["stage_ms"], 1e-9), 3)
    return res


def galerkin_orders(torch, S, L, reps):
    """R*(A*P) against (R*A)*P for the 2D 5-/9-point (1024^2) and 3D
    7-/27-point (101^3) stencils with unsmoothed 2^d aggregation, binary64:
    time of both products (analysis and computation each), their flops, and
    whether the two orders agree bit for bit (small-integer values: exact)."""
    res = {}
    for name in S.GALERKIN:
        dim, points, g = S.GALERKIN[name]
        A, P, R = S.galerkin(name)
        dA, dP, dR = (L.CsrMatrix.from_host(x) for x in (A, P, R))
        del A, P, R

        def right():
            AP, i1 = L.spgemm(dA, dP, return_info=True)
            C, i2 = L.spgemm(dR, AP, return_info=True)
            return C, int(i1.flops) + int(i2.flops)

        def left():
            RA, i1 = L.spgemm(dR, dA, return_info=True)
            C, i2 = L.spgemm(RA, dP, return_info=True)
            return C, int(i1.flops) + int(i2.flops)

        row = {"grid": "%d^%d" % (g, dim), "n_fine": g ** dim}
        outs = {}
        for key, f in (("R(AP)", right), ("(RA)P", left)):
            C, fl = f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                f()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            outs[key] = C
            row[key] = {"ms": round(ms, 3), "flops": fl, "gflops": round(fl / (ms * 1e-3) / 1e9, 2)}
        c1, c2 = outs["R(AP)"], outs["(RA)P"]
        row["nnz_coarse"] = int(c1.nnz)
        row["orders_equal"] = bool(torch.equal(c1.row_ptr, c2.row_ptr)
                                   and torch.equal(c1.col_idx, c2.col_idx)
                                   and torch.equal(c1.val, c2.val))
        row["faster"] = min(("R(AP)", "(RA)P"), key=lambda k: row[k]["ms"])
        res[name] = row
        del outs, c1, c2, dA, dP, dR
        torch.cuda.empty_cache()
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_block(args):
    """One worker of the host-cores baseline: the oracle, as it stands, on a
    block of rows of the workload (the worker draws the same seeded matrix).
    Returns (seconds of the oracle call, flops)."""
    n, r0, r1 = args
    import oracle
    import synthetic as S
    A, _ = S.config2(n=n) if n != 200000 else S.config2()
    blk = A.row_slice(r0, r1)
    t = time.perf_counter()
    ref = oracle.spgemm(blk.as_tuple(), A.as_tuple())
    return time.perf_counter() - t, ref.flops


def parallel_oracle(n):
    """The oracle on all host cores at once: the rows split into one block of
    equal flops per worker process, each running the unchanged oracle; the
    time is the slowest worker's (they run side by side)."""
    import multiprocessing as mp
    import synthetic as S
    workers = min(16, int(os.environ.get("OMP_NUM_THREADS", "16")), os.cpu_count() or 1)
    A, _ = S.config2(n=n) if n != 200000 else S.config2()
    deg = np.diff(A.row_ptr.astype(np.int64))
    u = np.bincount(np.repeat(np.arange(A.rows), deg), weights=deg[A.col_idx],
                    minlength=A.rows).astype(np.int64)
    cu = np.cumsum(u)
    cuts = [0] + [int(np.searchsorted(cu, cu[-1] * k / workers)) for k in range(1, workers)] \
        + [A.rows]
    blocks = [(n, cuts[k], cuts[k + 1]) for k in range(workers) if cuts[k + 1] > cuts[k]]
    with mp.get_context("spawn").Pool(len(blocks)) as pool:
        res = pool.map(_oracle_block, blocks)
    t = max(r[0] for r in res)
    fl = sum(r[1] for r in res)
    return {"value": round(fl / t / 1e9, 5), "unit": "GFLOP/s", "cores": len(blocks),
            "kind": "oracle", "sample": "the full workload once, rows split into %d blocks of "
            "equal flops, one process each (slowest block %.2f s)" % (len(blocks), t)}


def diff_forward():
    """The differentiable workload's forward product alone (A 500000^2 power
    law x B 500000x4096, binary32, default options)."""
    import torch

    import synthetic as S
    from paper_1504_05022_amd import lib as L

    L.load()
    torch.cuda.set_device(0)
    A, B = S.config5()
    dA, dB = L.CsrMatrix.from_host(A), L.CsrMatrix.from_host(B)
    del A, B
    for _ in range(2):
        C = L.spgemm(dA, dB)
        del C
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        C, info = L.spgemm(dA, dB, return_info=True)
        del C
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 3
    print(json.dumps({"workload": "A 500000^2 power law (2.2, mean 20) x B 500000x4096 (32/row), "
                                  "FP32", "forward_ms": round(ms, 3), "flops": int(info.flops)}),
          flush=True)


def diff_backward():
    """The differentiable workload's backward alone: dA and dB of a random
    dC on the forward's pattern (A 500000^2 power law x B 500000x4096,
    binary32)."""
    import torch

    import synthetic as S
    from paper_1504_05022_amd import lib as L

    L.load()
    torch.cuda.set_device(0)
    A, B = S.config5()
    dA, dB = L.CsrMatrix.from_host(A), L.CsrMatrix.from_host(B)
    del A, B
    plan = L.Plan(dA, dB)
    C = plan.compute()
    g = torch.Generator(device="cuda").manual_seed(5)
    dc = torch.randn(C.nnz, generator=g, dtype=torch.float32, device="cuda")
    plan.backward(C, dc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        plan.backward(C, dc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 3
    fl = int(plan.info.flops)
    plan.close()
    print(json.dumps({"workload": "A 500000^2 power law (2.2, mean 20) x B 500000x4096 (32/row), "
                                  "FP32", "backward_ms": round(ms, 3),
                      "backward_gflops": round(2 * fl / (ms * 1e-3) / 1e9, 2)}), flush=True)


def batch_one_shot():
    """spgemm_batch_multiply over the 512 banded problems alone."""
    import torch

    import synthetic as S
    from paper_1504_05022_amd import lib as L

    L.load()
    torch.cuda.set_device(0)
    probs = S.config4()
    dev = [(L.CsrMatrix.from_host(a), L.CsrMatrix.from_host(b)) for a, b in probs]
    del probs
    outs, st = L.batch_multiply(dev, return_stats=True)
    del outs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        outs = L.batch_multiply(dev)
        del outs
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 3
    print(json.dumps({"workload": "512 banded problems, n log-uniform in [1024, 65536], 4-32 "
                                  "nnz/row in a 5% band, FP64 even / FP32 odd",
                      "one_shot_ms": round(ms, 3), "items": st.items, "flops": st.flops}),
          flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.diff_forward:
        diff_forward()
        return
    if args.batch_one_shot:
        batch_one_shot()
        return
    if args.diff_backward:
        diff_backward()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import synthetic as S
    from paper_1504_05022_amd import lib as L

    L.load()
    torch.cuda.set_device(0)
    A, _ = S.config2(n=args.n) if args.n != 200000 else S.config2()
    dA = L.CsrMatrix.from_host(A)
    torch.cuda.synchronize()
    s = 8

    # inside the timed steps only the long-row kernels (the candidates for
    # the dominant kernel) carry event timers (each timed stage adds two
    # event records to the stream)
    wave_mask = ((1 << L.STAGES.index("long_wave")) | (1 << L.STAGES.index("long_sym"))
                 | (1 << L.STAGES.index("combine_wave")))

    def step(mask=wave_mask):
        return L.spgemm(dA, dA, return_info=True, timing=1, timing_mask=mask)

    for _ in range(args.warmup):
        C, info = step()
    torch.cuda.synchronize()
    crp = C.row_ptr.cpu().numpy()
    cci = C.col_idx.cpu().numpy()
    nnz_c = int(C.nnz)
    del C

    stage_ms = np.zeros(L.NSTAGES)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C, info = step()
        stage_ms += np.array(list(info.stage_ms))
        del C
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    stage_ms /= args.steps
    # the same steps with the L2 and Infinity Cache flushed before each (a
    # 512 MB write, outside the measured time): no input is cache-resident
    # when a step starts
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    flushed = 0.0
    for _ in range(args.steps):
        flush.fill_(1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        C, _ = step()
        torch.cuda.synchronize()
        flushed += time.perf_counter() - t
        del C
    del flush
    ms_flushed = flushed * 1e3 / args.steps
    # per-stage breakdown from untimed steps with every stage timer on
    full_ms = np.zeros(L.NSTAGES)
    for _ in range(2):
        C2, info2 = step(0)
        full_ms += np.array(list(info2.stage_ms))
        del C2
    torch.cuda.synchronize()
    full_ms /= 2
    flops = int(info.flops)
    gflops = flops / (ms * 1e-3) / 1e9
    bytes_comp = compulsory_bytes(A, nnz_c, s)
    stages = dict(zip(L.STAGES, [round(float(x), 4) for x in stage_ms]))
    breakdown = dict(zip(L.STAGES, [round(float(x), 4) for x in full_ms]))

    # dominant kernel: the longest of the long-row kernels of the method the
    # library takes for this product
    method = "window" if A.cols <= dense_cols(s) else "merge"
    if method == "window":
        part_b, sym_b, num_b = window_kernel_bytes(A, A, crp, s)
        cand = [("k_wpart (partition of long-row segments into column pieces)", part_b,
                 stages["long_wave"]),
                ("k_wsym (symbolic pass of the long-row windows)", sym_b, stages["long_sym"]),
                ("k_wnum (numeric pass of the long-row windows, into C)", num_b,
                 stages["combine_wave"])]
    else:
        seg_b, rng_b = merge_kernel_bytes(A, A, crp, cci, s)
        cand = [("k_long_w (512-product segments of split rows, one wavefront each)", seg_b,
                 stages["long_wave"]),
                ("k_combine_w (column ranges of split rows, 512-entry wavefront pass)", rng_b,
                 stages["combine_wave"])]
    name, kbytes, kms = max(cand, key=lambda c: c[2])
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0

    out = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "m": A.rows, "nnz_A": A.nnz, "flops": flops,
                   "nnz_C": nnz_c, "max_u": int(info.max_u),
                   "long_rows": int(info.bin_count[37])},
        "hbm_compulsory": {"bytes": bytes_comp,
                           "achieved_GBps": round(bytes_comp / (ms * 1e-3) / 1e9, 2),
                           "frac": round(bytes_comp / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                           "target_frac": 0.40,
                           "flushed_ms_per_step": round(ms_flushed, 4),
                           "flushed_frac": round(bytes_comp / (ms_flushed * 1e-3) / 1e9
                                                 / HBM_PEAK_GBS, 5)},
        "long_row_kernels_ms": {c[0].split()[0]: c[2] for c in cand},
        "stage_ms": breakdown,
        "roofline": {"kernel": name, "bound": "hbm", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(name, method),
                     "algorithmic_bytes": int(kbytes), "kernel_ms": round(kms, 4)},
    }
    out["memory"] = memory_accounting(row_upper_bounds(A, A), crp, info, s)
    if not args.no_cpu:
        import oracle
        # the oracle as it stands, single thread, on the whole workload,
        # repeated until about 10 s of CPU time have been measured
        runs, dt, flops = 0, 0.0, 0
        while runs == 0 or (dt < 10.0 and runs < 10):
            t = time.perf_counter()
            ref = oracle.spgemm(A.as_tuple(), A.as_tuple())
            dt += time.perf_counter() - t
            flops += ref.flops
            runs += 1
            del ref
        out["cpu_baseline"] = {"value": round(flops / dt / 1e9, 5), "unit": "GFLOP/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "the full workload, %d runs (%.1f s)" % (runs, dt),
                               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                               "host_cores": parallel_oracle(args.n)}
    if not args.no_ext:
        tiny = tiny_rows_ablation(torch, L, dA, int(sum(info.bin_count[2:33])))
        del dA
        torch.cuda.empty_cache()
        out["extensions"] = extensions(args, torch, S, L)
        out["extensions"]["tiny_rows"] = tiny
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
