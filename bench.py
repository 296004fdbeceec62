"""Benchmark: SpGEMM GFLOP/s on the irregular power-law squaring workload.

One step = the whole hot path on one MI355X: analyze (upper bounds, scan,
binning, C~ sizing) + compute (per-bin insert kernels, long-row merges,
row pointers, allocation of C, copy into C), inputs already resident in HBM.
Prints one JSON line (see the "metric" field); the roofline entry is for the
dominant kernel, timed with HIP events on the library's stream during the
timed steps.
"""
import argparse
import json
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--n", type=int, default=200000, help="rows (default: the full workload)")
    return ap.parse_args()


def compulsory_bytes(A, nnz_c, s=8):
    """sum over distinct inputs [4(rows+1) + nnz(4+s)] + 4(m+1) + nnz(C)(4+s)."""
    return 4 * (A.rows + 1) + A.nnz * (4 + s) + 4 * (A.rows + 1) + nnz_c * (4 + s)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import synthetic as S
    from paper_1504_05022_amd import CsrMatrix, Plan, lib

    lib.load()
    torch.cuda.set_device(0)
    A, _ = S.config2(n=args.n) if args.n != 200000 else S.config2()
    dA = CsrMatrix.from_host(A)
    torch.cuda.synchronize()
    s = 8

    # host-side per-row counts for the per-kernel byte model
    arp = A.row_ptr.astype(np.int64)
    deg = np.diff(arp)
    rowlen = deg  # A*A: row lengths of B are A's
    u = np.zeros(A.rows, np.int64)
    np.add.at(u, np.repeat(np.arange(A.rows), deg), rowlen[A.col_idx])

    def step(timing):
        plan = Plan(dA, dA, timing=timing)
        C = plan.compute()
        info = plan.info
        plan.close()
        return C, info

    for _ in range(args.warmup):
        C, info = step(1)
    torch.cuda.synchronize()
    cnnz = np.diff(C.row_ptr.cpu().numpy().astype(np.int64))
    nnz_c = int(C.nnz)
    del C

    stage_ms = np.zeros(8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C, info = step(1)
        stage_ms += np.array(list(info.stage_ms))
        del C
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    stage_ms /= args.steps
    flops = int(info.flops)
    gflops = flops / (ms * 1e-3) / 1e9
    bytes_comp = compulsory_bytes(A, nnz_c, s)

    # dominant kernel: the long-row merge kernel (one launch per step)
    long_rows = u > 512
    long_bytes = (int(np.sum(8 + deg[long_rows] * (4 + s)))          # its rows of A
                  + 4 * (A.rows + 1) + A.nnz * (4 + s)                  # B, read once
                  + int(np.sum(cnnz[long_rows])) * (4 + s))             # its output rows
    long_ms = float(stage_ms[4])
    stages = dict(zip(lib.STAGES, [round(float(x), 4) for x in stage_ms]))
    achieved = long_bytes / (long_ms * 1e-3) / 1e9 if long_ms > 0 else 0.0

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
                   "long_rows": int(long_rows.sum())},
        "hbm_compulsory": {"bytes": bytes_comp,
                           "achieved_GBps": round(bytes_comp / (ms * 1e-3) / 1e9, 2),
                           "frac": round(bytes_comp / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)},
        "stage_ms": stages,
        "roofline": {"kernel": "k_long (long-row merge method)", "bound": "hbm",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "algorithmic_bytes": long_bytes, "kernel_ms": round(long_ms, 4)},
    }
    if not args.no_cpu:
        import oracle
        # the oracle as it stands, single thread, on the whole workload
        t = time.perf_counter()
        ref = oracle.spgemm(A.as_tuple(), A.as_tuple())
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(ref.flops / dt / 1e9, 5), "unit": "GFLOP/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "the full workload once (%.1f s)" % dt}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
