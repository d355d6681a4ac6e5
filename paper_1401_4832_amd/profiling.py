"""Profiling helpers for the benchmark's roofline numbers.

python -m paper_1401_4832_amd.profiling drive [workload] [path]
    one reweight + one all-sites objective/gradient evaluation on the workload
    (evaluation path 2 unless given), then a 1 GiB device-to-device copy (the
    calibration kernel for the HBM byte counters); the program rocprofv3 runs
    for kernel traces and counters.
python -m paper_1401_4832_amd.profiling stats <kernel_stats.csv> <out.md> <command...>
    short markdown summary of a rocprofv3 --stats kernel table.
python -m paper_1401_4832_amd.profiling readbw
    reference stream rates of the device: a 2 GiB float32 tensor summed
    (read only), copied (read + write) and filled (write only), best of 5.
python -m paper_1401_4832_amd.profiling traffic <fetch.csv> <write.csv> <workload> <out_prefix>
    HBM bytes per launch of the forward and backward kernels from FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch), each scaled by what the same counter
    reads for the 1 GiB copy; writes <out_prefix>_<kernel>_<workload>.json.
python -m paper_1401_4832_amd.profiling onchip <l2.csv> <lds.csv> <workload> <out_prefix>
    L2 bytes per launch (TCC_READ_SECTORS_sum + TCC_WRITE_SECTORS_sum, scaled
    by what they read for the 1 GiB copy) and the LDS busy percentage
    (LdsUtil) of each kernel; writes <out_prefix>_<kernel>_<workload>.txt.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30
KERNELS = {"forward": "fwd_kernel", "backward": "bwd_kernel", "forward_mfma": "fwd_mfma_kernel",
           "backward_mfma": "bwd_mfma_kernel", "backward_g3": "bwd_g3_kernel", "backward_i8": "bwd_i8_kernel", "forward_i8": "fwd_i8_kernel",
           "jmax": "jmax_kernel", "jquant": "jquant_kernel", "lbfgs": "lbfgs_kernel",
           "reweight": "identity_kernel"}


# the source files each profiled kernel is compiled from
KERNEL_SOURCES = {"forward": ("k_gather.hip", "plm_internal.h"), "backward": ("k_gather.hip", "plm_internal.h"),
                  "forward_mfma": ("k_mfma.hip", "plm_internal.h"), "backward_mfma": ("k_mfma.hip", "plm_internal.h"),
                  "backward_g3": ("k_mfma.hip", "plm_internal.h"), "backward_i8": ("k_mfma.hip", "plm_internal.h"),
                  "forward_i8": ("k_fwd8.hip", "plm_internal.h"), "jmax": ("k_fwd8.hip", "plm_internal.h"),
                  "jquant": ("k_fwd8.hip", "plm_internal.h"),
                  "lbfgs": ("k_lbfgs.hip", "plm_internal.h"), "lbfgs_dir": ("k_lbfgs.hip", "plm_internal.h"),
                  "reweight": ("k_reweight.hip", "plm_internal.h")}


def source_hash(kernel: str | None = None) -> str:
    """Hash of the kernel's source files (of every library source without a kernel)."""
    csrc = os.path.join(ROOT, "paper_1401_4832_amd", "csrc")
    files = ([os.path.join(csrc, f) for f in KERNEL_SOURCES[kernel]] if kernel
             else sorted(glob.glob(os.path.join(csrc, "*"))))
    h = hashlib.sha256()
    for p in files:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def drive(workload: str = "potts_n500_b50000", path: str = "2"):
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import paper_1401_4832_amd as plm
    import synth
    s = synth.workload(workload)
    dev = torch.device("cuda:0")
    msa = torch.from_numpy(s.msa).to(dev)
    m, w, beff = plm.reweight(msa, theta=0.8)
    N, q = s.N, 21
    rng = np.random.default_rng(0)
    h = torch.from_numpy((0.1 * rng.standard_normal((N, q))).astype(np.float32)).to(dev)
    J = torch.from_numpy((0.1 * rng.standard_normal((N, N, q, q))).astype(np.float32)).to(dev)
    f, gh, gJ = plm.objgrad(msa, w, beff, h, J, path=int(path))
    plm.sync(dev)
    del gJ, J
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print("drive done", workload, float(f.sum()), flush=True)


def readbw():
    import json
    import torch
    dev = torch.device("cuda:0")
    n = (2 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn, nbytes in (("sum_read", lambda: a.sum(), 4 * n), ("copy_read_write", lambda: b.copy_(a), 8 * n),
                             ("fill_write", lambda: b.fill_(2.0), 4 * n)):
        best = 1e9
        for _ in range(5):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[name] = {"ms": best, "TB_per_s": nbytes / (best * 1e-3) / 1e12}
    print(json.dumps(out), flush=True)


def _rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def stats(csv_path: str, out_md: str, command: str):
    rows = _rows(csv_path)
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | total ms | average ms | % |", "|---|---|---|---|---|"]
    for r in rows[:24]:
        name = r.get("Name") or r.get("KERNEL_NAME") or r.get("name")
        calls = int(float(r.get("Calls") or r.get("calls")))
        tot = float(r.get("TotalDurationNs") or r.get("total_duration")) / 1e6
        avg = float(r.get("AverageNs") or r.get("average")) / 1e6
        pct = float(r.get("Percentage") or r.get("percentage"))
        lines.append(f"| `{name[:70]}` | {calls} | {tot:.3f} | {avg:.3f} | {pct:.1f} |")
    lines += ["", f"Kernel sources hash: `{source_hash()}`", ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def _per_kernel(rows, counter):
    out = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_csv: str, write_csv: str, workload: str, out_prefix: str, path: str = "6"):
    fr, wr = _rows(fetch_csv), _rows(write_csv)
    fk, wk = _per_kernel(fr, "FETCH_SIZE"), _per_kernel(wr, "WRITE_SIZE")

    def copy_value(d):
        vals = [v for k, vs in d.items() if "copy" in k.lower() or "elementwise" in k.lower()
                for v in vs if v > 0]
        return max(vals) if vals else None

    cf, cw = copy_value(fk), copy_value(wk)
    if not cf or not cw:
        raise SystemExit("copy calibration kernel not found in the counter files")
    sf, sw = COPY_BYTES / cf, COPY_BYTES / cw  # bytes per counter unit
    for kname, sym in KERNELS.items():
        h = source_hash(kname)
        f = [v for k, vs in fk.items() if sym in k for v in vs]
        w = [v for k, vs in wk.items() if sym in k for v in vs]
        if not f or not w:
            continue
        d = {"kernel": kname, "workload": workload, "source_hash": h,
             "fetch_kib_per_launch": sum(f) / len(f), "write_kib_per_launch": sum(w) / len(w),
             "copy_fetch_kib": cf, "copy_write_kib": cw,
             "bytes_per_launch": sum(f) / len(f) * sf + sum(w) / len(w) * sw,
             "commands": [
                 f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {os.path.dirname(fetch_csv)} -o run -- "
                 f"python3 -u -m paper_1401_4832_amd.profiling drive {workload} {path}",
                 f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {os.path.dirname(write_csv)} -o run -- "
                 f"python3 -u -m paper_1401_4832_amd.profiling drive {workload} {path}",
                 f"python -m paper_1401_4832_amd.profiling traffic {fetch_csv} {write_csv} {workload} {out_prefix}"
                 + ("" if path == "6" else f" {path}")],
             "note": f"one all-sites evaluation on evaluation path {path}; FETCH_SIZE scaled by {sf / 1024:.1f} "
                     f"and WRITE_SIZE by {sw / 1024:.1f} (the {COPY_BYTES >> 30} GiB copy calibration of the "
                     "same run)"}
        out = f"{out_prefix}_{kname}_{workload}.txt"
        with open(out, "w") as fh:
            json.dump(d, fh, indent=1)
        print(out, json.dumps(d))


def onchip(l2_csv: str, lds_csv: str, workload: str, out_prefix: str, path: str = "6"):
    """L2 bytes (TCC_READ_SECTORS_sum + TCC_WRITE_SECTORS_sum, 32-byte sectors,
    scaled by what they read for the calibration copy) and the LDS busy
    percentage (LdsUtil: SQ_LDS_IDX_ACTIVE over GRBM_GUI_ACTIVE x CUs) per
    launch of each kernel of one evaluation."""
    lr, dr = _rows(l2_csv), _rows(lds_csv)
    rk, wk = _per_kernel(lr, "TCC_READ_SECTORS_sum"), _per_kernel(lr, "TCC_WRITE_SECTORS_sum")
    uk = _per_kernel(dr, "LdsUtil")

    def copy_value(d):
        vals = [v for k, vs in d.items() if "copy" in k.lower() or "elementwise" in k.lower()
                for v in vs if v > 0]
        return max(vals) if vals else None

    cr, cw = copy_value(rk), copy_value(wk)
    if not cr or not cw:
        raise SystemExit("copy calibration kernel not found in the counter files")
    sr, sw = COPY_BYTES / cr, COPY_BYTES / cw  # bytes per sector as counted
    for kname, sym in KERNELS.items():
        rd = [v for k, vs in rk.items() if sym in k for v in vs]
        wr = [v for k, vs in wk.items() if sym in k for v in vs]
        ut = [v for k, vs in uk.items() if sym in k for v in vs]
        if not rd or not wr or not ut:
            continue
        d = {"kernel": kname, "workload": workload, "source_hash": source_hash(kname),
             "l2_read_bytes_per_launch": sum(rd) / len(rd) * sr,
             "l2_write_bytes_per_launch": sum(wr) / len(wr) * sw,
             "l2_bytes_per_launch": sum(rd) / len(rd) * sr + sum(wr) / len(wr) * sw,
             "lds_util_pct": sum(ut) / len(ut),
             "copy_read_sectors": cr, "copy_write_sectors": cw,
             "commands": [
                 f"rocprofv3 --pmc TCC_READ_SECTORS_sum TCC_WRITE_SECTORS_sum --output-format csv -d "
                 f"{os.path.dirname(l2_csv)} -o run -- python3 -u -m paper_1401_4832_amd.profiling drive "
                 f"{workload} {path}",
                 f"rocprofv3 --pmc LdsUtil --output-format csv -d {os.path.dirname(lds_csv)} -o run -- "
                 f"python3 -u -m paper_1401_4832_amd.profiling drive {workload} {path}",
                 f"python -m paper_1401_4832_amd.profiling onchip {l2_csv} {lds_csv} {workload} {out_prefix}"
                 + ("" if path == "6" else f" {path}")],
             "note": f"one all-sites evaluation on evaluation path {path}; sectors scaled by {sr:.1f} (read) and "
                     f"{sw:.1f} (write) bytes, from the {COPY_BYTES >> 30} GiB copy of the same run; LdsUtil is "
                     "the share of CU cycles the LDS was busy during the launch"}
        out = f"{out_prefix}_{kname}_{workload}.txt"
        with open(out, "w") as fh:
            json.dump(d, fh, indent=1)
        print(out, json.dumps(d))


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "readbw":
        readbw()
    elif cmd == "drive":
        drive(*(sys.argv[2:4]))
    elif cmd == "stats":
        stats(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif cmd == "traffic":
        traffic(*sys.argv[2:7])
    elif cmd == "onchip":
        onchip(*sys.argv[2:7])
    else:
        raise SystemExit(__doc__)
