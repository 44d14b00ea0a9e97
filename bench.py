#!/usr/bin/env python3
"""Benchmark: full lower-triangular CSR construction of K (integrate + assemble) on one MI355X.

Workload (default): 150^3 cubes split into 6 Kuhn tet4 each (20,250,000 elements,
3,442,951 nodes), interior jitter 0.2h, random node and element numbering,
c log-uniform in [1e-3, 1e3], FP32 integration with FP64 Jacobian fallback.
A step is one complete construction from device-resident E, C, c to device-resident
row_ptr / col_idx / vals.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1|c4|c5|c6|t2|fan] [--prec ...]
                    [--groups G] [--dof D] [--op mass] [--adjoint]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "elements/s for full lower-tri CSR K build (integrate+assemble), % HBM peak"
HBM_PEAK_GBS = 8000.0
# the paper's own figure for exactly this metric and workload (Table 2, 27M bricks: 115 s for
# the whole build, GPU integration + CPU assembly, on a Quadro 4000 + Xeon E5-2620)
PAPER_TABLE2_27M_ELEMENTS_PER_S = 27_000_000 / 115.0

WORKLOADS = {
    "c1": (1, "hex8 unit cube 10^3 (1,000 elements, 1,331 nodes), jitter 0.2h, c=1", "fp64"),
    "c2": (2, "hex8 box 100^3 (1,000,000 elements, 1,030,301 nodes), jitter 0.25h, random node numbering, "
              "c log-U[1e-2,1e2]", "fp32fb64"),
    "c3": (3, "tet4 Kuhn 6x150^3 (20,250,000 elements, 3,442,951 nodes), jitter 0.2h, random node and element "
              "numbering, c log-U[1e-3,1e3], 1-point rule", "fp32fb64"),
    "c5": (5, "hex8 box 64^3 (262,144 elements), jitter 0.2h, c log-U[1e-1,1e1]", "fp64"),
    "c4": (4, "256 hex8 boxes, cells per axis U{8..64}, h=1/64, jitter 0.2h, c log-U[1e-2,1e2], one batched "
              "build", "fp32fb64"),
    "t2": (7, "hex8 unit cube 300^3 (27,000,000 elements, 27,270,901 nodes), undistorted, c=1, natural numbering: "
              "the largest mesh of the paper's Table 2", "fp64"),
    "c6": (6, "tet4 Kuhn 6x337^3 (229,636,518 elements, 38,614,472 nodes, 2,296,365,180 element pairs: more than "
              "one pass indexes), jitter 0.2h, c log-U[1e-3,1e3], grouped build", "fp32fb64"),
    # not one of the paper's workloads: the heavy-row path under one node of valence 10^6
    "fan": ("fan", "tet4 fan of 1,000,000 tets around one node numbered last (3,000,001 nodes; its row holds "
                   "4,000,000 pairs and 3,000,001 entries), c log-U[e^-2,e^2]", "fp32fb64"),
}


def algorithmic_bytes(elem: int, n_elem: int, n_node: int, nnz: int, prec: str) -> dict:
    """Compulsory HBM bytes of each stage and of the whole path (per launch).

    Per stage: its inputs read once and its outputs written once, in the formats the
    stages exchange: (16-bit row within its bucket, col, value) after pass 1, (packed key,
    value) after pass 2.
    For the path: E, c and C read once (coordinates once per node), the lower values
    written once and read once, CSR written once.
    """
    vb = 8 if prec == "fp64" else 4
    nen = elem
    te = nen * (nen + 1) // 2
    T = n_elem * te
    conn = 4 * nen * n_elem
    coef = 8 * n_elem
    coords = 24 * n_node
    b = {
        "count": conn,                                            # E in (histogram out is small)
        "integrate": conn + coef + coords + (6 + vb) * T,         # E, c, C in; (row16, col, value) out
        "histogram": 2 * T,                                       # rows in (histograms out are small)
        "partition": (6 + vb) * T + (4 + vb) * T,                 # (row16, col, value) in, (key, value) out
        "reduce": (4 + vb) * T + (4 + vb) * nnz + 4 * n_node,     # pairs in; unique entries, row counts out
        "compress": 2 * (4 + vb) * nnz + 8 * n_node,              # unique entries in, CSR out
    }
    # the path as a whole: E, c, C in once, lower values once out and in, CSR out
    b["path"] = conn + coef + coords + 2 * vb * T + (4 + vb) * nnz + 4 * (n_node + 1)
    return b


# stages that are exactly one kernel: the roofline is reported for the slowest of them
SINGLE_KERNEL_STAGES = {"integrate": "k_pass1", "partition": "k_scatter2", "reduce": "k_pass3"}
PROFILE_DIR = os.path.join(ROOT, "profiles")
SOURCE_DIR = os.path.join(ROOT, "paper_1501_04784_amd", "csrc")


def source_digest() -> str:
    """sha256 over the HIP sources, to tell whether stored counters still apply."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(SOURCE_DIR)):
        with open(os.path.join(SOURCE_DIR, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def pass1_kernel(elem: int, prec: str, op: str) -> str:
    """The pass-1 kernel a build from coordinates launches: tets in the persistent tet
    kernel; bricks in FP64 two tiles per workgroup, in FP32 a lane pair per element for the
    stiffness matrix, else one lane per element."""
    if elem == 4:
        return "k_pass1_tet"
    if prec == "fp64":
        return "k_pass1_two"
    return "k_pass1_pair" if op == "stiffness" else "k_pass1"


def stored_traffic(kernel: str, workload: str, prec: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was
    taken on the current sources (else None).  The summary holds lines
    `traffic_bytes: N` and `source_sha256: H`."""
    path = os.path.join(PROFILE_DIR, f"counters_{workload}_{prec}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.strip().startswith(("traffic_bytes", "source_sha256")):
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    sec = [l for l in open(path).read().split("\n## ") if l.split("\n", 1)[0].strip() == kernel]
    if not sec or fields.get("source_sha256") != source_digest():
        return None
    for line in sec[0].splitlines():
        if line.strip().startswith("traffic_bytes:"):
            return float(line.split(":", 1)[1])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32", "fp32fb64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="elements in the oracle's timed sample (0: as many as make 202.5M lower pairs, i.e. the "
                         "whole 20.25M-tet workload)")
    ap.add_argument("--copy-mib", type=int, default=2048, help="size of the device copy timed as a ceiling (0: skip)")
    ap.add_argument("--profile-steps", action="store_true", help="no stage events (for profiler runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--op", default="stiffness", choices=["stiffness", "mass"],
                    help="element integrand: stiffness matrix (default) or consistent mass matrix")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the adjoint (dL/dc, dL/dX of L = sum W K, seeded N(0,1) weights), FP64")
    ap.add_argument("--groups", type=int, default=0,
                    help="build in this many element groups (Eq. 10; workload c6 needs at least 2, default 2)")
    ap.add_argument("--host-stream", action="store_true",
                    help="grouped builds: also time the groups streamed from pinned host memory (upload of group "
                         "g+1 overlapping the pass of group g; PCIe-inclusive, reported beside the value)")
    ap.add_argument("--dof", type=int, default=1, choices=[1, 2, 3],
                    help="also time the assembly of k ⊗ I_dof element matrices (several DOFs per node)")
    ap.add_argument("--block", type=int, default=0, help="tuning: element tile / block size")
    ap.add_argument("--bucket-bits", type=int, default=0, help="tuning: log2 rows per first-level bucket")
    ap.add_argument("--sub-bits", type=int, default=0, help="tuning: log2 rows per sub-bucket")
    ap.add_argument("--seg-pairs", type=int, default=0, help="tuning: pairs per sub-bucket partition segment")
    ap.add_argument("--table-slots", type=int, default=0, help="tuning: pass-3 hash-table slots per sub-bucket")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch and t2 workloads: time only the built-in tuning (no tuning search / cache lookup)")
    ap.add_argument("--tune-cache", default=None, help="JSON cache of tuning choices (default: KBUILD_TUNE_CACHE "
                                                       "or ~/.cache/kbuild/tuning.json)")
    return ap.parse_args()


def time_builds(kb, torch, mesh_dev, m, prec, steps, warmup, stage_events=True, tuning=None, op="stiffness",
                groups=0):
    if groups > 1:
        import meshgen

        conn, coords, coef = mesh_dev
        cap = meshgen.box_nnz(m.elem, m.meta["nx"], m.meta["ny"], m.meta["nz"])
        b = kb.GroupedBuilder(m.elem, m.n_elem, m.n_node, -(-m.n_elem // groups), cap, prec=prec, tuning=tuning,
                              op=op)
        run = lambda ev=None: b.run(conn, coords, coef, stage_events=ev)  # noqa: E731
        result = lambda: b.result(check=True, allow_flags=0)  # noqa: E731
    elif isinstance(mesh_dev, kb.Batch):
        b = kb.BatchBuilder(mesh_dev, prec=prec, tuning=tuning)
        run = lambda ev=None: b.run(stage_events=ev)  # noqa: E731
        result = lambda: b.results(check=True)  # noqa: E731
    else:
        conn, coords, coef = mesh_dev
        b = kb.Builder(m.elem, m.n_elem, m.n_node, prec=prec, tuning=tuning, op=op)
        run = lambda ev=None: b.run(conn, coords, coef, stage_events=ev)  # noqa: E731
        result = lambda: b.result(check=True, allow_flags=0)  # noqa: E731
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        run()
    res = result()
    n_ev = kb.KB_N_STAGES + 1
    evs = [kb._lib.HipEvents(n_ev) for _ in range(steps)] if stage_events else None
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for s in range(steps):
        run(evs[s].handles if evs else None)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1) / steps
    stages = None
    if evs:
        stages = {}
        for i, name in enumerate(kb.STAGE_NAMES):
            stages[name] = sum(evs[s].elapsed_ms(i, i + 1) for s in range(steps)) / steps
        for e in evs:
            e.close()
    res = result()
    if isinstance(res, list):  # a batch: totals over its meshes
        res = BatchTotals(sum(r.nnz for r in res), res[0].n_fallback if res else 0)
    return ms, wall / steps * 1e3, stages, res


def time_adjoint(kb, torch, mesh_dev, m, steps, warmup):
    """Backward of L = sum W_ij K_ij (FP64 forward pattern, seeded N(0,1) weights)."""
    import meshgen

    conn, coords, coef = mesh_dev
    r = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64")
    rp, col = r.row_ptr.clone(), r.col_idx.clone()
    w = torch.from_numpy(meshgen.loss_weights(r.nnz)).to(conn.device)
    a = kb.AdjointBuilder(m.elem, m.n_elem, m.n_node, device=conn.device)
    for _ in range(warmup):
        a.run(conn, coords, coef, rp, col, w)
    a.result()  # data errors raise here, before timing
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        a.run(conn, coords, coef, rp, col, w)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    return {"ms_per_step": ms, "value": m.n_elem / (ms * 1e-3), "unit": "elements/s",
            "note": "reusable context: workspace and gradients allocated once, before the timed calls"}


def time_host_stream(kb, torch, mesh_dev, m, prec, groups, steps, warmup, device_ms):
    """Grouped build with connectivity and coefficients streamed from pinned host memory:
    its time, the time of the uploads alone and how much of the shorter of the two
    (uploads, device-resident build) the streaming hides."""
    import meshgen

    conn_h = torch.from_numpy(m.conn).pin_memory()
    coef_h = torch.from_numpy(m.coef).pin_memory()
    cap = meshgen.box_nnz(m.elem, m.meta["nx"], m.meta["ny"], m.meta["nz"])
    sb = kb.StreamedGroupedBuilder(m.elem, m.n_elem, m.n_node, -(-m.n_elem // groups), cap, prec=prec)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        sb.run(conn_h, mesh_dev[1], coef_h)
    sb.result(check=True)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        sb.run(conn_h, mesh_dev[1], coef_h)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    # the uploads alone (same copies, same staging buffers, one stream)
    b = sb.base
    t0.record(stream)
    for g in range(sb.n_groups):
        e0, e1 = g * b.group, min(b.n_elem, (g + 1) * b.group)
        sb.stage_conn[g % 2][: e1 - e0].copy_(conn_h[e0:e1], non_blocking=True)
        sb.stage_coef[g % 2][: e1 - e0].copy_(coef_h[e0:e1], non_blocking=True)
    t1.record(stream)
    torch.cuda.synchronize()
    up_ms = t0.elapsed_time(t1)
    host_bytes = m.conn.nbytes + m.coef.nbytes
    hidden = (up_ms + device_ms - ms) / min(up_ms, device_ms)
    del sb, conn_h, coef_h
    torch.cuda.empty_cache()
    return {"ms_per_step": ms, "elements_per_s_pcie_inclusive": m.n_elem / (ms * 1e-3), "upload_ms": up_ms,
            "upload_GBps": host_bytes / (up_ms * 1e-3) / 1e9, "device_resident_ms": device_ms,
            "overlap_hidden_frac": hidden, "groups": sb_groups(m.n_elem, groups),
            "note": "connectivity and coefficients in pinned host memory, two device staging buffers, uploads on a "
                    "second stream; coordinates device-resident"}


def sb_groups(n_elem, groups):
    return -(-n_elem // -(-n_elem // groups))


def kron_values(torch, k1, elem, dof):
    """Packed lower triangles of k ⊗ I_dof from packed scalar ones (input preparation)."""
    src = []
    for p in range(elem * dof):
        for q in range(p + 1):
            a, c = divmod(p, dof)
            b, c2 = divmod(q, dof)
            src.append(a * (a + 1) // 2 + b if c == c2 else -1)
    src = torch.tensor(src, device=k1.device)
    out = k1[:, src.clamp(min=0)]
    return torch.where(src[None, :] >= 0, out, torch.zeros_like(out)).contiguous()


def time_dof(kb, torch, mesh_dev, m, prec, dof, steps, warmup, cpu_sample):
    """Assembly only of element matrices with ``dof`` components per node (k_e ⊗ I from the
    mesh's own stiffness values), timed per stage like the main build."""
    import numpy as np

    import oracle

    conn, coords, coef = mesh_dev
    k1, _ = kb.integrate_lower(conn, coords, coef, m.elem, prec=prec)
    kd = kron_values(torch, k1, m.elem, dof)
    del k1
    b = kb.Builder(m.elem, m.n_elem, m.n_node, prec=prec, dof=dof)
    for _ in range(warmup):
        b.run(conn, None, None, klow=kd)
    res = b.result(check=True)
    n_ev = kb.KB_N_STAGES + 1
    evs = [kb._lib.HipEvents(n_ev) for _ in range(steps)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for s in range(steps):
        b.run(conn, None, None, klow=kd, stage_events=evs[s].handles)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    stages = {name: sum(e.elapsed_ms(i, i + 1) for e in evs) / steps for i, name in enumerate(kb.STAGE_NAMES)}
    for e in evs:
        e.close()
    nd = m.elem * dof
    T = m.n_elem * nd * (nd + 1) // 2
    out = {"dof": dof, "ms_per_step": ms, "value": m.n_elem / (ms * 1e-3), "unit": "elements/s",
           "pairs_per_s": T / (ms * 1e-3), "n_pairs": T, "nnz": res.nnz, "rows": dof * m.n_node, "stages_ms": stages,
           "note": "assembly only (values given), k_e ⊗ I_dof from the mesh's stiffness values"}
    if cpu_sample:
        n = max(1, min(m.n_elem, cpu_sample))
        kh = kd[:n].double().cpu().numpy()
        ch = np.ascontiguousarray(m.conn[:n])
        oracle.lib()
        t = time.perf_counter()
        oracle.assemble_lower_csr_dof(m.elem, dof, ch, m.n_node, kh)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": n / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {n:,} of the {m.n_elem:,} elements, single-threaded FP64 C "
                                         f"oracle assembly (sort + CSR), {dt:.1f} s"}
    del kd, b
    torch.cuda.empty_cache()
    return out


class BatchTotals:
    def __init__(self, nnz, n_fallback):
        self.nnz, self.n_fallback = nnz, n_fallback


def default_cpu_sample(elem: int) -> int:
    """Elements of the oracle's timed sample: as many as make 202.5M lower pairs (the whole
    20.25M-tet workload; 5.6M bricks), about 10-30 s of single-threaded oracle work."""
    return 202_500_000 // (elem * (elem + 1) // 2)


def cpu_baseline(m, sample):
    """The single-threaded FP64 oracle timed on the first ``sample`` elements, then the
    all-cores harness (same element routine, parallel loops and sort) on the same
    sample.  Returns (single-threaded record, all-cores record, oracle CSR of the sample
    or None when the sample is part of the workload)."""
    import numpy as np

    import meshgen
    import oracle

    if isinstance(m, list):  # a batch: whole meshes in order until the sample is reached
        oracle.lib()
        done, k, t = 0, 0, time.perf_counter()
        while k < len(m) and done < sample:
            oracle.build_mesh(m[k])
            done += m[k].n_elem
            k += 1
        dt = time.perf_counter() - t
        single = {"value": done / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
                  "sample": f"the first {k} of {len(m)} meshes ({done:,} elements), each built separately by the "
                            f"single-threaded FP64 C oracle, {dt:.1f} s"}
        th = oracle.par_threads()
        t = time.perf_counter()
        for x in m[:k]:
            oracle.par_build_mesh(x)
        dtp = time.perf_counter() - t
        par = {"value": done / dtp, "unit": "elements/s", "cores": th, "kind": "oracle, all-cores harness",
               "sample": f"the same {k} meshes, {dtp:.1f} s"}
        return single, par, None
    n = min(sample, m.n_elem)
    whole = n == m.n_elem
    sub = m if whole else meshgen.Mesh(m.elem, np.ascontiguousarray(m.conn[:n]), m.coords,
                                       np.ascontiguousarray(m.coef[:n]))
    oracle.lib()
    t = time.perf_counter()
    ref = oracle.build_mesh(sub)
    dt = time.perf_counter() - t
    what = (f"all {n:,} elements" if whole else f"first {n:,} of the {m.n_elem:,} elements (all {m.n_node:,} "
            f"nodes)")
    single = {"value": n / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
              "sample": f"{what}, single-threaded FP64 C oracle, integrate + sort + CSR, {dt:.1f} s"}
    th = oracle.par_threads()
    t = time.perf_counter()
    oracle.par_build_mesh(sub)
    dtp = time.perf_counter() - t
    par = {"value": n / dtp, "unit": "elements/s", "cores": th, "kind": "oracle, all-cores harness",
           "sample": f"{what}, the oracle's element routine on {th} OpenMP threads with a parallel merge sort "
                     f"(oracle/timing_par.c), {dtp:.1f} s"}
    return single, par, (ref if whole else None)


def scaled_errors(results: dict, ref) -> dict:
    """Diagonal-scaled error max |dK_ij| / sqrt(K_ii K_jj) of each benched run against the
    oracle's matrix; the pattern must match exactly (else the error is reported as inf)."""
    import numpy as np

    orp, ocol, oval, _ = ref
    n = len(orp) - 1
    last = orp[1:] - 1
    diag = np.where(orp[1:] > orp[:-1], oval[np.maximum(last, 0)], 0.0)
    rows = np.repeat(np.arange(n), np.diff(orp))
    scale = np.sqrt(np.abs(diag[rows] * diag[ocol]))
    scale = np.where(scale > 0, scale, 1.0)
    out = {}
    for prec, (rp, col, val) in results.items():
        if not (np.array_equal(rp, orp) and np.array_equal(col, ocol)):
            out[prec] = float("inf")
            continue
        out[prec] = float(np.max(np.abs(val.astype(np.float64) - oval) / scale)) if len(oval) else 0.0
    return out


def copy_ceiling(torch, mib: int) -> dict:
    """Rate of a plain device-to-device copy (read + write bytes per second), the
    practical ceiling of a streaming kernel on this device."""
    src = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * (mib << 20), "ms": ms, "GBps": 2 * (mib << 20) / (ms * 1e-3) / 1e9}


class MeshTotals:
    def __init__(self, elem, n_elem, n_node):
        self.elem, self.n_elem, self.n_node = elem, n_elem, n_node


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import meshgen
    import paper_1501_04784_amd as kb

    if args.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cid, desc, default_prec = WORKLOADS[args.workload]
    prec = args.prec or default_prec
    groups = args.groups if args.groups else (2 if cid == 6 else 0)
    if groups > 1 and cid == 4:
        print("grouped builds apply to single meshes", file=sys.stderr)
        sys.exit(2)
    print(f"[bench] generating workload {args.workload}: {desc}", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    if cid == 4:
        meshes = meshgen.config4_batch()
        mesh_dev = kb.pack_batch([(x.conn, x.coords, x.coef) for x in meshes], 8, dev)
        m = MeshTotals(8, sum(x.n_elem for x in meshes), sum(x.n_node for x in meshes))
    else:
        m = meshgen.fan_mesh(1_000_000, True, seed=3) if cid == "fan" else meshgen.config_mesh(cid)
        mesh_dev = (torch.from_numpy(m.conn).to(dev), torch.from_numpy(m.coords).to(dev),
                    torch.from_numpy(m.coef).to(dev))
    torch.cuda.synchronize()
    print(f"[bench] {m.n_elem} elements, {m.n_node} nodes on device; timing {prec}", file=sys.stderr, flush=True)

    tuning = kb.Tuning(block=args.block, bucket_bits=args.bucket_bits, sub_bits=args.sub_bits,
                       seg_pairs=args.seg_pairs, table_slots=args.table_slots)
    tune = None
    if cid in (4, 7) and not args.no_tune and tuning == kb.Tuning() and groups <= 1:
        # the batch and the naturally numbered 27M bricks take the tuning search's choice
        # (cached per architecture, element, precision and size class); the built-in
        # choice is timed beside it below
        t0 = time.perf_counter()
        if cid == 4:
            tuning, entry = kb.tune_batch(mesh_dev, prec, cache_path=args.tune_cache)
        else:
            tuning, entry = kb.tune_build(*mesh_dev, m.elem, prec, op=args.op, cache_path=args.tune_cache)
        tune = {"tuning": entry["tuning"], "source": entry["source"], "key": entry["key"],
                "search_s": time.perf_counter() - t0, "candidates_timed": entry.get("candidates_timed")}
        print(f"[bench] tuning ({entry['source']}): {tuning}", file=sys.stderr, flush=True)
    ms, wall_ms, stages, res = time_builds(kb, torch, mesh_dev, m, prec, args.steps, args.warmup,
                                           stage_events=not args.profile_steps, tuning=tuning, op=args.op,
                                           groups=groups)
    nnz = res.nnz
    print(f"[bench] {prec}: {ms:.3f} ms/step, nnz {nnz}, fallback elements {res.n_fallback}", file=sys.stderr,
          flush=True)
    host = {}  # the benched runs' CSR on the host, for the error against the oracle
    if isinstance(res, kb.LowerCSR):
        host[prec] = (res.row_ptr.cpu().numpy(), res.col_idx.cpu().numpy(), res.vals.cpu().numpy())
    n_fallback = res.n_fallback
    del res
    value = m.n_elem / (ms * 1e-3)
    ab = algorithmic_bytes(m.elem, m.n_elem, m.n_node, nnz, prec)
    out = {
        "metric": METRIC, "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": value / PAPER_TABLE2_27M_ELEMENTS_PER_S if args.workload == "t2" else None,
        "dtype": "f64" if prec == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": desc if args.op == "stiffness" else desc + ", consistent mass matrix",
                   "n_elem": m.n_elem, "n_node": m.n_node, "nnz": nnz, "precision": prec,
                   "fp64_fallback_elements": n_fallback, "parallelism": "single GPU",
                   "tuning": {"block": tuning.block, "bucket_bits": tuning.bucket_bits, "sub_bits": tuning.sub_bits,
                              "seg_pairs": tuning.seg_pairs, "table_slots": tuning.table_slots},
                   "groups": groups if groups > 1 else 1},
        "path_hbm_frac": ab["path"] / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
    }
    if stages and groups > 1:
        # the stage events time the last group's pass only; its pairs include the carried sums
        out["roofline"] = None
        out["stages_ms_last_group"] = stages
    elif stages:
        dom = max(SINGLE_KERNEL_STAGES, key=lambda k: stages[k])
        kernel = SINGLE_KERNEL_STAGES[dom]
        if dom == "integrate":
            kernel = pass1_kernel(m.elem, prec, args.op)
        elif dom == "reduce" and args.workload == "fan":
            # its heavy row adds the heavy-path kernels to the stage
            kernel = "k_pass3 + heavy path (k_heavy_*, k_pass3_heavy_ranges, k_pass3_heavy_finish)"
        achieved = ab[dom] / (stages[dom] * 1e-3) / 1e9
        traffic = stored_traffic(kernel, args.workload, prec)
        out["roofline"] = {"bound": "hbm", "kernel": kernel, "stage": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel_ms": stages[dom], "algorithmic_bytes": ab[dom],
                           # measured bytes per launch over this run's kernel time: how busy the
                           # memory system is, wasted bytes (partly used lines) included
                           "traffic_frac": (traffic / (stages[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None}
        out["stages_ms"] = stages
        # every stage's algorithmic bytes over its time, against the HBM peak
        out["stage_hbm_frac"] = {k: ab[k] / (stages[k] * 1e-3) / (HBM_PEAK_GBS * 1e9)
                                 for k in ("count", "integrate", "histogram", "partition", "reduce", "compress")
                                 if stages.get(k, 0) > 0}
    if tune is not None:
        # the built-in tuning on the same batch, for comparison with the tuned value
        msd, _, _, _ = time_builds(kb, torch, mesh_dev, m, prec, args.steps, args.warmup, stage_events=False)
        tune["default_ms_per_step"] = msd
        tune["default_value"] = m.n_elem / (msd * 1e-3)
        tune["speedup_vs_default"] = msd / ms
        out["autotune"] = tune
        print(f"[bench] built-in tuning: {msd:.3f} ms/step", file=sys.stderr, flush=True)
    if args.copy_mib:
        cc = copy_ceiling(torch, args.copy_mib)
        out["copy_ceiling"] = {"GBps": cc["GBps"], "bytes": cc["bytes"], "ms": cc["ms"],
                               "path_frac": ab["path"] / (ms * 1e-3) / (cc["GBps"] * 1e9)}
        if out.get("roofline"):
            out["copy_ceiling"]["dominant_kernel_frac"] = out["roofline"]["achieved"] / cc["GBps"]
        print(f"[bench] device copy {cc['GBps']:.0f} GB/s", file=sys.stderr, flush=True)
    if not args.no_fp64 and prec != "fp64":
        ms64, _, st64, r64 = time_builds(kb, torch, mesh_dev, m, "fp64", max(3, args.steps // 2), 2,
                                         stage_events=False, tuning=kb.Tuning(bucket_bits=args.bucket_bits,
                                                                              sub_bits=args.sub_bits), op=args.op,
                                         groups=groups)
        out["fp64"] = {"ms_per_step": ms64, "value": m.n_elem / (ms64 * 1e-3)}
        if isinstance(r64, kb.LowerCSR):
            host["fp64"] = (r64.row_ptr.cpu().numpy(), r64.col_idx.cpu().numpy(), r64.vals.cpu().numpy())
        del r64
        out["speedup_vs_fp64"] = ms64 / ms
        print(f"[bench] fp64: {ms64:.3f} ms/step", file=sys.stderr, flush=True)
    if args.host_stream and groups > 1:
        out["host_stream"] = time_host_stream(kb, torch, mesh_dev, m, prec, groups, max(2, args.steps // 4), 1, ms)
        print(f"[bench] host-streamed groups: {out['host_stream']['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
    if args.adjoint and cid != 4:
        out["adjoint"] = time_adjoint(kb, torch, mesh_dev, m, args.steps, args.warmup)
        print(f"[bench] adjoint: {out['adjoint']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if args.dof > 1 and cid != 4:
        out["dof_assembly"] = time_dof(kb, torch, mesh_dev, m, prec, args.dof, args.steps, args.warmup,
                                       0 if args.no_cpu else max(1, 1_000_000 // (args.dof * args.dof)))
        print(f"[bench] dof {args.dof} assembly: {out['dof_assembly']['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
    if not args.no_cpu:
        sample = args.cpu_sample or default_cpu_sample(m.elem)
        print(f"[bench] timing the CPU oracle on {min(sample, m.n_elem):,} elements", file=sys.stderr, flush=True)
        single, par, ref = cpu_baseline(meshes if cid == 4 else m, sample)
        out["cpu_baseline"] = single
        out["cpu_baseline_all_cores"] = par
        if ref is not None and host and args.op == "stiffness":
            err = scaled_errors(host, ref)
            out["scaled_error"] = {"vs": "FP64 oracle, every entry", "metric": "max |dK_ij| / sqrt(K_ii K_jj)",
                                   **err, "tolerance": {k: (1e-12 if k == "fp64" else 5e-6) for k in err}}
            print(f"[bench] scaled error against the oracle: {err}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
