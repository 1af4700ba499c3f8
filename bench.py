#!/usr/bin/env python3
"""Benchmark of the nAIR hot path on one MI355X.

One step = the whole hot path on one synthetic upwind-DG transport system
already resident in HBM: hierarchy setup, solve A x = b to 1e-10 relative
residual, and the transposed solve A^T y = g to 1e-10.  `value` is DOFs/s of
setup + solve (the metric's definition: n / (t_setup + t_solve)); the
transposed solve is timed in the same steps and reported beside it, and
`ms_per_step` covers all three phases.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  The CPU-baseline leg times the plain CPU oracle (one
thread) on the same workload.  The batched leg ("batched") sets up and solves
64 discrete-ordinate systems on uneven meshes (17.7M DOFs) as one batched
hierarchy with a graph-replayed iteration, with the FP32-stored and the FP64
hierarchy, beside the same systems set up and solved one after another.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOFs/s setup+solve to 1e-10 rel. residual, FP64 vs batched FP32-hier; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def measured_traffic(workload: str, grid_threads: int):
    """HBM bytes per launch of an F sweep, pre-recorded: the committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs per launch shape, scaled by
    reference kernels), or None when there is none for this launch shape or
    the kernel source has changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_sweep_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1704_05001_amd", "csrc", "cycle.hip"), "rb").read()
    if d.get("cycle_hip_sha256") != hashlib.sha256(src).hexdigest():
        return None
    t = d.get("traffic_by_grid", {}).get(str(grid_threads))
    return float(t) if t is not None else None


def relax_level_bytes(lv: dict) -> dict:
    """Algorithmic HBM bytes of one F-relaxation sweep on a level: each operand
    read once, each output written once (int32 indices, FP64 values).  The
    sweep e_I = D_I^-1 (r_I - sum_{J != I} A_IJ e_J) reads every off-diagonal
    block of an F row (from A, where the diagonal block's column index and
    masks are read too, or from the level's sweep copy, which holds only the
    off-diagonal blocks); of e, the entries those blocks multiply, each once.
    With face rectangles an off-diagonal block costs the entries on its
    nonzero rows and columns plus its 8-byte row/column masks; a sweep copy
    without them stores each block by its nonzero rows (full width) with a
    4-byte row mask and a 4-byte offset."""
    import numpy as np
    rp = lv["rowptr"].cpu().numpy().astype(np.int64)
    cf = lv["cf"].cpu().numpy()
    bs = lv["bs"]
    bb = bs * bs
    rowlen = np.diff(rp)
    F = cf == 0
    nF = int(F.sum())
    nnzF = int(rowlen[F].sum())
    rows = np.repeat(np.arange(lv["nb"]), rowlen)
    ci = lv["colidx"].cpu().numpy()
    inF = F[rows]
    diag = ci == rows
    off = inF & ~diag
    copy = lv.get("sweep_nnzb", -1) >= 0
    if lv.get("face_meta") is not None:
        meta = lv["face_meta"].cpu().numpy().view(np.uint64)
        nr = np.bitwise_count(meta & np.uint64(0xFFFFFFFF)).astype(np.int64)
        nc = np.bitwise_count(meta >> np.uint64(32)).astype(np.int64)
        bytes_A = (0 if copy else nF * 12) + int((12 + 8 * nr * nc)[off].sum())
        # e entries needed: per neighbour J, the union of its blocks' nonzero columns
        cm = np.zeros(lv["nb"], dtype=np.uint64)
        np.bitwise_or.at(cm, ci[off], meta[off] >> np.uint64(32))
        bytes_e = int(np.bitwise_count(cm).astype(np.int64).sum()) * 8
    elif copy:
        nzr = nonzero_rows(lv["vals"])
        bytes_A = int((nzr[off] * bs * 8 + 12).sum())
        bytes_e = len(np.unique(ci[off])) * bs * 8
    else:
        bytes_A = nF * 4 + int(off.sum()) * (bb * 8 + 4)   # off-diagonal blocks (+ diagonal's index)
        bytes_e = len(np.unique(ci[off])) * bs * 8
    bytes_D = nF * bb * 8                  # D_F^{-1}
    bytes_idx = nF * 4 + nF * 8            # F list, rowptr pairs
    bytes_vec = bytes_e + nF * bs * 8 * 2  # e gathered (each needed entry once), r_F, e_out_F
    return dict(bytes=bytes_A + bytes_D + bytes_idx + bytes_vec, nF=nF, nnzF=nnzF,
                bytes_true_blocks=bytes_A + bytes_D, sweep_copy=copy)


def sweep_launch_shape(lv: dict, nF: int, tuning, level: int):
    """The F sweep launch on a level as the library issues it: (kernel, lane
    groups, grid threads).  A face-compressed copy runs k_sweep with G groups of
    bs lanes per row; a copy stored by nonzero rows with bs >= 8 on a level of
    32,768 lanes or more runs k_sweep_cr, R = max(1, 512 / (G bs)) rows per
    256-thread workgroup."""
    G = int(tuning[level][0]) if tuning is not None and len(tuning) > level else 0
    if G <= 0:
        avg_row = lv["nnzb"] / max(1, lv["nb"])
        G = 1 if avg_row <= 3.5 else (2 if avg_row <= 7.0 else (4 if avg_row <= 14.0 else 8))
    bs = lv["bs"]
    while G > 1 and G * bs > 256:
        G //= 2
    stored_rows = lv.get("face_meta") is None and lv.get("sweep_nnzb", -1) >= 0
    if stored_rows and bs >= 8 and nF * bs >= 32768:
        R = max(1, 512 // (G * bs))
        return "k_sweep_cr", G, -(-nF // R) * 256
    rows_per_wg = 256 // (G * bs)
    return "k_sweep", G, -(-nF // rows_per_wg) * 256


def H_level0_fields(H):
    return H.level(0, fields=("rowptr", "colidx", "cf", "face_meta", "vals"))


def host_relres(S, x) -> float:
    """||b - A x||_2 / ||b||_2 in FP64 on the host (numpy block products), an
    independent check of a GPU solution."""
    import numpy as np
    xb = x.detach().cpu().numpy().reshape(S.nb, S.bs)
    prod = np.einsum("tij,tj->ti", S.vals, xb[S.colidx])
    Ax = np.add.reduceat(prod, S.rowptr[:-1].astype(np.int64), axis=0)
    r = S.rhs - Ax.reshape(-1)
    return float(np.linalg.norm(r) / np.linalg.norm(S.rhs))


def nonzero_rows(vals):
    """Rows with a nonzero entry, per block of a (nnzb, bs, bs) array (on the host)."""
    v = vals.cpu().numpy()
    return (v != 0).any(axis=2).sum(axis=1).astype("int64")


def restrict_level_bytes(lv: dict) -> int:
    """Algorithmic HBM bytes of one restriction r_c = r_C + Z r_F on a level:
    Z's blocks and column indices, its row pointers, the C list, r_C read and
    r_c written, r_F gathered once.  Where the level has a sweep copy, Z is
    read from its row-compressed copy: each block's nonzero rows at full
    width, a 4-byte row mask and a 4-byte offset."""
    import numpy as np
    bs = lv["bs"]
    nc = int(lv["nc"])
    znnz = int(lv["z_rowptr"][-1].item()) if nc > 0 else 0
    nF = int((lv["cf"].cpu().numpy() == 0).sum())
    if znnz > 0 and lv.get("sweep_nnzb", -1) >= 0:
        bytes_Z = int((nonzero_rows(lv["z_vals"]) * bs * 8 + 12).sum())
    else:
        bytes_Z = znnz * (bs * bs * 8 + 4)
    return bytes_Z + (nc + 1) * 4 + nc * 4 + nc * bs * 16 + nF * bs * 8


def level_bandwidth(P, H, b, levels: int) -> list:
    """Per level: the forward solve's F sweep and restriction, average launch
    time from the library's HIP-event timer over one solve each, and the
    algorithmic GB/s."""
    out = []
    for l in range(levels):
        lv = H.level(l, fields=("rowptr", "colidx", "cf", "z_rowptr", "z_vals"))
        if lv["coarsest"]:
            break
        row = {"level": l, "nb": lv["nb"], "nnzb": lv["nnzb"]}
        for kind, nbytes in (("relax", relax_level_bytes(H.level(l, fields=("rowptr", "colidx", "cf", "face_meta", "vals")))["bytes"]),
                             ("restrict", restrict_level_bytes(lv))):
            P.timer_select(kind, l)
            H.solve(b)
            P.timer_select(None)
            n, ms = P.timer_read()
            us = ms * 1e3 / max(n, 1)
            row[f"{kind}_us"] = round(us, 2)
            row[f"{kind}_MB"] = round(nbytes / 1e6, 2)
            row[f"{kind}_GBs"] = round(nbytes / (us * 1e-6) / 1e9, 1) if n else None
        out.append(row)
    return out


FP64_PEAK_TFS = 78.6   # MI355X dense FP64 (matrix cores and vector units alike)


def setup_work(H, degree: int) -> dict:
    """Algorithmic work of one setup of hierarchy H, from its levels' patterns
    (host scipy on the block patterns; no values): block pairs of the Neumann
    products W_i = W_{i-1} T (T: the phi-strong F-F blocks, W_0 = A_cf) and of
    the coarse operator R (A P) (R = [Z I]; A P merges A's columns through the
    one-point map), the single block products T = -D^-1 A_ff and Z = -S D^-1
    (S = W_0 + ... + W_k, never stored: Z's product reads the k+1 terms),
    the block inverses, and the compulsory bytes of each (operands read once,
    outputs written once, 8-byte pair entries).  Flops: 2 bs^3 per block pair
    or block product, 2 bs^3 per block inverse (LU and the inverse from it)."""
    import numpy as np
    import scipy.sparse as sp
    info = H.info()
    w = {k: 0 for k in ("pairs_W", "pairs_RAP", "ident_RAP", "blocks_T", "blocks_Z", "blocks_W", "blocks_Wprev",
                        "blocks_W0", "blocks_K", "blocks_AP", "nb_inv")}
    bs = None
    for l in range(info["levels"]):
        lv = H.level(l, fields=("rowptr", "colidx", "mask", "cf", "pmap", "z_rowptr", "z_colidx"))
        if lv["coarsest"]:
            break
        bs = lv["bs"]
        nb = lv["nb"]
        rp = lv["rowptr"].cpu().numpy().astype(np.int64)
        ci = lv["colidx"].cpu().numpy().astype(np.int64)
        mask = lv["mask"].cpu().numpy()
        cf = lv["cf"].cpu().numpy()
        rows = np.repeat(np.arange(nb), np.diff(rp))
        F = cf == 0
        tm = F[rows] & F[ci] & (rows != ci) & ((mask & 2) != 0)
        T = sp.csr_matrix((np.ones(int(tm.sum())), (rows[tm], ci[tm])), shape=(nb, nb))
        cm = (cf[rows] == 1) & F[ci]
        W = sp.csr_matrix((np.ones(int(cm.sum())), (rows[cm], ci[cm])), shape=(nb, nb))
        tlen = np.diff(T.indptr)
        w["blocks_W0"] += W.nnz
        for _ in range(degree):
            w["pairs_W"] += int(tlen[W.indices].sum())
            w["blocks_Wprev"] += W.nnz
            W = (W @ T).tocsr()
            W.data[:] = 1.0
            w["blocks_W"] += W.nnz
        pm = lv["pmap"].cpu().numpy().astype(np.int64)
        kp = pm[ci] >= 0
        AP = sp.csr_matrix((np.ones(int(kp.sum())), (rows[kp], pm[ci[kp]])), shape=(nb, int(lv["nc"])))
        AP.sum_duplicates()
        aplen = np.diff(AP.indptr)
        zc = lv["z_colidx"].cpu().numpy().astype(np.int64)
        w["pairs_RAP"] += int(aplen[zc].sum())         # Z_ik (A P)_k. products
        w["ident_RAP"] += int(aplen[cf == 1].sum())    # (A P)_c. blocks added plainly
        w["blocks_T"] += T.nnz
        w["blocks_Z"] += len(zc)
        w["blocks_AP"] += AP.nnz
        w["nb_inv"] += nb
        w["blocks_K"] += H.level(l + 1, fields=())["nnzb"]
    w["bs"] = bs
    return w


def setup_roofline(P, make_hier, work: dict, reps: int = 1) -> list:
    """Per setup kernel kind: total launch time over `reps` setups (the
    library's HIP-event timer, all levels), the algorithmic flops and bytes of
    one setup (setup_work), and both fractions of MI355X's peaks; `bound` names
    the larger, the resource the kernel is nearer to."""
    bs = work["bs"]
    bb8 = 8 * bs * bs
    f3 = 2.0 * bs ** 3
    kinds = {
        "galerkin": dict(kernel="k_pair_sums (R (A P) block products summed into K blocks)",
                         flops=work["pairs_RAP"] * f3,
                         bytes=(work["blocks_Z"] + work["blocks_AP"] + work["blocks_K"]) * bb8
                         + 8 * (work["pairs_RAP"] + work["ident_RAP"])),
        "spgemm_numeric": dict(kernel="k_pair_sums (Neumann products W_i = W_(i-1) T)",
                               flops=work["pairs_W"] * f3,
                               bytes=(work["blocks_Wprev"] + work["blocks_T"] + work["blocks_W"]) * bb8
                               + 8 * work["pairs_W"]),
        # Z's product adds the terms W_0 .. W_k of the unstored sum S itself: each term block read once
        "block_product": dict(kernel="k_block_product_mfma (T = -D^-1 A_ff), k_sum_product_mfma "
                                     "(Z = -(W_0 + ... + W_k) D^-1)",
                              flops=(work["blocks_T"] + work["blocks_Z"]) * f3,
                              bytes=(3 * work["blocks_T"] + work["blocks_W0"] + work["blocks_W"]
                                     + 2 * work["blocks_Z"]) * bb8),
        "block_inverse": dict(kernel="k_block_inverse_rows (D^-1 by LU)", flops=work["nb_inv"] * f3,
                              bytes=work["nb_inv"] * 2 * bb8),
    }
    out = []
    for kind, d in kinds.items():
        P.timer_read()
        P.timer_select(kind, -1)
        for _ in range(reps):
            make_hier().close()
        P.timer_select(None)
        n, ms = P.timer_read()
        if n == 0 or ms <= 0:
            continue
        t = ms * 1e-3 / reps
        tf = d["flops"] / t / 1e12
        gb = d["bytes"] / t / 1e9
        fm, fh = tf / FP64_PEAK_TFS, gb / HBM_PEAK_GBS
        out.append({"kind": kind, "kernel": d["kernel"], "ms_per_setup": round(ms / reps, 3),
                    "launches_per_setup": n // reps, "gflop": round(d["flops"] / 1e9, 2),
                    "MB": round(d["bytes"] / 1e6, 1), "TFLOPs": round(tf, 2), "GBs": round(gb, 1),
                    "frac_fp64_peak": round(fm, 4), "frac_hbm_peak": round(fh, 4),
                    "bound": "mfma" if fm >= fh else "hbm"})
    return out


def batched_leg(args, P, torch, np):
    """Many discrete-ordinate systems in one hierarchy and one graph-replayed
    solve, FP32-stored and FP64, against the same systems set up and solved
    one after another."""
    from nair_inputs import make_batch, concat_systems
    t0 = time.time()
    workers = max(1, min(16, os.cpu_count() or 1))
    systems, degree = make_batch(args.batch_workload, workers=workers, check_acyclic=False)
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    ndof = int(rhs.size)
    log(f"batch {args.batch_workload}: {len(systems)} systems, {ndof} DOFs, nnzb {ci.size} "
        f"({time.time() - t0:.1f}s to generate)")
    dev = torch.device("cuda", 0)
    d_rp, d_ci, d_va = (torch.from_numpy(a).to(dev) for a in (rp, ci, va))
    d_b = torch.from_numpy(rhs).to(dev)
    x = torch.empty_like(d_b)
    stream = torch.cuda.current_stream()
    res = {"workload": args.batch_workload, "systems": len(systems), "dofs": ndof, "nnzb": int(ci.size),
           "meshes": sorted({int(S.N) for S in systems}), "steps": args.batch_steps,
           "step": "one batched setup + one batched solve of every system to 1e-10; value = dofs / (setup + solve)"}

    tables = {}

    def run(prec, graph):
        prm = P.Params(faces=not args.no_faces, degree=degree, precision=prec)
        if not args.no_tune:
            if prec not in tables:   # lane groups tuned once per precision on the batch hierarchy
                Ht = P.Hierarchy(d_rp, d_ci, d_va, 9, prm, sys_nb=sys_nb)
                tables[prec] = Ht.autotune(reps=10)
                Ht.close()
            prm = P.Params(faces=not args.no_faces, degree=degree, precision=prec, tuning=tables[prec])
        times, iters = [], None
        for i in range(1 + args.batch_steps):        # first step untimed (warm-up)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record(stream)
            H = P.Hierarchy(d_rp, d_ci, d_va, 9, prm, sys_nb=sys_nb)
            ev[1].record(stream)
            _, rr = H.solve_batch(d_b, x=x, rtol=args.rtol, graph=graph)
            ev[2].record(stream)
            torch.cuda.synchronize()
            if any(r.status != "OK" for r in rr):
                raise RuntimeError(f"batched solve: {[r.status for r in rr if r.status != 'OK'][:3]}")
            if i > 0:
                times.append((ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])))
            iters = [r.iters for r in rr]
            levels = H.info()["levels"]
            H.close()
        st = float(np.mean([t[0] for t in times]))
        sv = float(np.mean([t[1] for t in times]))
        return {"value": round(ndof / ((st + sv) * 1e-3), 1), "unit": "DOFs/s", "setup_ms": round(st, 3),
                "solve_ms": round(sv, 3), "iters_min": min(iters), "iters_max": max(iters), "levels": levels}

    res["fp32_hier_graph"] = run("fp32", True)
    x32 = x.clone()
    res["fp64_graph"] = run("fp64", True)
    res["fp64_eager"] = run("fp64", False)
    res["fp32_hier_max_rel_diff_vs_fp64"] = float((x32 - x).abs().max() / x.abs().max())
    log(f"batched: fp32 graph {res['fp32_hier_graph']['value']:.0f}, fp64 graph {res['fp64_graph']['value']:.0f}, "
        f"fp64 eager {res['fp64_eager']['value']:.0f} DOFs/s")

    res["tuned"] = not args.no_tune
    # the same systems one after another: setup + solve each with the plain entry points
    # (default lane groups: a tuning table fits one hierarchy structure)
    prm = P.Params(faces=not args.no_faces, degree=degree)
    per = []
    offs = np.concatenate(([0], np.cumsum([S.nnzb for S in systems])))
    boff = np.concatenate(([0], np.cumsum(sys_nb)))
    subs = []
    for k, S in enumerate(systems):
        subs.append((torch.from_numpy(S.rowptr).to(dev), torch.from_numpy(S.colidx).to(dev),
                     d_va[offs[k]:offs[k + 1]], d_b[boff[k] * 9:boff[k + 1] * 9], x[boff[k] * 9:boff[k + 1] * 9]))
    for i in range(1 + args.batch_steps):
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for (srp, sci, sva, sb, sx) in subs:
            H = P.Hierarchy(srp, sci, sva, 9, prm)
            _, r = H.solve(sb, x=sx, rtol=args.rtol)
            if r.status != "OK":
                raise RuntimeError(f"sequential solve {r.status}")
            H.close()
        ev[1].record(stream)
        torch.cuda.synchronize()
        if i > 0:
            per.append(ev[0].elapsed_time(ev[1]))
    seq_ms = float(np.mean(per))
    res["fp64_sequential"] = {"value": round(ndof / (seq_ms * 1e-3), 1), "unit": "DOFs/s", "ms": round(seq_ms, 3),
                              "what": "nair_setup + nair_solve per system, one after another"}
    res["speedup_fp32_graph_vs_fp64_sequential"] = round(res["fp32_hier_graph"]["value"] /
                                                         res["fp64_sequential"]["value"], 3)
    res["speedup_fp32_graph_vs_fp64_graph"] = round(res["fp32_hier_graph"]["value"] / res["fp64_graph"]["value"], 3)
    del d_rp, d_ci, d_va, d_b, x, subs
    torch.cuda.empty_cache()
    P.pool_trim()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dg_q4_512_jitter")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--roofline-kernel", default="relax")
    ap.add_argument("--roofline-level", type=int, default=1,
                    help="level of the roofline F sweep (1: the stored-row sweep, the step's dominant kernel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-hierarchy leg")
    ap.add_argument("--cpu-sample", default="auto",
                    help="'full', a mesh size N for the oracle sample, or 'auto' (full up to 1M DOFs, else N = 96)")
    ap.add_argument("--batch-workload", default="dg_q2_angles64_uneven")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-angles leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the default lane groups (no autotuning)")
    ap.add_argument("--no-setup-roofline", action="store_true", help="skip the per-kernel setup timing")
    ap.add_argument("--roofline-groups", type=int, default=0, metavar="G",
                    help="lane groups per row of the roofline kernel's F sweep (0: as tuned, or the default)")
    ap.add_argument("--no-faces", action="store_true",
                    help="read whole blocks of the finest operator (no face-compressed copy)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched leg and print its JSON (for profiling it alone)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="after the timed steps, fill, sum and copy a BYTES buffer (reference kernels of "
                         "known traffic for hardware counters)")
    ap.add_argument("--skip-transposed", action="store_true",
                    help="leave the transposed solve out of every step (for counter runs of the forward "
                         "cycle only; not a benchmark configuration)")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "one GPU only: run with --gpus 1 (the path is not sharded across GPUs)"}),
              flush=True)
        return 2

    import numpy as np
    import torch
    import paper_1704_05001_amd as P
    from nair_inputs import make_config

    if not os.path.exists(P.LIB_PATH):
        from paper_1704_05001_amd.build import build
        build()
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        return 3

    if args.batch_only:
        print(json.dumps(batched_leg(args, P, torch, np)), flush=True)
        return 0

    t0 = time.time()
    S, degree = make_config(args.workload)
    log(f"workload {args.workload}: {S.n} DOFs, nb={S.nb}, bs={S.bs}, nnzb={S.nnzb}, degree={degree} "
        f"({time.time() - t0:.1f}s to generate)")
    dev = torch.device("cuda", 0)
    rp = torch.from_numpy(S.rowptr).to(dev)
    ci = torch.from_numpy(S.colidx).to(dev)
    va = torch.from_numpy(S.vals).to(dev)
    b = torch.from_numpy(S.rhs).to(dev)
    g = torch.from_numpy(np.random.Generator(np.random.PCG64(300)).uniform(-1, 1, S.n)).to(dev)
    x = torch.empty_like(b)
    y = torch.empty_like(g)
    params = P.Params(faces=not args.no_faces, degree=degree)
    stream = torch.cuda.current_stream()

    def step(record, prm=params, xo=x, yo=y, timed=False):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        H = P.Hierarchy(rp, ci, va, S.bs, prm)
        ev[1].record(stream)
        if timed:   # the kernel timer brackets the forward solve's launches of the roofline kernel
            P.timer_select(args.roofline_kernel, args.roofline_level)
        _, r = H.solve(b, x=xo, rtol=args.rtol)
        if timed:
            P.timer_select(None)
        ev[2].record(stream)
        if args.skip_transposed:
            rT = r
        else:
            _, rT = H.solve_T(g, y=yo, rtol=args.rtol)
        ev[3].record(stream)
        if r.status != "OK" or rT.status != "OK":
            raise RuntimeError(f"solve status {r.status} / {rT.status}")
        if record is not None:
            record.append((ev, r, rT))
        return H

    for i in range(args.warmup):
        H = step(None)
        if i == 0:
            info = H.info()
            lvl = H.level(args.roofline_level)
            lvl0 = H.level(0, fields=())
            audit = [int(v) for v in np.sum([H.level(l, fields=())["margin"] for l in range(info["levels"])], axis=0)]
            log(f"levels {info['levels']} nb {info['nb']} OC {info['oc']:.2f} CC {info['cc']:.2f}")
        H.close()
    if args.warmup == 0:
        H = step(None)
        info = H.info()
        lvl = H.level(args.roofline_level)
        lvl0 = H.level(0, fields=())
        audit = [int(v) for v in np.sum([H.level(l, fields=())["margin"] for l in range(info["levels"])], axis=0)]
        H.close()

    tuning = None
    if not args.no_tune:
        # lane groups of the cycle kernels, tuned once on this matrix's hierarchy
        Ht = P.Hierarchy(rp, ci, va, S.bs, params)
        tuning = Ht.autotune(reps=20)
        Ht.close()
        params = P.Params(faces=not args.no_faces, degree=degree, tuning=tuning)
    if args.roofline_groups > 0:
        # the roofline kernel at a given launch shape (the rest as tuned or default)
        if tuning is None:
            tuning = np.zeros((64, len(P.TUNE_KINDS)), dtype=np.int8)
        tuning = np.array(tuning, dtype=np.int8)
        tuning[args.roofline_level][0] = args.roofline_groups
        params = P.Params(faces=not args.no_faces, degree=degree, tuning=tuning)
    if tuning is not None:
        for _ in range(max(1, args.warmup)):
            step(None, params).close()

    recs = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        H = step(recs, params, timed=True)
        H.close()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    launches, kernel_ms = P.timer_read()
    log(f"timed {args.steps} steps in {t_end - t_start:.3f}s")
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe // 8, dtype=torch.float64, device=dev)
        src.fill_(1.0)                       # writes BYTES
        total = float(src.sum())             # reads BYTES
        dst = torch.empty_like(src)
        dst.copy_(src)                       # reads and writes BYTES
        torch.cuda.synchronize()
        log(f"copy probe: fill, sum ({total:.0f}) and copy of {src.numel() * 8} bytes")
        del src, dst

    setup_ms = np.mean([e[0].elapsed_time(e[1]) for e, _, _ in recs])
    solve_ms = np.mean([e[1].elapsed_time(e[2]) for e, _, _ in recs])
    solveT_ms = np.mean([e[2].elapsed_time(e[3]) for e, _, _ in recs])
    wall_ms = (t_end - t_start) * 1e3 / args.steps
    iters = recs[-1][1].iters
    itersT = recs[-1][2].iters
    value = S.n / ((setup_ms + solve_ms) * 1e-3)

    def sweep_roof(level, lv, avg_ms, nlaunch):
        """Roofline entry of a level's forward F sweep from its average launch time."""
        rb = relax_level_bytes(lv)
        achieved = rb["bytes"] / (avg_ms * 1e-3) / 1e9
        name, G, grid_threads = sweep_launch_shape(lv, rb["nF"], tuning, level)
        return {"bound": "hbm", "kernel": f"{name} (level {level} F sweep)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, grid_threads),
                "traffic_source": "pre-recorded rocprofv3 FETCH_SIZE + WRITE_SIZE of this launch shape "
                                  "(profiles/), null when the kernel source changed since",
                "bytes_per_launch": rb["bytes"], "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches": nlaunch, "lane_groups": G, "grid_threads": grid_threads}

    roof = None
    if args.roofline_kernel == "relax" and launches > 0:
        roof = sweep_roof(args.roofline_level, lvl, kernel_ms / launches, launches)

    Hl = P.Hierarchy(rp, ci, va, S.bs, params)
    P.timer_read()
    levels_bw = level_bandwidth(P, Hl, b, info["levels"])
    Hl_work = Hl
    for r in levels_bw:
        log(f"level {r['level']}: relax {r['relax_us']} us {r['relax_GBs']} GB/s, "
            f"restrict {r['restrict_us']} us {r['restrict_GBs']} GB/s")
    # the finest level's face-compressed sweep, beside the roofline kernel
    roof0 = None
    if args.roofline_level != 0 and levels_bw and levels_bw[0].get("relax_us"):
        roof0 = sweep_roof(0, H_level0_fields(Hl), levels_bw[0]["relax_us"] * 1e-3, None)

    rT = recs[-1][2]
    r0 = recs[-1][1]
    import math as _m
    conv = {"iters": iters, "rho_avg": r0.rho_avg, "rho_last5": r0.rho_last5, "cc": round(info["cc"], 4),
            "oc": round(info["oc"], 4),
            "wpd": round(-info["cc"] / _m.log10(r0.rho_avg), 3) if 0 < r0.rho_avg < 1 else None,
            "iters_T": itersT, "rho_avg_T": rT.rho_avg, "rho_last5_T": rT.rho_last5,
            "what": "rho_avg = h_K^(1/K), rho_last5 = (h_K/h_(K-5))^(1/5), WPD = -CC/log10(rho_avg); "
                    "CC, OC in work units of one level-0 SpMV"}
    log(f"convergence: {iters} iterations, rho_avg {r0.rho_avg:.3f}, rho_last5 {r0.rho_last5:.3f}, "
        f"CC {info['cc']:.2f}, WPD {conv['wpd']}")

    setup_roof = None
    if not args.no_setup_roofline:
        work = setup_work(Hl_work, degree)
        setup_roof = setup_roofline(P, lambda: P.Hierarchy(rp, ci, va, S.bs, params), work)
        for r in setup_roof:
            log(f"setup {r['kind']}: {r['ms_per_setup']} ms, {r['TFLOPs']} TFLOP/s ({r['frac_fp64_peak']:.3f}), "
                f"{r['GBs']} GB/s ({r['frac_hbm_peak']:.3f})")
    Hl_work.close()

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "DOFs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "mesh": f"{S.N}x{S.N} quads", "dg_order": S.p,
                   "dofs": S.n, "block": S.bs, "nnzb": S.nnzb, "neumann_degree": degree,
                   "rtol": args.rtol, "levels": info["levels"], "oc": round(info["oc"], 3),
                   "cc": round(info["cc"], 3),
                   "face_blocks": ([lvl0["face_rmax"], lvl0["face_cmax"]] if lvl0["face_rmax"] > 0 else None)},
        "setup_ms": round(float(setup_ms), 3), "solve_ms": round(float(solve_ms), 3),
        "solve_T_ms": round(float(solveT_ms), 3), "iters": iters, "iters_T": itersT,
        "step": "setup + solve + transposed solve; value = dofs / (setup + solve)",
        "roofline": roof,
        "roofline_level0_sweep": roof0,
        "convergence": conv,
        "setup_roofline": setup_roof,
        "decision_margin_audit": dict(zip(("theta", "phi", "one_point", "drop"), audit)),
        "levels_bandwidth": levels_bw,
        "tuned": tuning is not None,
        "tuning": tuning.tolist() if tuning is not None else None,
        "tuning_kinds": list(P.TUNE_KINDS),
    }

    if not args.no_fp32:
        # the same steps with the FP32-stored hierarchy (FP64 setup, refinement and residuals)
        p32 = P.Params(faces=not args.no_faces, degree=degree, precision="fp32")
        if not args.no_tune:
            Ht = P.Hierarchy(rp, ci, va, S.bs, p32)
            p32 = P.Params(faces=not args.no_faces, degree=degree, precision="fp32", tuning=Ht.autotune(reps=20))
            Ht.close()
        x32, y32 = torch.empty_like(b), torch.empty_like(g)
        for _ in range(max(1, args.warmup)):
            step(None, p32, x32, y32).close()
        recs32 = []
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(args.steps):
            step(recs32, p32, x32, y32).close()
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        s32 = np.mean([e[0].elapsed_time(e[1]) for e, _, _ in recs32])
        v32 = np.mean([e[1].elapsed_time(e[2]) for e, _, _ in recs32])
        t32 = np.mean([e[2].elapsed_time(e[3]) for e, _, _ in recs32])
        err_x = float((x32 - x).abs().max() / x.abs().max())
        err_y = float((y32 - y).abs().max() / y.abs().max())
        out["fp32_hier"] = {"value": round(S.n / ((s32 + v32) * 1e-3), 1), "unit": "DOFs/s",
                            "ms_per_step": round((f1 - f0) * 1e3 / args.steps, 3),
                            "setup_ms": round(float(s32), 3), "solve_ms": round(float(v32), 3),
                            "solve_T_ms": round(float(t32), 3), "iters": recs32[-1][1].iters,
                            "iters_T": recs32[-1][2].iters, "relres": recs32[-1][1].relres,
                            "max_rel_diff_x_vs_fp64": err_x, "max_rel_diff_y_vs_fp64": err_y,
                            "relres_host_fp64": host_relres(S, x32), "relres_host_fp64_of_fp64_x": host_relres(S, x),
                            "speedup_vs_fp64": round((setup_ms + solve_ms) / (s32 + v32), 3)}
        log(f"fp32 hierarchy: {out['fp32_hier']['value']:.0f} DOFs/s, {out['fp32_hier']['iters']} iterations")

    if not args.no_batch:
        out["batched"] = batched_leg(args, P, torch, np)

    if not args.no_cpu_baseline:
        import oracle
        cs = args.cpu_sample
        if cs == "auto":
            cs = "full" if S.n <= 1_000_000 else "96"
        if cs == "full":
            So, dego = S, degree
            sample = f"full {args.workload} ({S.n} DOFs): one oracle setup + solve to {args.rtol:g}"
        else:
            So, dego = make_config(args.workload, N=int(cs))
            sample = (f"{args.workload} recipe at N={cs} ({So.n} DOFs, {So.nb} blocks of {So.bs}x{So.bs}): one "
                      f"oracle setup + solve to {args.rtol:g}; DOFs/s of that sample (its iteration count differs "
                      f"from the full mesh's)")
        log(f"cpu baseline: {sample}")
        c0 = time.perf_counter()
        O = oracle.Hierarchy(So.nb, So.bs, So.rowptr, So.colidx, So.vals, oracle.Params(degree=dego))
        c1 = time.perf_counter()
        xo, ho, so = O.solve(So.rhs, args.rtol, 500)
        c2 = time.perf_counter()
        out["cpu_baseline"] = {"value": round(So.n / (c2 - c0), 1), "unit": "DOFs/s", "cores": 1,
                               "kind": "oracle", "sample": sample,
                               "setup_s": round(c1 - c0, 3), "solve_s": round(c2 - c1, 3),
                               "iters": len(ho), "cpu": cpu_model(), "nproc": os.cpu_count()}
        if So is S:
            xg = x.cpu().numpy()
            out["cpu_baseline"]["max_rel_diff_x"] = float(np.abs(xg - xo).max() / np.abs(xo).max())
            out["cpu_baseline"]["same_iters"] = bool(len(ho) == iters)
            if "fp32_hier" in out:
                out["fp32_hier"]["max_rel_err_x_vs_fp64_oracle"] = float(
                    np.abs(x32.cpu().numpy() - xo).max() / np.abs(xo).max())
        else:
            # the GPU paths on the same sample, against the oracle's solution there
            srp, sci, sva, sb = (torch.from_numpy(a).to(dev) for a in (So.rowptr, So.colidx, So.vals, So.rhs))
            cmp = {}
            for prec in ("fp64", "fp32"):
                Hs = P.Hierarchy(srp, sci, sva, So.bs, P.Params(faces=not args.no_faces, degree=dego, precision=prec))
                xs, rs = Hs.solve(sb, rtol=args.rtol)
                Hs.close()
                cmp[prec] = {"max_rel_err_x_vs_fp64_oracle": float(np.abs(xs.cpu().numpy() - xo).max()
                                                                   / np.abs(xo).max()),
                             "iters": rs.iters, "oracle_iters": len(ho)}
            out["cpu_baseline"]["gpu_on_sample"] = cmp
            if "fp32_hier" in out:
                out["fp32_hier"]["max_rel_err_x_vs_fp64_oracle_on_sample"] = cmp["fp32"]["max_rel_err_x_vs_fp64_oracle"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
