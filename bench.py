"""Benchmark of the stiffness-operator apply on one MI355X.

One step = one application y = A x of the whole decomposed operator
(A = B + M + K~: CSR near field + weighted mass, dense near leaf blocks, H2
far field) to the workload's right-hand side(s), inputs resident in HBM.

Metric: DOF-matvecs/s = N * F * R * steps / elapsed.  The default workload is
the 2D unit square with 128 x 128 cells split in two (16129 dofs, 131072 cells
including the exterior band), jittered nodes, variable order and diffusivity,
leaf 64, 5 Chebyshev points per dimension, eta = 1, one right-hand side.

Prints one JSON line (see the contract in the repository docs) with a
roofline entry for the dominant kernel (k_near_up: CSR of B + M, packed near
leaf blocks, and the upsweep of the far field in the same launch) measured
with HIP events on the apply stream, and a CPU baseline of the oracle on a
bounded sample of rows of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def workload(name: str):
    from fpde_inputs import configs
    if name == "square":
        return configs.square(128), {"workload": "square-128x128-P1 (16129 dofs, 131072 cells), variable s and kappa",
                                     "n": 128, "leaf": 64, "cheb_p": 5, "eta": 1.0, "nrhs": 1, "fields": 1}
    if name == "square-small":
        return configs.square(32), {"workload": "square-32x32-P1", "n": 32, "nrhs": 1, "fields": 1}
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes_near(op, st, F, R, dim, p):
    """HBM bytes one launch of the near/upsweep kernel must move, no re-reads counted:
    the near leaf blocks (sum over near pairs of |s| |s'| FP64 entries), the nonzeros
    of B + M (FP64 values, int32 columns) and one 8-byte index per row, x read once,
    y written once, the leaf bases U (N x k FP64) and the transfers (D P^2 per
    cluster) read once, the cluster coefficients (k per cluster) written once.  The
    kernel reads B + M in an ELL form by leaf slot; its padding is not counted."""
    leafptr = op.export("K_LEAFPTR")
    sizes = leafptr[1:] - leafptr[:-1]
    pairs = op.export("K_NEAR").reshape(-1, 2)
    first = (1 << (int(st["k_levels"]) - 1)) - 1
    near_entries = int((sizes[pairs[:, 0] - first] * sizes[pairs[:, 1] - first]).sum())
    N = st["n_dofs"]
    nnz = st["csr_nnz"]
    b = F * near_entries * 8
    b += F * nnz * 8 + nnz * 4 + (N + 1) * 8
    b += 2 * F * N * R * 8
    k, ncl = int(st["k_rank"]), int(st["k_clusters"])
    b += N * k * 8 + ncl * dim * p * p * 8 + F * ncl * k * 8
    return b, near_entries


def measured_traffic(kernel_name):
    """HBM traffic of the dominant kernel from the committed rocprofv3 counter record,
    valid only while the kernel source is unchanged (else None)."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "traffic_%s_square128.json" % kernel_name)
    src = os.path.join(ROOT, "paper_2302_02863_amd", "csrc", "fpde_apply.hip")
    try:
        rec = json.load(open(rec_path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernel") != kernel_name or rec.get("source_sha256") != sha:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(P, seconds: float = 15.0):
    """Oracle rows of A_h x computed one by one on the host cores (bounded sample)."""
    import numpy as np
    from oracle.sampled import SampledOracle
    np.seterr(divide="ignore", invalid="ignore")
    t0 = time.perf_counter()
    so = SampledOracle(P.mesh, P.s[0], P.kappa[0], P.opts)
    t_setup = time.perf_counter() - t0
    rng = np.random.default_rng(11)
    rows = rng.choice(P.mesh.n_dofs, size=64, replace=False)
    done = 0
    t1 = time.perf_counter()
    for r in rows:
        so.row_apply([int(r)], P.x[0, :, 0])
        done += 1
        if time.perf_counter() - t1 > seconds:
            break
    el = time.perf_counter() - t1
    try:
        import threadpoolctl
        cores = max(i["num_threads"] for i in threadpoolctl.threadpool_info()) if threadpoolctl.threadpool_info() else 1
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": done / el, "unit": "DOF-matvecs/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{done} rows of A_h x on the same workload computed entry by entry by the FP64 oracle "
                      f"(tree/partition/basis setup {t_setup:.1f} s excluded, rows {el:.1f} s)"}


def time_applies(op, x, y, stream, steps, warmup, parts=None):
    import torch
    kw = {} if parts is None else {"parts": parts}
    for _ in range(warmup):
        op.apply(x, y, stream=stream, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        op.apply(x, y, stream=stream, **kw)          # the apply's kernels, launched directly
    torch.cuda.synchronize()
    return time.perf_counter() - t1


def mixed_and_solve(P, op64, x, y64, stream, steps, warmup):
    """Mixed-precision apply (FP32 near panels, bases, transfers, coupling; FP64 CSR of B + M)
    against the FP64 path on the same workload, and FP64 CG versus mixed CG with iterative
    refinement on the load vector of f = 1."""
    import numpy as np
    import torch
    import paper_2302_02863_amd as fp
    o = dict(P.opts)
    o["precision"] = "mixed"
    opm = fp.Operator(P.mesh, P.s, P.kappa, o)
    ym = torch.empty_like(x)
    el_m = time_applies(opm, x, ym, stream, steps, warmup)
    err = float(torch.linalg.vector_norm(ym - y64) / torch.linalg.vector_norm(y64))
    out = {"value": P.mesh.n_dofs * x.shape[0] * x.shape[2] * steps / el_m,
           "ms_per_step": el_m / steps * 1e3, "max_rel_err_vs_fp64": err}
    # solves: A u = F, F the load vector of f = 1 (computed by the library)
    F = op64.load_vector(torch.ones(P.mesh.n_nodes, dtype=torch.float64, device=x.device)).reshape(1, -1, 1)
    F = F.expand(x.shape[0], -1, -1).contiguous()
    res = {}
    for name, op in (("fp64", op64), ("mixed", opm)):
        op.solve(F, rtol=1e-10, maxit=20000)        # warm-up (captures the CG graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = op.solve(F, rtol=1e-10, maxit=20000)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0, u, info)
    uerr = float(torch.linalg.vector_norm(res["mixed"][1] - res["fp64"][1]) / torch.linalg.vector_norm(res["fp64"][1]))
    out["solve"] = {"rtol": 1e-10, "fp64_ms": res["fp64"][0] * 1e3, "mixed_ms": res["mixed"][0] * 1e3,
                    "fp64_iterations": res["fp64"][2]["iterations"],
                    "mixed_iterations": res["mixed"][2]["iterations"],
                    "mixed_refinements": res["mixed"][2]["refinements"],
                    "speedup": res["fp64"][0] / res["mixed"][0],
                    "mixed_vs_fp64_solution_rel_diff": uerr}
    opm.close()
    return out


def near_entries(op, st):
    leafptr = op.export("K_LEAFPTR")
    sizes = leafptr[1:] - leafptr[:-1]
    pairs = op.export("K_NEAR").reshape(-1, 2)
    first = (1 << (int(st["k_levels"]) - 1)) - 1
    return int((sizes[pairs[:, 0] - first] * sizes[pairs[:, 1] - first]).sum())


def batched(steps, warmup):
    """The batched workload: 256 x 256 squares (65025 dofs), 16 order fields x 64
    right-hand sides (FP32 vectors), FP64 operator against the mixed-precision one.
    The near-panel GEMM (k_near_mm) is MFMA-bound: 2 * entries * F * R flops."""
    import torch
    import paper_2302_02863_amd as fp
    from fpde_inputs import configs
    P = configs.batched(256, n_fields=16, nrhs=64)
    F, N, R = P.x.shape
    x = torch.tensor(P.x, device="cuda:0", dtype=torch.float32)
    out = {"workload": "square-256x256-P1 batched (65025 dofs), 16 order fields x 64 rhs, FP32 vectors"}
    ys = {}
    for prec, peak in (("fp64", 78.6), ("mixed", 157.3)):
        o = dict(P.opts)
        o["precision"] = prec
        t0 = time.perf_counter()
        op = fp.Operator(P.mesh, P.s, P.kappa, o)
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        y = torch.empty_like(x)
        el = time_applies(op, x, y, torch.cuda.current_stream(), steps, warmup)
        op.profile(True)
        for _ in range(3):
            op.apply(x, y)
        torch.cuda.synchronize()
        pr = op.profile(False)
        near_ms = pr["ms_out"] / pr["n_applies"]
        flops = 2.0 * near_entries(op, op.stats()) * F * R
        tf = flops / (near_ms * 1e-3) / 1e12
        out[prec] = {"value": N * F * R * steps / el, "ms_per_step": el / steps * 1e3, "build_s": build,
                     "near_mfma": {"kernel": "k_near_mm<%s>" % ("double" if prec == "fp64" else "float"),
                                   "avg_ms": near_ms, "tflops": tf, "peak_tflops": peak, "frac": tf / peak},
                     "phases_ms_per_apply": {k: pr[k] / pr["n_applies"] for k in ("ms_far", "ms_out", "ms_far_out",
                                                                                  "ms_total")}}
        ys[prec] = y.double()
        op.close()
    out["mixed_speedup"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    out["mixed_max_rel_err_vs_fp64"] = float((ys["mixed"] - ys["fp64"]).norm() / ys["fp64"].norm())
    return out


def scaling(steps, warmup, sizes=(32, 64, 128, 256)):
    """Build time and one-vector FP64 apply time of the square workload (same recipe:
    jitter, order and diffusivity fields) for growing n: linear scaling in N."""
    import torch
    import paper_2302_02863_amd as fp
    from fpde_inputs import configs
    out = []
    for n in sizes:
        P = configs.square(n)
        t0 = time.perf_counter()
        op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        st = op.stats()
        x = torch.tensor(P.x, device="cuda:0")
        y = torch.empty_like(x)
        el = time_applies(op, x, y, torch.cuda.current_stream(), steps, warmup)
        N = P.mesh.n_dofs
        out.append({"n": n, "n_dofs": N, "build_s": build_s,
                    "build_phase_ms": {k: st[k] for k in ("t_plan_ms", "t_singular_ms", "t_rho_ms", "t_mass_ms",
                                                          "t_bases_ms", "t_near_blocks_ms")},
                    "apply_us": el / steps * 1e6, "dof_matvecs_per_s": N * steps / el})
        op.close()
        del x, y
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="square")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision apply and the solves")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-field x 64-rhs batched workload")
    ap.add_argument("--no-scaling", action="store_true", help="skip the build and apply times of square 32..256")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 256 MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": a.numel() * 8,
                          "launches": args.steps}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(1)

    import numpy as np
    import torch
    import paper_2302_02863_amd as fp

    P, cfg = workload(args.workload)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    st = op.stats()
    F, N, R = P.x.shape
    x = torch.tensor(P.x, device=dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    el = time_applies(op, x, y, stream, args.steps, args.warmup)
    # same launches without the graph, HIP events on the apply stream between the phases
    op.profile(True)
    for _ in range(args.steps):
        op.apply(x, y, stream=stream)
    torch.cuda.synchronize()
    prof = op.profile(False)
    value = N * F * R * args.steps / el
    out_ms = prof["ms_out"] / max(1, prof["n_applies"])
    b_out, near_entries = algorithmic_bytes_near(op, st, F, R, P.mesh.dim, int(P.opts.get("cheb_p", 5)))
    achieved = b_out / (out_ms * 1e-3) / 1e9
    kname = "k_near_up"
    res = {
        "metric": "DOF-matvecs/s of stiffness apply at 1e-6 rel err; mixed vs FP64 path speedup",
        "value": value,
        "unit": "DOF-matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname),
                     "kernel": kname + " (B+M rows, dense near leaf blocks, far-field upsweep)",
                     "bytes_per_launch": b_out, "avg_ms": out_ms},
        "phases_ms_per_apply": {k: prof[k] / max(1, prof["n_applies"]) for k in ("ms_far", "ms_out", "ms_far_out",
                                                                               "ms_total")},
        "build_s": build_s,
        "build_phase_ms": {k: st[k] for k in ("t_plan_ms", "t_singular_ms", "t_rho_ms", "t_mass_ms", "t_bases_ms",
                                              "t_near_blocks_ms")},
        "counts": {k: st[k] for k in ("n_dofs", "csr_nnz", "k_near", "k_far", "k_leaves", "rho_near", "rho_far")},
    }
    if not args.no_mixed:
        mx = mixed_and_solve(P, op, x, y, stream, args.steps, args.warmup)
        mx["speedup_vs_fp64"] = mx["value"] / value
        res["mixed"] = mx
    if not args.no_batched:
        res["batched"] = batched(max(5, args.steps // 20), 3)
    if not args.no_scaling:
        res["scaling_in_n"] = scaling(max(20, args.steps // 4), 5)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(P)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
