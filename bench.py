"""Benchmark of the stiffness-operator apply on one MI355X.

One step = one application Y = A X of the whole decomposed operator
(A = B + M + K~: rows of B + M, dense near leaf blocks, H2 far field) to every
right-hand side of every order field of the workload, inputs resident in HBM.

Headline workload: the 2D unit square with 256 x 256 cells split in two
(65025 dofs, 524288 cells including the exterior band), 16 order fields
s_k = 0.5 + 0.3 sin(k pi x1) cos(pi x2), 64 right-hand sides each (FP32
vectors), leaf 64, 5 Chebyshev points per dimension, eta = 1, applied by the
mixed-precision operator (FP32 near panels, bases, transfers and coupling on
FP32 MFMA; FP64 rows of B + M and FP64 accumulation of each output).

Metric: DOF-matvecs/s = N * F * R * steps / elapsed of the mixed apply, which
counts only when its relative error against the FP64 apply (max over the
1024 vectors of ||y - y64|| / ||y64||) is within 1e-6; the FP64 path's time on
the same vectors gives the speedup.

Prints one JSON line with a roofline entry for the dominant kernel
(k_near_mm<float>, the near-panel GEMM on MFMA, timed with HIP events on the
apply stream), a CPU baseline of the oracle, and extras: the one-vector
square-128 apply, the disk solve (mixed CG with refinement against FP64 CG),
the batched solve, adjoint timings, the variable-order bump problem's
self-convergence and build/apply times for growing N.
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
FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6
MIXED_TOL = 1e-6
METRIC = "DOF-matvecs/s of stiffness apply at 1e-6 rel err; mixed vs FP64 path speedup"


# ---------------------------------------------------------------------------- helpers

def near_entries(op, st):
    """Sum over the near leaf pairs of |sigma| |sigma'| (entries of the dense near blocks)."""
    leafptr = op.export("K_LEAFPTR")
    sizes = leafptr[1:] - leafptr[:-1]
    pairs = op.export("K_NEAR").reshape(-1, 2)
    first = (1 << (int(st["k_levels"]) - 1)) - 1
    return int((sizes[pairs[:, 0] - first] * sizes[pairs[:, 1] - first]).sum())


def algorithmic_bytes_near(op, st, F, R, dim, p):
    """HBM bytes one launch of the one-vector near/upsweep kernel must move, no re-reads
    counted: the near leaf blocks (sum over near pairs of |s| |s'| FP64 entries), the
    nonzeros of B + M (FP64 values, int32 columns) and one 8-byte index per row, x read
    once, y written once, the leaf bases U (N x k FP64) and the transfers (D P^2 per
    cluster) read once, the cluster coefficients (k per cluster) written once.  The
    kernel reads B + M in an ELL form by leaf slot; its padding is not counted."""
    ne = near_entries(op, st)
    N = st["n_dofs"]
    nnz = st["csr_nnz"]
    b = F * ne * 8
    b += F * nnz * 8 + nnz * 4 + (N + 1) * 8
    b += 2 * F * N * R * 8
    k, ncl = int(st["k_rank"]), int(st["k_clusters"])
    b += N * k * 8 + ncl * dim * p * p * 8 + F * ncl * k * 8
    return b, ne


def algorithmic_flops_near_mm(op, st, F, R):
    """MFMA flops of one launch of the several-right-hand-side near kernel: the dense near
    panels times the gathered rows of X (2 x near entries x F x R) plus the far field's
    leaf output U Y^ (2 x N x k x F x R).  The FP64 rows of B + M (2 x nnz x F x R vector
    flops) run on the vector units and are not counted against the MFMA peak."""
    ne = near_entries(op, st)
    N, k = int(st["n_dofs"]), int(st["k_rank"])
    return 2.0 * ne * F * R + 2.0 * N * k * F * R, ne


def committed_record(name, sources):
    """A committed rocprofv3 record under profiles/, valid only while the listed kernel
    sources are unchanged (their sha256 is stored in the record); else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    try:
        rec = json.load(open(path))
        for src in sources:
            sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2302_02863_amd", "csrc", src), "rb").read()).hexdigest()
            if rec.get("source_sha256", {}).get(src) != sha:
                return None
    except (OSError, ValueError, AttributeError):
        return None
    return rec


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


def profiled(op, x, y, n=10):
    """Per-apply device times from HIP events on the apply stream (fpde_profile)."""
    import torch
    op.profile(True)
    for _ in range(n):
        op.apply(x, y)
    torch.cuda.synchronize()
    pr = op.profile(False)
    return {k: pr[k] / pr["n_applies"] for k in ("ms_far", "ms_out", "ms_far_out", "ms_total")}


def per_vector_rel_err(y, yref):
    """max over (field, rhs) of ||y - yref||_2 / ||yref||_2 (vectors along N)."""
    import torch
    d = torch.linalg.vector_norm((y.double() - yref.double()), dim=1)
    r = torch.linalg.vector_norm(yref.double(), dim=1)
    return float((d / r).max())


# ---------------------------------------------------------------------------- headline

def headline(steps, warmup):
    """Batched square 256: 16 order fields x 64 right-hand sides, mixed against FP64."""
    import torch
    import paper_2302_02863_amd as fp
    from fpde_inputs import configs
    P = configs.batched(256, n_fields=16, nrhs=64)
    F, N, R = P.x.shape
    x = torch.tensor(P.x, device="cuda:0", dtype=torch.float32)
    stream = torch.cuda.current_stream()
    out = {}
    ops, ys = {}, {}
    for prec in ("mixed", "fp64"):
        o = dict(P.opts)
        o["precision"] = prec
        o["jacobi"] = True   # only fpde_solve reads it (the batched solve extra); the apply is unchanged
        t0 = time.perf_counter()
        op = fp.Operator(P.mesh, P.s, P.kappa, o)
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        y = torch.empty_like(x)
        el = time_applies(op, x, y, stream, steps, warmup)
        ph = profiled(op, x, y)
        st = op.stats()
        flops, ne = algorithmic_flops_near_mm(op, st, F, R)
        kname = "k_near_mm<%s>" % ("float" if prec == "mixed" else "double")
        peak = FP32_MFMA_PEAK_TFLOPS if prec == "mixed" else FP64_MFMA_PEAK_TFLOPS
        tf = flops / (ph["ms_out"] * 1e-3) / 1e12
        out[prec] = {"value": N * F * R * steps / el, "ms_per_step": el / steps * 1e3, "build_s": build,
                     "phases_ms_per_apply": {"far_chain": ph["ms_far"], "near_kernel": ph["ms_out"],
                                             "total": ph["ms_total"]},
                     "near_kernel": {"kernel": kname, "avg_ms": ph["ms_out"], "flops_per_launch": flops,
                                     "tflops": tf, "peak_tflops": peak, "frac": tf / peak},
                     "build_phase_ms": {k: st[k] for k in ("t_plan_ms", "t_singular_ms", "t_rho_ms", "t_mass_ms",
                                                           "t_bases_ms", "t_near_blocks_ms")}}
        ops[prec] = op
        ys[prec] = y
    out["near_entries_per_field"] = ne
    out["counts"] = {k: st[k] for k in ("n_dofs", "csr_nnz", "k_near", "k_far", "k_leaves", "k_rank")}
    out["max_rel_err_vs_fp64"] = per_vector_rel_err(ys["mixed"], ys["fp64"])
    out["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    # the far field's own share of the mixed error (fpde_apply_parts with the far blocks only)
    yk = ops["mixed"].apply(x, parts=fp.PART_KFAR)
    yk64 = ops["mixed"].apply(x, parts=fp.PART_KFAR | fp.PART_FP64)
    ynear = ops["mixed"].apply(x, parts=fp.PART_KNEAR)
    ynear64 = ops["mixed"].apply(x, parts=fp.PART_KNEAR | fp.PART_FP64)
    nb = fp.PART_KNEAR | fp.PART_B | fp.PART_M   # with several rhs, B + M ride in the FP32 panels
    ynb = ops["mixed"].apply(x, parts=nb)
    ynb64 = ops["mixed"].apply(x, parts=nb | fp.PART_FP64)
    torch.cuda.synchronize()
    yref = ys["fp64"].double()
    yn = torch.linalg.vector_norm(yref, dim=1)
    out["error_budget"] = {
        "far_part_err_over_y": float((torch.linalg.vector_norm(yk.double() - yk64.double(), dim=1) / yn).max()),
        "near_panel_err_over_y": float((torch.linalg.vector_norm(ynear.double() - ynear64.double(), dim=1)
                                        / yn).max()),
        "far_part_norm_over_y": float((torch.linalg.vector_norm(yk64.double(), dim=1) / yn).max()),
        "near_panel_norm_over_y": float((torch.linalg.vector_norm(ynear64.double(), dim=1) / yn).max()),
        "near_panels_with_b_m_err_over_y": float((torch.linalg.vector_norm(ynb.double() - ynb64.double(), dim=1)
                                                  / yn).max())}
    out["_y_fp64"] = ys["fp64"]
    return P, x, ops, out


# ---------------------------------------------------------------------------- extras

def square128(steps, warmup):
    """One vector on the jittered square 128 (16129 dofs): FP64 and mixed, with the HBM
    roofline of the fused near/upsweep kernel k_near_up<2,5,double>."""
    import torch
    import paper_2302_02863_amd as fp
    from fpde_inputs import configs
    P = configs.square(128)
    F, N, R = P.x.shape
    x = torch.tensor(P.x, device="cuda:0")
    t0 = time.perf_counter()
    op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    st = op.stats()
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    el = time_applies(op, x, y, stream, steps, warmup)
    ph = profiled(op, x, y, n=steps)
    b, _ = algorithmic_bytes_near(op, st, F, R, P.mesh.dim, int(P.opts["cheb_p"]))
    ach = b / (ph["ms_out"] * 1e-3) / 1e9
    rec = committed_record("traffic_k_near_up_square128.json", ["fpde_apply.hip"])
    out = {"workload": "square-128x128-P1 (16129 dofs, 131072 cells), variable s and kappa, 1 rhs",
           "fp64": {"value": N * steps / el, "ms_per_step": el / steps * 1e3},
           "roofline": {"bound": "hbm", "kernel": "k_near_up<2,5,double>", "achieved": ach, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "bytes_per_launch": b, "avg_ms": ph["ms_out"],
                        "traffic": rec["traffic_bytes_per_launch"] if rec else None},
           "phases_ms_per_apply": ph, "build_s": build_s,
           "build_phase_ms": {k: st[k] for k in ("t_plan_ms", "t_singular_ms", "t_rho_ms", "t_mass_ms", "t_bases_ms",
                                                 "t_near_blocks_ms")}}
    o = dict(P.opts)
    o["precision"] = "mixed"
    opm = fp.Operator(P.mesh, P.s, P.kappa, o)
    ym = torch.empty_like(x)
    el_m = time_applies(opm, x, ym, stream, steps, warmup)
    out["mixed"] = {"value": N * steps / el_m, "ms_per_step": el_m / steps * 1e3,
                    "max_rel_err_vs_fp64": per_vector_rel_err(ym, y), "speedup_vs_fp64": el / el_m}
    # one-vector solve of the load vector of f = 1, plain and Jacobi-preconditioned CG
    Fv = op.load_vector(torch.ones(P.mesh.n_nodes, dtype=torch.float64, device=x.device)).reshape(1, -1, 1)
    out["solve"] = solve_pair(op, opm, Fv, rtol=1e-10)
    oj = dict(P.opts)
    oj["jacobi"] = True
    opj = fp.Operator(P.mesh, P.s, P.kappa, oj)
    oj["precision"] = "mixed"
    opjm = fp.Operator(P.mesh, P.s, P.kappa, oj)
    out["solve_jacobi"] = solve_pair(opj, opjm, Fv, rtol=1e-10)
    opj.close()
    opjm.close()
    # adjoint: gradient of w^T A u in every nodal s and kappa
    out["adjoint_ms"] = time_adjoint(op, x, x)
    opm.close()
    op.close()
    return out


def solve_pair(op64, opm, Fv, rtol, maxit=50000, ref_rtol=None):
    """FP64 CG against mixed CG with refinement on the FP64 residual, same rtol; the
    solution error of each against a reference solve (FP64 CG to ref_rtol) if given."""
    import torch
    res = {}
    uref = None
    if ref_rtol is not None:
        uref, rinfo = op64.solve(Fv, rtol=ref_rtol, maxit=maxit, raise_on_noconv=False)
        res["reference"] = {"rtol": ref_rtol, "rel_residual": rinfo["rel_residual"],
                            "iterations": rinfo["iterations"]}
    for name, op in (("fp64", op64), ("mixed", opm)):
        op.solve(Fv, rtol=rtol, maxit=maxit)        # warm-up (workspaces allocated on first use)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = op.solve(Fv, rtol=rtol, maxit=maxit)
        torch.cuda.synchronize()
        res[name] = {"ms": (time.perf_counter() - t0) * 1e3, "iterations": info["iterations"],
                     "refinements": info["refinements"], "rel_residual": info["rel_residual"],
                     "cond_estimate": info["cond_estimate"]}
        if uref is not None:
            res[name]["solution_rel_err"] = per_vector_rel_err(u, uref)
        res[name]["_u"] = u
    res["mixed_vs_fp64_solution_rel_diff"] = per_vector_rel_err(res["mixed"].pop("_u"), res["fp64"].pop("_u"))
    res["rtol"] = rtol
    res["speedup"] = res["fp64"]["ms"] / res["mixed"]["ms"]
    return res


def time_adjoint(op, w, u, n=3):
    import torch
    op.apply_adjoint(w, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        op.apply_adjoint(w, u)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / n * 1e3


def disk_solve():
    """The disk workload (elliptical 512 x 512 grid, 261121 dofs, tanh order profile,
    exterior beyond R = 1.1): FP64 CG against mixed CG with refinement, both stopped at
    rtol 1e-10, and their solution errors against a reference FP64 solve to rtol 1e-12."""
    import torch
    import paper_2302_02863_amd as fp
    from fpde_inputs import configs
    P = configs.disk(512)
    t0 = time.perf_counter()
    op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    o = dict(P.opts)
    o["precision"] = "mixed"
    opm = fp.Operator(P.mesh, P.s, P.kappa, o)
    x = torch.tensor(P.x, device="cuda:0")
    y = torch.empty_like(x)
    ym = torch.empty_like(x)
    el = time_applies(op, x, y, torch.cuda.current_stream(), 50, 5)
    el_m = time_applies(opm, x, ym, torch.cuda.current_stream(), 50, 5)
    Fv = op.load_vector(torch.ones(P.mesh.n_nodes, dtype=torch.float64, device=x.device)).reshape(1, -1, 1)
    out = {"workload": "disk-512 (261121 dofs), tanh order profile, exterior beyond R=1.1, f=1",
           "build_s": build_s, "apply_ms": {"fp64": el / 50 * 1e3, "mixed": el_m / 50 * 1e3},
           "apply_mixed_rel_err_vs_fp64": per_vector_rel_err(ym, y),
           "solve": solve_pair(op, opm, Fv, rtol=1e-10, ref_rtol=1e-12)}
    opm.close()
    op.close()
    oj = dict(P.opts)
    oj["jacobi"] = True
    opj = fp.Operator(P.mesh, P.s, P.kappa, oj)
    oj["precision"] = "mixed"
    opjm = fp.Operator(P.mesh, P.s, P.kappa, oj)
    out["solve_jacobi"] = solve_pair(opj, opjm, Fv, rtol=1e-10, ref_rtol=1e-12)
    opj.close()
    opjm.close()
    return out


def recompression(P, x, y64, tols=(1e-2, 1e-3, 1e-4)):
    """The headline workload's mixed apply with the far field's bases recompressed
    algebraically (closing remark of Sec. 5.3) at several tolerances: cluster ranks,
    far-chain and apply times, build cost and the error against the FP64 apply."""
    import torch
    import paper_2302_02863_amd as fp
    out = []
    for tol in tols:
        o = dict(P.opts)
        o["precision"] = "mixed"
        o["recompress_tol"] = tol
        op = fp.Operator(P.mesh, P.s, P.kappa, o)
        y = torch.empty_like(x)
        for _ in range(3):
            op.apply(x, y)
        ph = profiled(op, x, y)
        st = op.stats()
        out.append({"tol": tol, "rank": st["k_rank_rc"], "rank_mean": st["k_rank_rc_mean"],
                    "chebyshev_rank": st["k_rank"], "build_ms": st["t_recompress_ms"],
                    "far_chain_ms": ph["ms_far"], "apply_ms": ph["ms_total"],
                    "max_rel_err_vs_fp64": per_vector_rel_err(y, y64)})
        op.close()
    return out


def batched_solve_and_adjoint(P, x, ops):
    """The headline workload's 1024 systems A_f u = b (b = the N(0,1) vectors in FP64),
    Jacobi-preconditioned FP64 CG against mixed CG with refinement to rtol 1e-8; adjoint with
    one vector per field."""
    import torch
    b = x.double().contiguous()
    out = {"solve": solve_pair(ops["fp64"], ops["mixed"], b, rtol=1e-8, maxit=100000)}
    out["adjoint_ms_16_fields_1_rhs"] = time_adjoint(ops["fp64"], b[:, :, :1].contiguous(),
                                                     b[:, :, 1:2].contiguous(), n=2)
    torch.cuda.synchronize()
    return out


def build_and_adjoint():
    """The headline workload's FP64 operator built once and its adjoint run once with one
    vector pair per field (a short run for a kernel trace of the build and the adjoint)."""
    import torch
    import paper_2302_02863_amd as fp
    from fpde_inputs import configs
    P = configs.batched(256, n_fields=16, nrhs=2)
    t0 = time.perf_counter()
    op = fp.Operator(P.mesh, P.s, P.kappa, dict(P.opts))
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    st = op.stats()
    x = torch.tensor(P.x, device="cuda:0")
    ms = time_adjoint(op, x[:, :, :1].contiguous(), x[:, :, 1:2].contiguous(), n=1)
    op.close()
    return {"workload": "square-256x256-P1, 16 order fields, FP64 operator; adjoint with 1 vector pair per field",
            "build_s": build,
            "build_phase_ms": {k: st[k] for k in ("t_plan_ms", "t_singular_ms", "t_rho_ms", "t_mass_ms",
                                                  "t_bases_ms", "t_near_blocks_ms")},
            "adjoint_ms": ms}


def p1_l2_norm(mesh, u_dofs):
    """L2(Omega_i) norm of the P1 function with dof values u (zero on the other nodes):
    per cell, vol (sum u_a^2 + (sum u_a)^2) / ((d+1)(d+2)) is the exact integral of u^2."""
    import numpy as np
    u = np.zeros(mesh.n_nodes)
    u[:mesh.n_dofs] = u_dofs
    X = mesh.coords[:, mesh.cells]                 # (d, d+1, nc)
    d = mesh.dim
    J = X[:, 1:, :] - X[:, :1, :]                  # (d, d, nc)
    det = np.abs(np.linalg.det(np.moveaxis(J, -1, 0))) if d > 1 else np.abs(J[0, 0])
    vol = det / (2.0 if d == 2 else 1.0)
    uc = u[mesh.cells]
    return float(np.sqrt((vol * ((uc ** 2).sum(axis=0) + uc.sum(axis=0) ** 2) / ((d + 1) * (d + 2))).sum()))


def bump_self_convergence(levels=(3, 4, 5, 6, 7)):
    """The paper's variable-order bump problem (Sec. 7.2): build and FP64 solve (rtol 1e-11)
    on the uniform grids T_j, and the self-convergence e_j = U_{j+1} - I U_j in L2(Omega_i)
    and at the nodes, with fitted rates."""
    import numpy as np
    import torch
    import paper_2302_02863_amd as fp
    from fpde_inputs import configs
    from fpde_inputs.meshes import grid_values, prolong_p1
    sols, rows = {}, []
    for j in levels:
        P = configs.bump(j)
        t0 = time.perf_counter()
        op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        F = op.load_vector(torch.tensor(P.f, device="cuda:0")).reshape(1, -1, 1)
        op.solve(F, rtol=1e-11, maxit=50000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = op.solve(F, rtol=1e-11, maxit=50000)
        torch.cuda.synchronize()
        solve_ms = (time.perf_counter() - t0) * 1e3
        sols[j] = (P.mesh, u.cpu().numpy()[0, :, 0])
        rows.append({"j": j, "n_dofs": P.mesh.n_dofs, "cells": P.mesh.n_cells, "build_s": build_s,
                     "solve_ms": solve_ms, "cg_iterations": info["iterations"]})
        op.close()
    errs = []
    for j in levels[:-1]:
        (mc, uc), (mf, uf) = sols[j], sols[j + 1]
        Gf = prolong_p1(grid_values(mc, uc)[0])
        _, idx = grid_values(mf, uf)
        d = uf - Gf[idx[0, :mf.n_dofs], idx[1, :mf.n_dofs]]
        errs.append({"j": j, "h": mc.info["h"], "l2": p1_l2_norm(mf, d), "linf": float(np.abs(d).max())})
    hs = np.log([e["h"] for e in errs])
    return {"workload": "variable-order bump, s* = 0.7, eta = 0.2, l = 1, x^c = (-0.4, 0.4), f = 20, "
                        "Omega = (-2,2)^2, Omega_i = (-1,1)^2", "levels": rows, "self_convergence": errs,
            "rate_l2": float(np.polyfit(hs, np.log([e["l2"] for e in errs]), 1)[0]),
            "rate_linf": float(np.polyfit(hs, np.log([e["linf"] for e in errs]), 1)[0])}


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


def measured_denominators():
    """Achieved rates of plain library work on this GPU, next to the datasheet peaks:
    a 1 GiB device-to-device copy (torch) and an 8192^3 FP32 GEMM (torch.mm)."""
    import torch
    a = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    n = 20
    t0 = time.perf_counter()
    for _ in range(n):
        b.copy_(a)
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 8 * n / (time.perf_counter() - t0) / 1e9
    del a, b
    m = 8192
    A = torch.randn(m, m, device="cuda:0")
    B = torch.randn(m, m, device="cuda:0")
    C = A @ B
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        C = A @ B
    torch.cuda.synchronize()
    gemm_tf = 2 * m ** 3 * 5 / (time.perf_counter() - t0) / 1e12
    return {"copy_GBps": copy_gbs, "fp32_gemm_TFLOPs": gemm_tf, "hbm_peak_GBps": HBM_PEAK_GBS,
            "fp32_mfma_peak_TFLOPs": FP32_MFMA_PEAK_TFLOPS, "fp64_mfma_peak_TFLOPs": FP64_MFMA_PEAK_TFLOPS}


# ---------------------------------------------------------------------------- CPU baseline

def _host_info():
    import numpy as np          # noqa: F401  (loads the BLAS threadpoolctl reports)
    import scipy.linalg         # noqa: F401
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = []
    try:
        import threadpoolctl
        blas = [{k: i.get(k) for k in ("internal_api", "version", "num_threads", "threading_layer")}
                for i in threadpoolctl.threadpool_info()]
    except Exception:
        pass
    return model, blas


def _median(f, n):
    ts = []
    for _ in range(n):
        t0 = time.perf_counter()
        f()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2]


def cpu_baseline(P, seconds: float = 15.0):
    """The FP64 oracle on the host cores.

    value: rows of A_h x of the headline workload (field 0, one right-hand side),
    computed one by one by the sampled-row oracle (oracle.sampled) for about
    ``seconds``; its cluster-tree/partition setup is excluded and reported.
    dense: the dense oracle (assembly, A @ X and Cholesky, median of 5) on the 1D
    workload at full size (511 dofs), and its A @ X and Cholesky at the square-128
    size (16129 dofs, 2.1 GB) on an SPD matrix of that size, whose dense assembly
    by the oracle does not fit a bounded run (O(N^2) kernel evaluations)."""
    import numpy as np
    from fpde_inputs import configs
    from oracle.assembly import assemble_exact, assemble_split, load_vector
    from oracle.h2 import assemble_h2
    from oracle.sampled import SampledOracle
    from oracle.solve import solve_dense
    np.seterr(divide="ignore", invalid="ignore")
    model, blas = _host_info()
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
    dense = {}
    C1 = configs.interval(n_int=512)
    m = C1.mesh
    dense["interval512"] = {
        "n_dofs": m.n_dofs,
        "assembly_exact_s": _median(lambda: assemble_exact(m, C1.s[0], C1.kappa[0], C1.opts, all_columns=False), 5),
        "assembly_h2_consistent_s": _median(lambda: assemble_h2(m, C1.s[0], C1.kappa[0], C1.opts), 5)}
    ref = assemble_h2(m, C1.s[0], C1.kappa[0], C1.opts, split=assemble_split(m, C1.s[0], C1.kappa[0], C1.opts))
    A = ref["B"] + ref["K"] + ref["M"]
    X = np.random.default_rng(12).standard_normal((m.n_dofs, 64))
    Fv = load_vector(m, C1.f, C1.opts)
    dense["interval512"]["apply_64rhs_s"] = _median(lambda: A @ X, 5)
    dense["interval512"]["cholesky_solve_s"] = _median(lambda: solve_dense(A, Fv), 5)
    n2 = 16129
    G = np.random.default_rng(13).standard_normal((n2, n2))
    G = G + G.T
    G[np.diag_indices(n2)] += 4.0 * np.sqrt(n2) + 10.0      # SPD by diagonal dominance of the spectrum
    X2 = np.random.default_rng(14).standard_normal((n2, 64))
    x1 = X2[:, 0].copy()
    dense["square128_size"] = {"n_dofs": n2, "apply_1rhs_s": _median(lambda: G @ x1, 5),
                               "apply_64rhs_s": _median(lambda: G @ X2, 5),
                               "cholesky_solve_s": _median(lambda: solve_dense(G, x1), 3),
                               "note": "SPD matrix of the square-128 size; timings of the oracle's A @ X and "
                                       "Cholesky routines, which do not depend on the entries"}
    del G
    return {"value": done / el, "unit": "DOF-matvecs/s", "cores": os.cpu_count() or 1, "kind": "oracle",
            "sample": f"{done} rows of A_h x (field 0, one right-hand side) of the headline workload computed "
                      f"entry by entry by the FP64 sampled-row oracle in {el:.1f} s (its tree/partition/basis "
                      f"setup, {t_setup:.1f} s, excluded)",
            "cpu_model": model, "blas": blas, "dense_oracle": dense}


# ---------------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--no-square", action="store_true")
    ap.add_argument("--no-disk", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the batched solve and adjoint")
    ap.add_argument("--no-scaling", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 256 MiB (calibrates HBM byte counters)")
    ap.add_argument("--build-adjoint", action="store_true",
                    help="run only one build of the headline FP64 operator and one adjoint (kernel traces)")
    ap.add_argument("--square128-only", action="store_true",
                    help="run only the one-vector square-128 extra (kernel traces)")
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
        print(json.dumps({"error": "this library runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(1)
    if args.build_adjoint:
        print(json.dumps(build_and_adjoint()))
        return
    if args.square128_only:
        print(json.dumps(square128(max(100, args.steps), 20)))
        return

    P, x, ops, hl = headline(args.steps, args.warmup)
    ys_fp64 = hl.pop("_y_fp64")
    print("[bench] headline done", file=sys.stderr, flush=True)
    F, N, R = P.x.shape
    mixed = hl["mixed"]
    kn = mixed["near_kernel"]
    rec = committed_record("traffic_k_near_mm_float_batched256.json", ["fpde_near.hip"])
    res = {
        "metric": METRIC,
        "value": mixed["value"] if hl["max_rel_err_vs_fp64"] <= MIXED_TOL else 0.0,
        "unit": "DOF-matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "square-256x256-P1 batched: 65025 dofs, 16 order fields x 64 rhs (FP32 vectors), "
                               "mixed-precision operator",
                   "n": 256, "fields": F, "nrhs": R, "leaf": 64, "cheb_p": 5, "eta": 1.0, "precision": "mixed"},
        "roofline": {"bound": "mfma", "kernel": kn["kernel"] + " (near-panel GEMM + far leaf output on FP32 MFMA, "
                                                             "FP64 rows of B + M)",
                     "achieved": kn["tflops"], "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": kn["tflops"] / FP32_MFMA_PEAK_TFLOPS, "flops_per_launch": kn["flops_per_launch"],
                     "avg_ms": kn["avg_ms"], "traffic": rec["traffic_bytes_per_launch"] if rec else None},
        "max_rel_err_vs_fp64": hl["max_rel_err_vs_fp64"],
        "speedup_vs_fp64": hl["speedup_vs_fp64"],
        "headline": hl,
    }
    extras = {}

    def extra(name, fn, *a):
        # an extra that fails is reported, not fatal: the headline line still prints
        try:
            extras[name] = fn(*a)
        except Exception as exc:      # noqa: BLE001
            extras[name] = {"error": f"{type(exc).__name__}: {exc}"}
        print(f"[bench] {name} done", file=sys.stderr, flush=True)

    if not args.no_extras:
        extra("recompression", recompression, P, x, ys_fp64)
    if not args.no_extras and not args.no_solve:
        extra("batched_solve_adjoint", batched_solve_and_adjoint, P, x, ops)
    for op in ops.values():
        op.close()
    del ops, x
    if not args.no_extras:
        extra("measured_denominators", measured_denominators)
        if not args.no_square:
            extra("square128", square128, max(100, args.steps), 20)
        if not args.no_disk:
            extra("disk512", disk_solve)
        extra("bump", bump_self_convergence)
        if not args.no_scaling:
            extra("scaling_in_n", scaling, 50, 5)
    res["extras"] = extras
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(P)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
