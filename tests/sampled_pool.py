"""Sampled oracle rows of a full-size workload, spread over CPU worker processes (spawned
fresh: the workers import only numpy, the inputs and the oracle, never the GPU)."""
import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np

_cache = {}


def _worker(recipe, kwargs, field, rows, vecs):
    from fpde_inputs import configs
    from oracle.sampled import SampledOracle
    key = (recipe, tuple(sorted(kwargs.items())), field)
    if key not in _cache:
        P = getattr(configs, recipe)(**kwargs)
        _cache[key] = (P, SampledOracle(P.mesh, P.s[field], P.kappa[field], P.opts))
    P, so = _cache[key]
    out = []
    for v in vecs:
        x = P.x[field, :, v]
        r = so.row_apply(rows, x)
        out.append({k: r[k] for k in ("B", "K", "M", "total")})
    return rows, out


def sampled_rows(recipe, kwargs, field, rows, vecs=(0,), workers=None):
    """{part: array [len(vecs)][len(rows)]} of (A_h x_v) at the given rows, for the
    right-hand sides vecs of field `field` of configs.<recipe>(**kwargs)."""
    if workers is None:
        workers = max(1, min(8, (os.cpu_count() or 2) // 2, len(rows)))
    chunks = [list(c) for c in np.array_split(np.asarray(rows), workers) if len(c)]
    ctx = mp.get_context("spawn")
    res = {}
    with cf.ProcessPoolExecutor(max_workers=len(chunks), mp_context=ctx) as ex:
        futs = [ex.submit(_worker, recipe, kwargs, field, [int(i) for i in c], list(vecs)) for c in chunks]
        for fu in cf.as_completed(futs):
            rs, out = fu.result()
            for j, r in enumerate(rs):
                res[r] = {k: np.array([o[k][j] for o in out]) for k in ("B", "K", "M", "total")}
    return {k: np.stack([res[int(r)][k] for r in rows], axis=1) for k in ("B", "K", "M", "total")}
