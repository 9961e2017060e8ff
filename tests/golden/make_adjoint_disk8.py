"""Write tests/golden/adjoint_disk8_F2.txt: the oracle's gradient of
sum_r w_r^T A_h(s, kappa) u_r over every mesh node, for both fields of
``configs.adjoint_disk(8)`` (complex-step derivatives of the dense
H2-consistent assembly, ``oracle.adjoint.gradient``).

Calls only ``oracle/`` and the seeded input recipes.  About 10 CPU-minutes,
spread over the host cores:  python tests/golden/make_adjoint_disk8.py
"""
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from fpde_inputs import configs  # noqa: E402
from oracle.adjoint import directional  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_disk8_F2.txt")


def _one(task):
    f, j = task
    np.seterr(divide="ignore", invalid="ignore")
    P = configs.adjoint_disk(8)
    e = np.zeros(P.mesh.n_nodes)
    e[j] = 1.0
    w, u = P.extra["w"][f], P.x[f]
    gs = directional(P.mesh, P.s[f], P.kappa[f], P.opts, w, u, ds=e)
    gk = directional(P.mesh, P.s[f], P.kappa[f], P.opts, w, u, dk=e)
    return f, j, gs, gk


def main():
    P = configs.adjoint_disk(8)
    tasks = [(f, j) for f in range(2) for j in range(P.mesh.n_nodes)]
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(_one, tasks, chunksize=4)
    with open(OUT, "w") as fh:
        fh.write("# oracle gradient of sum_r w_r^T A_h u_r, configs.adjoint_disk(8); columns: field node d/ds d/dkappa\n")
        for f, j, gs, gk in sorted(res):
            fh.write(f"{f} {j} {gs:.17e} {gk:.17e}\n")


if __name__ == "__main__":
    main()
