"""CPU checks of bench.py's command-line contract (no GPU needed): more than one GPU
is refused with a JSON message and a non-zero exit; the algorithmic byte count of the
one-vector near kernel and the algorithmic MFMA flop count of the several-right-hand-side
near kernel (the headline's dominant kernel) follow their stated formulas."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = [ln for ln in r.stdout.splitlines() if ln.strip()][-1]
    msg = json.loads(line)
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_algorithmic_bytes_formula():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench

    class FakeOp:   # two leaves of 3 and 2 points, near pairs (0,0), (0,1), (1,1)
        def export(self, what):
            if what == "K_LEAFPTR":
                return np.array([0, 3, 5])
            if what == "K_NEAR":
                return np.array([1, 1, 1, 2, 2, 2])
            raise KeyError(what)

    st = {"k_levels": 2, "n_dofs": 5, "csr_nnz": 13, "k_rank": 4, "k_clusters": 3}   # leaves are heap ids 1, 2
    b, near = bench.algorithmic_bytes_near(FakeOp(), st, 1, 1, 2, 2)
    assert near == 3 * 3 + 3 * 2 + 2 * 2
    expect = near * 8 + 13 * (8 + 4) + 6 * 8 + 2 * 5 * 8 + 5 * 4 * 8 + 3 * 2 * 2 * 2 * 8 + 3 * 4 * 8
    assert b == expect


def test_algorithmic_flops_formula():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench

    class FakeOp:   # leaves of 3 and 2 points, near pairs (0,0), (0,1), (1,0), (1,1)
        def export(self, what):
            if what == "K_LEAFPTR":
                return np.array([0, 3, 5])
            if what == "K_NEAR":
                return np.array([1, 1, 1, 2, 2, 1, 2, 2])
            raise KeyError(what)

    st = {"k_levels": 2, "n_dofs": 5, "k_rank": 4}
    F, R = 3, 7
    fl, ne = bench.algorithmic_flops_near_mm(FakeOp(), st, F, R)
    assert ne == 9 + 6 + 6 + 4
    assert fl == 2.0 * ne * F * R + 2.0 * 5 * 4 * F * R


def test_oracle_only_in_cpu_baseline():
    """bench.py may run the oracle only in its CPU-baseline leg."""
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    for fn in ast.walk(tree):
        if not isinstance(fn, ast.FunctionDef):
            continue
        for node in ast.walk(fn):
            mods = []
            if isinstance(node, ast.ImportFrom):
                mods = [node.module or ""]
            elif isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            if any(m == "oracle" or m.startswith("oracle.") for m in mods):
                assert fn.name == "cpu_baseline", (fn.name, mods)


def test_bench_l2_norm_matches_oracle():
    import numpy as np
    import bench
    from fpde_inputs import configs
    from oracle.solve import l2_norm
    for P in (configs.bump(3), configs.interval(n_int=16, n_ext=4)):
        u = np.random.default_rng(0).standard_normal(P.mesh.n_dofs)
        assert abs(bench.p1_l2_norm(P.mesh, u) - l2_norm(P.mesh, u)) < 1e-13 * l2_norm(P.mesh, u)


def test_profile_commands_use_existing_bench_flags():
    """Every bench.py command quoted in profiles/ (the rocprofv3 summaries and counter
    records) names only flags bench.py accepts, so each record can be re-run as written."""
    import re
    src = open(os.path.join(ROOT, "bench.py")).read()
    known = set(re.findall(r'add_argument\("(--[a-z0-9-]+)"', src))
    assert "--steps" in known and "--build-adjoint" in known
    pdir = os.path.join(ROOT, "profiles")
    seen = 0
    for name in sorted(os.listdir(pdir)):
        text = open(os.path.join(pdir, name)).read().replace("\\\n", " ")
        for m in re.finditer(r"bench\.py((?:\s+--[a-z0-9-]+(?:\s+[0-9]+)?)*)", text):
            flags = re.findall(r"--[a-z0-9-]+", m.group(1))
            seen += 1
            assert set(flags) <= known, (name, sorted(set(flags) - known))
    assert seen >= 4
