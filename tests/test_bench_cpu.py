"""bench.py on the CPU: every module-level helper that main() calls exists (a
missing one would only surface on the GPU machine, mid-run), the host-side
helpers compute what they state, and a request for more than one GPU exits
with a message before any device work."""
import ast
import builtins
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_main_calls_only_defined_names():
    src = open(os.path.join(ROOT, "bench.py")).read()
    tree = ast.parse(src)
    defined = {n.name for n in tree.body if isinstance(n, (ast.FunctionDef, ast.ClassDef))}
    imported = set()
    for n in ast.walk(tree):
        if isinstance(n, ast.Import):
            imported |= {(a.asname or a.name).split(".")[0] for a in n.names}
        elif isinstance(n, ast.ImportFrom):
            imported |= {a.asname or a.name for a in n.names}
    main = next(n for n in tree.body if isinstance(n, ast.FunctionDef) and n.name == "main")
    local = {a.arg for a in main.args.args}
    for n in ast.walk(main):
        if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Store):
            local.add(n.id)
        elif isinstance(n, (ast.FunctionDef, ast.Lambda)) and n is not main:
            if isinstance(n, ast.FunctionDef):
                local.add(n.name)
            local |= {a.arg for a in n.args.args}
    called = {n.func.id for n in ast.walk(main) if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    missing = sorted(c for c in called
                     if c not in defined and c not in imported and c not in local and not hasattr(builtins, c))
    assert not missing, missing


def test_host_helpers():
    sys.path.insert(0, ROOT)
    import bench
    from oracle import schedule as OS
    assert bench.algo_flops([(4096, 14336)], 5) == 5 * (3.0 * 4096 ** 2 * 14336 + 4096.0 ** 3)
    assert bench.update_flops([(100, 300), (300, 100)]) == 2 * 2.0 * 100 ** 2 * 300
    abc = OS.greedy_schedule(1e-3, 5).abc
    r = np.random.Generator(np.random.PCG64(3))
    mats = [r.standard_normal((40, 90)), r.standard_normal((90, 40))]
    rec, ref = bench.cpu_baseline(mats, abc, 5)
    assert rec["kind"] == "oracle" and rec["cores"] >= 1 and rec["value"] > 0 and ref.shape == (90, 40)
    assert rec["sample"].startswith("2 of the workload's matrices (40x90, 90x40)")
    # the Appendix C prediction of an orthogonal input's error: |1 - phi(1/1.01)|
    sig = np.ones(16)
    x = 1.0 / (1.01 * 4.0 + 1e-7)
    y = x
    for a, b, c in abc:
        y = y * (a + y * y * (b + c * y * y))
    assert abs(bench.predicted_polar_error(sig, abc) - abs(1.0 - y)) < 1e-15


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert p.returncode != 0 and "GPU" in p.stdout
