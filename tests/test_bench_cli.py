"""The measurement script's contract that needs no GPU: several GPUs are
refused before any device work, and the counter-measured traffic is
reported only while the sweep source it was taken with is unchanged."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    table = {
        "fp32": {"source_hash": bench.sweep_source_hash(), "bytes_per_launch": 123},
        "fp16": {"source_hash": "0000000000000000", "bytes_per_launch": 456},
        "d3q19_256": {"source_hash": bench.sweep_source_hash(bench.D3_SOURCES), "bytes_per_launch": 789},
        "d3q19_256_mrt": {"source_hash": bench.sweep_source_hash(), "bytes_per_launch": 1},
    }
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(table))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(path))
    assert bench.measured_traffic("fp32") == 123
    assert bench.measured_traffic("fp16") is None              # taken with another source
    assert bench.measured_traffic("d3q19_256") == 789          # keyed by the D3Q19 source
    assert bench.measured_traffic("d3q19_256_mrt") is None     # the 2-D hash does not fit it
    assert bench.measured_traffic("unknown") is None


def test_committed_traffic_table_is_well_formed():
    d = json.load(open(os.path.join(ROOT, "profiles", "sweep_traffic_membrane4096.json")))
    for key, e in d.items():
        assert len(e["source_hash"]) == 16
        assert e["bytes_per_launch"] == round((e["fetch_kib_raw"] * e["fetch_scale"]
                                              + e["write_kib_raw"] * e["write_scale"]) * 1024)
        # counters within a few per cent of the algorithmic bytes
        assert 0.99 < e["bytes_per_launch"] / e["algorithmic_bytes_per_launch"] < 1.1


def _unbound_names(path):
    """Names a function of `path` reads that no enclosing scope, the module
    or the builtins bind (a NameError waiting for that code path)."""
    import ast
    import builtins
    tree = ast.parse(open(path).read())
    module = set(dir(builtins)) | {"__file__", "__name__"}
    for node in tree.body:
        if isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            module.add(node.name)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            module.update((a.asname or a.name).split(".")[0] for a in node.names)
        elif isinstance(node, (ast.Assign, ast.AnnAssign, ast.AugAssign)):
            targets = node.targets if isinstance(node, ast.Assign) else [node.target]
            module.update(n.id for t in targets for n in ast.walk(t) if isinstance(n, ast.Name))

    def bound(fn):
        b = {a.arg for a in ast.walk(fn.args) if isinstance(a, ast.arg)}
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
                b.add(n.id)
            elif isinstance(n, ast.FunctionDef) and n is not fn:
                b.add(n.name)
            elif isinstance(n, (ast.Import, ast.ImportFrom)):
                b.update((a.asname or a.name).split(".")[0] for a in n.names)
            elif isinstance(n, ast.ExceptHandler) and n.name:
                b.add(n.name)
            elif isinstance(n, ast.arg):
                b.add(n.arg)
        return b

    bad = []

    def visit(fn, outer):
        scope = outer | bound(fn)
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load) and n.id not in scope:
                bad.append((fn.name, n.id, n.lineno))
        for n in ast.walk(fn):
            if isinstance(n, ast.FunctionDef) and n is not fn:
                visit(n, scope)

    for node in tree.body:
        if isinstance(node, ast.FunctionDef):
            visit(node, module)
    return sorted(set(bad))


def test_bench_and_package_read_no_unbound_names():
    # every workload of the bench is a separate code path that the default
    # run never enters; a name left over from another function would only
    # fail when that workload runs
    for rel in ("bench.py", "__graft_entry__.py", os.path.join("paper_2003_12186_amd", "binding.py"),
                os.path.join("paper_2003_12186_amd", "workloads.py"),
                os.path.join("paper_2003_12186_amd", "train_learned.py"),
                os.path.join("paper_2003_12186_amd", "learned.py")):
        assert _unbound_names(os.path.join(ROOT, rel)) == [], rel
