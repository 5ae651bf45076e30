"""Host-side logic of bench.py that runs without a GPU: the one-GPU rule,
the rule that a committed HBM-traffic record is used only while the kernel
sources it was measured on are unchanged, and that its functions read only
names that exist."""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_traffic_record_is_used_only_for_unchanged_sources(monkeypatch):
    rec = bench.profiled_traffic("k_sweep_bit1_tiles")
    if rec is None:
        pytest.skip("flagship traffic record absent or stale")
    assert rec["hbm_read_bytes_per_launch"] > 0 and rec["hbm_write_bytes_per_launch"] > 0
    assert bench.profiled_traffic("k_halfsweep_bit1") is None  # another kernel's record
    monkeypatch.setattr(bench, "kernel_source_hash", lambda source: "0" * 64)
    assert bench.profiled_traffic("k_sweep_bit1_tiles") is None


def test_source_hash_covers_every_header_a_kernel_includes():
    """Each source listed for a traffic record hashes the headers it includes
    from the library's own sources, so an edit to any of them drops the record."""
    csrc = os.path.join(ROOT, "paper_2402_06415_amd", "csrc")
    for source, files in bench.KERNEL_SOURCES.items():
        seen, todo = set(), [source]
        while todo:
            f = todo.pop()
            if f in seen:
                continue
            seen.add(f)
            for line in open(os.path.join(csrc, f)):
                if line.startswith("#include \"") and os.path.exists(
                        os.path.join(csrc, line.split('"')[1])):
                    todo.append(line.split('"')[1])
        assert seen <= set(files), (source, sorted(seen - set(files)))


def test_committed_traffic_records_are_complete():
    recs = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")))
    assert recs
    for path in recs:
        rec = json.load(open(path))
        assert rec["kernel"].startswith("k_"), path
        assert len(rec["kernel_source_sha256"]) == 64, path
        assert rec["hbm_read_bytes_per_launch"] > 0 and rec["hbm_write_bytes_per_launch"] > 0
        assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0


@pytest.mark.parametrize("rel", ["bench.py", "__graft_entry__.py"] + sorted(
    os.path.relpath(f, ROOT) for f in glob.glob(os.path.join(ROOT, "paper_2402_06415_amd", "*.py"))
    + glob.glob(os.path.join(ROOT, "oracle", "*.py"))))
def test_functions_read_only_defined_names(rel):
    """Every name a function reads from its module's scope is defined there
    or is a builtin (Python's symbol tables): bench.py's workloads other than
    the default run only on a GPU, so a name left undefined in one of them
    would otherwise surface only there; the same holds for the package."""
    import builtins
    import symtable

    src = open(os.path.join(ROOT, rel)).read()
    top = symtable.symtable(src, rel, "exec")
    module_names = {s.get_name() for s in top.get_symbols() if s.is_assigned() or s.is_imported()}
    known = module_names | set(dir(builtins)) | {"__file__", "__name__"}
    missing = []

    def walk(table):
        for child in table.get_children():
            if child.get_type() == "function":
                for s in child.get_symbols():
                    if (s.is_referenced() and s.is_global() and not s.is_assigned()
                            and s.get_name() not in known):
                        missing.append(f"{child.get_name()}: {s.get_name()}")
            walk(child)

    walk(top)
    assert not missing, missing
