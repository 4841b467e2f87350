"""Host logic of bench.py: the committed traffic counters count only for the
stencil source and launch shape they were taken on."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _counter_fields(path):
    for line in open(path):
        if line.strip().startswith("counters:"):
            return dict(f.split("=", 1) for f in line.split()[1:])
    raise AssertionError("no counters line")


def test_committed_traffic_for_the_recorded_shape(bench):
    kv = _counter_fields(bench.COUNTERS)
    shape = [int(v) for v in kv["shape"].split(",")]
    want = (float(kv["fetch_kib"]) + float(kv["write_kib"])) * 1024.0 * float(kv.get("scale", 1.0))
    assert bench.committed_traffic(shape) == want


def test_committed_traffic_refused_for_another_shape(bench):
    kv = _counter_fields(bench.COUNTERS)
    shape = [int(v) for v in kv["shape"].split(",")]
    shape[1] += 1
    assert bench.committed_traffic(shape) is None


def test_committed_traffic_refused_for_another_source(bench, tmp_path, monkeypatch):
    """An edit inside the roofline kernel voids the counters; one elsewhere in
    the stencil file does not."""
    text = open(bench.STENCIL_SRC).read()
    kv = _counter_fields(bench.COUNTERS)
    shape = [int(v) for v in kv["shape"].split(",")]
    head = "void k_stencil_z2("
    i = text.index(head) + len(head)
    src = tmp_path / "stencil.hip"
    src.write_text(text[:i] + "/* changed */" + text[i:])
    monkeypatch.setattr(bench, "STENCIL_SRC", str(src))
    assert bench.committed_traffic(shape) is None
    src.write_text(text + "\n// changed elsewhere\n")
    assert bench.committed_traffic(shape) is not None


def test_more_than_one_gpu_is_refused(bench, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2


def test_oversize_grid_depth_matches_the_workload_hierarchies(bench):
    """The oversize control halves its grid down to 4 elements per axis, the
    depth of the 64^3 and 128^3 workloads."""
    import workloads as W
    assert bench.oversize_levels(W.C2.nelx) == W.C2.levels
    assert bench.oversize_levels(W.C3.nelx) == W.C3.levels
    assert bench.oversize_levels(256) == 7
    for n in (96, 160, 256, 384):
        L = bench.oversize_levels(n)
        assert n % (1 << (L - 1)) == 0           # every coarse grid has whole elements
        assert 2 <= n >> (L - 1) <= 4 or (n >> (L - 1)) % 2 == 1
