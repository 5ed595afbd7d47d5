"""Host logic of bench.py that needs no GPU: the HBM-traffic lookup that keys
measured counter values to the kernel source they were taken on and to the
node shape the bench tuned, and the refusal of several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write(path, sha, lines):
    with open(path, "w") as f:
        f.write(f"kernel_sha256_16: {sha}\n")
        for ln in lines:
            f.write(ln + "\n")


def test_traffic_reported_for_matching_source_and_shape(tmp_path, monkeypatch):
    p = tmp_path / "traffic.txt"
    _write(p, bench.kernel_sha(), [
        "shape 8,1,1: fetch_bytes_per_launch 1000.0 write_bytes_per_launch 250.5 dispatches 3",
        "shape 16,1,1: fetch_bytes_per_launch 7.0 write_bytes_per_launch 1.0 dispatches 3",
    ])
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic((8, 1, 1)) == pytest.approx(1250.5)
    assert bench.measured_traffic((16, 1, 1)) == pytest.approx(8.0)
    # a shape that was not measured has no traffic
    assert bench.measured_traffic((4, 2, 1)) is None


def test_traffic_withheld_once_the_kernel_source_changed(tmp_path, monkeypatch):
    p = tmp_path / "traffic.txt"
    stale = "0" * 16 if bench.kernel_sha() != "0" * 16 else "1" * 16
    _write(p, stale, ["shape 8,1,1: fetch_bytes_per_launch 1000.0 write_bytes_per_launch 250.5 dispatches 3"])
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic((8, 1, 1)) is None


def test_traffic_absent_or_malformed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic((8, 1, 1)) is None
    p = tmp_path / "bad.txt"
    _write(p, bench.kernel_sha(), ["shape 8,1,1: fetch_bytes_per_launch x write_bytes_per_launch 1 dispatches 3"])
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic((8, 1, 1)) is None


def test_committed_traffic_files_are_well_formed():
    # every line the bench may report carries both byte counts
    import glob
    files = glob.glob(os.path.join(bench.PROFILES, "k_node_*_traffic.txt"))
    assert files
    for path in files:
        text = open(path).read().splitlines()
        assert text[0].startswith("kernel_sha256_16: ")
        shapes = [ln for ln in text if ln.startswith("shape ")]
        assert shapes
        for ln in shapes:
            assert "fetch_bytes_per_launch" in ln and "write_bytes_per_launch" in ln


def test_group_rooflines():
    st = {"msg_launches": 10, "group_ms": [0.0, 2.0, 0.0, 0.0, 1.0], "group_pairs": [0.0, 8.0e9, 0.0, 0.0, 1.0e9]}
    g = bench.group_rooflines(st)
    assert set(g) == {"k_node<D=1>", "k_sep_pass+k_node_sep"}
    d1 = g["k_node<D=1>"]
    assert d1["achieved"] == pytest.approx(8.0e9 / 2.0e-3 / 1e9)
    assert d1["peak"] == pytest.approx(bench.pair_peak_gpairs(1))
    assert d1["frac"] == pytest.approx(d1["achieved"] / d1["peak"])
    assert d1["ms_per_stage"] == pytest.approx(0.2)
    assert g["k_sep_pass+k_node_sep"]["peak"] == pytest.approx(bench.pair_peak_gpairs(1))
    ex = bench.group_rooflines({"msg_launches": 1, "group_ms": [1.0, 0, 0, 0, 0], "group_pairs": [1e9, 0, 0, 0, 0]})
    assert ex["k_node<explicit>"]["unit"] == "GB/s" and ex["k_node<explicit>"]["achieved"] == pytest.approx(4000.0)


def test_uniform_grid_groups_price_one_fma_per_pair():
    """Groups 5 and 6 (the Horner kernels on uniform grids) take one FP64 FMA
    per pair: 1024 SIMDs x 2.4 GHz x 64 lanes / 4 cycles = 39.3e12 pairs/s."""
    assert bench.fma_peak_gpairs() == pytest.approx(1024 * 2.4e9 * 64 / 4 / 1e9)
    st = {"msg_launches": 4, "group_ms": [0, 0, 0, 0, 0, 0.4, 0.2], "group_pairs": [0, 0, 0, 0, 0, 4.0e9, 2.0e8]}
    g = bench.group_rooflines(st)
    assert set(g) == {bench.GRID_GROUP_NAME, "k_sep_horner+k_node_sep"}
    grid = g[bench.GRID_GROUP_NAME]
    assert grid["peak"] == pytest.approx(bench.fma_peak_gpairs())
    assert grid["achieved"] == pytest.approx(4.0e9 / 0.4e-3 / 1e9)
    assert grid["ms_per_stage"] == pytest.approx(0.1) and grid["pairs_per_stage"] == pytest.approx(1.0e9)
    assert g["k_sep_horner+k_node_sep"]["peak"] == pytest.approx(bench.fma_peak_gpairs())


def test_rocprof_summaries(tmp_path):
    st = tmp_path / "k_stats.csv"
    st.write_text("Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs,StdDev\n"
                  "k_a,4,400,100.0,80.0,90,110,1\nk_b,1,100,100.0,20.0,100,100,0\n")
    md = bench.summarize_stats(str(st))
    assert "| `k_a` | 4 | 400 | 100 | 80.00 | 90 | 110 |" in md
    pm = tmp_path / "pmc.csv"
    pm.write_text("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
                  "1,k_a,FETCH_SIZE,10\n2,k_a,FETCH_SIZE,30\n3,copy,FETCH_SIZE,5\n")
    md = bench.summarize_pmc(str(pm))
    assert "| `k_a` | FETCH_SIZE | 2 | 20.0 | 30.0 |" in md
    assert "| `copy` | FETCH_SIZE | 1 | 5.0 | 5.0 |" in md


def test_make_traffic_scales_by_the_calibration_copy(tmp_path):
    """Per-dispatch means of a kernel, scaled so the 1 GiB calibration copy
    reads 1 GiB; MIN_FRAC drops launches that did no work."""
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    f = tmp_path / "f.csv"
    f.write_text(hdr + "1,__amd_rocclr_copyBuffer,FETCH_SIZE,524288\n2,k_x<1>,FETCH_SIZE,1000\n"
                       "3,k_x<1>,FETCH_SIZE,3000\n4,k_x<1>,FETCH_SIZE,2\n5,k_y,FETCH_SIZE,7\n")
    w = tmp_path / "w.csv"
    w.write_text(hdr + "1,__amd_rocclr_copyBuffer,WRITE_SIZE,1048576\n2,k_x<1>,WRITE_SIZE,10\n"
                       "3,k_x<1>,WRITE_SIZE,30\n4,k_x<1>,WRITE_SIZE,2\n")
    n, mean, scale = bench.pmc_kernel_bytes(str(f), "k_x")
    assert n == 3 and scale == pytest.approx(2.0) and mean == pytest.approx((1000 + 3000 + 2) / 3 * 1024 * 2)
    n, mean, _ = bench.pmc_kernel_bytes(str(f), "k_x", 0.01)
    assert n == 2 and mean == pytest.approx(2000 * 1024 * 2)
    txt = bench.make_traffic(str(f), str(w), "k_x", "4,1,1", "0.01")
    line = txt.splitlines()[0]
    assert line.startswith("shape 4,1,1: fetch_bytes_per_launch 4096000.0 write_bytes_per_launch 14336.0")
    assert bench.pmc_kernel_bytes(str(f), "k_none") is None


def test_several_gpus_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _gpurun_excluded(rel):
    """Whether a path (relative to the repo root) matches a .gpurunignore
    pattern (tar semantics: './x' anchors at the top, other patterns match any
    path component)."""
    import fnmatch
    pats = [ln.strip() for ln in open(os.path.join(ROOT, ".gpurunignore")) if ln.strip() and not ln.startswith("#")]
    parts = rel.split("/")
    prefixes = ["./" + "/".join(parts[:i + 1]) for i in range(len(parts))]
    for pat in pats:
        if pat.startswith("./"):
            if any(fnmatch.fnmatch(pr, pat) for pr in prefixes):
                return True
        elif any(fnmatch.fnmatch(c, pat) for c in parts):
            return True
    return False


def test_files_the_gpu_runs_read_are_shipped():
    """The bench reads its HBM-traffic summaries from profiles/, the GPU tests
    read the stored references under tests/golden/; none may be left out of
    the tree copied to the GPU machine."""
    paths = [os.path.relpath(f, ROOT) for f in (bench.TRAFFIC_FILE, bench.GRID_TRAFFIC_FILE,
                                                  bench.GRID_CHAIN_TRAFFIC_FILE, bench.CHAIN_TRAFFIC_FILE)]
    for d in ("profiles", os.path.join("tests", "golden")):
        paths += [os.path.join(d, f) for f in os.listdir(os.path.join(ROOT, d))]
    for rel in paths:
        assert not _gpurun_excluded(rel), rel
    assert _gpurun_excluded("_work/probe.py")
