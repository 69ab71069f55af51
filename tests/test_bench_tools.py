"""Host logic of bench.py: the counter reduction that turns two rocprofv3
counter files into per-launch traffic, the validity checks of the stored
traffic records, and the one-GPU guard.  No GPU is used."""
import csv
import os
import subprocess
import sys

import pytest

import bench

HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]

COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(at::TensorIteratorBase&)>"
FWD = "void hsp::(anonymous namespace)::k_bstage_fwd<float, 32, 4, 2, 32>(hsp::BSeg const*, int, int)"
BWD = "void hsp::(anonymous namespace)::k_bstage_bwd<float, 32, 4>(hsp::BSeg const*, int, int)"
FWD8 = "void hsp::(anonymous namespace)::k_bstage_fwd<float, 32, 8, 2, 32>(hsp::BSeg const*, int, int)"
PROJ = "void hsp::(anonymous namespace)::k_bmultidot2<double>(hsp::cx<double> const*, unsigned long, hsp::BIdx, int)"
UPD = "void hsp::(anonymous namespace)::k_bdcgs_update<double>(hsp::cx<double>*, unsigned long, hsp::BIdx, int)"
MV = ("void hsp::(anonymous namespace)::k_stencil_multi<5, double, float, double, double>"
      "(hsp::LevelDev, int, hsp::cx<float> const*, hsp::cx<double> const*, hsp::cx<double>*)")
RES = ("void hsp::(anonymous namespace)::k_stencil_multi<5, double, double, double, double>"
       "(hsp::LevelDev, int, hsp::cx<double> const*, hsp::cx<double> const*, hsp::cx<double>*)")


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEADER)
        for i, (name, value) in enumerate(rows):
            w.writerow([i, i, 1, 1, 1, 1, 256, 1, name, 256, 0, 0, 8, 0, 16, counter, value, 0, 1])


def test_reduce_counters(tmp_path, capsys):
    # copy kernel: FETCH_SIZE sees half of the 256 MiB read, WRITE_SIZE all of
    # the 256 MiB written; two stages at tile 4 and one at tile 8 (ignored)
    kib = bench.COPY_BYTES / 1024
    fetch = [(COPY, kib / 2), (FWD, 150.0), (BWD, 25.0), (FWD, 450.0), (BWD, 75.0),
             (FWD8, 1e6), (PROJ, 1000.0), (PROJ, 3000.0), (UPD, 500.0), (UPD, 700.0),
             (MV, 80.0), (MV, 120.0), (RES, 1e6)]
    write = [(COPY, kib), (FWD, 30.0), (BWD, 30.0), (FWD, 30.0), (BWD, 30.0),
             (FWD8, 1e6), (PROJ, 1.0), (PROJ, 1.0), (UPD, 100.0), (UPD, 100.0),
             (MV, 50.0), (MV, 70.0), (RES, 1e6)]
    _write(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write(tmp_path / "w.csv", "WRITE_SIZE", write)
    bench.reduce_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), tile=4, nsrc=64, chunk=34)
    out = capsys.readouterr().out
    rec = {}
    for line in out.splitlines():
        if line.startswith("traffic-record:"):
            kv = dict(t.split("=") for t in line.split()[1:])
            rec[kv["kernel"]] = kv
    # stage: fetch (700 KiB over 2 stages) x 2 + write (120 KiB over 2 stages) x 1
    stage = float(rec["stage"]["bytes_per_launch"])
    assert stage == pytest.approx((700 / 2 * 2 + 120 / 2) * 1024, rel=1e-5)
    assert rec["stage"]["tile"] == "4" and rec["stage"]["sources"] == "64" and rec["stage"]["chunk"] == "34"
    assert rec["project"]["chunk"] == "0"
    assert rec["stage"]["digest"] == bench.sources_digest("stage")
    proj = float(rec["project"]["bytes_per_launch"])
    assert proj == pytest.approx((4000 / 2 * 2 + 2 / 2) * 1024, rel=1e-5)
    assert rec["project"]["digest"] == bench.sources_digest("project")
    upd = float(rec["update"]["bytes_per_launch"])
    assert upd == pytest.approx((1200 / 2 * 2 + 200 / 2) * 1024, rel=1e-5)
    # the batched matvec only (not the true-residual launches of the same kernel)
    mv = float(rec["matvec"]["bytes_per_launch"])
    assert mv == pytest.approx((200 / 2 * 2 + 120 / 2) * 1024, rel=1e-5)
    assert rec["matvec"]["digest"] == bench.sources_digest("matvec")


def test_reduce_counters_needs_copy(tmp_path):
    _write(tmp_path / "f.csv", "FETCH_SIZE", [(FWD, 1.0)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [(FWD, 1.0)])
    with pytest.raises(SystemExit):
        bench.reduce_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), tile=4, nsrc=64)


def test_recorded_traffic_validity(tmp_path, monkeypatch):
    rec = tmp_path / "traffic.md"
    ds, dp = bench.sources_digest("stage"), bench.sources_digest("project")
    rec.write_text("notes\n"
                   f"traffic-record: kernel=stage bytes_per_launch=1.5e+08 tile=4 chunk=34 sources=64 digest={ds}\n"
                   f"traffic-record: kernel=project bytes_per_launch=9.0e+09 tile=0 chunk=0 sources=64 digest={dp}\n")
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(rec))
    assert bench.recorded_traffic("stage", 4, 64, 34) == 1.5e8
    assert bench.recorded_traffic("stage", 8, 64, 34) is None  # other tile
    assert bench.recorded_traffic("stage", 4, 64, 24) is None  # other chunk length
    assert bench.recorded_traffic("stage", 4, 32, 34) is None  # other batch size
    assert bench.recorded_traffic("project", 8, 64) == 9.0e9  # tile and chunk do not matter
    rec.write_text(f"traffic-record: kernel=stage bytes_per_launch=1.5e+08 tile=4 chunk=34 sources=64 "
                   f"digest=0000{ds[4:]}\n")
    assert bench.recorded_traffic("stage", 4, 64, 34) is None  # kernel sources changed
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic("stage", 4, 64, 34) is None


def test_committed_records_parse():
    """The committed counter summary holds a record for each roofline kernel."""
    with open(bench.TRAFFIC_RECORD) as fh:
        txt = fh.read()
    for kernel in ("stage", "project", "update", "matvec"):
        assert f"traffic-record: kernel={kernel} " in txt


def test_committed_records_match_sources():
    """Every committed counter record was taken on the kernel sources as they
    stand (a kernel change without new counters would report traffic null)."""
    assert bench.recorded_traffic("stage", 4, 64, 34) is not None
    for kernel in ("project", "update", "matvec"):
        assert bench.recorded_traffic(kernel, 0, 64) is not None, kernel
    assert bench.recorded_traffic("nd_stage", 0, 1, 0, bench.ND_TRAFFIC_RECORD) is not None


def test_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
