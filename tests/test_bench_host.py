"""Host-side logic of bench.py (no GPU): the measured-traffic lookup only
returns counter values taken on the current kernel sources."""

import hashlib
import os

import bench


def test_traffic_lookup_follows_kernel_sources(tmp_path, monkeypatch):
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(bench.ROOT, "paper_2412_09734_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    good = tmp_path / "good.txt"
    good.write_text(f"x\nkernel-sources-sha256: {h.hexdigest()}\ntraffic-bytes k_primal: 1234\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(good))
    assert bench.measured_traffic("k_primal") == 1234
    assert bench.measured_traffic("k_dual") is None
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel-sources-sha256: 00\ntraffic-bytes k_primal: 1234\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert bench.measured_traffic("k_primal") is None


def test_multi_gpu_request_exits(monkeypatch, capsys):
    import sys
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
