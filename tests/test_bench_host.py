"""Host-side logic of bench.py (no GPU): the HBM traffic recorded in the
committed rocprofv3 summary is reported only while the kernel sources still
hash to the value it was taken on."""
import os
import shutil

import bench


def test_recorded_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "profiles", "denoiser_step_4096sq_bf16.md")
    text = open(src).read()
    h = bench.kernel_source_hash()
    assert len(h) == 64
    row = "conv_pair_ws_kernel"
    # a summary taken on the current sources: the row's read + write bytes
    cur = tmp_path / "cur.md"
    shutil.copy(src, cur)
    body = text
    import re
    body = re.sub(r"`[0-9a-f]{64}`", f"`{h}`", body)
    cur.write_text(body)
    monkeypatch.setattr(bench, "PROFILE_MD", str(cur))
    t = bench.recorded_traffic(row)
    assert t is not None and 1e9 < t < 1e11
    line = next(l for l in body.splitlines() if f"pnp::{row}(" in l and l.count("|") == 6)
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert abs(t - (float(cells[3]) + float(cells[4])) * 1e9) < 1.0
    # a kernel with no row
    assert bench.recorded_traffic("no_such_kernel") is None
    # sources changed since: no figure
    stale = tmp_path / "stale.md"
    stale.write_text(re.sub(r"`[0-9a-f]{64}`", "`" + "0" * 64 + "`", body))
    monkeypatch.setattr(bench, "PROFILE_MD", str(stale))
    assert bench.recorded_traffic(row) is None
    # no summary at all
    monkeypatch.setattr(bench, "PROFILE_MD", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic(row) is None


def test_gpus_above_one_is_refused(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    try:
        bench.main()
    except SystemExit as e:
        assert e.code == 2
    else:
        raise AssertionError("bench.py --gpus 2 must exit")
    assert "one GPU" in capsys.readouterr().out
