"""Host-side checks of the profile summariser: counter calibration, traffic per
launch and the SQ-counter figures, on small synthetic profiler databases."""
import sqlite3
import subprocess
import sys

import pytest

K = "void nd::k_cube_stage<0, double, 4, 1, false>(nd::NetDesc const*)"


def _db(path, rows, kind):
    con = sqlite3.connect(path)
    if kind == "trace":
        con.execute("create table kernels(name text, duration int)")
        con.executemany("insert into kernels values(?, ?)", rows)
    else:
        con.execute("create table counters_collection(kernel_name text, counter_name text, value real)")
        con.executemany("insert into counters_collection values(?, ?, ?)", rows)
    con.commit()
    con.close()
    return str(path)


def _run(args):
    r = subprocess.run([sys.executable, "-m", "paper_2410_19075_amd.profsum", *args], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_traffic_from_calibrated_counters(tmp_path):
    """A 1 GiB copy that reads FETCH_SIZE = 0.5 GiB scales FETCH by 2; traffic per
    launch = 2 x FETCH + WRITE (KiB -> bytes), averaged over dispatches."""
    gib = 1 << 30
    cf = _db(tmp_path / "cf.db", [("copyBuffer", "FETCH_SIZE", gib / 2 / 1024)], "pmc")
    cw = _db(tmp_path / "cw.db", [("copyBuffer", "WRITE_SIZE", gib / 1024)], "pmc")
    f = _db(tmp_path / "f.db", [(K, "FETCH_SIZE", 1000.0), (K, "FETCH_SIZE", 3000.0)], "pmc")
    w = _db(tmp_path / "w.db", [(K, "WRITE_SIZE", 500.0)], "pmc")
    out = _run(["--out", str(tmp_path / "o.md"), "--filter", "k_cube_stage", "--sources", "cube.hip",
                "--fetch", f, "--write", w, "--copy-fetch", cf, "--copy-write", cw, "--copy-bytes", str(gib)])
    line = [l for l in out.splitlines() if l.startswith("traffic-per-launch-bytes k_cube_stage f64")][0]
    assert float(line.split(": ")[1]) == pytest.approx((2 * 2000.0 + 500.0) * 1024)


def test_sq_figures(tmp_path):
    """VALU busy = SQ_ACTIVE_INST_VALU / (256 CUs x cycles); issue share =
    SQ_INSTS_VALU x 4 / (1024 SIMDs x cycles); conflict share =
    SQ_LDS_BANK_CONFLICT / (256 x cycles); per access = conflicts / (idx - conflicts)."""
    t = _db(tmp_path / "t.db", [(K, 100000), (K, 100000)], "trace")  # 100 us = 240000 cycles
    cyc = 100e-6 * 2.4e9
    s = _db(tmp_path / "s.db", [(K, "SQ_ACTIVE_INST_VALU", 0.5 * 256 * cyc), (K, "SQ_INSTS_VALU", 0.25 * 1024 * cyc / 4),
                                (K, "SQ_LDS_BANK_CONFLICT", 0.1 * 256 * cyc), (K, "SQ_LDS_IDX_ACTIVE", 0.5 * 256 * cyc)],
            "pmc")
    out = _run(["--out", str(tmp_path / "o.md"), "--filter", "k_cube_stage", "--sources", "cube.hip",
                "--trace", t, "--sq", s])
    row = [l for l in out.splitlines() if l.startswith("| `k_cube_stage") and l.count("|") == 7][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1:] == ["100.00", "0.50", "0.25", "0.10", "0.250"]
