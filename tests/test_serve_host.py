"""Host-side behaviour of the serving API (no GPU work is started)."""
import numpy as np
import pytest

from paper_2410_19075_amd import inputs

nd = pytest.importorskip("paper_2410_19075_amd.nd")


def kur(n=1024, P=256):
    return nd.problem(nd.ND_KURAMOTO, nd.ND_RING, n, [0.0, 1.0, 1.46], radius=P)


def test_config_validation():
    with pytest.raises(nd.NDError):
        nd.nd_server_create(0)
    with pytest.raises(nd.NDError):
        nd.nd_server_create(1 << 30, max_slots=0)
    with pytest.raises(nd.NDError):
        nd.nd_server_create(1 << 30, grid=12)
    s = nd.nd_server_create(1 << 30)
    nd.nd_server_destroy(s)


def test_submit_rejections_fail_alone():
    s = nd.nd_server_create(1 << 20, max_slots=4)
    try:
        good = nd.nd_server_submit(s, kur(), inputs.kuramoto_phases(1, 1024), 0.01, 10)
        y = inputs.kuramoto_phases(2, 1024)
        y[17] = np.nan
        with pytest.raises(nd.NDError) as ei:
            nd.nd_server_submit(s, kur(), y, 0.01, 10)
        assert ei.value.status == nd.ND_ERR_NUMERIC
        with pytest.raises(nd.NDError) as ei:  # footprint above the budget
            nd.nd_server_submit(s, kur(1 << 20, 1000), inputs.kuramoto_phases(3, 1 << 20), 0.01, 10)
        assert ei.value.status == nd.ND_ERR_INVALID_ARG and "budget" in str(ei.value)
        with pytest.raises(nd.NDError):
            nd.nd_server_submit(s, kur(), inputs.kuramoto_phases(1, 1000), 0.01, 10)  # wrong length
        with pytest.raises(nd.NDError):
            nd.nd_server_submit(s, kur(), inputs.kuramoto_phases(1, 1024), 0.0, 10)
        st = nd.nd_server_stats(s)
        assert st.submitted == 1 and st.queued == 1
        info = nd.nd_server_info(s, good)
        assert info.state == nd.ND_REQ_QUEUED and info.admitted == -1.0
    finally:
        nd.nd_server_destroy(s)


def test_cancel_queued_request_without_gpu_work():
    s = nd.nd_server_create(1 << 30)
    try:
        r = nd.nd_server_submit(s, kur(), inputs.kuramoto_phases(1, 1024), 0.01, 10, arrival=0.0)
        nd.nd_server_cancel(s, r)
        assert nd.nd_server_pump(s) == 0  # only the cancelled head: nothing is launched
        assert nd.nd_server_info(s, r).state == nd.ND_REQ_CANCELLED
        with pytest.raises(nd.NDError) as ei:
            nd.nd_server_result(s, r, np.empty(1024))
        assert ei.value.status == nd.ND_ERR_NOT_READY
    finally:
        nd.nd_server_destroy(s)


def test_tune_cache_roundtrip(tmp_path):
    f = tmp_path / "tune.txt"
    f.write_text("# arch model topo precision log2n width h tile block grid chunk tile_y tile_z\n"
                 "gfx950 1 0 0 16 2 0 512 128 0 64 0 0\n"
                 "gfx950 0 1 1 23 0 4 24 832 0 32 24 100\n")
    nd.nd_tune_clear()
    nd.nd_tune_load(str(f))
    out = tmp_path / "out.txt"
    nd.nd_tune_save(str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert sorted(lines) == sorted(["gfx950 0 1 1 23 0 4 24 832 0 32 24 100", "gfx950 1 0 0 16 2 0 512 128 0 64 0 0"])
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 1 0\n")
    with pytest.raises(nd.NDError):
        nd.nd_tune_load(str(bad))
    nd.nd_tune_clear()


def test_footprint_follows_the_tuned_configuration(tmp_path):
    """nd_footprint (and the server's admission) sizes a problem with the
    configuration nd_create will use: a cached autotuner entry changes the tile
    count of a ring, and with it the per-tile sum buffers."""
    n, P = 1 << 16, 1 << 13
    p = nd.problem(nd.ND_FHN, nd.ND_RING, n, [0.05, 0.5, 0.1, 1.47], radius=P)
    nd.nd_tune_clear()
    base = nd.nd_footprint(p)
    f = tmp_path / "tune.txt"
    # width bucket floor(8 P / n) = 1, log2 n = 16; the same entry for a host without a device
    f.write_text("".join(f"{arch} 1 0 0 16 1 0 128 64 0 64 0 0\n" for arch in ("unknown", "gfx950")))
    nd.nd_tune_load(str(f))
    try:
        tuned = nd.nd_footprint(p)
    finally:
        nd.nd_tune_clear()
    # tiles of 128 instead of 512: three more per-tile pairs of doubles per 128 elements x 3 buffers
    assert tuned - base == 3 * 2 * 8 * (n // 128 - n // 512)
