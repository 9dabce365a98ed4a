"""Host-side checks of the C-ABI library: it loads, exports what include/nd.h
declares, and rejects bad arguments before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_19075_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:nd_status|const char\*)\s+(nd_\w+)\s*\(", txt, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2410_19075_amd import nd
    lib = ctypes.CDLL(nd.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    from paper_2410_19075_amd import nd
    assert nd.nd_status_str(0) == "ok"
    assert nd.nd_status_str(-1) == "invalid argument"


@pytest.mark.parametrize("kw,needle", [
    (dict(model=0, topo=0, n=10, radius=5), "2P+1"),
    (dict(model=0, topo=0, n=10, radius=0), "2P+1"),
    (dict(model=2, topo=0, n=10, radius=2), "CSR"),
    (dict(model=0, topo=1, n=8 ** 3, radius=4, dims=(8, 8, 8)), "2h+1"),
    (dict(model=0, topo=1, n=999, radius=4, dims=(10, 10, 10)), "n1*n2*n3"),
    (dict(model=1, topo=1, n=1000, radius=1, dims=(10, 10, 10)), "Kuramoto"),
    (dict(model=7, topo=0, n=10, radius=1), "model"),
    (dict(model=1, topo=3, n=1000, radius=1, dims=(10, 10, 10)), "Kuramoto"),
    (dict(model=0, topo=3, n=20 ** 3, radius=9, dims=(20, 20, 20)), "ball radius"),
    (dict(model=0, topo=3, n=8 ** 3, radius=4, dims=(8, 8, 8)), "2P+1"),
    (dict(model=3, topo=0, n=100, radius=3, zero_mass=True), "mass"),
])
def test_invalid_problems_are_rejected_on_the_host(kw, needle):
    from paper_2410_19075_amd import nd
    prm = [1.0, 1.0, 1.0, 0.0 if kw.get("zero_mass") else 0.5, 0, 0, 0, 0, 0, 1.0]
    p = nd.problem(kw["model"], kw["topo"], kw["n"], prm, radius=kw["radius"], dims=kw.get("dims", (0, 0, 0)))
    with pytest.raises(nd.NDError) as ei:
        nd.nd_footprint(p)
    assert ei.value.status == nd.ND_ERR_INVALID_ARG
    assert needle in str(ei.value)


def test_nonfinite_parameters_rejected():
    from paper_2410_19075_amd import nd
    p = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, 100, [0.0, float("nan"), 1.0], radius=3)
    with pytest.raises(nd.NDError):
        nd.nd_footprint(p)


def test_csr_validation():
    from paper_2410_19075_amd import nd
    rp = np.array([0, 1, 2], dtype=np.int64)
    prm = [1, 120, 36, 0.3, 50, -77, -54.387, 0, 0, 2]
    good = nd.problem(nd.ND_HH, nd.ND_CSR, 2, prm, row_ptr=rp, col=np.array([1, 0]), weight=np.array([.1, .1]),
                      per_elem=np.zeros(2))
    assert nd.nd_footprint(good) > 0
    bad = nd.problem(nd.ND_HH, nd.ND_CSR, 2, prm, row_ptr=rp, col=np.array([1, 5]), weight=np.array([.1, .1]),
                     per_elem=np.zeros(2))
    with pytest.raises(nd.NDError):
        nd.nd_footprint(bad)


def test_size_limits_of_rings_and_lattices():
    """Rings and lattices hold at most 2^29 - 1 elements (32-bit element
    offsets with headroom for window ends); one more is rejected on the host."""
    from paper_2410_19075_amd import nd
    top = 2 ** 29 - 1
    ring = lambda n: nd.problem(nd.ND_KURAMOTO, nd.ND_RING, n, [0.0, 1.0, 1.46], radius=n // 4)
    assert nd.nd_footprint(ring(top)) > 6 * top * 8
    with pytest.raises(nd.NDError):
        nd.nd_footprint(ring(top + 1))
    cube = lambda e: nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, e ** 3, [0.0, 1.0, 0.8], radius=4, dims=(e, e, e))
    assert nd.nd_footprint(cube(800)) > 0
    with pytest.raises(nd.NDError):
        nd.nd_footprint(cube(813))  # 813^3 > 2^29


def test_footprint_grows_with_precision_and_size():
    from paper_2410_19075_amd import nd
    f64 = nd.nd_footprint(nd.problem(nd.ND_FHN, nd.ND_RING, 65536, [0.05, 0.5, 0.1, 1.47], radius=22937))
    f32 = nd.nd_footprint(nd.problem(nd.ND_FHN, nd.ND_RING, 65536, [0.05, 0.5, 0.1, 1.47], radius=22937,
                                     precision=nd.ND_FP32_BULK))
    assert f64 > f32 > 2 * 65536 * 8 * 3


# ------------------------------------------------------------ input generators
def test_generators_are_deterministic_and_in_range():
    a = inputs.kuramoto_phases(7, 1000)
    assert np.array_equal(a, inputs.kuramoto_phases(7, 1000))
    assert not np.array_equal(a, inputs.kuramoto_phases(8, 1000))
    assert a.min() >= -np.pi and a.max() < np.pi
    assert abs(a.mean()) < 0.2
    u = inputs.uniform(1, 1, 200000)
    assert abs(u.mean() - 0.5) < 0.005 and abs(u.var() - 1 / 12) < 0.002
    y = inputs.fhn_circle(3, 500)
    assert np.allclose(y[:500] ** 2 + y[500:] ** 2, 4.0)


def test_splitmix64_reference_values():
    """SplitMix64 as published: state += 0x9E3779B97F4A7C15, then the two
    xor-shift-multiply rounds.  From state 0 the first outputs are the
    generator's well-known test vector."""
    z = np.array([0x9E3779B97F4A7C15, 2 * 0x9E3779B97F4A7C15 % 2 ** 64], dtype=np.uint64)
    out = inputs._mix(z)
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


def test_random_graph_structure():
    rp, col, w = inputs.random_out_graph(5, 2000, 30)
    assert rp[0] == 0 and rp[-1] == 2000 * 30 and np.all(np.diff(rp) >= 0)
    tgt = np.repeat(np.arange(2000), np.diff(rp))
    assert np.all(col != tgt)
    # distinct targets per source, ascending sources per target
    assert len(set(zip(col.tolist(), tgt.tolist()))) == col.size
    for i in range(0, 2000, 97):
        seg = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)
    assert np.all(np.bincount(col, minlength=2000) == 30)
    assert w.min() >= 0 and w.max() < 0.1


def test_patch_is_planted():
    phi = inputs.cube_phases_with_patch(3, 20)
    vals, counts = np.unique(phi, return_counts=True)
    big = counts.max()
    # a ball of radius 4 holds 257 lattice points
    assert big == 257


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_ball_link_counts_and_footprint():
    """Ball problems are accepted up to P = 8 and cost the same state memory as
    cube problems of the lattice size (up to the per-work-item sums).  The
    normalisation by the closed-ball count (925 at P = 6) is checked on the GPU
    against the oracle, whose count is pinned to the paper's."""
    from paper_2410_19075_amd import nd
    for P, count in ((2, 33), (6, 925)):
        pb = nd.problem(nd.ND_KURAMOTO, nd.ND_BALL3D, 40 ** 3, [0.0, 1.0, 0.4], radius=P, dims=(40, 40, 40))
        pc = nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, 40 ** 3, [0.0, 1.0, 0.4], radius=min(P, 4), dims=(40, 40, 40))
        fb, fc = nd.nd_footprint(pb), nd.nd_footprint(pc)
        assert abs(fb - fc) < 2e5
    r = np.arange(-6, 7)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    assert int(np.sum(X ** 2 + Y ** 2 + Z ** 2 <= 36)) == 925


# ------------------------------------------- compressed coupling matrix (host)
def _oracle_compress(n, rp, col):
    from oracle import compress as CM
    return CM.compress(n, rp, col)


@pytest.mark.parametrize("case", ["random", "ring", "small_world", "lattice", "disk", "empty_rows"])
def test_links_compression_matches_the_oracle(case):
    """The library's Alg. 2 (host C++) gives exactly the oracle's common vector,
    difference table (same order) and row entries."""
    from paper_2410_19075_amd import nd
    if case == "random":
        n, (rp, col) = 61, inputs.random_links(5, 61, 0.2)
    elif case == "ring":
        n, (rp, col) = 100, inputs.ring_links(100, 17)
    elif case == "small_world":
        n, (rp, col) = 500, inputs.small_world_links(9, 500, 6, 40)
    elif case == "lattice":
        n, (rp, col) = 9 * 10 * 11, inputs.lattice_ball_links(9, 10, 11, 3)
    elif case == "disk":
        n, (rp, col) = 15 * 13, inputs.lattice_ball_links(15, 13, 1, 4)
    else:
        n = 30
        rp0, col0 = inputs.random_links(8, n, 0.3)
        rows = [col0[rp0[i]:rp0[i + 1]] if i % 2 else col0[:0] for i in range(n)]  # even rows empty
        rp = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64)
        col = np.concatenate(rows).astype(np.int32)
    V, dptr, dpos, C, info = nd.nd_compress_links(n, rp, col)
    Vo, Do, Co = _oracle_compress(n, rp, col)
    assert list(V) == Vo and np.array_equal(C, Co)
    assert info.entries == len(Do) and [list(dpos[dptr[k]:dptr[k + 1]]) for k in range(info.entries)] == Do
    assert info.v_bits == len(Vo) and info.d_bits == sum(len(d) for d in Do)


def test_links_unsorted_rows_compress_like_sorted_ones():
    from paper_2410_19075_amd import nd
    n, (rp, col) = 80, inputs.small_world_links(4, 80, 3, 10)
    shuffled = col.copy()
    for i in range(n):
        shuffled[rp[i]:rp[i + 1]] = shuffled[rp[i]:rp[i + 1]][::-1]
    a, b = nd.nd_compress_links(n, rp, col), nd.nd_compress_links(n, rp, shuffled)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


def test_links_paper_3d_radius_6_table_is_small():
    """Ball of radius 6 (925 links) on a flattened periodic lattice: 13^2 = 169
    entries, so the per-row index dominates the compressed size."""
    from paper_2410_19075_amd import nd
    n1 = 26
    rp, col = inputs.lattice_ball_links(n1, n1, n1, 6)
    _, _, _, _, info = nd.nd_compress_links(n1 ** 3, rp, col)
    assert info.v_bits == 925 and info.entries == 169
    # V's positions, the table (offsets, positions, 1/links) and one entry index per row
    assert info.bytes == 4 * 925 + 4 * 170 + 4 * info.d_bits + 8 * 169 + 4 * n1 ** 3


@pytest.mark.parametrize("bad", ["duplicate", "range", "decreasing"])
def test_links_malformed_rows_are_rejected(bad):
    from paper_2410_19075_amd import nd
    n = 6
    rp = np.array([0, 2, 4, 6, 8, 10, 12], dtype=np.int64)
    col = np.array([1, 2, 0, 2, 0, 1, 4, 5, 3, 5, 3, 4], dtype=np.int32)
    if bad == "duplicate":
        col[3] = 0
    elif bad == "range":
        col[5] = 6
    else:
        rp[2] = 1
    with pytest.raises(nd.NDError) as ei:
        nd.nd_compress_links(n, rp, col)
    assert ei.value.status == nd.ND_ERR_INVALID_ARG
    if bad != "decreasing":
        p = nd.problem(nd.ND_KURAMOTO, nd.ND_LINKS, n, [0, 1, 0.5], row_ptr=rp, col=col)
        with pytest.raises(nd.NDError):
            nd.nd_footprint(p)


def test_header_is_plain_c_and_host_calls_work_from_c(tmp_path):
    """include/nd.h compiles as C99, and a C program linked against libnd.so
    calls the host-only entry points (compression of a ring: one empty table
    entry; error reporting) without a GPU."""
    import subprocess
    from paper_2410_19075_amd import nd
    src = tmp_path / "use_nd.c"
    src.write_text(r"""
#include <stdio.h>
#include <stdint.h>
#include "nd.h"
int main(void) {
    enum { N = 40, P = 3 };
    int64_t row_ptr[N + 1];
    int32_t col[N * 2 * P];
    for (int i = 0; i <= N; ++i) row_ptr[i] = (int64_t)i * 2 * P;
    for (int i = 0; i < N; ++i) {
        int c = 0;
        for (int k = -P; k <= P; ++k)
            if (k) col[i * 2 * P + c++] = (int32_t)((i + k + N) % N);
    }
    nd_links_info info;
    nd_status s = nd_compress_links(N, row_ptr, col, NULL, 0, NULL, 0, NULL, 0, NULL, 0, &info);
    printf("%d %lld %lld %lld\n", (int)s, (long long)info.v_bits, (long long)info.entries, (long long)info.d_bits);
    col[1] = col[0];  /* a source listed twice */
    s = nd_compress_links(N, row_ptr, col, NULL, 0, NULL, 0, NULL, 0, NULL, 0, &info);
    printf("%d %s\n", (int)s, nd_status_str(s));
    return 0;
}
""")
    exe = tmp_path / "use_nd"
    libdir = os.path.dirname(nd.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                    "-L", libdir, "-l:libnd.so", "-Wl,-rpath," + libdir], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    assert out[0].split() == ["0", "6", "1", "0"]
    assert out[1].startswith("-1 invalid argument")


@pytest.mark.parametrize("bad", ["float32", "strided", "int64", "list"])
def test_binding_refuses_buffers_the_library_would_overrun(bad):
    """The C side copies len * 8 bytes of FP64, so the binding refuses anything
    that is not a contiguous float64 buffer before the call (no handle needed)."""
    from paper_2410_19075_amd import nd
    a = {"float32": np.zeros(8, dtype=np.float32), "strided": np.zeros(16)[::2],
         "int64": np.zeros(8, dtype=np.int64), "list": [0.0] * 8}[bad]
    for call in (lambda: nd.nd_get_state(None, a), lambda: nd.nd_set_state(None, a),
                 lambda: nd.nd_get_observables(None, R=a), lambda: nd.nd_server_result(None, 1, a)):
        with pytest.raises((TypeError, ValueError)):
            call()


def test_binding_refuses_mixed_or_mislabelled_locations():
    import torch
    from paper_2410_19075_amd import nd
    host = np.zeros(8)
    with pytest.raises(ValueError):
        nd.nd_get_state(None, host, on_device=1)
    with pytest.raises(TypeError):
        nd.nd_set_state(None, torch.zeros(8, dtype=torch.float32))
    with pytest.raises(ValueError):
        nd.nd_set_state(None, torch.zeros(8, 2, dtype=torch.float64).t())
    assert nd._on_device("x", None, False, None) == 0
    with pytest.raises(ValueError):
        nd._on_device("x", None, False, True)
