"""GPU parity of the Hodgkin-Huxley CSR path against the FP64 CPU oracle,
through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_19075_amd import inputs

pytestmark = pytest.mark.gpu

HH_PRM = [1.0, 120.0, 36.0, 0.3, 50.0, -77.0, -54.387, 0.0, 0.0, 2.0]


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_19075_amd import nd as _nd
    return _nd


def normwise(a, ref):
    a = a.reshape(4, -1)
    ref = ref.reshape(4, -1)
    return max(np.max(np.abs(a[v] - ref[v])) / np.max(np.abs(ref[v])) for v in range(4))


def hh_case(nd, n, deg, seed, steps, prec=0, cfg=None, dt=0.01):
    rp, col, w = inputs.random_out_graph(seed, n, deg)
    iapp = inputs.hh_iapp(seed, n)
    y0 = inputs.hh_state(seed, n)
    p = nd.problem(nd.ND_HH, nd.ND_CSR, n, HH_PRM, precision=prec, row_ptr=rp, col=col, weight=w, per_elem=iapp)
    h = nd.nd_create(p)
    try:
        if cfg:
            c = nd.nd_get_config(h)
            for k, v in cfg.items():
                setattr(c, k, v)
            nd.nd_set_config(h, c)
        nd.nd_set_state(h, y0, on_device=0)
        nd.nd_run(h, dt, steps)
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
    finally:
        nd.nd_destroy(h)
    ref, _, _ = O.run(O.csr(n, rp, col, w, HH_PRM, iapp), y0, dt, steps)
    return y, ref


@pytest.mark.parametrize("n,deg,steps", [(50, 7, 300), (2000, 50, 200), (1000, 999 // 10, 100), (777, 1, 50)])
def test_hh_fp64_parity(nd, n, deg, steps):
    print(f"case hh n={n} deg={deg}", flush=True)
    y, ref = hh_case(nd, n, deg, n + deg, steps)
    assert normwise(y, ref) < 1e-12


@pytest.mark.parametrize("ept", [2, 4, 8, 16])
def test_hh_edges_per_thread(nd, ept):
    print(f"case hh ept={ept}", flush=True)
    y, ref = hh_case(nd, 3000, 100, 5, 20, cfg=dict(tile_y=ept))
    assert normwise(y, ref) < 1e-12


def test_hh_edges_per_thread_bitwise(nd):
    """Every row's products are added in edge order whatever the chunking, so the
    result does not depend on the edges-per-thread setting at all."""
    ys = [hh_case(nd, 2500, 60, 9, 10, cfg=dict(tile_y=e))[0] for e in (2, 4, 8, 16)]
    for y in ys[1:]:
        assert np.array_equal(y, ys[0])


def hub_graph(n, deg, hub, empty, seed):
    """Random out-degree `deg` graph plus every node feeding `hub`, with the rows
    in `empty` stripped of all in-edges; CSR by target, sources ascending."""
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, size=src.size)
    keep = dst != src
    src, dst = src[keep], dst[keep]
    src = np.concatenate([src, np.delete(np.arange(n), hub)])
    dst = np.concatenate([dst, np.full(n - 1, hub)])
    keep = ~np.isin(dst, empty)
    src, dst = src[keep], dst[keep]
    order = np.lexsort((src, dst))
    src, dst = src[order], dst[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(np.bincount(dst, minlength=n))
    w = rng.uniform(0.0, 0.1, size=src.size)
    return rp, src.astype(np.int32), w


@pytest.mark.parametrize("ept", [2, 16])
def test_hh_hub_row_spans_chunks(nd, ept):
    """A row whose in-edges of one source block exceed a whole chunk (hub with
    in-degree n-1, ~5000 edges per block), and rows with no in-edges at all."""
    n = 40000
    rp, col, w = hub_graph(n, 3, 7, np.arange(100, 300), 11)
    assert np.diff(rp)[100:300].max() == 0 and np.diff(rp)[7] >= n - 1
    iapp = inputs.hh_iapp(11, n)
    y0 = inputs.hh_state(11, n)
    p = nd.problem(nd.ND_HH, nd.ND_CSR, n, HH_PRM, row_ptr=rp, col=col, weight=w, per_elem=iapp)
    h = nd.nd_create(p)
    try:
        c = nd.nd_get_config(h)
        c.tile_y = ept
        nd.nd_set_config(h, c)
        nd.nd_set_state(h, y0, on_device=0)
        nd.nd_run(h, 0.01, 5)
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
    finally:
        nd.nd_destroy(h)
    ref, _, _ = O.run(O.csr(n, rp, col, w, HH_PRM, iapp), y0, 0.01, 5)
    assert normwise(y, ref) < 1e-12


def test_hh_persistent_grid_and_chunks(nd):
    y, ref = hh_case(nd, 5000, 30, 6, 45, cfg=dict(grid=8, chunk=7))
    assert normwise(y, ref) < 1e-12


def test_hh_large_graph_few_steps(nd):
    """10^5 neurons with out-degree 100 (10^7 synapses)."""
    y, ref = hh_case(nd, 100000, 100, 7, 3)
    assert normwise(y, ref) < 1e-12


def test_hh_fp32_bulk(nd):
    y, ref = hh_case(nd, 2000, 50, 8, 200, prec=1)
    e = normwise(y, ref)
    print(f"hh fp32 error {e:.3e}")
    assert e < 1e-4


def test_hh_fp32_bulk_1e5_deg100_200_steps(nd):
    """FP32-bulk over the 200-step horizon at the benchmark's out-degree (10^5
    neurons, 10^7 synapses; the launch configuration of the 10^6 network:
    source blocks per XCD, 256 rows per work item, 8 edges per thread)
    against the oracle."""
    print("case hh 1e5 x 100 fp32-bulk, 200 steps", flush=True)
    y, ref = hh_case(nd, 100000, 100, 9, 200, prec=1)
    e = normwise(y, ref)
    print(f"hh 1e5 fp32-bulk 200-step error {e:.3e}")
    assert e < 1e-4


@pytest.fixture(scope="module")
def hh_full():
    """The benchmark's network (10^6 neurons, out-degree 100) and the oracle's
    state after two steps, shared by the FP64 and FP32-bulk full-size tests."""
    n, deg, seed = 1000000, 100, 1
    rp, col, w = inputs.random_out_graph(seed, n, deg)
    iapp = inputs.hh_iapp(seed, n)
    y0 = inputs.hh_state(seed, n)
    ref, _, _ = O.run(O.csr(n, rp, col, w, HH_PRM, iapp), y0, 0.01, 2)
    return n, rp, col, w, iapp, y0, ref


def hh_run(nd, net, prec, steps):
    n, rp, col, w, iapp, y0, _ = net
    p = nd.problem(nd.ND_HH, nd.ND_CSR, n, HH_PRM, precision=prec, row_ptr=rp, col=col, weight=w, per_elem=iapp)
    y, _, _ = nd.simulate(p, y0, 0.01, steps)
    return y


def test_hh_full_size_two_steps(nd, hh_full):
    """The benchmark's workload at full size and in its launch configuration:
    10^6 neurons, out-degree 100 (10^8 synapses), two steps against the oracle."""
    print("case full HH 1e6 x 100, two steps", flush=True)
    assert normwise(hh_run(nd, hh_full, 0, 2), hh_full[-1]) < 1e-12


def test_hh_full_size_fp32_bulk_two_steps(nd, hh_full):
    """FP32-bulk at full size (FP32 weights and activations, FP64 synaptic sums
    and state), two steps against the oracle."""
    print("case full HH 1e6 x 100 fp32-bulk, two steps", flush=True)
    e = normwise(hh_run(nd, hh_full, 1, 2), hh_full[-1])
    print(f"hh 1e6 fp32-bulk two-step error {e:.3e}")
    assert e < 1e-4


def test_hh_full_size_fp32_bulk_200_steps_against_fp64(nd, hh_full):
    """FP32-bulk at full size over the 200-step horizon against the FP64 path,
    which the two-step oracle test holds at this size."""
    print("case full HH 1e6 x 100 fp32-bulk vs fp64, 200 steps", flush=True)
    e = normwise(hh_run(nd, hh_full, 1, 200), hh_run(nd, hh_full, 0, 200))
    print(f"hh 1e6 fp32-bulk vs fp64 after 200 steps {e:.3e}")
    assert e < 1e-4
