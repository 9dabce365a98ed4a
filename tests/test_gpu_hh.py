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


@pytest.mark.parametrize("lanes", [4, 8, 16, 32, 64])
def test_hh_lane_groups(nd, lanes):
    print(f"case hh lanes={lanes}", flush=True)
    y, ref = hh_case(nd, 3000, 100, 5, 20, cfg=dict(tile_y=lanes))
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
