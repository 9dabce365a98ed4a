"""GPU parity of the 3D lattice path (Kuramoto-Sakaguchi, cube neighbourhood)
against the FP64 CPU oracle and against closed forms, through the C ABI."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_19075_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_19075_amd import nd as _nd
    return _nd


def rel(a, ref):
    return np.max(np.abs(a - ref)) / np.max(np.abs(ref))


def cube_problem(nd, dims, h, prm, prec=0):
    n1, n2, n3 = dims
    return nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, n1 * n2 * n3, prm, precision=prec, radius=h, dims=dims)


def run_cfg(nd, p, y0, dt, steps, cfg=None, record_every=0, mv=-1):
    h = nd.nd_create(p)
    try:
        if cfg:
            c = nd.nd_get_config(h)
            for k, v in cfg.items():
                setattr(c, k, v)
            nd.nd_set_config(h, c)
        nd.nd_set_state(h, y0, on_device=0)
        nd.nd_run(h, dt, steps, nd.observe(record_every, mv))
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
        R = np.empty(steps // record_every + 1) if record_every else None
        M = np.empty(p.n) if mv >= 0 else None
        if R is not None or M is not None:
            nd.nd_get_observables(h, R=R, mean_vel=M, on_device=0)
        return y, R, M
    finally:
        nd.nd_destroy(h)


@pytest.mark.parametrize("dims,h", [((9, 9, 9), 4), ((10, 10, 10), 1), ((12, 11, 13), 2), ((23, 9, 17), 3),
                                    ((40, 40, 40), 4), ((7, 7, 7), 3)])
def test_cube_fp64_parity(nd, dims, h):
    print(f"case cube dims={dims} h={h}", flush=True)
    prm = [0.1, 1.0, 0.8]
    n = dims[0] * dims[1] * dims[2]
    y0 = inputs.kuramoto_phases(sum(dims) + h, n)
    steps = 2 if n > 20000 else 12
    y, R, _ = run_cfg(nd, cube_problem(nd, dims, h, prm), y0, 0.05, steps, record_every=1)
    net = O.cube(dims[0], h, prm, n2=dims[1], n3=dims[2])
    ref, Rref, _ = O.run(net, y0, 0.05, steps, record_every=1)
    assert rel(y, ref) < 1e-12
    assert np.max(np.abs(R - Rref)) < 1e-12


@pytest.mark.parametrize("cfg", [dict(tile=20, tile_y=20, tile_z=40), dict(tile=7, tile_y=13, tile_z=5),
                                 dict(tile=23, tile_y=3, tile_z=17), dict(tile=16, tile_y=16, tile_z=9, grid=8),
                                 dict(tile=9, tile_y=9, tile_z=2, grid=24, chunk=3)])
def test_cube_tilings(nd, cfg):
    """Ragged tiles in x, y and z, persistent grids and graph chunks that do not
    divide the step count all reproduce the oracle."""
    print(f"case cube cfg={cfg}", flush=True)
    dims, h = (23, 20, 17), 4
    prm = [0.0, 1.0, 0.8]
    y0 = inputs.kuramoto_phases(5, dims[0] * dims[1] * dims[2])
    y, R, _ = run_cfg(nd, cube_problem(nd, dims, h, prm), y0, 0.05, 7, cfg=cfg, record_every=2)
    ref, Rref, _ = O.run(O.cube(dims[0], h, prm, n2=dims[1], n3=dims[2]), y0, 0.05, 7, record_every=2)
    assert rel(y, ref) < 1e-12
    assert np.max(np.abs(R - Rref)) < 1e-12


def dirichlet(h, th):
    if abs(math.sin(th / 2)) < 1e-300:
        return 2 * h + 1.0
    return math.sin((h + 0.5) * th) / math.sin(th / 2)


@pytest.mark.parametrize("q", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (5, 0, 0), (3, -2, 7)])
def test_plane_waves_full_200_cube(nd, q):
    """On the full 200^3 lattice (h = 4, alpha = 0.8) a plane wave rotates rigidly
    at omega - mu sin(alpha) (prod_a D_4(theta_a) - 1) / 728 (closed form)."""
    print(f"case plane wave {q}", flush=True)
    n1, h, alpha = 200, 4, 0.8
    idx = np.arange(n1 ** 3)
    x, y, z = idx % n1, (idx // n1) % n1, idx // (n1 * n1)
    y0 = 2 * math.pi * (q[0] * x + q[1] * y + q[2] * z) / n1
    prod = 1.0
    for qa in q:
        prod *= dirichlet(h, 2 * math.pi * qa / n1)
    om = -math.sin(alpha) * (prod - 1) / 728
    dt, steps = 0.05, 10
    yt, R, _ = run_cfg(nd, cube_problem(nd, (n1,) * 3, h, [0.0, 1.0, alpha]), y0, dt, steps, record_every=5)
    assert np.max(np.abs((yt - y0) - om * dt * steps)) < 1e-12 + 1e-14 * np.max(np.abs(y0))
    assert np.max(np.abs(R - (1.0 if q == (0, 0, 0) else 0.0))) < 1e-12


def test_cube_fp32_bulk_within_1e4(nd):
    dims, h = (16, 16, 16), 4
    prm = [0.0, 1.0, 0.8]
    y0 = inputs.cube_phases_with_patch(3, 16)
    y, R, _ = run_cfg(nd, cube_problem(nd, dims, h, prm, prec=1), y0, 0.05, 100, record_every=1)
    ref, Rref, _ = O.run(O.cube(16, h, prm), y0, 0.05, 100, record_every=1)
    e = rel(y, ref)
    print(f"cube fp32-bulk error {e:.3e}")
    assert e < 1e-4
    assert np.max(np.abs(R - Rref)) < 1e-4


def test_cube_mean_velocity_and_checkpoint(nd):
    dims, h = (12, 12, 12), 2
    prm = [0.3, 1.0, 0.8]
    p = cube_problem(nd, dims, h, prm)
    y0 = inputs.kuramoto_phases(8, 12 ** 3)
    y, _, mv = run_cfg(nd, p, y0, 0.05, 40, mv=10)
    ref, _, mvref = O.run(O.cube(12, h, prm), y0, 0.05, 40, mv_start=10)
    assert rel(y, ref) < 1e-12
    assert np.max(np.abs(mv - mvref)) < 1e-10
    a, _, _ = run_cfg(nd, p, y0, 0.05, 15)
    b, _, _ = run_cfg(nd, p, a, 0.05, 25)
    assert np.array_equal(b, y)


def test_cube_batch_equals_solo(nd):
    cases = [((12, 12, 12), 2, 3), ((9, 10, 11), 4, 4), ((30, 30, 30), 4, 5)]
    solos, hs = [], []
    try:
        for dims, h, seed in cases:
            n = dims[0] * dims[1] * dims[2]
            y0 = inputs.kuramoto_phases(seed, n)
            solos.append((y0, run_cfg(nd, cube_problem(nd, dims, h, [0.0, 1.0, 0.8]), y0, 0.05, 9)[0]))
            hh = nd.nd_create(cube_problem(nd, dims, h, [0.0, 1.0, 0.8]))
            nd.nd_set_state(hh, y0, on_device=0)
            hs.append(hh)
        nd.nd_run_batch(hs, [0.05] * 3, [9] * 3)
        for hh, (y0, ys) in zip(hs, solos):
            y = np.empty_like(y0)
            nd.nd_get_state(hh, y, on_device=0)
            assert np.array_equal(y, ys)
    finally:
        for hh in hs:
            nd.nd_destroy(hh)


@pytest.fixture(scope="module")
def cube200_one_step():
    """The benchmark's 200^3 state (h = 4, uniform phases with a planted coherent
    ball) and the oracle's result after one step (about half a minute of oracle
    time), shared by the FP64 and FP32-bulk full-size tests."""
    n1 = 200
    y0 = inputs.cube_phases_with_patch(1000, n1)
    prm = [0.0, 1.0, 0.8]
    ref, Rref, _ = O.run(O.cube(n1, 4, prm), y0, 0.05, 1, record_every=1)
    return n1, prm, y0, ref, Rref


def test_cube_full_200_random_state_one_step(nd, cube200_one_step):
    """The benchmark's workload at full size and in its launch configuration:
    200^3, h = 4, one step, every element against the oracle."""
    print("case full 200^3 cube, one step", flush=True)
    n1, prm, y0, ref, Rref = cube200_one_step
    y, R, _ = run_cfg(nd, cube_problem(nd, (n1,) * 3, 4, prm), y0, 0.05, 1, record_every=1)
    assert rel(y, ref) < 1e-12
    assert np.max(np.abs(R - Rref)) < 1e-12


def test_cube_full_200_fp32_bulk_one_step(nd, cube200_one_step):
    """FP32-bulk at full size in the benchmark's launch configuration (the
    default tiling with its two-plane prefetch), one step, every element against
    the oracle."""
    print("case full 200^3 cube fp32-bulk, one step", flush=True)
    n1, prm, y0, ref, Rref = cube200_one_step
    y, R, _ = run_cfg(nd, cube_problem(nd, (n1,) * 3, 4, prm, prec=1), y0, 0.05, 1, record_every=1)
    e = rel(y, ref)
    print(f"cube 200^3 fp32-bulk one-step error {e:.3e}")
    assert e < 1e-4
    assert np.max(np.abs(R - Rref)) < 1e-4


def test_cube_fp32_bulk_benchmark_tiling_200_steps(nd):
    """FP32-bulk over the 200-step horizon against the oracle, with the tile
    extents the 200^3 lattice runs with (25 x 20 columns per work item) on a
    30^3 lattice, so the same kernel shape meets ragged tiles in x and y and
    ragged z runs (tile_z = 13)."""
    print("case cube 30^3 fp32-bulk with the 200^3 tiling, 200 steps", flush=True)
    n1, h, prm = 30, 4, [0.0, 1.0, 0.8]
    y0 = inputs.cube_phases_with_patch(77, n1)
    cfg = dict(tile=25, tile_y=20, tile_z=13)
    y, R, _ = run_cfg(nd, cube_problem(nd, (n1,) * 3, h, prm, prec=1), y0, 0.05, 200, cfg=cfg, record_every=1)
    ref, Rref, _ = O.run(O.cube(n1, h, prm), y0, 0.05, 200, record_every=1)
    e = rel(y, ref)
    print(f"cube 30^3 fp32-bulk 200-step error {e:.3e}")
    assert e < 1e-4
    assert np.max(np.abs(R - Rref)) < 1e-4


def test_cube_full_200_fp32_bulk_200_steps_against_fp64(nd):
    """FP32-bulk at full size over the 200-step horizon against the FP64 path
    (itself held to the oracle at this size by the one-step test and by the
    plane-wave closed forms): the oracle's O(N L) sums cannot follow 200 steps
    of 8e6 elements."""
    print("case full 200^3 cube fp32-bulk vs fp64, 200 steps", flush=True)
    n1, prm = 200, [0.0, 1.0, 0.8]
    y0 = inputs.cube_phases_with_patch(1001, n1)
    y64, R64, _ = run_cfg(nd, cube_problem(nd, (n1,) * 3, 4, prm), y0, 0.05, 200, record_every=1)
    y32, R32, _ = run_cfg(nd, cube_problem(nd, (n1,) * 3, 4, prm, prec=1), y0, 0.05, 200, record_every=1)
    e = rel(y32, y64)
    print(f"cube 200^3 fp32-bulk vs fp64 after 200 steps {e:.3e}")
    assert e < 1e-4
    assert np.max(np.abs(R32 - R64)) < 1e-4
