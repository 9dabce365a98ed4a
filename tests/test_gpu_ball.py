"""GPU parity of the ball neighbourhood (lattice points within distance P,
centre included: the paper's 3D topology) for both Kuramoto models against the
FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_19075_amd import inputs

pytestmark = pytest.mark.gpu

KUR = [0.1, 1.0, 0.45]
INERT = [0.1, 1.0, 0.45, 1.0, 0.05]


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_19075_amd import nd as _nd
    return _nd


def normwise(a, ref, nvars):
    a, ref = a.reshape(nvars, -1), ref.reshape(nvars, -1)
    return max(np.max(np.abs(a[v] - ref[v])) / np.max(np.abs(ref[v])) for v in range(nvars))


def case(nd, model, dims, P, seed, steps, prec=0, cfg=None, record_every=0, mv=-1, dt=0.05):
    n1, n2, n3 = dims
    n = n1 * n2 * n3
    phases = inputs.kuramoto_phases(seed, n)
    if model == "inertia":
        y0 = np.concatenate([phases, inputs.uniform_range(seed, inputs.TAG_MISC, n, -0.5, 0.5)])
        code, ocode, prm, nv = nd.ND_KURAMOTO_INERTIA, O.INERTIA, INERT, 2
    else:
        y0, code, ocode, prm, nv = phases, nd.ND_KURAMOTO, O.KURAMOTO, KUR, 1
    p = nd.problem(code, nd.ND_BALL3D, n, prm, precision=prec, radius=P, dims=dims)
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
        R = mvel = None
        if record_every or mv >= 0:
            R = np.empty(steps // record_every + 1) if record_every else None
            mvel = np.empty(n) if mv >= 0 else None
            nd.nd_get_observables(h, R=R, mean_vel=mvel, on_device=0)
    finally:
        nd.nd_destroy(h)
    ref, Rref, mvref = O.run(O.ball(n1, P, prm, n2=n2, n3=n3, model=ocode), y0, dt, steps,
                             record_every=record_every, mv_start=mv if mv >= 0 else None)
    return y, ref, R, Rref, mvel, mvref, nv


@pytest.mark.parametrize("model", ["kuramoto", "inertia"])
@pytest.mark.parametrize("dims,P", [((12, 12, 12), 1), ((20, 18, 16), 2), ((13, 14, 15), 3), ((13, 13, 13), 6),
                                    ((11, 30, 9), 4), ((15, 11, 12), 5), ((15, 16, 15), 7), ((17, 18, 17), 8)])
def test_ball_fp64_parity(nd, model, dims, P):
    print(f"case ball {model} dims={dims} P={P}", flush=True)
    y, ref, R, Rref, mv, mvref, nv = case(nd, model, dims, P, sum(dims) + P, 25, record_every=5, mv=10)
    assert normwise(y, ref, nv) < 1e-12
    assert np.max(np.abs(R - Rref)) < 1e-12
    assert np.max(np.abs(mv - mvref)) < 1e-10


@pytest.mark.parametrize("cfg", [dict(tile=7, tile_y=5, tile_z=3), dict(tile=24, tile_y=9, tile_z=17),
                                 dict(tile=1, tile_y=1, tile_z=1), dict(tile=16, tile_y=16, tile_z=4, grid=8, chunk=3)])
def test_ball_tilings(nd, cfg):
    """Ragged tiles in every direction, single-element tiles, a persistent grid
    smaller than the work and graph chunks that do not divide the steps."""
    print(f"case ball cfg={cfg}", flush=True)
    y, ref, _, _, _, _, nv = case(nd, "inertia", (24, 22, 20), 2, 3, 11, cfg=cfg)
    assert normwise(y, ref, nv) < 1e-12


@pytest.mark.parametrize("model", ["kuramoto", "inertia"])
def test_ball_fp32_bulk(nd, model):
    y, ref, _, _, _, _, nv = case(nd, model, (16, 16, 16), 3, 4, 200, prec=1)
    e = normwise(y, ref, nv)
    print(f"ball {model} fp32-bulk error {e:.3e}")
    assert e < 1e-4


def test_ball_restart_is_bitwise(nd):
    n1, P = 18, 2
    n = n1 ** 3
    y0 = np.concatenate([inputs.cube_phases_with_patch(5, n1), np.zeros(n)])
    p = nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, n, INERT, radius=P, dims=(n1,) * 3)
    a, _, _ = nd.simulate(p, y0, 0.05, 30)
    b, _, _ = nd.simulate(p, y0, 0.05, 12)
    c, _, _ = nd.simulate(p, b, 0.05, 18)
    assert np.array_equal(a, c)


@pytest.mark.parametrize("n1,P,steps", [(100, 2, 2), (60, 6, 1)])
def test_ball_paper_performance_shapes(nd, n1, P, steps):
    """The paper's performance state (Sec. V, Fig. 6c): Kuramoto with inertia,
    m = 1, eps = 0.05, mu = 0.01, alpha = 0.45, ball radius 2 (33 links) on
    100^3, and radius 6 (925 links) on 60^3; psi = 0 initially."""
    n = n1 ** 3
    prm = [0.0, 0.01, 0.45, 1.0, 0.05]
    y0 = np.concatenate([inputs.cube_phases_with_patch(6, n1), np.zeros(n)])
    p = nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, n, prm, radius=P, dims=(n1,) * 3)
    y, _, _ = nd.simulate(p, y0, 0.05, steps)
    ref, _, _ = O.run(O.ball(n1, P, prm, model=O.INERTIA), y0, 0.05, steps)
    assert normwise(y, ref, 2) < 1e-12


def run_cfg(nd, model, dims, P, seed, steps, prec, cfg):
    """Final state and R(t) of one run with the given kernel configuration."""
    n = dims[0] * dims[1] * dims[2]
    phases = inputs.kuramoto_phases(seed, n)
    if model == "inertia":
        y0 = np.concatenate([phases, inputs.uniform_range(seed, inputs.TAG_MISC, n, -0.5, 0.5)])
        code, prm = nd.ND_KURAMOTO_INERTIA, INERT
    else:
        y0, code, prm = phases, nd.ND_KURAMOTO, KUR
    p = nd.problem(code, nd.ND_BALL3D, n, prm, precision=prec, radius=P, dims=dims)
    h = nd.nd_create(p)
    try:
        c = nd.nd_get_config(h)
        for k, v in cfg.items():
            setattr(c, k, v)
        nd.nd_set_config(h, c)
        assert nd.nd_get_config(h).block == cfg["block"]
        nd.nd_set_state(h, y0, on_device=0)
        nd.nd_run(h, 0.05, steps, nd.observe(3, -1))
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
        R = np.empty(steps // 3 + 1)
        nd.nd_get_observables(h, R=R, on_device=0)
    finally:
        nd.nd_destroy(h)
    return y, R


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("model", ["kuramoto", "inertia"])
@pytest.mark.parametrize("dims,P,scatter,gather", [
    ((12, 12, 12), 1, dict(tile=12, tile_y=12, tile_z=3, block=512), dict(tile=12, tile_y=12, tile_z=12, block=1024)),
    ((20, 18, 16), 2, dict(tile=20, tile_y=18, tile_z=5, block=512), dict(tile=20, tile_y=18, tile_z=16, block=1024)),
    ((20, 18, 16), 2, dict(tile=7, tile_y=5, tile_z=3, block=512), dict(tile=7, tile_y=4, tile_z=7, block=256)),
    ((13, 14, 15), 6, dict(tile=13, tile_y=14, tile_z=4, block=512), dict(tile=13, tile_y=12, tile_z=15, block=1024)),
    ((16, 15, 14), 6, dict(tile=5, tile_y=3, tile_z=1, block=512), dict(tile=5, tile_y=7, tile_z=3, block=1024))])
def test_ball_scatter_matches_gather_bitwise(nd, prec, model, dims, P, scatter, gather):
    """The plane-scatter form (block 512) adds every output's runs in the
    gather form's (dz, dy) order, so with the same x tiling (the row prefix
    sums start at the same halo column) the two give bitwise equal states for
    any y and z tilings (ragged tiles, z runs shorter than the 2P lead-in); R
    sums the per-work-item partials in tile order, so it agrees to rounding."""
    print(f"case ball scatter/gather {model} prec={prec} dims={dims} P={P} {scatter} {gather}", flush=True)
    ys, Rs = run_cfg(nd, model, dims, P, 21 + P, 7, prec, scatter)
    yg, Rg = run_cfg(nd, model, dims, P, 21 + P, 7, prec, gather)
    assert np.array_equal(ys, yg)
    assert np.max(np.abs(Rs - Rg)) < 1e-13


def test_ball_scatter_other_x_tiling(nd):
    """Different x tilings move the row prefix origins, so the forms then
    agree to rounding (both are checked against the oracle elsewhere)."""
    ys, _ = run_cfg(nd, "inertia", (20, 18, 16), 2, 23, 7, 0, dict(tile=7, tile_y=5, tile_z=3, block=512))
    yg, _ = run_cfg(nd, "inertia", (20, 18, 16), 2, 23, 7, 0, dict(tile=9, tile_y=4, tile_z=7, block=256))
    assert np.max(np.abs(ys - yg)) < 1e-12


@pytest.mark.parametrize("cfg", [dict(tile=1, tile_y=1, tile_z=1, block=512),
                                 dict(tile=52, tile_y=9, tile_z=2, block=512),
                                 dict(tile=11, tile_y=20, tile_z=40, grid=5, chunk=2, block=512)])
def test_ball_scatter_tilings_p6(nd, cfg):
    """Plane-scatter form at P = 6 against the oracle: single-element tiles
    (every output plane a lead-in edge case), the widest halo row (HX = 64) and
    a z run longer than the lattice, under a persistent grid and graph chunks."""
    print(f"case ball scatter P=6 cfg={cfg}", flush=True)
    y, ref, _, _, _, _, nv = case(nd, "inertia", (52, 20, 13), 6, 8, 5, cfg=cfg)
    assert normwise(y, ref, nv) < 1e-12


def test_ball_default_config_forms(nd):
    """Balls of radius 3 and more default to the plane-scatter form (block 512),
    radius 1 and 2 and the disk to the gather form; the scatter block can be
    chosen for any ball radius, and is refused for the disk."""
    def make(topo, P, dims):
        n = dims[0] * dims[1] * dims[2]
        return nd.nd_create(nd.problem(nd.ND_KURAMOTO, topo, n, KUR, radius=P, dims=dims))
    for P in (1, 2, 3, 4, 6, 8):
        h = make(nd.ND_BALL3D, P, (30, 30, 30))
        try:
            c = nd.nd_get_config(h)
            assert c.block == 512 if P >= 3 else c.block in (256, 1024), (P, c.block)
            if c.block != 512:
                c.block, c.tile, c.tile_y = 512, 8, 8
                nd.nd_set_config(h, c)
                assert nd.nd_get_config(h).block == 512
        finally:
            nd.nd_destroy(h)
    h = make(nd.ND_DISK2D, 6, (40, 40, 1))
    try:
        c = nd.nd_get_config(h)
        assert c.block in (256, 1024)
        c.block = 512
        with pytest.raises(nd.NDError):
            nd.nd_set_config(h, c)
    finally:
        nd.nd_destroy(h)


@pytest.fixture(scope="module")
def ball100_p6_one_step():
    """The ball workload's state (100^3, radius 6, 925 links, Sec. V: m = 1,
    eps = 0.05, mu = 0.01, alpha = 0.45, planted coherent ball, psi = 0) and the
    oracle's result after one step."""
    n1, P = 100, 6
    n = n1 ** 3
    prm = [0.0, 0.01, 0.45, 1.0, 0.05]
    y0 = np.concatenate([inputs.cube_phases_with_patch(1000, n1), np.zeros(n)])
    ref, Rref, _ = O.run(O.ball(n1, P, prm, model=O.INERTIA), y0, 0.05, 1, record_every=1)
    return n1, P, prm, y0, ref, Rref


@pytest.mark.parametrize("prec", [0, 1])
def test_ball_full_100_p6_one_step(nd, ball100_p6_one_step, prec):
    """The ball workload at full size in its launch configuration (the default:
    plane-scatter form, two workgroups per CU), one step, every element and R
    against the oracle."""
    print(f"case full 100^3 ball P=6 prec={prec}, one step", flush=True)
    n1, P, prm, y0, ref, Rref = ball100_p6_one_step
    n = n1 ** 3
    p = nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, n, prm, precision=prec, radius=P, dims=(n1,) * 3)
    h = nd.nd_create(p)
    try:
        assert nd.nd_get_config(h).block == 512
        nd.nd_set_state(h, y0, on_device=0)
        nd.nd_run(h, 0.05, 1, nd.observe(1, -1))
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
        R = np.empty(2)
        nd.nd_get_observables(h, R=R, on_device=0)
    finally:
        nd.nd_destroy(h)
    e = normwise(y, ref, 2)
    print(f"ball 100^3 P=6 prec={prec} one-step error {e:.3e}")
    assert e < (1e-12 if prec == 0 else 1e-4)
    assert np.max(np.abs(R - Rref)) < (1e-12 if prec == 0 else 1e-4)


def case2d(nd, model, n1, n2, P, seed, steps, prec=0, cfg=None, record_every=0):
    n = n1 * n2
    phases = inputs.kuramoto_phases(seed, n)
    if model == "inertia":
        y0 = np.concatenate([phases, inputs.uniform_range(seed, inputs.TAG_MISC, n, -0.5, 0.5)])
        code, ocode, prm, nv = nd.ND_KURAMOTO_INERTIA, O.INERTIA, INERT, 2
    else:
        y0, code, ocode, prm, nv = phases, nd.ND_KURAMOTO, O.KURAMOTO, KUR, 1
    p = nd.problem(code, nd.ND_DISK2D, n, prm, precision=prec, radius=P, dims=(n1, n2, 1))
    h = nd.nd_create(p)
    try:
        if cfg:
            c = nd.nd_get_config(h)
            for k, v in cfg.items():
                setattr(c, k, v)
            nd.nd_set_config(h, c)
        nd.nd_set_state(h, y0, on_device=0)
        nd.nd_run(h, 0.05, steps, nd.observe(record_every, -1))
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
        R = None
        if record_every:
            R = np.empty(steps // record_every + 1)
            nd.nd_get_observables(h, R=R, on_device=0)
    finally:
        nd.nd_destroy(h)
    ref, Rref, _ = O.run(O.disk(n1, P, prm, n2=n2, model=ocode), y0, 0.05, steps, record_every=record_every)
    return y, ref, R, Rref, nv


@pytest.mark.parametrize("model", ["kuramoto", "inertia"])
@pytest.mark.parametrize("n1,n2,P,cfg", [(40, 36, 2, None), (17, 19, 6, None), (64, 64, 1, None),
                                         (30, 25, 3, dict(tile=7, tile_y=5, tile_z=1)),
                                         (50, 40, 4, dict(tile=32, tile_y=8, tile_z=1, block=256))])
def test_disk_fp64_parity(nd, model, n1, n2, P, cfg):
    print(f"case disk {model} {n1}x{n2} P={P} cfg={cfg}", flush=True)
    y, ref, R, Rref, nv = case2d(nd, model, n1, n2, P, n1 + P, 40, cfg=cfg, record_every=4)
    assert normwise(y, ref, nv) < 1e-12
    assert np.max(np.abs(R - Rref)) < 1e-12


def test_disk_fp32_bulk(nd):
    y, ref, _, _, nv = case2d(nd, "inertia", 48, 48, 3, 9, 200, prec=1)
    e = normwise(y, ref, nv)
    print(f"disk fp32-bulk error {e:.3e}")
    assert e < 1e-4
