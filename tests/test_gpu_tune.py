"""Autotuner on the GPU: picks a valid configuration, later networks of the
same key use it, and results stay exact."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_19075_amd import inputs

pytestmark = pytest.mark.gpu
FHN_PRM = [0.05, 0.5, 0.1, math.pi / 2 - 0.1]


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_19075_amd import nd as _nd
    return _nd


def test_tune_ring_and_cube(nd, tmp_path):
    nd.nd_tune_clear()
    try:
        n, P = 20000, 7000
        p = nd.problem(nd.ND_FHN, nd.ND_RING, n, FHN_PRM, radius=P)
        y0 = inputs.fhn_circle(1, n)
        best, ms = nd.nd_tune(p, y0, 0.01, 8)
        assert best.tile in (128, 256, 512, 1024, 2048) and ms > 0
        h = nd.nd_create(p)
        try:
            assert nd.nd_get_config(h).tile == best.tile
        finally:
            nd.nd_destroy(h)
        y, _, _ = nd.simulate(p, y0, 0.01, 20)
        ref, _, _ = O.run(O.ring(O.FHN, n, P, FHN_PRM), y0, 0.01, 20)
        assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-12
        pc = nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, 24 ** 3, [0.0, 1.0, 0.8], radius=4, dims=(24, 24, 24))
        bc, msc = nd.nd_tune(pc, inputs.kuramoto_phases(2, 24 ** 3), 0.05, 4)
        assert (bc.tile + 8) * (bc.tile_y + 8) <= 1024 and msc > 0
        f = tmp_path / "t.txt"
        nd.nd_tune_save(str(f))
        assert len([l for l in f.read_text().splitlines() if not l.startswith("#")]) == 2
    finally:
        nd.nd_tune_clear()


def test_tune_ball_chooses_between_forms(nd):
    """The tuner times the plane-scatter form's tilings and the gather form's;
    a network created afterwards uses the winner and matches the oracle."""
    nd.nd_tune_clear()
    try:
        n1, P = 20, 6
        n = n1 ** 3
        prm = [0.1, 1.0, 0.45, 1.0, 0.05]
        p = nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, n, prm, radius=P, dims=(n1,) * 3)
        y0 = np.concatenate([inputs.kuramoto_phases(3, n), np.zeros(n)])
        best, ms = nd.nd_tune(p, y0, 0.05, 2)
        assert best.block in (256, 512, 1024) and ms > 0
        h = nd.nd_create(p)
        try:
            c = nd.nd_get_config(h)
            assert (c.block, c.tile, c.tile_y, c.tile_z) == (best.block, best.tile, best.tile_y, best.tile_z)
        finally:
            nd.nd_destroy(h)
        y, _, _ = nd.simulate(p, y0, 0.05, 4)
        ref, _, _ = O.run(O.ball(n1, P, prm, model=O.INERTIA), y0, 0.05, 4)
        assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-12
    finally:
        nd.nd_tune_clear()
