"""The entry point that allocates nothing (nd_run_batch_noalloc) against
nd_run_batch on the same inputs: bitwise equal states and order parameters on
two calls in a row, the second with a smaller batch, and its size limits."""
import math

import numpy as np
import pytest

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


def cases(nd, small):
    if small:
        return [(nd.problem(nd.ND_FHN, nd.ND_RING, 3000, FHN_PRM, radius=1000), inputs.fhn_circle(61, 3000), 0.01)]
    return [
        (nd.problem(nd.ND_FHN, nd.ND_RING, 9000, FHN_PRM, radius=3000), inputs.fhn_circle(62, 9000), 0.01),
        (nd.problem(nd.ND_KURAMOTO, nd.ND_RING, 1000, [0.0, 1.0, 1.46], radius=250), inputs.kuramoto_phases(63, 1000),
         0.01),
        (nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, 20 ** 3, [0.0, 1.0, 0.8], radius=3, dims=(20,) * 3),
         inputs.kuramoto_phases(64, 20 ** 3), 0.05),
        (nd.problem(nd.ND_FHN, nd.ND_RING, 9000, FHN_PRM, precision=1, radius=2500), inputs.fhn_circle(65, 9000),
         0.01),
        # a ball in plane-scatter form (radius 3)
        (nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, 14 ** 3, [0.0, 0.5, 0.45, 1.0, 0.05], radius=3,
                    dims=(14,) * 3),
         np.concatenate([inputs.kuramoto_phases(66, 14 ** 3), np.zeros(14 ** 3)]), 0.05),
    ]


def run_both(nd, cs, steps, re):
    """nd_run_batch on one set of handles, nd_run_batch_noalloc on another
    (whose observable buffers an earlier run sized); returns both results."""
    obs = [nd.observe(re, -1)] * len(cs)
    out = []
    for noalloc in (False, True):
        hs = [nd.nd_create(p) for p, _, _ in cs]
        try:
            if noalloc:  # size the R buffers with an ordinary run first
                for h, (_, y0, _) in zip(hs, cs):
                    nd.nd_set_state(h, y0, on_device=0)
                nd.nd_run_batch(hs, [dt for _, _, dt in cs], [steps] * len(cs), obs)
            for h, (_, y0, _) in zip(hs, cs):
                nd.nd_set_state(h, y0, on_device=0)
            run = nd.nd_run_batch_noalloc if noalloc else nd.nd_run_batch
            run(hs, [dt for _, _, dt in cs], [steps] * len(cs), obs)
            res = []
            for h, (_, y0, _) in zip(hs, cs):
                y = np.empty_like(y0)
                nd.nd_get_state(h, y, on_device=0)
                R = np.empty(steps // re + 1)
                nd.nd_get_observables(h, R=R, on_device=0)
                res.append((y, R))
            out.append(res)
        finally:
            for h in hs:
                nd.nd_destroy(h)
    return out


def test_noalloc_equals_batch_twice_second_smaller(nd):
    print("case noalloc: mixed batch, then one smaller ring", flush=True)
    for small, steps in ((False, 150), (True, 70)):
        ref, got = run_both(nd, cases(nd, small), steps, 1)
        for (ya, Ra), (yb, Rb) in zip(ref, got):
            assert np.array_equal(ya, yb)
            assert np.array_equal(Ra, Rb)


def test_noalloc_limits(nd):
    print("case noalloc limits", flush=True)
    p, y0, dt = cases(nd, True)[0]
    h = nd.nd_create(p)
    try:
        nd.nd_set_state(h, y0, on_device=0)
        # R buffers never sized for this handle: refused, nothing enqueued
        with pytest.raises(nd.NDError) as ei:
            nd.nd_run_batch_noalloc([h], [dt], [10], [nd.observe(1, -1)])
        assert ei.value.status == nd.ND_ERR_INVALID_ARG
        # more networks than the fixed tables hold
        with pytest.raises(nd.NDError) as ei:
            nd.nd_run_batch_noalloc([h] * (nd.ND_NOALLOC_MAX_NETS + 1), [dt] * (nd.ND_NOALLOC_MAX_NETS + 1),
                                    [1] * (nd.ND_NOALLOC_MAX_NETS + 1))
        assert ei.value.status == nd.ND_ERR_INVALID_ARG
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
        assert np.array_equal(y, y0)
    finally:
        nd.nd_destroy(h)
