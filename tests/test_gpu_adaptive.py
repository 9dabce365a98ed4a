"""GPU parity of the on-device Dormand-Prince 5(4) stepping (step-size control
per ring) against the oracle's Dormand-Prince run, through the C ABI."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_19075_amd import inputs

pytestmark = pytest.mark.gpu

FHN = [0.05, 0.5, 0.1, math.pi / 2 - 0.1]
KUR = [0.2, 1.0, 1.46]
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


def net(nd, model, n, P, seed):
    if model == "kuramoto":
        return (nd.problem(nd.ND_KURAMOTO, nd.ND_RING, n, KUR, radius=P), O.ring(O.KURAMOTO, n, P, KUR),
                inputs.kuramoto_phases(seed, n), 1)
    if model == "fhn":
        return nd.problem(nd.ND_FHN, nd.ND_RING, n, FHN, radius=P), O.ring(O.FHN, n, P, FHN), inputs.fhn_circle(seed, n), 2
    y0 = np.concatenate([inputs.kuramoto_phases(seed, n), inputs.uniform_range(seed, inputs.TAG_MISC, n, -0.5, 0.5)])
    return (nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_RING, n, INERT, radius=P), O.ring(O.INERTIA, n, P, INERT), y0, 2)


def run_gpu(nd, probs, y0s, t_end, dt0, rtol, atol, max_steps=10 ** 7):
    hs = [nd.nd_create(p) for p in probs]
    try:
        for h, y0 in zip(hs, y0s):
            nd.nd_set_state(h, y0, on_device=0)
        st = nd.nd_run_adaptive(hs, t_end, dt0, rtol, atol, max_steps)
        ys = []
        for h, y0 in zip(hs, y0s):
            y = np.empty_like(y0)
            nd.nd_get_state(h, y, on_device=0)
            ys.append(y)
        return ys, st
    finally:
        for h in hs:
            nd.nd_destroy(h)


@pytest.mark.parametrize("model,n,P,t_end,rtol", [("kuramoto", 1000, 300, 5.0, 1e-8), ("fhn", 512, 179, 2.0, 1e-7),
                                                  ("inertia", 777, 200, 4.0, 1e-9), ("kuramoto", 37, 5, 3.0, 1e-6),
                                                  ("fhn", 1024, 358, 1.0, 1e-10)])
def test_adaptive_matches_oracle(nd, model, n, P, t_end, rtol):
    """Same accepted / rejected steps as the oracle's controller and the same state."""
    print(f"case adaptive {model} n={n} rtol={rtol}", flush=True)
    p, onet, y0, nv = net(nd, model, n, P, n + P)
    (y,), (st,) = run_gpu(nd, [p], [y0], [t_end], [1e-3], rtol, rtol * 1e-2)
    ref, t, acc, rej, hnext = O.run_dopri(onet, y0, t_end, rtol, rtol * 1e-2, 1e-3)
    print(f"  gpu {st.accepted}/{st.rejected}  oracle {acc}/{rej}", flush=True)
    assert st.accepted == acc and st.rejected == rej
    assert st.t == t == pytest.approx(t_end, abs=0)
    assert normwise(y, ref, nv) < 1e-10
    # the proposal follows err^(-1/5); at tight tolerances err itself carries the
    # rounding of the stage slopes, so only its leading digits are shared
    assert st.h_next == pytest.approx(hnext, rel=1e-4)


def test_adaptive_fixed_steps_match_oracle(nd):
    p, onet, y0, nv = net(nd, "inertia", 600, 150, 3)
    (y,), (st,) = run_gpu(nd, [p], [y0], [2.0], [0.01], -1.0, 0.0)
    ref, t, acc, rej, _ = O.run_dopri(onet, y0, 2.0, -1.0, 0.0, 0.01)
    assert st.accepted == acc == 200 and st.rejected == rej == 0
    assert normwise(y, ref, nv) < 1e-12


def test_adaptive_batch_of_rings_each_controls_its_step(nd):
    """Five rings with different sizes, radii, horizons and initial steps in one
    launch; each matches its own oracle run."""
    cases = [(900, 250, 4.0, 1e-3), (128, 20, 1.5, 1e-2), (1024, 511, 2.5, 1e-4), (300, 1, 3.0, 1e-3),
             (64, 31, 0.0, 1e-3)]
    probs, onets, y0s = [], [], []
    for i, (n, P, _, _) in enumerate(cases):
        p, onet, y0, _ = net(nd, "kuramoto", n, P, 40 + i)
        probs.append(p)
        onets.append(onet)
        y0s.append(y0)
    ys, st = run_gpu(nd, probs, y0s, [c[2] for c in cases], [c[3] for c in cases], 1e-8, 1e-10)
    for y, s, onet, y0, c in zip(ys, st, onets, y0s, cases):
        ref, t, acc, rej, _ = O.run_dopri(onet, y0, c[2], 1e-8, 1e-10, c[3])
        assert (s.accepted, s.rejected) == (acc, rej)
        assert s.t == t
        assert np.max(np.abs(y - ref)) / max(1.0, np.max(np.abs(ref))) < 1e-10


def test_adaptive_step_budget(nd):
    p, onet, y0, nv = net(nd, "fhn", 256, 50, 7)
    (y,), (st,) = run_gpu(nd, [p], [y0], [100.0], [1e-3], 1e-8, 1e-10, max_steps=25)
    ref, t, acc, rej, _ = O.run_dopri(onet, y0, 100.0, 1e-8, 1e-10, 1e-3, max_steps=25)
    assert st.accepted + st.rejected == 25 == acc + rej
    # the time reached is the sum of the accepted steps, whose sizes agree to the
    # leading digits of the error estimate (see above)
    assert st.t < 100.0 and st.t == pytest.approx(t, rel=1e-6)
    assert normwise(y, ref, nv) < 1e-6


def test_adaptive_rejects_unsupported(nd):
    f32 = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, 500, KUR, precision=nd.ND_FP32_BULK, radius=10)
    cube = nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, 9 ** 3, KUR, radius=1, dims=(9, 9, 9))
    for p in (f32, cube):
        h = nd.nd_create(p)
        try:
            with pytest.raises(nd.NDError) as ei:
                nd.nd_run_adaptive([h], [1.0], [1e-3], 1e-6, 1e-9)
            assert ei.value.status == nd.ND_ERR_UNSUPPORTED
        finally:
            nd.nd_destroy(h)
    h = nd.nd_create(nd.problem(nd.ND_KURAMOTO, nd.ND_RING, 500, KUR, radius=10))
    try:
        with pytest.raises(nd.NDError):
            nd.nd_run_adaptive([h], [1.0], [1e-3], 1e-6, 0.0)  # atol must be > 0 with rtol > 0
    finally:
        nd.nd_destroy(h)


# ---------------------------------------------------------------- dense output
@pytest.mark.parametrize("model,n,P,t_end,rtol,t_out", [("kuramoto", 1000, 300, 5.0, 1e-8, 0.1),
                                                        ("fhn", 512, 179, 2.0, 1e-7, 0.05),
                                                        ("inertia", 777, 200, 4.0, 1e-9, 0.3)])
def test_dense_output_matches_oracle(nd, model, n, P, t_end, rtol, t_out):
    """R and the state at every output time from the continuous extension, and
    the same steps as without outputs."""
    print(f"case dense {model} n={n} t_out={t_out}", flush=True)
    p, onet, y0, nv = net(nd, model, n, P, 5 * n + P)
    h = nd.nd_create(p)
    try:
        nd.nd_set_state(h, y0, on_device=0)
        (st,), R, Y = nd.nd_run_adaptive_dense([h], [t_end], [1e-3], rtol, rtol * 1e-2, t_out, state_len=nv * n)
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
    finally:
        nd.nd_destroy(h)
    ref, t, acc, rej, _, Rref, Yref = O.run_dopri_dense(onet, y0, t_end, rtol, rtol * 1e-2, 1e-3, t_out, states=True)
    assert (st.accepted, st.rejected) == (acc, rej) and st.t == t
    K = int(np.floor(t_end / t_out))
    assert R.shape == (1, K + 1) and not np.any(np.isnan(R))
    # the step sizes agree to the rounding of err^(-1/5), so the outputs, which
    # interpolate inside those steps, are held to 1e-9 (the interpolant's own
    # error at these tolerances is ~1e-8)
    assert np.max(np.abs(R[0] - Rref)) < 1e-9
    Yg = Y[0].reshape(K + 1, nv * n)
    for k in range(K + 1):
        assert normwise(Yg[k], Yref[k], nv) < 1e-9
    assert normwise(y, ref, nv) < 1e-10


def test_dense_output_batch_and_budget(nd):
    """Rings with different horizons in one call: each gets its own number of
    outputs (the rest of its row untouched by the run reads NaN); a ring whose
    step budget runs out leaves its later outputs NaN."""
    cases = [(600, 100, 3.0), (256, 40, 1.2), (1024, 300, 0.0)]
    probs, onets, y0s = [], [], []
    for i, (n, P, _) in enumerate(cases):
        p, onet, y0, _ = net(nd, "kuramoto", n, P, 70 + i)
        probs.append(p)
        onets.append(onet)
        y0s.append(y0)
    hs = [nd.nd_create(p) for p in probs]
    try:
        for h, y0 in zip(hs, y0s):
            nd.nd_set_state(h, y0, on_device=0)
        st, R, _ = nd.nd_run_adaptive_dense(hs, [c[2] for c in cases], [1e-3] * 3, 1e-8, 1e-10, 0.2)
    finally:
        for h in hs:
            nd.nd_destroy(h)
    assert R.shape == (3, 16)
    for i, (c, onet, y0) in enumerate(zip(cases, onets, y0s)):
        _, _, acc, rej, _, Rref, _ = O.run_dopri_dense(onet, y0, c[2], 1e-8, 1e-10, 1e-3, 0.2)
        K = int(np.floor(c[2] / 0.2))
        assert (st[i].accepted, st[i].rejected) == (acc, rej)
        assert np.max(np.abs(R[i, :K + 1] - Rref)) < 1e-9
        assert np.all(np.isnan(R[i, K + 1:]))
    p, onet, y0, _ = net(nd, "fhn", 300, 60, 9)
    h = nd.nd_create(p)
    try:
        nd.nd_set_state(h, y0, on_device=0)
        (s1,), R1, _ = nd.nd_run_adaptive_dense([h], [50.0], [1e-3], 1e-8, 1e-10, 0.5, max_steps=40)
    finally:
        nd.nd_destroy(h)
    _, t, _, _, _, Rref, _ = O.run_dopri_dense(onet, y0, 50.0, 1e-8, 1e-10, 1e-3, 0.5, max_steps=40)
    reached = ~np.isnan(Rref)
    assert s1.t < 50.0 and np.array_equal(~np.isnan(R1[0]), reached)
    assert np.max(np.abs(R1[0][reached] - Rref[reached])) < 1e-8


def test_dense_output_rejects_bad_arguments(nd):
    h = nd.nd_create(nd.problem(nd.ND_KURAMOTO, nd.ND_RING, 100, KUR, radius=10))
    try:
        with pytest.raises(nd.NDError):
            nd.nd_run_adaptive_dense([h], [1.0], [1e-3], 1e-6, 1e-9, 0.0)
        hs = (nd._c_vp * 1)(h)
        te = (nd._c_dbl * 1)(1.0)
        d0 = (nd._c_dbl * 1)(1e-3)
        st = (nd.nd_adaptive_stats * 1)()
        R = np.empty(5)
        rc = nd._lib.nd_run_adaptive_dense(hs, 1, te, d0, 1e-6, 1e-9, 1000, 0.1, R.ctypes.data, 5, None, 0, st, None)
        assert rc == nd.ND_ERR_INVALID_ARG  # 11 outputs do not fit r_stride 5
    finally:
        nd.nd_destroy(h)


# ------------------------------------------------- rings beyond one workgroup
@pytest.mark.parametrize("model,n,P,t_end,rtol", [("kuramoto", 5000, 1000, 2.0, 1e-8), ("fhn", 2049, 700, 1.0, 1e-7),
                                                  ("inertia", 3000, 500, 3.0, 1e-9), ("kuramoto", 1025, 3, 1.5, 1e-6)])
def test_tiled_adaptive_matches_oracle(nd, model, n, P, t_end, rtol):
    """Rings larger than one workgroup take the tiled path: the same accepted and
    rejected steps as the oracle's controller and the same state."""
    print(f"case tiled adaptive {model} n={n}", flush=True)
    p, onet, y0, nv = net(nd, model, n, P, n + 3 * P)
    (y,), (st,) = run_gpu(nd, [p], [y0], [t_end], [1e-3], rtol, rtol * 1e-2)
    ref, t, acc, rej, hnext = O.run_dopri(onet, y0, t_end, rtol, rtol * 1e-2, 1e-3)
    print(f"  gpu {st.accepted}/{st.rejected}  oracle {acc}/{rej}", flush=True)
    assert st.accepted == acc and st.rejected == rej
    assert st.t == t
    assert normwise(y, ref, nv) < 1e-10
    assert st.h_next == pytest.approx(hnext, rel=1e-4)


def test_tiled_adaptive_long_ring_and_mixed_batch(nd):
    """Rings of more than 2048 tiles of 512 take their tile offsets from a launch
    of their own, shorter rings scan them inside the RHS launch: an FHN ring of
    2048 * 512 + 1000 elements alone and in a batch with a ring of 3000, each
    against the oracle's accepted and rejected steps and state."""
    n, P = 2048 * 512 + 1000, 4
    print(f"case tiled long ring n={n}", flush=True)
    p, onet, y0, nv = net(nd, "fhn", n, P, 12)
    ref, t, acc, rej, _ = O.run_dopri(onet, y0, 0.2, 1e-6, 1e-8, 1e-3)
    (y,), (st,) = run_gpu(nd, [p], [y0], [0.2], [1e-3], 1e-6, 1e-8)
    assert (st.accepted, st.rejected) == (acc, rej) and st.t == t
    assert normwise(y, ref, nv) < 1e-10
    p2, onet2, y02, _ = net(nd, "fhn", 3000, 900, 13)
    ref2, t2, acc2, rej2, _ = O.run_dopri(onet2, y02, 0.3, 1e-6, 1e-8, 1e-3)
    ys, sts = run_gpu(nd, [p, p2], [y0, y02], [0.2, 0.3], [1e-3, 1e-3], 1e-6, 1e-8)
    assert (sts[0].accepted, sts[0].rejected) == (acc, rej)
    assert (sts[1].accepted, sts[1].rejected) == (acc2, rej2) and sts[1].t == t2
    assert normwise(ys[0], ref, nv) < 1e-10 and normwise(ys[1], ref2, nv) < 1e-10


def test_tiled_adaptive_batch_fixed_steps_and_budget(nd):
    """A batch with a small and two large rings (all on the tiled path), one of
    them with t_end = 0; then fixed steps, and a step budget."""
    cases = [(700, 100, 2.0, 1e-3), (4000, 1300, 1.0, 1e-2), (2500, 30, 0.0, 1e-3)]
    probs, onets, y0s = [], [], []
    for i, (n, P, _, _) in enumerate(cases):
        p, onet, y0, _ = net(nd, "kuramoto", n, P, 90 + i)
        probs.append(p)
        onets.append(onet)
        y0s.append(y0)
    ys, st = run_gpu(nd, probs, y0s, [c[2] for c in cases], [c[3] for c in cases], 1e-8, 1e-10)
    for y, s, onet, y0, c in zip(ys, st, onets, y0s, cases):
        ref, t, acc, rej, _ = O.run_dopri(onet, y0, c[2], 1e-8, 1e-10, c[3])
        assert (s.accepted, s.rejected) == (acc, rej) and s.t == t
        assert np.max(np.abs(y - ref)) / max(1.0, np.max(np.abs(ref))) < 1e-10
    p, onet, y0, nv = net(nd, "fhn", 3000, 900, 4)
    (y,), (s,) = run_gpu(nd, [p], [y0], [0.5], [0.01], -1.0, 0.0)
    ref, t, acc, rej, _ = O.run_dopri(onet, y0, 0.5, -1.0, 0.0, 0.01)
    assert s.accepted == acc == 50 and s.rejected == 0
    assert normwise(y, ref, nv) < 1e-12
    (y,), (s,) = run_gpu(nd, [p], [y0], [100.0], [1e-3], 1e-8, 1e-10, max_steps=21)
    ref, t, acc, rej, _ = O.run_dopri(onet, y0, 100.0, 1e-8, 1e-10, 1e-3, max_steps=21)
    assert s.accepted + s.rejected == 21 == acc + rej
    assert s.t == pytest.approx(t, rel=1e-6) and normwise(y, ref, nv) < 1e-6


@pytest.mark.parametrize("case", ["ring", "links"])
def test_tiled_dense_output_matches_oracle(nd, case):
    """Dense output on the tiled path (a ring of 3000, a compressed small-world
    matrix): R and the state at every output time, as the oracle's."""
    print(f"case tiled dense {case}", flush=True)
    if case == "ring":
        p, onet, y0, nv = net(nd, "kuramoto", 3000, 700, 31)
        t_end, rtol, t_out = 2.0, 1e-8, 0.1
    else:
        p, onet, y0, nv = links_net(nd, "fhn", "small_world", 32)
        t_end, rtol, t_out = 1.0, 1e-7, 0.05
    n = y0.size // nv
    h = nd.nd_create(p)
    try:
        nd.nd_set_state(h, y0, on_device=0)
        (st,), R, Y = nd.nd_run_adaptive_dense([h], [t_end], [1e-3], rtol, rtol * 1e-2, t_out, state_len=nv * n)
        y = np.empty_like(y0)
        nd.nd_get_state(h, y, on_device=0)
    finally:
        nd.nd_destroy(h)
    ref, t, acc, rej, _, Rref, Yref = O.run_dopri_dense(onet, y0, t_end, rtol, rtol * 1e-2, 1e-3, t_out, states=True)
    assert (st.accepted, st.rejected) == (acc, rej) and st.t == t
    K = int(np.floor(t_end / t_out))
    assert not np.any(np.isnan(R[0]))
    assert np.max(np.abs(R[0] - Rref)) < 1e-9
    Yg = Y[0].reshape(K + 1, nv * n)
    for k in range(K + 1):
        assert normwise(Yg[k], Yref[k], nv) < 1e-9
    assert normwise(y, ref, nv) < 1e-10


def links_net(nd, model, kind, seed):
    if kind == "small_world":
        n = 2000
        rp, col = inputs.small_world_links(seed, n, 25, 60)
    elif kind == "random":
        n = 300
        rp0, col0 = inputs.random_links(seed, n, 0.05)
        rows = [col0[rp0[i]:rp0[i + 1]] if i % 7 else col0[:0] for i in range(n)]  # some rows empty
        rp = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64)
        col = np.concatenate(rows).astype(np.int32)
    else:
        n = 12 * 11 * 10
        rp, col = inputs.lattice_ball_links(12, 11, 10, 2)
    if model == "kuramoto":
        code, ocode, prm, y0, nv = nd.ND_KURAMOTO, O.KURAMOTO, KUR, inputs.kuramoto_phases(seed, n), 1
    elif model == "fhn":
        code, ocode, prm, y0, nv = nd.ND_FHN, O.FHN, FHN, inputs.fhn_circle(seed, n), 2
    else:
        code, ocode, prm, nv = nd.ND_KURAMOTO_INERTIA, O.INERTIA, INERT, 2
        y0 = np.concatenate([inputs.kuramoto_phases(seed, n), inputs.uniform_range(seed, inputs.TAG_MISC, n, -0.5, 0.5)])
    return (nd.problem(code, nd.ND_LINKS, n, prm, row_ptr=rp, col=col), O.links(ocode, n, rp, col, np.array(prm)),
            y0, nv)


@pytest.mark.parametrize("model,kind,t_end,rtol", [("fhn", "small_world", 1.0, 1e-7), ("kuramoto", "random", 3.0, 1e-8),
                                                   ("inertia", "lattice", 2.0, 1e-9)])
def test_adaptive_on_compressed_coupling_matrices(nd, model, kind, t_end, rtol):
    """Dormand-Prince on arbitrary coupling matrices (the tiled path with the
    compressed rows): the oracle's steps and state."""
    print(f"case adaptive links {model} {kind}", flush=True)
    p, onet, y0, nv = links_net(nd, model, kind, 13)
    (y,), (st,) = run_gpu(nd, [p], [y0], [t_end], [1e-3], rtol, rtol * 1e-2)
    ref, t, acc, rej, _ = O.run_dopri(onet, y0, t_end, rtol, rtol * 1e-2, 1e-3)
    print(f"  gpu {st.accepted}/{st.rejected}  oracle {acc}/{rej}", flush=True)
    assert (st.accepted, st.rejected) == (acc, rej) and st.t == t
    assert normwise(y, ref, nv) < 1e-10
