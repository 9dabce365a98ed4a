"""Runtime behaviour of the C ABI on the GPU: nd_run is enqueued without a host
wait and ordered on the caller's stream, a network whose state turns
non-finite is reported by the next synchronising call (and only that network),
the server fails such a request alone, and Dormand-Prince runs stop promptly on
a non-finite state."""
import math
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_19075_amd import inputs

pytestmark = pytest.mark.gpu
FHN_PRM = [0.05, 0.5, 0.1, math.pi / 2 - 0.1]
HH_PRM = [1.0, 120.0, 36.0, 0.3, 50.0, -77.0, -54.387, 0.0, 0.0, 2.0]
INERT = [0.0, 0.5, 0.45, 1.0, 0.05]


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_19075_amd import nd as _nd
    return _nd


def test_run_returns_before_the_device_and_is_stream_ordered(nd):
    """nd_run on torch's current stream returns long before the device work it
    enqueued ends; a torch op enqueued after it on the same stream, with no host
    wait in between, sees the final state.  The lattice (120^3, h = 4) starts
    from a plane wave, which rotates rigidly at
    -sin(alpha) (prod_a D_4(theta_a) - 1) / 728 (D_H the Dirichlet kernel), so
    the expected state holds at this size without the oracle's O(N L) sums."""
    import torch
    n1, h, alpha, steps, q = 120, 4, 0.8, 40, (2, -1, 3)
    n = n1 ** 3

    def dirichlet(H, th):
        return 2 * H + 1 if th == 0 else math.sin((H + 0.5) * th) / math.sin(th / 2)

    idx = np.arange(n, dtype=np.int64)
    y0 = (2 * math.pi / n1) * (q[0] * (idx % n1) + q[1] * ((idx // n1) % n1) + q[2] * (idx // (n1 * n1)))
    prod = 1.0
    for qa in q:
        prod *= dirichlet(h, 2 * math.pi * qa / n1)
    om = -math.sin(alpha) * (prod - 1) / 728
    p = nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, n, [0.0, 1.0, alpha], radius=h, dims=(n1,) * 3)
    st = torch.cuda.current_stream()
    hd = nd.nd_create(p)
    try:
        dev = torch.from_numpy(y0).cuda()
        nd.nd_set_state(hd, dev, stream=st)
        nd.nd_run(hd, 0.05, 2, stream=st)  # warm the kernels
        nd.nd_set_state(hd, dev, stream=st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        t0 = time.perf_counter()
        nd.nd_run(hd, 0.05, steps, stream=st)
        host_s = time.perf_counter() - t0
        out = torch.empty_like(dev)
        nd.nd_get_state(hd, out, stream=st)   # device-to-device, stream ordered
        doubled = out * 2.0                    # a torch op on the same stream, no host wait
        e1.record(st)
        torch.cuda.synchronize()
        gpu_s = e0.elapsed_time(e1) / 1e3
        got = doubled.cpu().numpy() / 2.0
    finally:
        nd.nd_destroy(hd)
    assert host_s < 0.5 * gpu_s, (host_s, gpu_s)
    err = np.max(np.abs(got - y0 - om * 0.05 * steps))
    assert err < 1e-12 + 1e-14 * np.max(np.abs(y0)), err


def _cases(nd):
    rp, col, w = inputs.random_out_graph(21, 500, 10)
    sw = inputs.small_world_links(22, 900, 8, 20)
    return {
        "ring_resident": (nd.problem(nd.ND_KURAMOTO, nd.ND_RING, 1000, [0.0, 1.0, 1.46], radius=200),
                          inputs.kuramoto_phases(23, 1000), 0.01),
        "ring_tiled": (nd.problem(nd.ND_FHN, nd.ND_RING, 9000, FHN_PRM, radius=3000), inputs.fhn_circle(24, 9000),
                       0.01),
        "cube": (nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, 14 ** 3, [0.0, 1.0, 0.8], radius=3, dims=(14,) * 3),
                 inputs.kuramoto_phases(25, 14 ** 3), 0.05),
        "ball": (nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, 12 ** 3, INERT, radius=2, dims=(12,) * 3),
                 np.concatenate([inputs.kuramoto_phases(26, 12 ** 3), np.zeros(12 ** 3)]), 0.05),
        # radius 3: the plane-scatter form
        "ball_scatter": (nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, 13 ** 3, INERT, radius=3, dims=(13,) * 3),
                         np.concatenate([inputs.kuramoto_phases(28, 13 ** 3), np.zeros(13 ** 3)]), 0.05),
        "links": (nd.problem(nd.ND_FHN, nd.ND_LINKS, 900, FHN_PRM, row_ptr=sw[0], col=sw[1]),
                  inputs.fhn_circle(27, 900), 0.01),
        "csr": (nd.problem(nd.ND_HH, nd.ND_CSR, 500, HH_PRM, row_ptr=rp, col=col, weight=w,
                           per_elem=inputs.hh_iapp(21, 500)), inputs.hh_state(21, 500), 0.01),
    }


def test_destroy_waits_for_that_network_only(nd):
    """nd_destroy and nd_set_config wait for the network's own work (its event)
    and return its buffers to the stream-ordered pool; long torch work queued on
    another stream keeps running meanwhile.  A network created afterwards reuses
    pool memory and still matches its oracle run."""
    import torch
    p = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, 1024, [0.0, 1.0, 1.46], radius=256)
    y0 = inputs.kuramoto_phases(31, 1024)
    h = nd.nd_create(p)
    nd.nd_set_state(h, y0, on_device=0)
    nd.nd_run(h, 0.01, 10)
    nd.nd_sync(h)
    other = torch.cuda.Stream()
    a = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(other):
        e0.record()
        b = a
        for _ in range(60):
            b = torch.mm(b, a) * 1e-3
        e1.record()
    t0 = time.perf_counter()
    c = nd.nd_get_config(h)
    nd.nd_set_config(h, c)   # rebuilds the per-work-item buffers
    nd.nd_destroy(h)
    host_s = time.perf_counter() - t0
    other.synchronize()
    gpu_s = e0.elapsed_time(e1) / 1e3
    print(f"destroy {host_s * 1e3:.2f} ms while the other stream ran {gpu_s * 1e3:.1f} ms")
    assert gpu_s > 0.05 and host_s < 0.25 * gpu_s
    y, _, _ = nd.simulate(p, y0, 0.01, 10)
    ref, _, _ = O.run(O.ring(O.KURAMOTO, 1024, 256, [0.0, 1.0, 1.46]), y0, 0.01, 10)
    assert np.max(np.abs(y - ref)) < 1e-12


@pytest.mark.parametrize("kind", ["ring_resident", "ring_tiled", "cube", "ball", "ball_scatter", "links", "csr"])
def test_nonfinite_state_is_reported_for_that_network_only(nd, kind):
    """A NaN planted in one network's device state: after a batched run the next
    synchronising call on it returns ND_ERR_NUMERIC, the other network of the
    batch is unaffected (bitwise equal to its run alone), and a new state clears
    the flag."""
    import torch
    p, y0, dt = _cases(nd)[kind]
    steps = 7
    bad = y0.copy()
    bad[len(bad) // 3] = np.nan
    ha, hb = nd.nd_create(p), nd.nd_create(p)
    try:
        nd.nd_set_state(ha, torch.from_numpy(y0).cuda())
        nd.nd_set_state(hb, torch.from_numpy(bad).cuda())
        nd.nd_run_batch([ha, hb], [dt, dt], [steps, steps])
        ya = np.empty_like(y0)
        nd.nd_get_state(ha, ya, on_device=0)
        nd.nd_sync(ha)
        yb = np.empty_like(y0)
        with pytest.raises(nd.NDError) as ei:
            nd.nd_get_state(hb, yb, on_device=0)
        assert ei.value.status == nd.ND_ERR_NUMERIC
        assert not np.all(np.isfinite(yb))
        with pytest.raises(nd.NDError) as ei:
            nd.nd_sync(hb)
        assert ei.value.status == nd.ND_ERR_NUMERIC
        nd.nd_set_state(hb, y0, on_device=0)
        nd.nd_sync(hb)
        nd.nd_run(hb, dt, steps)
        ys = np.empty_like(y0)
        nd.nd_get_state(hb, ys, on_device=0)
    finally:
        nd.nd_destroy(ha)
        nd.nd_destroy(hb)
    assert np.array_equal(ya, ys)


def test_server_fails_a_diverging_request_alone(nd):
    """An FHN request with a step far beyond the model's stability limit blows up
    within a few steps; the server fails it at the next chunk boundary with
    ND_ERR_NUMERIC (well before its horizon) while the request beside it
    completes with the result of its run alone."""
    n, P = 4000, 1400
    y0 = inputs.fhn_circle(31, n)
    good = nd.problem(nd.ND_FHN, nd.ND_RING, n, FHN_PRM, radius=P)
    s = nd.nd_server_create(1 << 30, max_slots=8, chunk_steps=16)
    try:
        rb = nd.nd_server_submit(s, good, y0, 2.0, 5000)
        rg = nd.nd_server_submit(s, good, y0, 0.01, 100)
        for _ in range(1000):
            if nd.nd_server_pump(s) == 0:
                break
        ib, ig = nd.nd_server_info(s, rb), nd.nd_server_info(s, rg)
        assert ib.state == nd.ND_REQ_FAILED and ib.status == nd.ND_ERR_NUMERIC
        assert ib.steps_done < 5000
        assert ig.state == nd.ND_REQ_DONE
        y = np.empty_like(y0)
        nd.nd_server_result(s, rg, y)
    finally:
        nd.nd_server_destroy(s)
    alone, _, _ = nd.simulate(good, y0, 0.01, 100)
    assert np.array_equal(y, alone)


@pytest.mark.parametrize("n", [300, 4000])
def test_adaptive_run_stops_on_a_nonfinite_state(nd, n):
    """Dormand-Prince on a ring whose state holds a NaN: the non-finite error
    estimate stops the run at the first attempt (one workgroup per ring for
    n <= 1024, the tiled path above) instead of rejecting until max_steps; the
    other ring of the batch finishes, and the call returns ND_ERR_NUMERIC with
    the failed network marked."""
    P = n // 5
    p = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, n, [0.0, 1.0, 1.46], radius=P)
    y0 = inputs.kuramoto_phases(32, n)
    bad = y0.copy()
    bad[7] = np.nan
    hs = [nd.nd_create(p), nd.nd_create(p)]
    try:
        nd.nd_set_state(hs[0], y0, on_device=0)
        nd.nd_set_state(hs[1], bad, on_device=0)
        t0 = time.perf_counter()
        with pytest.raises(nd.NDError) as ei:
            nd.nd_run_adaptive(hs, [1.0, 1.0], [1e-3, 1e-3], 1e-8, 1e-10, max_steps=10 ** 7)
        wall = time.perf_counter() - t0
        st = ei.value.stats
    finally:
        for h in hs:
            nd.nd_destroy(h)
    assert ei.value.status == nd.ND_ERR_NUMERIC
    assert wall < 30.0
    assert st[1].failed == 1 and st[1].accepted == 0 and st[1].t == 0.0
    assert st[0].failed == 0 and st[0].t == 1.0
    _, t, acc, rej, _ = O.run_dopri(O.ring(O.KURAMOTO, n, P, [0.0, 1.0, 1.46]), y0, 1.0, 1e-8, 1e-10, 1e-3)
    assert (st[0].accepted, st[0].rejected) == (acc, rej)
