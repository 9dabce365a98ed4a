"""GPU runs at the largest sizes the library accepts (2^29 - 1 elements for
rings and lattices; the paper's workloads reach 10^8 elements), checked by
closed forms and by properties that hold at any size: the oracle's O(N P)
window sums cannot follow at these sizes."""
import math

import numpy as np
import pytest

from paper_2410_19075_amd import inputs

pytestmark = pytest.mark.gpu

NMAX = 2 ** 29 - 1  # odd: every tiling ends in a ragged tail


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_19075_amd import nd as _nd
    return _nd


def test_twisted_state_at_the_maximum_ring(nd):
    """Kuramoto ring of 2^29 - 1 elements, P = n/4: a 3-twisted state rotates
    rigidly at -sin(alpha) C / P, C = sum_{k=1..P} cos(k theta) (closed form),
    and its order parameter stays 0."""
    n, P, q, alpha = NMAX, NMAX // 4, 3, 1.46
    print(f"case twisted ring n={n} P={P} q={q}", flush=True)
    y0 = inputs.twisted_state(n, q)
    th = 2 * math.pi * q / n
    csum = math.sin((P + 0.5) * th) / (2 * math.sin(th / 2)) - 0.5
    om = -math.sin(alpha) * csum / P
    dt, steps = 0.01, 4
    p = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, n, [0.0, 1.0, alpha], radius=P)
    y, R, _ = nd.simulate(p, y0, dt, steps, record_every=2)
    y -= y0
    y -= om * dt * steps
    assert np.max(np.abs(y)) < 1e-12
    assert np.max(np.abs(R)) < 1e-12


@pytest.mark.parametrize("model", ["kur", "fhn"])
def test_translation_equivariance_at_large_rings(nd, model):
    """A ring is translation invariant: integrating the state rotated by s
    gives the rotated result (to the FP64 bar), whatever the tiling.  A wrong
    window offset or tile boundary anywhere breaks it.  Kuramoto at 2^29 - 1
    elements, FitzHugh-Nagumo at 2^28 + 3 (two variables per element), with a
    shift that is no multiple of any tile."""
    if model == "kur":
        n = NMAX
        P = int(0.3 * n)
        p = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, n, [0.0, 1.0, 1.46], radius=P)
        y0 = inputs.kuramoto_phases(11, n)
        nv = 1
    else:
        n = 2 ** 28 + 3
        P = int(0.35 * n)
        p = nd.problem(nd.ND_FHN, nd.ND_RING, n, [0.05, 0.5, 0.1, math.pi / 2 - 0.1], radius=P)
        y0 = inputs.fhn_circle(12, n)
        nv = 2
    s = 12345677
    print(f"case equivariance {model} n={n} P={P} s={s}", flush=True)
    a, Ra, _ = nd.simulate(p, y0, 0.01, 2, record_every=1)
    y0 = np.roll(y0.reshape(nv, n), s, axis=1).reshape(-1)
    b, Rb, _ = nd.simulate(p, y0, 0.01, 2, record_every=1)
    del y0
    a = np.roll(a.reshape(nv, n), s, axis=1)
    b = b.reshape(nv, n)
    for v in range(nv):
        assert np.max(np.abs(a[v] - b[v])) <= 1e-12 * np.max(np.abs(a[v]))
    assert np.max(np.abs(Ra - Rb)) < 1e-12


def test_plane_wave_at_the_largest_cube(nd):
    """3D Kuramoto lattice 800^3 (5.12e8 elements, the largest cube below
    2^29), h = 4: a plane wave rotates rigidly at
    -sin(alpha) (prod_a D_4(theta_a) - 1) / 728 with D_H the Dirichlet kernel."""
    n1, h, alpha, q = 800, 4, 0.8, (3, -2, 7)
    print(f"case plane wave {n1}^3 q={q}", flush=True)

    def dirichlet(H, th):
        return 2 * H + 1 if th == 0 else math.sin((H + 0.5) * th) / math.sin(th / 2)

    idx = np.arange(n1 ** 3, dtype=np.int64)
    y0 = (2 * math.pi / n1) * (q[0] * (idx % n1) + q[1] * ((idx // n1) % n1) + q[2] * (idx // (n1 * n1)))
    del idx
    prod = 1.0
    for qa in q:
        prod *= dirichlet(h, 2 * math.pi * qa / n1)
    om = -math.sin(alpha) * (prod - 1) / 728
    dt, steps = 0.05, 2
    p = nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, n1 ** 3, [0.0, 1.0, alpha], radius=h, dims=(n1, n1, n1))
    y, R, _ = nd.simulate(p, y0, dt, steps, record_every=1)
    bound = 1e-12 + 1e-14 * np.max(np.abs(y0))
    y -= y0
    y -= om * dt * steps
    assert np.max(np.abs(y)) < bound
    assert np.max(np.abs(R)) < 1e-12
