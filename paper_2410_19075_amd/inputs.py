"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds random-number generation and data layout only (no model
arithmetic), so both the HIP path and the CPU oracle receive bit-identical
inputs from it.  Every draw comes from SplitMix64 (Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) used as a
counter-based generator: value i of stream (seed, tag) is
mix(base + (i + 1) * GAMMA) with base = mix(seed * GAMMA + tag), and a uniform
double in [0, 1) is (x >> 11) * 2^-53.

Shapes follow the workloads the paper studies (Sec. IV): rings of ~10^3 and
more oscillators with non-local radius P, periodic 3D lattices with a
coherent patch, and sparse directed neuron graphs.
"""
import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream tags: one independent stream per quantity
TAG_PHASE, TAG_FHN, TAG_PATCH, TAG_HH_STATE, TAG_HH_IAPP, TAG_GRAPH, TAG_WEIGHT, TAG_MISC, TAG_LINKS = range(1, 10)


def _mix(z):
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def raw(seed, tag, n, offset=0):
    """n raw 64-bit draws of stream (seed, tag), starting at counter `offset`."""
    with np.errstate(over="ignore"):
        base = _mix(np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GAMMA + np.uint64(tag)],
                             dtype=np.uint64))[0]
        ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        return _mix(base + ctr * GAMMA)


def uniform(seed, tag, n, offset=0):
    """n doubles uniform on [0, 1)."""
    return (raw(seed, tag, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_range(seed, tag, n, lo, hi, offset=0):
    return lo + (hi - lo) * uniform(seed, tag, n, offset)


# ------------------------------------------------------------------ phases
def kuramoto_phases(seed, n):
    """phi_i i.i.d. uniform on [-pi, pi)."""
    return -math.pi + 2.0 * math.pi * uniform(seed, TAG_PHASE, n)


def fhn_circle(seed, n, radius=2.0):
    """(u, v) on the circle u^2 + v^2 = radius^2 at i.i.d. uniform angles;
    returned variable-major: u[0..n) then v[0..n)."""
    th = 2.0 * math.pi * uniform(seed, TAG_FHN, n)
    return np.concatenate([radius * np.cos(th), radius * np.sin(th)])


def cube_phases_with_patch(seed, n1, patch_radius=None):
    """Uniform phases on an n1^3 periodic lattice plus one spherical patch of a
    single common phase.  Patch centre uniform over sites, radius n1/5 in
    minimum-image Euclidean distance, patch phase uniform on [-pi, pi)."""
    n = n1 ** 3
    phi = kuramoto_phases(seed, n)
    r = n1 / 5.0 if patch_radius is None else float(patch_radius)
    u = uniform(seed, TAG_PATCH, 4)
    cx, cy, cz = (np.floor(u[:3] * n1).astype(np.int64))
    phase = -math.pi + 2.0 * math.pi * u[3]
    ax = np.arange(n1)

    def md(a, c):
        d = np.abs(a - c)
        return np.minimum(d, n1 - d).astype(np.float64)

    dx2 = md(ax, cx) ** 2
    dy2 = md(ax, cy) ** 2
    dz2 = md(ax, cz) ** 2
    # index x + n1*y + n1*n1*z  ->  array [z, y, x]
    d2 = dz2[:, None, None] + dy2[None, :, None] + dx2[None, None, :]
    phi = phi.reshape(n1, n1, n1)
    phi[d2 <= r * r] = phase
    return phi.ravel()


def twisted_state(n, q):
    """phi_i = 2 pi q i / n (a q-twisted state on a ring)."""
    return 2.0 * math.pi * q * np.arange(n, dtype=np.float64) / n


# --------------------------------------------------------- Hodgkin-Huxley
def hh_state(seed, n):
    """(V, m, h, n) variable-major: V ~ U[-70, -60] mV and gating variables
    uniform in ranges that bracket their resting values (m in [0.03, 0.07],
    h in [0.55, 0.65], n in [0.29, 0.35])."""
    u = uniform(seed, TAG_HH_STATE, 4 * n).reshape(4, n)
    V = -70.0 + 10.0 * u[0]
    m = 0.03 + 0.04 * u[1]
    h = 0.55 + 0.10 * u[2]
    nn = 0.29 + 0.06 * u[3]
    return np.concatenate([V, m, h, nn])


def hh_iapp(seed, n, lo=8.0, hi=12.0):
    return uniform_range(seed, TAG_HH_IAPP, n, lo, hi)


def random_out_graph(seed, n, out_degree, wmax=0.1):
    """Directed graph: each source picks `out_degree` distinct targets other than
    itself, uniformly; weights uniform on [0, wmax).  Returned as CSR by
    target (row_ptr int64[n+1], col int32 sources ascending, w float64)."""
    if out_degree > n - 1:
        raise ValueError("out_degree must be < n")
    d = out_degree
    src = np.repeat(np.arange(n, dtype=np.int64), d).reshape(n, d)
    # target = src + 1 + floor(u * (n - 1)) mod n  (never the source itself)
    tgt = (src + 1 + (uniform(seed, TAG_GRAPH, n * d).reshape(n, d) * (n - 1)).astype(np.int64)) % n
    offset = n * d
    rows = np.arange(n)
    while True:  # redraw whole rows that hold a repeated target
        s = np.sort(tgt[rows], axis=1)
        bad = rows[(s[:, 1:] == s[:, :-1]).any(axis=1)]
        if bad.size == 0:
            break
        draw = uniform(seed, TAG_GRAPH, bad.size * d, offset).reshape(bad.size, d)
        offset += bad.size * d
        tgt[bad] = (bad[:, None] + 1 + (draw * (n - 1)).astype(np.int64)) % n
        rows = bad
    w = wmax * uniform(seed, TAG_WEIGHT, n * d)
    tgt = tgt.ravel().astype(np.int32)
    del src
    # edges are generated source-major, so a stable sort by target leaves the
    # sources of every row ascending
    order = np.argsort(tgt, kind="stable")
    col = (order // d).astype(np.int32)
    w = w[order]
    counts = np.bincount(tgt, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, col, w


# ------------------------------------------------- binary coupling matrices
# Rows of a binary coupling matrix L (row i lists the j with L_ij = 1) as CSR:
# row_ptr int64[n+1], col int32 ascending within each row.
def _csr_from_mask(mask):
    n = mask.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    col = np.nonzero(mask)[1].astype(np.int32)
    return row_ptr, col


def random_links(seed, n, density):
    """Every entry L_ij (self links included) set independently with
    probability `density`; empty rows can occur.  For small n (n^2 draws)."""
    mask = uniform(seed, TAG_LINKS, n * n).reshape(n, n) < density
    return _csr_from_mask(mask)


def ring_links(n, P):
    """Ring: row i holds i-P..i-1 and i+1..i+P (mod n)."""
    off = np.concatenate([np.arange(-P, 0), np.arange(1, P + 1)])
    j = (np.arange(n)[:, None] + off[None, :]) % n
    col = np.sort(j, axis=1).astype(np.int32).ravel()
    return np.arange(0, n * 2 * P + 1, 2 * P, dtype=np.int64), col


def small_world_links(seed, n, P, shortcuts):
    """Ring of radius P plus `shortcuts` extra links placed on random rows to
    random sources (a row may get several; duplicates of existing links and
    self links are skipped), so most rows share the ring's structure and a few
    differ."""
    off = np.concatenate([np.arange(-P, 0), np.arange(1, P + 1)])
    rows = [set(((i + off) % n).tolist()) for i in range(n)]
    u = uniform(seed, TAG_LINKS, 2 * shortcuts)
    for s_ in range(shortcuts):
        i = int(u[2 * s_] * n)
        j = int(u[2 * s_ + 1] * n)
        if j != i:
            rows[i].add(j)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([j for r in rows for j in sorted(r)], dtype=np.int32)
    return row_ptr, col


def lattice_ball_links(n1, n2, n3, P, include_self=True):
    """Periodic n1 x n2 x n3 lattice (index x + n1*y + n1*n2*z), row i holding
    every lattice point within Euclidean distance P of element i (the element
    itself when include_self).  n3 = 1 gives the plane with the disk."""
    r = np.arange(-P, P + 1)
    dz_r = r if n3 > 1 else np.array([0])
    DX, DY, DZ = np.meshgrid(r, r, dz_r, indexing="ij")
    keep = DX ** 2 + DY ** 2 + DZ ** 2 <= P * P
    if not include_self:
        keep &= (DX != 0) | (DY != 0) | (DZ != 0)
    dx, dy, dz = DX[keep], DY[keep], DZ[keep]
    i = np.arange(n1 * n2 * n3, dtype=np.int64)
    x, y, z = i % n1, (i // n1) % n2, i // (n1 * n2)
    L = dx.size
    col = np.empty((i.size, L), dtype=np.int64)
    for q in range(L):
        col[:, q] = (x + dx[q]) % n1 + n1 * ((y + dy[q]) % n2) + n1 * n2 * ((z + dz[q]) % n3)
    col.sort(axis=1)
    row_ptr = np.arange(0, i.size * L + 1, L, dtype=np.int64)
    return row_ptr, col.astype(np.int32).ravel()
