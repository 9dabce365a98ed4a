"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
solutions, invariants of the equations, textbook constants, a dense-matrix
brute force written in a different formulation, or a library integrator.
None of these tests needs a GPU.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from paper_2410_19075_amd import inputs

RING_1024 = dict(n=1024, P=256, omega=0.0, mu=1.0, alpha=1.46)


def kur(omega, mu, alpha):
    return np.array([omega, mu, alpha])


# ----------------------------------------------------------- closed forms
def ring_twist_frequency(n, P, q, omega, mu, alpha):
    """Rotation frequency of the q-twisted state phi_i = 2 pi q i / n.
    sum_{0<|k|<=P} sin(theta k - alpha) = -2 sin(alpha) sum_{k=1}^{P} cos(k theta),
    and sum_{k=1}^{P} cos(k theta) = sin((P + 1/2) theta) / (2 sin(theta/2)) - 1/2
    (Dirichlet kernel), which is P at theta = 0."""
    th = 2.0 * math.pi * q / n
    if q % n == 0:
        csum = float(P)
    else:
        csum = math.sin((P + 0.5) * th) / (2.0 * math.sin(th / 2.0)) - 0.5
    return omega - mu * math.sin(alpha) * csum / P


def dirichlet(h, th):
    """sum_{d=-h}^{h} cos(d th) = sin((h + 1/2) th) / sin(th / 2)."""
    if abs(math.sin(th / 2.0)) < 1e-300:
        return 2.0 * h + 1.0
    return math.sin((h + 0.5) * th) / math.sin(th / 2.0)


def cube_wave_frequency(dims, h, q, omega, mu, alpha):
    """Plane wave phi = 2 pi (q1 x / n1 + q2 y / n2 + q3 z / n3) on the periodic
    lattice: the cube sum of exp(i theta.d) factorises into a product of
    Dirichlet kernels, so the sum over the cube minus the centre of
    sin(theta.d - alpha) equals -sin(alpha) (prod D_h(theta_a) - 1)."""
    L = (2 * h + 1) ** 3 - 1
    prod = 1.0
    for qa, na in zip(q, dims):
        prod *= dirichlet(h, 2.0 * math.pi * qa / na)
    return omega - mu * math.sin(alpha) * (prod - 1.0) / L


def test_closed_form_twist_values_ring_1024():
    # q = 0 is the synchronous state: Omega = -sin(alpha); q = 4 with P = n/4:
    # sin(257 * 2pi*4/1024 ...) makes the Dirichlet sum -1/2 - 1/2 + ... = 0
    assert ring_twist_frequency(1024, 256, 0, 0.0, 1.0, 1.46) == pytest.approx(-math.sin(1.46), abs=1e-15)
    assert abs(ring_twist_frequency(1024, 256, 4, 0.0, 1.0, 1.46)) < 1e-15


# ------------------------------------------------------------ Kuramoto ring
@pytest.mark.parametrize("q", [0, 1, 2, 3, 4, 17])
def test_ring_twisted_state_rotates_rigidly(q):
    """A q-twisted state is an exact solution rotating at Omega_q; RK4 keeps it
    exactly (all stage slopes equal), so phi(t) - phi(0) = Omega_q t."""
    n, P = RING_1024["n"], RING_1024["P"]
    net = O.ring(O.KURAMOTO, n, P, kur(0.0, 1.0, 1.46))
    y0 = inputs.twisted_state(n, q)
    dt, steps = 0.01, 200
    y, R, _ = O.run(net, y0, dt, steps, record_every=1)
    om = ring_twist_frequency(n, P, q, 0.0, 1.0, 1.46)
    # phases are unwrapped, so rounding scales with their magnitude
    assert np.max(np.abs((y - y0) - om * dt * steps)) < 1e-13 + 1e-14 * np.max(np.abs(y0))
    # order parameter of a twisted state is 0 (q != 0) or 1 (q == 0) at all times
    target = 1.0 if q == 0 else 0.0
    assert np.max(np.abs(R - target)) < 1e-12


def test_ring_zero_coupling_is_free_rotation():
    """mu = 0: phi_i(t) = phi_i(0) + omega t exactly up to rounding."""
    n = 257
    net = O.ring(O.KURAMOTO, n, 40, kur(0.73, 0.0, 1.46))
    y0 = inputs.kuramoto_phases(5, n)
    y, _, mv = O.run(net, y0, 0.01, 300, mv_start=100)
    assert np.max(np.abs(y - (y0 + 0.73 * 3.0))) < 1e-13
    assert np.max(np.abs(mv - 0.73)) < 1e-12


def test_ring_sign_forms_agree():
    """The configs write -(mu/2P) sum sin(phi_i - phi_j + alpha); Eq. (3) writes
    +mu sum sin(phi_j - phi_i - alpha) normalised by the link count. The two
    are the same function."""
    n, P = 64, 9
    net = O.ring(O.KURAMOTO, n, P, kur(0.2, 1.3, 0.9))
    z = inputs.kuramoto_phases(11, n)
    f = O.rhs(net, z)
    g = np.empty(n)
    for i in range(n):
        s = 0.0
        for k in list(range(-P, 0)) + list(range(1, P + 1)):
            s += math.sin(z[i] - z[(i + k) % n] + 0.9)
        g[i] = 0.2 - 1.3 / (2 * P) * s
    assert np.max(np.abs(f - g)) < 1e-14


def test_ring_mean_phase_invariant_alpha0():
    """alpha = 0, omega = 0: sum_i f_i = 0 (antisymmetric pairs) and RK4
    preserves linear invariants, so the mean phase is constant even though
    individual phases move."""
    n, P = 300, 70
    net = O.ring(O.KURAMOTO, n, P, kur(0.0, 1.0, 0.0))
    y0 = inputs.kuramoto_phases(3, n)
    y, _, _ = O.run(net, y0, 0.05, 400)
    assert np.max(np.abs(y - y0)) > 1e-2
    assert abs(np.mean(y) - np.mean(y0)) < 1e-13


def test_rk4_fourth_order():
    """Error after T = 2 falls by ~16 per halving of dt (classical RK4)."""
    n, P = 64, 8
    net = O.ring(O.KURAMOTO, n, P, kur(0.0, 1.0, 1.46))
    y0 = inputs.kuramoto_phases(1, n)
    ref, _, _ = O.run(net, y0, 0.1 / 64, 64 * 20)
    errs = []
    for k in range(4):
        dt = 0.1 / 2 ** k
        y, _, _ = O.run(net, y0, dt, 20 * 2 ** k)
        errs.append(np.max(np.abs(y - ref)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 14.0 < r < 18.5, ratios


def test_ring_cyclic_shift_and_reflection_symmetry():
    n, P = 97, 13
    net = O.ring(O.KURAMOTO, n, P, kur(0.1, 1.0, 1.2))
    y0 = inputs.kuramoto_phases(8, n)
    y, _, _ = O.run(net, y0, 0.02, 50)
    ys, _, _ = O.run(net, np.roll(y0, 5), 0.02, 50)
    assert np.array_equal(np.roll(y, 5), ys)  # neighbour order is relative to i
    yr, _, _ = O.run(net, y0[::-1].copy(), 0.02, 50)
    assert np.max(np.abs(yr[::-1] - y)) < 1e-12
    # global phase shift: phi -> phi + c commutes with the flow
    yc, _, _ = O.run(net, y0 + 0.7, 0.02, 50)
    assert np.max(np.abs(yc - 0.7 - y)) < 1e-12


def test_ring_rejects_overlapping_window():
    net = O.ring(O.KURAMOTO, 10, 5, kur(0, 1, 1))
    with pytest.raises(ValueError):
        O.rhs(net, np.zeros(10))


# ------------------------------------------------------------ dense brute force
def ring_adjacency(n, P):
    A = np.zeros((n, n))
    for i in range(n):
        for k in range(1, P + 1):
            A[i, (i + k) % n] = 1.0
            A[i, (i - k) % n] = 1.0
    return A


def cube_adjacency(dims, h):
    n1, n2, n3 = dims
    n = n1 * n2 * n3
    idx = np.arange(n)
    x, y, z = idx % n1, (idx // n1) % n2, idx // (n1 * n2)
    A = np.zeros((n, n))
    for dz in range(-h, h + 1):
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                if dx == dy == dz == 0:
                    continue
                j = (x + dx) % n1 + n1 * (((y + dy) % n2) + n2 * ((z + dz) % n3))
                A[idx, j] += 1.0
    return A


def dense_rk4(F, y, dt, steps):
    for _ in range(steps):
        k1 = F(y)
        k2 = F(y + dt / 2 * k1)
        k3 = F(y + dt / 2 * k2)
        k4 = F(y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def kuramoto_dense(A, omega, mu, alpha):
    L = A.sum(axis=1)

    def F(phi):
        # sum_j A_ij sin(phi_j - phi_i - alpha) = Im(exp(-i(phi_i + alpha)) (A exp(i phi))_i)
        return omega + mu * np.imag(np.exp(-1j * (phi + alpha)) * (A @ np.exp(1j * phi))) / L

    return F


@pytest.mark.parametrize("n,P", [(16, 1), (16, 7), (33, 3), (33, 16), (64, 7), (64, 31)])
def test_ring_dense_brute_force(n, P):
    A = ring_adjacency(n, P)
    assert np.all(A.sum(axis=1) == 2 * P)
    F = kuramoto_dense(A, 0.3, 1.1, 1.46)
    y0 = inputs.kuramoto_phases(n + P, n)
    ref = dense_rk4(F, y0, 0.01, 100)
    y, _, _ = O.run(O.ring(O.KURAMOTO, n, P, kur(0.3, 1.1, 1.46)), y0, 0.01, 100)
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-13


@pytest.mark.parametrize("dims,h", [((9, 9, 9), 4), ((10, 10, 10), 1), ((5, 7, 9), 2)])
def test_cube_dense_brute_force(dims, h):
    A = cube_adjacency(dims, h)
    assert np.all(A.sum(axis=1) == (2 * h + 1) ** 3 - 1)
    F = kuramoto_dense(A, 0.0, 1.0, 0.8)
    n = dims[0] * dims[1] * dims[2]
    y0 = inputs.kuramoto_phases(7, n)
    ref = dense_rk4(F, y0, 0.05, 20)
    net = O.cube(dims[0], h, kur(0.0, 1.0, 0.8), n2=dims[1], n3=dims[2])
    y, _, _ = O.run(net, y0, 0.05, 20)
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-13


@pytest.mark.parametrize("q", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (2, -1, 3)])
def test_cube_plane_wave_closed_form(q):
    """Plane waves rotate rigidly at the Dirichlet-product frequency.  Distinct
    extents per axis catch any mix-up of the index map."""
    dims, h = (11, 12, 13), 2
    n1, n2, n3 = dims
    idx = np.arange(n1 * n2 * n3)
    x, y, z = idx % n1, (idx // n1) % n2, idx // (n1 * n2)
    y0 = 2 * math.pi * (q[0] * x / n1 + q[1] * y / n2 + q[2] * z / n3)
    net = O.cube(n1, h, kur(0.25, 1.0, 0.8), n2=n2, n3=n3)
    dt, steps = 0.05, 20
    yt, _, _ = O.run(net, y0, dt, steps)
    om = cube_wave_frequency(dims, h, q, 0.25, 1.0, 0.8)
    assert np.max(np.abs((yt - y0) - om * dt * steps)) < 1e-12


def test_cube_200_plane_wave_frequencies_h4():
    """The closed form for the 200^3, h = 4, alpha = 0.8 lattice at q = 0 is
    -sin(alpha); the oracle's RHS on a plane wave matches the closed form."""
    assert cube_wave_frequency((200,) * 3, 4, (0, 0, 0), 0, 1, 0.8) == pytest.approx(-math.sin(0.8), abs=1e-15)
    dims = (20, 20, 20)
    n = 8000
    idx = np.arange(n)
    x, y, z = idx % 20, (idx // 20) % 20, idx // 400
    for q in [(1, 0, 0), (1, 1, 0), (1, 1, 1), (5, 0, 0)]:
        phi = 2 * math.pi * (q[0] * x + q[1] * y + q[2] * z) / 20
        f = O.rhs(O.cube(20, 4, kur(0.0, 1.0, 0.8)), phi)
        assert np.max(np.abs(f - cube_wave_frequency(dims, 4, q, 0.0, 1.0, 0.8))) < 1e-14


def test_cube_cyclic_shift_symmetry():
    n1 = 10
    net = O.cube(n1, 2, kur(0.0, 1.0, 0.8))
    y0 = inputs.kuramoto_phases(2, n1 ** 3)
    y, _, _ = O.run(net, y0, 0.05, 5)
    sh = np.roll(y0.reshape(n1, n1, n1), (1, 2, 3), axis=(0, 1, 2)).ravel()
    ys, _, _ = O.run(net, sh, 0.05, 5)
    assert np.array_equal(np.roll(y.reshape(n1, n1, n1), (1, 2, 3), axis=(0, 1, 2)).ravel(), ys)


def test_sphere_link_counts_of_the_paper(golden):
    """Reading of the paper's link counts: its 3D sphere neighbourhoods of radius
    P = 2 and 6 have 33 and 925 links, which are the lattice-point counts of the
    closed ball including the centre.  The cube neighbourhood used here excludes
    the centre, as the 1D ring with mu = 1/2P does."""
    for P, count in golden("sphere_link_counts.txt"):
        r = np.arange(-P, P + 1)
        X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
        assert int(np.sum(X ** 2 + Y ** 2 + Z ** 2 <= P * P)) == count


# ---------------------------------------------------------- FitzHugh-Nagumo
FHN_PRM = np.array([0.05, 0.5, 0.1, math.pi / 2 - 0.1])


def fhn_local(u, v, eps, a):
    return np.array([(u - u ** 3 / 3 - v) / eps, u + a])


def test_fhn_rest_point_is_fixed():
    """(u*, v*) = (-a, -a + a^3/3) is an equilibrium of the uncoupled and of the
    uniformly coupled network."""
    n, P = 128, 44
    net = O.ring(O.FHN, n, P, FHN_PRM)
    a = 0.5
    y0 = np.concatenate([np.full(n, -a), np.full(n, -a + a ** 3 / 3)])
    f = O.rhs(net, y0)
    assert np.max(np.abs(f)) < 1e-15
    y, _, _ = O.run(net, y0, 0.01, 200)
    assert np.max(np.abs(y - y0)) < 1e-12


def test_fhn_jacobian_at_rest():
    """Finite differences of the RHS at the rest point reproduce the hand-derived
    Jacobian [[(1 - a^2)/eps, -1/eps], [1, 0]] of one uncoupled element."""
    eps, a = 0.05, 0.5
    n, P = 16, 3
    net = O.ring(O.FHN, n, P, np.array([eps, a, 0.0, 0.3]))
    y0 = np.concatenate([np.full(n, -a), np.full(n, -a + a ** 3 / 3)])
    J = np.array([[(1 - a * a) / eps, -1 / eps], [1.0, 0.0]])
    d = 1e-6
    for c in range(2):
        yp = y0.copy()
        ym = y0.copy()
        yp[c * n + 5] += d
        ym[c * n + 5] -= d
        col = (O.rhs(net, yp) - O.rhs(net, ym)) / (2 * d)
        assert abs(col[5] - J[0, c]) < 1e-6 * max(1, abs(J[0, c]))
        assert abs(col[n + 5] - J[1, c]) < 1e-6


def test_fhn_rotational_coupling_single_neighbour():
    """Uniform state with one neighbour j of element i displaced by (du, dv):
    the change of f_i is (kappa/eps) (cos phi du + sin phi dv) in u and
    kappa (-sin phi du + cos phi dv) in v, kappa = sigma / 2P."""
    n, P = 40, 6
    eps, a, sigma, phi = 0.05, 0.5, 0.1, math.pi / 2 - 0.1
    net = O.ring(O.FHN, n, P, np.array([eps, a, sigma, phi]))
    base = np.concatenate([np.full(n, 0.3), np.full(n, -0.2)])
    f0 = O.rhs(net, base)
    du, dv = 0.25, -0.4
    y = base.copy()
    y[10 + 3] += du
    y[n + 10 + 3] += dv
    f1 = O.rhs(net, y)
    kap = sigma / (2 * P)
    assert abs((f1[10] - f0[10]) - kap * (math.cos(phi) * du + math.sin(phi) * dv) / eps) < 1e-13
    assert abs((f1[n + 10] - f0[n + 10]) - kap * (-math.sin(phi) * du + math.cos(phi) * dv)) < 1e-14
    # an element outside the window (distance P + 1) is untouched
    assert f1[10 + 3 + P + 1] == f0[10 + 3 + P + 1]


def test_fhn_coupling_sums_to_zero():
    """The coupling is antisymmetric in (i, j) and linear, so summed over all
    elements it vanishes for any state."""
    n, P = 200, 70
    eps, a = 0.05, 0.5
    net = O.ring(O.FHN, n, P, FHN_PRM)
    y = inputs.fhn_circle(4, n)
    f = O.rhs(net, y)
    u, v = y[:n], y[n:]
    loc = fhn_local(u, v, eps, a)
    cu = eps * f[:n] - eps * loc[0]
    cv = f[n:] - loc[1]
    assert abs(cu.sum()) < 1e-13 * np.abs(cu).sum() + 1e-15
    assert abs(cv.sum()) < 1e-13 * np.abs(cv).sum() + 1e-15


def test_fhn_uniform_network_is_one_oscillator():
    """A uniform state has zero coupling, so each element follows the single
    FitzHugh-Nagumo oscillator; compare with scipy's DOP853 at tight tolerance."""
    n, P = 64, 20
    eps, a = 0.05, 0.5
    net = O.ring(O.FHN, n, P, FHN_PRM)
    u0, v0 = 1.3, -0.4
    y0 = np.concatenate([np.full(n, u0), np.full(n, v0)])
    dt, steps = 0.001, 2000
    y, _, _ = O.run(net, y0, dt, steps)
    sol = solve_ivp(lambda t, s: fhn_local(s[0], s[1], eps, a), (0, dt * steps), [u0, v0],
                    method="DOP853", rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1]
    assert np.all(y[:n] == y[0]) and np.all(y[n:] == y[n])
    assert abs(y[0] - ref[0]) < 1e-8 and abs(y[n] - ref[1]) < 1e-8


def test_fhn_dense_brute_force():
    n, P = 33, 11
    eps, a, sigma, phi = FHN_PRM
    A = ring_adjacency(n, P)
    L = 2 * P
    B = np.array([[math.cos(phi), math.sin(phi)], [-math.sin(phi), math.cos(phi)]])

    def F(s):
        u, v = s[:n], s[n:]
        Du = A @ u - L * u
        Dv = A @ v - L * v
        cu = sigma / L * (B[0, 0] * Du + B[0, 1] * Dv)
        cv = sigma / L * (B[1, 0] * Du + B[1, 1] * Dv)
        return np.concatenate([(u - u ** 3 / 3 - v + cu) / eps, u + a + cv])

    y0 = inputs.fhn_circle(9, n)
    ref = dense_rk4(F, y0, 0.01, 200)
    y, _, _ = O.run(O.ring(O.FHN, n, P, FHN_PRM), y0, 0.01, 200)
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-12


def test_fhn_order_parameter_uses_geometric_phase():
    n = 50
    th = np.full(n, 0.7)
    y = np.concatenate([2 * np.cos(th), 2 * np.sin(th)])
    assert O.order_parameter(O.FHN, n, y) == pytest.approx(1.0, abs=1e-15)
    th = 2 * math.pi * np.arange(n) / n
    y = np.concatenate([3 * np.cos(th), 3 * np.sin(th)])
    assert O.order_parameter(O.FHN, n, y) < 1e-14


# ----------------------------------------------------------- Hodgkin-Huxley
HH_PRM = np.array([1.0, 120.0, 36.0, 0.3, 50.0, -77.0, -54.387, 0.0, 0.0, 2.0])


def hh_net(n, row_ptr, col, w, iapp):
    return O.csr(n, row_ptr, col, w, HH_PRM, iapp)


def empty_csr(n):
    return np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0)


def hh_rates_via_rhs(V):
    """Read alpha_x(V) and beta_x(V) off the RHS: with x = 0, dx/dt = alpha_x;
    with x = 1, dx/dt = -beta_x."""
    rp, c, w = empty_csr(2)
    net = hh_net(2, rp, c, w, np.zeros(2))
    z0 = np.array([V, V, 0, 1, 0, 1, 0, 1], dtype=np.float64)  # V, m, h, n (2 neurons)
    f = O.rhs(net, z0)
    return dict(am=f[2], bm=-f[3], ah=f[4], bh=-f[5], an=f[6], bn=-f[7])


def test_hh_textbook_resting_state():
    """Squid axon at rest (modern convention): V = -65 mV with the textbook
    steady-state gates m = 0.0529, h = 0.5961, n = 0.3177; the leak reversal
    -54.387 mV makes the net ionic current vanish there."""
    rp, c, w = empty_csr(1)
    net = hh_net(1, rp, c, w, np.zeros(1))
    f = O.rhs(net, np.array([-65.0, 0.0529, 0.5961, 0.3177]))
    assert abs(f[0]) < 0.02          # mV/ms, 4-digit gates
    assert abs(f[1]) < 5e-4 and abs(f[2]) < 5e-4 and abs(f[3]) < 5e-4


def test_hh_rate_special_values():
    r = hh_rates_via_rhs(-65.0)
    assert r["bm"] == pytest.approx(4.0, rel=1e-15)
    assert r["ah"] == pytest.approx(0.07, rel=1e-15)
    assert r["bn"] == pytest.approx(0.125, rel=1e-15)
    # removable singularities: alpha_m(-40) = 1, alpha_n(-55) = 0.1
    assert hh_rates_via_rhs(-40.0)["am"] == pytest.approx(1.0, rel=1e-15)
    assert hh_rates_via_rhs(-55.0)["an"] == pytest.approx(0.1, rel=1e-15)
    # continuity across the singularity
    assert hh_rates_via_rhs(-40.0 + 1e-6)["am"] == pytest.approx(1.0 + 0.5e-7, rel=1e-12)
    assert hh_rates_via_rhs(-35.0)["bh"] == pytest.approx(0.5, rel=1e-15)
    # far from the singularity alpha_m = 0.1 (V + 40) / (1 - exp(-(V + 40)/10))
    assert hh_rates_via_rhs(-20.0)["am"] == pytest.approx(2.0 / (1 - math.exp(-2.0)), rel=1e-14)


def test_hh_synapse_direction_and_sigmoid():
    """One edge 0 -> 1 with weight w: neuron 1 gets (Esyn - V1) w S(V0) with
    S(0 mV) = 1/2; neuron 0 is unaffected (CSR rows are targets)."""
    n = 2
    row_ptr = np.array([0, 0, 1], dtype=np.int64)
    col = np.array([0], dtype=np.int32)
    w = np.array([0.08])
    z = np.array([0.0, -60.0, 0.05, 0.05, 0.6, 0.6, 0.3, 0.3])
    f = O.rhs(hh_net(n, row_ptr, col, w, np.zeros(n)), z)
    rp, c, ww = empty_csr(n)
    g = O.rhs(hh_net(n, rp, c, ww, np.zeros(n)), z)
    assert f[0] == g[0]
    assert f[1] - g[1] == pytest.approx((0.0 - (-60.0)) * 0.08 * 0.5, rel=1e-14)
    z2 = z.copy()
    z2[0] = 4.0  # S(4 mV) = 1 / (1 + e^-2)
    f2 = O.rhs(hh_net(n, row_ptr, col, w, np.zeros(n)), z2)
    g2 = O.rhs(hh_net(n, rp, c, ww, np.zeros(n)), z2)
    assert f2[1] - g2[1] == pytest.approx(60.0 * 0.08 / (1 + math.exp(-2.0)), rel=1e-13)


def test_hh_uncoupled_neuron_matches_library_integrator():
    """With no synapses each neuron is the single HH model; compare the oracle's
    RK4 with scipy's DOP853 over 20 ms of repetitive firing (I = 10)."""
    n = 3
    rp, c, w = empty_csr(n)
    iapp = np.array([0.0, 10.0, 6.5])
    net = hh_net(n, rp, c, w, iapp)
    y0 = np.concatenate([np.full(n, -65.0), np.full(n, 0.0529), np.full(n, 0.5961), np.full(n, 0.3177)])
    dt, steps = 0.001, 20000
    y, _, _ = O.run(net, y0, dt, steps)

    def am(V):
        x = (V + 40) / 10
        return x / (-math.expm1(-x))

    def an(V):
        x = (V + 55) / 10
        return 0.1 * x / (-math.expm1(-x))

    def F(t, s, I):
        V, m, h, nn = s
        dV = I - 120 * m ** 3 * h * (V - 50) - 36 * nn ** 4 * (V + 77) - 0.3 * (V + 54.387)
        return [dV, am(V) * (1 - m) - 4 * math.exp(-(V + 65) / 18) * m,
                0.07 * math.exp(-(V + 65) / 20) * (1 - h) - h / (1 + math.exp(-(V + 35) / 10)),
                an(V) * (1 - nn) - 0.125 * math.exp(-(V + 65) / 80) * nn]

    for i in range(n):
        sol = solve_ivp(F, (0, dt * steps), y0[i::n], args=(iapp[i],), method="DOP853",
                        rtol=1e-12, atol=1e-12)
        ref = sol.y[:, -1]
        got = y[i::n]
        assert np.max(np.abs(got - ref) / np.array([100, 1, 1, 1])) < 1e-7, (i, got, ref)
    # the driven neuron spiked (V went far above rest at some point is implied by
    # the library agreeing on a state away from rest)
    assert abs(y[1] - (-65.0)) > 1.0


def test_hh_dense_brute_force():
    n = 50
    row_ptr, col, w = inputs.random_out_graph(3, n, 7, wmax=0.1)
    W = np.zeros((n, n))
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            W[i, col[e]] += w[e]
    # every source has exactly 7 distinct targets, none itself
    assert np.all((W > 0).sum(axis=0) == 7) and np.all(np.diag(W) == 0)
    iapp = inputs.hh_iapp(3, n)
    y0 = inputs.hh_state(3, n)
    base = hh_net(n, *empty_csr(n), iapp)
    full = hh_net(n, row_ptr, col, w, iapp)

    def F(s):
        # uncoupled RHS from the oracle, synaptic term added as a dense matvec
        f = O.rhs(base, s)
        V = s[:n]
        S = 1.0 / (1.0 + np.exp(-V / 2.0))
        f[:n] += (0.0 - V) * (W @ S)
        return f

    ref = dense_rk4(F, y0, 0.01, 300)
    y, _, _ = O.run(full, y0, 0.01, 300)
    assert np.max(np.abs(y - ref) / np.array([100.0] * n + [1.0] * 3 * n)) < 1e-12


# ------------------------------------------------------------- self floor
def test_fp64_self_floor_ring_1024():
    """Reversing the neighbour summation order changes the N = 1024 ring's result only at the
    rounding level after 200 steps (the FP64 floor behind the 1e-12 gate)."""
    net = O.ring(O.KURAMOTO, RING_1024["n"], RING_1024["P"], kur(0.0, 1.0, 1.46))
    y0 = inputs.kuramoto_phases(1, RING_1024["n"])
    a, Ra, _ = O.run(net, y0, 0.01, 200, record_every=1)
    b, Rb, _ = O.run(net, y0, 0.01, 200, record_every=1, reverse=True)
    e = np.max(np.abs(a - b)) / np.max(np.abs(a))
    assert 0 < e < 1e-13
    assert np.max(np.abs(Ra - Rb)) < 1e-13


# ------------------------------------------------- Kuramoto with inertia, Eq. (3)
def inert(omega, mu, alpha, m, eps):
    return np.array([omega, mu, alpha, m, eps])


def test_inertia_zero_coupling_closed_form():
    """mu = 0: m psi' = omega - eps psi is linear, so
    psi(t) = w + (psi0 - w) e^{-eps t/m},  phi(t) = phi0 + w t + (psi0 - w)(m/eps)(1 - e^{-eps t/m}),
    w = omega/eps.  Checks the placement of m, eps and omega."""
    n, P = 40, 3
    omega, m, eps = 0.7, 2.5, 0.4
    phi0 = inputs.kuramoto_phases(5, n)
    psi0 = inputs.uniform_range(6, inputs.TAG_MISC, n, -1.0, 1.0)
    dt, steps = 0.01, 500
    y, _, _ = O.run(O.ring(O.INERTIA, n, P, inert(omega, 0.0, 1.0, m, eps)), np.concatenate([phi0, psi0]), dt, steps)
    t = dt * steps
    w = omega / eps
    decay = math.exp(-eps * t / m)
    psi = w + (psi0 - w) * decay
    phi = phi0 + w * t + (psi0 - w) * (m / eps) * (1.0 - decay)
    assert np.max(np.abs(y[n:] - psi)) < 1e-12
    assert np.max(np.abs(y[:n] - phi)) < 1e-11


@pytest.mark.parametrize("q", [0, 1, 3, 7])
def test_inertia_ring_twisted_state_steady_rotation(q):
    """A q-twisted state with psi = Omega everywhere is an exact solution when
    eps Omega = omega + mu * (coupling of the twist) = eps * (first-order
    twist frequency with omega -> omega, i.e. Omega = f_q / eps)."""
    n, P = 60, 11
    omega, mu, alpha, m, eps = 0.3, 1.2, 0.45, 1.0, 0.05
    f = ring_twist_frequency(n, P, q, omega, mu, alpha)  # omega + mu * coupling
    Om = f / eps
    phi0 = 2 * math.pi * q * np.arange(n) / n
    y0 = np.concatenate([phi0, np.full(n, Om)])
    dt, steps = 0.01, 100
    y, _, _ = O.run(O.ring(O.INERTIA, n, P, inert(omega, mu, alpha, m, eps)), y0, dt, steps)
    assert np.max(np.abs(y[n:] - Om)) < 1e-10 * max(1.0, abs(Om))
    assert np.max(np.abs((y[:n] - phi0) - Om * dt * steps)) < 1e-10 * max(1.0, abs(Om))


def test_inertia_cube_plane_wave_steady_rotation():
    dims, h = (9, 10, 11), 2
    n1, n2, n3 = dims
    idx = np.arange(n1 * n2 * n3)
    x, yy, z = idx % n1, (idx // n1) % n2, idx // (n1 * n2)
    q = (1, -2, 1)
    phi0 = 2 * math.pi * (q[0] * x / n1 + q[1] * yy / n2 + q[2] * z / n3)
    omega, mu, alpha, m, eps = 0.1, 0.9, 0.45, 1.0, 0.5
    Om = cube_wave_frequency(dims, h, q, omega, mu, alpha) / eps
    y0 = np.concatenate([phi0, np.full(phi0.size, Om)])
    net = O.cube(n1, h, inert(omega, mu, alpha, m, eps), n2=n2, n3=n3, model=O.INERTIA)
    y, _, _ = O.run(net, y0, 0.05, 20)
    assert np.max(np.abs(y[phi0.size:] - Om)) < 1e-12
    assert np.max(np.abs((y[:phi0.size] - phi0) - Om * 1.0)) < 1e-12


def test_inertia_time_rescaling_invariance():
    """Multiplying m, eps, mu and omega by the same factor leaves the equations
    unchanged (every term of m psi' = ... scales alike)."""
    n, P = 50, 6
    y0 = np.concatenate([inputs.kuramoto_phases(8, n), inputs.uniform_range(9, inputs.TAG_MISC, n, -0.5, 0.5)])
    a, _, _ = O.run(O.ring(O.INERTIA, n, P, inert(0.2, 1.0, 0.45, 1.0, 0.05)), y0, 0.01, 200)
    b, _, _ = O.run(O.ring(O.INERTIA, n, P, inert(0.2 * 4, 1.0 * 4, 0.45, 1.0 * 4, 0.05 * 4)), y0, 0.01, 200)
    assert np.max(np.abs(a - b)) < 1e-13


def inertia_dense(A, omega, mu, alpha, m, eps):
    L = A.sum(axis=1)
    n = A.shape[0]

    def F(y):
        phi, psi = y[:n], y[n:]
        coup = np.imag(np.exp(-1j * (phi + alpha)) * (A @ np.exp(1j * phi))) / L
        return np.concatenate([psi, (omega - eps * psi + mu * coup) / m])

    return F


@pytest.mark.parametrize("topo", ["ring", "cube"])
def test_inertia_dense_brute_force(topo):
    prm = (0.15, 1.3, 0.45, 1.7, 0.3)
    if topo == "ring":
        n, P = 40, 9
        A = ring_adjacency(n, P)
        net = O.ring(O.INERTIA, n, P, inert(*prm))
    else:
        dims, h = (6, 7, 8), 2
        n = 6 * 7 * 8
        A = cube_adjacency(dims, h)
        net = O.cube(6, h, inert(*prm), n2=7, n3=8, model=O.INERTIA)
    y0 = np.concatenate([inputs.kuramoto_phases(11, n), inputs.uniform_range(12, inputs.TAG_MISC, n, -1.0, 1.0)])
    ref = dense_rk4(inertia_dense(A, *prm), y0, 0.02, 100)
    y, _, _ = O.run(net, y0, 0.02, 100)
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-13


# ------------------------------------------ ball neighbourhood (3D lattice)
def ball_offsets(P):
    r = np.arange(-P, P + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    keep = X ** 2 + Y ** 2 + Z ** 2 <= P * P
    return X[keep], Y[keep], Z[keep]


@pytest.mark.parametrize("P", [2, 6])
def test_ball_link_count_matches_the_paper(golden, P):
    """Perturb one element inside the ball of element 0 and one outside it; the
    RHS of element 0 changes by mu/L (sin(d - alpha) + sin alpha) for the inside
    one and not at all for the outside one, which measures L: the paper's link
    count (33 for P = 2, 925 for P = 6, centre included)."""
    count = dict(golden("sphere_link_counts.txt"))[P]
    n1 = 2 * P + 3
    omega, mu, alpha, d = 0.2, 1.3, 0.45, 0.9
    net = O.ball(n1, P, kur(omega, mu, alpha))
    base = O.rhs(net, np.zeros(n1 ** 3))[0]
    assert base == pytest.approx(omega - mu * math.sin(alpha), abs=1e-13)
    inside = np.zeros(n1 ** 3)
    inside[1 + n1 * 1] = d  # offset (1, 1, 0): |d|^2 = 2 <= P^2
    L = mu * (math.sin(d - alpha) + math.sin(alpha)) / (O.rhs(net, inside)[0] - base)
    assert L == pytest.approx(count, rel=1e-9)
    outside = np.zeros(n1 ** 3)
    outside[P + n1 * P] = d  # offset (P, P, 0): |d|^2 = 2 P^2 > P^2
    assert O.rhs(net, outside)[0] == pytest.approx(base, abs=1e-13)


@pytest.mark.parametrize("P,q", [(2, (1, 0, 0)), (2, (1, -1, 2)), (3, (0, 2, 1)), (1, (1, 1, 1))])
def test_ball_plane_wave_rotates_at_closed_form(P, q):
    """On a plane wave phi = theta . x the ball sum of sin(theta.d - alpha) is
    -sin(alpha) sum_d cos(theta.d) (the sine part cancels between d and -d), so
    every element rotates at omega - mu sin(alpha) <cos(theta.d)>_ball."""
    dims = (9, 10, 11)
    n1, n2, n3 = dims
    idx = np.arange(n1 * n2 * n3)
    x, y, z = idx % n1, (idx // n1) % n2, idx // (n1 * n2)
    th = [2 * math.pi * q[0] / n1, 2 * math.pi * q[1] / n2, 2 * math.pi * q[2] / n3]
    phi0 = th[0] * x + th[1] * y + th[2] * z
    omega, mu, alpha = 0.1, 0.8, 0.45
    dx, dy, dz = ball_offsets(P)
    om = omega - mu * math.sin(alpha) * float(np.mean(np.cos(th[0] * dx + th[1] * dy + th[2] * dz)))
    yt, _, _ = O.run(O.ball(n1, P, kur(omega, mu, alpha), n2=n2, n3=n3), phi0, 0.05, 20)
    assert np.max(np.abs((yt - phi0) - om * 1.0)) < 1e-12


def ball_adjacency(dims, P):
    n1, n2, n3 = dims
    n = n1 * n2 * n3
    idx = np.arange(n)
    x, y, z = idx % n1, (idx // n1) % n2, idx // (n1 * n2)
    A = np.zeros((n, n))
    for ox, oy, oz in zip(*ball_offsets(P)):
        j = (x + ox) % n1 + n1 * (((y + oy) % n2) + n2 * ((z + oz) % n3))
        A[idx, j] += 1.0
    return A


@pytest.mark.parametrize("model", ["kuramoto", "inertia"])
def test_ball_dense_brute_force(model):
    dims, P = (7, 8, 9), 3
    n = 7 * 8 * 9
    A = ball_adjacency(dims, P)
    assert np.all(A.sum(axis=1) == 123)  # lattice points within distance 3
    if model == "kuramoto":
        prm = kur(0.2, 1.1, 0.45)
        F = kuramoto_dense(A, *prm)
        y0 = inputs.kuramoto_phases(13, n)
        net = O.ball(7, P, prm, n2=8, n3=9)
    else:
        prm = inert(0.2, 1.1, 0.45, 1.5, 0.2)
        F = inertia_dense(A, *prm)
        y0 = np.concatenate([inputs.kuramoto_phases(13, n), inputs.uniform_range(14, inputs.TAG_MISC, n, -1, 1)])
        net = O.ball(7, P, prm, n2=8, n3=9, model=O.INERTIA)
    ref = dense_rk4(F, y0, 0.05, 30)
    y, _, _ = O.run(net, y0, 0.05, 30)
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-13


def test_ball_axis_permutation_symmetry():
    """The ball is invariant under permutations of the axes: on a cubic lattice,
    transposing the initial state transposes the result (up to the changed
    summation order of the neighbour sum)."""
    n1, P = 9, 2
    net = O.ball(n1, P, kur(0.0, 1.0, 0.45))
    y0 = inputs.kuramoto_phases(15, n1 ** 3)
    y, _, _ = O.run(net, y0, 0.05, 10)
    perm = (2, 0, 1)
    yp, _, _ = O.run(net, np.transpose(y0.reshape(n1, n1, n1), perm).ravel().copy(), 0.05, 10)
    assert np.max(np.abs(np.transpose(y.reshape(n1, n1, n1), perm).ravel() - yp)) < 1e-13


# ------------------------------------------------ disk neighbourhood (2D plane)
def disk_offsets(P):
    r = np.arange(-P, P + 1)
    X, Y = np.meshgrid(r, r, indexing="ij")
    keep = X ** 2 + Y ** 2 <= P * P
    return X[keep], Y[keep]


@pytest.mark.parametrize("P,count", [(1, 5), (2, 13), (3, 29), (6, 113)])
def test_disk_link_count(P, count):
    """Gauss circle counts N(P) = #{x^2 + y^2 <= P^2}: 5, 13, 29, 113; the oracle's
    normalisation is recovered from a single perturbed neighbour."""
    assert len(disk_offsets(P)[0]) == count
    n1 = 2 * P + 3
    omega, mu, alpha, d = 0.2, 1.3, 0.45, 0.9
    net = O.disk(n1, P, kur(omega, mu, alpha))
    base = O.rhs(net, np.zeros(n1 * n1))[0]
    z = np.zeros(n1 * n1)
    z[1] = d  # offset (1, 0), inside every disk
    L = mu * (math.sin(d - alpha) + math.sin(alpha)) / (O.rhs(net, z)[0] - base)
    assert L == pytest.approx(count, rel=1e-9)


@pytest.mark.parametrize("P,q", [(2, (1, 0)), (3, (1, -2)), (5, (2, 3))])
def test_disk_plane_wave_rotates_at_closed_form(P, q):
    n1, n2 = 17, 19
    idx = np.arange(n1 * n2)
    x, y = idx % n1, idx // n1
    th = (2 * math.pi * q[0] / n1, 2 * math.pi * q[1] / n2)
    phi0 = th[0] * x + th[1] * y
    omega, mu, alpha = 0.1, 0.8, 0.45
    dx, dy = disk_offsets(P)
    om = omega - mu * math.sin(alpha) * float(np.mean(np.cos(th[0] * dx + th[1] * dy)))
    yt, _, _ = O.run(O.disk(n1, P, kur(omega, mu, alpha), n2=n2), phi0, 0.05, 20)
    assert np.max(np.abs((yt - phi0) - om * 1.0)) < 1e-12


def test_disk_dense_brute_force_inertia():
    n1, n2, P = 11, 13, 3
    n = n1 * n2
    idx = np.arange(n)
    x, y = idx % n1, idx // n1
    A = np.zeros((n, n))
    for ox, oy in zip(*disk_offsets(P)):
        A[idx, (x + ox) % n1 + n1 * ((y + oy) % n2)] += 1.0
    prm = inert(0.2, 1.1, 0.45, 1.5, 0.2)
    y0 = np.concatenate([inputs.kuramoto_phases(16, n), inputs.uniform_range(17, inputs.TAG_MISC, n, -1, 1)])
    ref = dense_rk4(inertia_dense(A, *prm), y0, 0.05, 30)
    yy, _, _ = O.run(O.disk(n1, P, prm, n2=n2, model=O.INERTIA), y0, 0.05, 30)
    assert np.max(np.abs(yy - ref)) / np.max(np.abs(ref)) < 1e-13


# ------------------------------------------------ Dormand-Prince 5(4) stepping
def test_dopri_fixed_step_is_fifth_order():
    """Fixed steps (no control): the error of the inertia zero-coupling closed
    form falls by ~2^5 per halving of the step."""
    n, P = 20, 3
    omega, m, eps = 0.7, 0.5, 0.9
    phi0 = inputs.kuramoto_phases(31, n)
    psi0 = inputs.uniform_range(32, inputs.TAG_MISC, n, -1.0, 1.0)
    t = 4.0
    w = omega / eps
    decay = math.exp(-eps * t / m)
    exact = np.concatenate([phi0 + w * t + (psi0 - w) * (m / eps) * (1 - decay), w + (psi0 - w) * decay])
    errs = []
    for steps in (20, 40, 80):
        y, tr, acc, rej, _ = O.run_dopri(O.ring(O.INERTIA, n, P, inert(omega, 0.0, 1.0, m, eps)),
                                         np.concatenate([phi0, psi0]), t, -1.0, 0.0, t / steps)
        assert acc == steps and rej == 0 and tr == pytest.approx(t, abs=1e-12)
        errs.append(np.max(np.abs(y - exact)))
    assert 28 < errs[0] / errs[1] < 50 and 28 < errs[1] / errs[2] < 50


def test_dopri_constant_field_is_exact():
    """With zero coupling the Kuramoto field is the constant omega: every stage
    and both embedded solutions are exact, so the error estimate is 0 and each
    step is accepted with the largest growth factor."""
    n, P = 30, 4
    y0 = inputs.kuramoto_phases(33, n)
    y, t, acc, rej, hlast = O.run_dopri(O.ring(O.KURAMOTO, n, P, kur(0.37, 0.0, 1.0)), y0, 10.0, 1e-9, 1e-12, 0.01)
    assert np.max(np.abs(y - (y0 + 0.37 * 10.0))) < 1e-12
    assert rej == 0 and t == pytest.approx(10.0, abs=1e-12)


@pytest.mark.parametrize("rtol", [1e-6, 1e-9])
def test_dopri_tolerance_proportionality_against_library(rtol):
    """Adaptive runs of a coupled FHN ring agree with scipy's DOP853 at a tight
    tolerance to within a small multiple of the requested rtol."""
    n, P = 40, 6
    prm = np.array([0.05, 0.5, 0.1, math.pi / 2 - 0.1])
    y0 = inputs.fhn_circle(34, n)
    net = O.ring(O.FHN, n, P, prm)
    y, t, acc, rej, _ = O.run_dopri(net, y0, 2.0, rtol, rtol * 1e-3, 1e-3)
    sol = solve_ivp(lambda _t, yy: O.rhs(net, yy), (0.0, 2.0), y0, method="DOP853", rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1]
    assert t == pytest.approx(2.0, abs=1e-12) and acc > 0
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 100 * rtol


def scipy_rk45_run(net, y0, t_end, rtol, atol, h0):
    """Step scipy's RK45 (the same Dormand-Prince pair and textbook controller)
    to t_end; returns (y, t, accepted, rejected, next proposed step). Every
    attempt costs six right-hand-side calls after the first one at t = 0."""
    from scipy.integrate import RK45
    s = RK45(lambda _t, yy: O.rhs(net, yy), 0.0, np.array(y0, dtype=np.float64), t_end, rtol=rtol, atol=atol,
             first_step=h0)
    acc = 0
    while s.status == "running":
        s.step()
        acc += 1
    assert s.status == "finished"
    attempts = (s.nfev - 1) // 6
    assert s.nfev == 1 + 6 * attempts
    return s.y, s.t, acc, attempts - acc, s.h_abs


@pytest.mark.parametrize("case", ["fhn", "kuramoto", "inertia"])
def test_dopri_controller_takes_the_library_steps(case):
    """The step-size controller (error norm, accept test, growth and shrink
    factors, facmax = 1 after a rejection, the last step cut to t_end) follows
    the textbook Dormand-Prince controller that scipy's RK45 implements: the
    same accepted and rejected step counts, the same next proposed step and the
    same final state. A wrong exponent, safety factor or norm, or a missing
    facmax = 1 after a rejection, changes the step sequence."""
    if case == "fhn":
        n, P, prm = 48, 9, np.array([0.05, 0.5, 0.1, math.pi / 2 - 0.1])
        net, y0, t_end, rtol, atol, h0 = O.ring(O.FHN, n, P, prm), inputs.fhn_circle(41, n), 3.0, 1e-7, 1e-9, 0.05
    elif case == "kuramoto":
        n, P = 64, 16
        net = O.ring(O.KURAMOTO, n, P, kur(0.0, 1.0, 1.46))
        y0, t_end, rtol, atol, h0 = inputs.kuramoto_phases(42, n), 20.0, 1e-9, 1e-11, 0.5
    else:
        n, P = 40, 5
        net = O.ring(O.INERTIA, n, P, inert(0.1, 1.0, 0.45, 1.0, 0.05))
        y0 = np.concatenate([inputs.kuramoto_phases(43, n), np.zeros(n)])
        t_end, rtol, atol, h0 = 10.0, 1e-6, 1e-8, 1.0
    y, t, acc, rej, h = O.run_dopri(net, y0, t_end, rtol, atol, h0)
    ys, ts, accs, rejs, hs = scipy_rk45_run(net, y0, t_end, rtol, atol, h0)
    assert rej > 0, "the case must exercise rejections"
    assert (acc, rej) == (accs, rejs)
    assert t == ts == t_end
    # err is a small difference of two solutions, so its rounding (summation order)
    # moves the proposed steps at the 1e-8 level; a wrong exponent or factor moves them by O(1)
    assert h == pytest.approx(hs, rel=1e-6)
    assert np.max(np.abs(y - ys)) / np.max(np.abs(ys)) < 1e-12


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_dopri_non_finite_state_fails_at_once(bad):
    """A non-finite state gives a non-finite error estimate; the controlled run
    stops at the first attempt instead of rejecting until max_steps."""
    n, P = 32, 4
    y0 = inputs.kuramoto_phases(44, n)
    y0[5] = bad
    with pytest.raises(O.DopriFailure) as ei:
        O.run_dopri(O.ring(O.KURAMOTO, n, P, kur(0.0, 1.0, 1.46)), y0, 1.0, 1e-8, 1e-10, 0.01, max_steps=10 ** 6)
    _, t, acc, rej, _ = ei.value.result
    assert (t, acc, rej) == (0.0, 0, 0)


def test_dopri_step_floor():
    """A proposed step below 10 units in the last place of t ends the run (the
    floor of scipy's solvers); at t = 0 that floor is 10 times the smallest
    subnormal, and a step just above it is taken."""
    n, P = 32, 4
    net = O.ring(O.KURAMOTO, n, P, kur(0.3, 0.0, 1.46))
    y0 = inputs.kuramoto_phases(45, n)
    tiny = 10 * np.nextafter(0.0, 1.0)
    with pytest.raises(O.DopriFailure):
        O.run_dopri(net, y0, 1.0, 1e-8, 1e-10, tiny / 2)
    _, t, acc, _, _ = O.run_dopri(net, y0, 1.0, 1e-8, 1e-10, tiny * 2)
    assert t == 1.0 and acc > 0


def test_fhn_mean_phase_velocity_unwraps_the_geometric_phase():
    """Uncoupled FHN oscillators (sigma = 0) on a limit cycle around the origin:
    the oracle's mean phase velocity (atan2(v, u) unwrapped step by step) equals
    the slope of np.unwrap(atan2(v, u)) sampled densely along an independent
    DOP853 solution, over many cycles. Without the unwrap the value would be off
    by 2 pi x cycles / time; a sign error flips it."""
    n = 6
    eps, a = 0.05, 0.5
    prm = np.array([eps, a, 0.0, math.pi / 2 - 0.1])
    net = O.ring(O.FHN, n, 1, prm)
    y0 = inputs.fhn_circle(46, n)
    dt, steps, mv0 = 0.01, 6000, 1500
    _, _, mv = O.run(net, y0, dt, steps, mv_start=mv0)
    t0, t1 = mv0 * dt, steps * dt
    ts = np.linspace(0.0, t1, 600001)
    ref = np.empty(n)
    for j in range(n):
        sol = solve_ivp(lambda _t, s: fhn_local(s[0], s[1], eps, a), (0.0, t1), [y0[j], y0[n + j]],
                        method="DOP853", rtol=1e-12, atol=1e-12, t_eval=ts)
        th = np.unwrap(np.arctan2(sol.y[1], sol.y[0]))
        i0 = int(round(t0 / (t1 / 600000)))
        ref[j] = (th[-1] - th[i0]) / (t1 - t0)
    cycles = np.abs(ref) * (t1 - t0) / (2 * math.pi)
    assert np.all(cycles > 5), "the horizon must cover several cycles"
    assert np.max(np.abs(mv - ref)) < 1e-4 * np.max(np.abs(ref))


# ------------------------------------------- compressed coupling matrix (Alg. 2)
from oracle import compress as CM  # noqa: E402


def test_compress_full_mesh_is_all_ones_and_one_empty_entry():
    """Sec. III.C: a full mesh compresses to a common vector with every bit set
    and a single difference-table entry with no bit set."""
    n = 12
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    V, D, C = CM.compress(n, rp, col)
    assert V == list(range(n)) and D == [[]] and np.all(C == 0)
    # without self links every row shifts onto row 0 as well
    col = np.array([j for i in range(n) for j in range(n) if j != i], dtype=np.int32)
    rp = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64)
    V, D, C = CM.compress(n, rp, col)
    assert V == list(range(1, n)) and D == [[]] and np.all(C == 0)


@pytest.mark.parametrize("n,P", [(10, 1), (33, 7), (64, 31)])
def test_compress_ring_has_one_entry(n, P):
    """A ring is translation invariant: one (empty) entry, V = row 0."""
    V, D, C = CM.compress(n, *inputs.ring_links(n, P))
    assert V == list(range(1, P + 1)) + list(range(n - P, n))
    assert D == [[]] and np.all(C == 0)


@pytest.mark.parametrize("density", [0.0, 0.05, 0.3, 0.9, 1.0])
def test_compress_extract_round_trip_random(density):
    """EXTRACT inverts COMPRESS on every row of arbitrary matrices (brute force
    over all rows; self links and empty rows included)."""
    n = 37
    rp, col = inputs.random_links(int(100 * density) + 3, n, density)
    V, D, C = CM.compress(n, rp, col)
    rp2, col2 = CM.extract_all(n, V, D, C)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    assert len(D) == len({tuple(d) for d in D}) <= n and D[0] == []


def test_compress_small_world_round_trip_and_entries():
    """A ring with a few shortcuts: the rows without a shortcut share the empty
    entry, every row with shortcuts has an entry holding exactly its shortcuts
    (shifted onto row 0's frame)."""
    n, P = 200, 5
    rp, col = inputs.small_world_links(11, n, P, 12)
    V, D, C = CM.compress(n, rp, col)
    rp2, col2 = CM.extract_all(n, V, D, C)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    ring_rows = CM.rows_of(n, *inputs.ring_links(n, P))
    rows = CM.rows_of(n, rp, col)
    for i in range(n):
        extra = rows[i] - ring_rows[i]
        assert sorted((j - i) % n for j in extra) == D[C[i]]


def boundary_pattern(i, n1, n2, n3, P):
    """Which coordinates of element i lie within P of a lattice face; with a
    periodic flattened index, a wrap in z shifts by n1*n2*n3 = n (a multiple of
    n), a wrap in y (on a 3D lattice) or x does not."""
    x, y = i % n1, (i // n1) % n2
    px = x if x < P else (x - n1 if x >= n1 - P else None)
    py = None if n3 == 1 else (y if y < P else (y - n2 if y >= n2 - P else None))
    return px, py


@pytest.mark.parametrize("dims,P", [((9, 8, 7), 2), ((11, 10, 5), 1), ((13, 9, 1), 3), ((7, 7, 7), 3)])
def test_compress_lattice_entries_are_boundary_patterns(dims, P):
    """On the flattened periodic lattice with the ball (disk) neighbourhood two
    rows share an entry exactly when they share a boundary pattern: (2P+1)^2
    entries in 3D, 2P+1 on the plane."""
    n1, n2, n3 = dims
    n = n1 * n2 * n3
    V, D, C = CM.compress(n, *inputs.lattice_ball_links(n1, n2, n3, P))
    pats = [boundary_pattern(i, n1, n2, n3, P) for i in range(n)]
    assert len(D) == len(set(pats)) == ((2 * P + 1) ** 2 if n3 > 1 else 2 * P + 1)
    first = {}
    for i, p in enumerate(pats):
        assert first.setdefault(p, C[i]) == C[i]


def test_links_rhs_reduces_to_the_structured_topologies():
    """Given the rows of a ring, a ball or a disk, the row-list RHS equals the
    oracle's ring / ball / disk RHS (pinned above) up to summation order."""
    prm = kur(0.2, 1.1, 0.9)
    n, P = 57, 9
    z = inputs.kuramoto_phases(5, n)
    a = O.rhs(O.links(O.KURAMOTO, n, *inputs.ring_links(n, P), prm), z)
    assert np.max(np.abs(a - O.rhs(O.ring(O.KURAMOTO, n, P, prm), z))) < 1e-14
    dims, P = (9, 8, 7), 2
    n = 9 * 8 * 7
    z = inputs.kuramoto_phases(6, n)
    a = O.rhs(O.links(O.KURAMOTO, n, *inputs.lattice_ball_links(*dims, P), prm), z)
    assert np.max(np.abs(a - O.rhs(O.ball(9, P, prm, n2=8, n3=7), z))) < 1e-14
    n = 13 * 11
    z = inputs.kuramoto_phases(7, n)
    a = O.rhs(O.links(O.KURAMOTO, n, *inputs.lattice_ball_links(13, 11, 1, 3), prm), z)
    assert np.max(np.abs(a - O.rhs(O.disk(13, 3, prm, n2=11), z))) < 1e-14
    fhn = np.array([0.05, 0.5, 0.1, math.pi / 2 - 0.1])
    n, P = 40, 13
    z = inputs.fhn_circle(8, n)
    a = O.rhs(O.links(O.FHN, n, *inputs.ring_links(n, P), fhn), z)
    b = O.rhs(O.ring(O.FHN, n, P, fhn), z)
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-14


def links_dense(A, model, prm):
    """Dense formulation with per-row link counts (an empty row: no coupling)."""
    n = A.shape[0]
    L = A.sum(axis=1)
    Linv = np.where(L > 0, 1.0 / np.maximum(L, 1), 0.0)
    if model == O.FHN:
        eps, a, sigma, phi = prm
        B = np.array([[math.cos(phi), math.sin(phi)], [-math.sin(phi), math.cos(phi)]])

        def F(s):
            u, v = s[:n], s[n:]
            Du, Dv = A @ u - L * u, A @ v - L * v
            cu = sigma * Linv * (B[0, 0] * Du + B[0, 1] * Dv)
            cv = sigma * Linv * (B[1, 0] * Du + B[1, 1] * Dv)
            return np.concatenate([(u - u ** 3 / 3 - v + cu) / eps, u + a + cv])
        return F
    omega, mu, alpha = prm[:3]

    def coup(phi):
        return np.imag(np.exp(-1j * (phi + alpha)) * (A @ np.exp(1j * phi))) * Linv
    if model == O.KURAMOTO:
        return lambda phi: omega + mu * coup(phi)
    m, eps = prm[3], prm[4]
    return lambda y: np.concatenate([y[n:], (omega - eps * y[n:] + mu * coup(y[:n])) / m])


@pytest.mark.parametrize("model", [O.KURAMOTO, O.INERTIA, O.FHN])
def test_links_dense_brute_force(model):
    n = 45
    rp, col = inputs.random_links(21, n, 0.15)
    A = np.zeros((n, n))
    for i in range(n):
        if i % 11 != 3:  # rows 3, 14, 25, 36 are left empty
            A[i, col[rp[i]:rp[i + 1]]] = 1.0
    rp = np.concatenate([[0], np.cumsum(A.sum(axis=1))]).astype(np.int64)
    col = np.nonzero(A)[1].astype(np.int32)
    assert np.any(A.sum(axis=1) == 0) and np.any(np.diag(A) == 1)  # empty rows and self links occur
    prm = {O.KURAMOTO: [0.3, 1.2, 1.1], O.INERTIA: [0.3, 1.2, 1.1, 0.8, 0.2],
           O.FHN: [0.05, 0.5, 0.1, math.pi / 2 - 0.1]}[model]
    if model == O.FHN:
        y0 = inputs.fhn_circle(4, n)
    elif model == O.INERTIA:
        y0 = np.concatenate([inputs.kuramoto_phases(4, n), inputs.uniform_range(4, inputs.TAG_MISC, n, -0.5, 0.5)])
    else:
        y0 = inputs.kuramoto_phases(4, n)
    ref = dense_rk4(links_dense(A, model, prm), y0, 0.01, 100)
    y, _, _ = O.run(O.links(model, n, rp, col, np.array(prm)), y0, 0.01, 100)
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-12


# ------------------------------------------------ Dormand-Prince dense output
def test_dopri_dense_weights_match_the_library_interpolant():
    """The fourth-order continuous extension equals scipy's RK45 interpolant
    (its P matrix) at every theta, vanishes at theta = 0 and gives the
    fifth-order weights at theta = 1."""
    from scipy.integrate._ivp.rk import RK45
    for th in np.linspace(0.0, 1.0, 41):
        ref = RK45.P @ np.array([th, th ** 2, th ** 3, th ** 4])
        assert np.max(np.abs(O.dopri_dense_weights(th) - ref)) < 2e-15
    b = np.array([35 / 384, 0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0])
    assert np.max(np.abs(O.dopri_dense_weights(1.0) - b)) < 1e-15
    assert np.all(O.dopri_dense_weights(0.0) == 0.0)


def test_dopri_dense_output_follows_the_inertia_closed_form():
    """mu = 0: the dense outputs between accepted steps follow the damped-rotor
    closed form to the tolerance's order, and R is the order parameter of the
    interpolated state."""
    n, P = 30, 3
    omega, m, eps = 0.7, 2.5, 0.4
    phi0 = inputs.kuramoto_phases(15, n)
    psi0 = inputs.uniform_range(16, inputs.TAG_MISC, n, -1.0, 1.0)
    net = O.ring(O.INERTIA, n, P, inert(omega, 0.0, 1.0, m, eps))
    t_end, t_out = 7.3, 0.25
    y, t, acc, rej, _, R, Y = O.run_dopri_dense(net, np.concatenate([phi0, psi0]), t_end, 1e-10, 1e-12, 1e-3,
                                                t_out, states=True)
    K = int(t_end / t_out)
    assert t == t_end and acc < 3 * K  # steps are longer than the output spacing
    w = omega / eps
    for k in range(K + 1):
        tk = k * t_out
        decay = math.exp(-eps * tk / m)
        psi = w + (psi0 - w) * decay
        phi = phi0 + w * tk + (psi0 - w) * (m / eps) * (1.0 - decay)
        assert np.max(np.abs(Y[k, n:] - psi)) < 1e-8
        assert np.max(np.abs(Y[k, :n] - phi)) < 1e-8
        assert R[k] == pytest.approx(O.order_parameter(O.INERTIA, n, Y[k]), abs=1e-15)


def test_dopri_dense_output_at_step_ends_is_the_step_state():
    """Fixed steps (rtol <= 0) with outputs on step ends: theta = 1 gives the
    state the solver reached there (a separate run to that time)."""
    n, P = 40, 9
    fhn = np.array([0.05, 0.5, 0.1, math.pi / 2 - 0.1])
    net = O.ring(O.FHN, n, P, fhn)
    y0 = inputs.fhn_circle(17, n)
    _, _, acc, _, _, R, Y = O.run_dopri_dense(net, y0, 1.0, -1.0, 0.0, 0.02, 0.1, states=True)
    assert acc == 50
    for k in (1, 4, 10):
        ref, _, _, _, _ = O.run_dopri(net, y0, 0.1 * k, -1.0, 0.0, 0.02)
        assert np.max(np.abs(Y[k] - ref)) < 1e-12
    assert np.array_equal(Y[0], y0)
