"""ctypes wrapper around liboracle.so (the plain FP64 CPU oracle, oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.

Model / topology codes and parameter vectors follow oracle.c:
  Kuramoto  params = (omega, mu, alpha)                       Eq. (3), m=0, eps=1
  FHN       params = (eps, a, sigma, phi)                     Eq. (2) + rotational coupling
  HH        params = (C, gNa, gK, gL, ENa, EK, EL, Esyn, theta_s, k_s)   Eq. (1)
  Inertia   params = (omega, mu, alpha, m, eps)                Eq. (3), m != 0; state (phi, psi)
"""
import ctypes
import os

import numpy as np

KURAMOTO, FHN, HH, INERTIA = 0, 1, 2, 3
RING, CUBE, CSR, BALL, DISK, LINKS = 0, 1, 2, 3, 4, 5
NVARS = {KURAMOTO: 1, FHN: 2, HH: 4, INERTIA: 2}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_rhs.restype = i32
        L.orc_rhs.argtypes = [i32, i32, i64, i64, i64, i64, i64, dp, dp, dp, dp, dp, i32, dp, dp]
        L.orc_run.restype = i32
        L.orc_run.argtypes = [i32, i32, i64, i64, i64, i64, i64, dp, dp, dp, dp, dp, i32,
                              dp, ctypes.c_double, i64, dp, i64, dp, i64]
        L.orc_run_dopri.restype = i32
        L.orc_run_dopri.argtypes = [i32, i32, i64, i64, i64, i64, i64, dp, dp, dp, dp, dp, dp,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, i64, dp]
        L.orc_run_dopri_dense.restype = i32
        L.orc_run_dopri_dense.argtypes = [i32, i32, i64, i64, i64, i64, i64, dp, dp, dp, dp, dp, dp,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, i64,
                                          dp, ctypes.c_double, dp, dp]
        L.orc_dopri_dense_weights.restype = None
        L.orc_dopri_dense_weights.argtypes = [ctypes.c_double, dp]
        L.orc_order_parameter.restype = ctypes.c_double
        L.orc_order_parameter.argtypes = [i32, i64, dp]
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Net:
    """A network description for the oracle (plain data, no arithmetic)."""

    def __init__(self, model, topo, n, params, radius=0, dims=(0, 0, 0), row_ptr=None,
                 col=None, w=None, per_elem=None):
        self.model, self.topo, self.n, self.radius = int(model), int(topo), int(n), int(radius)
        self.dims = tuple(int(d) for d in dims)
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.row_ptr = None if row_ptr is None else np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = None if col is None else np.ascontiguousarray(col, dtype=np.int32)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        self.per_elem = None if per_elem is None else np.ascontiguousarray(per_elem, dtype=np.float64)

    @property
    def nvars(self):
        return NVARS[self.model]

    def _args(self):
        n1, n2, n3 = self.dims
        return (self.model, self.topo, self.n, self.radius, n1, n2, n3, _p(self.row_ptr),
                _p(self.col), _p(self.w), _p(self.params), _p(self.per_elem))


def ring(model, n, P, params):
    return Net(model, RING, n, params, radius=P)


def cube(n1, h, params, n2=None, n3=None, model=KURAMOTO):
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    return Net(model, CUBE, n1 * n2 * n3, params, radius=h, dims=(n1, n2, n3))


def ball(n1, P, params, n2=None, n3=None, model=KURAMOTO):
    """Periodic lattice, neighbours = lattice points within distance P, centre included."""
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    return Net(model, BALL, n1 * n2 * n3, params, radius=P, dims=(n1, n2, n3))


def disk(n1, P, params, n2=None, model=KURAMOTO):
    """Periodic n1 x n2 plane, neighbours = lattice points within distance P, centre included."""
    n2 = n1 if n2 is None else n2
    return Net(model, DISK, n1 * n2, params, radius=P, dims=(n1, n2, 1))


def links(model, n, row_ptr, col, params):
    """Arbitrary binary coupling matrix by rows: row i lists the j with L_ij = 1
    (summed in the listed order, divided by the row's link count)."""
    return Net(model, LINKS, n, params, row_ptr=row_ptr, col=col)


def csr(n, row_ptr, col, w, params, i_app):
    return Net(HH, CSR, n, params, row_ptr=row_ptr, col=col, w=w, per_elem=i_app)


def rhs(net, z, reverse=False):
    z = np.ascontiguousarray(z, dtype=np.float64)
    assert z.size == net.nvars * net.n
    f = np.empty_like(z)
    rc = lib().orc_rhs(*net._args(), int(reverse), _p(z), _p(f))
    if rc != 0:
        raise ValueError(f"orc_rhs failed ({rc})")
    return f


def run(net, y0, dt, steps, record_every=0, mv_start=None, reverse=False):
    """Integrate with classical RK4; returns (y, R or None, mean_velocity or None)."""
    y = np.array(y0, dtype=np.float64, copy=True).ravel()
    assert y.size == net.nvars * net.n
    R = np.empty(steps // record_every + 1) if record_every else None
    mv = np.empty(net.n) if mv_start is not None else None
    rc = lib().orc_run(*net._args(), int(reverse), _p(y), float(dt), int(steps), _p(R),
                       int(record_every), _p(mv), int(mv_start or 0))
    if rc != 0:
        raise ValueError(f"orc_run failed ({rc})")
    return y, R, mv


def order_parameter(model, n, y):
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_order_parameter(int(model), int(n), _p(y))


class DopriFailure(FloatingPointError):
    """A controlled Dormand-Prince run stopped: its error estimate was not finite
    or its proposed step fell below 10 units in the last place of t.  `result`
    holds (y, t reached, accepted, rejected, last proposed step) at the stop."""

    def __init__(self, result):
        super().__init__(f"Dormand-Prince run failed at t={result[1]!r} after {result[2]} accepted steps")
        self.result = result


ORC_ENUMERIC = -5


def run_dopri(net, y0, t_end, rtol, atol, dt0, max_steps=10 ** 7):
    """Dormand-Prince 5(4) with step-size control (rtol <= 0: fixed steps of dt0);
    returns (y, t reached, accepted steps, rejected steps, last proposed step).
    Raises DopriFailure when a controlled run fails (non-finite error estimate,
    step below its floor)."""
    y = np.array(y0, dtype=np.float64, copy=True).ravel()
    assert y.size == net.nvars * net.n
    st = np.zeros(4)
    n1, n2, n3 = net.dims
    rc = lib().orc_run_dopri(net.model, net.topo, net.n, net.radius, n1, n2, n3, _p(net.row_ptr), _p(net.col),
                             _p(net.w), _p(net.params), _p(net.per_elem), _p(y), float(t_end), float(rtol),
                             float(atol), float(dt0), int(max_steps), _p(st))
    if rc == ORC_ENUMERIC:
        raise DopriFailure((y, st[0], int(st[1]), int(st[2]), st[3]))
    if rc != 0:
        raise ValueError(f"oracle dopri run failed ({rc})")
    return y, st[0], int(st[1]), int(st[2]), st[3]


def run_dopri_dense(net, y0, t_end, rtol, atol, dt0, t_out, states=False, max_steps=10 ** 7):
    """Dormand-Prince as run_dopri, plus R (and, with states=True, the state) at the
    output times k * t_out from the dense output; returns
    (y, t, accepted, rejected, h_next, R, Y or None)."""
    y = np.array(y0, dtype=np.float64, copy=True).ravel()
    K = int(np.floor(t_end / t_out))
    R = np.full(K + 1, np.nan)
    Y = np.full((K + 1, y.size), np.nan) if states else None
    st = np.zeros(4)
    n1, n2, n3 = net.dims
    rc = lib().orc_run_dopri_dense(net.model, net.topo, net.n, net.radius, n1, n2, n3, _p(net.row_ptr),
                                   _p(net.col), _p(net.w), _p(net.params), _p(net.per_elem), _p(y), float(t_end),
                                   float(rtol), float(atol), float(dt0), int(max_steps), _p(st), float(t_out),
                                   _p(R), _p(Y))
    if rc == ORC_ENUMERIC:
        raise DopriFailure((y, st[0], int(st[1]), int(st[2]), st[3]))
    if rc != 0:
        raise ValueError(f"oracle dense dopri run failed ({rc})")
    return y, st[0], int(st[1]), int(st[2]), st[3], R, Y


def dopri_dense_weights(theta):
    w = np.empty(7)
    lib().orc_dopri_dense_weights(float(theta), _p(w))
    return w
