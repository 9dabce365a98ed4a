/*
 * FP64 CPU oracle for the network-dynamics hot path of Sudakov & Maistrenko,
 * "Parallelization of Network Dynamics Computations in Heterogeneous
 * Distributed Environment" (arXiv 2410.19075).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The product path (the HIP library) never links, includes or
 * calls it, and it never includes anything from the product path.
 *
 * What it computes is the plain definition: every right-hand side takes each
 * neighbour term directly, in a fixed order, exactly as the per-oscillator
 * link loop of the paper's model API does (Sec. III.B, Alg. 1: accumulate
 * sin(phi_j - phi_i - alpha) over the links, then divide by the link count),
 * and the integrator is the classical fixed-step fourth-order Runge-Kutta
 * scheme.  Arithmetic is IEEE double with libm sin/cos/exp/expm1/atan2.
 * OpenMP splits the element loop only; every element's sum runs serially in
 * the stated order, so results do not depend on the thread count.
 *
 * Models (state is variable-major: all of variable 0, then variable 1, ...):
 *   Kuramoto-Sakaguchi phase oscillators, Eq. (3) with m = 0, eps = 1 plus a
 *     natural frequency omega (zero reproduces the paper):
 *       dphi_i/dt = omega + (mu / L) * sum_{j in nbr(i)} sin(phi_j - phi_i - alpha)
 *     on a ring (neighbours i+-1..i+-P, L = 2P, Sec. IV 1D study, mu = 1/2P)
 *     or on a periodic n1 x n2 x n3 lattice with the cube neighbourhood of
 *     half-width h minus the element itself (L = (2h+1)^3 - 1); lattice index
 *     x + n1*y + n1*n2*z as in the paper's 3D index map (Sec. IV).
 *   Kuramoto-Sakaguchi with inertia, Eq. (3) with m != 0 (plus omega), as a
 *     first-order system in (phi, psi = dphi/dt), same neighbourhoods:
 *       dphi_i/dt = psi_i
 *       m dpsi_i/dt = omega - eps psi_i + (mu / L) * sum_j sin(phi_j - phi_i - alpha)
 *   Both Kuramoto models also run on the periodic lattice with the ball
 *     neighbourhood of the paper's 3D studies: every lattice point within
 *     Euclidean distance P, the element itself included (Sec. V counts 33 links
 *     for P = 2 and 925 for P = 6), L = that count, taken in lexicographic
 *     (dz, dy, dx) order; and on the periodic n1 x n2 plane with the disk of
 *     radius P (the 2D studies), centre included, in (dy, dx) order.
 *   FitzHugh-Nagumo, Eq. (2) with tau = 0, D = 0, I_app = 0 and a rotational
 *     coupling matrix B(phi) acting on (u_j - u_i, v_j - v_i), averaged over
 *     the 2P ring neighbours and placed inside the eps-scaled fast equation:
 *       eps du_i/dt = u_i - u_i^3/3 - v_i + k * sum_j ( cos phi du_j + sin phi dv_j)
 *           dv_i/dt = u_i + a         + k * sum_j (-sin phi du_j + cos phi dv_j)
 *     with k = sigma / (2P).
 *   The Kuramoto models and FitzHugh-Nagumo also run on an arbitrary binary
 *     coupling matrix given by rows (topology LINKS: row i lists the
 *     presynaptic elements j with L_ij = 1, Sec. III.C), each sum divided by
 *     the row's own link count Omega_i as Alg. 1 divides by its link count; a
 *     row without links contributes no coupling.  The links are taken in the
 *     order the row lists them.
 *   Hodgkin-Huxley, Eq. (1) specialised to the squid axon (Na, K, leak) with
 *     an instantaneous sigmoidal synapse S(V) on a directed graph stored as
 *     CSR by target (sources ascending):
 *       C dV_i/dt = I_i - gNa m^3 h (V-ENa) - gK n^4 (V-EK) - gL (V-EL)
 *                   + (Esyn - V_i) * sum_{e in in(i)} w_e S(V_src(e))
 *       dx/dt = alpha_x(V)(1 - x) - beta_x(V) x,  x in {m, h, n}
 *     The paper leaves the channel kinetics generic; the textbook squid rate
 *     functions in the modern (rest = -65 mV) convention are used.
 *
 * parity: every function here is pinned by tests/test_oracle_pins.py
 * (closed forms, invariants, dense brute force, library integrators).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENUMERIC -5 /* Dormand-Prince: non-finite error estimate or step below its floor */

enum { ORC_KURAMOTO = 0, ORC_FHN = 1, ORC_HH = 2, ORC_INERTIA = 3 };
enum { ORC_RING = 0, ORC_CUBE = 1, ORC_CSR = 2, ORC_BALL = 3, ORC_DISK = 4, ORC_LINKS = 5 };

typedef struct {
    int model, topo;
    int64_t n;          /* elements */
    int64_t radius;     /* ring: P; cube: h */
    int64_t n1, n2, n3; /* cube extents */
    const int64_t* row_ptr; /* CSR by target, n+1 entries */
    const int32_t* col;     /* source of each in-edge, ascending per row */
    const double* w;        /* weight of each in-edge */
    const double* prm;      /* model parameters */
    const double* per_elem; /* HH: applied current per neuron */
    int reverse;            /* 1: take every neighbour sum in reverse order */
} orc_net;

static int64_t wrapi(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* ---------------------------------------------------------------- Kuramoto */
/* Coupling term of element i: (1/L) sum_{j in nbr(i)} sin(phi_j - phi_i - alpha),
 * the neighbour sum of Eq. (3) divided by the link count (Alg. 1). */
static double kuramoto_ring_coupling(const orc_net* m, const double* z, int64_t i, double alpha) {
    const int64_t n = m->n, P = m->radius;
    double s = 0.0;
    /* neighbour order: i-P, ..., i-1, i+1, ..., i+P (or reversed) */
    for (int64_t t = 0; t < 2 * P; ++t) {
        int64_t q = m->reverse ? (2 * P - 1 - t) : t;
        int64_t k = (q < P) ? (q - P) : (q - P + 1);
        int64_t j = wrapi(i + k, n);
        s += sin(z[j] - z[i] - alpha);
    }
    return s * (1.0 / (double)(2 * P));
}

/* Kuramoto, prm = {omega, mu, alpha} */
static void rhs_kuramoto_ring(const orc_net* m, const double* z, double* f) {
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->n; ++i) f[i] = omega + mu * kuramoto_ring_coupling(m, z, i, alpha);
}

/* Kuramoto with inertia, prm = {omega, mu, alpha, m, eps}; z = (phi, psi) */
static void rhs_inertia_ring(const orc_net* m, const double* z, double* f) {
    const int64_t n = m->n;
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2], mass = m->prm[3], eps = m->prm[4];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double psi = z[n + i];
        f[i] = psi;
        f[n + i] = (omega - eps * psi + mu * kuramoto_ring_coupling(m, z, i, alpha)) / mass;
    }
}

static double kuramoto_cube_coupling(const orc_net* m, const double* z, int64_t i, double alpha) {
    const int64_t n1 = m->n1, n2 = m->n2, n3 = m->n3, h = m->radius;
    const int64_t side = 2 * h + 1;
    const int64_t links = side * side * side - 1;
    const int64_t x = i % n1, y = (i / n1) % n2, zz = i / (n1 * n2);
    double s = 0.0;
    /* lexicographic dz, dy, dx in [-h, h], self skipped (or reversed) */
    for (int64_t t = 0; t < side * side * side; ++t) {
        int64_t q = m->reverse ? (side * side * side - 1 - t) : t;
        int64_t dz = q / (side * side) - h;
        int64_t dy = (q / side) % side - h;
        int64_t dx = q % side - h;
        if (dx == 0 && dy == 0 && dz == 0) continue;
        int64_t j = wrapi(x + dx, n1) + n1 * (wrapi(y + dy, n2) + n2 * wrapi(zz + dz, n3));
        s += sin(z[j] - z[i] - alpha);
    }
    return s * (1.0 / (double)links);
}

/* Ball neighbourhood: lattice offsets with dx^2 + dy^2 + dz^2 <= P^2, the
 * centre included, lexicographic (dz, dy, dx) (or reversed). */
static int64_t ball_links(int64_t P) {
    int64_t c = 0;
    for (int64_t dz = -P; dz <= P; ++dz)
        for (int64_t dy = -P; dy <= P; ++dy)
            for (int64_t dx = -P; dx <= P; ++dx)
                if (dx * dx + dy * dy + dz * dz <= P * P) ++c;
    return c;
}

static int64_t disk_links(int64_t P) {
    int64_t c = 0;
    for (int64_t dy = -P; dy <= P; ++dy)
        for (int64_t dx = -P; dx <= P; ++dx)
            if (dx * dx + dy * dy <= P * P) ++c;
    return c;
}

/* The ball (3D) or the disk (2D: the z offset is always 0). */
static double kuramoto_ball_coupling(const orc_net* m, const double* z, int64_t i, double alpha) {
    const int64_t n1 = m->n1, n2 = m->n2, n3 = m->n3, P = m->radius;
    const int disk = m->topo == ORC_DISK;
    const int64_t side = 2 * P + 1, cells = disk ? side * side : side * side * side;
    const int64_t x = i % n1, y = (i / n1) % n2, zz = i / (n1 * n2);
    double s = 0.0;
    for (int64_t t = 0; t < cells; ++t) {
        int64_t q = m->reverse ? (cells - 1 - t) : t;
        int64_t dz = disk ? 0 : q / (side * side) - P;
        int64_t dy = (q / side) % side - P;
        int64_t dx = q % side - P;
        if (dx * dx + dy * dy + dz * dz > P * P) continue;
        int64_t j = wrapi(x + dx, n1) + n1 * (wrapi(y + dy, n2) + n2 * wrapi(zz + dz, n3));
        s += sin(z[j] - z[i] - alpha);
    }
    return s * (1.0 / (double)(disk ? disk_links(P) : ball_links(P)));
}

static void rhs_kuramoto_ball(const orc_net* m, const double* z, double* f) {
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->n; ++i) f[i] = omega + mu * kuramoto_ball_coupling(m, z, i, alpha);
}

static void rhs_inertia_ball(const orc_net* m, const double* z, double* f) {
    const int64_t n = m->n;
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2], mass = m->prm[3], eps = m->prm[4];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double psi = z[n + i];
        f[i] = psi;
        f[n + i] = (omega - eps * psi + mu * kuramoto_ball_coupling(m, z, i, alpha)) / mass;
    }
}

static void rhs_inertia_cube(const orc_net* m, const double* z, double* f) {
    const int64_t n = m->n;
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2], mass = m->prm[3], eps = m->prm[4];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double psi = z[n + i];
        f[i] = psi;
        f[n + i] = (omega - eps * psi + mu * kuramoto_cube_coupling(m, z, i, alpha)) / mass;
    }
}

static void rhs_kuramoto_cube(const orc_net* m, const double* z, double* f) {
    const int64_t n1 = m->n1, n2 = m->n2, n3 = m->n3, h = m->radius;
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2];
    const int64_t side = 2 * h + 1;
    const int64_t links = side * side * side - 1;
    const double inv_links = 1.0 / (double)links;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->n; ++i) {
        const int64_t x = i % n1, y = (i / n1) % n2, zz = i / (n1 * n2);
        double s = 0.0;
        /* lexicographic dz, dy, dx in [-h, h], self skipped (or reversed) */
        for (int64_t t = 0; t < side * side * side; ++t) {
            int64_t q = m->reverse ? (side * side * side - 1 - t) : t;
            int64_t dz = q / (side * side) - h;
            int64_t dy = (q / side) % side - h;
            int64_t dx = q % side - h;
            if (dx == 0 && dy == 0 && dz == 0) continue;
            int64_t j = wrapi(x + dx, n1) + n1 * (wrapi(y + dy, n2) + n2 * wrapi(zz + dz, n3));
            s += sin(z[j] - z[i] - alpha);
        }
        f[i] = omega + mu * (s * inv_links);
    }
}

/* --------------------------------------------------------- FitzHugh-Nagumo */
/* prm = {eps, a, sigma, phi}; z = u[0..n) then v[0..n) */
static void rhs_fhn_ring(const orc_net* m, const double* z, double* f) {
    const int64_t n = m->n, P = m->radius;
    const double eps = m->prm[0], a = m->prm[1], sigma = m->prm[2], phi = m->prm[3];
    const double buu = cos(phi), buv = sin(phi), bvu = -sin(phi), bvv = cos(phi);
    const double kappa = sigma / (double)(2 * P);
    const double* u = z;
    const double* v = z + n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double cu = 0.0, cv = 0.0;
        for (int64_t t = 0; t < 2 * P; ++t) {
            int64_t q = m->reverse ? (2 * P - 1 - t) : t;
            int64_t k = (q < P) ? (q - P) : (q - P + 1);
            int64_t j = wrapi(i + k, n);
            double du = u[j] - u[i], dv = v[j] - v[i];
            cu += buu * du + buv * dv;
            cv += bvu * du + bvv * dv;
        }
        f[i] = (u[i] - u[i] * u[i] * u[i] / 3.0 - v[i] + kappa * cu) / eps;
        f[n + i] = u[i] + a + kappa * cv;
    }
}

/* ------------------------------------------------ binary coupling matrix rows */
/* Kuramoto coupling of element i over the links of its row:
 * (1/Omega_i) sum_{j in row i} sin(phi_j - phi_i - alpha), 0 for an empty row. */
static double kuramoto_links_coupling(const orc_net* m, const double* z, int64_t i, double alpha) {
    const int64_t b = m->row_ptr[i], e = m->row_ptr[i + 1];
    if (e == b) return 0.0;
    double s = 0.0;
    for (int64_t t = 0; t < e - b; ++t) {
        const int64_t q = m->reverse ? (e - 1 - t) : (b + t);
        s += sin(z[m->col[q]] - z[i] - alpha);
    }
    return s * (1.0 / (double)(e - b));
}

static void rhs_kuramoto_links(const orc_net* m, const double* z, double* f) {
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->n; ++i) f[i] = omega + mu * kuramoto_links_coupling(m, z, i, alpha);
}

static void rhs_inertia_links(const orc_net* m, const double* z, double* f) {
    const int64_t n = m->n;
    const double omega = m->prm[0], mu = m->prm[1], alpha = m->prm[2], mass = m->prm[3], eps = m->prm[4];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double psi = z[n + i];
        f[i] = psi;
        f[n + i] = (omega - eps * psi + mu * kuramoto_links_coupling(m, z, i, alpha)) / mass;
    }
}

/* FitzHugh-Nagumo with the rotational coupling averaged over the row's links,
 * k = sigma / Omega_i (no coupling for an empty row). */
static void rhs_fhn_links(const orc_net* m, const double* z, double* f) {
    const int64_t n = m->n;
    const double eps = m->prm[0], a = m->prm[1], sigma = m->prm[2], phi = m->prm[3];
    const double buu = cos(phi), buv = sin(phi), bvu = -sin(phi), bvv = cos(phi);
    const double* u = z;
    const double* v = z + n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t b = m->row_ptr[i], e = m->row_ptr[i + 1];
        double cu = 0.0, cv = 0.0;
        for (int64_t t = 0; t < e - b; ++t) {
            const int64_t q = m->reverse ? (e - 1 - t) : (b + t);
            const int64_t j = m->col[q];
            double du = u[j] - u[i], dv = v[j] - v[i];
            cu += buu * du + buv * dv;
            cv += bvu * du + bvv * dv;
        }
        const double kappa = e > b ? sigma / (double)(e - b) : 0.0;
        f[i] = (u[i] - u[i] * u[i] * u[i] / 3.0 - v[i] + kappa * cu) / eps;
        f[n + i] = u[i] + a + kappa * cv;
    }
}

/* ---------------------------------------------------------- Hodgkin-Huxley */
/* x / (1 - exp(-x)), the removable singularity at x = 0 taken by its series */
static double xoverexpm1(double x) {
    if (fabs(x) < 1e-7) return 1.0 + 0.5 * x;
    return x / (-expm1(-x));
}
static double hh_am(double V) { return xoverexpm1((V + 40.0) / 10.0); }
static double hh_bm(double V) { return 4.0 * exp(-(V + 65.0) / 18.0); }
static double hh_ah(double V) { return 0.07 * exp(-(V + 65.0) / 20.0); }
static double hh_bh(double V) { return 1.0 / (1.0 + exp(-(V + 35.0) / 10.0)); }
static double hh_an(double V) { return 0.1 * xoverexpm1((V + 55.0) / 10.0); }
static double hh_bn(double V) { return 0.125 * exp(-(V + 65.0) / 80.0); }

/* prm = {C, gNa, gK, gL, ENa, EK, EL, Esyn, theta_s, k_s}; z = V, m, h, n */
static void rhs_hh_csr(const orc_net* m, const double* z, double* f) {
    const int64_t n = m->n;
    const double C = m->prm[0], gNa = m->prm[1], gK = m->prm[2], gL = m->prm[3];
    const double ENa = m->prm[4], EK = m->prm[5], EL = m->prm[6], Esyn = m->prm[7];
    const double th = m->prm[8], ks = m->prm[9];
    const double *V = z, *M = z + n, *H = z + 2 * n, *Nn = z + 3 * n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t b = m->row_ptr[i], e = m->row_ptr[i + 1];
        double g = 0.0;
        for (int64_t t = 0; t < e - b; ++t) {
            int64_t q = m->reverse ? (e - 1 - t) : (b + t);
            double Vs = V[m->col[q]];
            g += m->w[q] * (1.0 / (1.0 + exp(-(Vs - th) / ks)));
        }
        const double v = V[i], mm = M[i], hh = H[i], nn = Nn[i];
        const double iion = gNa * mm * mm * mm * hh * (v - ENa) + gK * nn * nn * nn * nn * (v - EK) +
                            gL * (v - EL);
        f[i] = (m->per_elem[i] - iion + (Esyn - v) * g) / C;
        f[n + i] = hh_am(v) * (1.0 - mm) - hh_bm(v) * mm;
        f[2 * n + i] = hh_ah(v) * (1.0 - hh) - hh_bh(v) * hh;
        f[3 * n + i] = hh_an(v) * (1.0 - nn) - hh_bn(v) * nn;
    }
}

static int nvars(int model) {
    return model == ORC_KURAMOTO ? 1 : (model == ORC_HH ? 4 : 2);
}

static int rhs(const orc_net* m, const double* z, double* f) {
    if (m->model == ORC_KURAMOTO && m->topo == ORC_RING) rhs_kuramoto_ring(m, z, f);
    else if (m->model == ORC_KURAMOTO && m->topo == ORC_CUBE) rhs_kuramoto_cube(m, z, f);
    else if (m->model == ORC_INERTIA && m->topo == ORC_RING) rhs_inertia_ring(m, z, f);
    else if (m->model == ORC_INERTIA && m->topo == ORC_CUBE) rhs_inertia_cube(m, z, f);
    else if (m->model == ORC_KURAMOTO && (m->topo == ORC_BALL || m->topo == ORC_DISK)) rhs_kuramoto_ball(m, z, f);
    else if (m->model == ORC_INERTIA && (m->topo == ORC_BALL || m->topo == ORC_DISK)) rhs_inertia_ball(m, z, f);
    else if (m->model == ORC_FHN && m->topo == ORC_RING) rhs_fhn_ring(m, z, f);
    else if (m->model == ORC_HH && m->topo == ORC_CSR) rhs_hh_csr(m, z, f);
    else if (m->model == ORC_KURAMOTO && m->topo == ORC_LINKS) rhs_kuramoto_links(m, z, f);
    else if (m->model == ORC_INERTIA && m->topo == ORC_LINKS) rhs_inertia_links(m, z, f);
    else if (m->model == ORC_FHN && m->topo == ORC_LINKS) rhs_fhn_links(m, z, f);
    else return ORC_EINVAL;
    return ORC_OK;
}

static int validate(const orc_net* m) {
    if (m->n <= 0) return ORC_EINVAL;
    if (m->topo == ORC_RING) {
        if (m->radius < 1 || 2 * m->radius + 1 > m->n) return ORC_EINVAL;
    } else if (m->topo == ORC_DISK) {
        int64_t side = 2 * m->radius + 1;
        if (m->radius < 1 || m->n1 < side || m->n2 < side || m->n3 != 1) return ORC_EINVAL;
        if (m->n1 * m->n2 != m->n) return ORC_EINVAL;
    } else if (m->topo == ORC_CUBE || m->topo == ORC_BALL) {
        int64_t side = 2 * m->radius + 1;
        if (m->radius < 1 || m->n1 < side || m->n2 < side || m->n3 < side) return ORC_EINVAL;
        if (m->n1 * m->n2 * m->n3 != m->n) return ORC_EINVAL;
    } else if (m->topo == ORC_CSR || m->topo == ORC_LINKS) {
        if (m->topo == ORC_CSR && (!m->col || !m->w || !m->per_elem)) return ORC_EINVAL;
        if (!m->row_ptr || m->row_ptr[0] != 0) return ORC_EINVAL;
        for (int64_t i = 0; i < m->n; ++i) {
            if (m->row_ptr[i + 1] < m->row_ptr[i]) return ORC_EINVAL;
            for (int64_t q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q)
                if (m->col[q] < 0 || m->col[q] >= m->n) return ORC_EINVAL;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------- observables */
/* Global order parameter R = |sum_j exp(i theta_j)| / n, theta = phi for the
 * Kuramoto model and the geometric phase atan2(v, u) for FitzHugh-Nagumo. */
static double order_parameter(int model, int64_t n, const double* y) {
    double c = 0.0, s = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double th = (model == ORC_FHN) ? atan2(y[n + j], y[j]) : y[j];
        c += cos(th);
        s += sin(th);
    }
    return sqrt(c * c + s * s) / (double)n;
}

static double wrap_pi(double d) {
    /* map an angle difference to (-pi, pi] */
    while (d > M_PI) d -= 2.0 * M_PI;
    while (d <= -M_PI) d += 2.0 * M_PI;
    return d;
}

/* ------------------------------------------------------------------ driver */
static orc_net make_net(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2,
                        int64_t n3, const int64_t* row_ptr, const int32_t* col, const double* w,
                        const double* prm, const double* per_elem, int reverse) {
    orc_net m;
    m.model = model; m.topo = topo; m.n = n; m.radius = radius;
    m.n1 = n1; m.n2 = n2; m.n3 = n3;
    m.row_ptr = row_ptr; m.col = col; m.w = w;
    m.prm = prm; m.per_elem = per_elem; m.reverse = reverse;
    return m;
}

/* One right-hand-side evaluation f = F(z). */
int orc_rhs(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
            const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
            const double* per_elem, int reverse, const double* z, double* f) {
    orc_net m = make_net(model, topo, n, radius, n1, n2, n3, row_ptr, col, w, prm, per_elem, reverse);
    int rc = validate(&m);
    if (rc) return rc;
    return rhs(&m, z, f);
}

/*
 * Classical RK4 with fixed step dt, `steps` steps, in place on y:
 *   k1 = F(y), k2 = F(y + dt/2 k1), k3 = F(y + dt/2 k2), k4 = F(y + dt k3)
 *   y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4)
 * R (if non-NULL) receives the order parameter at t = 0, r, 2r, ... (r =
 * record_every), i.e. steps / r + 1 values.  mean_vel (if non-NULL) receives
 * per element (theta(t_end) - theta(t_start)) / (t_end - t_start) with
 * t_start = mv_start * dt, on unwrapped phases (Kuramoto: phi itself;
 * FitzHugh-Nagumo: atan2(v, u) unwrapped by accumulating each step's increment
 * mapped to (-pi, pi]).
 */
int orc_run(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
            const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
            const double* per_elem, int reverse, double* y, double dt, int64_t steps, double* R,
            int64_t record_every, double* mean_vel, int64_t mv_start) {
    orc_net m = make_net(model, topo, n, radius, n1, n2, n3, row_ptr, col, w, prm, per_elem, reverse);
    int rc = validate(&m);
    if (rc) return rc;
    if (!(dt > 0.0) || steps < 0) return ORC_EINVAL;
    if (R && record_every < 1) return ORC_EINVAL;
    if (mean_vel && (model == ORC_HH || mv_start < 0 || mv_start >= steps)) return ORC_EINVAL;
    const int64_t len = (int64_t)nvars(model) * n;
    double* k1 = (double*)malloc(sizeof(double) * len);
    double* k2 = (double*)malloc(sizeof(double) * len);
    double* k3 = (double*)malloc(sizeof(double) * len);
    double* k4 = (double*)malloc(sizeof(double) * len);
    double* z = (double*)malloc(sizeof(double) * len);
    double* unwrap = mean_vel ? (double*)malloc(sizeof(double) * n) : NULL;
    double* th_prev = (mean_vel && model == ORC_FHN) ? (double*)malloc(sizeof(double) * n) : NULL;
    if (!k1 || !k2 || !k3 || !k4 || !z || (mean_vel && !unwrap) ||
        (mean_vel && model == ORC_FHN && !th_prev)) {
        free(k1); free(k2); free(k3); free(k4); free(z); free(unwrap); free(th_prev);
        return ORC_ENOMEM;
    }
    if (R) R[0] = order_parameter(model, n, y);
    if (mean_vel && model == ORC_FHN) {
        for (int64_t j = 0; j < n; ++j) { th_prev[j] = atan2(y[n + j], y[j]); unwrap[j] = th_prev[j]; }
    }
    double* start = mean_vel ? (double*)malloc(sizeof(double) * n) : NULL;
    if (mean_vel && !start) {
        free(k1); free(k2); free(k3); free(k4); free(z); free(unwrap); free(th_prev);
        return ORC_ENOMEM;
    }
    for (int64_t step = 0; step < steps; ++step) {
        if (mean_vel && step == mv_start) {
            for (int64_t j = 0; j < n; ++j) start[j] = (model == ORC_FHN) ? unwrap[j] : y[j];
        }
        rhs(&m, y, k1);
        for (int64_t q = 0; q < len; ++q) z[q] = y[q] + (dt / 2.0) * k1[q];
        rhs(&m, z, k2);
        for (int64_t q = 0; q < len; ++q) z[q] = y[q] + (dt / 2.0) * k2[q];
        rhs(&m, z, k3);
        for (int64_t q = 0; q < len; ++q) z[q] = y[q] + dt * k3[q];
        rhs(&m, z, k4);
        for (int64_t q = 0; q < len; ++q)
            y[q] = y[q] + (dt / 6.0) * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
        if (mean_vel && model == ORC_FHN) {
            for (int64_t j = 0; j < n; ++j) {
                double th = atan2(y[n + j], y[j]);
                unwrap[j] += wrap_pi(th - th_prev[j]);
                th_prev[j] = th;
            }
        }
        if (R && (step + 1) % record_every == 0) R[(step + 1) / record_every] = order_parameter(model, n, y);
    }
    if (mean_vel) {
        const double span = (double)(steps - mv_start) * dt;
        for (int64_t j = 0; j < n; ++j) {
            double end = (model == ORC_FHN) ? unwrap[j] : y[j];
            mean_vel[j] = (end - start[j]) / span;
        }
    }
    free(k1); free(k2); free(k3); free(k4); free(z); free(unwrap); free(th_prev); free(start);
    return ORC_OK;
}

/* Order parameter of a state, exposed for the observable pins. */
double orc_order_parameter(int model, int64_t n, const double* y) { return order_parameter(model, n, y); }

/* ------------------------------------------------- Dormand-Prince 5(4) stepping
 * The embedded explicit Runge-Kutta pair of Dormand & Prince (1980), the
 * paper's default solver (Sec. III.A), with the usual step-size control
 * (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4):
 *   err = sqrt(mean_i ((y5_i - y4_i) / (atol + rtol * max(|y_i|, |y5_i|)))^2),
 *   accept when err <= 1; new h = h * min(facmax, max(0.2, 0.9 * err^(-1/5))),
 *   facmax = 10, and 1 right after a rejection; the step that reaches t_end
 *   (to within a relative 1e-12 of h) is shortened to end exactly on it.
 * The fifth-order solution propagates and the last stage is the first stage of
 * the next step (first same as last).  rtol <= 0 selects fixed steps of dt0
 * with no control (used by the order pin).
 * Failure (controlled runs only): an attempt whose proposed step h lies below
 * 10 units in the last place of t (the floor scipy's solvers use), or whose
 * error estimate is not finite (a NaN or Inf in the state or the slopes), ends
 * the run with ORC_ENUMERIC; y keeps the last accepted state and the failed
 * attempt is not counted.
 * stats[4] = {t reached, accepted steps, rejected steps, last proposed h}. */
static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
/* fifth minus fourth order weights */
static const double DP_E[7] = {71.0 / 57600, 0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200, 22.0 / 525, -1.0 / 40};
/* coefficients of the fourth-order continuous extension (dense output) */
static const double DP_D[7] = {-12715105075.0 / 11282082432.0, 0.0, 87487479700.0 / 32700410799.0,
                               -10690763975.0 / 1880347072.0, 701980252875.0 / 199316789632.0,
                               -1453857185.0 / 822651844.0, 69997945.0 / 29380423.0};

/* Dense output of an accepted step from (t, y) with stages k[0..6] and size h
 * (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.6, the continuous
 * extension of order 4 of the Dormand-Prince pair):
 *   y(t + theta h) = y + h sum_i b_i(theta) k_i,
 *   b_i(theta) = theta (b_i + (1 - theta) (e1_i - b_i + theta (2 b_i - e1_i - e7_i + (1 - theta) d_i)))
 * with b the fifth-order weights, e1 / e7 the first / last unit vectors and d
 * the coefficients above; b_i(0) = 0 and b_i(1) = b_i. */
void orc_dopri_dense_weights(double theta, double* wt) {
    for (int i = 0; i < 7; ++i) {
        const double b = i < 6 ? DP_A[6][i] : 0.0; /* the fifth-order weights are the last row of A */
        const double e1 = i == 0 ? 1.0 : 0.0, e7 = i == 6 ? 1.0 : 0.0;
        wt[i] = theta * (b + (1.0 - theta) * (e1 - b + theta * (2.0 * b - e1 - e7 + (1.0 - theta) * DP_D[i])));
    }
}

static int dopri_core(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
                      const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
                      const double* per_elem, double* y, double t_end, double rtol, double atol, double dt0,
                      int64_t max_steps, double* stats, double t_out, double* Rout, double* Yout);

int orc_run_dopri(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
                  const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
                  const double* per_elem, double* y, double t_end, double rtol, double atol, double dt0,
                  int64_t max_steps, double* stats) {
    return dopri_core(model, topo, n, radius, n1, n2, n3, row_ptr, col, w, prm, per_elem, y, t_end, rtol, atol,
                      dt0, max_steps, stats, 0.0, NULL, NULL);
}

/* As orc_run_dopri, and at the output times t_k = k t_out, k = 0 .. floor(t_end / t_out),
 * the order parameter Rout[k] and (Yout non-NULL) the state Yout[k * nvars * n ..] from
 * the dense output of the accepted step that contains t_k (t_0 = 0: the initial state).
 * The step that ends on t_end provides every output left, theta clamped to 1. */
int orc_run_dopri_dense(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
                        const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
                        const double* per_elem, double* y, double t_end, double rtol, double atol, double dt0,
                        int64_t max_steps, double* stats, double t_out, double* Rout, double* Yout) {
    if (!(t_out > 0.0) || !Rout) return ORC_EINVAL;
    return dopri_core(model, topo, n, radius, n1, n2, n3, row_ptr, col, w, prm, per_elem, y, t_end, rtol, atol,
                      dt0, max_steps, stats, t_out, Rout, Yout);
}

static int dopri_core(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
                      const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
                      const double* per_elem, double* y, double t_end, double rtol, double atol, double dt0,
                      int64_t max_steps, double* stats, double t_out, double* Rout, double* Yout) {
    orc_net m = make_net(model, topo, n, radius, n1, n2, n3, row_ptr, col, w, prm, per_elem, 0);
    int rc = validate(&m);
    if (rc) return rc;
    if (!(dt0 > 0.0) || !(t_end >= 0.0) || max_steps < 0) return ORC_EINVAL;
    const int64_t len = (int64_t)nvars(model) * n;
    double* k[7];
    double* z = (double*)malloc(sizeof(double) * len);
    int ok = z != NULL;
    for (int s = 0; s < 7; ++s) {
        k[s] = (double*)malloc(sizeof(double) * len);
        ok = ok && k[s];
    }
    if (!ok) {
        free(z);
        for (int s = 0; s < 7; ++s) free(k[s]);
        return ORC_ENOMEM;
    }
    (void)DP_C;
    double t = 0.0, h = dt0, facmax = 10.0;
    int64_t acc = 0, rej = 0;
    const int64_t K = t_out > 0.0 ? (int64_t)floor(t_end / t_out) : -1;
    int64_t next = 0;
    double* yt = t_out > 0.0 ? (double*)malloc(sizeof(double) * len) : NULL;
    if (t_out > 0.0 && !yt) {
        free(z);
        for (int s = 0; s < 7; ++s) free(k[s]);
        return ORC_ENOMEM;
    }
    if (K >= 0) {
        Rout[0] = order_parameter(model, n, y);
        if (Yout) memcpy(Yout, y, sizeof(double) * len);
        next = 1;
    }
    rhs(&m, y, k[0]);
    int failed = 0;
    while (t < t_end && acc + rej < max_steps) {
        if (rtol > 0.0 && h < 10.0 * (nextafter(t, INFINITY) - t)) {
            failed = 1;
            break;
        }
        /* the step that reaches t_end (within a relative 1e-12 of h) ends on it */
        const int last = t_end - t <= h * (1.0 + 1e-12);
        const double hs = last ? t_end - t : h;
        for (int s = 1; s < 7; ++s) {
            for (int64_t i = 0; i < len; ++i) {
                double a = 0.0;
                for (int q = 0; q < s; ++q) a += DP_A[s][q] * k[q][i];
                z[i] = y[i] + hs * a;
            }
            rhs(&m, z, k[s]);
        }
        /* z now holds the fifth-order solution (stage 7 uses the weights b) */
        int accept = 1;
        double f = 1.0;
        if (rtol > 0.0) {
            double sum = 0.0;
            for (int64_t i = 0; i < len; ++i) {
                double e = 0.0;
                for (int q = 0; q < 7; ++q) e += DP_E[q] * k[q][i];
                e *= hs;
                const double sc = atol + rtol * fmax(fabs(y[i]), fabs(z[i]));
                sum += (e / sc) * (e / sc);
            }
            const double err = sqrt(sum / (double)len);
            if (!isfinite(err)) {
                failed = 1;
                break;
            }
            f = 0.9 * pow(err, -0.2);
            accept = err <= 1.0;
        }
        if (accept) {
            /* outputs inside (t, t + hs]; the last step takes every one left */
            const double tn = last ? t_end : t + hs;
            for (; next <= K; ++next) {
                const double tk = (double)next * t_out;
                if (tk > tn && !last) break;
                double theta = (tk - t) / hs, wt[7];
                if (theta > 1.0) theta = 1.0;
                orc_dopri_dense_weights(theta, wt);
                for (int64_t i = 0; i < len; ++i) {
                    double a = 0.0;
                    for (int q = 0; q < 7; ++q) a += wt[q] * k[q][i];
                    yt[i] = y[i] + hs * a;
                }
                Rout[next] = order_parameter(model, n, yt);
                if (Yout) memcpy(Yout + next * len, yt, sizeof(double) * len);
            }
        }
        if (rtol <= 0.0) {
            memcpy(y, z, sizeof(double) * len);
            memcpy(k[0], k[6], sizeof(double) * len);
            t = last ? t_end : t + hs;
            ++acc;
            continue;
        }
        if (accept) {
            memcpy(y, z, sizeof(double) * len);
            memcpy(k[0], k[6], sizeof(double) * len);
            t = last ? t_end : t + hs;
            ++acc;
            h = hs * fmin(facmax, fmax(0.2, f));
            facmax = 10.0;
        } else {
            ++rej;
            h = hs * fmax(0.2, fmin(1.0, f));
            facmax = 1.0;
        }
    }
    stats[0] = t;
    stats[1] = (double)acc;
    stats[2] = (double)rej;
    stats[3] = h;
    free(z);
    free(yt);
    for (int s = 0; s < 7; ++s) free(k[s]);
    return failed ? ORC_ENUMERIC : ORC_OK;
}
