// Ring-window stage kernels (Kuramoto-Sakaguchi and FitzHugh-Nagumo on a ring of
// radius P) for gfx950.
//
// Each element i couples to the 2P elements i-P..i-1, i+1..i+P (periodic); the
// paper's 1D chimera study uses exactly this topology with mu = 1/2P (Sec. IV).
// Per RK4 stage the kernel needs, for every element, the window sum of the mapped
// stage values x_j = map(z_j) (Kuramoto: (cos z, sin z); FHN: (u, v)).  Instead of
// the paper's per-link loop (Alg. 1, O(P) work per element) a tile of T outputs
// [t0, t0+T) gets its sums from
//   W_incl(t0 + d) = W_incl(t0) + sum_{m < d} (x_{t0+P+1+m} - x_{t0-P+m}),
// i.e. one exclusive scan over the two window-end ranges, and W_incl(t0) from the
// per-tile sums written by the previous stage plus the partial tiles at both
// ends.  The window sum then excludes the element itself.  Everything summed is
// double; the sums are re-associations of the direct neighbour sum.
//
// RK4 access schedule per step (y double-buffered, k in the bulk type):
//   stage 1: z = y               -> write k1
//   stage 2: z = y + dt/2 k1     -> write k2, acc = y + dt/6 k1 + dt/3 k2
//   stage 3: z = y + dt/2 k2     -> write k3
//   stage 4: z = y + dt k3       -> y' = acc + dt/3 k3 + dt/6 k4
// and every stage also writes the per-tile sums of map(z) for the next stage.
#include "nd_dev.h"
#include "runtime.h"

namespace nd {

// ------------------------------------------------------------------ models
template <int MODEL, class KT>
struct RingModel;

// Kuramoto-Sakaguchi, Eq. (3) with m = 0, eps = 1:
//   k_i = omega + mu/(2P) sum_j sin(z_j - z_i - alpha)
//       = omega + mu/(2P) [cos(z_i + alpha) S_i - sin(z_i + alpha) C_i]
// with (C_i, S_i) the window sums of (cos z_j, sin z_j).
// p = {omega, mu/(2P), cos alpha, sin alpha}
template <class KT>
struct RingModel<ND_KURAMOTO, KT> {
    static constexpr int V = 1;
    __device__ static __forceinline__ double2 map(const double* z) {
        double s, c;
        if constexpr (sizeof(KT) == 8) {
            sincos(z[0], &s, &c);
        } else {
            // bulk float: reduce to revolutions in double, then the hardware
            // sin/cos (their argument is in revolutions)
            double r = z[0] * 0.15915494309189535;  // 1 / (2 pi)
            r -= rint(r);
            float rf = (float)r;
            s = (double)__builtin_amdgcn_sinf(rf);
            c = (double)__builtin_amdgcn_cosf(rf);
        }
        return make_double2(c, s);
    }
    __device__ static __forceinline__ void rhs(const NetDesc& d, const double* z, double2 xo, double2 W,
                                               double* k) {
        (void)z;
        if constexpr (sizeof(KT) == 8) {
            const double ca = xo.x * d.p[2] - xo.y * d.p[3];
            const double sa = xo.y * d.p[2] + xo.x * d.p[3];
            k[0] = d.p[0] + d.p[1] * (ca * W.y - sa * W.x);
        } else {
            const float cf = (float)xo.x, sf = (float)xo.y;
            const float ca = cf * (float)d.p[2] - sf * (float)d.p[3];
            const float sa = sf * (float)d.p[2] + cf * (float)d.p[3];
            k[0] = d.p[0] + d.p[1] * ((double)ca * W.y - (double)sa * W.x);
        }
    }
};

// FitzHugh-Nagumo, Eq. (2) (tau = 0, D = 0, I_app = 0) with the rotational
// coupling B(phi) on (u_j - u_i, v_j - v_i), kappa = sigma / 2P:
//   eps du = u - u^3/3 - v + kappa ( cos phi Du + sin phi Dv)
//       dv = u + a         + kappa (-sin phi Du + cos phi Dv)
// Du = sum_j u_j - 2P u_i, Dv likewise (double, before any rounding to float).
// p = {eps, a, kappa, cos phi, sin phi, 2P}
template <class KT>
struct RingModel<ND_FHN, KT> {
    static constexpr int V = 2;
    __device__ static __forceinline__ double2 map(const double* z) { return make_double2(z[0], z[1]); }
    __device__ static __forceinline__ void rhs(const NetDesc& d, const double* z, double2 xo, double2 W,
                                               double* k) {
        (void)xo;
        const double u = z[0], v = z[1];
        const double Du = W.x - d.p[5] * u;
        const double Dv = W.y - d.p[5] * v;
        if constexpr (sizeof(KT) == 8) {
            const double cu = d.p[2] * (d.p[3] * Du + d.p[4] * Dv);
            const double cv = d.p[2] * (d.p[3] * Dv - d.p[4] * Du);
            k[0] = (u - u * u * u / 3.0 - v + cu) / d.p[0];
            k[1] = u + d.p[1] + cv;
        } else {
            const float uf = (float)u, vf = (float)v, duf = (float)Du, dvf = (float)Dv;
            const float kap = (float)d.p[2], cph = (float)d.p[3], sph = (float)d.p[4];
            const float cu = kap * (cph * duf + sph * dvf);
            const float cv = kap * (cph * dvf - sph * duf);
            k[0] = (double)((uf - uf * uf * uf / 3.0f - vf + cu) / (float)d.p[0]);
            k[1] = (double)(uf + (float)d.p[1] + cv);
        }
    }
};

template <class KT>
__device__ __forceinline__ double kq(double k) {
    return (double)(KT)k;  // the value that is stored (and that every reader sees)
}

// Stage value z_v(idx) = y + c dt k_prev (stage 1: y).  Written once here so the
// producer of the tile sums and every reader of the window ends agree bitwise.
template <int V, class KT>
__device__ __forceinline__ void stage_z(const double* __restrict__ y, const KT* __restrict__ kp, double cdt,
                                        int64_t n, int64_t idx, double* z) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const double yy = y[v * n + idx];
        z[v] = kp ? fma(cdt, (double)kp[v * n + idx], yy) : yy;
    }
}

// ------------------------------------------------------------ prologue
// Tile sums of map(y) for the first stage of a run (networks with g0 == 0).
template <int MODEL, class KT, int BS, int EPT>
__global__ __launch_bounds__(BS) void k_ring_prologue(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                      const int* __restrict__ nwork_p) {
    using M = RingModel<MODEL, KT>;
    constexpr int V = M::V, T = BS * EPT, NW = BS / kWave;
    __shared__ double lds[4 * NW];
    const int nwork = *nwork_p;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (d.g0 != 0 || d.nsteps <= 0) continue;
        const int64_t n = d.n, t0 = (int64_t)wk.y * T;
        const int cnt = (int)min((int64_t)T, n - t0);
        const double* y = d.y[d.ypar];
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int m = threadIdx.x * EPT + e;
            if (m < cnt) {
                double z[V];
                stage_z<V, KT>(y, (const KT*)nullptr, 0.0, n, t0 + m, z);
                const double2 x = M::map(z);
                s[0] += x.x;
                s[1] += x.y;
                if constexpr (MODEL == ND_FHN) {
                    const double r = sqrt(z[0] * z[0] + z[1] * z[1]);
                    s[2] += z[0] / r;
                    s[3] += z[1] / r;
                }
            }
        }
        block_sum<BS, 4>(s, lds);
        if (threadIdx.x == 0) {
            d.tsum[0][2 * wk.y] = s[0];
            d.tsum[0][2 * wk.y + 1] = s[1];
            if constexpr (MODEL == ND_FHN) {
                d.rsum[2 * wk.y] = s[2];
                d.rsum[2 * wk.y + 1] = s[3];
            }
        }
    }
}

// ---------------------------------------------------------------- stage
template <int MODEL, class KT, int BS, int EPT>
__global__ __launch_bounds__(BS) void k_ring_stage(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                   const int* __restrict__ nwork_p, int stage, int j) {
    using M = RingModel<MODEL, KT>;
    constexpr int V = M::V, T = BS * EPT, NW = BS / kWave;
    __shared__ double lds[8 * NW];
    const int nwork = *nwork_p;
    const int tid = threadIdx.x;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;  // uniform over the block
        const int64_t n = d.n, P = d.P;
        const int G = d.G, tile = wk.y;
        const int64_t t0 = (int64_t)tile * T;
        const int cnt = (int)min((int64_t)T, n - t0);
        const int64_t g = d.g0 + j;
        const int par = (d.ypar + j) & 1;
        const double* __restrict__ y = d.y[par];
        const KT* __restrict__ kp = stage == 1 ? nullptr : (const KT*)d.k[stage - 2];
        const double dt = d.dt;
        const double cdt = stage == 4 ? dt : 0.5 * dt;
        const double* __restrict__ tin = d.tsum[(stage - 1) & 1];

        // ---- order parameter R(g) from the tile sums of map(y) (tile 0)
        if (stage == 1 && tile == 0 && (d.obs & OBS_R) && (g % d.r_every) == 0) {
            const double* src = (MODEL == ND_FHN) ? d.rsum : tin;
            double s[2] = {0.0, 0.0};
            for (int u = tid; u < G; u += BS) {
                s[0] += src[2 * u];
                s[1] += src[2 * u + 1];
            }
            block_sum<BS, 2>(s, lds);
            if (tid == 0) d.R[g / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }

        // ---- window ends: x over [A, A+T) and [B, B+T), A = t0-P, B = t0+P+1
        const int64_t A = t0 - P, B = t0 + P + 1;
        const int64_t a = A < 0 ? A + n : A;
        const int64_t b = B >= n ? B - n : B;
        const int ta = (int)(a / T), tb = (int)(b / T);
        const int hlen = (int)(min((int64_t)ta * T + T, n) - a);
        const int tlen = (int)(min((int64_t)tb * T + T, n) - b);
        const int ua = (A < 0 ? -G : 0) + ta;
        const int ub = (B >= n ? G : 0) + tb;
        // elements of each end range that are used: the partial tile (head /
        // tail remainder) and the first cnt - 1 scan terms; both stay inside
        // one period of the ring, so a single conditional wrap is exact
        const int lneed = max(hlen, cnt), rneed = max(tlen, cnt);

        double red[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // head(2), tail remainder(2), tiles(2)
        double dl[EPT][2];
        double dsum[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int m = tid * EPT + e;
            double2 xl = make_double2(0.0, 0.0), xr = make_double2(0.0, 0.0);
            if (m < lneed) {
                double z[V];
                stage_z<V, KT>(y, kp, cdt, n, ring_wrap(A + m, n), z);
                xl = M::map(z);
            }
            if (m < rneed) {
                double z[V];
                stage_z<V, KT>(y, kp, cdt, n, ring_wrap(B + m, n), z);
                xr = M::map(z);
            }
            if (m < hlen) {
                red[0] += xl.x;
                red[1] += xl.y;
            }
            if (m < tlen) {
                red[2] += xr.x;
                red[3] += xr.y;
            }
            dl[e][0] = xr.x - xl.x;
            dl[e][1] = xr.y - xl.y;
            dsum[0] += dl[e][0];
            dsum[1] += dl[e][1];
        }
        for (int u = ua + 1 + tid; u <= ub; u += BS) {
            const int uu = u < 0 ? u + G : (u >= G ? u - G : u);
            red[4] += tin[2 * uu];
            red[5] += tin[2 * uu + 1];
        }
        block_sum_and_exscan<BS, 6, 2>(red, dsum, lds);
        const double w0x = (red[0] + red[4]) - red[2];
        const double w0y = (red[1] + red[5]) - red[3];

        // ---- own elements: RHS and RK bookkeeping
        double nx[4] = {0.0, 0.0, 0.0, 0.0};  // next-stage tile sums (2) + FHN phase vectors (2)
        double run0 = dsum[0], run1 = dsum[1];  // exclusive prefix of d before this thread's first element
        const KT* __restrict__ k1 = (const KT*)d.k[0];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int m = tid * EPT + e;
            if (m < cnt) {
                const int64_t i = t0 + m;
                double z[V];
                stage_z<V, KT>(y, kp, cdt, n, i, z);
                const double2 xo = M::map(z);
                const double2 W = make_double2((w0x + run0) - xo.x, (w0y + run1) - xo.y);
                double k[V];
                M::rhs(d, z, xo, W, k);
                double zn[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int64_t q = v * n + i;
                    const double yy = y[q];
                    const double kk = kq<KT>(k[v]);
                    if (stage == 1) {
                        ((KT*)d.k[0])[q] = (KT)kk;
                        zn[v] = fma(0.5 * dt, kk, yy);
                    } else if (stage == 2) {
                        ((KT*)d.k[1])[q] = (KT)kk;
                        d.acc[q] = fma(dt / 3.0, kk, fma(dt / 6.0, (double)k1[q], yy));
                        zn[v] = fma(0.5 * dt, kk, yy);
                    } else if (stage == 3) {
                        ((KT*)d.k[2])[q] = (KT)kk;
                        zn[v] = fma(dt, kk, yy);
                    } else {
                        const double yo = fma(dt / 6.0, kk, fma(dt / 3.0, (double)kp[q], d.acc[q]));
                        d.y[par ^ 1][q] = yo;
                        zn[v] = yo;
                    }
                }
                const double2 xn = M::map(zn);
                nx[0] += xn.x;
                nx[1] += xn.y;
                if constexpr (MODEL == ND_FHN) {
                    if (stage == 4) {
                        const double r = sqrt(zn[0] * zn[0] + zn[1] * zn[1]);
                        nx[2] += zn[0] / r;
                        nx[3] += zn[1] / r;
                    }
                }
                // mean phase velocity
                if ((d.obs & OBS_MV) && g >= d.mv_start) {
                    if constexpr (MODEL == ND_KURAMOTO) {
                        if (stage == 1 && g == d.mv_start) d.mv[i] = y[i];
                    } else {
                        if (stage == 4) {
                            const double uo = y[i], vo = y[n + i];
                            const double un = zn[0], vn = zn[1];
                            const double dth = atan2(uo * vn - vo * un, uo * un + vo * vn);
                            d.mv[i] = (g == d.mv_start ? 0.0 : d.mv[i]) + dth;
                        }
                    }
                }
            }
            run0 += dl[e][0];
            run1 += dl[e][1];
        }
        block_sum<BS, 4>(nx, lds);
        if (tid == 0) {
            double* tout = d.tsum[stage & 1];
            tout[2 * tile] = nx[0];
            tout[2 * tile + 1] = nx[1];
            if constexpr (MODEL == ND_FHN) {
                if (stage == 4) {
                    d.rsum[2 * tile] = nx[2];
                    d.rsum[2 * tile + 1] = nx[3];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- epilogue
// After the last step of a run: R at the final step and the mean phase velocity.
// `chunk` is the number of steps of the chunk that just ran.
template <int MODEL, class KT, int BS, int EPT>
__global__ __launch_bounds__(BS) void k_ring_epilogue(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                      const int* __restrict__ nwork_p, int chunk) {
    constexpr int T = BS * EPT, NW = BS / kWave;
    __shared__ double lds[2 * NW];
    const int nwork = *nwork_p;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (d.nsteps <= 0 || d.nsteps > chunk) continue;
        const int64_t n = d.n, gend = d.g0 + d.nsteps;
        const int par = (d.ypar + (int)d.nsteps) & 1;
        if (wk.y == 0 && (d.obs & OBS_R) && (gend % d.r_every) == 0) {
            const double* src = (MODEL == ND_FHN) ? d.rsum : d.tsum[0];
            double s[2] = {0.0, 0.0};
            for (int u = threadIdx.x; u < d.G; u += BS) {
                s[0] += src[2 * u];
                s[1] += src[2 * u + 1];
            }
            block_sum<BS, 2>(s, lds);
            if (threadIdx.x == 0) d.R[gend / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }
        if (d.obs & OBS_MV) {
            const int64_t t0 = (int64_t)wk.y * T;
            const int cnt = (int)min((int64_t)T, n - t0);
            const double* y = d.y[par];
            for (int m = threadIdx.x; m < cnt; m += BS) {
                const int64_t i = t0 + m;
                if constexpr (MODEL == ND_KURAMOTO)
                    d.mv[i] = (y[i] - d.mv[i]) * d.mv_scale;
                else
                    d.mv[i] = d.mv[i] * d.mv_scale;
            }
        }
    }
}

// ------------------------------------------------------------------ launch


template <int MODEL, class KT, int BS, int EPT>
static RingLaunch ring_entry() {
    RingLaunch r;
    r.prologue = k_ring_prologue<MODEL, KT, BS, EPT>;
    r.stage = k_ring_stage<MODEL, KT, BS, EPT>;
    r.epilogue = k_ring_epilogue<MODEL, KT, BS, EPT>;
    r.bs = BS;
    r.tile = BS * EPT;
    return r;
}

template <int MODEL, class KT>
static bool ring_pick(int tile, RingLaunch* out) {
    switch (tile) {
        case 1024: *out = ring_entry<MODEL, KT, 256, 4>(); return true;
        case 2048: *out = ring_entry<MODEL, KT, 256, 8>(); return true;
        case 4096: *out = ring_entry<MODEL, KT, 512, 8>(); return true;
        case 512: *out = ring_entry<MODEL, KT, 128, 4>(); return true;
        default: return false;
    }
}

bool ring_select(int model, int prec, int tile, RingLaunch* out) {
    if (model == ND_KURAMOTO)
        return prec == ND_FP64 ? ring_pick<ND_KURAMOTO, double>(tile, out) : ring_pick<ND_KURAMOTO, float>(tile, out);
    if (model == ND_FHN)
        return prec == ND_FP64 ? ring_pick<ND_FHN, double>(tile, out) : ring_pick<ND_FHN, float>(tile, out);
    return false;
}

hipError_t ring_launch_prologue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork) {
    hipLaunchKernelGGL(L.prologue, dim3(grid), dim3(L.bs), 0, s, D, work, nwork);
    return hipGetLastError();
}
hipError_t ring_launch_stage(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                             const int* nwork, int stage, int j) {
    hipLaunchKernelGGL(L.stage, dim3(grid), dim3(L.bs), 0, s, D, work, nwork, stage, j);
    return hipGetLastError();
}
hipError_t ring_launch_epilogue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork, int chunk) {
    hipLaunchKernelGGL(L.epilogue, dim3(grid), dim3(L.bs), 0, s, D, work, nwork, chunk);
    return hipGetLastError();
}

}  // namespace nd
