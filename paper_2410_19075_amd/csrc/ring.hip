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
#include "models.h"
#include "runtime.h"

namespace nd {

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
        const ND_GLOBAL double* y = gp(d.y[d.ypar]);
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            // same element order and grouping as the stage kernel's next-stage
            // sums, so a restarted run reproduces a continuous one bitwise
            const int m = e * BS + threadIdx.x;
            if (m < cnt) {
                double z[V];
                stage_z<V, KT>(y, (const ND_GLOBAL KT*)nullptr, 0.0, n, t0 + m, z);
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
            gp(d.tsum[0])[2 * wk.y] = s[0];
            gp(d.tsum[0])[2 * wk.y + 1] = s[1];
            if constexpr (MODEL == ND_FHN) {
                gp(d.rsum)[2 * wk.y] = s[2];
                gp(d.rsum)[2 * wk.y + 1] = s[3];
            }
        }
    }
}

// ---------------------------------------------------------------- stage
template <int MODEL, class KT, int BS, int EPT, int STAGE, bool MV>
__global__ __launch_bounds__(BS) void k_ring_stage(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                   const int* __restrict__ nwork_p, int j) {
    constexpr int stage = STAGE;
    using M = RingModel<MODEL, KT>;
    constexpr int V = M::V, T = BS * EPT, NW = BS / kWave;
    __shared__ double2 sd[T];  // x_right - x_left, then the inclusive window sums
    // own y and k_prev, kept for the RK update, only where the stage uses them
    constexpr bool kNeedY = STAGE != 4 || MV, kNeedK = STAGE == 2 || STAGE == 4;
    __shared__ double sy[kNeedY ? V * T : 1], sk[kNeedK ? V * T : 1];
    __shared__ double lds[8 * NW];
    const int nwork = *nwork_p;
    const int tid = threadIdx.x;
    // virtual block ids keep blockIdx.x % 8 (grid is a multiple of 8 or == nwork)
    const int nvb = ((nwork + 7) >> 3) << 3;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int w = xcd_work(vb, nwork);
        if (w < 0) continue;
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;  // uniform over the block
        // element indices and the per-variable offsets below are 32-bit (rings
        // hold fewer than 2^29 elements, so every byte offset fits 32 bits):
        // loads and stores then take a uniform 64-bit base plus a lane offset
        const int n = (int)d.n, P = (int)d.P;
        const int G = d.G, tile = wk.y;
        const int t0 = tile * T;
        const int cnt = min(T, n - t0);
        const int64_t g = d.g0 + j;
        const int par = (d.ypar + j) & 1;
        const ND_GLOBAL double* yb[V];
        const ND_GLOBAL KT* kb[V];
        const ND_GLOBAL double* ab[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            yb[v] = gp(d.y[par]) + (int64_t)v * n;
            kb[v] = stage == 1 ? nullptr : gp((const KT*)d.k[stage > 1 ? stage - 2 : 0]) + (int64_t)v * n;
            ab[v] = gp(d.acc) + (int64_t)v * n;
        }
        const double dt = d.dt;
        const double cdt = stage == 4 ? dt : 0.5 * dt;
        const ND_GLOBAL double* __restrict__ tin = gp(d.tsum[(stage - 1) & 1]);

        // ---- order parameter R(g) from the tile sums of map(y) (tile 0)
        if (stage == 1 && tile == 0 && (d.obs & OBS_R) && (g % d.r_every) == 0) {
            const ND_GLOBAL double* src = (MODEL == ND_FHN) ? gp((const double*)d.rsum) : tin;
            double s[2] = {0.0, 0.0};
            for (int u = tid; u < G; u += BS) {
                s[0] += src[2 * u];
                s[1] += src[2 * u + 1];
            }
            block_sum<BS, 2>(s, lds);
            if (tid == 0) gp(d.R)[g / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }

        // ---- geometry of the window ends [A, A+T) and [B, B+T)
        const int A = t0 - P, B = t0 + P + 1;
        const int a = A < 0 ? A + n : A;
        const int b = B >= n ? B - n : B;
        const int ta = a / T, tb = b / T;
        const int hlen = min(ta * T + T, n) - a;
        const int tlen = min(tb * T + T, n) - b;
        const int ua = (A < 0 ? -G : 0) + ta;
        const int ub = (B >= n ? G : 0) + tb;
        // elements of each end range that are used: the partial tile (head /
        // tail remainder) and the first cnt - 1 scan terms; both stay inside
        // one period of the ring, so a single conditional wrap is exact
        const int lneed = max(hlen, cnt), rneed = max(tlen, cnt);

        // ---- phase 1 (coalesced, element m = e*BS + tid): own stage values,
        // window-end differences into LDS, head / tail-remainder partial sums
        // per lane: head partial + whole tiles - tail remainder (both components)
        double red[2] = {0.0, 0.0};
        double zo[EPT][V];
        double2 xo[EPT];
        auto stage_val = [&](uint32_t i, double* z) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double yy = ld32(yb[v], i);
                z[v] = stage == 1 ? yy : fma(cdt, (double)ld32(kb[v], i), yy);
            }
        };
        {
            // all loads first, from always-valid (clamped) indices, so they are
            // issued back to back; masks are applied to the values afterwards
            double zl[EPT][V], zr[EPT][V];
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int m = e * BS + tid;
                const int il = m < lneed ? ring_wrap32(A + m, n) : t0;
                const int ir = m < rneed ? ring_wrap32(B + m, n) : t0;
                const int io = m < cnt ? t0 + m : t0;
                stage_val(il, zl[e]);
                stage_val(ir, zr[e]);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const double yy = ld32(yb[v], io);
                    const double kk = stage == 1 ? 0.0 : (double)ld32(kb[v], io);
                    zo[e][v] = stage == 1 ? yy : fma(cdt, kk, yy);
                    if constexpr (kNeedY) sy[v * T + m] = yy;
                    if constexpr (kNeedK) sk[v * T + m] = kk;
                }
            }
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int m = e * BS + tid;
                double2 xl = M::map(zl[e]), xr = M::map(zr[e]);
                xo[e] = M::map(zo[e]);
                if (m >= lneed) xl = make_double2(0.0, 0.0);
                if (m >= rneed) xr = make_double2(0.0, 0.0);
                if (m < hlen) {
                    red[0] += xl.x;
                    red[1] += xl.y;
                }
                if (m < tlen) {
                    red[0] -= xr.x;
                    red[1] -= xr.y;
                }
                sd[m] = make_double2(xr.x - xl.x, xr.y - xl.y);
            }
        }
        // whole tiles inside the window (several per lane for long windows;
        // unrolled so their loads are in flight together, order unchanged)
#pragma unroll 4
        for (int u = ua + 1 + tid; u <= ub; u += BS) {
            const int uu = u < 0 ? u + G : (u >= G ? u - G : u);
            typedef double d2v __attribute__((ext_vector_type(2)));
            const d2v ts = *(const ND_GLOBAL d2v*)(tin + 2 * uu);
            red[0] += ts.x;
            red[1] += ts.y;
        }
        lds_barrier();

        // stage 4 needs the accumulator: issue its loads before the scan
        double av[EPT][V];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int m = e * BS + tid;
            const int i = t0 + (m < cnt ? m : 0);
#pragma unroll
            for (int v = 0; v < V; ++v) av[e][v] = stage == 4 ? ld32(ab[v], i) : 0.0;
        }
        // ---- phase 2 (blocked, elements EPT*tid ..): exclusive scan of the
        // differences; LDS then holds the inclusive window sum of every element
        double2 dv[EPT];
        double tot[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            dv[e] = sd[tid * EPT + e];
            tot[0] += dv[e].x;
            tot[1] += dv[e].y;
        }
        block_sum_and_exscan<BS, 2, 2>(red, tot, lds);
        {
            const double w0x = red[0], w0y = red[1];
            double r0 = tot[0], r1 = tot[1];
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                sd[tid * EPT + e] = make_double2(w0x + r0, w0y + r1);
                r0 += dv[e].x;
                r1 += dv[e].y;
            }
        }
        lds_barrier();

        // ---- phase 3 (coalesced): RHS, RK bookkeeping, next-stage tile sums
        // (loads from clamped indices issue together; only stores are masked)
        double nx[4] = {0.0, 0.0, 0.0, 0.0};
        double yv[EPT][V], kv[EPT][V];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int m = e * BS + tid;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                yv[e][v] = kNeedY ? sy[v * T + m] : 0.0;
                kv[e][v] = kNeedK ? sk[v * T + m] : 0.0;
            }
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int m = e * BS + tid;
            if (m < cnt) {
                const int i = t0 + m;
                const double2 wi = sd[m];
                const double2 W = make_double2(wi.x - xo[e].x, wi.y - xo[e].y);
                double k[V];
                M::rhs(d, zo[e], xo[e], W, k);
                double zn[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const double yy = yv[e][v];
                    const double kk = kq<KT>(k[v]);
                    if (stage <= 3) {
                        st32(gp((KT*)d.k[stage - 1]) + (int64_t)v * n, i, (KT)kk);
                        zn[v] = fma(stage == 3 ? dt : 0.5 * dt, kk, yy);
                        if (stage == 2) st32((ND_GLOBAL double*)ab[v], i, fma(d.dt3, kk, fma(d.dt6, kv[e][v], yy)));
                    } else {
                        const double yo = fma(d.dt6, kk, fma(d.dt3, kv[e][v], av[e][v]));
                        st32(gp(d.y[par ^ 1]) + (int64_t)v * n, i, yo);
                        flag_nonfinite(d, yo);
                        zn[v] = yo;
                    }
                }
                const double2 xn = M::map(zn);
                nx[0] += xn.x;
                nx[1] += xn.y;
                if constexpr (MODEL == ND_FHN) {
                    if (stage == 4 && (d.obs & OBS_R)) {
                        const double r = sqrt(zn[0] * zn[0] + zn[1] * zn[1]);
                        nx[2] += zn[0] / r;
                        nx[3] += zn[1] / r;
                    }
                }
                // mean phase velocity (compiled only into the MV variants)
                if (MV && (d.obs & OBS_MV) && g >= d.mv_start) {
                    if constexpr (MODEL != ND_FHN) {  // phase models: unwrapped phase is variable 0
                        if (stage == 1 && g == d.mv_start) gp(d.mv)[i] = yv[e][0];
                    } else {
                        if (stage == 4) {
                            const double uo = yv[e][0], vo = yv[e][1];
                            const double un = zn[0], vn = zn[1];
                            const double dth = atan2(uo * vn - vo * un, uo * un + vo * vn);
                            gp(d.mv)[i] = (g == d.mv_start ? 0.0 : gp(d.mv)[i]) + dth;
                        }
                    }
                }
            }
        }
        // FHN's stage 4 also sums the unit vectors for R; otherwise two sums
        block_sum<BS, (MODEL == ND_FHN && STAGE == 4) ? 4 : 2>(
            *reinterpret_cast<double(*)[(MODEL == ND_FHN && STAGE == 4) ? 4 : 2]>(nx), lds);
        if (tid == 0) {
            ND_GLOBAL double* tout = gp(d.tsum[stage & 1]);
            tout[2 * tile] = nx[0];
            tout[2 * tile + 1] = nx[1];
            if constexpr (MODEL == ND_FHN) {
                if (stage == 4) {
                    gp(d.rsum)[2 * tile] = nx[2];
                    gp(d.rsum)[2 * tile + 1] = nx[3];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- resident
// Rings small enough for one workgroup (n <= BS*EPT): the state stays in
// registers for a whole chunk of steps.  Per stage the mapped values are
// prefix-summed in LDS (double) and every window sum is a difference of two
// prefix values (wrapping through the ring total); no global memory traffic
// between stages.  Each thread owns EPT consecutive elements.  The prefix
// array holds element k at k + k / EPT, so the lanes' stride-EPT accesses land
// on distinct LDS banks (stride EPT + 1 doubles, at any offset).
template <int MODEL, class KT, int BS, int EPT, bool MV>
__global__ __launch_bounds__(BS) void k_ring_resident(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                      const int* __restrict__ nwork_p, int chunk) {
    using M = RingModel<MODEL, KT>;
    constexpr int V = M::V, T = BS * EPT, NW = BS / kWave, TP = T + BS;
    auto px = [](int k) { return k + k / EPT; };  // padded position of element k
    extern __shared__ double pf[];  // [2][TP]: inclusive prefix sums of the two map components (padded)
    __shared__ double lds[8 * NW];
    const int nwork = *nwork_p;
    const int tid = threadIdx.x;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (d.nsteps <= 0) continue;
        const int steps = (int)min((int64_t)chunk, d.nsteps);
        const int n = (int)d.n, P = (int)d.P;
        const double dt = d.dt;
        const ND_GLOBAL double* yin = gp(d.y[d.ypar]);
        double y[EPT][V], acc[EPT][V], kp[EPT][V], dth[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid * EPT + e;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                y[e][v] = i < n ? yin[(int64_t)v * n + i] : 0.0;
                acc[e][v] = 0.0;
                kp[e][v] = 0.0;
            }
            dth[e] = 0.0;
        }
        for (int j = 0; j < steps; ++j) {
            const int64_t g = d.g0 + j;
#pragma unroll
            for (int s = 1; s <= 4; ++s) {
                const double cdt = s == 4 ? dt : 0.5 * dt;
                double z[EPT][V];
                double2 x[EPT];
                double tot[2] = {0.0, 0.0};
                double ru[2] = {0.0, 0.0};  // FHN: unit phase vectors for R
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const int i = tid * EPT + e;
#pragma unroll
                    for (int v = 0; v < V; ++v) z[e][v] = s == 1 ? y[e][v] : fma(cdt, kp[e][v], y[e][v]);
                    x[e] = M::map(z[e]);
                    if (i >= n) x[e] = make_double2(0.0, 0.0);
                    tot[0] += x[e].x;
                    tot[1] += x[e].y;
                    // thread-local inclusive prefix, completed below with the
                    // block-exclusive offset of this thread
                    pf[px(tid * EPT + e)] = tot[0];
                    pf[TP + px(tid * EPT + e)] = tot[1];
                    if constexpr (MODEL == ND_FHN) {
                        if (s == 1 && i < n) {
                            const double r = sqrt(z[e][0] * z[e][0] + z[e][1] * z[e][1]);
                            ru[0] += z[e][0] / r;
                            ru[1] += z[e][1] / r;
                        }
                    }
                }
                if constexpr (MODEL == ND_FHN)
                    block_sum_and_exscan<BS, 2, 2>(ru, tot, lds);
                else
                    block_exscan<BS, 2>(tot, lds);  // R comes from the prefix totals
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    pf[px(tid * EPT + e)] = tot[0] + pf[px(tid * EPT + e)];
                    pf[TP + px(tid * EPT + e)] = tot[1] + pf[TP + px(tid * EPT + e)];
                }
                lds_barrier();
                const double t0 = pf[px(n - 1)], t1 = pf[TP + px(n - 1)];
                if (s == 1 && tid == 0 && (d.obs & OBS_R) && (g % d.r_every) == 0) {
                    const double c = MODEL == ND_FHN ? ru[0] : t0, sn = MODEL == ND_FHN ? ru[1] : t1;
                    gp(d.R)[g / d.r_every] = sqrt(c * c + sn * sn) / (double)n;
                }
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const int i = tid * EPT + e;
                    if (i < n) {
                        // prefix(k) = sum_{j<k} x_j; window [i-P, i+P] through the ring total
                        const int lo = i - P, hi = i + P + 1;
                        auto pre = [&](int k, int c) { return k == 0 ? 0.0 : pf[c * TP + px(k - 1)]; };
                        double w0, w1;
                        if (lo < 0) {
                            w0 = pre(hi, 0) + (t0 - pre(lo + n, 0));
                            w1 = pre(hi, 1) + (t1 - pre(lo + n, 1));
                        } else if (hi > n) {
                            w0 = (t0 - pre(lo, 0)) + pre(hi - n, 0);
                            w1 = (t1 - pre(lo, 1)) + pre(hi - n, 1);
                        } else {
                            w0 = pre(hi, 0) - pre(lo, 0);
                            w1 = pre(hi, 1) - pre(lo, 1);
                        }
                        const double2 W = make_double2(w0 - x[e].x, w1 - x[e].y);
                        double k[V];
                        M::rhs(d, z[e], x[e], W, k);
                        if (MV && (d.obs & OBS_MV) && g == d.mv_start && s == 1 && MODEL != ND_FHN)
                            gp(d.mv)[i] = y[e][0];
                        double yo[V];
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            const double kk = kq<KT>(k[v]);
                            if (s == 2) acc[e][v] = fma(d.dt3, kk, fma(d.dt6, kp[e][v], y[e][v]));
                            yo[v] = s == 4 ? fma(d.dt6, kk, fma(d.dt3, kp[e][v], acc[e][v])) : y[e][v];
                            kp[e][v] = kk;
                        }
                        if constexpr (MODEL == ND_FHN) {
                            if (MV && s == 4 && (d.obs & OBS_MV) && g >= d.mv_start) {
                                const double uo = y[e][0], vo = y[e][1], un = yo[0], vn = yo[1];
                                dth[e] += atan2(uo * vn - vo * un, uo * un + vo * vn);
                            }
                        }
#pragma unroll
                        for (int v = 0; v < V; ++v) y[e][v] = yo[v];
                    }
                }
                lds_barrier();
            }
        }
        if constexpr (MODEL == ND_FHN) {
            // unwrapped-phase increments of this chunk's steps at or after mv_start
            if (MV && (d.obs & OBS_MV) && d.mv_start < d.g0 + steps) {
                const bool first = d.mv_start >= d.g0;
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const int i = tid * EPT + e;
                    if (i < n) gp(d.mv)[i] = (first ? 0.0 : gp(d.mv)[i]) + dth[e];
                }
            }
        }
        // write the state back into the buffer the chunk ends on, plus the map
        // sums the epilogue turns into the final R
        ND_GLOBAL double* yout = gp(d.y[(d.ypar + steps) & 1]);
        double sums[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid * EPT + e;
            if (i < n) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    yout[(int64_t)v * n + i] = y[e][v];
                    flag_nonfinite(d, y[e][v]);
                }
                const double2 xm = M::map(y[e]);
                sums[0] += xm.x;
                sums[1] += xm.y;
                if constexpr (MODEL == ND_FHN) {
                    const double r = sqrt(y[e][0] * y[e][0] + y[e][1] * y[e][1]);
                    sums[2] += y[e][0] / r;
                    sums[3] += y[e][1] / r;
                }
            }
        }
        block_sum<BS, 4>(sums, lds);
        if (tid == 0) {
            gp(d.tsum[0])[0] = sums[0];
            gp(d.tsum[0])[1] = sums[1];
            gp(d.rsum)[0] = sums[2];
            gp(d.rsum)[1] = sums[3];
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
            // a ring held by one work item (resident kernel) is finalised whole
            const int cnt = d.G == 1 ? (int)n : (int)min((int64_t)T, n - t0);
            const double* y = d.y[par];
            for (int m = threadIdx.x; m < cnt; m += BS) {
                const int64_t i = t0 + m;
                if constexpr (MODEL != ND_FHN)
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
    r.stage[0] = k_ring_stage<MODEL, KT, BS, EPT, 1, false>;
    r.stage[1] = k_ring_stage<MODEL, KT, BS, EPT, 2, false>;
    r.stage[2] = k_ring_stage<MODEL, KT, BS, EPT, 3, false>;
    r.stage[3] = k_ring_stage<MODEL, KT, BS, EPT, 4, false>;
    r.stage_mv[0] = k_ring_stage<MODEL, KT, BS, EPT, 1, true>;
    r.stage_mv[1] = k_ring_stage<MODEL, KT, BS, EPT, 2, true>;
    r.stage_mv[2] = k_ring_stage<MODEL, KT, BS, EPT, 3, true>;
    r.stage_mv[3] = k_ring_stage<MODEL, KT, BS, EPT, 4, true>;
    r.epilogue = k_ring_epilogue<MODEL, KT, BS, EPT>;
    r.bs = BS;
    r.tile = BS * EPT;
    r.resident = nullptr;
    r.resident_mv = nullptr;
    r.smem = 0;
    return r;
}

template <int MODEL, class KT, int BS, int EPT>
static RingLaunch resident_entry() {
    // every kernel of this entry is launched with BS threads, so each one is
    // instantiated for BS (launch bounds and LDS sizing follow the block size)
    RingLaunch r;
    r.prologue = k_ring_prologue<MODEL, KT, BS, EPT>;
    for (auto& f : r.stage) f = nullptr;
    for (auto& f : r.stage_mv) f = nullptr;
    r.epilogue = k_ring_epilogue<MODEL, KT, BS, EPT>;
    r.resident = k_ring_resident<MODEL, KT, BS, EPT, false>;
    r.resident_mv = k_ring_resident<MODEL, KT, BS, EPT, true>;
    r.bs = BS;
    r.tile = -BS * EPT;
    r.smem = 2 * (BS * EPT + BS) * sizeof(double);  // padded prefix arrays
    return r;
}

template <int MODEL, class KT>
static bool ring_pick(int tile, RingLaunch* out) {
    switch (tile) {
        case -1024: *out = resident_entry<MODEL, KT, 256, 4>(); return true;
        case -2048: *out = resident_entry<MODEL, KT, 256, 8>(); return true;
        case -4096: *out = resident_entry<MODEL, KT, 512, 8>(); return true;
        case 2048: *out = ring_entry<MODEL, KT, 256, 8>(); return true;
        case 1024: *out = ring_entry<MODEL, KT, 256, 4>(); return true;
        case 512: *out = ring_entry<MODEL, KT, 256, 2>(); return true;
        case 256: *out = ring_entry<MODEL, KT, 128, 2>(); return true;
        case 128: *out = ring_entry<MODEL, KT, 64, 2>(); return true;
        default: return false;
    }
}

bool ring_select(int model, int prec, int tile, RingLaunch* out) {
    if (model == ND_KURAMOTO)
        return prec == ND_FP64 ? ring_pick<ND_KURAMOTO, double>(tile, out) : ring_pick<ND_KURAMOTO, float>(tile, out);
    if (model == ND_FHN)
        return prec == ND_FP64 ? ring_pick<ND_FHN, double>(tile, out) : ring_pick<ND_FHN, float>(tile, out);
    if (model == ND_KURAMOTO_INERTIA)
        return prec == ND_FP64 ? ring_pick<ND_KURAMOTO_INERTIA, double>(tile, out)
                               : ring_pick<ND_KURAMOTO_INERTIA, float>(tile, out);
    return false;
}

hipError_t ring_launch_prologue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork) {
    hipLaunchKernelGGL(L.prologue, dim3(grid), dim3(L.bs), 0, s, D, work, nwork);
    return hipGetLastError();
}
hipError_t ring_launch_stage(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                             const int* nwork, int stage, int j, bool mv) {
    hipLaunchKernelGGL(mv ? L.stage_mv[stage - 1] : L.stage[stage - 1], dim3(grid), dim3(L.bs), 0, s, D, work,
                       nwork, j);
    return hipGetLastError();
}
hipError_t ring_launch_resident(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork, int chunk, bool mv) {
    auto f = mv ? L.resident_mv : L.resident;
    if (L.smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.smem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(f, dim3(grid), dim3(L.bs), L.smem, s, D, work, nwork, chunk);
    return hipGetLastError();
}

hipError_t ring_launch_epilogue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork, int chunk) {
    hipLaunchKernelGGL(L.epilogue, dim3(grid), dim3(L.bs), 0, s, D, work, nwork, chunk);
    return hipGetLastError();
}

}  // namespace nd
