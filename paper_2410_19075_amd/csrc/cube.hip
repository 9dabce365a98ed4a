// Kuramoto-Sakaguchi on a periodic n1 x n2 x n3 lattice, stage kernels for gfx950.
//
// Element (x, y, z) (index x + n1*y + n1*n2*z, the paper's 3D index map, Sec. IV)
// couples to every element of the cube [x-H, x+H] x [y-H, y+H] x [z-H, z+H]
// except itself; the sum of sin(z_j - z_i - alpha) is normalised by the
// (2H+1)^3 - 1 neighbours, as Alg. 1 divides by its link count.  The paper's
// own 3D runs use a ball neighbourhood; the cube is the separable case.
//
// Each work item owns a cx x cy column tile and a run of cz planes and streams
// through z (a 2.5D scheme):
//   * one thread per halo column (cx+2H) x (cy+2H) maps its stage values
//     (cos z, sin z) plane by plane and keeps the last 2H+1 of them in
//     registers; the z-direction sum is a running sum (new plane in, oldest
//     out) in double;
//   * the z-sums go to LDS; an x-pass (H <= 2: one thread per output column
//     and halo row, 2H+1 terms; longer windows: sliding along runs of 4
//     outputs) and a
//     y-pass (2H+1 terms) finish the cube sum for the cx x cy outputs;
//   * the RHS and the RK bookkeeping follow the 13-access schedule of the ring
//     kernels (y double-buffered, k in the bulk type).
// The coming planes' column values and RK operands are prefetched one to three
// planes ahead (as registers allow), and the plane loop synchronises through
// LDS-only barriers so those loads stay in flight.  In FP64 runs (the inertia
// model up to half-width 2) the three passes work on consecutive planes at once
// (the z-sums of plane i, the x-pass of plane i-1, the outputs of plane i-2)
// with one barrier per plane.  All sums are double and every sum has a fixed order.
#include <type_traits>

#include "models.h"
#include "runtime.h"

namespace nd {

__device__ __forceinline__ int wrapm(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Block sum for a runtime block size (<= 1024). lds: NV * 16 doubles.
template <int NV>
__device__ __forceinline__ void block_sum_rt(double (&v)[NV], double* lds) {
    const int nw = (blockDim.x + kWave - 1) / kWave;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[q * 16 + wid] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[q * 16 + w];
        v[q] = s;
    }
    __syncthreads();
}

template <int MODEL, class KT, int H, int STAGE, bool MV>
__global__ __launch_bounds__(1024) void k_cube_stage(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                    const int* __restrict__ nwork_p, int j) {
    using M = RingModel<MODEL, KT>;  // Kuramoto (phi) or Kuramoto with inertia (phi, psi)
    constexpr int V = M::V;
    constexpr int S = 2 * H + 1;
    constexpr int stage = STAGE;
    extern __shared__ double2 smem[];
    __shared__ double lds[2 * 16];
    const int nwork = *nwork_p;
    const int nvb = ((nwork + 7) >> 3) << 3;
    const int tid = threadIdx.x;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int w = xcd_work(vb, nwork);
        if (w < 0) continue;
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;  // uniform over the block
        const int n1 = d.n1, n2 = d.n2, n3 = d.n3;
        const int64_t n = d.n;
        // 32-bit element offsets (lattices below 2^29 elements) on uniform bases
        const uint32_t plane = (uint32_t)n1 * (uint32_t)n2;
        const int cx = d.cx, cy = d.cy, cz = d.cz, gx = d.gx, gy = d.gy;
        const int HX = cx + 2 * H, HY = cy + 2 * H;
        const int t = wk.y;
        const int tx = t % gx, ty = (t / gx) % gy, tz = t / (gx * gy);
        const int x0 = tx * cx, y0 = ty * cy, z0 = tz * cz;
        const int ex = min(cx, n1 - x0), ey = min(cy, n2 - y0);
        const int nz = min(cz, n3 - z0);
        const int64_t g = d.g0 + j;
        const int par = (d.ypar + j) & 1;
        const ND_GLOBAL double* __restrict__ y = gp(d.y[par]);
        const ND_GLOBAL KT* __restrict__ kp =
            stage == 1 ? nullptr : gp((const KT*)d.k[stage > 1 ? stage - 2 : 0]);
        const ND_GLOBAL double* __restrict__ acc = gp(d.acc);
        const double dt = d.dt;
        const double cdt = stage == 4 ? dt : 0.5 * dt;

        // ---- order parameter R(g) from the stage-1 partial sums (stage 2, item 0)
        if (stage == 2 && t == 0 && (d.obs & OBS_R) && (g % d.r_every) == 0) {
            double s[2] = {0.0, 0.0};
            const ND_GLOBAL double* ts = gp(d.tsum[0]);
            for (int u = tid; u < d.G; u += blockDim.x) {
                s[0] += ts[2 * u];
                s[1] += ts[2 * u + 1];
            }
            block_sum_rt<2>(s, lds);
            if (tid == 0) gp(d.R)[g / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }

        // The plane loop runs in one of two schedules that do the same arithmetic
        // per output.  Two-phase: the column threads' z-sums of plane i, a
        // barrier, the x-pass of plane i, a barrier, the y-pass and RHS of plane i
        // (two LDS buffers per array).  Pipelined (FP64: the one-variable model,
        // and the inertia model for half-widths up to 2, where registers allow):
        // in one phase the column threads do plane i, the x-pass plane i-1 and
        // the output threads plane i-2, then one barrier (three LDS buffers).
        // Each schedule is written out in full: sharing the passes as lambdas
        // changed the register allocation and cost FP32-bulk 10 %.
        constexpr bool kPipe = sizeof(KT) == 8 && (V == 1 || H <= 2);
        constexpr int NB = kPipe ? 3 : 2;    // LDS buffers per array (cube_lds_buffers)
        double2* S1 = smem;                  // [NB][HY][HX] z-sums per halo column
        double2* S0 = S1 + NB * HX * HY;     // [NB][cy][cx] mapped centre values
        double2* S2 = S0 + NB * cx * cy;     // [NB][HY][cx] x-pass sums

        // halo-column thread
        const bool col = tid < HX * HY;
        const int hx = col ? tid % HX : 0, hy = col ? tid / HX : 0;
        const bool inner = col && hx >= H && hx < H + cx && hy >= H && hy < H + cy;
        const uint32_t colbase = (uint32_t)wrapm(x0 - H + hx, n1) + (uint32_t)n1 * (uint32_t)wrapm(y0 - H + hy, n2);
        // output thread
        const bool outv = tid < cx * cy && (tid % cx) < ex && (tid / cx) < ey;
        const int ox = outv ? tid % cx : 0, oy = outv ? tid / cx : 0;
        const uint32_t obase = (uint32_t)(x0 + ox) + (uint32_t)n1 * (uint32_t)(y0 + oy);
        // x-pass thread. Short windows (H <= 2): one output column of one halo
        // row (HY * cx <= HX * HY threads), consecutive lanes on consecutive LDS
        // entries. Longer windows: a run of up to kRunX consecutive outputs of
        // one row, sliding the window along it (fewer LDS reads per output).
        constexpr bool kDirectX = H <= 2;
        constexpr int kRunX = 4;
        const int nsx = (cx + kRunX - 1) / kRunX;
        const bool xr = kDirectX ? tid < HY * cx : tid < HY * nsx;
        const int xrow = xr ? (kDirectX ? tid / cx : tid / nsx) : 0;
        const int xs0 = xr ? (kDirectX ? tid - xrow * cx : (tid - xrow * nsx) * kRunX) : 0;
        const int xcnt = kDirectX ? 1 : (xr ? min(kRunX, cx - xs0) : 0);

        auto zval = [&](uint32_t i) {
            const double yy = ld32(y, i);
            return stage == 1 ? yy : fma(cdt, (double)ld32(kp, i), yy);
        };
        // the last 2H+1 mapped planes of this column; in the bulk type, which is
        // exact (FP32-bulk maps are computed in float)
        using RB = typename std::conditional<sizeof(KT) == 8, double2, float2>::type;
        auto to_rb = [](double2 v) {
            RB r;
            r.x = v.x;
            r.y = v.y;
            return r;
        };
        RB rb[S];
        // running z-sum of the planes in the window that are already mapped
        double zsx = 0.0, zsy = 0.0;
#pragma unroll
        for (int u = 0; u < 2 * H; ++u) {
            double z[1] = {zval(colbase + plane * (uint32_t)wrapm(z0 - H + u, n3))};
            rb[u] = to_rb(M::map(z));
            zsx += (double)rb[u].x;
            zsy += (double)rb[u].y;
        }
        rb[2 * H] = to_rb(make_double2(0.0, 0.0));
        double part[2] = {0.0, 0.0};  // stage 1: sums of map(y) for R
        if constexpr (!kPipe) {
            // two-phase schedule; prefetched operands PF planes ahead (a shift
            // queue with static indices): the column value of the plane entering
            // the z window and the RK operands of the output plane, as far ahead as
            // 128 VGPRs allow: three planes in FP32-bulk for the one-variable model;
            // the inertia model (its psi operands besides) one in FP64, two in FP32-bulk
            constexpr int PF = V == 1 ? 3 : (sizeof(KT) == 8 ? 1 : 2);
            double qy[PF], qk[PF], qry[PF], qrk[PF], qra[PF];
            auto fetch = [&](int ahead, double& cy_, double& ck_, double& ry_, double& rk_, double& ra_) {
                // operands of output plane z0 + ahead (clamped inside this work item)
                const int zo_ = z0 + min(ahead, nz - 1);
                const uint32_t ci = colbase + plane * (uint32_t)wrapm(zo_ + H, n3);
                cy_ = ld32(y, ci);
                ck_ = stage != 1 ? (double)ld32(kp, ci) : 0.0;
                const uint32_t oi = obase + plane * (uint32_t)zo_;
                ry_ = ld32(y, oi);
                rk_ = (stage == 2 || stage == 4) ? (double)ld32(kp, oi) : 0.0;
                ra_ = stage == 4 ? ld32(acc, oi) : 0.0;
            };
#pragma unroll
            for (int f = 0; f < PF; ++f) fetch(f, qy[f], qk[f], qry[f], qrk[f], qra[f]);
            for (int zb = 0; zb < nz; zb += S) {
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    if (zb + u < nz) {
                        const int zo = z0 + zb + u;
                        const double zc = stage == 1 ? qy[0] : fma(cdt, qk[0], qy[0]);
                        const double cry = qry[0], crk = qrk[0], cra = qra[0];
#pragma unroll
                        for (int f = 0; f + 1 < PF; ++f) {
                            qy[f] = qy[f + 1];
                            qk[f] = qk[f + 1];
                            qry[f] = qry[f + 1];
                            qrk[f] = qrk[f + 1];
                            qra[f] = qra[f + 1];
                        }
                        fetch(zb + u + PF, qy[PF - 1], qk[PF - 1], qry[PF - 1], qrk[PF - 1], qra[PF - 1]);
                        // z window of output plane zo: planes zo-H .. zo+H; the new
                        // plane enters the running sum, the oldest leaves it after
                        {
                            double z[1] = {zc};
                            rb[(u + 2 * H) % S] = to_rb(M::map(z));
                        }
                        const double2 sz = make_double2(zsx + (double)rb[(u + 2 * H) % S].x,
                                                        zsy + (double)rb[(u + 2 * H) % S].y);
                        zsx = sz.x - (double)rb[u % S].x;
                        zsy = sz.y - (double)rb[u % S].y;
                        const int buf = (zb + u) & 1;
                        if (col) S1[buf * HX * HY + tid] = sz;
                        if (inner)
                            S0[buf * cx * cy + (hy - H) * cx + (hx - H)] =
                                make_double2((double)rb[(u + H) % S].x, (double)rb[(u + H) % S].y);
                        lds_barrier();
                        // x-pass over the HY rows
                        if (xr) {
                            const double2* src = S1 + buf * HX * HY + xrow * HX + xs0;
                            double2* dst = S2 + buf * HY * cx + xrow * cx + xs0;
                            double2 a = make_double2(0.0, 0.0);
#pragma unroll
                            for (int dx = 0; dx < S; ++dx) {
                                a.x += src[dx].x;
                                a.y += src[dx].y;
                            }
                            dst[0] = a;
                            if constexpr (!kDirectX) {
#pragma unroll
                                for (int r = 1; r < kRunX; ++r) {
                                    if (r < xcnt) {
                                        const double2 in = src[r + 2 * H], out = src[r - 1];
                                        a.x = (a.x + in.x) - out.x;
                                        a.y = (a.y + in.y) - out.y;
                                        dst[r] = a;
                                    }
                                }
                            }
                        }
                        lds_barrier();
                        // y-pass, RHS, RK bookkeeping
                        if (outv) {
                            const double2* src = S2 + buf * HY * cx + oy * cx + ox;
                            double2 bsum = make_double2(0.0, 0.0);
#pragma unroll
                            for (int dy = 0; dy < S; ++dy) {
                                bsum.x += src[dy * cx].x;
                                bsum.y += src[dy * cx].y;
                            }
                            const double2 xo = S0[buf * cx * cy + oy * cx + ox];
                            const double2 W = make_double2(bsum.x - xo.x, bsum.y - xo.y);
                            const uint32_t q = obase + plane * (uint32_t)zo;
                            // variable 1 (psi, inertia only): operands read here, not prefetched
                            double y1 = 0.0, kp1 = 0.0, a1 = 0.0;
                            double zz[V];
                            zz[0] = 0.0;  // the phase enters through xo
                            if constexpr (V == 2) {
                                y1 = ld32(y + n, q);
                                kp1 = stage != 1 ? (double)ld32(kp + n, q) : 0.0;
                                a1 = stage == 4 ? ld32(acc + n, q) : 0.0;
                                zz[V - 1] = stage == 1 ? y1 : fma(cdt, kp1, y1);
                            }
                            double k[V];
                            M::rhs(d, zz, xo, W, k);
                            const double kk = kq<KT>(k[0]);
                            if constexpr (V == 2) {
                                const double kk1 = kq<KT>(k[1]);
                                if (stage <= 3) st32(gp((KT*)d.k[stage - 1]) + n, q, (KT)kk1);
                                if (stage == 2) st32(gp(d.acc) + n, q, fma(d.dt3, kk1, fma(d.dt6, kp1, y1)));
                                if (stage == 4) {
                                    const double yo1 = fma(d.dt6, kk1, fma(d.dt3, kp1, a1));
                                    st32(gp(d.y[par ^ 1]) + n, q, yo1);
                                    flag_nonfinite(d, yo1);
                                }
                            }
                            if (stage == 1) {
                                st32(gp((KT*)d.k[0]), q, (KT)kk);
                                part[0] += xo.x;
                                part[1] += xo.y;
                                if (MV && (d.obs & OBS_MV) && g == d.mv_start) st32(gp(d.mv), q, cry);
                            } else if (stage == 2) {
                                st32(gp((KT*)d.k[1]), q, (KT)kk);
                                st32(gp(d.acc), q, fma(d.dt3, kk, fma(d.dt6, crk, cry)));
                            } else if (stage == 3) {
                                st32(gp((KT*)d.k[2]), q, (KT)kk);
                            } else {
                                const double yo = fma(d.dt6, kk, fma(d.dt3, crk, cra));
                                st32(gp(d.y[par ^ 1]), q, yo);
                                flag_nonfinite(d, yo);
                            }
                        }
                    }
                }
            }
        } else {
            // pipelined schedule: column values PF planes ahead of the column
            // pass, RK operands PF planes ahead of the output pass (two planes in
            // stages 1 and 3, one in 2 and 4, within 128 VGPRs)
            constexpr int PF = (STAGE == 1 || STAGE == 3) ? 2 : 1;
            double qy[PF], qk[PF], qry[PF], qrk[PF], qra[PF];
            auto fetch_col = [&](int ahead, double& cy_, double& ck_) {
                const int zo_ = z0 + min(ahead, nz - 1);
                const uint32_t ci = colbase + plane * (uint32_t)wrapm(zo_ + H, n3);
                cy_ = ld32(y, ci);
                ck_ = stage != 1 ? (double)ld32(kp, ci) : 0.0;
            };
            auto fetch_rk = [&](int ahead, double& ry_, double& rk_, double& ra_) {
                const int zo_ = z0 + min(ahead, nz - 1);
                const uint32_t oi = obase + plane * (uint32_t)zo_;
                ry_ = ld32(y, oi);
                rk_ = (stage == 2 || stage == 4) ? (double)ld32(kp, oi) : 0.0;
                ra_ = stage == 4 ? ld32(acc, oi) : 0.0;
            };
#pragma unroll
            for (int f = 0; f < PF; ++f) fetch_col(f, qy[f], qk[f]);
#pragma unroll
            for (int f = 0; f < PF; ++f) fetch_rk(f, qry[f], qrk[f], qra[f]);
            const int nit = nz + 2;
            for (int zb = 0; zb < nit; zb += S) {
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    const int i = zb + u;
                    if (i >= nit) continue;  // uniform
                    if (i < nz) {  // column pass, plane i
                        const double zc = stage == 1 ? qy[0] : fma(cdt, qk[0], qy[0]);
#pragma unroll
                        for (int f = 0; f + 1 < PF; ++f) {
                            qy[f] = qy[f + 1];
                            qk[f] = qk[f + 1];
                        }
                        fetch_col(i + PF, qy[PF - 1], qk[PF - 1]);
                        {
                            double z[1] = {zc};
                            rb[(u + 2 * H) % S] = to_rb(M::map(z));
                        }
                        const double2 sz = make_double2(zsx + (double)rb[(u + 2 * H) % S].x,
                                                        zsy + (double)rb[(u + 2 * H) % S].y);
                        zsx = sz.x - (double)rb[u % S].x;
                        zsy = sz.y - (double)rb[u % S].y;
                        const int buf = i % NB;
                        if (col) S1[buf * HX * HY + tid] = sz;
                        if (inner)
                            S0[buf * cx * cy + (hy - H) * cx + (hx - H)] =
                                make_double2((double)rb[(u + H) % S].x, (double)rb[(u + H) % S].y);
                    }
                    if (i >= 1 && i - 1 < nz) {  // x-pass over the HY rows, plane i - 1
                        const int buf = (i - 1) % NB;
                        if (xr) {
                            const double2* src = S1 + buf * HX * HY + xrow * HX + xs0;
                            double2* dst = S2 + buf * HY * cx + xrow * cx + xs0;
                            double2 a = make_double2(0.0, 0.0);
#pragma unroll
                            for (int dx = 0; dx < S; ++dx) {
                                a.x += src[dx].x;
                                a.y += src[dx].y;
                            }
                            dst[0] = a;
                            if constexpr (!kDirectX) {
#pragma unroll
                                for (int r = 1; r < kRunX; ++r) {
                                    if (r < xcnt) {
                                        const double2 in = src[r + 2 * H], out = src[r - 1];
                                        a.x = (a.x + in.x) - out.x;
                                        a.y = (a.y + in.y) - out.y;
                                        dst[r] = a;
                                    }
                                }
                            }
                        }
                    }
                    if (i >= 2) {                                    // output plane i - 2
                        const int io = i - 2;
                        const double cry = qry[0], crk = qrk[0], cra = qra[0];
#pragma unroll
                        for (int f = 0; f + 1 < PF; ++f) {
                            qry[f] = qry[f + 1];
                            qrk[f] = qrk[f + 1];
                            qra[f] = qra[f + 1];
                        }
                        fetch_rk(io + PF, qry[PF - 1], qrk[PF - 1], qra[PF - 1]);
                        const int zo = z0 + io, buf = io % NB;
                        if (outv) {
                            const double2* src = S2 + buf * HY * cx + oy * cx + ox;
                            double2 bsum = make_double2(0.0, 0.0);
#pragma unroll
                            for (int dy = 0; dy < S; ++dy) {
                                bsum.x += src[dy * cx].x;
                                bsum.y += src[dy * cx].y;
                            }
                            const double2 xo = S0[buf * cx * cy + oy * cx + ox];
                            const double2 W = make_double2(bsum.x - xo.x, bsum.y - xo.y);
                            const uint32_t q = obase + plane * (uint32_t)zo;
                            // variable 1 (psi, inertia only): operands read here, not prefetched
                            double y1 = 0.0, kp1 = 0.0, a1 = 0.0;
                            double zz[V];
                            zz[0] = 0.0;  // the phase enters through xo
                            if constexpr (V == 2) {
                                y1 = ld32(y + n, q);
                                kp1 = stage != 1 ? (double)ld32(kp + n, q) : 0.0;
                                a1 = stage == 4 ? ld32(acc + n, q) : 0.0;
                                zz[V - 1] = stage == 1 ? y1 : fma(cdt, kp1, y1);
                            }
                            double k[V];
                            M::rhs(d, zz, xo, W, k);
                            const double kk = kq<KT>(k[0]);
                            if constexpr (V == 2) {
                                const double kk1 = kq<KT>(k[1]);
                                if (stage <= 3) st32(gp((KT*)d.k[stage - 1]) + n, q, (KT)kk1);
                                if (stage == 2) st32(gp(d.acc) + n, q, fma(d.dt3, kk1, fma(d.dt6, kp1, y1)));
                                if (stage == 4) {
                                    const double yo1 = fma(d.dt6, kk1, fma(d.dt3, kp1, a1));
                                    st32(gp(d.y[par ^ 1]) + n, q, yo1);
                                    flag_nonfinite(d, yo1);
                                }
                            }
                            if (stage == 1) {
                                st32(gp((KT*)d.k[0]), q, (KT)kk);
                                part[0] += xo.x;
                                part[1] += xo.y;
                                if (MV && (d.obs & OBS_MV) && g == d.mv_start) st32(gp(d.mv), q, cry);
                            } else if (stage == 2) {
                                st32(gp((KT*)d.k[1]), q, (KT)kk);
                                st32(gp(d.acc), q, fma(d.dt3, kk, fma(d.dt6, crk, cry)));
                            } else if (stage == 3) {
                                st32(gp((KT*)d.k[2]), q, (KT)kk);
                            } else {
                                const double yo = fma(d.dt6, kk, fma(d.dt3, crk, cra));
                                st32(gp(d.y[par ^ 1]), q, yo);
                                flag_nonfinite(d, yo);
                            }
                        }
                    }
                    lds_barrier();
                }
            }
        }
        if (stage == 1) {
            block_sum_rt<2>(part, lds);
            if (tid == 0) {
                gp(d.tsum[0])[2 * t] = part[0];
                gp(d.tsum[0])[2 * t + 1] = part[1];
            }
        } else {
            __syncthreads();  // LDS reuse by the next work item
        }
    }
}

// ------------------------------------------------------------------ ball
// Ball neighbourhood of the paper's 3D studies: every lattice point within
// Euclidean distance P, the element itself included (L = that count); the
// disk of the 2D studies is the same kernel with a z half-width of 0 on an
// n1 x n2 x 1 lattice.  The
// ball is the union over (dy, dz) with dy^2 + dz^2 <= P^2 of x-runs of
// half-width r = floor(sqrt(P^2 - dy^2 - dz^2)), so with per-row prefix sums
// along x every run is one difference of two prefix values.
// Each work item owns a cx x cy output tile and a run of cz planes and streams
// through z.  Per plane, wave w of W maps halo rows w, w+W, ... (one lane per x of
// the HX = cx + 2P <= 64 halo columns), scans each row with DPP and stores
// the row's inclusive prefix in a ring of 2P+2 prefix planes in LDS.  After
// one LDS-only barrier every output sums its 2 * (#(dy, dz) pairs) prefix
// differences over the 2P+1 planes of its window, re-maps its own stage
// value for the RHS and does the RK bookkeeping.  The ring holds one spare
// plane, so the next plane's rows are written while this plane's sums read.
constexpr int kBallRowsPerWave = 4;
constexpr int kBallUnroll = 8;
constexpr int kBallMaxRuns = 224;  // (dy, dz) runs of the largest ball (P = 8: 197), padded to kBallUnroll

template <int MODEL, class KT, int BS, int STAGE, bool MV>
__global__ __launch_bounds__(BS) void k_ball_stage(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                    const int* __restrict__ nwork_p, int j) {
    using M = RingModel<MODEL, KT>;
    constexpr int V = M::V;
    constexpr int stage = STAGE;
    constexpr int kBallWaves = BS / kWave;
    extern __shared__ double2 smem[];
    __shared__ double lds[2 * 16];
    // the (dy, dz) runs of the ball: {dz, dy, r + 1, -r}, padded with empty runs
    // ({0, 0, 0, 0}: hi - lo = 0 exactly) to a multiple of kBallUnroll
    __shared__ int4 runs[kBallMaxRuns];
    __shared__ int nruns;
    const int nwork = *nwork_p;
    const int nvb = ((nwork + 7) >> 3) << 3;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int w = xcd_work(vb, nwork);
        if (w < 0) continue;
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;  // uniform over the block
        const int n1 = d.n1, n2 = d.n2, n3 = d.n3, P = (int)d.P;
        const int64_t n = d.n;
        const uint32_t plane = (uint32_t)n1 * (uint32_t)n2;
        const int cx = d.cx, cy = d.cy, cz = d.cz, gx = d.gx, gy = d.gy;
        const int PZ = d.pz;  // z half-width: P (ball) or 0 (disk)
        const int HX = cx + 2 * P, HY = cy + 2 * P, NS = 2 * PZ + 2, RW = HX + 1;
        const int t = wk.y;
        const int tx = t % gx, ty = (t / gx) % gy, tz = t / (gx * gy);
        const int x0 = tx * cx, y0 = ty * cy, z0 = tz * cz;
        const int ex = min(cx, n1 - x0), ey = min(cy, n2 - y0);
        const int nz = min(cz, n3 - z0);
        const int64_t g = d.g0 + j;
        const int par = (d.ypar + j) & 1;
        const ND_GLOBAL double* __restrict__ y = gp(d.y[par]);
        const ND_GLOBAL KT* __restrict__ kp =
            stage == 1 ? nullptr : gp((const KT*)d.k[stage > 1 ? stage - 2 : 0]);
        const ND_GLOBAL double* __restrict__ acc = gp(d.acc);
        const double dt = d.dt;
        const double cdt = stage == 4 ? dt : 0.5 * dt;

        if (stage == 2 && t == 0 && (d.obs & OBS_R) && (g % d.r_every) == 0) {
            double s[2] = {0.0, 0.0};
            const ND_GLOBAL double* ts = gp(d.tsum[0]);
            for (int u = tid; u < d.G; u += blockDim.x) {
                s[0] += ts[2 * u];
                s[1] += ts[2 * u + 1];
            }
            block_sum_rt<2>(s, lds);
            if (tid == 0) gp(d.R)[g / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }
        if (tid == 0) {
            int c = 0;
            for (int dz = -PZ; dz <= PZ; ++dz)
                for (int dy = -P; dy <= P; ++dy) {
                    const int q = P * P - dz * dz - dy * dy;
                    if (q < 0) continue;
                    int r = 0;
                    while ((r + 1) * (r + 1) <= q) ++r;
                    runs[c++] = make_int4(dz, dy, r + 1, -r);
                }
            while (c % kBallUnroll) runs[c++] = make_int4(0, 0, 0, 0);
            nruns = c;
        }

        // mapper rows of this wave (lane = halo x); columns beyond the halo or
        // rows beyond HY load a valid element and contribute nothing
        const bool lx = lane < HX;
        const uint32_t xcol = (uint32_t)wrapm(x0 - P + (lx ? lane : 0), n1);
        uint32_t rowbase[kBallRowsPerWave];
        bool rv[kBallRowsPerWave];
#pragma unroll
        for (int k = 0; k < kBallRowsPerWave; ++k) {
            const int r = wave + k * kBallWaves;
            rv[k] = r < HY;
            rowbase[k] = xcol + (uint32_t)n1 * (uint32_t)wrapm(y0 - P + (rv[k] ? r : 0), n2);
        }
        auto zval = [&](uint32_t i) {
            const double yy = ld32(y, i);
            return stage == 1 ? yy : fma(cdt, (double)ld32(kp, i), yy);
        };
        // map plane q (relative: absolute z = z0 - P + q) into ring slot q % NS
        double qz[kBallRowsPerWave];
        auto load_plane = [&](int q) {
            const uint32_t zb = plane * (uint32_t)wrapm(z0 - PZ + min(q, nz + 2 * PZ - 1), n3);
#pragma unroll
            for (int k = 0; k < kBallRowsPerWave; ++k)
                if (rv[k]) qz[k] = zval(rowbase[k] + zb);
        };
        auto store_plane = [&](int q) {
            double2* pre = smem + (size_t)(q % NS) * HY * RW;
#pragma unroll
            for (int k = 0; k < kBallRowsPerWave; ++k) {
                if (!rv[k]) continue;  // uniform over the wave
                double z[1] = {qz[k]};
                double2 m = M::map(z);
                if (!lx) m = make_double2(0.0, 0.0);
                const double px = wave_incl_scan(m.x), py = wave_incl_scan(m.y);
                double2* row = pre + (size_t)(wave + k * kBallWaves) * RW;
                if (lx) row[lane + 1] = make_double2(px, py);
                if (lane == 0) row[0] = make_double2(0.0, 0.0);
            }
        };
        for (int q = 0; q < 2 * PZ; ++q) {
            load_plane(q);
            store_plane(q);
        }
        load_plane(2 * PZ);

        // output thread
        const bool outv = tid < cx * cy && (tid % cx) < ex && (tid / cx) < ey;
        const int ox = outv ? tid % cx : 0, oy = outv ? tid / cx : 0;
        const uint32_t obase = (uint32_t)(x0 + ox) + (uint32_t)n1 * (uint32_t)(y0 + oy);
        double part[2] = {0.0, 0.0};
        // own RK operands, one plane ahead
        double ny[V], nk[V], na[V];
        auto own = [&](int i) {
            const uint32_t q = obase + plane * (uint32_t)(z0 + min(i, nz - 1));
#pragma unroll
            for (int v = 0; v < V; ++v) {
                ny[v] = nk[v] = na[v] = 0.0;
                if (outv) {
                    ny[v] = ld32(y + (int64_t)v * n, q);
                    nk[v] = stage != 1 ? (double)ld32(kp + (int64_t)v * n, q) : 0.0;
                    na[v] = stage == 4 ? ld32(acc + (int64_t)v * n, q) : 0.0;
                }
            }
        };
        own(0);
        for (int i = 0; i < nz; ++i) {
            const int zo = z0 + i;
            const uint32_t q = obase + plane * (uint32_t)zo;
            double yv[V], kv[V], av[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                yv[v] = ny[v];
                kv[v] = nk[v];
                av[v] = na[v];
            }
            own(i + 1);
            store_plane(i + 2 * PZ);   // the plane entering the window of output plane zo
            load_plane(i + 2 * PZ + 1);
            lds_barrier();
            if (outv) {
                // runs in (dz, dy) order, kBallUnroll at a time so their LDS
                // reads are in flight together; the sum order is fixed
                double2 W = make_double2(0.0, 0.0);
                const int s0 = (i + PZ) % NS;  // slot of the centre plane
                const double2* centre = smem + (size_t)(oy + P) * RW + ox + P;
                const int nr = nruns;
                for (int k0 = 0; k0 < nr; k0 += kBallUnroll) {
                    double2 hi[kBallUnroll], lo[kBallUnroll];
#pragma unroll
                    for (int u = 0; u < kBallUnroll; ++u) {
                        const int4 e = runs[k0 + u];
                        int sl = s0 + e.x;
                        sl += sl < 0 ? NS : 0;
                        sl -= sl >= NS ? NS : 0;
                        const double2* row = centre + (size_t)sl * HY * RW + e.y * RW;
                        hi[u] = row[e.z];
                        lo[u] = row[e.w];
                    }
#pragma unroll
                    for (int u = 0; u < kBallUnroll; ++u) {
                        W.x += hi[u].x - lo[u].x;
                        W.y += hi[u].y - lo[u].y;
                    }
                }
                double zz[V];
#pragma unroll
                for (int v = 0; v < V; ++v) zz[v] = stage == 1 ? yv[v] : fma(cdt, kv[v], yv[v]);
                const double2 xo = M::map(zz);
                double k[V];
                M::rhs(d, zz, xo, W, k);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const double kk = kq<KT>(k[v]);
                    if (stage <= 3) st32(gp((KT*)d.k[stage - 1]) + (int64_t)v * n, q, (KT)kk);
                    if (stage == 2) st32(gp(d.acc) + (int64_t)v * n, q, fma(d.dt3, kk, fma(d.dt6, kv[v], yv[v])));
                    if (stage == 4) {
                        const double yo = fma(d.dt6, kk, fma(d.dt3, kv[v], av[v]));
                        st32(gp(d.y[par ^ 1]) + (int64_t)v * n, q, yo);
                        flag_nonfinite(d, yo);
                    }
                }
                if (stage == 1) {
                    part[0] += xo.x;
                    part[1] += xo.y;
                    if (MV && (d.obs & OBS_MV) && g == d.mv_start) st32(gp(d.mv), q, yv[0]);
                }
            }
        }
        if (stage == 1) {
            block_sum_rt<2>(part, lds);
            if (tid == 0) {
                gp(d.tsum[0])[2 * t] = part[0];
                gp(d.tsum[0])[2 * t + 1] = part[1];
            }
        } else {
            __syncthreads();  // LDS reuse by the next work item
        }
    }
}

// After the last step of a run: partial sums of map(y) over flat element ranges
// (one per work item) and the mean phase velocity.
template <class KT>
__global__ __launch_bounds__(256) void k_cube_final_partials(const NetDesc* __restrict__ D,
                                                             const int2* __restrict__ work,
                                                             const int* __restrict__ nwork_p, int chunk) {
    using M = RingModel<ND_KURAMOTO, KT>;
    __shared__ double lds[2 * 16];
    const int nwork = *nwork_p;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (d.nsteps <= 0 || d.nsteps > chunk) continue;
        const int64_t n = d.n;
        const int64_t per = (n + d.G - 1) / d.G;
        const int64_t b = (int64_t)wk.y * per, e = min(n, b + per);
        const double* y = d.y[(d.ypar + (int)d.nsteps) & 1];
        double s[2] = {0.0, 0.0};
        for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
            double z[1] = {y[i]};
            const double2 x = M::map(z);
            s[0] += x.x;
            s[1] += x.y;
            if (d.obs & OBS_MV) d.mv[i] = (y[i] - d.mv[i]) * d.mv_scale;
        }
        block_sum_rt<2>(s, lds);
        if (threadIdx.x == 0) {
            d.tsum[1][2 * wk.y] = s[0];
            d.tsum[1][2 * wk.y + 1] = s[1];
        }
    }
}

__global__ __launch_bounds__(256) void k_cube_final_R(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                      const int* __restrict__ nwork_p, int chunk) {
    __shared__ double lds[2 * 16];
    const int nwork = *nwork_p;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (wk.y != 0 || d.nsteps <= 0 || d.nsteps > chunk || !(d.obs & OBS_R)) continue;
        const int64_t gend = d.g0 + d.nsteps;
        if (gend % d.r_every) continue;
        double s[2] = {0.0, 0.0};
        for (int u = threadIdx.x; u < d.G; u += blockDim.x) {
            s[0] += d.tsum[1][2 * u];
            s[1] += d.tsum[1][2 * u + 1];
        }
        block_sum_rt<2>(s, lds);
        if (threadIdx.x == 0) d.R[gend / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)d.n;
    }
}

// ------------------------------------------------------------------ launch
template <int MODEL, class KT, int H>
static void cube_entry(CubeLaunch* r) {
    r->stage[0] = k_cube_stage<MODEL, KT, H, 1, false>;
    r->stage[1] = k_cube_stage<MODEL, KT, H, 2, false>;
    r->stage[2] = k_cube_stage<MODEL, KT, H, 3, false>;
    r->stage[3] = k_cube_stage<MODEL, KT, H, 4, false>;
    r->stage_mv[0] = k_cube_stage<MODEL, KT, H, 1, true>;
    r->stage_mv[1] = k_cube_stage<MODEL, KT, H, 2, true>;
    r->stage_mv[2] = k_cube_stage<MODEL, KT, H, 3, true>;
    r->stage_mv[3] = k_cube_stage<MODEL, KT, H, 4, true>;
    r->final_partials = k_cube_final_partials<KT>;
    r->final_R = k_cube_final_R;
}

template <int MODEL>
static bool cube_pick(int prec, int h, CubeLaunch* out) {
    if (prec == ND_FP64) {
        switch (h) {
            case 1: cube_entry<MODEL, double, 1>(out); break;
            case 2: cube_entry<MODEL, double, 2>(out); break;
            case 3: cube_entry<MODEL, double, 3>(out); break;
            default: cube_entry<MODEL, double, 4>(out); break;
        }
    } else {
        switch (h) {
            case 1: cube_entry<MODEL, float, 1>(out); break;
            case 2: cube_entry<MODEL, float, 2>(out); break;
            case 3: cube_entry<MODEL, float, 3>(out); break;
            default: cube_entry<MODEL, float, 4>(out); break;
        }
    }
    return true;
}

template <int MODEL, class KT, int BS>
static void ball_entry(CubeLaunch* r) {
    r->stage[0] = k_ball_stage<MODEL, KT, BS, 1, false>;
    r->stage[1] = k_ball_stage<MODEL, KT, BS, 2, false>;
    r->stage[2] = k_ball_stage<MODEL, KT, BS, 3, false>;
    r->stage[3] = k_ball_stage<MODEL, KT, BS, 4, false>;
    r->stage_mv[0] = k_ball_stage<MODEL, KT, BS, 1, true>;
    r->stage_mv[1] = k_ball_stage<MODEL, KT, BS, 2, true>;
    r->stage_mv[2] = k_ball_stage<MODEL, KT, BS, 3, true>;
    r->stage_mv[3] = k_ball_stage<MODEL, KT, BS, 4, true>;
    r->final_partials = k_cube_final_partials<KT>;
    r->final_R = k_cube_final_R;
}

template <int MODEL, class KT>
static bool ball_pick(int block, CubeLaunch* out) {
    if (block == 256) ball_entry<MODEL, KT, 256>(out);
    else if (block == 1024) ball_entry<MODEL, KT, 1024>(out);
    else return false;
    return true;
}

bool ball_select(int model, int prec, int block, CubeLaunch* out) {
    if (model == ND_KURAMOTO)
        return prec == ND_FP64 ? ball_pick<ND_KURAMOTO, double>(block, out) : ball_pick<ND_KURAMOTO, float>(block, out);
    if (model == ND_KURAMOTO_INERTIA)
        return prec == ND_FP64 ? ball_pick<ND_KURAMOTO_INERTIA, double>(block, out)
                               : ball_pick<ND_KURAMOTO_INERTIA, float>(block, out);
    return false;
}

size_t ball_smem_bytes(int P, int pz, int cx, int cy) {
    return (size_t)(2 * pz + 2) * (cy + 2 * P) * (cx + 2 * P + 1) * sizeof(double2);
}

bool cube_select(int model, int prec, int h, CubeLaunch* out) {
    if (h < 1 || h > 4) return false;
    if (model == ND_KURAMOTO) return cube_pick<ND_KURAMOTO>(prec, h, out);
    if (model == ND_KURAMOTO_INERTIA) return cube_pick<ND_KURAMOTO_INERTIA>(prec, h, out);
    return false;
}

int cube_lds_buffers(int model, int prec, int h) {
    return prec == ND_FP64 && (model == ND_KURAMOTO || h <= 2) ? 3 : 2;
}

size_t cube_smem_bytes(int h, int cx, int cy, int nb) {
    const size_t HX = cx + 2 * h, HY = cy + 2 * h;
    return (nb * HX * HY + nb * (size_t)cx * cy + nb * HY * cx) * sizeof(double2);
}

int cube_block(int h, int cx, int cy) {
    const int cols = (cx + 2 * h) * (cy + 2 * h);
    return ((cols + kWave - 1) / kWave) * kWave;
}

hipError_t cube_launch_stage(const CubeLaunch& L, int grid, int block, size_t smem, hipStream_t s, NetDesc* D,
                             const int2* work, const int* nwork, int stage, int j, bool mv) {
    auto f = mv ? L.stage_mv[stage - 1] : L.stage[stage - 1];
    if (smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(f, dim3(grid), dim3(block), smem, s, D, work, nwork, j);
    return hipGetLastError();
}

hipError_t cube_launch_final(const CubeLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                             const int* nwork, int chunk) {
    hipLaunchKernelGGL(L.final_partials, dim3(grid), dim3(256), 0, s, D, work, nwork, chunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(L.final_R, dim3(grid), dim3(256), 0, s, D, work, nwork, chunk);
    return hipGetLastError();
}

}  // namespace nd
