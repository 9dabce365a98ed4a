// Ball neighbourhood of the paper's 3D studies (every lattice point within
// Euclidean distance P, the element itself included; Sec. IV and V), in a
// plane-scatter form for a compile-time radius.
//
// The ball is the union over (dy, dz), dy^2 + dz^2 <= P^2, of x-runs of
// half-width r = floor(sqrt(P^2 - dy^2 - dz^2)); with per-row prefix sums
// along x every run is the difference of two prefix values.  The gather form
// (k_ball_stage) keeps the 2P+1 planes of an output plane's window in LDS, so
// at P = 6 a CU holds ~200 outputs and a few waves carry all the prefix reads.
// Here each work item streams through z and keeps only the plane just mapped
// (double-buffered) in LDS:
//   * waves map halo rows of the incoming plane (one lane per x of the
//     HX = cx + 2P <= 64 halo columns, up to 4 rows per wave), scan each row
//     with DPP and store the inclusive prefix;
//   * after one LDS-only barrier every output thread adds the plane's runs to
//     the 2P+1 output planes the plane reaches, held as running sums in
//     registers: plane q reaches output plane q - dz through the runs of dz,
//     and the runs of dz and -dz are the same (dy, r) set, so one pair of
//     prefix reads serves both;
//   * the output plane whose window is complete gets the RHS and the RK
//     bookkeeping of the 13-access schedule; its own operands were prefetched
//     one output plane ahead.
// Each output's sum visits the runs in (dz, dy) order, the order of the gather
// form, so both forms give bitwise identical stage values when their x tilings
// agree (the row prefix sums then start at the same halo column).  With the radius
// fixed at compile time every run's LDS offset is a constant relative to the
// thread's row base, so the sums carry no per-run address arithmetic.
#include <utility>

#include "models.h"
#include "runtime.h"

namespace nd {

constexpr int kScatterWaves = kBallScatterBlock / kWave;
constexpr int kScatterRows = 4;  // halo rows per wave (HY <= 32)

constexpr int isqrt_floor(int q) {
    int r = 0;
    while ((r + 1) * (r + 1) <= q) ++r;
    return r;
}

__device__ __forceinline__ int wrap_index(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// One run (|dz| = A, dy) of the plane: the x-run of half-width r around the
// output column, added to the output planes reached through dz = +A (s1) and,
// for A > 0, dz = -A (s2).  row0 points at the output's centre in the plane's
// prefix array; RW is the prefix row stride.
template <int P, int A, int DY>
__device__ __forceinline__ void scatter_run(const double2* row0, int RW, double2& s1, double2& s2) {
    constexpr int r = isqrt_floor(P * P - A * A - DY * DY);
    const double2* row = row0 + DY * RW;
    const double2 hi = row[r + 1], lo = row[-r];
    const double ex = hi.x - lo.x, ey = hi.y - lo.y;
    s1.x += ex;
    s1.y += ey;
    if constexpr (A > 0) {
        s2.x += ex;
        s2.y += ey;
    }
}

template <int P, int A, int... I>
__device__ __forceinline__ void scatter_dz(const double2* row0, int RW, double2& s1, double2& s2,
                                           std::integer_sequence<int, I...>) {
    constexpr int rz = isqrt_floor(P * P - A * A);
    (scatter_run<P, A, I - rz>(row0, RW, s1, s2), ...);
}

// Runs of |dz| = A, when at least one of the two output planes they reach is
// one of this work item's outputs (acc[k] holds output plane q - 2P + k; an
// output plane outside [0, nz) collects values nobody reads).
template <int P, int A>
__device__ __forceinline__ void scatter_group(const double2* row0, int RW, int q, int nz, double2 (&acc)[2 * P + 1]) {
    const int o1 = q - P - A, o2 = q - P + A;  // dz = +A, dz = -A
    const bool need = (o1 >= 0 && o1 < nz) || (A > 0 && o2 >= 0 && o2 < nz);
    if (!need) return;  // uniform over the block
    constexpr int rz = isqrt_floor(P * P - A * A);
    scatter_dz<P, A>(row0, RW, acc[P - A], acc[P + A], std::make_integer_sequence<int, 2 * rz + 1>{});
}

template <int P, int... A>
__device__ __forceinline__ void scatter_plane(const double2* row0, int RW, int q, int nz, double2 (&acc)[2 * P + 1],
                                              std::integer_sequence<int, A...>) {
    (scatter_group<P, A>(row0, RW, q, nz, acc), ...);
}

// Radii up to kBallScatterPairedMaxP are built for two workgroups per CU (at most
// 128 VGPRs: the 2P+1 running sums of the FP64 inertia model then spill a few
// words at P = 6, which still measured faster than one workgroup per CU);
// larger radii keep one workgroup per CU.
template <int MODEL, class KT, int P, int STAGE, bool MV>
__global__ __launch_bounds__(kBallScatterBlock) __attribute__((amdgpu_waves_per_eu(P <= kBallScatterPairedMaxP ? 4 : 2)))
void k_ball_scatter(const NetDesc* __restrict__ D, const int2* __restrict__ work, const int* __restrict__ nwork_p,
                    int j) {
    using M = RingModel<MODEL, KT>;
    constexpr int V = M::V;
    constexpr int stage = STAGE;
    constexpr int S = 2 * P + 1;
    extern __shared__ double2 smem[];  // [2][HY][RW] row prefix planes
    __shared__ double lds[2 * kScatterWaves];
    const int nwork = *nwork_p;
    const int nvb = ((nwork + 7) >> 3) << 3;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int w = xcd_work(vb, nwork);
        if (w < 0) continue;
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;  // uniform over the block
        const int n1 = d.n1, n2 = d.n2, n3 = d.n3;
        const int64_t n = d.n;
        const uint32_t plane = (uint32_t)n1 * (uint32_t)n2;
        const int cx = d.cx, cy = d.cy, cz = d.cz, gx = d.gx, gy = d.gy;
        const int HX = cx + 2 * P, HY = cy + 2 * P, RW = HX + 1;
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
            for (int u = tid; u < d.G; u += kBallScatterBlock) {
                s[0] += ts[2 * u];
                s[1] += ts[2 * u + 1];
            }
            block_sum<kBallScatterBlock, 2>(s, lds);
            if (tid == 0) gp(d.R)[g / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }

        // mapper rows of this wave (lane = halo x); columns beyond the halo or
        // rows beyond HY load a valid element and contribute nothing
        const bool lx = lane < HX;
        const uint32_t xcol = (uint32_t)wrap_index(x0 - P + (lx ? lane : 0), n1);
        uint32_t rowbase[kScatterRows];
        bool rv[kScatterRows];
#pragma unroll
        for (int k = 0; k < kScatterRows; ++k) {
            const int r = wave + k * kScatterWaves;
            rv[k] = r < HY;
            rowbase[k] = xcol + (uint32_t)n1 * (uint32_t)wrap_index(y0 - P + (rv[k] ? r : 0), n2);
        }
        const int nq = nz + 2 * P;  // planes z0 - P .. z0 + nz - 1 + P
        auto zval = [&](uint32_t i) {
            const double yy = ld32(y, i);
            return stage == 1 ? yy : fma(cdt, (double)ld32(kp, i), yy);
        };
        double qz[kScatterRows];
        auto load_plane = [&](int q) {
            const uint32_t zb = plane * (uint32_t)wrap_index(z0 - P + min(q, nq - 1), n3);
#pragma unroll
            for (int k = 0; k < kScatterRows; ++k)
                if (rv[k]) qz[k] = zval(rowbase[k] + zb);
        };
        auto store_plane = [&](int q) {
            double2* pre = smem + (size_t)(q & 1) * HY * RW;
#pragma unroll
            for (int k = 0; k < kScatterRows; ++k) {
                if (!rv[k]) continue;  // uniform over the wave
                double z[1] = {qz[k]};
                double2 m = M::map(z);
                if (!lx) m = make_double2(0.0, 0.0);
                const double px = wave_incl_scan(m.x), py = wave_incl_scan(m.y);
                double2* row = pre + (size_t)(wave + k * kScatterWaves) * RW;
                if (lx) row[lane + 1] = make_double2(px, py);
                if (lane == 0) row[0] = make_double2(0.0, 0.0);
            }
        };

        // output thread
        const bool outv = tid < cx * cy && (tid % cx) < ex && (tid / cx) < ey;
        const int ox = outv ? tid % cx : 0, oy = outv ? tid / cx : 0;
        const uint32_t obase = (uint32_t)(x0 + ox) + (uint32_t)n1 * (uint32_t)(y0 + oy);
        double part[2] = {0.0, 0.0};
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
        // acc_[k]: running sum of output plane q - 2P + k over the planes added so far
        double2 acc_[S];
#pragma unroll
        for (int k = 0; k < S; ++k) acc_[k] = make_double2(0.0, 0.0);
        load_plane(0);
        own(0);
        for (int q = 0; q < nq; ++q) {
            store_plane(q);
            load_plane(q + 1);
            lds_barrier();
            if (outv) {
                const double2* row0 = smem + (size_t)(q & 1) * HY * RW + (size_t)(oy + P) * RW + ox + P;
                scatter_plane<P>(row0, RW, q, nz, acc_, std::make_integer_sequence<int, P + 1>{});
            }
            if (q >= 2 * P) {  // output plane o = q - 2P has its whole window
                const int o = q - 2 * P;
                double yv[V], kv[V], av[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    yv[v] = ny[v];
                    kv[v] = nk[v];
                    av[v] = na[v];
                }
                own(o + 1);
                if (outv) {
                    const uint32_t qi = obase + plane * (uint32_t)(z0 + o);
                    const double2 W = acc_[0];
                    double zz[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) zz[v] = stage == 1 ? yv[v] : fma(cdt, kv[v], yv[v]);
                    const double2 xo = M::map(zz);
                    double k[V];
                    M::rhs(d, zz, xo, W, k);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const double kk = kq<KT>(k[v]);
                        if (stage <= 3) st32(gp((KT*)d.k[stage - 1]) + (int64_t)v * n, qi, (KT)kk);
                        if (stage == 2)
                            st32(gp(d.acc) + (int64_t)v * n, qi, fma(d.dt3, kk, fma(d.dt6, kv[v], yv[v])));
                        if (stage == 4) {
                            const double yo = fma(d.dt6, kk, fma(d.dt3, kv[v], av[v]));
                            st32(gp(d.y[par ^ 1]) + (int64_t)v * n, qi, yo);
                            flag_nonfinite(d, yo);
                        }
                    }
                    if (stage == 1) {
                        part[0] += xo.x;
                        part[1] += xo.y;
                        if (MV && (d.obs & OBS_MV) && g == d.mv_start) st32(gp(d.mv), qi, yv[0]);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k + 1 < S; ++k) acc_[k] = acc_[k + 1];
            acc_[S - 1] = make_double2(0.0, 0.0);
        }
        if (stage == 1) {
            block_sum<kBallScatterBlock, 2>(part, lds);
            if (tid == 0) {
                gp(d.tsum[0])[2 * t] = part[0];
                gp(d.tsum[0])[2 * t + 1] = part[1];
            }
        } else {
            __syncthreads();  // LDS reuse by the next work item
        }
    }
}

template <int MODEL, class KT, int P>
static void scatter_entry(CubeLaunch* r, const CubeLaunch& finals) {
    r->stage[0] = k_ball_scatter<MODEL, KT, P, 1, false>;
    r->stage[1] = k_ball_scatter<MODEL, KT, P, 2, false>;
    r->stage[2] = k_ball_scatter<MODEL, KT, P, 3, false>;
    r->stage[3] = k_ball_scatter<MODEL, KT, P, 4, false>;
    r->stage_mv[0] = k_ball_scatter<MODEL, KT, P, 1, true>;
    r->stage_mv[1] = k_ball_scatter<MODEL, KT, P, 2, true>;
    r->stage_mv[2] = k_ball_scatter<MODEL, KT, P, 3, true>;
    r->stage_mv[3] = k_ball_scatter<MODEL, KT, P, 4, true>;
    r->final_partials = finals.final_partials;
    r->final_R = finals.final_R;
}

template <int MODEL, class KT>
static bool scatter_pick(int P, CubeLaunch* out) {
    CubeLaunch finals;
    if (!ball_select(MODEL, sizeof(KT) == 8 ? ND_FP64 : ND_FP32_BULK, 1024, &finals)) return false;
    switch (P) {
        case 1: scatter_entry<MODEL, KT, 1>(out, finals); return true;
        case 2: scatter_entry<MODEL, KT, 2>(out, finals); return true;
        case 3: scatter_entry<MODEL, KT, 3>(out, finals); return true;
        case 4: scatter_entry<MODEL, KT, 4>(out, finals); return true;
        case 5: scatter_entry<MODEL, KT, 5>(out, finals); return true;
        case 6: scatter_entry<MODEL, KT, 6>(out, finals); return true;
        case 7: scatter_entry<MODEL, KT, 7>(out, finals); return true;
        case 8: scatter_entry<MODEL, KT, 8>(out, finals); return true;
        default: return false;
    }
}
static_assert(kBallMaxP == 8, "plane-scatter radii");

bool ball_scatter_available(int P) { return P >= 1 && P <= kBallMaxP; }

bool ball_scatter_select(int model, int prec, int P, CubeLaunch* out) {
    if (model == ND_KURAMOTO)
        return prec == ND_FP64 ? scatter_pick<ND_KURAMOTO, double>(P, out) : scatter_pick<ND_KURAMOTO, float>(P, out);
    if (model == ND_KURAMOTO_INERTIA)
        return prec == ND_FP64 ? scatter_pick<ND_KURAMOTO_INERTIA, double>(P, out)
                               : scatter_pick<ND_KURAMOTO_INERTIA, float>(P, out);
    return false;
}

size_t ball_scatter_smem_bytes(int P, int cx, int cy) {
    return (size_t)2 * (cy + 2 * P) * (cx + 2 * P + 1) * sizeof(double2);
}

}  // namespace nd
