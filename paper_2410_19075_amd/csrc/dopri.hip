// Dormand-Prince 5(4) with step-size control on the device: rings held by one
// workgroup each, and (further below) rings of any size and compressed
// coupling matrices tiled over workgroups.
//
// The paper's default solver is the adaptive embedded pair of Dormand and
// Prince (Sec. III.A).  Every ring of up to 1024 elements is integrated
// by one workgroup from t = 0 to its own t_end: the state and the seven stage
// slopes stay in registers, each stage's window sums come from LDS prefix sums
// of the mapped stage values (as in the resident RK4 kernel), and the step
// control is the usual one (Hairer, Norsett & Wanner, Solving ODEs I, II.4):
//   err = sqrt(mean_i ((y5_i - y4_i) / (atol + rtol max(|y_i|, |y5_i|)))^2),
//   accept when err <= 1, new h = h min(facmax, max(0.2, 0.9 err^(-1/5))),
//   facmax = 10, or 1 right after a rejection; the step that reaches t_end
//   (to within a relative 1e-12 of h) ends on it; rtol <= 0 means fixed steps.
// A controlled run stops as failed when its error estimate is not finite (a
// NaN or Inf in the state or the slopes) or its proposed step falls below 10
// units in the last place of t; the state stays at the last accepted step.
// The fifth-order solution propagates, and the last stage is the first stage
// of the next step.  The error norm is one fixed-order block reduction, so the
// accept/reject decisions are the same in every run.  Each ring decides for
// itself: a batch of rings with different parameters and horizons runs in one
// launch without host round trips.
#include <cmath>

#include "models.h"
#include "runtime.h"

namespace nd {

namespace {
constexpr int kDpBS = 512, kDpEPT = 2, kDpCap = kDpBS * kDpEPT;  // ring capacity 1024
constexpr int kDpStats = 5;  // per ring: t, accepted, rejected, next h, failed

__device__ __constant__ double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
// fifth- minus fourth-order weights
__device__ __constant__ double kDpE[7] = {71.0 / 57600, 0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200,
                                           22.0 / 525, -1.0 / 40};
// continuous extension of order 4 (dense output; Hairer, Norsett & Wanner, Solving ODEs I, II.6)
__device__ __constant__ double kDpD[7] = {-12715105075.0 / 11282082432.0, 0.0, 87487479700.0 / 32700410799.0,
                                           -10690763975.0 / 1880347072.0, 701980252875.0 / 199316789632.0,
                                           -1453857185.0 / 822651844.0, 69997945.0 / 29380423.0};
}  // namespace

// Where the dense output goes: R (and optionally the state) of network b at
// output k is R[b * r_stride + k] (Y[b * y_stride + k * V * n + v * n + i]).
struct DenseOut {
    double t_out;  // output spacing (> 0: outputs at k * t_out, k = 0 .. floor(t_end / t_out))
    double* R;
    int64_t r_stride;
    double* Y;     // may be NULL
    int64_t y_stride;
};

template <int MODEL, bool DENSE>
__device__ __forceinline__ void ring_dopri(const NetDesc* __restrict__ D, const double* __restrict__ t_end,
                                           double rtol, double atol, int64_t max_steps, double* __restrict__ stats,
                                           DenseOut out) {
    using M = RingModel<MODEL, double>;
    constexpr int V = M::V, T = kDpCap, EPT = kDpEPT, NW = kDpBS / kWave;
    __shared__ double pf[2 * T];  // inclusive prefix sums of the two map components
    __shared__ double lds[8 * NW];
    const int tid = threadIdx.x;
    const NetDesc& d = D[blockIdx.x];
    const int n = (int)d.n, P = (int)d.P;
    ND_GLOBAL double* y_g = gp(d.y[d.ypar]);
    double y[EPT][V], k[7][EPT][V];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = tid * EPT + e;
#pragma unroll
        for (int v = 0; v < V; ++v) y[e][v] = i < n ? y_g[(int64_t)v * n + i] : 0.0;
    }
    // slopes of stage value z: map, block prefix sums, window sums, RHS
    auto slopes = [&](const double (&z)[EPT][V], double (&kout)[EPT][V]) {
        double2 x[EPT];
        double tot[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid * EPT + e;
            x[e] = M::map(z[e]);
            if (i >= n) x[e] = make_double2(0.0, 0.0);
            tot[0] += x[e].x;
            tot[1] += x[e].y;
            pf[tid * EPT + e] = tot[0];
            pf[T + tid * EPT + e] = tot[1];
        }
        block_exscan<kDpBS, 2>(tot, lds);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            pf[tid * EPT + e] += tot[0];
            pf[T + tid * EPT + e] += tot[1];
        }
        lds_barrier();
        const double t0 = pf[n - 1], t1 = pf[T + n - 1];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid * EPT + e;
#pragma unroll
            for (int v = 0; v < V; ++v) kout[e][v] = 0.0;
            if (i < n) {
                const int lo = i - P, hi = i + P + 1;
                auto pre = [&](int q, int c) { return q == 0 ? 0.0 : pf[c * T + q - 1]; };
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
                M::rhs(d, z[e], x[e], W, kout[e]);
            }
        }
        lds_barrier();  // pf is rewritten by the next stage
    };
    // dense output k: the state y + hs sum_q w_q(theta) k_q (theta = 0: y itself), its
    // order parameter by a fixed-order block reduction
    auto emit = [&](int64_t kout, double theta, double hs) {
        double wt[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double b = q < 6 ? kDpA[6][q] : 0.0, e1 = q == 0 ? 1.0 : 0.0, e7 = q == 6 ? 1.0 : 0.0;
            wt[q] = theta * (b + (1.0 - theta) * (e1 - b + theta * (2.0 * b - e1 - e7 + (1.0 - theta) * kDpD[q])));
        }
        double s2[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid * EPT + e;
            if (i >= n) continue;
            double yt[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                double a = 0.0;
#pragma unroll
                for (int q = 0; q < 7; ++q) a += wt[q] * k[q][e][v];
                yt[v] = theta == 0.0 ? y[e][v] : y[e][v] + hs * a;
                if (out.Y) gp(out.Y)[blockIdx.x * out.y_stride + kout * V * n + (int64_t)v * n + i] = yt[v];
            }
            if constexpr (MODEL == ND_FHN) {
                const double r = sqrt(yt[0] * yt[0] + yt[1] * yt[1]);
                s2[0] += yt[0] / r;
                s2[1] += yt[1] / r;
            } else {
                const double2 x = M::map(yt);
                s2[0] += x.x;
                s2[1] += x.y;
            }
        }
        block_sum<kDpBS, 2>(s2, lds);
        if (tid == 0) gp(out.R)[blockIdx.x * out.r_stride + kout] = sqrt(s2[0] * s2[0] + s2[1] * s2[1]) / (double)n;
    };
    slopes(y, k[0]);
    const double tend = t_end[blockIdx.x];
    double t = 0.0, h = d.dt, facmax = 10.0;
    int64_t acc = 0, rej = 0;
    const int64_t K = DENSE ? (int64_t)floor(tend / out.t_out) : -1;
    int64_t next = 0;
    if (DENSE && K >= 0) {
        emit(0, 0.0, 0.0);
        next = 1;
    }
    // every wave leaves the loop together: t, h, err and the counters are uniform
    bool failed = false;
    while (t < tend && acc + rej < max_steps) {
        if (rtol > 0.0 && h < 10.0 * (nextafter(t, INFINITY) - t)) {  // step below its floor
            failed = true;
            break;
        }
        const bool last = tend - t <= h * (1.0 + 1e-12);
        const double hs = last ? tend - t : h;
        double z[EPT][V];
#pragma unroll
        for (int s = 1; s < 7; ++s) {
#pragma unroll
            for (int e = 0; e < EPT; ++e)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    double a = 0.0;
#pragma unroll
                    for (int q = 0; q < s; ++q) a += kDpA[s][q] * k[q][e][v];
                    z[e][v] = y[e][v] + hs * a;
                }
            slopes(z, k[s]);
        }
        // z is the fifth-order solution (stage 7 uses the weights b)
        bool accept = true;
        double f = 1.0;
        if (rtol > 0.0) {
            double sum[1] = {0.0};
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                if (tid * EPT + e >= n) continue;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    double er = 0.0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) er += kDpE[q] * k[q][e][v];
                    er *= hs;
                    const double sc = atol + rtol * fmax(fabs(y[e][v]), fabs(z[e][v]));
                    sum[0] += (er / sc) * (er / sc);
                }
            }
            block_sum<kDpBS, 1>(sum, lds);
            const double err = sqrt(sum[0] / (double)(V * n));
            if (!isfinite(err)) {  // a NaN or Inf in the state or the slopes
                failed = true;
                break;
            }
            f = 0.9 * pow(err, -0.2);
            accept = err <= 1.0;
        }
        if (accept) {
            if constexpr (DENSE) {
                // outputs inside (t, t + hs]; the last step takes every one left
                const double tn = last ? tend : t + hs;
                for (; next <= K; ++next) {
                    const double tk = (double)next * out.t_out;
                    if (tk > tn && !last) break;
                    emit(next, fmin((tk - t) / hs, 1.0), hs);
                }
            }
#pragma unroll
            for (int e = 0; e < EPT; ++e)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    y[e][v] = z[e][v];
                    k[0][e][v] = k[6][e][v];
                }
            t = last ? tend : t + hs;
            ++acc;
            if (rtol > 0.0) h = hs * fmin(facmax, fmax(0.2, f));
            facmax = 10.0;
        } else {
            ++rej;
            h = hs * fmax(0.2, fmin(1.0, f));
            facmax = 1.0;
        }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = tid * EPT + e;
        if (i < n) {
#pragma unroll
            for (int v = 0; v < V; ++v) y_g[(int64_t)v * n + i] = y[e][v];
        }
    }
    if (tid == 0) {
        ND_GLOBAL double* st = gp(stats) + kDpStats * blockIdx.x;
        st[0] = t;
        st[1] = (double)acc;
        st[2] = (double)rej;
        st[3] = h;
        st[4] = failed ? 1.0 : 0.0;
    }
}

template <int MODEL, bool DENSE>
__global__ __launch_bounds__(kDpBS) void k_ring_dopri(const NetDesc* __restrict__ D,
                                                      const double* __restrict__ t_end, double rtol, double atol,
                                                      int64_t max_steps, double* __restrict__ stats, DenseOut out) {
    ring_dopri<MODEL, DENSE>(D, t_end, rtol, atol, max_steps, stats, out);
}

// The Kuramoto ring without dense output fits 128 registers per lane, so two
// rings (workgroups of 8 waves) share a CU and hide each other's barriers.
__global__ __launch_bounds__(kDpBS) __attribute__((amdgpu_waves_per_eu(4))) void k_ring_dopri_kuramoto(
    const NetDesc* __restrict__ D, const double* __restrict__ t_end, double rtol, double atol, int64_t max_steps,
    double* __restrict__ stats, DenseOut out) {
    ring_dopri<ND_KURAMOTO, false>(D, t_end, rtol, atol, max_steps, stats, out);
}


// ------------------------------------------------------------ tiled rings
// Rings larger than one workgroup: the same method and step control, with
// every stage spread over tiles of 512 elements in three launches (stage value,
// its map and the tile's prefix sums; the tiles' offsets; window sums, RHS and,
// at the last stage, the error terms), and one controller launch per step
// attempt that takes the accept / reject decision on the device.  The host
// replays attempts in groups and only reads back whether every ring is done.
// Window sums come from global prefix sums of the map: the prefix of element k
// is its tile's offset (fixed-order scan of the tile totals) plus its
// in-tile inclusive prefix.
constexpr int kDtBS = 256, kDtEPT = 2, kDtT = kDtBS * kDtEPT;
// rings of at most this many tiles get their tile offsets in each RHS workgroup
// (a scan of the tile totals into LDS); longer rings in a launch of their own
constexpr int kDtScanMax = 2048;

// Per-ring control block, advanced by the controller on the device.
struct DtCtl {
    double t, h, hs, facmax;
    int64_t acc, rej;
    int32_t done, last, f, ypar;  // f: physical buffer of k1 (k_q lives at (f + q - 1) mod 7)
    // dense output: outputs [out_lo, out_hi) lie in the step just accepted, which
    // started at t_prev with size hs_prev, state y[ypar_prev] and k1 at f_prev
    int64_t next, out_lo, out_hi;
    double t_prev, hs_prev;
    int32_t f_prev, ypar_prev;
    int32_t failed, pad_;  // failed: non-finite error estimate or step below its floor
};

// Per-ring buffers of one call.
struct DtNet {
    int32_t n, P, G, V;
    int32_t gather;   // the RHS reads other elements' maps (compressed coupling matrix)
    double tend;
    double* y[2];     // state, and the fifth-order solution of the attempt
    double* k[7];     // stage slopes (physical buffers)
    double* Z;        // stage value of stages 1 .. 5 (stage 0 is y, stage 6 goes to y[ypar ^ 1])
    double* M;        // [n] map of the current stage value, as double2 (written when gather is set)
    double* pre;      // [2][n] in-tile inclusive prefix of M
    double* tot;      // [2][G] tile totals, then (after the offsets launch) exclusive offsets
    double* errp;     // [G] error partial sums of the attempt
    DtCtl* ctl;
    int64_t K;        // dense output: last output index (-1: none)
    double* Rpart;    // dense output: [K + 1][G][2] per-tile sums of the order parameter
    double* R;        // dense output: R of outputs 0 .. K (device)
    double* Y;        // dense output: states at the outputs (device, may be NULL)
};

// Stage value z of stage S (S = 0: the state; S = 6: the fifth-order
// solution, kept in y[ypar ^ 1]), its map and the tile's inclusive prefix.
// Element e * kDtBS + tid of the tile belongs to thread tid, so every access
// of a wave is one contiguous run; the stage is a template parameter so the
// slopes' loads are all issued before the sums that use them.
template <int MODEL, int S>
__global__ __launch_bounds__(kDtBS) void k_dt_map(const DtNet* __restrict__ R, const int2* __restrict__ work) {
    using M = RingModel<MODEL, double>;
    constexpr int V = M::V, NW = kDtBS / kWave, NE = 2 * kDtEPT;
    __shared__ double lds[2 * NE * NW];
    const int2 wk = work[blockIdx.x];
    const DtNet& r = R[wk.x];
    const DtCtl c = *r.ctl;
    if (c.done) return;
    const int n = r.n, t0 = wk.y * kDtT, tid = threadIdx.x;
    const double* __restrict__ y = r.y[c.ypar];
    const double* kq[S > 0 ? S : 1];
#pragma unroll
    for (int q = 0; q < S; ++q) kq[q] = r.k[(c.f + q) % 7];
    double* __restrict__ zo = S == 6 ? r.y[c.ypar ^ 1] : r.Z;
    double xs[NE];
#pragma unroll
    for (int e = 0; e < kDtEPT; ++e) {
        const int i = t0 + e * kDtBS + tid;
        double2 x = make_double2(0.0, 0.0);
        if (i < n) {
            double z[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int64_t o = (int64_t)v * n + i;
                double a = 0.0;
#pragma unroll
                for (int q = 0; q < S; ++q) a += kDpA[S][q] * kq[q][o];
                z[v] = S == 0 ? y[o] : y[o] + c.hs * a;
            }
            x = M::map(z);
            if (S > 0) {  // kept for the RHS launch of this stage
#pragma unroll
                for (int v = 0; v < V; ++v) zo[(int64_t)v * n + i] = z[v];
            }
            if (r.gather) ((double2*)r.M)[i] = x;
        }
        xs[2 * e] = x.x;
        xs[2 * e + 1] = x.y;
    }
    // block sums and thread-exclusive prefixes of each element run
    double bs[NE], ex[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) bs[q] = ex[q] = xs[q];
    block_sum_and_exscan<kDtBS, NE, NE>(bs, ex, lds);
    double off0 = 0.0, off1 = 0.0;
#pragma unroll
    for (int e = 0; e < kDtEPT; ++e) {
        const int i = t0 + e * kDtBS + tid;
        if (i < n) {
            r.pre[i] = off0 + (ex[2 * e] + xs[2 * e]);
            r.pre[n + i] = off1 + (ex[2 * e + 1] + xs[2 * e + 1]);
        }
        off0 += bs[2 * e];
        off1 += bs[2 * e + 1];
    }
    if (tid == 0) {
        r.tot[wk.y] = off0;
        r.tot[r.G + wk.y] = off1;
    }
}

// Exclusive offsets of the tiles (one workgroup per ring, fixed order).
__global__ __launch_bounds__(kDtBS) void k_dt_offsets(const DtNet* __restrict__ R) {
    const DtNet& r = R[blockIdx.x];
    if (r.ctl->done || r.G <= kDtScanMax) return;
    __shared__ double lds[4 * (kDtBS / kWave)];
    __shared__ double chunk[2];
    double carry0 = 0.0, carry1 = 0.0;
    for (int b0 = 0; b0 < r.G; b0 += kDtBS) {
        const int q = b0 + (int)threadIdx.x;
        const double own0 = q < r.G ? r.tot[q] : 0.0, own1 = q < r.G ? r.tot[r.G + q] : 0.0;
        double v[2] = {own0, own1};
        block_exscan<kDtBS, 2>(v, lds);  // v: exclusive prefix in this chunk
        if (threadIdx.x == kDtBS - 1) {
            chunk[0] = v[0] + own0;
            chunk[1] = v[1] + own1;
        }
        if (q < r.G) {
            r.tot[q] = carry0 + v[0];
            r.tot[r.G + q] = carry1 + v[1];
        }
        __syncthreads();
        carry0 += chunk[0];
        carry1 += chunk[1];
        __syncthreads();
    }
}

// Neighbour sums (ring: windows from the global prefix; links: the compressed
// coupling matrix's rows, extracted as in the stage kernels of that topology),
// the RHS of stage s into k_{s+1} and, at the last stage, the error terms of
// the attempt.
template <int MODEL, int TOPO>
__global__ __launch_bounds__(kDtBS) void k_dt_rhs(const DtNet* __restrict__ R, const NetDesc* __restrict__ D,
                                                  const int2* __restrict__ work, int nwork, int s, double rtol,
                                                  double atol) {
    using M = RingModel<MODEL, double>;
    constexpr int V = M::V, NW = kDtBS / kWave;
    __shared__ double lds[3 * NW];
    extern __shared__ double dt_off[];  // [2][G]: exclusive tile offsets (rings of <= kDtScanMax tiles)
    // row tiles that share gathers stay on one XCD (its own L2)
    const int w = xcd_work(blockIdx.x, nwork);
    if (w < 0) return;
    const int2 wk = work[w];
    const DtNet& r = R[wk.x];
    const NetDesc& d = D[wk.x];
    const DtCtl c = *r.ctl;
    if (c.done) return;
    const int n = r.n, P = r.P, t0 = wk.y * kDtT, tid = threadIdx.x;
    const int G = r.G;
    const bool local = TOPO == ND_RING && G <= kDtScanMax;  // uniform over the block
    if (local) {
        // each thread adds a run of consecutive tile totals; the block scans the
        // runs' sums; every workgroup of the ring computes the same offsets
        const int per = (G + kDtBS - 1) / kDtBS, u0 = min(tid * per, G), u1 = min(u0 + per, G);
        double v[2] = {0.0, 0.0};
        for (int u = u0; u < u1; ++u) {
            v[0] += r.tot[u];
            v[1] += r.tot[G + u];
        }
        block_exscan<kDtBS, 2>(v, lds);
        for (int u = u0; u < u1; ++u) {
            dt_off[u] = v[0];
            dt_off[G + u] = v[1];
            v[0] += r.tot[u];
            v[1] += r.tot[G + u];
        }
        __syncthreads();
    }
    auto S = [&](int k, int comp) {  // inclusive global prefix of element k (k = -1: 0)
        if (k < 0) return 0.0;
        const double o = local ? dt_off[comp * G + k / kDtT] : r.tot[comp * G + k / kDtT];
        return o + r.pre[comp * n + k];
    };
    double es[1] = {0.0};
#pragma unroll
    for (int e = 0; e < kDtEPT; ++e) {
        const int i = t0 + e * kDtBS + tid;
        if (i >= n) continue;
        // the stage value as the map launch computed it
        const double* zs = s == 0 ? r.y[c.ypar] : (s == 6 ? r.y[c.ypar ^ 1] : r.Z);
        double z[V];
#pragma unroll
        for (int v = 0; v < V; ++v) z[v] = zs[(int64_t)v * n + i];
        // the element's own map: stored by the map launch where the rows gather
        // maps anyway, else recomputed from the same stage value (same bits)
        const double2 x = TOPO == ND_LINKS ? ((const double2*)r.M)[i] : M::map(z);
        double2 W;
        if constexpr (TOPO == ND_RING) {
            const int lo = i - P, hi = i + P;
            double w0, w1;
            if (lo < 0) {
                w0 = S(hi, 0) + (S(n - 1, 0) - S(lo + n - 1, 0));
                w1 = S(hi, 1) + (S(n - 1, 1) - S(lo + n - 1, 1));
            } else if (hi >= n) {
                w0 = (S(n - 1, 0) - S(lo - 1, 0)) + S(hi - n, 0);
                w1 = (S(n - 1, 1) - S(lo - 1, 1)) + S(hi - n, 1);
            } else {
                w0 = S(hi, 0) - S(lo - 1, 0);
                w1 = S(hi, 1) - S(lo - 1, 1);
            }
            W = make_double2(w0 - x.x, w1 - x.y);
        } else {
            // row i = (V XOR D[C_i]) shifted by i: V's positions, then the entry's
            // signed positions, divided by the row's link count
            const double2* __restrict__ mp = (const double2*)r.M;
            double w0 = 0.0, w1 = 0.0;
#pragma unroll 8
            for (int q = 0; q < d.lnv; ++q) {
                int j = i + d.lvpos[q];
                j -= j >= n ? n : 0;
                const double2 m = mp[j];
                w0 += m.x;
                w1 += m.y;
            }
            const int ke = d.lrow[i];
            for (int e2 = d.ldptr[ke]; e2 < d.ldptr[ke + 1]; ++e2) {
                const int32_t v = d.ldpos[e2];
                int j = i + (v & ~kLinksRemove);
                j -= j >= n ? n : 0;
                const double sg = (v & kLinksRemove) ? -1.0 : 1.0;
                const double2 m = mp[j];
                w0 += sg * m.x;
                w1 += sg * m.y;
            }
            const double inv = d.linv[ke];
            W = inv != 0.0 ? make_double2(w0 * inv, w1 * inv)
                           : (MODEL == ND_FHN ? make_double2(z[0], z[V - 1]) : make_double2(0.0, 0.0));
        }
        double k[V];
        M::rhs(d, z, x, W, k);
        double* ko = r.k[(c.f + s) % 7];
#pragma unroll
        for (int v = 0; v < V; ++v) ko[(int64_t)v * n + i] = k[v];
        if (s == 6 && rtol > 0.0) {
            const double* y = r.y[c.ypar];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                double er = 0.0;
                for (int q = 0; q < 7; ++q) er += kDpE[q] * r.k[(c.f + q) % 7][(int64_t)v * n + i];
                er *= c.hs;
                const double sc = atol + rtol * fmax(fabs(y[(int64_t)v * n + i]), fabs(z[v]));
                es[0] += (er / sc) * (er / sc);
            }
        }
    }
    if (s == 6) {
        block_sum<kDtBS, 1>(es, lds);
        if (tid == 0) r.errp[wk.y] = es[0];
    }
}

// The accept / reject decision of the attempt and the next step (one wave per
// ring: lane l adds the error partials of tiles l, l + 64, ... in order, the
// wave adds the lanes' sums in a fixed tree; lane 0 decides).
__global__ __launch_bounds__(kWave) void k_dt_control(const DtNet* __restrict__ R, double rtol, int64_t max_steps,
                                                       double t_out) {
    const DtNet& r = R[blockIdx.x];
    double sum = 0.0;
    if (rtol > 0.0 && !r.ctl->done) {  // uniform over the wave
        for (int q = threadIdx.x; q < r.G; q += kWave) sum += r.errp[q];
        sum = wave_sum(sum);
    }
    if (threadIdx.x != 0) return;
    DtCtl c = *r.ctl;
    if (c.done) {
        if (c.out_hi != c.out_lo) {  // nothing more to emit
            c.out_lo = c.out_hi = 0;
            *r.ctl = c;
        }
        return;
    }
    c.out_lo = c.out_hi = 0;
    bool accept = true;
    double f = 1.0;
    if (rtol > 0.0) {
        const double err = sqrt(sum / ((double)r.V * (double)r.n));
        if (!isfinite(err)) {  // a NaN or Inf in the state or the slopes: stop, state kept
            c.failed = 1;
            c.done = 1;
            *r.ctl = c;
            return;
        }
        f = 0.9 * pow(err, -0.2);
        accept = err <= 1.0;
    }
    if (accept) {
        if (r.K >= 0) {  // outputs inside (t, t + hs]; the last step takes every one left
            const double tn = c.last ? r.tend : c.t + c.hs;
            c.out_lo = c.next;
            while (c.next <= r.K && ((double)c.next * t_out <= tn || c.last)) ++c.next;
            c.out_hi = c.next;
            c.t_prev = c.t;
            c.hs_prev = c.hs;
            c.f_prev = c.f;
            c.ypar_prev = c.ypar;
        }
        c.t = c.last ? r.tend : c.t + c.hs;
        ++c.acc;
        if (rtol > 0.0) c.h = c.hs * fmin(c.facmax, fmax(0.2, f));
        c.facmax = 10.0;
        c.ypar ^= 1;
        c.f = (c.f + 6) % 7;  // k1 of the next step is this step's k7
    } else {
        ++c.rej;
        c.h = c.hs * fmax(0.2, fmin(1.0, f));
        c.facmax = 1.0;
    }
    c.done = !(c.t < r.tend && c.acc + c.rej < max_steps);
    if (!c.done && rtol > 0.0 && c.h < 10.0 * (nextafter(c.t, INFINITY) - c.t)) {  // step below its floor
        c.failed = 1;
        c.done = 1;
    }
    if (!c.done) {
        c.last = r.tend - c.t <= c.h * (1.0 + 1e-12);
        c.hs = c.last ? r.tend - c.t : c.h;
    }
    *r.ctl = c;
}

// Dense output of the step just accepted: for each of its outputs, the
// continuous extension on the tile's elements (the state, when requested) and
// the tile's sums of the order parameter's unit vectors.
template <int MODEL>
__global__ __launch_bounds__(kDtBS) void k_dt_emit(const DtNet* __restrict__ R, const int2* __restrict__ work,
                                                   double t_out) {
    using M = RingModel<MODEL, double>;
    constexpr int V = M::V, NW = kDtBS / kWave;
    __shared__ double lds[2 * NW];
    const int2 wk = work[blockIdx.x];
    const DtNet& r = R[wk.x];
    const DtCtl c = *r.ctl;
    if (c.out_hi <= c.out_lo) return;
    const int n = r.n, t0 = wk.y * kDtT, tid = threadIdx.x;
    const double* y = r.y[c.ypar_prev];
    for (int64_t ko = c.out_lo; ko < c.out_hi; ++ko) {
        const double theta = fmin(((double)ko * t_out - c.t_prev) / c.hs_prev, 1.0);
        double wt[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double b = q < 6 ? kDpA[6][q] : 0.0, e1 = q == 0 ? 1.0 : 0.0, e7 = q == 6 ? 1.0 : 0.0;
            wt[q] = theta * (b + (1.0 - theta) * (e1 - b + theta * (2.0 * b - e1 - e7 + (1.0 - theta) * kDpD[q])));
        }
        double s2[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < kDtEPT; ++e) {
            const int i = t0 + e * kDtBS + tid;
            if (i >= n) continue;
            double yt[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                yt[v] = y[(int64_t)v * n + i];
                if (theta != 0.0) {  // theta = 0: the initial state (no stage slopes yet)
                    double a = 0.0;
                    for (int q = 0; q < 7; ++q) a += wt[q] * r.k[(c.f_prev + q) % 7][(int64_t)v * n + i];
                    yt[v] += c.hs_prev * a;
                }
                if (r.Y) r.Y[ko * V * n + (int64_t)v * n + i] = yt[v];
            }
            if constexpr (MODEL == ND_FHN) {
                const double rr = sqrt(yt[0] * yt[0] + yt[1] * yt[1]);
                s2[0] += yt[0] / rr;
                s2[1] += yt[1] / rr;
            } else {
                const double2 x = M::map(yt);
                s2[0] += x.x;
                s2[1] += x.y;
            }
        }
        block_sum<kDtBS, 2>(s2, lds);
        if (tid == 0) {
            r.Rpart[(ko * r.G + wk.y) * 2] = s2[0];
            r.Rpart[(ko * r.G + wk.y) * 2 + 1] = s2[1];
        }
    }
}

// R of every emitted output from the tiles' sums: block (ring, y) takes outputs
// y, y + kDtRBlocks, ...; thread l adds tiles l, l + kDtBS, ... in order and
// the block adds the threads' sums in a fixed order.
constexpr int kDtRBlocks = 64;
__global__ __launch_bounds__(kDtBS) void k_dt_reduce_R(const DtNet* __restrict__ R) {
    constexpr int NW = kDtBS / kWave;
    __shared__ double lds[2 * NW];
    const DtNet& r = R[blockIdx.x];
    const int64_t emitted = min(r.ctl->next, r.K + 1);
    for (int64_t ko = blockIdx.y; ko < emitted; ko += kDtRBlocks) {  // uniform over the block
        double s2[2] = {0.0, 0.0};
        for (int q = threadIdx.x; q < r.G; q += kDtBS) {
            s2[0] += r.Rpart[(ko * r.G + q) * 2];
            s2[1] += r.Rpart[(ko * r.G + q) * 2 + 1];
        }
        block_sum<kDtBS, 2>(s2, lds);
        if (threadIdx.x == 0) r.R[ko] = sqrt(s2[0] * s2[0] + s2[1] * s2[1]) / (double)r.n;
    }
}
}  // namespace nd

using namespace nd;

typedef void (*DtMapFn)(const DtNet*, const int2*);
template <int MODEL>
static DtMapFn dt_map_of_model(int s) {
    switch (s) {
        case 0: return k_dt_map<MODEL, 0>;
        case 1: return k_dt_map<MODEL, 1>;
        case 2: return k_dt_map<MODEL, 2>;
        case 3: return k_dt_map<MODEL, 3>;
        case 4: return k_dt_map<MODEL, 4>;
        case 5: return k_dt_map<MODEL, 5>;
        default: return k_dt_map<MODEL, 6>;
    }
}
static DtMapFn dt_map_kernel(int model, int s) {
    if (model == ND_KURAMOTO) return dt_map_of_model<ND_KURAMOTO>(s);
    if (model == ND_FHN) return dt_map_of_model<ND_FHN>(s);
    return dt_map_of_model<ND_KURAMOTO_INERTIA>(s);
}

// Rings beyond one workgroup: buffers per ring, the stage / controller launches
// replayed in groups of attempts until every ring is done.
static nd_status run_adaptive_tiled(const std::vector<Net*>& nets, int model, int topo, const double* t_end,
                                    const double* dt0, double rtol, double atol, int64_t max_steps,
                                    nd_adaptive_stats* stats, hipStream_t st, double t_out, double* Rh,
                                    int64_t r_stride, double* Yh, int64_t y_stride) {
    const bool dense = t_out > 0.0;
    const int count = (int)nets.size();
    std::vector<DtNet> rs(count);
    std::vector<DtCtl> cs(count);
    std::vector<NetDesc> descs(count);
    std::vector<int2> work;
    size_t bytes = 0;
    for (int b = 0; b < count; ++b) {
        const Net* nt = nets[b];
        const int64_t n = nt->prob.n, len = nvars_of(nt->prob.model) * n, G = (n + kDtT - 1) / kDtT;
        bytes += (size_t)(9 * len + 4 * n + 3 * G) * 8 + sizeof(DtCtl);
        if (dense) bytes += (size_t)(2 * ((int64_t)std::floor(t_end[b] / t_out) + 1) * G) * 8;
        for (int64_t t = 0; t < G; ++t) work.push_back(make_int2(b, (int)t));
    }
    const size_t bd = (size_t)count * sizeof(DtNet), bn = (size_t)count * sizeof(NetDesc),
                 bw = work.size() * sizeof(int2);
    const size_t br = dense ? (size_t)count * r_stride * 8 : 0, by = dense && Yh ? (size_t)count * y_stride * 8 : 0;
    bytes += br + by;
    char* buf = nullptr;
    hipError_t e = hipMallocAsync((void**)&buf, bd + bn + bw + bytes + 256, st);
    if (e != hipSuccess) return hip_fail(e, "adaptive scratch");
    DtNet* d_r = (DtNet*)buf;
    NetDesc* d_desc = (NetDesc*)(buf + bd);
    int2* d_work = (int2*)(buf + bd + bn);
    char* p = buf + ((bd + bn + bw + 255) / 256) * 256;
    auto take = [&](size_t nbytes) {
        char* q = p;
        p += (nbytes + 7) / 8 * 8;
        return q;
    };
    for (int b = 0; b < count; ++b) {
        const Net* nt = nets[b];
        const int64_t n = nt->prob.n, len = nvars_of(nt->prob.model) * n;
        DtNet& r = rs[b];
        r.n = (int32_t)n;
        r.P = (int32_t)nt->prob.radius;
        r.gather = topo == ND_LINKS;
        r.G = (int32_t)((n + kDtT - 1) / kDtT);
        r.V = nvars_of(nt->prob.model);
        r.tend = t_end[b];
        descs[b] = nt->run_desc(dt0[b], 0);
        r.y[0] = descs[b].y[descs[b].ypar];
        r.y[1] = (double*)take(len * 8);
        for (int q = 0; q < 7; ++q) r.k[q] = (double*)take(len * 8);
        r.Z = (double*)take(len * 8);
        r.M = (double*)take(2 * n * 8);
        r.pre = (double*)take(2 * n * 8);
        r.tot = (double*)take(2 * r.G * 8);
        r.errp = (double*)take(r.G * 8);
        r.ctl = (DtCtl*)take(sizeof(DtCtl));
        r.K = dense ? (int64_t)std::floor(t_end[b] / t_out) : -1;
        r.Rpart = dense ? (double*)take(2 * (r.K + 1) * r.G * 8) : nullptr;
        r.R = nullptr;
        r.Y = nullptr;
        DtCtl& c = cs[b];
        c = DtCtl{};
        c.h = dt0[b];
        c.facmax = 10.0;
        c.done = !(0.0 < t_end[b] && max_steps > 0);
        if (!c.done && rtol > 0.0 && c.h < 10.0 * std::nextafter(0.0, INFINITY)) {  // step below its floor
            c.failed = 1;
            c.done = 1;
        }
        c.last = t_end[b] <= c.h * (1.0 + 1e-12);
        c.hs = c.last ? t_end[b] : c.h;
        if (r.K >= 0) {  // output 0 is the initial state (theta = 0)
            c.out_lo = 0;
            c.out_hi = 1;
            c.next = 1;
            c.hs_prev = 1.0;
        }
    }
    double* d_R = dense ? (double*)take(br) : nullptr;
    double* d_Y = by ? (double*)take(by) : nullptr;
    for (int b = 0; b < count; ++b) {
        if (d_R) rs[b].R = d_R + (size_t)b * r_stride;
        if (d_Y) rs[b].Y = d_Y + (size_t)b * y_stride;
    }
    const int tiles = (int)work.size();
    // tile offsets: in the RHS launch (LDS) for rings of up to kDtScanMax tiles
    bool long_rings = false;
    int local_g = 0;
    for (const DtNet& r : rs) {
        if (r.G > kDtScanMax) long_rings = true;
        else local_g = std::max(local_g, (int)r.G);
    }
    const size_t off_bytes = topo == ND_RING ? (size_t)2 * local_g * 8 : 0;
    auto stage = [&](int s) {
        const DtMapFn map = dt_map_kernel(model, s);
        hipLaunchKernelGGL(map, dim3(tiles), dim3(kDtBS), 0, st, d_r, d_work);
        if (topo == ND_RING && long_rings) hipLaunchKernelGGL(k_dt_offsets, dim3(count), dim3(kDtBS), 0, st, d_r);
        auto rhs = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((tiles + 7) / 8 * 8), dim3(kDtBS), off_bytes, st, d_r, d_desc, d_work, tiles, s,
                               rtol, atol);
        };
        if (topo == ND_RING) {
            if (model == ND_KURAMOTO) rhs(k_dt_rhs<ND_KURAMOTO, ND_RING>);
            else if (model == ND_FHN) rhs(k_dt_rhs<ND_FHN, ND_RING>);
            else rhs(k_dt_rhs<ND_KURAMOTO_INERTIA, ND_RING>);
        } else {
            if (model == ND_KURAMOTO) rhs(k_dt_rhs<ND_KURAMOTO, ND_LINKS>);
            else if (model == ND_FHN) rhs(k_dt_rhs<ND_FHN, ND_LINKS>);
            else rhs(k_dt_rhs<ND_KURAMOTO_INERTIA, ND_LINKS>);
        }
        return hipGetLastError();
    };
    auto emit = [&]() {
        if (model == ND_KURAMOTO) hipLaunchKernelGGL(k_dt_emit<ND_KURAMOTO>, dim3(tiles), dim3(kDtBS), 0, st, d_r, d_work, t_out);
        else if (model == ND_FHN) hipLaunchKernelGGL(k_dt_emit<ND_FHN>, dim3(tiles), dim3(kDtBS), 0, st, d_r, d_work, t_out);
        else hipLaunchKernelGGL(k_dt_emit<ND_KURAMOTO_INERTIA>, dim3(tiles), dim3(kDtBS), 0, st, d_r, d_work, t_out);
        return hipGetLastError();
    };
    // outputs a run does not reach read as NaN (all bits set)
    if (dense) e = hipMemsetAsync(d_R, 0xff, br + by, st);
    // the control blocks live inside the scratch: write them with the descriptors
    for (int b = 0; b < count && e == hipSuccess; ++b)
        e = hipMemcpyAsync(rs[b].ctl, &cs[b], sizeof(DtCtl), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_r, rs.data(), bd, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_desc, descs.data(), bn, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_work, work.data(), bw, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && dense) e = emit();  // output 0
    if (e == hipSuccess) e = stage(0);            // k1 = f(y)
    constexpr int kAttempts = 8;        // attempts launched between checks of the done flags
    while (e == hipSuccess) {
        for (int a = 0; a < kAttempts && e == hipSuccess; ++a) {
            for (int s = 1; s <= 6 && e == hipSuccess; ++s) e = stage(s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_dt_control, dim3(count), dim3(kWave), 0, st, d_r, rtol, max_steps,
                                   t_out);
                e = hipGetLastError();
                if (e == hipSuccess && dense) e = emit();
            }
        }
        for (int b = 0; b < count && e == hipSuccess; ++b)
            e = hipMemcpyAsync(&cs[b], rs[b].ctl, sizeof(DtCtl), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        bool all = true;
        for (const DtCtl& c : cs) all = all && c.done;
        if (all) break;
    }
    if (e == hipSuccess && dense) {
        hipLaunchKernelGGL(k_dt_reduce_R, dim3(count, kDtRBlocks), dim3(kDtBS), 0, st, d_r);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(Rh, d_R, br, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && by) e = hipMemcpyAsync(Yh, d_Y, by, hipMemcpyDeviceToHost, st);
    }
    // a state that ended in the scratch buffer goes back to the network
    for (int b = 0; b < count && e == hipSuccess; ++b)
        if (cs[b].ypar)
            e = hipMemcpyAsync(rs[b].y[0], rs[b].y[1], (size_t)rs[b].V * rs[b].n * 8, hipMemcpyDeviceToDevice, st);
    const hipError_t ef = hipFreeAsync(buf, st);
    const hipError_t es = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adaptive run (tiled)");
    if (ef != hipSuccess) return hip_fail(ef, "adaptive scratch free");
    if (es != hipSuccess) return hip_fail(es, "adaptive run (tiled)");
    int bad = -1;
    for (int b = 0; b < count; ++b) {
        stats[b].t = cs[b].t;
        stats[b].accepted = cs[b].acc;
        stats[b].rejected = cs[b].rej;
        stats[b].h_next = cs[b].h;
        stats[b].failed = cs[b].failed;
        stats[b].reserved = 0;
        if (cs[b].failed && bad < 0) bad = b;
    }
    if (bad >= 0)
        return fail(ND_ERR_NUMERIC, "adaptive run: network %d stopped at t = %.17g (non-finite error estimate or "
                                    "step below its floor)", bad, cs[bad].t);
    return ND_OK;
}

static nd_status run_adaptive(const nd_handle* hs, int32_t count, const double* t_end, const double* dt0,
                              double rtol, double atol, int64_t max_steps, nd_adaptive_stats* stats, void* stream,
                              double t_out, double* R, int64_t r_stride, double* Y, int64_t y_stride) {
    if (!hs || !t_end || !dt0 || !stats || count < 0) return fail(ND_ERR_INVALID_ARG, "bad adaptive-run arguments");
    if (!std::isfinite(rtol) || !std::isfinite(atol) || atol < 0.0 || (rtol > 0.0 && atol == 0.0))
        return fail(ND_ERR_INVALID_ARG, "rtol must be finite; atol finite, and > 0 when rtol > 0");
    if (max_steps < 0) return fail(ND_ERR_INVALID_ARG, "max_steps must be >= 0");
    const bool dense = t_out != 0.0;
    if (dense && (!(t_out > 0.0) || !std::isfinite(t_out) || !R || r_stride < 1))
        return fail(ND_ERR_INVALID_ARG, "dense output needs t_out > 0, R and r_stride >= 1");
    if (count == 0) return ND_OK;
    int model = -1, topo = -1;
    bool tiled = false;
    std::vector<NetDesc> descs(count);
    std::vector<Net*> nets(count);
    for (int i = 0; i < count; ++i) {
        Net* n = reinterpret_cast<Net*>(hs[i]);
        if (!n) return fail(ND_ERR_INVALID_ARG, "NULL handle at %d", i);
        nets[i] = n;
        if ((n->prob.topo != ND_RING && n->prob.topo != ND_LINKS) || n->prob.precision != ND_FP64 ||
            n->prob.model == ND_HH)
            return fail(ND_ERR_UNSUPPORTED, "adaptive stepping runs FP64 rings and compressed coupling matrices");
        if (topo >= 0 && n->prob.topo != topo) return fail(ND_ERR_INVALID_ARG, "one adaptive batch holds one topology");
        topo = n->prob.topo;
        tiled = tiled || n->prob.n > kDpCap || topo == ND_LINKS;
        if (model >= 0 && n->prob.model != model)
            return fail(ND_ERR_INVALID_ARG, "one adaptive batch holds one model");
        model = n->prob.model;
        if (!(t_end[i] >= 0.0) || !std::isfinite(t_end[i]) || !(dt0[i] > 0.0) || !std::isfinite(dt0[i]))
            return fail(ND_ERR_INVALID_ARG, "t_end must be finite and >= 0, dt0 finite and > 0 (network %d)", i);
        if (dense) {
            const int64_t outs = (int64_t)std::floor(t_end[i] / t_out) + 1;
            if (outs > r_stride)
                return fail(ND_ERR_INVALID_ARG, "network %d has %lld outputs, r_stride is %lld", i, (long long)outs,
                            (long long)r_stride);
            if (Y && outs * nvars_of(n->prob.model) * n->prob.n > y_stride)
                return fail(ND_ERR_INVALID_ARG, "network %d needs y_stride >= %lld", i,
                            (long long)(outs * nvars_of(n->prob.model) * n->prob.n));
        }
        descs[i] = n->run_desc(dt0[i], 0);
    }
    if (tiled) {
        return run_adaptive_tiled(nets, model, topo, t_end, dt0, rtol, atol, max_steps, stats, (hipStream_t)stream,
                                  dense ? t_out : 0.0, R, r_stride, Y, y_stride);
    }
    hipStream_t st = (hipStream_t)stream;
    void* buf = nullptr;
    const size_t bd = (size_t)count * sizeof(NetDesc), bt = (size_t)count * 8, bs = (size_t)count * kDpStats * 8;
    const size_t br = dense ? (size_t)count * r_stride * 8 : 0, by = dense && Y ? (size_t)count * y_stride * 8 : 0;
    hipError_t e = hipMallocAsync(&buf, bd + bt + bs + br + by, st);
    if (e != hipSuccess) return hip_fail(e, "adaptive scratch");
    NetDesc* d_desc = (NetDesc*)buf;
    double* d_tend = (double*)((char*)buf + bd);
    double* d_stats = (double*)((char*)buf + bd + bt);
    DenseOut o{dense ? t_out : 0.0, dense ? (double*)((char*)buf + bd + bt + bs) : nullptr, r_stride,
               by ? (double*)((char*)buf + bd + bt + bs + br) : nullptr, y_stride};
    std::vector<double> h_stats((size_t)count * kDpStats);
    // outputs a run does not reach (max_steps) read as NaN (all bits set)
    if (dense) e = hipMemsetAsync(o.R, 0xff, br + by, st);
    if (e == hipSuccess && (e = hipMemcpyAsync(d_desc, descs.data(), bd, hipMemcpyHostToDevice, st)) == hipSuccess &&
        (e = hipMemcpyAsync(d_tend, t_end, bt, hipMemcpyHostToDevice, st)) == hipSuccess) {
        auto launch = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(count), dim3(kDpBS), 0, st, d_desc, d_tend, rtol, atol, max_steps, d_stats, o);
        };
        if (model == ND_KURAMOTO)
            dense ? launch(k_ring_dopri<ND_KURAMOTO, true>) : launch(k_ring_dopri_kuramoto);
        else if (model == ND_FHN)
            dense ? launch(k_ring_dopri<ND_FHN, true>) : launch(k_ring_dopri<ND_FHN, false>);
        else
            dense ? launch(k_ring_dopri<ND_KURAMOTO_INERTIA, true>) : launch(k_ring_dopri<ND_KURAMOTO_INERTIA, false>);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h_stats.data(), d_stats, bs, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && dense) e = hipMemcpyAsync(R, o.R, br, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && by) e = hipMemcpyAsync(Y, o.Y, by, hipMemcpyDeviceToHost, st);
    }
    const hipError_t ef = hipFreeAsync(buf, st);
    const hipError_t es = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adaptive run");
    if (ef != hipSuccess) return hip_fail(ef, "adaptive scratch free");
    if (es != hipSuccess) return hip_fail(es, "adaptive run");
    int bad = -1;
    for (int i = 0; i < count; ++i) {
        const double* q = h_stats.data() + kDpStats * i;
        stats[i].t = q[0];
        stats[i].accepted = (int64_t)q[1];
        stats[i].rejected = (int64_t)q[2];
        stats[i].h_next = q[3];
        stats[i].failed = q[4] != 0.0;
        stats[i].reserved = 0;
        if (stats[i].failed && bad < 0) bad = i;
    }
    if (bad >= 0)
        return fail(ND_ERR_NUMERIC, "adaptive run: network %d stopped at t = %.17g (non-finite error estimate or "
                                    "step below its floor)", bad, stats[bad].t);
    return ND_OK;
}

extern "C" nd_status nd_run_adaptive(const nd_handle* hs, int32_t count, const double* t_end, const double* dt0,
                                     double rtol, double atol, int64_t max_steps, nd_adaptive_stats* stats,
                                     void* stream) {
    return run_adaptive(hs, count, t_end, dt0, rtol, atol, max_steps, stats, stream, 0.0, nullptr, 0, nullptr, 0);
}

extern "C" nd_status nd_run_adaptive_dense(const nd_handle* hs, int32_t count, const double* t_end,
                                           const double* dt0, double rtol, double atol, int64_t max_steps,
                                           double t_out, double* R, int64_t r_stride, double* Y, int64_t y_stride,
                                           nd_adaptive_stats* stats, void* stream) {
    if (!(t_out > 0.0)) return fail(ND_ERR_INVALID_ARG, "t_out must be > 0");
    return run_adaptive(hs, count, t_end, dt0, rtol, atol, max_steps, stats, stream, t_out, R, r_stride, Y, y_stride);
}
