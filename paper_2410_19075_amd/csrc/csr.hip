// Hodgkin-Huxley neurons coupled through a sparse directed graph (CSR by
// target), stage kernels for gfx950.
//
// Eq. (1) of the paper specialised to the squid axon (Na, K and leak currents
// with the textbook rate functions) and an instantaneous sigmoidal synapse:
//   C dV_i/dt = I_i - gNa m^3 h (V-ENa) - gK n^4 (V-EK) - gL (V-EL)
//               + (Esyn - V_i) sum_{e in in(i)} w_e S(V_src(e))
//   dx/dt = alpha_x(V) (1 - x) - beta_x(V) x,   x in {m, h, n}
// The coupling matrix L_ik of Eq. (1) with weights is the CSR graph.
//
// Per stage the activations s_j = S(V_j) of the stage values are computed
// once per neuron by the previous stage (the exchanged quantity), and each
// work item (256 target rows) does:
//   phase A: the in-edges are split into 8 source blocks (one per XCD); per
//            (row tile, block) the tile's edges are streamed coalesced, the
//            products w_e s_src(e) are formed in double and every row's
//            products are added in edge order, giving one partial per block;
//   phase B: one thread per neuron adds the 8 partials in block order,
//            evaluates the HH right-hand side, does the 13-access RK
//            bookkeeping and writes S of its next stage value.
#include "models.h"
#include "runtime.h"

namespace nd {

constexpr int kCsrRows = 256;
constexpr int kSrcBlocks = kCsrSourceBlocks;  // source blocks, one per XCD

// x / (1 - exp(-x)) with the removable singularity at 0 taken by its series
template <class T>
__device__ __forceinline__ T xoverexpm1(T x) {
    if (fabs(x) < (T)1e-7) return (T)1 + (T)0.5 * x;
    return x / (-expm1(-x));
}

// HH right-hand side of one neuron; z = (V, m, h, n), G = synaptic sum.
// p = {C, gNa, gK, gL, ENa, EK, EL, Esyn, theta_s, k_s}
template <class T>
__device__ __forceinline__ void hh_rhs(const double* p, double Iapp, const double* z, double G, double* k) {
    const T v = (T)z[0], mm = (T)z[1], hh = (T)z[2], nn = (T)z[3];
    const T am = xoverexpm1<T>((v + (T)40) / (T)10);
    const T bm = (T)4 * exp(-(v + (T)65) / (T)18);
    const T ah = (T)0.07 * exp(-(v + (T)65) / (T)20);
    const T bh = (T)1 / ((T)1 + exp(-(v + (T)35) / (T)10));
    const T an = (T)0.1 * xoverexpm1<T>((v + (T)55) / (T)10);
    const T bn = (T)0.125 * exp(-(v + (T)65) / (T)80);
    const T iion = (T)p[1] * mm * mm * mm * hh * (v - (T)p[4]) + (T)p[2] * nn * nn * nn * nn * (v - (T)p[5]) +
                   (T)p[3] * (v - (T)p[6]);
    // the synaptic current uses the double sum G
    k[0] = (double)(((T)Iapp - iion) + (T)(((double)p[7] - z[0]) * G)) / p[0];
    k[1] = (double)(am * ((T)1 - mm) - bm * mm);
    k[2] = (double)(ah * ((T)1 - hh) - bh * hh);
    k[3] = (double)(an * ((T)1 - nn) - bn * nn);
}

template <class T>
__device__ __forceinline__ T synapse(const double* p, double V) {
    return (T)1 / ((T)1 + exp(-((T)V - (T)p[8]) / (T)p[9]));
}

// Activations of the run's initial state (networks with g0 == 0).
template <class KT>
__global__ __launch_bounds__(256) void k_csr_prologue(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                     const int* __restrict__ nwork_p) {
    const int nwork = *nwork_p;
    // one row tile per workgroup: the tile's work items are 8 consecutive
    // entries starting at a multiple of 8; spreading the tiles over the
    // workgroups (rather than taking every 8th workgroup) keeps all XCDs busy
    for (int v = blockIdx.x; v < nwork / kSrcBlocks; v += gridDim.x) {
        const int2 wk = work[v * kSrcBlocks];
        const NetDesc& d = D[wk.x];
        if (d.g0 != 0 || d.nsteps <= 0) continue;
        const int64_t i = (int64_t)(wk.y / kSrcBlocks) * kCsrRows + threadIdx.x;
        if (i < d.n) gp((KT*)d.sx[0])[i] = (KT)synapse<KT>(d.p, gp(d.y[d.ypar])[i]);
    }
}

// Phase A: synaptic partial sums of one source block for 256 target rows.
// Work item (row tile t, block x) is entry 8t + x; with the work map aligned
// to multiples of 8 and the grid a multiple of 8, block x always lands on XCD x
// (workgroups go to the XCDs round-robin), whose L2 then holds that block's
// slice of the activations.
// The tile's in-edges of block x are one contiguous range of the block-major
// edge arrays.  It is streamed in chunks of 256*U edges: every thread loads U
// edges (coalesced col and w, then the U gathers, all in flight together) and
// leaves the products in LDS; then the owner thread of each row adds its
// row's products in ascending edge order.  The sum of a row therefore does not
// depend on U or on the chunking.
template <class KT, int U>
__global__ __launch_bounds__(256) void k_csr_gather(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                   const int* __restrict__ nwork_p, int stage, int j) {
    constexpr int BS = 256, CH = BS * U;
    __shared__ double prod[CH];
    __shared__ int64_t rb[kCsrRows + 1];
    const int nwork = *nwork_p;
    const int tid = threadIdx.x;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;  // uniform over the block
        const int64_t n = d.n;
        const int x = wk.y % kSrcBlocks;
        const int64_t r0 = (int64_t)(wk.y / kSrcBlocks) * kCsrRows;
        const int nrows = (int)min((int64_t)kCsrRows, n - r0);
        const ND_GLOBAL int64_t* __restrict__ bp = gp(d.row_ptr) + (int64_t)x * (n + 1) + r0;
        const ND_GLOBAL int32_t* __restrict__ col = gp(d.col);
        const ND_GLOBAL KT* __restrict__ wt = gp((const KT*)d.w);
        const ND_GLOBAL KT* __restrict__ sin_ = gp((const KT*)d.sx[(stage - 1) & 1]);
        if (tid <= nrows) rb[tid] = bp[tid];
        if (tid == 0 && nrows == BS) rb[BS] = bp[BS];
        __syncthreads();
        const int64_t E0 = rb[0], E1 = rb[nrows];
        const int64_t mb = tid < nrows ? rb[tid] : E1, me = tid < nrows ? rb[tid + 1] : E1;
        double a = 0.0;
        for (int64_t c0 = E0; c0 < E1; c0 += CH) {
            int c[U];
            double wv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = c0 + u * BS + tid;
                const bool ok = q < E1;
                c[u] = col[ok ? q : E0];
                wv[u] = ok ? (double)wt[q] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) prod[u * BS + tid] = wv[u] * (double)sin_[c[u]];
            __syncthreads();
            const int64_t lo = max(mb, c0), hi = min(me, c0 + CH);
            for (int64_t q = lo; q < hi; ++q) a += prod[q - c0];
            __syncthreads();
        }
        if (tid < nrows) gp(d.acc_part)[(int64_t)x * n + r0 + tid] = a;
    }
}

// Phase B: one thread per neuron sums the source-block partials (fixed order),
// evaluates the HH right-hand side, does the 13-access RK bookkeeping and
// writes S of its next stage value.
template <class KT, int STAGE>
__global__ __launch_bounds__(256) void k_csr_update(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                   const int* __restrict__ nwork_p, int j) {
    constexpr int stage = STAGE;
    const int nwork = *nwork_p;
    const int tid = threadIdx.x;
    for (int v = blockIdx.x; v < nwork / kSrcBlocks; v += gridDim.x) {  // one row tile per workgroup
        const int2 wk = work[v * kSrcBlocks];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;
        const int64_t n = d.n;
        const int64_t i = (int64_t)(wk.y / kSrcBlocks) * kCsrRows + tid;
        if (i >= n) continue;
        const int par = (d.ypar + j) & 1;
        const ND_GLOBAL double* __restrict__ y = gp(d.y[par]);
        const ND_GLOBAL KT* __restrict__ kp =
            stage == 1 ? nullptr : gp((const KT*)d.k[stage > 1 ? stage - 2 : 0]);
        const ND_GLOBAL double* __restrict__ part = gp(d.acc_part);
        const double dt = d.dt;
        const double cdt = stage == 4 ? dt : 0.5 * dt;
        double G = 0.0;
#pragma unroll
        for (int x = 0; x < kSrcBlocks; ++x) G += part[(int64_t)x * n + i];
        double z[4], yv[4], kv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t q = v * n + i;
            yv[v] = y[q];
            if (stage != 1) kv[v] = (double)kp[q];
            z[v] = stage == 1 ? yv[v] : fma(cdt, kv[v], yv[v]);
        }
        double k[4];
        if constexpr (sizeof(KT) == 8)
            hh_rhs<double>(d.p, gp(d.iapp)[i], z, G, k);
        else
            hh_rhs<float>(d.p, gp(d.iapp)[i], z, G, k);
        double zn[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t q = v * n + i;
            const double kk = kq<KT>(k[v]);
            if (stage == 1) {
                gp((KT*)d.k[0])[q] = (KT)kk;
                zn[v] = fma(0.5 * dt, kk, yv[v]);
            } else if (stage == 2) {
                gp((KT*)d.k[1])[q] = (KT)kk;
                gp(d.acc)[q] = fma(d.dt3, kk, fma(d.dt6, kv[v], yv[v]));
                zn[v] = fma(0.5 * dt, kk, yv[v]);
            } else if (stage == 3) {
                gp((KT*)d.k[2])[q] = (KT)kk;
                zn[v] = fma(dt, kk, yv[v]);
            } else {
                const double yo = fma(d.dt6, kk, fma(d.dt3, kv[v], gp(d.acc)[q]));
                gp(d.y[par ^ 1])[q] = yo;
                flag_nonfinite(d, yo);
                zn[v] = yo;
            }
        }
        gp((KT*)d.sx[stage & 1])[i] = (KT)synapse<KT>(d.p, zn[0]);
    }
}

// ------------------------------------------------------------------ launch
template <class KT, int U>
static void csr_entry_l(CsrLaunch* r) {
    r->gather = k_csr_gather<KT, U>;
    r->update[0] = k_csr_update<KT, 1>;
    r->update[1] = k_csr_update<KT, 2>;
    r->update[2] = k_csr_update<KT, 3>;
    r->update[3] = k_csr_update<KT, 4>;
    r->prologue = k_csr_prologue<KT>;
}

template <class KT>
static bool csr_entry(int ept, CsrLaunch* r) {
    switch (ept) {
        case 2: csr_entry_l<KT, 2>(r); return true;
        case 4: csr_entry_l<KT, 4>(r); return true;
        case 8: csr_entry_l<KT, 8>(r); return true;
        case 16: csr_entry_l<KT, 16>(r); return true;
        default: return false;
    }
}

bool csr_select(int prec, int ept, CsrLaunch* out) {
    return prec == ND_FP64 ? csr_entry<double>(ept, out) : csr_entry<float>(ept, out);
}

hipError_t csr_launch_prologue(const CsrLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                               const int* nwork) {
    hipLaunchKernelGGL(L.prologue, dim3((grid + kSrcBlocks - 1) / kSrcBlocks), dim3(256), 0, s, D, work, nwork);
    return hipGetLastError();
}

hipError_t csr_launch_stage(const CsrLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                            const int* nwork, int stage, int j) {
    hipLaunchKernelGGL(L.gather, dim3(grid), dim3(256), 0, s, D, work, nwork, stage, j);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(L.update[stage - 1], dim3((grid + kSrcBlocks - 1) / kSrcBlocks), dim3(256), 0, s, D, work, nwork,
                       j);
    return hipGetLastError();
}

}  // namespace nd
