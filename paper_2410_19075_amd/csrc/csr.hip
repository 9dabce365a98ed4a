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
//   phase A: groups of L lanes walk the in-edges of one row each, accumulate
//            w_e s_src(e) in double, reduce within the group (fixed tree),
//            row sums to LDS;
//   phase B: one thread per neuron evaluates the HH right-hand side, does the
//            13-access RK bookkeeping and writes S of its next stage value.
#include "models.h"
#include "runtime.h"

namespace nd {

constexpr int kCsrRows = 256;

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
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (d.g0 != 0 || d.nsteps <= 0) continue;
        const int64_t i = (int64_t)wk.y * kCsrRows + threadIdx.x;
        if (i < d.n) gp((KT*)d.sx[0])[i] = (KT)synapse<KT>(d.p, gp(d.y[d.ypar])[i]);
    }
}

template <class KT, int STAGE, int L>
__global__ __launch_bounds__(256) void k_csr_stage(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                  const int* __restrict__ nwork_p, int j) {
    constexpr int stage = STAGE;
    constexpr int BS = 256;
    __shared__ double gsum[kCsrRows];
    const int nwork = *nwork_p;
    const int nvb = ((nwork + 7) >> 3) << 3;
    const int tid = threadIdx.x;
    const int lane = tid & (L - 1), grp = tid / L;
    constexpr int NG = BS / L;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int wi = xcd_work(vb, nwork);
        if (wi < 0) continue;
        const int2 wk = work[wi];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;
        const int64_t n = d.n;
        const int64_t r0 = (int64_t)wk.y * kCsrRows;
        const int nrows = (int)min((int64_t)kCsrRows, n - r0);
        const int par = (d.ypar + j) & 1;
        const ND_GLOBAL double* __restrict__ y = gp(d.y[par]);
        const ND_GLOBAL KT* __restrict__ kp =
            stage == 1 ? nullptr : gp((const KT*)d.k[stage > 1 ? stage - 2 : 0]);
        const ND_GLOBAL KT* __restrict__ sin_ = gp((const KT*)d.sx[(stage - 1) & 1]);
        ND_GLOBAL KT* __restrict__ sout = gp((KT*)d.sx[stage & 1]);
        const ND_GLOBAL int64_t* __restrict__ rp = gp(d.row_ptr);
        const ND_GLOBAL int32_t* __restrict__ col = gp(d.col);
        const ND_GLOBAL KT* __restrict__ wt = gp((const KT*)d.w);
        const ND_GLOBAL double* __restrict__ accp = gp(d.acc);
        const double dt = d.dt;
        const double cdt = stage == 4 ? dt : 0.5 * dt;

        // ---- phase A: synaptic sums, L lanes per row
        for (int r = grp; r < nrows; r += NG) {
            const int64_t b = rp[r0 + r], e = rp[r0 + r + 1];
            double a = 0.0;
            // four independent gathers in flight per lane: the column and weight
            // loads of a group of 4L edges are issued first (clamped indices,
            // zero weight past the row end), then the activations they select
            for (int64_t q0 = b + lane; q0 < e; q0 += 4 * L) {
                int c[4];
                double wv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t q = q0 + u * L;
                    const bool ok = q < e;
                    const int64_t qq = ok ? q : q0;
                    c[u] = col[qq];
                    wv[u] = ok ? (double)wt[qq] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) a += wv[u] * (double)sin_[c[u]];
            }
#pragma unroll
            for (int o = L / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, kWave);
            if (lane == 0) gsum[r] = a;
        }
        __syncthreads();

        // ---- phase B: one neuron per thread
        if (tid < nrows) {
            const int64_t i = r0 + tid;
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
                hh_rhs<double>(d.p, gp(d.iapp)[i], z, gsum[tid], k);
            else
                hh_rhs<float>(d.p, gp(d.iapp)[i], z, gsum[tid], k);
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
                    gp(d.acc)[q] = fma(dt / 3.0, kk, fma(dt / 6.0, kv[v], yv[v]));
                    zn[v] = fma(0.5 * dt, kk, yv[v]);
                } else if (stage == 3) {
                    gp((KT*)d.k[2])[q] = (KT)kk;
                    zn[v] = fma(dt, kk, yv[v]);
                } else {
                    const double yo = fma(dt / 6.0, kk, fma(dt / 3.0, kv[v], accp[q]));
                    gp(d.y[par ^ 1])[q] = yo;
                    zn[v] = yo;
                }
            }
            sout[i] = (KT)synapse<KT>(d.p, zn[0]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launch
template <class KT, int L>
static void csr_entry_l(CsrLaunch* r) {
    r->stage[0] = k_csr_stage<KT, 1, L>;
    r->stage[1] = k_csr_stage<KT, 2, L>;
    r->stage[2] = k_csr_stage<KT, 3, L>;
    r->stage[3] = k_csr_stage<KT, 4, L>;
    r->prologue = k_csr_prologue<KT>;
}

template <class KT>
static bool csr_entry(int lanes, CsrLaunch* r) {
    switch (lanes) {
        case 4: csr_entry_l<KT, 4>(r); return true;
        case 8: csr_entry_l<KT, 8>(r); return true;
        case 16: csr_entry_l<KT, 16>(r); return true;
        case 32: csr_entry_l<KT, 32>(r); return true;
        case 64: csr_entry_l<KT, 64>(r); return true;
        default: return false;
    }
}

bool csr_select(int prec, int lanes, CsrLaunch* out) {
    return prec == ND_FP64 ? csr_entry<double>(lanes, out) : csr_entry<float>(lanes, out);
}

hipError_t csr_launch_prologue(const CsrLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                               const int* nwork) {
    hipLaunchKernelGGL(L.prologue, dim3(grid), dim3(256), 0, s, D, work, nwork);
    return hipGetLastError();
}

hipError_t csr_launch_stage(const CsrLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                            const int* nwork, int stage, int j) {
    hipLaunchKernelGGL(L.stage[stage - 1], dim3(grid), dim3(256), 0, s, D, work, nwork, j);
    return hipGetLastError();
}

}  // namespace nd
