// Shared host/device definitions of libnd: the per-network descriptor that every
// kernel reads, and wave/block primitives for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nd.h"

namespace nd {

constexpr int kWave = 64;
constexpr int kCsrSourceBlocks = 8;  // CSR in-edges split by source range, one block per XCD
constexpr int kLinksRows = 256;          // compressed coupling matrix: rows per work item
constexpr int32_t kLinksRemove = 1 << 30;  // entry position flag: the entry removes a link of V

// Per-network descriptor, one per network of a batch, resident in device memory.
// The chunk-position fields (g0, nsteps, ypar) advance on the device at the end
// of every chunk, so a captured chunk graph can be replayed without host writes.
struct NetDesc {
    int64_t n;          // elements
    int64_t P;          // ring radius / cube half-width
    int32_t n1, n2, n3; // cube extents
    int32_t G;          // ring: number of tiles
    int32_t model, prec, obs, tile;
    int32_t cx, cy, cz; // cube: output tile extents per work item (x, y, z)
    int32_t gx, gy;     // cube: tiles along x and y
    int32_t pz;         // ball / disk: z half-width of the neighbourhood (P, or 0 for the disk)
    double dt;
    double dt3, dt6;    // dt/3 and dt/6 (rounded once, on the host)
    double p[12];       // derived model constants (layout per model, see runtime)
    double* y[2];       // state, double-buffered across steps
    double* acc;        // RK accumulator y + dt/6 k1 + dt/3 k2
    void* k[3];         // k1, k2, k3 in the bulk type (double or float)
    double* tsum[2];    // ring: per-tile sums of the mapped stage values, 2 comps
    double* rsum;       // FHN: per-tile sums of the unit phase vectors (u, v)/|(u, v)|
    void* sx[2];        // HH: exchanged synaptic activations S(V) per stage
    const int64_t* row_ptr;  // CSR: per source block b, row offsets at [b*(n+1), (b+1)*(n+1))
    const int32_t* col;      // CSR: sources, block-major, ascending within each row and block
    const void* w;           // CSR: weights in the bulk type, same order
    double* acc_part;        // CSR: per source block synaptic partial sums [blocks][n]
    const double* iapp;
    const int32_t* lrow;     // links: difference-table entry of every row
    const int32_t* ldptr;    // links: entry k's positions at [ldptr[k], ldptr[k+1])
    const int32_t* ldpos;    // links: position, | kLinksRemove when V holds it
    const double* linv;      // links: 1 / link count of the rows of entry k (0: no links)
    const int32_t* lvpos;    // links: positions of the common vector, ascending
    int32_t lnv;             // links: number of positions of the common vector
    double* R;          // order parameter per recorded step
    int64_t r_every;
    double* mv;         // mean phase velocity accumulator / result
    int64_t mv_start;
    double mv_scale;    // 1 / (t_end - t_start)
    int64_t g0;         // run step index at the start of the current chunk
    int64_t nsteps;     // steps still to do at the start of the current chunk
    int32_t ypar;       // which y buffer holds the state at the start of the chunk
    int32_t* status;    // the network's status word: stage 4 stores 1 there when it produces a
                        // non-finite state value (cleared when a new state is set)
};


enum : int32_t { OBS_R = 1, OBS_MV = 2 };

// Buffers reached through the descriptor are generic pointers to the compiler;
// casting them to the global address space gives global (not flat) memory
// instructions, whose completion is tracked apart from LDS traffic.
#define ND_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ ND_GLOBAL T* gp(T* p) {
    return (ND_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const ND_GLOBAL T* gp(const T* p) {
    return (const ND_GLOBAL T*)p;
}

// Flag a non-finite new state value in the network's status word (a plain
// store of 1 from every lane that sees one; the host reads the word back).
__device__ __forceinline__ void flag_nonfinite(const NetDesc& d, double v) {
    if (!__builtin_isfinite(v)) *gp(d.status) = 1;
}

__device__ __forceinline__ int ring_wrap32(int i, int n) {
    // valid for i in [-n, 2n)
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Element access through a uniform base and a 32-bit byte offset (arrays
// below 4 GiB), which maps onto the scalar-base + lane-offset global memory
// forms instead of a 64-bit address per lane.
template <class T>
__device__ __forceinline__ T ld32(const ND_GLOBAL T* base, uint32_t i) {
    return *(const ND_GLOBAL T*)((const ND_GLOBAL char*)base + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st32(ND_GLOBAL T* base, uint32_t i, T v) {
    *(ND_GLOBAL T*)((ND_GLOBAL char*)base + i * (uint32_t)sizeof(T)) = v;
}

__device__ __forceinline__ int64_t ring_wrap(int64_t i, int64_t n) {
    // valid for i in [-n, 2n)
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Work item -> tile mapping that keeps consecutive work items (the tiles of one
// ring) on one XCD: workgroups are dispatched to the 8 XCDs round-robin by id,
// so block b runs on XCD b % 8; XCD x takes the contiguous work range
// [start(x), start(x) + cnt(x)).  A bijection on [0, nwork) when the number of
// virtual blocks is nwork.
__device__ __forceinline__ int xcd_work(int vb, int nwork) {
    const int x = vb & 7, s = vb >> 3;
    const int q = nwork >> 3, r = nwork & 7;
    const int cnt = q + (x < r ? 1 : 0);
    return s < cnt ? x * q + min(x, r) + s : -1;
}

// Barrier for exchanges through LDS only: waits for this wave's LDS traffic
// but lets outstanding global loads stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- wave/block
// All reductions below use a fixed combination tree, so every lane and every
// launch produces bitwise identical sums for identical inputs.
// Cross-lane moves of a double through DPP (data-parallel primitives): each half
// is moved with the same control; lanes whose source is outside the pattern,
// or whose row / bank is masked off, receive 0.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, BANK_MASK, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, BANK_MASK, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive scan over the 64 lanes: shifts of 1, 2, 4, 8 inside each row of 16
// lanes, then the row totals are carried by the row broadcasts of lanes 15 and
// 31.  A fixed combination tree, so the result is deterministic.
__device__ __forceinline__ double wave_incl_scan(double x) {
    x += dpp_move<0x111>(x);          // row_shr:1
    x += dpp_move<0x112>(x);          // row_shr:2
    x += dpp_move<0x114>(x);          // row_shr:4
    x += dpp_move<0x118>(x);          // row_shr:8
    x += dpp_move<0x142, 0xa>(x);     // row_bcast:15 into rows 1 and 3
    x += dpp_move<0x143, 0xc>(x);     // row_bcast:31 into rows 2 and 3
    return x;
}

// Exclusive value of an inclusive scan: the previous lane's value (lane 0: 0).
__device__ __forceinline__ double wave_shift_up1(double x) { return dpp_move<0x138>(x); }  // wave_shr:1

__device__ __forceinline__ double wave_bcast(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave, identical in every lane (the scan's last lane, broadcast).
__device__ __forceinline__ double wave_sum(double x) { return wave_bcast(wave_incl_scan(x), kWave - 1); }

// Sum NV values over the block (result in every thread). lds: NV * (BS/64) doubles.
template <int BS, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
    constexpr int NW = BS / kWave;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[q * NW + wid] = v[q];
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += lds[q * NW + w];
        v[q] = s;
    }
    lds_barrier();
}

// One pass over LDS that returns, in every thread, the block sums of NR values
// and the block-exclusive prefix of NS values (thread order).
// lds: (NR + NS) * (BS/64) doubles.
template <int BS, int NR, int NS>
__device__ __forceinline__ void block_sum_and_exscan(double (&r)[NR], double (&s)[NS], double* lds) {
    constexpr int NW = BS / kWave;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int q = 0; q < NR; ++q) r[q] = wave_sum(r[q]);
    double incl[NS], excl[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        incl[q] = wave_incl_scan(s[q]);
        excl[q] = wave_shift_up1(incl[q]);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NR; ++q) lds[q * NW + wid] = r[q];
    }
    if (lane == kWave - 1) {
#pragma unroll
        for (int q = 0; q < NS; ++q) lds[(NR + q) * NW + wid] = incl[q];
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) a += lds[q * NW + w];
        r[q] = a;
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double a = 0.0;
        for (int w = 0; w < wid; ++w) a += lds[(NR + q) * NW + w];
        s[q] = a + excl[q];
    }
    lds_barrier();
}

// Block-exclusive prefix (thread order) of NS values, in every thread: the scan
// half of block_sum_and_exscan, for callers with no block sums to take along.
// lds: NS * (BS/64) doubles.
template <int BS, int NS>
__device__ __forceinline__ void block_exscan(double (&s)[NS], double* lds) {
    constexpr int NW = BS / kWave;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    double incl[NS], excl[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        incl[q] = wave_incl_scan(s[q]);
        excl[q] = wave_shift_up1(incl[q]);
    }
    if (lane == kWave - 1) {
#pragma unroll
        for (int q = 0; q < NS; ++q) lds[q * NW + wid] = incl[q];
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double a = 0.0;
        for (int w = 0; w < wid; ++w) a += lds[q * NW + w];
        s[q] = a + excl[q];
    }
    lds_barrier();
}

}  // namespace nd
