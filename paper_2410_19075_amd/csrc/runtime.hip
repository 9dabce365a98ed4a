// Host runtime of libnd: argument validation, device buffers, batched launch
// sequences and the C ABI declared in include/nd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "nd_dev.h"
#include "runtime.h"

namespace nd {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

nd_status fail(nd_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

nd_status hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return fail(ND_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
    return fail(ND_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPC(expr)                                        \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

// ------------------------------------------------------------ validation
int nvars_of(int model) { return model == ND_KURAMOTO ? 1 : (model == ND_HH ? 4 : 2); }

static bool finite_all(const double* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

nd_status validate_problem(const nd_problem* p) {
    if (!p) return fail(ND_ERR_INVALID_ARG, "problem is NULL");
    if (p->reserved != 0) return fail(ND_ERR_INVALID_ARG, "reserved field must be 0");
    if (p->precision != ND_FP64 && p->precision != ND_FP32_BULK)
        return fail(ND_ERR_INVALID_ARG, "unknown precision %d", p->precision);
    if (p->n < 1) return fail(ND_ERR_INVALID_ARG, "n must be >= 1 (got %lld)", (long long)p->n);
    if (p->n > (int64_t(1) << 31) - 1) return fail(ND_ERR_INVALID_ARG, "n must be < 2^31");
    if (p->model < 0 || p->model > 3) return fail(ND_ERR_INVALID_ARG, "unknown model %d", p->model);
    const int np = p->model == ND_KURAMOTO ? 3 : (p->model == ND_FHN ? 4 : (p->model == ND_HH ? 10 : 5));
    if (!finite_all(p->params, np)) return fail(ND_ERR_INVALID_ARG, "model parameters must be finite");
    if (p->model == ND_FHN && p->params[0] == 0.0) return fail(ND_ERR_INVALID_ARG, "FHN eps must be non-zero");
    if (p->model == ND_KURAMOTO_INERTIA && p->params[3] == 0.0)
        return fail(ND_ERR_INVALID_ARG, "the mass m must be non-zero (m = 0 is ND_KURAMOTO)");
    if (p->model == ND_HH && (p->params[0] == 0.0 || p->params[9] == 0.0))
        return fail(ND_ERR_INVALID_ARG, "HH C and k_s must be non-zero");
    switch (p->topo) {
        case ND_RING:
            if (p->model == ND_HH) return fail(ND_ERR_INVALID_ARG, "HH needs the CSR topology");
            if (p->radius < 1 || 2 * p->radius + 1 > p->n)
                return fail(ND_ERR_INVALID_ARG, "ring radius P must satisfy 1 <= P and 2P+1 <= n (n=%lld, P=%lld)",
                            (long long)p->n, (long long)p->radius);
            if (p->n >= (int64_t(1) << 29))
                return fail(ND_ERR_INVALID_ARG, "ring networks hold at most 2^29 - 1 elements (n=%lld)", (long long)p->n);
            break;
        case ND_CUBE3D: {
            if (p->model != ND_KURAMOTO && p->model != ND_KURAMOTO_INERTIA)
                return fail(ND_ERR_INVALID_ARG, "the cube topology is for the Kuramoto models");
            const int64_t side = 2 * p->radius + 1;
            if (p->radius < 1 || p->n1 < side || p->n2 < side || p->n3 < side)
                return fail(ND_ERR_INVALID_ARG, "cube extents must be >= 2h+1");
            if (p->n1 * p->n2 * p->n3 != p->n) return fail(ND_ERR_INVALID_ARG, "n must equal n1*n2*n3");
            if (p->n >= (int64_t(1) << 29))
                return fail(ND_ERR_INVALID_ARG, "lattices hold at most 2^29 - 1 elements (n=%lld)", (long long)p->n);
            break;
        }
        case ND_BALL3D: {
            if (p->model != ND_KURAMOTO && p->model != ND_KURAMOTO_INERTIA)
                return fail(ND_ERR_INVALID_ARG, "the ball topology is for the Kuramoto models");
            const int64_t side = 2 * p->radius + 1;
            if (p->radius < 1 || p->radius > kBallMaxP)
                return fail(ND_ERR_INVALID_ARG, "ball radius must be in [1, %d]", kBallMaxP);
            if (p->n1 < side || p->n2 < side || p->n3 < side)
                return fail(ND_ERR_INVALID_ARG, "lattice extents must be >= 2P+1");
            if (p->n1 * p->n2 * p->n3 != p->n) return fail(ND_ERR_INVALID_ARG, "n must equal n1*n2*n3");
            if (p->n >= (int64_t(1) << 29))
                return fail(ND_ERR_INVALID_ARG, "lattices hold at most 2^29 - 1 elements (n=%lld)", (long long)p->n);
            break;
        }
        case ND_DISK2D: {
            if (p->model != ND_KURAMOTO && p->model != ND_KURAMOTO_INERTIA)
                return fail(ND_ERR_INVALID_ARG, "the disk topology is for the Kuramoto models");
            const int64_t side = 2 * p->radius + 1;
            if (p->radius < 1 || p->radius > kBallMaxP)
                return fail(ND_ERR_INVALID_ARG, "disk radius must be in [1, %d]", kBallMaxP);
            if (p->n1 < side || p->n2 < side || p->n3 != 1)
                return fail(ND_ERR_INVALID_ARG, "the disk needs n1, n2 >= 2P+1 and n3 = 1");
            if (p->n1 * p->n2 != p->n) return fail(ND_ERR_INVALID_ARG, "n must equal n1*n2");
            if (p->n >= (int64_t(1) << 29))
                return fail(ND_ERR_INVALID_ARG, "lattices hold at most 2^29 - 1 elements (n=%lld)", (long long)p->n);
            break;
        }
        case ND_LINKS: {
            if (p->model == ND_HH) return fail(ND_ERR_INVALID_ARG, "HH needs the CSR topology (weighted links)");
            if (!p->row_ptr || (p->nnz > 0 && !p->col))
                return fail(ND_ERR_INVALID_ARG, "the links topology needs row_ptr and col");
            if (p->row_ptr[0] != 0 || p->row_ptr[p->n] != p->nnz)
                return fail(ND_ERR_INVALID_ARG, "row_ptr must start at 0 and end at nnz");
            if (p->n >= (int64_t(1) << 29))
                return fail(ND_ERR_INVALID_ARG, "link matrices hold at most 2^29 - 1 elements (n=%lld)", (long long)p->n);
            // row order and ranges are checked while compressing
            break;
        }
        case ND_CSR: {
            if (p->model != ND_HH) return fail(ND_ERR_INVALID_ARG, "the CSR topology is for HH");
            if (!p->row_ptr || (p->nnz > 0 && (!p->col || !p->weight)) || !p->per_elem)
                return fail(ND_ERR_INVALID_ARG, "CSR needs row_ptr, col, weight and per_elem");
            if (p->row_ptr[0] != 0 || p->row_ptr[p->n] != p->nnz)
                return fail(ND_ERR_INVALID_ARG, "row_ptr must start at 0 and end at nnz");
            for (int64_t i = 0; i < p->n; ++i)
                if (p->row_ptr[i + 1] < p->row_ptr[i]) return fail(ND_ERR_INVALID_ARG, "row_ptr must be non-decreasing");
            for (int64_t e = 0; e < p->nnz; ++e)
                if (p->col[e] < 0 || p->col[e] >= p->n) return fail(ND_ERR_INVALID_ARG, "col[%lld] out of range", (long long)e);
            if (!finite_all(p->weight, (int)std::min<int64_t>(p->nnz, INT32_MAX)))
                return fail(ND_ERR_INVALID_ARG, "weights must be finite");
            if (!finite_all(p->per_elem, (int)p->n)) return fail(ND_ERR_INVALID_ARG, "per_elem must be finite");
            break;
        }
        default:
            return fail(ND_ERR_INVALID_ARG, "unknown topology %d", p->topo);
    }
    return ND_OK;
}

// Lattice points within distance P of the origin, the origin included.
int64_t disk_points(int64_t P) {
    int64_t c = 0;
    for (int64_t dy = -P; dy <= P; ++dy)
        for (int64_t dx = -P; dx <= P; ++dx) c += dx * dx + dy * dy <= P * P;
    return c;
}

int64_t ball_points(int64_t P) {
    int64_t c = 0;
    for (int64_t dz = -P; dz <= P; ++dz)
        for (int64_t dy = -P; dy <= P; ++dy)
            for (int64_t dx = -P; dx <= P; ++dx) c += dx * dx + dy * dy + dz * dz <= P * P;
    return c;
}

// (dy, dz) runs of the ball of radius P, padded to the kernel's unroll of 8.
static int ball_runs(int P, int pz) {
    int c = 0;
    for (int dz = -pz; dz <= pz; ++dz)
        for (int dy = -P; dy <= P; ++dy) c += dz * dz + dy * dy <= P * P;
    return (c + 7) / 8 * 8;
}

// Ball tiling and workgroup size.  Halo rows of HX = cx + 2P <= 64 lanes, at
// most 4 rows per wave and one output per thread, the prefix ring within the
// LDS budget.  A 256-thread workgroup leaves room for up to 4 per CU (LDS
// permitting), a 1024-thread one holds the CU alone.  The estimated time is
// (rounds of workgroups over the CU slots) x (planes per work item incl. the
// 2P lead-in) x (halo rows per wave + the outputs' prefix reads / 10).
// Plane-scatter form: 512-thread workgroups, two per CU where the radius is
// built for it and the two prefix planes fit twice in LDS.  Per plane every wave
// maps up to 4 halo rows (~720 clocks of issue per row and SIMD), then the
// outputs read two prefix values per (|dz|, dy) run pair: the larger of the
// pairs' VALU issue (~48 clocks per pair and SIMD) and their LDS traffic (cx*cy
// outputs x 32 bytes per pair at 128 bytes per clock).  Work items pay the 2P
// lead-in planes in mapping only; a CU running two work items at once is
// counted at 0.8 of running them one after the other (measured at P = 6).
// The default for radii from kBallScatterMinP (at smaller radii the gather
// form measured faster).
constexpr int kBallScatterMinP = 3;
static bool ball_tiles_scatter(const nd_problem* p, int cus, int* cx_, int* cy_, int* cz_) {
    const int P = (int)p->radius;
    if (p->topo != ND_BALL3D || !ball_scatter_available(P) || P < kBallScatterMinP) return false;
    const int n1 = (int)p->n1, n2 = (int)p->n2, n3 = (int)p->n3;
    const int waves = kBallScatterBlock / 64;
    int pairs = 0;  // runs of dz >= 0 (those of -dz share their reads)
    for (int dz = 0; dz <= P; ++dz)
        for (int dy = -P; dy <= P; ++dy) pairs += dz * dz + dy * dy <= P * P;
    double best = 1e300;
    bool found = false;
    for (int cx = 1; cx <= std::min(n1, 64 - 2 * P); ++cx) {
        for (int cy = 1; cy <= std::min(n2, 4 * waves - 2 * P); ++cy) {
            if (cx * cy > kBallScatterBlock) break;
            const size_t sm = ball_scatter_smem_bytes(P, cx, cy);
            if (sm > kBallSmemMax) break;
            const int per_cu = P <= kBallScatterPairedMaxP && 2 * sm <= kBallSmemMax ? 2 : 1;
            const double overlap = per_cu == 2 ? 0.8 : 1.0;
            const int64_t tiles = (int64_t)((n1 + cx - 1) / cx) * ((n2 + cy - 1) / cy);
            const double map = 720.0 * ((cy + 2 * P + waves - 1) / waves);
            const double sums = std::max(48.0 * pairs, (double)cx * cy * pairs * 32.0 / 128.0);
            for (int zt = 1; zt <= std::min(n3, 256); ++zt) {
                const int cz = (n3 + zt - 1) / zt;
                if (zt > 1 && (n3 + cz - 1) / cz != zt) continue;
                const int64_t rounds = (tiles * zt + (int64_t)cus * per_cu - 1) / ((int64_t)cus * per_cu);
                const double cost =
                    (double)rounds * per_cu * overlap * ((cz + 2 * P) * map + cz * sums) - 1e-6 * cx * cy;
                if (cost < best) {
                    best = cost;
                    found = true;
                    *cx_ = cx, *cy_ = cy, *cz_ = cz;
                }
            }
        }
    }
    return found;
}

static void ball_tiles_gather(const nd_problem* p, int cus, int* cx_, int* cy_, int* cz_, int* bs_) {
    const int P = (int)p->radius, pz = ball_pz(p->topo, p->radius);
    const int n1 = (int)p->n1, n2 = (int)p->n2, n3 = (int)p->n3;
    const double reads = 0.1 * ball_runs(P, pz);
    double best = 1e300;
    *cx_ = 1, *cy_ = 1, *cz_ = n3, *bs_ = 1024;
    for (int bs : {256, 1024}) {
        const int waves = bs / 64;
        for (int cx = 1; cx <= std::min(n1, 64 - 2 * P); ++cx) {
            for (int cy = 1; cy <= std::min(n2, 4 * waves - 2 * P); ++cy) {
                if (cx * cy > bs) break;
                const size_t sm = ball_smem_bytes(P, pz, cx, cy);
                if (sm > kBallSmemMax) break;
                const int per_cu = bs == 1024 ? 1 : std::max(1, std::min<int>(4, (int)(kBallSmemMax / sm)));
                const int64_t tiles = (int64_t)((n1 + cx - 1) / cx) * ((n2 + cy - 1) / cy);
                const double plane_cost = (double)((cy + 2 * P + waves - 1) / waves) + reads;
                for (int zt = 1; zt <= std::min(n3, 256); ++zt) {
                    const int cz = (n3 + zt - 1) / zt;
                    if (zt > 1 && (n3 + cz - 1) / cz != zt) continue;
                    const int64_t rounds = (tiles * zt + (int64_t)cus * per_cu - 1) / ((int64_t)cus * per_cu);
                    const double cost = (double)rounds * (cz + 2 * pz) * plane_cost - 1e-6 * cx * cy;
                    if (cost < best) {
                        best = cost;
                        *cx_ = cx, *cy_ = cy, *cz_ = cz, *bs_ = bs;
                    }
                }
            }
        }
    }
}

static void ball_tiles(const nd_problem* p, int cus, int* cx_, int* cy_, int* cz_, int* bs_) {
    if (ball_tiles_scatter(p, cus, cx_, cy_, cz_)) {
        *bs_ = kBallScatterBlock;
        return;
    }
    ball_tiles_gather(p, cus, cx_, cy_, cz_, bs_);
}

nd_kernel_config ball_gather_config(const nd_problem* p) {
    nd_kernel_config c = default_config(p);
    int cx, cy, cz, bs;
    ball_tiles_gather(p, device_cu_count(), &cx, &cy, &cz, &bs);
    c.tile = cx;
    c.tile_y = cy;
    c.tile_z = cz;
    c.block = bs;
    return c;
}

// ------------------------------------------------------------ configuration
// Compute units of the current device (256 on MI355X; also the answer when no
// device can be queried, e.g. for footprint estimates on a host without GPU).
int device_cu_count() {
    static const int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
            (void)hipGetLastError();
            return 256;
        }
        return n;
    }();
    return cus;
}

// Cube tiling.  One workgroup of (cx+2h)(cy+2h) column threads holds a CU, and
// the time of a stage is about (rounds of workgroups over the CUs) x (planes
// per work item, including the 2h lead-in) x (threads per workgroup), so the
// tiling minimising that product is taken (ties: fewer halo columns, then
// wider x for coalescing).
static void cube_tiles(const nd_problem* p, int cus, int* cx_, int* cy_, int* cz_) {
    const int h = (int)p->radius;
    const int n1 = (int)p->n1, n2 = (int)p->n2, n3 = (int)p->n3;
    double best = 1e300;
    *cx_ = 1, *cy_ = 1, *cz_ = n3;
    for (int cx = 1; cx <= std::min(n1, 64); ++cx) {
        for (int cy = 1; cy <= std::min(n2, 64); ++cy) {
            const int halo = (cx + 2 * h) * (cy + 2 * h);
            if (halo > 1024) break;
            const int64_t threads = (halo + 63) / 64 * 64;
            const int64_t tiles = (int64_t)((n1 + cx - 1) / cx) * ((n2 + cy - 1) / cy);
            for (int zt = 1; zt <= std::min(n3, 256); ++zt) {
                const int cz = (n3 + zt - 1) / zt;
                if (zt > 1 && (n3 + cz - 1) / cz != zt) continue;  // same split as a smaller zt
                const int64_t G = tiles * zt;
                const int64_t rounds = (G + cus - 1) / cus;
                const double cost = (double)rounds * (cz + 2 * h) * threads + 1e-2 * halo - 1e-4 * cx;
                if (cost < best) {
                    best = cost;
                    *cx_ = cx, *cy_ = cy, *cz_ = cz;
                }
            }
        }
    }
}

nd_kernel_config default_config(const nd_problem* p) {
    nd_kernel_config c{};
    c.grid = 0;
    c.chunk = 64;
    if (p->topo == ND_RING) {
        // rings up to 4096 elements stay resident in one workgroup (negative tile =
        // resident capacity); larger rings use the per-stage tiled kernel
        if (p->n <= 1024) c.tile = -1024;
        else if (p->n <= 2048) c.tile = -2048;
        else if (p->n <= 4096) c.tile = -4096;
        else c.tile = p->n <= (int64_t(1) << 20) ? 512 : 1024;
        c.block = ring_block(c.tile);
    } else if (p->topo == ND_CUBE3D) {
        // e.g. 25 x 20 x 67 on a 200^3 lattice at h = 4: 240 work items, one round
        const int h = (int)p->radius;
        int cx, cy, cz;
        cube_tiles(p, device_cu_count(), &cx, &cy, &cz);
        c.tile = cx;
        c.tile_y = cy;
        c.tile_z = cz;
        c.block = cube_block(h, cx, cy);
    } else if (p->topo == ND_BALL3D || p->topo == ND_DISK2D) {
        int cx, cy, cz, bs;
        ball_tiles(p, device_cu_count(), &cx, &cy, &cz, &bs);
        c.tile = cx;
        c.tile_y = cy;
        c.tile_z = cz;
        c.block = bs;
    } else if (p->topo == ND_LINKS) {
        c.tile = kLinksRows;  // rows per work item
        c.block = 256;
    } else {
        c.tile = 256;    // target rows per work item
        c.tile_y = 8;    // edges per thread per chunk
        c.block = 256;
    }
    return c;
}

nd_kernel_config config_for(const nd_problem* p) {
    nd_kernel_config c = default_config(p);
    nd_kernel_config tuned;
    if (tuned_config(p, &tuned)) c = tuned;
    return c;
}

int ring_block(int tile) {
    if (tile < 0) return tile == -4096 ? 512 : 256;
    return tile == 128 ? 64 : (tile == 256 ? 128 : 256);  // two elements per thread up to 512
}

static int64_t bulk_bytes(int prec) { return prec == ND_FP64 ? 8 : 4; }

static int64_t ring_tiles(int64_t n, int tile) { return tile < 0 ? 1 : (n + tile - 1) / tile; }

int64_t footprint_bytes(const nd_problem* p, const nd_kernel_config& c) {
    const int64_t V = nvars_of(p->model), n = p->n, kb = bulk_bytes(p->precision);
    int64_t b = 3 * V * n * 8 + 3 * V * n * kb;  // y[2], acc, k[3]
    if (p->topo == ND_RING) b += 3 * 2 * ring_tiles(n, c.tile) * 8;
    if (p->topo == ND_CUBE3D || p->topo == ND_BALL3D || p->topo == ND_DISK2D)
        b += 3 * 2 * 8 * ((p->n1 + c.tile - 1) / c.tile) * ((p->n2 + c.tile_y - 1) / c.tile_y) *
             ((p->n3 + c.tile_z - 1) / c.tile_z);
    if (p->topo == ND_CSR)
        b += kCsrSourceBlocks * (n + 1) * 8 + p->nnz * (4 + kb) + n * 8 + 2 * n * kb + kCsrSourceBlocks * n * 8;
    if (p->topo == ND_LINKS) {
        // the compressed matrix (sized by compressing it), the two exchanged-map buffers and
        // the per-work-item sums
        LinksCompressed lc;
        if (compress_links(n, p->row_ptr, p->col, &lc) == ND_OK) b += links_device_bytes(lc);
        b += 2 * n * (int64_t)links_map_bytes(p->model, p->precision) + 3 * 2 * 8 * ((n + kLinksRows - 1) / kLinksRows);
    }
    b += sizeof(NetDesc) + 64;
    return b;
}

// -------------------------------------------------------------- allocation
// Buffers of networks the caller owns come from the device's stream-ordered
// pool, allocated and freed on a stream of the library's own (one per device,
// non-blocking, default priority).  A network's buffers are freed only after its
// own work has completed (its event), so destroying or reconfiguring a network
// waits for that network alone; hipFree would wait for the whole device.
constexpr int kMaxDevices = 64;
static std::mutex g_ls_mu;
static hipStream_t g_ls[kMaxDevices] = {};

static nd_status lib_stream(int dev, hipStream_t* out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(ND_ERR_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_ls_mu);
    if (!g_ls[dev]) {
        int cur = 0;
        HIPC(hipGetDevice(&cur));
        if (cur != dev) HIPC(hipSetDevice(dev));
        const hipError_t e = hipStreamCreateWithFlags(&g_ls[dev], hipStreamNonBlocking);
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate (allocation stream)");
    }
    *out = g_ls[dev];
    return ND_OK;
}

nd_status Net::alloc(void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e;
    if (astream) {
        e = hipMallocAsync(ptr, bytes, astream);
    } else {
        hipStream_t ls;
        const nd_status s = lib_stream(dev, &ls);
        if (s) return s;
        // ready for use on any stream once the allocation stream has passed it
        e = hipMallocAsync(ptr, bytes, ls);
        if (e == hipSuccess) e = hipStreamSynchronize(ls);
    }
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    allocs.push_back(*ptr);
    return ND_OK;
}

// Pinned host words for the networks' status read-backs, carved from blocks
// that live until the process ends (hipHostFree would wait for the device).
static std::mutex g_pin_mu;
static std::vector<int32_t*> g_pin_free;

static nd_status pinned_word(int32_t** out) {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (g_pin_free.empty()) {
        constexpr int kWords = 4096;
        int32_t* blk = nullptr;
        HIPC(hipHostMalloc((void**)&blk, kWords * sizeof(int32_t)));
        for (int i = kWords - 1; i >= 0; --i) g_pin_free.push_back(blk + i);
    }
    *out = g_pin_free.back();
    g_pin_free.pop_back();
    return ND_OK;
}

static void pinned_word_put(int32_t* w) {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(w);
}

// Return one of this network's buffers to the pool; the device no longer uses
// it (the caller has waited for the network's work, or owns astream's order).
void Net::free_buf(void* q) {
    if (astream) {
        (void)hipFreeAsync(q, astream);
        return;
    }
    hipStream_t ls;
    if (lib_stream(dev, &ls) == ND_OK) (void)hipFreeAsync(q, ls);
}

RunEvent::~RunEvent() {
    if (ev) (void)hipEventDestroy(ev);
}

void Net::quiesce() {
    if (ev_recorded) {
        (void)hipEventSynchronize(batch_ev ? batch_ev->ev : last_ev);
        ev_recorded = false;
    }
    batch_ev.reset();
}

nd_status Net::touch(hipStream_t st) {
    batch_ev.reset();
    hipError_t e = hipEventRecord(last_ev, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ev_recorded = true;
    return ND_OK;
}

void Net::touch_shared(const std::shared_ptr<RunEvent>& ev) {
    batch_ev = ev;
    ev_recorded = true;
}

void Net::drop_graphs() {
    for (auto& g : solo_graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

Net::~Net() {
    // server networks: the owner has seen the last work complete and the frees
    // are ordered on astream; others: wait for this network's own work
    if (!astream) quiesce();
    drop_graphs();
    for (void* q : allocs) free_buf(q);
    if (status_host && own_status_host) pinned_word_put(status_host);
    if (last_ev) (void)hipEventDestroy(last_ev);
}

// Host-to-device copy of set-up data (sources are host temporaries): synchronous,
// or on astream, waiting for that stream only, not for the device.
static hipError_t setup_copy(hipStream_t astream, void* dst, const void* src, size_t bytes) {
    if (!astream) return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, astream);
    return e != hipSuccess ? e : hipStreamSynchronize(astream);
}

static void derive_params(const nd_problem* p, NetDesc& d) {
    std::memset(d.p, 0, sizeof d.p);
    if (p->model == ND_KURAMOTO || p->model == ND_KURAMOTO_INERTIA) {
        // links: the kernels divide each row's sum by its own link count
        const double L = p->topo == ND_RING     ? 2.0 * (double)p->radius
                         : p->topo == ND_BALL3D ? (double)ball_points(p->radius)
                         : p->topo == ND_DISK2D ? (double)disk_points(p->radius)
                         : p->topo == ND_LINKS  ? 1.0
                                                : std::pow(2.0 * (double)p->radius + 1.0, 3.0) - 1.0;
        d.p[0] = p->params[0];
        d.p[1] = p->params[1] / L;
        d.p[2] = std::cos(p->params[2]);
        d.p[3] = std::sin(p->params[2]);
        if (p->model == ND_KURAMOTO_INERTIA) {
            d.p[4] = p->params[4];        // eps
            d.p[5] = 1.0 / p->params[3];  // 1/m
        }
    } else if (p->model == ND_FHN) {
        d.p[0] = p->params[0];
        d.p[1] = p->params[1];
        // links: the kernels pass the row's mean, so kappa = sigma and the count is 1
        const double L = p->topo == ND_LINKS ? 1.0 : 2.0 * (double)p->radius;
        d.p[2] = p->params[2] / L;
        d.p[3] = std::cos(p->params[3]);
        d.p[4] = std::sin(p->params[3]);
        d.p[5] = L;
        d.p[6] = 1.0 / p->params[0];
    } else {
        for (int i = 0; i < 10; ++i) d.p[i] = p->params[i];
    }
}

nd_status Net::create(const nd_problem* pr) {
    HIPC(hipGetDevice(&dev));
    prob = *pr;
    prob.row_ptr = nullptr;
    prob.col = nullptr;
    prob.weight = nullptr;
    prob.per_elem = nullptr;
    cfg = config_for(pr);
    const int64_t V = nvars_of(pr->model), n = pr->n, kb = bulk_bytes(pr->precision);
    std::memset(&tmpl, 0, sizeof tmpl);
    NetDesc& d = tmpl;
    d.n = n;
    d.P = pr->radius;
    d.n1 = (int32_t)pr->n1;
    d.n2 = (int32_t)pr->n2;
    d.n3 = (int32_t)pr->n3;
    d.model = pr->model;
    d.prec = pr->precision;
    derive_params(pr, d);
    nd_status s;
    for (int b = 0; b < 2; ++b)
        if ((s = alloc((void**)&d.y[b], V * n * 8))) return s;
    if ((s = alloc((void**)&d.acc, V * n * 8))) return s;
    for (int b = 0; b < 3; ++b)
        if ((s = alloc(&d.k[b], V * n * kb))) return s;
    if (pr->topo == ND_CSR) {
        // split every row's in-edges by source block (sources ascending, so each
        // block keeps its order) and lay the blocks out one after the other
        const int B = kCsrSourceBlocks;
        const int64_t nnz = pr->nnz;
        std::vector<int64_t> bptr((size_t)B * (n + 1), 0);
        auto block_of = [&](int64_t src) { return (int)std::min<int64_t>(B - 1, src * B / n); };
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = pr->row_ptr[i]; e < pr->row_ptr[i + 1]; ++e) ++bptr[(size_t)block_of(pr->col[e]) * (n + 1) + i + 1];
        int64_t base = 0;
        for (int b = 0; b < B; ++b) {
            int64_t* p = bptr.data() + (size_t)b * (n + 1);
            p[0] = base;
            for (int64_t i = 0; i < n; ++i) p[i + 1] += p[i];
            base = p[n];
        }
        std::vector<int64_t> pos(bptr);
        std::vector<int32_t> col2((size_t)std::max<int64_t>(nnz, 1));
        std::vector<double> w2((size_t)std::max<int64_t>(nnz, 1));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = pr->row_ptr[i]; e < pr->row_ptr[i + 1]; ++e) {
                const int b = block_of(pr->col[e]);
                const int64_t dst = pos[(size_t)b * (n + 1) + i]++;
                col2[dst] = pr->col[e];
                w2[dst] = pr->weight[e];
            }
        if ((s = alloc((void**)&d.row_ptr, (size_t)B * (n + 1) * 8))) return s;
        if ((s = alloc((void**)&d.col, std::max<int64_t>(nnz, 1) * 4))) return s;
        if ((s = alloc((void**)&d.w, std::max<int64_t>(nnz, 1) * kb))) return s;
        if ((s = alloc((void**)&d.acc_part, (size_t)B * n * 8))) return s;
        if ((s = alloc((void**)&d.iapp, n * 8))) return s;
        for (int b = 0; b < 2; ++b)
            if ((s = alloc(&d.sx[b], n * kb))) return s;
        HIPC(setup_copy(astream, (void*)d.row_ptr, bptr.data(), bptr.size() * 8));
        if (nnz > 0) {
            HIPC(setup_copy(astream, (void*)d.col, col2.data(), nnz * 4));
            if (kb == 8) {
                HIPC(setup_copy(astream, (void*)d.w, w2.data(), nnz * 8));
            } else {
                std::vector<float> wf(nnz);
                for (int64_t e = 0; e < nnz; ++e) wf[e] = (float)w2[e];
                HIPC(setup_copy(astream, (void*)d.w, wf.data(), nnz * 4));
            }
        }
        HIPC(setup_copy(astream, (void*)d.iapp, pr->per_elem, n * 8));
    }
    if (pr->topo == ND_LINKS) {
        LinksCompressed lc;
        if ((s = compress_links(n, pr->row_ptr, pr->col, &lc))) return s;
        if ((int64_t)lc.dpos.size() >= (int64_t(1) << 31))
            return fail(ND_ERR_UNSUPPORTED, "links: the difference table holds 2^31 or more positions");
        LinksDeviceForm f;
        links_device_form(lc, &f);
        const size_t K = f.inv.size();
        if ((s = alloc((void**)&d.lrow, n * 4))) return s;
        if ((s = alloc((void**)&d.lvpos, lc.V.size() * 4))) return s;
        if ((s = alloc((void**)&d.ldptr, (K + 1) * 4))) return s;
        if ((s = alloc((void**)&d.ldpos, f.dsig.size() * 4))) return s;
        if ((s = alloc((void**)&d.linv, K * 8))) return s;
        for (int b = 0; b < 2; ++b)
            if ((s = alloc(&d.sx[b], n * (int64_t)links_map_bytes(pr->model, pr->precision)))) return s;
        d.lnv = (int32_t)lc.V.size();
        HIPC(setup_copy(astream, (void*)d.lrow, lc.C.data(), n * 4));
        if (!lc.V.empty()) HIPC(setup_copy(astream, (void*)d.lvpos, lc.V.data(), lc.V.size() * 4));
        HIPC(setup_copy(astream, (void*)d.ldptr, f.dptr.data(), (K + 1) * 4));
        if (!f.dsig.empty()) HIPC(setup_copy(astream, (void*)d.ldpos, f.dsig.data(), f.dsig.size() * 4));
        HIPC(setup_copy(astream, (void*)d.linv, f.inv.data(), K * 8));
    }
    if ((s = alloc((void**)&solo_desc, sizeof(NetDesc)))) return s;
    if ((s = alloc((void**)&solo_count, 2 * sizeof(int)))) return s;
    if ((s = alloc((void**)&status_dev, sizeof(int32_t)))) return s;
    HIPC(astream ? hipMemsetAsync(status_dev, 0, sizeof(int32_t), astream) : hipMemset(status_dev, 0, sizeof(int32_t)));
    if (own_status_host && (s = pinned_word(&status_host))) return s;
    *status_host = 0;
    HIPC(hipEventCreateWithFlags(&last_ev, hipEventDisableTiming));
    d.status = status_dev;
    return apply_config(cfg);
}

// (Re)build everything that depends on the kernel configuration: the work
// decomposition, the per-work-item sum buffers and the single-network work map.
nd_status Net::apply_config(const nd_kernel_config& c) {
    quiesce();  // the buffers below may be in use by enqueued work
    drop_graphs();
    auto release = [&](void*& q) {
        if (!q) return;
        free_buf(q);
        allocs.erase(std::find(allocs.begin(), allocs.end(), q));
        q = nullptr;
    };
    release((void*&)tmpl.tsum[0]);
    release((void*&)tmpl.tsum[1]);
    release((void*&)tmpl.rsum);
    release((void*&)solo_work);
    cfg = c;
    const int64_t n = prob.n;
    if (prob.topo == ND_RING) {
        cfg.block = ring_block(cfg.tile);
        tmpl.tile = cfg.tile;
        tmpl.G = (int32_t)ring_tiles(n, cfg.tile);
    } else if (prob.topo == ND_CUBE3D || prob.topo == ND_BALL3D || prob.topo == ND_DISK2D) {
        const int h = (int)prob.radius;
        if (prob.topo == ND_CUBE3D) cfg.block = cube_block(h, cfg.tile, cfg.tile_y);
        tmpl.cx = cfg.tile;
        tmpl.cy = cfg.tile_y;
        tmpl.cz = cfg.tile_z;
        tmpl.gx = (int32_t)((prob.n1 + cfg.tile - 1) / cfg.tile);
        tmpl.gy = (int32_t)((prob.n2 + cfg.tile_y - 1) / cfg.tile_y);
        tmpl.pz = ball_pz(prob.topo, prob.radius);
        const int32_t gz = (int32_t)((prob.n3 + cfg.tile_z - 1) / cfg.tile_z);
        tmpl.G = tmpl.gx * tmpl.gy * gz;
    } else if (prob.topo == ND_LINKS) {
        cfg.block = 256;
        cfg.tile = kLinksRows;  // rows per work item (fixed by the kernel)
        tmpl.tile = kLinksRows;
        tmpl.G = (int32_t)((n + kLinksRows - 1) / kLinksRows);
    } else {
        cfg.block = 256;
        cfg.tile = 256;  // rows per work item (fixed by the kernel)
        tmpl.tile = 256;
        tmpl.G = (int32_t)(kCsrSourceBlocks * ((n + 255) / 256));  // (row tile, source block)
    }
    nd_status s;
    if (prob.topo != ND_CSR) {
        for (int b = 0; b < 2; ++b)
            if ((s = alloc((void**)&tmpl.tsum[b], 2 * (int64_t)tmpl.G * 8))) return s;
        if ((s = alloc((void**)&tmpl.rsum, 2 * (int64_t)tmpl.G * 8))) return s;
    }
    std::vector<int2> wk;
    append_work(0, wk);
    if ((s = alloc((void**)&solo_work, wk.size() * sizeof(int2)))) return s;
    HIPC(setup_copy(astream, solo_work, wk.data(), wk.size() * sizeof(int2)));
    int cnt[2] = {(int)wk.size(), 1};
    HIPC(setup_copy(astream, solo_count, cnt, sizeof cnt));
    return ND_OK;
}

int64_t Net::work_items() const { return tmpl.G; }

void Net::append_work(int desc_index, std::vector<int2>& wk) const {
    const int64_t m = work_items();
    for (int64_t t = 0; t < m; ++t) wk.push_back(make_int2(desc_index, (int)t));
}

nd_status Net::prepare_observe(int64_t steps, const nd_observe* obs, bool may_alloc) {
    last_steps = steps;
    r_every = 0;
    mv_start = -1;
    if (!obs) return ND_OK;
    if (obs->record_every < 0) return fail(ND_ERR_INVALID_ARG, "record_every must be >= 0");
    if (obs->mv_start_step < -1) return fail(ND_ERR_INVALID_ARG, "mv_start_step must be >= -1");
    const bool want_r = obs->record_every > 0, want_mv = obs->mv_start_step >= 0;
    if ((want_r || want_mv) && prob.model == ND_HH)
        return fail(ND_ERR_INVALID_ARG, "R and mean phase velocity are not defined for HH");
    if ((want_r || want_mv) && steps < 1) return fail(ND_ERR_INVALID_ARG, "recording observables needs steps >= 1");
    if (want_mv && obs->mv_start_step >= steps) return fail(ND_ERR_INVALID_ARG, "mv_start_step must be < steps");
    nd_status s;
    if (want_r) {
        const int64_t len = steps / obs->record_every + 1;
        if (len > R_cap && !may_alloc)
            return fail(ND_ERR_INVALID_ARG,
                        "recording %lld values of R needs a buffer an earlier run sized (it holds %lld)",
                        (long long)len, (long long)R_cap);
        if (len > R_cap) {
            if (R_dev) {
                quiesce();  // earlier runs may still record into it
                free_buf(R_dev);
                allocs.erase(std::find(allocs.begin(), allocs.end(), (void*)R_dev));
            }
            if ((s = alloc((void**)&R_dev, len * 8))) return s;
            R_cap = len;
        }
        r_every = obs->record_every;
    }
    if (want_mv) {
        if (!mv_dev && !may_alloc)
            return fail(ND_ERR_INVALID_ARG, "recording the mean phase velocity needs a buffer an earlier run sized");
        if (!mv_dev && (s = alloc((void**)&mv_dev, prob.n * 8))) return s;
        mv_start = obs->mv_start_step;
    }
    return ND_OK;
}

NetDesc Net::run_desc(double dt, int64_t steps) const {
    NetDesc d = tmpl;
    d.dt = dt;
    d.dt3 = dt / 3.0;
    d.dt6 = dt / 6.0;
    d.obs = (r_every > 0 ? OBS_R : 0) | (mv_start >= 0 ? OBS_MV : 0);
    d.R = R_dev;
    d.r_every = r_every > 0 ? r_every : 1;
    d.mv = mv_dev;
    d.mv_start = mv_start;
    d.mv_scale = mv_start >= 0 ? 1.0 / ((double)(steps - mv_start) * dt) : 0.0;
    d.g0 = 0;
    d.nsteps = steps;
    d.ypar = ypar;
    return d;
}

nd_status Net::begin_run(double dt, int64_t steps, const nd_observe* obs) {
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ND_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (steps < 1) return fail(ND_ERR_INVALID_ARG, "steps must be >= 1");
    nd_status s = prepare_observe(steps, obs);
    if (s) return s;
    run_dt = dt;
    run_total = steps;
    run_done = 0;
    return ND_OK;
}

NetDesc Net::chunk_desc() const {
    NetDesc d = run_desc(run_dt, run_total);
    d.g0 = run_done;
    d.nsteps = run_total - run_done;
    return d;
}

// ----------------------------------------------------------- launch groups
__global__ void k_advance(NetDesc* D, int ndesc, int chunk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ndesc) {
        NetDesc& d = D[i];
        if (d.nsteps > 0) {
            const int64_t done = d.nsteps < chunk ? d.nsteps : (int64_t)chunk;
            d.g0 += done;
            d.nsteps -= done;
            d.ypar ^= (int)(done & 1);
        }
    }
}

// Enqueue one chunk of `chunk` steps for a group of networks of one kernel
// class.  Each network runs min(chunk, remaining) steps.
nd_status enqueue_chunk(const Group& g, int chunk, hipStream_t st) {
    const int grid = g.grid;
    hipError_t e;
    if (g.topo == ND_RING) {
        RingLaunch L;
        if (!ring_select(g.model, g.prec, g.tile, &L)) return fail(ND_ERR_UNSUPPORTED, "no ring kernel for tile %d", g.tile);
        if (g.tile < 0) {
            if (!L.resident || L.bs * 4 > -g.tile) return fail(ND_ERR_UNSUPPORTED, "bad resident ring entry");
            if ((e = ring_launch_resident(L, grid, st, g.desc, g.work, g.nwork, chunk, g.mv)) != hipSuccess)
                return hip_fail(e, "ring resident");
        } else {
            if ((e = ring_launch_prologue(L, grid, st, g.desc, g.work, g.nwork)) != hipSuccess)
                return hip_fail(e, "ring prologue");
            for (int j = 0; j < chunk; ++j)
                for (int s = 1; s <= 4; ++s)
                    if ((e = ring_launch_stage(L, grid, st, g.desc, g.work, g.nwork, s, j, g.mv)) != hipSuccess)
                        return hip_fail(e, "ring stage");
        }
        if ((e = ring_launch_epilogue(L, grid, st, g.desc, g.work, g.nwork, chunk)) != hipSuccess)
            return hip_fail(e, "ring epilogue");
    } else if (g.topo == ND_CUBE3D) {
        CubeLaunch L;
        if (!cube_select(g.model, g.prec, g.h, &L))
            return fail(ND_ERR_UNSUPPORTED, "no cube kernel for model %d, h = %d", g.model, g.h);
        const int block = cube_block(g.h, g.tile, g.tile_y);
        const size_t smem = cube_smem_bytes(g.h, g.tile, g.tile_y, cube_lds_buffers(g.model, g.prec, g.h));
        for (int j = 0; j < chunk; ++j)
            for (int s = 1; s <= 4; ++s)
                if ((e = cube_launch_stage(L, grid, block, smem, st, g.desc, g.work, g.nwork, s, j, g.mv)) != hipSuccess)
                    return hip_fail(e, "cube stage");
        if ((e = cube_launch_final(L, grid, st, g.desc, g.work, g.nwork, chunk)) != hipSuccess)
            return hip_fail(e, "cube final");
    } else if (g.topo == ND_BALL3D || g.topo == ND_DISK2D) {
        CubeLaunch L;
        const bool scatter = g.block == kBallScatterBlock;
        if (scatter ? !ball_scatter_select(g.model, g.prec, g.h, &L) : !ball_select(g.model, g.prec, g.block, &L))
            return fail(ND_ERR_UNSUPPORTED, "no ball kernel for model %d, block %d, radius %d", g.model, g.block, g.h);
        const size_t smem = scatter ? ball_scatter_smem_bytes(g.h, g.tile, g.tile_y)
                                    : ball_smem_bytes(g.h, ball_pz(g.topo, g.h), g.tile, g.tile_y);
        for (int j = 0; j < chunk; ++j)
            for (int s = 1; s <= 4; ++s)
                if ((e = cube_launch_stage(L, grid, g.block, smem, st, g.desc, g.work, g.nwork, s, j, g.mv)) != hipSuccess)
                    return hip_fail(e, "ball stage");
        if ((e = cube_launch_final(L, grid, st, g.desc, g.work, g.nwork, chunk)) != hipSuccess)
            return hip_fail(e, "ball final");
    } else if (g.topo == ND_LINKS) {
        LinksLaunch L;
        if (!links_select(g.model, g.prec, &L)) return fail(ND_ERR_UNSUPPORTED, "no links kernel for model %d", g.model);
        if ((e = links_launch_chunk(L, grid, st, g.desc, g.work, g.nwork, chunk, g.mv)) != hipSuccess)
            return hip_fail(e, "links chunk");
    } else {
        CsrLaunch L;
        if (!csr_select(g.prec, g.tile_y, &L)) return fail(ND_ERR_UNSUPPORTED, "no CSR kernel for %d edges per thread", g.tile_y);
        if ((e = csr_launch_prologue(L, grid, st, g.desc, g.work, g.nwork)) != hipSuccess) return hip_fail(e, "csr prologue");
        for (int j = 0; j < chunk; ++j)
            for (int s = 1; s <= 4; ++s)
                if ((e = csr_launch_stage(L, grid, st, g.desc, g.work, g.nwork, s, j)) != hipSuccess)
                    return hip_fail(e, "csr stage");
    }
    hipLaunchKernelGGL(k_advance, dim3((g.ndesc + 255) / 256), dim3(256), 0, st, g.desc, g.ndesc, chunk);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "advance");
    return ND_OK;
}

bool graphs_enabled() {
    static const bool on = [] {
        const char* v = getenv("ND_GRAPHS");
        return !(v && v[0] == '0');
    }();
    return on;
}

// Capture one chunk of K steps of group g into an executable graph.
nd_status capture_chunk(const Group& g, int K, hipGraphExec_t* out) {
    hipStream_t cap;
    HIPC(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    nd_status s = enqueue_chunk(g, K, cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    if (s) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return ND_OK;
}

// State values per launch from which a group runs without graph capture.
constexpr int64_t kEagerValues = int64_t(1) << 20;

__global__ void k_put_desc(NetDesc* dst, NetDesc d) { *dst = d; }
__global__ void k_clear_status(int32_t* status) { *status = 0; }

hipError_t put_desc(NetDesc* dst, const NetDesc& d, hipStream_t st) {
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(1), 0, st, dst, d);
    return hipGetLastError();
}

hipError_t clear_status(int32_t* status, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, st, status);
    return hipGetLastError();
}

// Pinned host staging for the descriptor tables and work maps of batched runs.
// A block is handed out again only after the event recorded behind its upload
// has completed, so a run returns without waiting for the device and the host
// never rewrites a block a pending copy still reads.
namespace {
struct Staging {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool busy = false;      // handed out, upload not yet recorded
    bool pending = false;   // an upload from it may still be in flight
};
std::mutex g_stage_mu;
std::vector<std::unique_ptr<Staging>> g_stage;

// Graph executables of batched runs, destroyed once their last replay is done.
struct DeadGraph {
    hipGraphExec_t exec;
    hipEvent_t ev;
};
std::mutex g_dead_mu;
std::vector<DeadGraph> g_dead;

void reap_graphs() {
    std::lock_guard<std::mutex> lk(g_dead_mu);
    std::vector<DeadGraph> keep;
    for (const DeadGraph& d : g_dead) {
        if (hipEventQuery(d.ev) == hipSuccess) {
            (void)hipGraphExecDestroy(d.exec);
            (void)hipEventDestroy(d.ev);
        } else {
            keep.push_back(d);
        }
    }
    g_dead.swap(keep);
}

nd_status retire_graph(hipGraphExec_t exec, hipStream_t st) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e != hipSuccess) {  // fall back to waiting here
        (void)hipStreamSynchronize(st);
        (void)hipGraphExecDestroy(exec);
        return hip_fail(e, "graph retirement event");
    }
    std::lock_guard<std::mutex> lk(g_dead_mu);
    g_dead.push_back({exec, ev});
    return ND_OK;
}

nd_status staging_get(size_t bytes, Staging** out) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (auto& b : g_stage) {
        if (b->busy || b->cap < bytes) continue;
        if (b->pending) {
            if (hipEventQuery(b->ev) != hipSuccess) continue;
            b->pending = false;
        }
        b->busy = true;
        *out = b.get();
        return ND_OK;
    }
    auto b = std::make_unique<Staging>();
    b->cap = std::max<size_t>(bytes, 64 * 1024);
    hipError_t e = hipHostMalloc(&b->p, b->cap);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc (staging)");
    e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipHostFree(b->p);
        return hip_fail(e, "hipEventCreate (staging)");
    }
    b->busy = true;
    *out = b.get();
    g_stage.push_back(std::move(b));
    return ND_OK;
}

// The uploads from `b` are enqueued on st: record that and release the block.
nd_status staging_put(Staging* b, hipStream_t st) {
    hipError_t e = hipEventRecord(b->ev, st);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    b->busy = false;
    b->pending = true;
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        b->pending = false;
        return hip_fail(e, "hipEventRecord (staging)");
    }
    return ND_OK;
}
}  // namespace

// Run a set of networks (possibly of different classes) for their own step
// counts.  Everything is enqueued on st and the call returns without waiting
// for the device: descriptors of a single network travel as a kernel argument,
// those of batches through pinned staging blocks; each network records an event
// behind its work so that reconfiguring or destroying it waits for exactly that.
nd_status run_nets(Net* const* nets, int count, const double* dt, const int64_t* steps, const nd_observe* obs,
                   hipStream_t st) {
    // validate and prepare observables
    for (int i = 0; i < count; ++i) {
        if (!nets[i]) return fail(ND_ERR_INVALID_ARG, "handle %d is NULL", i);
        if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(ND_ERR_INVALID_ARG, "dt must be finite and > 0");
        if (steps[i] < 0) return fail(ND_ERR_INVALID_ARG, "steps must be >= 0");
    }
    {
        std::vector<Net*> sorted(nets, nets + count);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(ND_ERR_INVALID_ARG, "a handle appears twice in one batch");
    }
    reap_graphs();
    nd_status s;
    for (int i = 0; i < count; ++i)
        if ((s = nets[i]->prepare_observe(steps[i], obs ? &obs[i] : nullptr))) return s;
    // group by kernel class
    std::map<std::tuple<int, int, int, int, int, int, int>, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        if (steps[i] == 0) continue;
        const Net* n = nets[i];
        const int h = n->prob.topo == ND_CUBE3D || n->prob.topo == ND_BALL3D || n->prob.topo == ND_DISK2D
                          ? (int)n->prob.radius : 0;
        const int bs = (n->prob.topo == ND_BALL3D || n->prob.topo == ND_DISK2D) ? n->cfg.block : 0;
        groups[std::make_tuple(n->prob.model, n->prob.topo, n->prob.precision, n->cfg.tile, n->cfg.tile_y, h, bs)]
            .push_back(i);
    }
    for (auto& kv : groups) {
        const std::vector<int>& idx = kv.second;
        Group g{};
        g.model = std::get<0>(kv.first);
        g.topo = std::get<1>(kv.first);
        g.prec = std::get<2>(kv.first);
        g.tile = std::get<3>(kv.first);
        g.tile_y = std::get<4>(kv.first);
        g.h = std::get<5>(kv.first);
        g.block = std::get<6>(kv.first);
        g.ndesc = (int)idx.size();
        int64_t maxsteps = 0, nwork = 0;
        g.mv = false;
        for (int q : idx) {
            g.mv = g.mv || nets[q]->mv_start >= 0;
            nwork += nets[q]->work_items();
            maxsteps = std::max(maxsteps, steps[q]);
        }
        const bool solo = idx.size() == 1;
        void* scratch = nullptr;
        hipError_t e;
        if (solo) {
            Net* n = nets[idx[0]];
            g.desc = n->solo_desc;
            g.work = n->solo_work;
            g.nwork = n->solo_count;
            if ((e = put_desc(g.desc, n->run_desc(dt[idx[0]], steps[idx[0]]), st)) != hipSuccess)
                return hip_fail(e, "descriptor upload");
        } else {
            const size_t bd = idx.size() * sizeof(NetDesc), bw = (size_t)nwork * sizeof(int2);
            Staging* sb = nullptr;
            if ((s = staging_get(bd + bw + 16, &sb))) return s;
            NetDesc* hd = (NetDesc*)sb->p;
            int2* hw = (int2*)((char*)sb->p + bd);
            int w = 0;
            for (int q = 0; q < (int)idx.size(); ++q) {
                Net* n = nets[idx[q]];
                hd[q] = n->run_desc(dt[idx[q]], steps[idx[q]]);
                const int64_t m = n->work_items();
                for (int64_t t = 0; t < m; ++t) hw[w++] = make_int2(q, (int)t);
            }
            *(int*)((char*)sb->p + bd + bw) = w;
            e = hipMallocAsync(&scratch, bd + bw + 16, st);
            if (e == hipSuccess) e = hipMemcpyAsync(scratch, sb->p, bd + bw + 16, hipMemcpyHostToDevice, st);
            const nd_status sp = staging_put(sb, st);
            if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
            if (sp) return sp;
            g.desc = (NetDesc*)scratch;
            g.work = (int2*)((char*)scratch + bd);
            g.nwork = (int*)((char*)scratch + bd + bw);
        }
        const Net* n0 = nets[idx[0]];
        const int cfg_grid = n0->cfg.grid;
        g.grid = cfg_grid > 0 ? (int)std::min<int64_t>(cfg_grid, nwork) : (int)nwork;
        const int K = std::max(1, n0->cfg.chunk);
        // Replaying a captured chunk saves the host's per-launch cost, which matters
        // for short kernels; groups whose stage kernels are long (many state values
        // per launch) run eagerly, which measured a few percent faster per launch.
        // Rings resident in one workgroup always take the chunked path.
        int64_t values = 0;
        for (int q : idx) values += nets[q]->prob.n * nvars_of(nets[q]->prob.model);
        const bool eager = values >= kEagerValues && !(g.topo == ND_RING && g.tile < 0);
        if (maxsteps <= K || !graphs_enabled() || eager) {
            // one eager chunk covering every network's steps
            if ((s = enqueue_chunk(g, (int)std::min<int64_t>(maxsteps, 1 << 30), st))) return s;
        } else {
            // replay a captured K-step chunk; the descriptors advance on the
            // device, so every replay continues where the last one stopped
            const int64_t reps = (maxsteps + K - 1) / K;
            hipGraphExec_t exec = nullptr;
            Net* so = solo ? nets[idx[0]] : nullptr;
            const int slot = g.mv ? 1 : 0;
            if (so && so->solo_graph[slot] && so->solo_graph_key[slot][0] == K &&
                so->solo_graph_key[slot][1] == g.grid) {
                exec = so->solo_graph[slot];
            } else {
                if ((s = capture_chunk(g, K, &exec))) return s;
                if (so) {
                    if (so->solo_graph[slot]) (void)retire_graph(so->solo_graph[slot], st);
                    so->solo_graph[slot] = exec;
                    so->solo_graph_key[slot][0] = K;
                    so->solo_graph_key[slot][1] = g.grid;
                }
            }
            e = hipSuccess;
            for (int64_t r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(exec, st);
            if (!so) {
                const nd_status rs = retire_graph(exec, st);
                if (e == hipSuccess && rs) return rs;
            }
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        }
        if (scratch) HIPC(hipFreeAsync(scratch, st));
    }
    for (int i = 0; i < count; ++i) nets[i]->ypar ^= (int)(steps[i] & 1);
    if (count == 1) return nets[0]->touch(st);
    // one event behind the whole batch, shared by its networks
    auto ev = std::make_shared<RunEvent>();
    HIPC(hipEventCreateWithFlags(&ev->ev, hipEventDisableTiming));
    HIPC(hipEventRecord(ev->ev, st));
    for (int i = 0; i < count; ++i) nets[i]->touch_shared(ev);
    return ND_OK;
}

// ------------------------------------------------- runs that allocate nothing
// nd_run_batch_noalloc keeps the descriptor tables, the per-group work counts and
// the work maps in `scratch`, one fixed array per GPU, instead of memory taken per
// call.  Layout: ND_NOALLOC_MAX_NETS descriptors, then ND_NOALLOC_MAX_NETS work
// counts, then ND_NOALLOC_MAX_WORK work items; a call lays its groups out one
// after the other.  Host code reaches the array only through the address
// hipGetSymbolAddress returns for the current device (the symbol itself is a
// host-side stand-in, not a device address).
constexpr size_t kNaDescBytes = ((size_t)ND_NOALLOC_MAX_NETS * sizeof(NetDesc) + 255) / 256 * 256;
constexpr size_t kNaCountBytes = ((size_t)ND_NOALLOC_MAX_NETS * sizeof(int) + 255) / 256 * 256;
constexpr size_t kNaBytes = kNaDescBytes + kNaCountBytes + (size_t)ND_NOALLOC_MAX_WORK * sizeof(int2);
static_assert(kNaBytes <= (size_t)ND_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds its stated size");
static __device__ __align__(256) unsigned char scratch[ND_NOALLOC_SCRATCH_BYTES];

constexpr int kNaMaxDevices = 64;
static std::mutex g_na_mu;
static unsigned char* g_na_ptr[kNaMaxDevices] = {};

// The scratch array's device address on the current device, looked up once per
// device (with that device current) and kept.
static nd_status noalloc_scratch(unsigned char** out) {
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(ND_ERR_UNSUPPORTED, "device %d beyond %d devices", dev, kNaMaxDevices);
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (no-allocation scratch)");
        g_na_ptr[dev] = (unsigned char*)p;
    }
    *out = g_na_ptr[dev];
    return ND_OK;
}

// Work map of one group, built on the device from its descriptors (the same
// order as the host-built map of nd_run_batch: networks in turn, tiles ascending).
__global__ void k_noalloc_work(const NetDesc* D, int ndesc, int2* work, int* nwork) {
    __shared__ int off[ND_NOALLOC_MAX_NETS + 1];
    if (threadIdx.x == 0) {
        int o = 0;
        for (int q = 0; q < ndesc; ++q) {
            off[q] = o;
            o += D[q].G;
        }
        off[ndesc] = o;
        *nwork = o;
    }
    __syncthreads();
    for (int q = 0; q < ndesc; ++q) {
        const int G = off[q + 1] - off[q];
        for (int t = threadIdx.x; t < G; t += blockDim.x) work[off[q] + t] = make_int2(q, t);
    }
}

// nd_run_batch without allocation: the same groups, descriptors, work maps and
// kernels as run_nets, with the tables in `scratch`, descriptors passed to the
// device as kernel arguments and chunks launched eagerly (no graph capture).
// Fixed-size host arrays only; nothing is allocated on the success path.
static nd_status run_nets_noalloc(Net* const* nets, int count, const double* dt, const int64_t* steps,
                                  const nd_observe* obs, hipStream_t st) {
    if (count > ND_NOALLOC_MAX_NETS)
        return fail(ND_ERR_INVALID_ARG, "%d networks, the no-allocation run takes at most %d", count,
                    ND_NOALLOC_MAX_NETS);
    int64_t total_work = 0;
    for (int i = 0; i < count; ++i) {
        if (!nets[i]) return fail(ND_ERR_INVALID_ARG, "handle %d is NULL", i);
        if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(ND_ERR_INVALID_ARG, "dt must be finite and > 0");
        if (steps[i] < 0) return fail(ND_ERR_INVALID_ARG, "steps must be >= 0");
        for (int k = 0; k < i; ++k)
            if (nets[k] == nets[i]) return fail(ND_ERR_INVALID_ARG, "a handle appears twice in one batch");
        if (steps[i] > 0) total_work += nets[i]->work_items();
    }
    if (total_work > ND_NOALLOC_MAX_WORK)
        return fail(ND_ERR_INVALID_ARG, "%lld work items, the no-allocation run takes at most %d",
                    (long long)total_work, ND_NOALLOC_MAX_WORK);
    unsigned char* base = nullptr;
    nd_status s = noalloc_scratch(&base);
    if (s) return s;
    for (int i = 0; i < count; ++i)
        if ((s = nets[i]->prepare_observe(steps[i], obs ? &obs[i] : nullptr, false))) return s;
    NetDesc* descs = (NetDesc*)base;
    int* counts = (int*)(base + kNaDescBytes);
    int2* works = (int2*)(base + kNaDescBytes + kNaCountBytes);
    // groups of one kernel class, in order of first appearance
    int key[ND_NOALLOC_MAX_NETS][7];
    int grp[ND_NOALLOC_MAX_NETS];
    int ngroups = 0;
    for (int i = 0; i < count; ++i) {
        grp[i] = -1;
        if (steps[i] == 0) continue;
        const Net* n = nets[i];
        const bool lattice = n->prob.topo == ND_CUBE3D || n->prob.topo == ND_BALL3D || n->prob.topo == ND_DISK2D;
        const bool ball = n->prob.topo == ND_BALL3D || n->prob.topo == ND_DISK2D;
        const int k[7] = {n->prob.model, n->prob.topo, n->prob.precision, n->cfg.tile, n->cfg.tile_y,
                          lattice ? (int)n->prob.radius : 0, ball ? n->cfg.block : 0};
        int gi = 0;
        while (gi < ngroups && std::memcmp(key[gi], k, sizeof k) != 0) ++gi;
        if (gi == ngroups) std::memcpy(key[ngroups++], k, sizeof k);
        grp[i] = gi;
    }
    int dnext = 0;
    int64_t wnext = 0;
    hipError_t e;
    for (int gi = 0; gi < ngroups; ++gi) {
        Group g{};
        g.model = key[gi][0];
        g.topo = key[gi][1];
        g.prec = key[gi][2];
        g.tile = key[gi][3];
        g.tile_y = key[gi][4];
        g.h = key[gi][5];
        g.block = key[gi][6];
        g.desc = descs + dnext;
        g.work = works + wnext;
        g.nwork = counts + gi;
        g.mv = false;
        int64_t maxsteps = 0, nwork = 0, values = 0;
        int first = -1;
        for (int i = 0; i < count; ++i) {
            if (grp[i] != gi) continue;
            if (first < 0) first = i;
            const Net* n = nets[i];
            if ((e = put_desc(g.desc + g.ndesc, n->run_desc(dt[i], steps[i]), st)) != hipSuccess)
                return hip_fail(e, "descriptor upload");
            ++g.ndesc;
            g.mv = g.mv || n->mv_start >= 0;
            nwork += n->work_items();
            values += n->prob.n * nvars_of(n->prob.model);
            maxsteps = std::max(maxsteps, steps[i]);
        }
        hipLaunchKernelGGL(k_noalloc_work, dim3(1), dim3(256), 0, st, g.desc, g.ndesc, g.work, g.nwork);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "work map");
        dnext += g.ndesc;
        wnext += nwork;
        const Net* n0 = nets[first];
        const int cfg_grid = n0->cfg.grid;
        g.grid = cfg_grid > 0 ? (int)std::min<int64_t>(cfg_grid, nwork) : (int)nwork;
        // the chunking of nd_run_batch: one chunk, or chunks of K steps where that
        // call replays a captured K-step graph (here launched directly)
        const int K = std::max(1, n0->cfg.chunk);
        const bool eager = values >= kEagerValues && !(g.topo == ND_RING && g.tile < 0);
        if (maxsteps <= K || !graphs_enabled() || eager) {
            if ((s = enqueue_chunk(g, (int)std::min<int64_t>(maxsteps, 1 << 30), st))) return s;
        } else {
            const int64_t reps = (maxsteps + K - 1) / K;
            for (int64_t r = 0; r < reps; ++r)
                if ((s = enqueue_chunk(g, K, st))) return s;
        }
    }
    for (int i = 0; i < count; ++i) {
        nets[i]->ypar ^= (int)(steps[i] & 1);
        if ((s = nets[i]->touch(st))) return s;
    }
    return ND_OK;
}

}  // namespace nd

// =================================================================== C ABI
using namespace nd;

extern "C" {

nd_status nd_create(const nd_problem* p, nd_handle* out) {
    if (!out) return fail(ND_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    nd_status s = validate_problem(p);
    if (s) return s;
    Net* n = new (std::nothrow) Net();
    if (!n) return fail(ND_ERR_OUT_OF_MEMORY, "host allocation failed");
    if ((s = n->create(p))) {
        delete n;
        return s;
    }
    *out = reinterpret_cast<nd_handle>(n);
    return ND_OK;
}

nd_status nd_footprint(const nd_problem* p, int64_t* bytes) {
    if (!bytes) return fail(ND_ERR_INVALID_ARG, "bytes is NULL");
    nd_status s = validate_problem(p);
    if (s) return s;
    if (p->topo == ND_LINKS) {  // malformed rows show up while compressing
        LinksCompressed lc;
        if ((s = compress_links(p->n, p->row_ptr, p->col, &lc))) return s;
    }
    *bytes = footprint_bytes(p, config_for(p));
    return ND_OK;
}

static Net* as_net(nd_handle h) { return reinterpret_cast<Net*>(h); }

nd_status nd_set_state(nd_handle h, const double* y, int64_t len, int32_t on_device, void* stream) {
    Net* n = as_net(h);
    if (!n || !y) return fail(ND_ERR_INVALID_ARG, "NULL handle or state");
    const int64_t want = nvars_of(n->prob.model) * n->prob.n;
    if (len != want) return fail(ND_ERR_INVALID_ARG, "state length %lld, expected %lld", (long long)len, (long long)want);
    hipStream_t st = (hipStream_t)stream;
    HIPC(hipMemcpyAsync(n->tmpl.y[n->ypar], y, len * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    HIPC(clear_status(n->status_dev, st));  // a new state starts with a clean status word
    if (!on_device) HIPC(hipStreamSynchronize(st));
    return n->touch(st);
}

// After the work enqueued on st so far: ND_ERR_NUMERIC when a stage kernel
// flagged a non-finite state value in this network (synchronises st).
static nd_status sync_status(Net* n, hipStream_t st, const char* what) {
    HIPC(hipMemcpyAsync(n->status_host, n->status_dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (*n->status_host)
        return fail(ND_ERR_NUMERIC, "%s: the state holds a non-finite value (a run produced NaN or Inf)", what);
    return ND_OK;
}

nd_status nd_get_state(nd_handle h, double* y, int64_t len, int32_t on_device, void* stream) {
    Net* n = as_net(h);
    if (!n || !y) return fail(ND_ERR_INVALID_ARG, "NULL handle or state");
    const int64_t want = nvars_of(n->prob.model) * n->prob.n;
    if (len != want) return fail(ND_ERR_INVALID_ARG, "state length %lld, expected %lld", (long long)len, (long long)want);
    hipStream_t st = (hipStream_t)stream;
    HIPC(hipMemcpyAsync(y, n->tmpl.y[n->ypar], len * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    if (!on_device) return sync_status(n, st, "nd_get_state");
    return n->touch(st);
}

nd_status nd_run(nd_handle h, double dt, int64_t steps, const nd_observe* obs, void* stream) {
    Net* n = as_net(h);
    if (!n) return fail(ND_ERR_INVALID_ARG, "NULL handle");
    return run_nets(&n, 1, &dt, &steps, obs, (hipStream_t)stream);
}

nd_status nd_run_batch(const nd_handle* hs, int32_t count, const double* dt, const int64_t* steps,
                       const nd_observe* obs, void* stream) {
    if (!hs || !dt || !steps || count < 0) return fail(ND_ERR_INVALID_ARG, "bad batch arguments");
    std::vector<Net*> nets(count);
    for (int i = 0; i < count; ++i) nets[i] = as_net(hs[i]);
    return run_nets(nets.data(), count, dt, steps, obs, (hipStream_t)stream);
}

nd_status nd_run_batch_noalloc(const nd_handle* hs, int32_t count, const double* dt, const int64_t* steps,
                               const nd_observe* obs, void* stream) {
    if (!hs || !dt || !steps || count < 0) return fail(ND_ERR_INVALID_ARG, "bad batch arguments");
    if (count > ND_NOALLOC_MAX_NETS)
        return fail(ND_ERR_INVALID_ARG, "%d networks, the no-allocation run takes at most %d", count,
                    ND_NOALLOC_MAX_NETS);
    Net* nets[ND_NOALLOC_MAX_NETS];
    for (int i = 0; i < count; ++i) nets[i] = as_net(hs[i]);
    return run_nets_noalloc(nets, count, dt, steps, obs, (hipStream_t)stream);
}

nd_status nd_get_observables(nd_handle h, double* R, int64_t r_len, double* mean_vel, int64_t mv_len,
                             int32_t on_device, void* stream) {
    Net* n = as_net(h);
    if (!n) return fail(ND_ERR_INVALID_ARG, "NULL handle");
    hipStream_t st = (hipStream_t)stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (R) {
        if (n->r_every <= 0) return fail(ND_ERR_INVALID_ARG, "the last run recorded no R");
        const int64_t want = n->last_steps / n->r_every + 1;
        if (r_len != want) return fail(ND_ERR_INVALID_ARG, "r_len %lld, expected %lld", (long long)r_len, (long long)want);
        HIPC(hipMemcpyAsync(R, n->R_dev, want * 8, kind, st));
    }
    if (mean_vel) {
        if (n->mv_start < 0) return fail(ND_ERR_INVALID_ARG, "the last run recorded no mean velocity");
        if (mv_len != n->prob.n) return fail(ND_ERR_INVALID_ARG, "mv_len must equal n");
        HIPC(hipMemcpyAsync(mean_vel, n->mv_dev, mv_len * 8, kind, st));
    }
    if (!on_device) return sync_status(n, st, "nd_get_observables");
    return n->touch(st);
}

nd_status nd_sync(nd_handle h, void* stream) {
    Net* n = as_net(h);
    if (!n) return fail(ND_ERR_INVALID_ARG, "NULL handle");
    return sync_status(n, (hipStream_t)stream, "nd_sync");
}

nd_status nd_destroy(nd_handle h) {
    Net* n = as_net(h);
    if (!n) return fail(ND_ERR_INVALID_ARG, "NULL handle");
    delete n;  // waits for the work enqueued for this network only
    return ND_OK;
}

nd_status nd_get_config(nd_handle h, nd_kernel_config* cfg) {
    Net* n = as_net(h);
    if (!n || !cfg) return fail(ND_ERR_INVALID_ARG, "NULL argument");
    *cfg = n->cfg;
    return ND_OK;
}

nd_status nd_set_config(nd_handle h, const nd_kernel_config* cfg) {
    Net* n = as_net(h);
    if (!n || !cfg) return fail(ND_ERR_INVALID_ARG, "NULL argument");
    if (cfg->grid < 0 || cfg->chunk < 1) return fail(ND_ERR_INVALID_ARG, "grid must be >= 0 and chunk >= 1");
    nd_kernel_config c = *cfg;
    const nd_problem& p = n->prob;
    if (p.topo == ND_RING) {
        RingLaunch L;
        if (!ring_select(p.model, p.precision, c.tile, &L))
            return fail(ND_ERR_INVALID_ARG, "no ring kernel for tile %d", c.tile);
        if (c.tile < 0 && -c.tile < p.n)
            return fail(ND_ERR_INVALID_ARG, "a resident ring needs n <= %d", -c.tile);
    } else if (p.topo == ND_CUBE3D) {
        const int h = (int)p.radius;
        if (c.tile < 1 || c.tile_y < 1 || c.tile_z < 1)
            return fail(ND_ERR_INVALID_ARG, "cube tile extents must be >= 1");
        c.tile = (int32_t)std::min<int64_t>(c.tile, p.n1);
        c.tile_y = (int32_t)std::min<int64_t>(c.tile_y, p.n2);
        c.tile_z = (int32_t)std::min<int64_t>(c.tile_z, p.n3);
        if ((c.tile + 2 * h) * (c.tile_y + 2 * h) > 1024)
            return fail(ND_ERR_INVALID_ARG, "cube tile: (tile+2h)*(tile_y+2h) must be <= 1024");
    } else if (p.topo == ND_BALL3D || p.topo == ND_DISK2D) {
        const int P = (int)p.radius, pz = ball_pz(p.topo, p.radius);
        if (c.tile < 1 || c.tile_y < 1 || c.tile_z < 1)
            return fail(ND_ERR_INVALID_ARG, "ball tile extents must be >= 1");
        c.tile = (int32_t)std::min<int64_t>(c.tile, p.n1);
        c.tile_y = (int32_t)std::min<int64_t>(c.tile_y, p.n2);
        c.tile_z = (int32_t)std::min<int64_t>(c.tile_z, p.n3);
        if (c.block == kBallScatterBlock) {
            if (p.topo != ND_BALL3D || !ball_scatter_available(P))
                return fail(ND_ERR_INVALID_ARG, "block %d (plane-scatter ball) is not built for this radius or topology",
                            kBallScatterBlock);
        } else if (c.block != 256 && c.block != 1024) {
            c.block = 1024;
        }
        const int rows = 4 * (c.block / 64);
        const size_t sm = c.block == kBallScatterBlock ? ball_scatter_smem_bytes(P, c.tile, c.tile_y)
                                                       : ball_smem_bytes(P, pz, c.tile, c.tile_y);
        if (c.tile + 2 * P > 64 || c.tile_y + 2 * P > rows || c.tile * c.tile_y > c.block || sm > kBallSmemMax)
            return fail(ND_ERR_INVALID_ARG, "ball tile: need tile+2P <= 64, tile_y+2P <= 4*block/64, "
                                            "tile*tile_y <= block and the prefix planes within LDS");
    } else if (p.topo == ND_LINKS) {
        if (c.tile != kLinksRows) return fail(ND_ERR_INVALID_ARG, "links work items hold %d rows (tile must be %d)",
                                              kLinksRows, kLinksRows);
    } else {
        if (c.tile != 256) return fail(ND_ERR_INVALID_ARG, "CSR work items hold 256 rows (tile must be 256)");
        if (c.tile_y < 2 || c.tile_y > 16 || (c.tile_y & (c.tile_y - 1)))
            return fail(ND_ERR_INVALID_ARG, "CSR edges per thread must be 2, 4, 8 or 16");
    }
    return n->apply_config(c);
}

const char* nd_status_str(nd_status s) {
    switch (s) {
        case ND_OK: return "ok";
        case ND_ERR_INVALID_ARG: return "invalid argument";
        case ND_ERR_OUT_OF_MEMORY: return "out of device memory";
        case ND_ERR_DEVICE: return "device error";
        case ND_ERR_NOT_READY: return "not ready";
        case ND_ERR_NUMERIC: return "non-finite value";
        case ND_ERR_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* nd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
