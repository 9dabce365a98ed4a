// Arbitrary binary coupling matrices, held in the paper's differentially
// compressed form (Sec. III.C, Alg. 2) and extracted on the fly in the stage
// kernels.
//
// Compression (host, once per network).  Row i of the coupling matrix is the
// set of positions j with L_ij = 1.  Shifted circularly left by i (position p
// goes to (p - i) mod n) and XORed with the common vector V = row 0, it leaves
// a difference vector d; the difference table keeps each distinct d once (in
// order of first appearance) and row i stores only the index C_i of its
// entry.  EXTRACT is the inverse: row i = ROR(V XOR D[C_i], i).  A
// translation-invariant topology (ring, full mesh) has a single, empty entry;
// a periodic lattice stored with the flattened index has one entry per
// boundary pattern.
//
// Evaluation (device, every stage).  The coupling sum of row i over
// V XOR D_k, shifted by i, is the sum over V shifted by i, minus the positions
// of D_k that V holds, plus those it does not:
//   sum_{j in row i} x_j = sum_{p in V} x_{i+p} + sum_{p in D_k} s_kp x_{i+p},
//   s_kp = -1 if p in V else +1   (indices mod n).
// V is stored as its positions (uniform over a workgroup: every lane walks
// the same positions from consecutive elements, so the gathers of a wave are
// contiguous, and several are in flight per lane); each entry of the table as
// its signed positions.  The exchanged values x_j = map(z_j) of the stage (Kuramoto:
// (cos z, sin z); FHN: (u, v)) are written once per element by the previous
// stage, so every gather reads one vector and no sin/cos is evaluated per
// link.  One thread per element adds its row's terms in a fixed order (V's
// positions ascending, then the entry's positions), evaluates the RHS with
// the sum divided by the row's link count, does the 13-access RK bookkeeping
// and writes the map of its next stage value.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "models.h"
#include "runtime.h"

namespace nd {

// ------------------------------------------------------------ compression
namespace {

uint64_t hash_positions(const int32_t* p, size_t m) {
    uint64_t h = 1469598103934665603ull ^ (uint64_t)m;  // FNV-1a over the positions
    for (size_t q = 0; q < m; ++q) {
        h ^= (uint32_t)p[q];
        h *= 1099511628211ull;
    }
    return h;
}

// Sorted symmetric difference of two sorted position lists.
void sym_diff(const std::vector<int32_t>& a, const std::vector<int32_t>& b, std::vector<int32_t>& out) {
    out.clear();
    size_t x = 0, y = 0;
    while (x < a.size() && y < b.size()) {
        if (a[x] < b[y]) out.push_back(a[x++]);
        else if (b[y] < a[x]) out.push_back(b[y++]);
        else ++x, ++y;
    }
    while (x < a.size()) out.push_back(a[x++]);
    while (y < b.size()) out.push_back(b[y++]);
}

}  // namespace

nd_status compress_links(int64_t n, const int64_t* row_ptr, const int32_t* col, LinksCompressed* out) {
    if (n < 1 || !row_ptr) return fail(ND_ERR_INVALID_ARG, "links: n >= 1 and row_ptr are required");
    if (row_ptr[0] != 0) return fail(ND_ERR_INVALID_ARG, "links: row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return fail(ND_ERR_INVALID_ARG, "links: row_ptr must be non-decreasing");
    if (row_ptr[n] > 0 && !col) return fail(ND_ERR_INVALID_ARG, "links: col is NULL");
    LinksCompressed& c = *out;
    c.n = n;
    c.V.clear();
    c.dptr.assign(1, 0);
    c.dpos.clear();
    c.C.assign((size_t)n, 0);
    std::vector<int32_t> r, d;
    // rotated row i: positions (j - i) mod n, ascending
    auto rotated = [&](int64_t i) -> nd_status {
        const int64_t b = row_ptr[i], e = row_ptr[i + 1];
        r.clear();
        bool sorted = true;
        for (int64_t q = b; q < e; ++q) {
            const int32_t j = col[q];
            if (j < 0 || j >= n) return fail(ND_ERR_INVALID_ARG, "links: col[%lld] = %d out of range", (long long)q, j);
            if (q > b && col[q - 1] >= j) sorted = false;
        }
        if (sorted) {
            // an ascending row stays ascending after the shift, up to a rotation:
            // the positions j >= i come first
            const int32_t* lo = std::lower_bound(col + b, col + e, (int32_t)i);
            for (const int32_t* p = lo; p != col + e; ++p) r.push_back((int32_t)(*p - i));
            for (const int32_t* p = col + b; p != lo; ++p) r.push_back((int32_t)(*p - i + n));
        } else {
            for (int64_t q = b; q < e; ++q) r.push_back((int32_t)((col[q] - i + n) % n));
            std::sort(r.begin(), r.end());
            for (size_t q = 1; q < r.size(); ++q)
                if (r[q] == r[q - 1]) return fail(ND_ERR_INVALID_ARG, "links: row %lld lists a source twice", (long long)i);
        }
        return ND_OK;
    };
    nd_status s;
    if ((s = rotated(0))) return s;
    c.V = r;
    // open-addressing table of entry indices keyed by the difference vector
    std::vector<int32_t> slot(1024, -1);
    std::vector<uint64_t> entry_hash;
    auto find_or_add = [&](const std::vector<int32_t>& v) -> int32_t {
        const uint64_t h = hash_positions(v.data(), v.size());
        size_t mask = slot.size() - 1;
        for (size_t q = h & mask;; q = (q + 1) & mask) {
            const int32_t k = slot[q];
            if (k < 0) break;
            if (entry_hash[k] == h && (size_t)(c.dptr[k + 1] - c.dptr[k]) == v.size() &&
                std::equal(v.begin(), v.end(), c.dpos.begin() + c.dptr[k]))
                return k;
        }
        const int32_t k = (int32_t)entry_hash.size();
        entry_hash.push_back(h);
        c.dpos.insert(c.dpos.end(), v.begin(), v.end());
        c.dptr.push_back((int64_t)c.dpos.size());
        if (2 * entry_hash.size() > slot.size()) {  // keep the load below 1/2
            slot.assign(slot.size() * 2, -1);
            mask = slot.size() - 1;
            for (int32_t e = 0; e < (int32_t)entry_hash.size(); ++e) {
                size_t q = entry_hash[e] & mask;
                while (slot[q] >= 0) q = (q + 1) & mask;
                slot[q] = e;
            }
        } else {
            size_t q = h & mask;
            while (slot[q] >= 0) q = (q + 1) & mask;
            slot[q] = k;
        }
        return k;
    };
    for (int64_t i = 0; i < n; ++i) {
        if ((s = rotated(i))) return s;
        sym_diff(r, c.V, d);
        c.C[(size_t)i] = find_or_add(d);
    }
    return ND_OK;
}

// Device form of the table: signed entry positions, 1 / link count per entry.
void links_device_form(const LinksCompressed& c, LinksDeviceForm* f) {
    const size_t K = c.dptr.size() - 1;
    f->dptr.assign(K + 1, 0);
    f->dsig.assign(c.dpos.size(), 0);
    f->inv.assign(K, 0.0);
    for (size_t k = 0; k < K; ++k) {
        int64_t links = (int64_t)c.V.size();
        for (int64_t q = c.dptr[k]; q < c.dptr[k + 1]; ++q) {
            const int32_t p = c.dpos[q];
            const bool in_v = std::binary_search(c.V.begin(), c.V.end(), p);
            f->dsig[q] = in_v ? (p | kLinksRemove) : p;
            links += in_v ? -1 : 1;
        }
        f->dptr[k + 1] = (int32_t)c.dptr[k + 1];
        f->inv[k] = links > 0 ? 1.0 / (double)links : 0.0;
    }
}

int64_t links_device_bytes(const LinksCompressed& c) {
    const int64_t K = (int64_t)c.dptr.size() - 1;
    return (int64_t)c.V.size() * 4 + (K + 1) * 4 + (int64_t)c.dpos.size() * 4 + K * 8 + c.n * 4;
}

// ------------------------------------------------------------------ kernels
// Clang vector types load and store through global-address-space pointers
// directly (one 16- or 8-byte access).
typedef double ldv2 __attribute__((ext_vector_type(2)));
typedef float lfv2 __attribute__((ext_vector_type(2)));

template <int MODEL, class KT>
struct LinksTypes {
    // FHN exchanges the stage values themselves (kept in double); the Kuramoto
    // models exchange (cos z, sin z) in the bulk type (exact in float for the
    // float map)
    using MT2 = typename std::conditional<MODEL == ND_FHN || sizeof(KT) == 8, ldv2, lfv2>::type;
};

template <class MT2>
__device__ __forceinline__ MT2 pack2(double2 v) {
    MT2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}

// Maps of the run's initial state (networks with g0 == 0) and, when R is
// recorded, the per-work-item sums R(0) is formed from.
template <int MODEL, class KT>
__global__ __launch_bounds__(256) void k_links_prologue(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                       const int* __restrict__ nwork_p) {
    using M = RingModel<MODEL, KT>;
    using MT2 = typename LinksTypes<MODEL, KT>::MT2;
    constexpr int V = M::V;
    __shared__ double lds[2 * 4];
    const int nwork = *nwork_p;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (d.g0 != 0 || d.nsteps <= 0) continue;
        const int64_t n = d.n;
        const int64_t i = (int64_t)wk.y * kLinksRows + threadIdx.x;
        double part[2] = {0.0, 0.0};
        if (i < n) {
            double z[V];
#pragma unroll
            for (int v = 0; v < V; ++v) z[v] = gp(d.y[d.ypar])[v * n + i];
            const double2 x = M::map(z);
            gp((MT2*)d.sx[0])[i] = pack2<MT2>(x);
            if constexpr (MODEL == ND_FHN) {
                const double r = sqrt(z[0] * z[0] + z[1] * z[1]);
                part[0] = z[0] / r;
                part[1] = z[1] / r;
            } else {
                part[0] = (double)pack2<MT2>(x).x;
                part[1] = (double)pack2<MT2>(x).y;
            }
        }
        if (d.obs & OBS_R) {
            block_sum<256, 2>(part, lds);
            if (threadIdx.x == 0) {
                gp(d.tsum[0])[2 * wk.y] = part[0];
                gp(d.tsum[0])[2 * wk.y + 1] = part[1];
            }
        }
    }
}

template <int MODEL, class KT, int STAGE, bool MV>
__global__ __launch_bounds__(256) void k_links_stage(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                    const int* __restrict__ nwork_p, int j) {
    using M = RingModel<MODEL, KT>;
    using MT2 = typename LinksTypes<MODEL, KT>::MT2;
    constexpr int V = M::V, stage = STAGE;
    __shared__ double lds[2 * 4];
    const int nwork = *nwork_p;
    const int tid = threadIdx.x;
    // neighbouring row tiles share most of their gathers: keep them on one XCD
    const int nvb = ((nwork + 7) >> 3) << 3;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int w = xcd_work(vb, nwork);
        if (w < 0) continue;
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (j >= d.nsteps) continue;  // uniform over the block
        const int64_t n = d.n, g = d.g0 + j;
        const int t = wk.y;

        // ---- order parameter R(g) from the sums of map(y_g) (stage 1, item 0)
        if (stage == 1 && t == 0 && (d.obs & OBS_R) && (g % d.r_every) == 0) {
            double s[2] = {0.0, 0.0};
            const ND_GLOBAL double* ts = gp(d.tsum[0]);
            for (int u = tid; u < d.G; u += 256) {
                s[0] += ts[2 * u];
                s[1] += ts[2 * u + 1];
            }
            block_sum<256, 2>(s, lds);
            if (tid == 0) gp(d.R)[g / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }

        const int64_t i = (int64_t)t * kLinksRows + tid;
        const bool valid = i < n;
        const int par = (d.ypar + j) & 1;
        const ND_GLOBAL double* __restrict__ y = gp(d.y[par]);
        const ND_GLOBAL KT* __restrict__ kp = stage == 1 ? nullptr : gp((const KT*)d.k[stage > 1 ? stage - 2 : 0]);
        const ND_GLOBAL MT2* __restrict__ mi = gp((const MT2*)d.sx[(stage - 1) & 1]);
        const double dt = d.dt;
        const double cdt = stage == 4 ? dt : 0.5 * dt;
        const uint32_t un = (uint32_t)n, ui = (uint32_t)(valid ? i : 0);

        // ---- coupling sum over the extracted row
        double wx = 0.0, wy = 0.0;
        double inv = 0.0;
        if (valid) {
            // the common vector's positions are uniform over the workgroup (scalar
            // loads); the gathers of consecutive positions are independent, so
            // several are in flight per lane
            const ND_GLOBAL int32_t* __restrict__ vpos = gp(d.lvpos);
            const int nv = d.lnv;
#pragma unroll 8
            for (int q = 0; q < nv; ++q) {
                uint32_t jj = ui + (uint32_t)vpos[q];
                if (jj >= un) jj -= un;
                const MT2 x = ld32(mi, jj);
                wx += (double)x.x;
                wy += (double)x.y;
            }
            const int k = ld32(gp(d.lrow), ui);
            const int e0 = ld32(gp(d.ldptr), (uint32_t)k), e1 = ld32(gp(d.ldptr), (uint32_t)k + 1);
            for (int e = e0; e < e1; ++e) {
                const int32_t v = ld32(gp(d.ldpos), (uint32_t)e);
                uint32_t jj = ui + (uint32_t)(v & ~kLinksRemove);
                if (jj >= un) jj -= un;
                const MT2 x = ld32(mi, jj);
                if (v & kLinksRemove) {
                    wx -= (double)x.x;
                    wy -= (double)x.y;
                } else {
                    wx += (double)x.x;
                    wy += (double)x.y;
                }
            }
            inv = ld32(gp(d.linv), (uint32_t)k);
        }

        double part[2] = {0.0, 0.0};
        if (valid) {
            double yv[V], kv[V], z[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                yv[v] = ld32(y + (int64_t)v * n, ui);
                kv[v] = stage == 1 ? 0.0 : (double)ld32(kp + (int64_t)v * n, ui);
                z[v] = stage == 1 ? yv[v] : fma(cdt, kv[v], yv[v]);
            }
            // the element's own map was written with its stage value (same bits)
            const MT2 own = ld32(mi, ui);
            const double2 xo = make_double2((double)own.x, (double)own.y);
            double2 W;
            if (inv != 0.0) {
                W = make_double2(wx * inv, wy * inv);
            } else {
                // no links: no coupling (FHN's coupling acts on W - x_i)
                W = MODEL == ND_FHN ? make_double2(z[0], z[V - 1]) : make_double2(0.0, 0.0);
            }
            double k[V];
            M::rhs(d, z, xo, W, k);
            double zn[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double kk = kq<KT>(k[v]);
                ND_GLOBAL double* accp = gp(d.acc) + (int64_t)v * n;
                if (stage <= 3) st32(gp((KT*)d.k[stage - 1]) + (int64_t)v * n, ui, (KT)kk);
                if (stage == 1) {
                    zn[v] = fma(0.5 * dt, kk, yv[v]);
                } else if (stage == 2) {
                    st32(accp, ui, fma(d.dt3, kk, fma(d.dt6, kv[v], yv[v])));
                    zn[v] = fma(0.5 * dt, kk, yv[v]);
                } else if (stage == 3) {
                    zn[v] = fma(dt, kk, yv[v]);
                } else {
                    const double yo = fma(d.dt6, kk, fma(d.dt3, kv[v], ld32(accp, ui)));
                    st32(gp(d.y[par ^ 1]) + (int64_t)v * n, ui, yo);
                    flag_nonfinite(d, yo);
                    zn[v] = yo;
                }
            }
            const MT2 xn = pack2<MT2>(M::map(zn));
            st32(gp((MT2*)d.sx[stage & 1]), ui, xn);
            if (stage == 4 && (d.obs & OBS_R)) {
                if constexpr (MODEL == ND_FHN) {
                    const double r = sqrt(zn[0] * zn[0] + zn[1] * zn[1]);
                    part[0] = zn[0] / r;
                    part[1] = zn[1] / r;
                } else {
                    part[0] = (double)xn.x;
                    part[1] = (double)xn.y;
                }
            }
            // mean phase velocity (compiled only into the MV variants)
            if (MV && (d.obs & OBS_MV) && g >= d.mv_start) {
                if constexpr (MODEL != ND_FHN) {  // phase models: unwrapped phase is variable 0
                    if (stage == 1 && g == d.mv_start) st32(gp(d.mv), ui, yv[0]);
                } else if (stage == 4) {
                    const double uo = yv[0], vo = yv[V - 1], un_ = zn[0], vn = zn[V - 1];
                    const double dth = atan2(uo * vn - vo * un_, uo * un_ + vo * vn);
                    st32(gp(d.mv), ui, (g == d.mv_start ? 0.0 : ld32(gp(d.mv), ui)) + dth);
                }
            }
        }
        if (stage == 4 && (d.obs & OBS_R)) {
            block_sum<256, 2>(part, lds);
            if (tid == 0) {
                gp(d.tsum[0])[2 * t] = part[0];
                gp(d.tsum[0])[2 * t + 1] = part[1];
            }
        }
    }
}

// After the last step of a run: R at the final step and the mean phase velocity.
template <int MODEL>
__global__ __launch_bounds__(256) void k_links_final(const NetDesc* __restrict__ D, const int2* __restrict__ work,
                                                    const int* __restrict__ nwork_p, int chunk) {
    __shared__ double lds[2 * 4];
    const int nwork = *nwork_p;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 wk = work[w];
        const NetDesc& d = D[wk.x];
        if (d.nsteps <= 0 || d.nsteps > chunk) continue;
        const int64_t n = d.n, gend = d.g0 + d.nsteps;
        if (wk.y == 0 && (d.obs & OBS_R) && (gend % d.r_every) == 0) {
            double s[2] = {0.0, 0.0};
            for (int u = threadIdx.x; u < d.G; u += 256) {
                s[0] += d.tsum[0][2 * u];
                s[1] += d.tsum[0][2 * u + 1];
            }
            block_sum<256, 2>(s, lds);
            if (threadIdx.x == 0) d.R[gend / d.r_every] = sqrt(s[0] * s[0] + s[1] * s[1]) / (double)n;
        }
        if (d.obs & OBS_MV) {
            const int64_t i = (int64_t)wk.y * kLinksRows + threadIdx.x;
            if (i < n) {
                const double* y = d.y[(d.ypar + (int)d.nsteps) & 1];
                if constexpr (MODEL != ND_FHN)
                    d.mv[i] = (y[i] - d.mv[i]) * d.mv_scale;
                else
                    d.mv[i] = d.mv[i] * d.mv_scale;
            }
        }
    }
}

// ------------------------------------------------------------------ launch
template <int MODEL, class KT>
static void links_entry(LinksLaunch* r) {
    r->prologue = k_links_prologue<MODEL, KT>;
    r->stage[0] = k_links_stage<MODEL, KT, 1, false>;
    r->stage[1] = k_links_stage<MODEL, KT, 2, false>;
    r->stage[2] = k_links_stage<MODEL, KT, 3, false>;
    r->stage[3] = k_links_stage<MODEL, KT, 4, false>;
    r->stage_mv[0] = k_links_stage<MODEL, KT, 1, true>;
    r->stage_mv[1] = k_links_stage<MODEL, KT, 2, true>;
    r->stage_mv[2] = k_links_stage<MODEL, KT, 3, true>;
    r->stage_mv[3] = k_links_stage<MODEL, KT, 4, true>;
    r->final = k_links_final<MODEL>;
}

bool links_select(int model, int prec, LinksLaunch* out) {
    const bool f64 = prec == ND_FP64;
    switch (model) {
        case ND_KURAMOTO: f64 ? links_entry<ND_KURAMOTO, double>(out) : links_entry<ND_KURAMOTO, float>(out); return true;
        case ND_KURAMOTO_INERTIA:
            f64 ? links_entry<ND_KURAMOTO_INERTIA, double>(out) : links_entry<ND_KURAMOTO_INERTIA, float>(out);
            return true;
        case ND_FHN: f64 ? links_entry<ND_FHN, double>(out) : links_entry<ND_FHN, float>(out); return true;
        default: return false;
    }
}

size_t links_map_bytes(int model, int prec) {
    return model == ND_FHN || prec == ND_FP64 ? 16 : 8;
}

hipError_t links_launch_chunk(const LinksLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                              const int* nwork, int chunk, bool mv) {
    hipLaunchKernelGGL(L.prologue, dim3(grid), dim3(256), 0, s, D, work, nwork);
    hipError_t e = hipGetLastError();
    for (int j = 0; j < chunk && e == hipSuccess; ++j)
        for (int st = 0; st < 4 && e == hipSuccess; ++st) {
            hipLaunchKernelGGL(mv ? L.stage_mv[st] : L.stage[st], dim3(grid), dim3(256), 0, s, D, work, nwork, j);
            e = hipGetLastError();
        }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(L.final, dim3(grid), dim3(256), 0, s, D, work, nwork, chunk);
    return hipGetLastError();
}

}  // namespace nd

// =================================================================== C ABI
extern "C" nd_status nd_compress_links(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t* V,
                                       int64_t v_cap, int64_t* d_ptr, int64_t d_ptr_cap, int32_t* d_pos,
                                       int64_t d_pos_cap, int32_t* C, int64_t c_cap, nd_links_info* info) {
    using namespace nd;
    if (!info) return fail(ND_ERR_INVALID_ARG, "info is NULL");
    if (n >= (int64_t(1) << 29)) return fail(ND_ERR_INVALID_ARG, "links: n must be < 2^29");
    LinksCompressed c;
    nd_status s = compress_links(n, row_ptr, col, &c);
    if (s) return s;
    const int64_t K = (int64_t)c.dptr.size() - 1;
    std::memset(info, 0, sizeof *info);
    info->v_bits = (int64_t)c.V.size();
    info->entries = K;
    info->d_bits = (int64_t)c.dpos.size();
    info->bytes = links_device_bytes(c);
    for (size_t q = 0; q < c.V.size(); ++q) info->runs += (q == 0 || c.V[q] != c.V[q - 1] + 1);
    if (V) {
        if (v_cap < info->v_bits) return fail(ND_ERR_INVALID_ARG, "V holds %lld, need %lld", (long long)v_cap, (long long)info->v_bits);
        std::copy(c.V.begin(), c.V.end(), V);
    }
    if (d_ptr) {
        if (d_ptr_cap < K + 1) return fail(ND_ERR_INVALID_ARG, "d_ptr holds %lld, need %lld", (long long)d_ptr_cap, (long long)(K + 1));
        std::copy(c.dptr.begin(), c.dptr.end(), d_ptr);
    }
    if (d_pos) {
        if (d_pos_cap < info->d_bits)
            return fail(ND_ERR_INVALID_ARG, "d_pos holds %lld, need %lld", (long long)d_pos_cap, (long long)info->d_bits);
        std::copy(c.dpos.begin(), c.dpos.end(), d_pos);
    }
    if (C) {
        if (c_cap < n) return fail(ND_ERR_INVALID_ARG, "C holds %lld, need %lld", (long long)c_cap, (long long)n);
        std::copy(c.C.begin(), c.C.end(), C);
    }
    return ND_OK;
}
