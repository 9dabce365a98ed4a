// Autotuner: times candidate kernel configurations of a problem on the device
// and caches the fastest per (architecture, model, topology, precision, size
// bucket, coupling-width bucket, half-width).  nd_create consults the cache.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.h"

namespace nd {

#define HIPC(expr)                                        \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

using TuneKey = std::tuple<std::string, int, int, int, int, int, int>;

static std::mutex g_tune_mu;
static std::map<TuneKey, nd_kernel_config>& cache() {
    static std::map<TuneKey, nd_kernel_config> m;
    return m;
}

static std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

static int log2_bucket(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

static TuneKey tune_key(const nd_problem* p, const std::string& arch) {
    // ring: width bucket = floor(8 P / n) (P/n in eighths); cube: half-width h
    const int wb = p->topo == ND_RING ? (int)(8 * p->radius / p->n) : 0;
    const int h = p->topo == ND_CUBE3D || p->topo == ND_BALL3D || p->topo == ND_DISK2D ? (int)p->radius : 0;
    return TuneKey(arch, p->model, p->topo, p->precision, log2_bucket(p->n), wb, h);
}

bool tuned_config(const nd_problem* p, nd_kernel_config* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (cache().empty()) return false;
    auto it = cache().find(tune_key(p, arch_name()));
    if (it == cache().end()) return false;
    *out = it->second;
    return true;
}

static std::vector<nd_kernel_config> candidates(const nd_problem* p) {
    std::vector<nd_kernel_config> v;
    nd_kernel_config base = default_config(p);
    if (p->topo == ND_RING) {
        for (int t : {128, 256, 512, 1024, 2048}) {
            nd_kernel_config c = base;
            c.tile = t;
            v.push_back(c);
        }
    } else if (p->topo == ND_CUBE3D) {
        const int h = (int)p->radius;
        v.push_back(base);  // the cost-model tiling (one round of workgroups where possible)
        const int shapes[][2] = {{20, 20}, {24, 24}, {32, 16}, {16, 16}, {40, 10}, {25, 20}};
        for (auto& sh : shapes) {
            if ((sh[0] + 2 * h) * (sh[1] + 2 * h) > 1024) continue;
            for (int cz : {base.tile_z, 40, 100}) {
                nd_kernel_config c = base;
                c.tile = (int)std::min<int64_t>(sh[0], p->n1);
                c.tile_y = (int)std::min<int64_t>(sh[1], p->n2);
                c.tile_z = (int)std::min<int64_t>(cz, p->n3);
                v.push_back(c);
            }
        }
    } else if (p->topo == ND_BALL3D || p->topo == ND_DISK2D) {
        std::vector<nd_kernel_config> bases{base};  // the cost-model tiling
        if (base.block == kBallScatterBlock) bases.push_back(ball_gather_config(p));  // and the gather form's
        for (const nd_kernel_config& b : bases) {
            v.push_back(b);
            for (int cz : {b.tile_z * 2, (b.tile_z + 1) / 2}) {
                nd_kernel_config c = b;
                c.tile_z = (int)std::max<int64_t>(1, std::min<int64_t>(cz, p->n3));
                v.push_back(c);
            }
        }
    } else if (p->topo == ND_LINKS) {
        v.push_back(base);  // one kernel shape
    } else {
        for (int l : {4, 8, 16}) {
            nd_kernel_config c = base;
            c.tile_y = l;
            v.push_back(c);
        }
    }
    return v;
}

nd_status tune(const nd_problem* p, const double* y0, int64_t len, double dt, int32_t steps, hipStream_t st,
               nd_kernel_config* best, double* best_ms) {
    nd_status s = validate_problem(p);
    if (s) return s;
    if (!y0 || len != nvars_of(p->model) * p->n) return fail(ND_ERR_INVALID_ARG, "y0 must hold nvars*n values");
    if (steps < 1 || !(dt > 0.0)) return fail(ND_ERR_INVALID_ARG, "steps >= 1 and dt > 0 required");
    Net* n = new (std::nothrow) Net();
    if (!n) return fail(ND_ERR_OUT_OF_MEMORY, "host allocation failed");
    if ((s = n->create(p))) {
        delete n;
        return s;
    }
    double best_t = 1e300;
    nd_kernel_config best_c = n->cfg;
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    for (const nd_kernel_config& c : candidates(p)) {
        if ((s = n->apply_config(c))) break;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && !s; ++rep) {  // the first repetition warms up
            hipError_t e = hipMemcpyAsync(n->tmpl.y[n->ypar], y0, len * 8, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) s = hip_fail(e, "state upload");
            if (!s) e = hipEventRecord(e0, st);
            int64_t sx = steps;
            if (!s) s = run_nets(&n, 1, &dt, &sx, nullptr, st);
            if (!s) e = hipEventRecord(e1, st);
            if (!s) e = hipEventSynchronize(e1);
            if (!s && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (!s && e != hipSuccess) s = hip_fail(e, "timing");
        }
        if (s) break;
        const double per = ms / steps;
        if (per < best_t) {
            best_t = per;
            best_c = n->cfg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    delete n;
    if (s) return s;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        cache()[tune_key(p, arch_name())] = best_c;
    }
    if (best) *best = best_c;
    if (best_ms) *best_ms = best_t;
    return ND_OK;
}

}  // namespace nd

using namespace nd;

extern "C" {

nd_status nd_tune(const nd_problem* p, const double* y0, int64_t len, double dt, int32_t steps, void* stream,
                  nd_kernel_config* best, double* best_ms) {
    return tune(p, y0, len, dt, steps, (hipStream_t)stream, best, best_ms);
}

nd_status nd_tune_save(const char* path) {
    if (!path) return fail(ND_ERR_INVALID_ARG, "NULL path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE* f = fopen(path, "w");
    if (!f) return fail(ND_ERR_INVALID_ARG, "cannot write %s", path);
    fprintf(f, "# arch model topo precision log2n width h tile block grid chunk tile_y tile_z\n");
    for (auto& kv : cache()) {
        const TuneKey& k = kv.first;
        const nd_kernel_config& c = kv.second;
        fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k),
                std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), c.tile, c.block, c.grid, c.chunk,
                c.tile_y, c.tile_z);
    }
    fclose(f);
    return ND_OK;
}

nd_status nd_tune_load(const char* path) {
    if (!path) return fail(ND_ERR_INVALID_ARG, "NULL path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(ND_ERR_INVALID_ARG, "cannot read %s", path);
    std::map<TuneKey, nd_kernel_config> m;
    char line[512];
    int lineno = 0;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[64];
        int v[12];
        nd_kernel_config c{};
        if (sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d %d", arch, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                   &c.tile, &c.block, &c.grid, &c.chunk, &c.tile_y, &c.tile_z) != 13) {
            fclose(f);
            return fail(ND_ERR_INVALID_ARG, "%s:%d: malformed entry", path, lineno);
        }
        m[TuneKey(arch, v[0], v[1], v[2], v[3], v[4], v[5])] = c;
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& kv : m) cache()[kv.first] = kv.second;
    return ND_OK;
}

nd_status nd_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    cache().clear();
    return ND_OK;
}

}  // extern "C"
