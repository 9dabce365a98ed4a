// Host paths of libnd under AddressSanitizer and UndefinedBehaviorSanitizer,
// built from the library sources with host code only (no device code, no GPU):
// argument validation, footprints, the differential compression of coupling
// matrices, the server's queue (submit, reject, cancel, a pump that admits
// nothing), the tuning cache file.  Exits non-zero on the first failed check;
// the sanitizers abort on the first error they find.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "nd.h"

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static nd_problem ring(int model, int64_t n, int64_t P) {
    nd_problem p;
    std::memset(&p, 0, sizeof p);
    p.model = model;
    p.topo = ND_RING;
    p.n = n;
    p.radius = P;
    if (model == ND_FHN)  // eps, a, sigma, phi
        p.params[0] = 0.05, p.params[1] = 0.5, p.params[2] = 0.1, p.params[3] = 1.4707963267948966;
    else  // omega, mu, alpha
        p.params[0] = 0.0, p.params[1] = 1.0, p.params[2] = 1.46;
    return p;
}

// random binary coupling matrix in CSR-by-row form: density q, optional self links
static void random_links(std::mt19937_64& g, int64_t n, double q, std::vector<int64_t>& rp, std::vector<int32_t>& col) {
    std::uniform_real_distribution<double> u(0.0, 1.0);
    rp.assign(1, 0);
    col.clear();
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j)
            if (u(g) < q) col.push_back((int32_t)j);
        rp.push_back((int64_t)col.size());
    }
}

int main() {
    // ---- status strings and validation before any device work
    CHECK(std::strcmp(nd_status_str(ND_OK), "ok") == 0);
    nd_handle h = nullptr;
    nd_problem bad = ring(ND_KURAMOTO, 10, 5);  // 2P+1 > n
    CHECK(nd_create(&bad, &h) == ND_ERR_INVALID_ARG && h == nullptr);
    CHECK(std::strlen(nd_last_error()) > 0);
    bad = ring(ND_KURAMOTO, 10, 0);
    CHECK(nd_create(&bad, &h) == ND_ERR_INVALID_ARG);
    bad = ring(ND_HH, 10, 2);  // HH needs a CSR graph
    CHECK(nd_create(&bad, &h) == ND_ERR_INVALID_ARG);
    bad = ring(ND_KURAMOTO, 1000, 10);
    bad.params[1] = NAN;
    CHECK(nd_create(&bad, &h) == ND_ERR_INVALID_ARG);
    CHECK(nd_create(nullptr, &h) == ND_ERR_INVALID_ARG);

    // ---- footprints of every topology
    int64_t bytes = 0;
    nd_problem p = ring(ND_FHN, 65536, 22937);
    CHECK(nd_footprint(&p, &bytes) == ND_OK && bytes > 65536 * 2 * 8 * 6);
    nd_problem c;
    std::memset(&c, 0, sizeof c);
    c.model = ND_KURAMOTO, c.topo = ND_CUBE3D, c.n1 = c.n2 = c.n3 = 20, c.n = 8000, c.radius = 4;
    c.params[1] = 1.0;
    CHECK(nd_footprint(&c, &bytes) == ND_OK && bytes > 0);
    c.topo = ND_BALL3D;
    c.radius = 2;
    c.model = ND_KURAMOTO_INERTIA;
    c.params[3] = 1.0, c.params[4] = 0.05;
    CHECK(nd_footprint(&c, &bytes) == ND_OK && bytes > 0);
    c.n1 = 20, c.n2 = 17, c.n3 = 1, c.n = 340, c.topo = ND_DISK2D;
    CHECK(nd_footprint(&c, &bytes) == ND_OK && bytes > 0);
    {
        std::vector<int64_t> rp{0};
        std::vector<int32_t> col;
        std::vector<double> w, iapp(300, 10.0);
        std::mt19937_64 g(3);
        for (int i = 0; i < 300; ++i) {
            for (int k = 0; k < 7; ++k) {
                col.push_back((int32_t)((i * 13 + k * 41) % 300));
                w.push_back(0.01 * k);
            }
            rp.push_back((int64_t)col.size());
        }
        nd_problem hh;
        std::memset(&hh, 0, sizeof hh);
        hh.model = ND_HH, hh.topo = ND_CSR, hh.n = 300, hh.row_ptr = rp.data(), hh.col = col.data();
        hh.weight = w.data(), hh.nnz = (int64_t)col.size(), hh.per_elem = iapp.data();
        const double prm[10] = {1.0, 120.0, 36.0, 0.3, 50.0, -77.0, -54.387, 0.0, 0.0, 2.0};
        std::memcpy(hh.params, prm, sizeof prm);
        CHECK(nd_footprint(&hh, &bytes) == ND_OK && bytes > 0);
        col[5] = 300;  // source out of range
        CHECK(nd_create(&hh, &h) == ND_ERR_INVALID_ARG);
    }

    // ---- differential compression of binary coupling matrices (Alg. 2)
    std::mt19937_64 g(7);
    for (int64_t n : {1, 2, 17, 64, 200}) {
        for (double q : {0.0, 0.05, 0.5, 1.0}) {
            std::vector<int64_t> rp;
            std::vector<int32_t> col;
            random_links(g, n, q, rp, col);
            nd_links_info info;
            CHECK(nd_compress_links(n, rp.data(), col.data(), nullptr, 0, nullptr, 0, nullptr, 0, nullptr, 0, &info) ==
                  ND_OK);
            std::vector<int32_t> V(info.v_bits + 1), dpos(info.d_bits + 1), C(n);
            std::vector<int64_t> dptr(info.entries + 1);
            CHECK(nd_compress_links(n, rp.data(), col.data(), V.data(), (int64_t)V.size(), dptr.data(),
                                    (int64_t)dptr.size(), dpos.data(), (int64_t)dpos.size(), C.data(), n,
                                    &info) == ND_OK);
            // extraction: row i = shift (V xor D[C[i]]) right by i, must equal row i of the input
            for (int64_t i = 0; i < n; ++i) {
                std::vector<char> bits(n, 0), want(n, 0);
                for (int64_t k = 0; k < info.v_bits; ++k) bits[V[k]] ^= 1;
                const int32_t e = C[i];
                CHECK(e >= 0 && e < info.entries);
                for (int64_t k = dptr[e]; k < dptr[e + 1]; ++k) bits[dpos[k]] ^= 1;
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) want[col[k]] = 1;
                for (int64_t pidx = 0; pidx < n; ++pidx) CHECK(bits[pidx] == want[(pidx + i) % n]);
            }
            if (info.v_bits > 0) {  // arrays one short are refused
                CHECK(nd_compress_links(n, rp.data(), col.data(), V.data(), info.v_bits - 1, dptr.data(),
                                        (int64_t)dptr.size(), dpos.data(), (int64_t)dpos.size(), C.data(), n,
                                        &info) == ND_ERR_INVALID_ARG);
            }
        }
    }
    {  // a source listed twice is refused
        std::vector<int64_t> rp{0, 2, 2};
        std::vector<int32_t> col{1, 1};
        nd_links_info info;
        CHECK(nd_compress_links(2, rp.data(), col.data(), nullptr, 0, nullptr, 0, nullptr, 0, nullptr, 0, &info) ==
              ND_ERR_INVALID_ARG);
    }

    // ---- the server's queue on the host: nothing here starts device work
    nd_server_config sc;
    std::memset(&sc, 0, sizeof sc);
    sc.hbm_budget_bytes = 1 << 20, sc.max_slots = 4, sc.chunk_steps = 16;
    nd_server_h s = nullptr;
    sc.max_slots = 0;
    CHECK(nd_server_create(&sc, &s) == ND_ERR_INVALID_ARG);
    sc.max_slots = 4;
    sc.grid = 12;
    CHECK(nd_server_create(&sc, &s) == ND_ERR_INVALID_ARG);
    sc.grid = 0;
    CHECK(nd_server_create(&sc, &s) == ND_OK);
    std::vector<double> y0(1024);
    for (int i = 0; i < 1024; ++i) y0[i] = std::sin(0.37 * i);
    nd_problem k = ring(ND_KURAMOTO, 1024, 256);
    std::vector<nd_req> ids;
    for (int r = 0; r < 6; ++r) {
        nd_req id = 0;
        CHECK(nd_server_submit(s, &k, y0.data(), 1024, 0.01, 10 + r, nullptr, 0.0, &id) == ND_OK);
        ids.push_back(id);
    }
    nd_req id = 0;
    CHECK(nd_server_submit(s, &k, y0.data(), 1000, 0.01, 10, nullptr, 0.0, &id) == ND_ERR_INVALID_ARG);
    CHECK(nd_server_submit(s, &k, y0.data(), 1024, 0.0, 10, nullptr, 0.0, &id) == ND_ERR_INVALID_ARG);
    y0[17] = NAN;
    CHECK(nd_server_submit(s, &k, y0.data(), 1024, 0.01, 10, nullptr, 0.0, &id) == ND_ERR_NUMERIC);
    y0[17] = 0.5;
    nd_problem big = ring(ND_KURAMOTO, 1 << 20, 1000);
    std::vector<double> yb((size_t)1 << 20, 0.0);
    CHECK(nd_server_submit(s, &big, yb.data(), 1 << 20, 0.01, 10, nullptr, 0.0, &id) == ND_ERR_INVALID_ARG);
    for (nd_req r : ids) CHECK(nd_server_cancel(s, r) == ND_OK);
    int64_t pending = -1;
    CHECK(nd_server_pump(s, nullptr, &pending) == ND_OK && pending == 0);
    nd_request_info info;
    for (nd_req r : ids) {
        CHECK(nd_server_info(s, r, &info) == ND_OK && info.state == ND_REQ_CANCELLED);
        CHECK(nd_server_result(s, r, y0.data(), 1024, nullptr, 0) == ND_ERR_NOT_READY);
    }
    CHECK(nd_server_info(s, 999999, &info) == ND_ERR_INVALID_ARG);
    nd_server_counters st;
    CHECK(nd_server_stats(s, &st) == ND_OK && st.submitted == 6 && st.cancelled == 6 && st.queued == 0);
    for (int r = 0; r < 3; ++r) CHECK(nd_server_submit(s, &k, y0.data(), 1024, 0.01, 5, nullptr, -1.0, &id) == ND_OK);
    CHECK(nd_server_destroy(s) == ND_OK);  // with requests still queued

    // ---- tuning cache file round trip
    const char* path = "tune_cache.txt";
    std::FILE* f = std::fopen(path, "w");
    CHECK(f != nullptr);
    std::fprintf(f, "# arch model topo precision log2n width h tile block grid chunk tile_y tile_z\n");
    std::fprintf(f, "gfx950 1 0 0 16 2 0 512 128 0 64 0 0\n");
    std::fprintf(f, "gfx950 0 1 1 23 0 4 24 832 0 32 24 100\n");
    std::fclose(f);
    CHECK(nd_tune_clear() == ND_OK);
    CHECK(nd_tune_load(path) == ND_OK);
    CHECK(nd_tune_save(path) == ND_OK);
    CHECK(nd_tune_load(path) == ND_OK);
    CHECK(nd_tune_load("does-not-exist.txt") != ND_OK);
    CHECK(nd_tune_clear() == ND_OK);
    std::remove(path);
    std::printf("host paths clean\n");
    return 0;
}
