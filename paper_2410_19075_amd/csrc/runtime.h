// Host-side internals of libnd shared by the runtime, the kernels' launchers,
// the batch scheduler and the autotuner.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "nd.h"
#include "nd_dev.h"

namespace nd {

nd_status fail(nd_status s, const char* fmt, ...);
nd_status hip_fail(hipError_t e, const char* what);
int nvars_of(int model);
nd_status validate_problem(const nd_problem* p);
nd_kernel_config default_config(const nd_problem* p);
int device_cu_count();
bool tuned_config(const nd_problem* p, nd_kernel_config* out);
// The configuration nd_create gives `p`: the autotuner's cached entry when there
// is one, else the default.  Footprints and admission use the same resolution.
nd_kernel_config config_for(const nd_problem* p);
int ring_block(int tile);
int64_t footprint_bytes(const nd_problem* p, const nd_kernel_config& c);

// An event recorded once behind a batch's work and shared by its networks (one
// record per batch instead of one per network).
struct RunEvent {
    hipEvent_t ev = nullptr;
    ~RunEvent();
};

// A network handle (nd_handle).
struct Net {
    nd_problem prob{};        // copy without host pointers
    nd_kernel_config cfg{};
    NetDesc tmpl{};           // device pointers and derived constants
    int ypar = 0;             // y buffer holding the current state
    int64_t last_steps = 0;
    int64_t r_every = 0;
    int64_t mv_start = -1;
    double* R_dev = nullptr;
    int64_t R_cap = 0;
    double* mv_dev = nullptr;
    NetDesc* solo_desc = nullptr;  // launch arrays for running this network alone
    int2* solo_work = nullptr;
    int* solo_count = nullptr;
    int32_t* status_dev = nullptr;   // status word the stage kernels flag (non-finite state)
    int32_t* status_host = nullptr;  // pinned copy, read after a synchronising call
    hipEvent_t last_ev = nullptr;    // recorded after the last work enqueued for this network alone
    std::shared_ptr<RunEvent> batch_ev;  // else the event of the batch that last ran it
    bool ev_recorded = false;
    // chunk graph of this network alone, replayed by every nd_run with the same
    // chunk length, grid and mean-velocity setting (rebuilt when the config changes)
    hipGraphExec_t solo_graph[2] = {nullptr, nullptr};
    int solo_graph_key[2][2] = {{0, 0}, {0, 0}};
    std::vector<void*> allocs;
    // Buffers come from the device's stream-ordered pool.  Networks the server
    // owns allocate and free on `astream`, enqueue their set-up copies on it and
    // use a pinned status word the owner supplies; others allocate on the
    // library's own stream and free there after their last work (free_buf).
    hipStream_t astream = nullptr;
    bool own_status_host = true;
    int dev = 0;  // device the network's buffers live on

    ~Net();
    // wait until the device no longer uses this network's buffers
    void quiesce();
    // mark the network's buffers as used by the work enqueued on st so far
    nd_status touch(hipStream_t st);
    // the same, through an event already recorded behind a batch holding this network
    void touch_shared(const std::shared_ptr<RunEvent>& ev);
    void drop_graphs();
    nd_status alloc(void** ptr, size_t bytes);
    void free_buf(void* ptr);
    nd_status create(const nd_problem* p);
    nd_status apply_config(const nd_kernel_config& c);
    int64_t work_items() const;
    void append_work(int desc_index, std::vector<int2>& wk) const;
    nd_status prepare_observe(int64_t steps, const nd_observe* obs, bool may_alloc = true);
    NetDesc run_desc(double dt, int64_t steps) const;
    // chunked runs (serving): the run's step counter lives on the host and each
    // chunk's descriptor starts where the previous chunk stopped
    double run_dt = 0.0;
    int64_t run_total = 0, run_done = 0;
    nd_status begin_run(double dt, int64_t steps, const nd_observe* obs);
    NetDesc chunk_desc() const;
};

// Networks of one kernel class launched together.
struct Group {
    int model, topo, prec, tile;
    int tile_y, h;  // cube: y tile extent and half-width (kernel shape)
    int block;      // ball: workgroup size (256 or 1024)
    bool mv;        // some network records the mean phase velocity
    int ndesc;
    int grid;
    NetDesc* desc;  // device
    int2* work;     // device
    int* nwork;     // device
};

nd_status enqueue_chunk(const Group& g, int chunk, hipStream_t st);
// Write one descriptor into device memory in stream order (the value travels as a
// kernel argument, so no host buffer has to outlive the call).
hipError_t put_desc(NetDesc* dst, const NetDesc& d, hipStream_t st);
// Clear a network's status word in stream order.
hipError_t clear_status(int32_t* status, hipStream_t st);
nd_status capture_chunk(const Group& g, int K, hipGraphExec_t* out);
bool graphs_enabled();
nd_status run_nets(Net* const* nets, int count, const double* dt, const int64_t* steps, const nd_observe* obs,
                   hipStream_t st);

// ring kernels (ring.hip)
struct RingLaunch {
    void (*prologue)(const NetDesc*, const int2*, const int*);
    void (*stage[4])(const NetDesc*, const int2*, const int*, int);
    void (*stage_mv[4])(const NetDesc*, const int2*, const int*, int);  // with mean-velocity recording
    void (*epilogue)(const NetDesc*, const int2*, const int*, int);
    void (*resident)(const NetDesc*, const int2*, const int*, int);  // whole ring per workgroup
    void (*resident_mv)(const NetDesc*, const int2*, const int*, int);
    int bs, tile;
    size_t smem;
};
bool ring_select(int model, int prec, int tile, RingLaunch* out);
hipError_t ring_launch_prologue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork);
hipError_t ring_launch_stage(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                             const int* nwork, int stage, int j, bool mv);
hipError_t ring_launch_resident(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork, int chunk, bool mv);
hipError_t ring_launch_epilogue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork, int chunk);

// cube kernels (cube.hip)
struct CubeLaunch {
    void (*stage[4])(const NetDesc*, const int2*, const int*, int);
    void (*stage_mv[4])(const NetDesc*, const int2*, const int*, int);
    void (*final_partials)(const NetDesc*, const int2*, const int*, int);
    void (*final_R)(const NetDesc*, const int2*, const int*, int);
};
bool cube_select(int model, int prec, int h, CubeLaunch* out);
// Ball neighbourhood (3D lattice, radius P <= kBallMaxP): workgroups of 256 or
// 1024 threads (up to 4 halo rows per wave, one output per thread); LDS =
// ball_smem_bytes.
constexpr int kBallMaxP = 8;
bool ball_select(int model, int prec, int block, CubeLaunch* out);
size_t ball_smem_bytes(int P, int pz, int cx, int cy);
// Ball in plane-scatter form (ball.hip): 3D balls of the radii it is built for,
// workgroups of kBallScatterBlock threads (config block = kBallScatterBlock
// selects it), halo rows of HX = cx + 2P <= 64 lanes, HY = cy + 2P <= 32, one
// output per thread, two prefix planes in LDS (ball_scatter_smem_bytes).
constexpr int kBallScatterBlock = 512;
constexpr int kBallScatterPairedMaxP = 6;  // radii built for two workgroups per CU
bool ball_scatter_available(int P);
bool ball_scatter_select(int model, int prec, int P, CubeLaunch* out);
size_t ball_scatter_smem_bytes(int P, int cx, int cy);
// The gather form's configuration for a ball or disk problem (the tuner's
// alternative where the default is the plane-scatter form).
nd_kernel_config ball_gather_config(const nd_problem* p);
inline int ball_pz(int topo, int64_t P) { return topo == ND_DISK2D ? 0 : (int)P; }
constexpr size_t kBallSmemMax = 156 * 1024;  // LDS for the prefix ring (160 KB per CU, minus statics)
int64_t ball_points(int64_t P);
int64_t disk_points(int64_t P);
// LDS buffers per array of the cube stage kernel: 3 in its pipelined schedule
// (FP64: the one-variable model, and the inertia model for h <= 2), else 2
int cube_lds_buffers(int model, int prec, int h);
size_t cube_smem_bytes(int h, int cx, int cy, int nb);
int cube_block(int h, int cx, int cy);
hipError_t cube_launch_stage(const CubeLaunch& L, int grid, int block, size_t smem, hipStream_t s, NetDesc* D,
                             const int2* work, const int* nwork, int stage, int j, bool mv);
hipError_t cube_launch_final(const CubeLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                             const int* nwork, int chunk);

// CSR kernels (csr.hip): work items of 256 target rows
struct CsrLaunch {
    void (*gather)(const NetDesc*, const int2*, const int*, int, int);
    void (*update[4])(const NetDesc*, const int2*, const int*, int);
    void (*prologue)(const NetDesc*, const int2*, const int*);
};
bool csr_select(int prec, int ept, CsrLaunch* out);
hipError_t csr_launch_prologue(const CsrLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                               const int* nwork);
hipError_t csr_launch_stage(const CsrLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                            const int* nwork, int stage, int j);

// Binary coupling matrices in the paper's compressed form (links.hip)
struct LinksCompressed {
    int64_t n = 0;
    std::vector<int32_t> V;     // common vector: sorted positions of row 0
    std::vector<int64_t> dptr;  // difference table: entry k at [dptr[k], dptr[k+1]) of dpos
    std::vector<int32_t> dpos;  // sorted positions of every entry
    std::vector<int32_t> C;     // entry of every row
};
struct LinksDeviceForm {
    std::vector<int32_t> dptr;  // as LinksCompressed::dptr
    std::vector<int32_t> dsig;  // positions, | kLinksRemove where V holds the position
    std::vector<double> inv;    // 1 / link count per entry (0 for an empty row)
};
nd_status compress_links(int64_t n, const int64_t* row_ptr, const int32_t* col, LinksCompressed* out);
void links_device_form(const LinksCompressed& c, LinksDeviceForm* f);
int64_t links_device_bytes(const LinksCompressed& c);
struct LinksLaunch {
    void (*prologue)(const NetDesc*, const int2*, const int*);
    void (*stage[4])(const NetDesc*, const int2*, const int*, int);
    void (*stage_mv[4])(const NetDesc*, const int2*, const int*, int);
    void (*final)(const NetDesc*, const int2*, const int*, int);
};
bool links_select(int model, int prec, LinksLaunch* out);
size_t links_map_bytes(int model, int prec);
hipError_t links_launch_chunk(const LinksLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                              const int* nwork, int chunk, bool mv);

}  // namespace nd
