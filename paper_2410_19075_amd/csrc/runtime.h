// Host-side internals of libnd shared by the runtime, the kernels' launchers,
// the batch scheduler and the autotuner.
#pragma once

#include <hip/hip_runtime.h>

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
int64_t footprint_bytes(const nd_problem* p, const nd_kernel_config& c);

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
    std::vector<void*> allocs;

    ~Net();
    nd_status alloc(void** ptr, size_t bytes);
    nd_status create(const nd_problem* p);
    int64_t work_items() const;
    void append_work(int desc_index, std::vector<int2>& wk) const;
    nd_status prepare_observe(int64_t steps, const nd_observe* obs);
    NetDesc run_desc(double dt, int64_t steps) const;
};

// Networks of one kernel class launched together.
struct Group {
    int model, topo, prec, tile;
    int ndesc;
    int grid;
    NetDesc* desc;  // device
    int2* work;     // device
    int* nwork;     // device
};

nd_status enqueue_chunk(const Group& g, int chunk, hipStream_t st);
nd_status run_nets(Net* const* nets, int count, const double* dt, const int64_t* steps, const nd_observe* obs,
                   hipStream_t st);

// ring kernels (ring.hip)
struct RingLaunch {
    void (*prologue)(const NetDesc*, const int2*, const int*);
    void (*stage)(const NetDesc*, const int2*, const int*, int, int);
    void (*epilogue)(const NetDesc*, const int2*, const int*, int);
    int bs, tile;
};
bool ring_select(int model, int prec, int tile, RingLaunch* out);
hipError_t ring_launch_prologue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork);
hipError_t ring_launch_stage(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                             const int* nwork, int stage, int j);
hipError_t ring_launch_epilogue(const RingLaunch& L, int grid, hipStream_t s, NetDesc* D, const int2* work,
                                const int* nwork, int chunk);

}  // namespace nd
