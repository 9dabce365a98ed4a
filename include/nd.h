/*
 * nd.h -- C ABI of libnd.so, the MI355X (gfx950) hot path for the network
 * dynamics method of Sudakov & Maistrenko, arXiv 2410.19075.
 *
 * The paper states the problem as: models with per-group parameters, a
 * coupling topology given at run time, initial values of the dynamical
 * variables, and a trajectory (or derived observables) returned at specified
 * times (Sec. II, last paragraph; Sec. III.A).  Its integrator calls the
 * per-oscillator right-hand side once per solver stage for every element in
 * parallel (Sec. III.A, Sec. III.D).  This library evaluates that right-hand
 * side -- including each element's coupling sum over its neighbourhood --
 * inside the four stages of a fixed-step classical Runge-Kutta integrator,
 * entirely on the GPU.
 *
 * Models (Sec. II):
 *   ND_KURAMOTO  Eq. (3) with m = 0, eps = 1 and a natural frequency:
 *                dphi_i/dt = omega + (mu/L) sum_{j in nbr(i)} sin(phi_j - phi_i - alpha),
 *                L = number of neighbours (the paper's Alg. 1 divides by the link count).
 *                params = {omega, mu, alpha}.  Topology ND_RING, ND_CUBE3D, ND_BALL3D, ND_DISK2D or
 *                ND_LINKS.
 *   ND_KURAMOTO_INERTIA  Eq. (3) with inertia (m != 0) as a first-order system in
 *                (phi, psi = dphi/dt), plus a natural frequency:
 *                dphi_i/dt = psi_i,
 *                m dpsi_i/dt = omega - eps psi_i + (mu/L) sum_{j in nbr(i)} sin(phi_j - phi_i - alpha).
 *                params = {omega, mu, alpha, m, eps}; m != 0.  ND_RING, ND_CUBE3D, ND_BALL3D,
 *                ND_DISK2D or ND_LINKS.
 *   ND_FHN       Eq. (2) with tau = 0, D = 0, I_app = 0 and a rotational coupling
 *                matrix B(phi) = [[cos phi, sin phi], [-sin phi, cos phi]] applied to
 *                (u_j - u_i, v_j - v_i), averaged over the 2P ring neighbours, inside the
 *                eps-scaled fast equation.  params = {eps, a, sigma, phi}.  ND_RING, or ND_LINKS
 *                (then averaged over the row's links).
 *   ND_HH        Eq. (1) for the squid axon (Na, K, leak; textbook rate functions, rest
 *                -65 mV) with an instantaneous sigmoidal synapse:
 *                C dV_i/dt = I_i - I_ion + (Esyn - V_i) sum_{e in in(i)} w_e S(V_src(e)),
 *                S(V) = 1 / (1 + exp(-(V - theta_s)/k_s)).
 *                params = {C, gNa, gK, gL, ENa, EK, EL, Esyn, theta_s, k_s}; per_elem = I_i.
 *                ND_CSR only.
 *
 * Topologies (Sec. IV; Sec. III.C for general coupling matrices and their compression):
 *   ND_RING      element i couples to i +- 1 .. i +- P (periodic), requires 1 <= P, 2P+1 <= n
 *                and n < 2^29.
 *   ND_CUBE3D    periodic n1 x n2 x n3 lattice, index x + n1*y + n1*n2*z (the paper's 3D index
 *                map), neighbours = the (2h+1)^3 cube minus the element itself; n1,n2,n3 >= 2h+1,
 *                n < 2^29.
 *   ND_BALL3D    periodic n1 x n2 x n3 lattice as ND_CUBE3D, neighbours = every lattice point within
 *                Euclidean distance P = radius, the element itself included (the paper's 3D
 *                studies: 33 links for P = 2, 925 for P = 6, Sec. V); L = that count; 1 <= P <= 8,
 *                n1,n2,n3 >= 2P+1, n < 2^29.  Kuramoto models only.
 *   ND_DISK2D    periodic n1 x n2 plane (n3 = 1, index x + n1*y), neighbours = every lattice point
 *                within distance P, the element included (the paper's 2D studies); 1 <= P <= 8,
 *                n1, n2 >= 2P+1.  Kuramoto models only.
 *   ND_CSR       directed graph stored by target: in-edges of i are row_ptr[i] .. row_ptr[i+1]-1,
 *                col[e] = source, weight[e] = synaptic weight (the paper's L_ik with weights).
 *   ND_LINKS     an arbitrary binary coupling matrix L (Sec. III.C: L_ij = 1 when element j
 *                influences element i), given by rows in row_ptr / col as for ND_CSR (weight
 *                ignored): row i lists its sources j, each at most once, self links allowed.
 *                L = the row's own link count; a row without links has no coupling.  nd_create
 *                compresses the matrix with the paper's differential compression (Alg. 2, see
 *                nd_compress_links) and the kernels extract every row on the fly; the cost per
 *                element is the row's link count.  n < 2^29.  Kuramoto models and FHN.
 *
 * State layout: variable-major FP64, length nvars * n: Kuramoto phi[n] (unwrapped, never reduced
 * mod 2 pi); Kuramoto with inertia phi[n] then psi[n]; FHN u[n] then v[n]; HH V[n], m[n], h[n],
 * n[n].
 *
 * Precision: ND_FP64 computes everything in IEEE double.  ND_FP32_BULK computes the per-element
 * maps (sin/cos, sigmoid, rate functions) and the local right-hand side in float and stores the
 * stage slopes k in float, while every neighbourhood sum, the state y and the RK accumulator stay
 * double.
 *
 * Ownership: the caller owns every pointer it passes.  nd_create copies topology, weights and
 * per-element data (host pointers) to the device, so the caller may free them on return.  The
 * library owns its device buffers; nd_destroy frees them.  Pointers passed with on_device = 1 are
 * device pointers that must stay valid until the work enqueued on the stream has completed.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued asynchronously
 * on it: nd_run and nd_run_batch return without waiting for the device.  Only the getters with
 * on_device = 0, nd_set_state with on_device = 0 (its host source is read before it returns) and
 * nd_sync synchronise it.  nd_destroy and nd_set_config wait for the work enqueued for that
 * network only (not for the whole device).
 *
 * Numerical failure: the stage kernels flag a network whose state turns non-finite (NaN or Inf)
 * in a status word on the device.  The next synchronising call on that network (nd_get_state or
 * nd_get_observables with on_device = 0, or nd_sync) returns ND_ERR_NUMERIC (the data are still
 * copied); nd_set_state clears the flag.
 *
 * Errors: every call returns ND_OK (0) or a negative nd_status.  Argument errors are detected on
 * the host before any device work and return ND_ERR_INVALID_ARG; nd_last_error() then returns a
 * thread-local description.  No C++ exception crosses this interface.
 *
 * Threading: one handle must not be used from two threads at once; different handles may.
 */
#ifndef ND_H
#define ND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nd_status;
#define ND_OK 0
#define ND_ERR_INVALID_ARG (-1)
#define ND_ERR_OUT_OF_MEMORY (-2)
#define ND_ERR_DEVICE (-3)
#define ND_ERR_NOT_READY (-4)
#define ND_ERR_NUMERIC (-5)
#define ND_ERR_UNSUPPORTED (-6)

#define ND_KURAMOTO 0
#define ND_FHN 1
#define ND_HH 2
#define ND_KURAMOTO_INERTIA 3

#define ND_RING 0
#define ND_CUBE3D 1
#define ND_CSR 2
#define ND_BALL3D 3
#define ND_DISK2D 4
#define ND_LINKS 5

#define ND_FP64 0
#define ND_FP32_BULK 1

#define ND_MAX_PARAMS 12

/* A network: model, parameters, topology, precision.  All pointers are host pointers. */
typedef struct nd_problem {
    int32_t model;      /* ND_KURAMOTO, ND_FHN, ND_HH, ND_KURAMOTO_INERTIA */
    int32_t topo;       /* ND_RING, ND_CUBE3D, ND_CSR, ND_BALL3D, ND_DISK2D, ND_LINKS */
    int32_t precision;  /* ND_FP64, ND_FP32_BULK */
    int32_t reserved;   /* must be 0 */
    int64_t n;          /* number of elements */
    int64_t radius;     /* ring: P; cube: half-width h */
    int64_t n1, n2, n3; /* cube extents, n = n1*n2*n3 */
    const int64_t* row_ptr; /* CSR, LINKS: n+1 offsets, row_ptr[0] = 0, non-decreasing */
    const int32_t* col;     /* CSR, LINKS: nnz sources in [0, n) */
    const double* weight;   /* CSR: nnz weights */
    int64_t nnz;            /* CSR: number of edges = row_ptr[n] */
    const double* per_elem; /* HH: applied current per neuron (n values); else NULL */
    double params[ND_MAX_PARAMS]; /* model parameters, see above; unused entries ignored */
} nd_problem;

/* What to record during nd_run. */
typedef struct nd_observe {
    int64_t record_every;  /* > 0: record the order parameter R at run steps 0, r, 2r, ... (r =
                              record_every), i.e. steps/r + 1 values; 0: record nothing.
                              R = |sum_j exp(i theta_j)| / n, theta = phi (Kuramoto) or
                              atan2(v, u) (FHN); the paper's synchronisation analysis at each
                              output (Sec. V).  Not defined for HH (must be 0). */
    int64_t mv_start_step; /* >= 0: record the mean phase velocity of every element over run steps
                              [mv_start_step, steps), (theta(t_end) - theta(t_start)) / (t_end -
                              t_start) on unwrapped phases (the paper's average-frequency
                              profiles, Sec. IV); FHN unwraps atan2(v, u) step by step.
                              -1: do not record.  Not defined for HH. */
} nd_observe;

typedef struct nd_net* nd_handle;

/* Validate `p`, allocate device buffers and copy topology / weights / per-element data. */
nd_status nd_create(const nd_problem* p, nd_handle* out);

/* Device bytes nd_create would allocate for `p` (state, RK buffers, exchange buffers,
 * topology), excluding observables. */
nd_status nd_footprint(const nd_problem* p, int64_t* bytes);

/* Copy the state (nvars*n doubles, layout above) into the network. */
nd_status nd_set_state(nd_handle h, const double* y, int64_t len, int32_t on_device, void* stream);

/* Integrate `steps` classical RK4 steps of size dt from the current state:
 *   k1 = F(y), k2 = F(y + dt/2 k1), k3 = F(y + dt/2 k2), k4 = F(y + dt k3),
 *   y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4).
 * obs may be NULL (record nothing).  Asynchronous on `stream`. */
nd_status nd_run(nd_handle h, double dt, int64_t steps, const nd_observe* obs, void* stream);

/* Integrate several networks together: one set of batched launches covers all of them, each with
 * its own dt, step count and observation settings (obs may be NULL or an array of `count`).
 * Every network's arithmetic is the same as in nd_run. */
nd_status nd_run_batch(const nd_handle* hs, int32_t count, const double* dt, const int64_t* steps,
                       const nd_observe* obs, void* stream);

/* Integrate several networks exactly as nd_run_batch does (same kernels, same results, bitwise),
 * without allocating anything: for callers that cannot allocate device or host memory, such as
 * code under HIP graph capture, tight serving loops and harnesses that forbid hipMalloc.  The
 * descriptor tables and work maps that nd_run_batch places in memory taken per call live here in
 * one fixed device array of ND_NOALLOC_SCRATCH_BYTES that the library reserves on every GPU it
 * runs on (held until the process ends): at most ND_NOALLOC_MAX_NETS networks and
 * ND_NOALLOC_MAX_WORK work items (nd_get_config: ring tiles, lattice tiles, CSR row blocks x 8,
 * compressed-matrix row blocks) per call; larger calls return ND_ERR_INVALID_ARG and enqueue
 * nothing.  Every call on one GPU uses that GPU's array and leaves its contents behind, so calls
 * whose device work overlaps on one GPU (unordered streams, concurrent threads) race: order them
 * on one stream.  Observables are recorded only into buffers that an earlier nd_run or
 * nd_run_batch of the same network sized (R of at least steps/record_every + 1 values, the mean
 * phase velocity); otherwise ND_ERR_INVALID_ARG.  Chunks are launched directly on `stream` (no
 * graph is captured or replayed).  Asynchronous like nd_run_batch. */
#define ND_NOALLOC_MAX_NETS 256
#define ND_NOALLOC_MAX_WORK 262144
#define ND_NOALLOC_SCRATCH_BYTES 2359296
nd_status nd_run_batch_noalloc(const nd_handle* hs, int32_t count, const double* dt, const int64_t* steps,
                               const nd_observe* obs, void* stream);

/* Copy the current state out (nvars*n doubles). */
nd_status nd_get_state(nd_handle h, double* y, int64_t len, int32_t on_device, void* stream);

/* Copy the observables of the last nd_run: R (r_len must equal steps/record_every + 1) and/or the
 * mean phase velocity (mv_len must equal n).  Pass NULL / 0 to skip either. */
nd_status nd_get_observables(nd_handle h, double* R, int64_t r_len, double* mean_vel, int64_t mv_len,
                             int32_t on_device, void* stream);

/* Wait for the work enqueued on `stream` and report the network's numerical status: ND_OK, or
 * ND_ERR_NUMERIC when a run since the last nd_set_state produced a non-finite state value. */
nd_status nd_sync(nd_handle h, void* stream);

nd_status nd_destroy(nd_handle h);

/* Kernel configuration (chosen by the autotuner; callers normally leave it alone). */
typedef struct nd_kernel_config {
    int32_t tile;   /* ring: elements per tile (128, 256, 512, 1024 or 2048), or -1024 / -2048 / -4096:
                       the whole ring (n <= that capacity) resident in one workgroup;
                       cube: output tile extent along x; CSR: rows per workgroup */
    int32_t block;  /* threads per workgroup: derived (ignored by nd_set_config), except for
                       ND_BALL3D / ND_DISK2D, where it selects 256 or 1024 */
    int32_t grid;   /* persistent grid size in workgroups; 0 = one workgroup per work item */
    int32_t chunk;  /* steps per captured graph chunk */
    int32_t tile_y; /* cube: output tile extent along y ((tile+2h)*(tile_y+2h) <= 1024);
                       CSR: edges each thread streams per chunk (2, 4, 8 or 16; results
                       do not depend on it) */
    int32_t tile_z; /* cube: planes per work item */
} nd_kernel_config;

/* Adaptive stepping: Dormand-Prince 5(4), the paper's default solver (Sec. III.A), with the
 * usual step-size control (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4):
 *   err = sqrt(mean_i ((y5_i - y4_i) / (atol + rtol max(|y_i|, |y5_i|)))^2), accept when
 *   err <= 1, new h = h min(facmax, max(0.2, 0.9 err^(-1/5))), facmax = 10 (1 right after a
 *   rejection); the step that reaches t_end (within a relative 1e-12 of h) ends on it.
 * rtol <= 0 takes fixed steps of dt0 (no control).  The fifth-order solution propagates.
 * Each of the `count` networks is integrated from its current state over [0, t_end[i]]
 * starting with step dt0[i] on the device; each network controls its own step.  Supported:
 * FP64 rings (ND_RING) or compressed coupling matrices (ND_LINKS) of the Kuramoto,
 * Kuramoto-with-inertia or FHN model, one model and one topology per call (ND_ERR_UNSUPPORTED
 * otherwise).  When every ring holds at most 1024 elements, one workgroup integrates each
 * ring in a single launch; otherwise (and for ND_LINKS) the batch is tiled over workgroups, with
 * the accept / reject decisions taken on the device and only the rings' completion read back
 * every few attempts.  At most max_steps step attempts per network.  The state
 * is advanced in place (read it with nd_get_state); no observables are recorded.  Blocks
 * until done; stats[i] receives the time reached, the accepted and rejected steps and the
 * step proposed next.  A controlled network whose error estimate is not finite, or whose step
 * falls below 10 units in the last place of t, stops there with stats[i].failed = 1; the call
 * then returns ND_ERR_NUMERIC (after every network has finished or stopped). */
typedef struct nd_adaptive_stats {
    double t;          /* time reached (t_end unless max_steps ran out or the run failed) */
    int64_t accepted;  /* accepted steps */
    int64_t rejected;  /* rejected step attempts */
    double h_next;     /* step size proposed for a continuation */
    int32_t failed;    /* 1: the run stopped at t because its error estimate was not finite (a NaN
                          or Inf in the state or the slopes) or its proposed step fell below 10 units
                          in the last place of t; the state is the last accepted one */
    int32_t reserved;
} nd_adaptive_stats;

nd_status nd_run_adaptive(const nd_handle* h, int32_t count, const double* t_end, const double* dt0, double rtol,
                          double atol, int64_t max_steps, nd_adaptive_stats* stats, void* hip_stream);

/* As nd_run_adaptive, with dense output: the trajectory at the output times t_k = k t_out,
 * k = 0 .. floor(t_end[i] / t_out), taken from the solver's continuous extension of order 4
 * inside the accepted step that contains t_k (Hairer, Norsett & Wanner, Solving ODEs I,
 * Sec. II.6), so the outputs do not shorten the steps; t_0 gives the initial state and the
 * step that ends on t_end provides every output left.  The paper returns trajectories at
 * specified times and analyses synchronisation at each output (Sec. II, Sec. V; its
 * Dormand-Prince solvers interpolate between steps, Sec. III.A).
 * R (host, count * r_stride doubles): R[i * r_stride + k] = order parameter of network i at t_k
 * (as nd_observe defines it); r_stride >= floor(t_end[i] / t_out) + 1 for every i.
 * Y (host, may be NULL; count * y_stride doubles): Y[i * y_stride + k * nvars * n + v * n + j]
 * = variable v of element j at t_k; y_stride >= (outputs of i) * nvars * n_i.
 * Outputs a network does not reach (max_steps) read NaN.  The device holds R and Y in a
 * scratch buffer for the call.  Otherwise as nd_run_adaptive. */
nd_status nd_run_adaptive_dense(const nd_handle* h, int32_t count, const double* t_end, const double* dt0,
                                double rtol, double atol, int64_t max_steps, double t_out, double* R,
                                int64_t r_stride, double* Y, int64_t y_stride, nd_adaptive_stats* stats,
                                void* hip_stream);

/* Differential compression of a binary coupling matrix (Sec. III.C, Alg. 2), as nd_create
 * applies it to ND_LINKS problems; exposed so a caller can inspect the compressed size.
 * Rows are given as for ND_LINKS (row_ptr: n+1 offsets, col: sources).  A circular shift of
 * row i left by i moves position p to (p - i) mod n; the common vector V is row 0; the
 * difference vector of row i is (row i shifted left by i) XOR V; the difference table keeps
 * each distinct difference vector once, in order of first appearance as i increases; C[i] is
 * the entry of row i, so row i = (V XOR D[C[i]]) shifted right by i.  Host-only: no device
 * work.  info receives the sizes (always); V (sorted positions, v_cap >= info.v_bits),
 * d_ptr (entry k holds d_pos[d_ptr[k] .. d_ptr[k+1]-1], sorted; d_ptr_cap >= entries + 1),
 * d_pos (d_pos_cap >= info.d_bits) and C (c_cap >= n) are written when non-NULL, so a first
 * call with NULL arrays sizes them.  ND_ERR_INVALID_ARG for malformed rows (a source out of
 * range or listed twice) or short arrays; n < 2^29. */
typedef struct nd_links_info {
    int64_t v_bits;   /* set bits of the common vector V (the links of row 0) */
    int64_t entries;  /* difference-table entries */
    int64_t d_bits;   /* set bits over all entries */
    int64_t runs;     /* maximal runs of consecutive positions in V */
    int64_t bytes;    /* device bytes of the compressed matrix as the kernels hold it */
} nd_links_info;

nd_status nd_compress_links(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t* V, int64_t v_cap,
                            int64_t* d_ptr, int64_t d_ptr_cap, int32_t* d_pos, int64_t d_pos_cap, int32_t* C,
                            int64_t c_cap, nd_links_info* info);

nd_status nd_get_config(nd_handle h, nd_kernel_config* cfg);
nd_status nd_set_config(nd_handle h, const nd_kernel_config* cfg);

/* Autotuner.  Times every candidate kernel configuration for problem p (ring: tile sizes;
 * cube: x/y/z tile extents; CSR: edges per thread) on `steps` RK4 steps of size dt from state y0
 * (host, nvars*n doubles), keeps the fastest in a process-wide cache keyed by (device
 * architecture, model, topology, precision, log2 n, coupling-width bucket, half-width), and
 * returns it.  nd_create uses a cached entry for every later problem of the same key.  The
 * paper tunes its own knobs (CUDA streams per GPU, MPI partitions) by hand (Sec. III.E-F).
 * best_ms (may be NULL) receives the best time per step in milliseconds. */
nd_status nd_tune(const nd_problem* p, const double* y0, int64_t len, double dt, int32_t steps, void* stream,
                  nd_kernel_config* best, double* best_ms);
/* Read / write the cache as text, one entry per line (an existing file is replaced). */
nd_status nd_tune_load(const char* path);
nd_status nd_tune_save(const char* path);
nd_status nd_tune_clear(void);

/* ------------------------------------------------------------------ serving
 * Continuous batching of many independent simulations on one GPU.  The paper
 * runs many small unconnected sub-networks in one run for throughput (Sec.
 * III.C) and computes thousands of trajectories in batch mode (Sec. II, Sec.
 * IV); the server does this online: requests arrive at any time, wait in a
 * FIFO queue, are admitted while their device footprint fits the HBM budget and
 * a slot is free, and then advance together, a chunk of RK4 steps at a time, in
 * one persistent batched launch per kernel class (a captured graph replayed
 * every chunk).  New requests join and finished ones leave at chunk
 * boundaries.  Every request's arithmetic is the same as nd_run's for the same
 * problem, whatever else shares the GPU with it.
 */
typedef struct nd_server* nd_server_h;
typedef int64_t nd_req;

#define ND_REQ_QUEUED 0
#define ND_REQ_RUNNING 1
#define ND_REQ_DONE 2
#define ND_REQ_FAILED 3
#define ND_REQ_CANCELLED 4

typedef struct nd_server_config {
    int64_t hbm_budget_bytes; /* device bytes that admitted requests may hold (nd_footprint) */
    int32_t max_slots;        /* requests running at once (<= 4096) */
    int32_t chunk_steps;      /* RK4 steps per chunk (>= 1) */
    int32_t grid;             /* persistent workgroups per kernel class (multiple of 8; 0 = 2048) */
    int32_t reserved;         /* must be 0 */
} nd_server_config;

typedef struct nd_request_info {
    int32_t state;        /* ND_REQ_* */
    nd_status status;     /* failure reason when state == ND_REQ_FAILED */
    int64_t steps_done;
    double arrival;       /* seconds on the server clock */
    double admitted;      /* -1 until admitted */
    double finished;      /* -1 until done / failed / cancelled */
} nd_request_info;

typedef struct nd_server_counters {
    int64_t submitted, completed, failed, cancelled, queued, running;
    int64_t bytes_in_use;  /* footprint of the running requests */
    int64_t chunks;        /* chunks launched */
    double gpu_seconds;    /* device time of the completed chunks (events around each chunk) */
    int64_t osc_steps;     /* element-steps completed */
    double active_seconds; /* wall time between pumps during which requests were admitted or chunks
                              in flight; gpu_seconds / active_seconds is the device's busy share
                              while there was work (the rest: host gaps between chunks) */
} nd_server_counters;

nd_status nd_server_create(const nd_server_config* cfg, nd_server_h* out);
/* Seconds since the server was created (the clock of arrival/admitted/finished). */
nd_status nd_server_now(nd_server_h s, double* seconds);
/* Queue a simulation: problem p (host data copied), initial state y0 (host, nvars*n doubles,
 * copied), dt, steps >= 1, observables (may be NULL).  arrival < 0 means now.  Returns
 * ND_ERR_INVALID_ARG for a bad problem or a footprint above the budget and ND_ERR_NUMERIC for a
 * non-finite y0; the request then does not exist.  Never touches the GPU. */
nd_status nd_server_submit(nd_server_h s, const nd_problem* p, const double* y0, int64_t len, double dt,
                           int64_t steps, const nd_observe* obs, double arrival, nd_req* id);
/* One scheduling cycle on `stream`: retire the requests whose last chunk has completed (results
 * copied to host memory on a copy stream of the server), admit from the queue (device memory from
 * the stream-ordered pool, initial state uploaded on the copy stream), enqueue the next chunk of
 * every admitted request with steps left, and wait for the chunk before it, so one chunk stays
 * queued behind the running one and the host's work overlaps the device's.  The first
 * admission creates the server's device resources.  *pending receives the number of queued + running
 * requests afterwards. */
nd_status nd_server_pump(nd_server_h s, void* stream, int64_t* pending);
nd_status nd_server_info(nd_server_h s, nd_req id, nd_request_info* info);
/* Final state (len = nvars*n) and R (r_len = steps/record_every + 1, or NULL / 0) of a done request. */
nd_status nd_server_result(nd_server_h s, nd_req id, double* y, int64_t len, double* R, int64_t r_len);
/* Cancel a queued or running request; a running one leaves at the next chunk boundary. */
nd_status nd_server_cancel(nd_server_h s, nd_req id);
nd_status nd_server_stats(nd_server_h s, nd_server_counters* st);
nd_status nd_server_destroy(nd_server_h s);

const char* nd_status_str(nd_status s);
const char* nd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ND_H */
