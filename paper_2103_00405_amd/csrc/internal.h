// internal.h -- library-internal types shared by the host code and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rtssa.h"

// Reaction encoding in the device tables: react[k].x = s0 | (kind << 29),
// react[k].y = s1, with kind
//   0: h = 1                       (no reactant)
//   1: h = X[s0]                   (one molecule of s0)
//   2: h = X[s0] (X[s0] - 1) / 2   (two molecules of s0)
//   3: h = X[s0] X[s1]             (one each of s0 != s1)
enum { RT_H_ZERO = 0, RT_H_ONE = 1, RT_H_PAIR = 2, RT_H_TWO = 3 };
#define RT_SPECIES_MASK 0x1FFFFFFF

// Largest network the thread-per-trajectory mapping handles (registers).
#define RT_THREAD_MAX_M 8
#define RT_THREAD_MAX_N 8

struct rt_net_dev {
    int32_t N, M;
    const int2* react;       // [M]
    const double* c;         // [M]
    const int32_t* nu_ptr;   // [M+1] net change v_k as (species, delta) lists
    const int32_t* nu_sp;
    const int32_t* nu_dl;
    const int32_t* dep_ptr;  // [M+1] dependency graph D(mu)
    const int32_t* dep_idx;
    const int32_t* nu_dense; // [M][N], only for networks of the thread mapping
    // piecewise-constant rates: c applies on [0, sched_t[0]); row i of
    // sched_c ([B][M]) from sched_t[i] on (sched_B = 0: constant rates)
    int32_t sched_B;
    const double* sched_t;
    const double* sched_c;
    // lazy form, fixed-stride rows (built on first use): touch[mu*64] = the
    // number of channels of D(mu) other than mu, touch[mu*64 + q] (q = 1..63)
    // the q-th of them or -1; touch_more[mu] = the CSR position of the 64th
    // (dep_ptr[mu+1] if none); nu_fixed[mu*nu_stride + i] = (species, change)
    // of the jump v_mu, (-1, 0) past its end
    const int32_t* touch;
    const int32_t* touch_more;
    const int2* nu_fixed;
    int32_t nu_stride;
    // workgroup mapping, fixed-stride dependency records (built on first
    // use): grow[mu*64 + q] = (k, react[k].x, react[k].y, w) for q = 0 (k = mu,
    // w = the number of channels of D(mu) other than mu) and q >= 1 (the q-th
    // other channel, k = -1 past the end; q = 1: w = the CSR position of the
    // 64th other channel, dep_ptr[mu+1] if none); growc[mu*64 + q] = c_k;
    // gdel[mu*64 + q] = the change of the record's reactant species s0, s1
    // under v_mu (0 for a species the record's kind does not read)
    const int4* grow;
    const double* growc;
    const int2* gdel;
};

struct rtssa_network {
    int32_t N = 0, M = 0;
    std::vector<int2> react;
    std::vector<double> c;
    std::vector<int32_t> nu_ptr, nu_sp, nu_dl, dep_ptr, dep_idx, nu_dense;
    int32_t max_nu = 0;      // largest |v_k| support
    int32_t max_dep = 0;     // largest |D(mu)|
    int device = -1;
    void* dev_block = nullptr;  // one allocation holding every device table
    void* sched_block = nullptr;  // device copy of the rate schedule (times, rates)
    void* lazy_block = nullptr;   // the lazy form's fixed-stride rows
    void* group_block = nullptr;  // the workgroup mapping's dependency records
    int32_t batch_refs = 0;       // batch items holding this network's device pointers
    rt_net_dev dev{};
};


// One network and its run parameters, in device memory: the unit of work
// description of every kernel (a single run is a batch of one item).
struct rt_item_dev {
    rt_net_dev net;
    const int32_t* x0;
    int32_t x0_per_traj;
    int32_t G;
    double t_end;
    const double* s;
    uint32_t net_id, traj_offset;
    int64_t R;
    int32_t* samples;
    int64_t ss_r, ss_g, ss_n;
    uint32_t* n_out;
    double* T_out;
    int32_t* x_final;
    double* t_last;
    uint8_t* status;
    unsigned long long* seq_hash;
    uint32_t* tie_step;
};

// Device workspace of one launch (or one class of a batch): counters written
// by the kernels, the work-queue heads, and the Philox key.
struct rt_ws {
    unsigned long long firings, near_ties, clamps, slow_logs;
    unsigned long long status_count[4];
    unsigned long long next_unit;    // trajectory units or items handed out
    uint32_t key0, key1;
    unsigned long long bad_input;    // 1: a single run's sample grid failed its check
    unsigned long long pad[5];
};

// A class of items run by one persistent kernel: items[0 .. count); the
// trajectory units of item i are unit_start[i] .. unit_start[i+1]-1.
// item_next[i] counts the trajectories of item i handed to lanes of the
// thread mapping.  exclusive = 1: one wavefront takes a whole item (batches,
// so that a wavefront's lanes share one network); 0: every wavefront works
// on item 0 (a single run).
struct rt_class_dev {
    const rt_item_dev* items;
    const int64_t* unit_start;
    unsigned long long* item_next;
    rt_ws* ws;
    int32_t count;
    int32_t exclusive;
    int32_t max_N;
    int32_t max_M;
    uint32_t max_firings;
    int32_t has_schedule;   // some item's network has a rate schedule
};

// Device workspace of one single run: counters, its item descriptor and
// unit range, the per-item trajectory counter; the lazy form's channel
// records follow at the next 256-byte boundary.
struct rt_run_scratch {
    rt_ws ws;
    rt_item_dev item;
    int64_t unit_start[2];
    unsigned long long item_next[2];
};

inline size_t rt_align256(size_t x) { return (x + 255) & ~(size_t)255; }

// error reporting and mapping choice (api.cpp)
int rt_fail(int code, const std::string& msg);
int rt_auto_mapping(const rtssa_network* net);
int rt_auto_group_size(int M);
int rt_launch_class(int mapping, int max_M, int max_N, int max_nu, const rt_class_dev& C,
                    int block, int grid, int64_t lanes, hipStream_t stream, int* block_used,
                    int* grid_used, int method = RTSSA_METHOD_RANDOM_TIME);
rt_item_dev rt_make_item(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                         double t_end, const double* sample_t, int32_t G, uint32_t net_id,
                         uint64_t traj_offset, int64_t R, int32_t* samples, int64_t s_stride_r,
                         int64_t s_stride_g, int64_t s_stride_n, uint32_t* n_out, double* T_out,
                         int32_t* x_final, double* t_last, uint8_t* status, uint64_t* seq_hash,
                         uint32_t* tie_step);
// host-side checks of one run's arguments (no device access)
int rt_check_run(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj, double t_end,
                 const double* sample_t, int32_t G, uint64_t traj_offset, int64_t R);
// reads a sample grid from the device and checks it (synchronous; batch creation)
int rt_check_grid_host(const double* sample_t, int32_t G, double t_end);
void rt_fill_stats(rtssa_stats* stats, const rt_ws& h);
int check_hip(hipError_t e, const char* what);

// kernels: launchers take a class descriptor whose pointers are device memory
// method: RTSSA_METHOD_RANDOM_TIME or RTSSA_METHOD_DIRECT
int rt_launch_thread(int M, int N, const rt_class_dev& C, int block, int grid,
                     hipStream_t stream, int* grid_used, int64_t lanes, int method);
int rt_launch_setup(rt_ws* ws, unsigned long long* extra, int64_t n_extra, uint32_t key0,
                    uint32_t key1, const uint32_t* key_src, const rt_item_dev* item,
                    rt_item_dev* item_dst, int64_t* unit_start, hipStream_t stream);
size_t rt_score_grad_workspace_bytes(int64_t R, int32_t M);
int rt_launch_score_grad(const double* f, const uint32_t* n, const double* T, int64_t R,
                         int32_t M, int32_t baseline, double* grad, double* se,
                         void* workspace, hipStream_t stream);
int rt_launch_debug_neglog(const uint64_t* m, double* out, uint8_t* slow, int64_t count,
                           int force, hipStream_t stream);
int rt_launch_debug_select(const double* v, int32_t M, int64_t count, int32_t mapping,
                           int32_t lanes, int32_t* mu, double* v1, double* v2, uint8_t* near,
                           hipStream_t stream);
int rt_launch_debug_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                           int64_t count, hipStream_t stream);
int rt_thread_supported(int M, int N);
int rt_launch_group(int M, int max_N, int max_M, const rt_class_dev& C, int L, int grid,
                    hipStream_t stream, int* grid_used);
int rt_group_slots(int M, int L);
// true when a workgroup kernel with L threads exists for M channels
bool rt_group_supported(int M, int L);
size_t rt_group_lds_bytes(int N, int M, int L);
int rt_launch_subwave(int max_M, const rt_class_dev& C, int L, int grid, hipStream_t stream,
                      int* grid_used);
// the workgroup mapping with the propensities in LDS (kernels_group_lds.hip):
// the kernel for a class, or nullptr when its LDS does not fit; it reads the
// network's fixed-stride rows (rt_lazy_prepare), which every item must have
const void* rt_group_lds_kernel_for(int M, int max_N, int L, bool sched);
size_t rt_group_lds2_bytes(int N, int L, int S);
int rt_launch_group_lds(int M, int max_N, const rt_class_dev& C, int L, int grid,
                        hipStream_t stream, int* grid_used);
// the fixed-stride rows a run of this network with these options reads:
// 0 none, 1 the lazy form's rows (tree methods; the random-time sub-wave
// mapping), 2 those and the workgroup
// mapping's dependency records (random-time workgroup mapping)
int rt_run_rows(const rtssa_network* net, const rtssa_options& o);
bool rt_rows_ready(const rtssa_network* net, int rows);
int rt_rows_prepare(rtssa_network* net, int rows);
// the lazy form (one wavefront per trajectory, LDS tree)
// workspace: NULL to allocate it stream-ordered for this launch, else at
// least rt_lazy_workspace_bytes(grid, max_M) bytes for the grid that
// rt_lazy_grid returns (the same grid the launch then uses)
int rt_launch_lazy(const rt_class_dev& C, int max_N, int max_M, int grid, int64_t units,
                   hipStream_t stream, int* grid_used, void* workspace = nullptr);
// sched: the class has a rate schedule (C.has_schedule), which picks the kernel;
// max_per_cu > 0 caps the resident wavefronts per CU of a grid the call sizes
// (a batch's lazy classes leave room for the classes running beside them)
int rt_lazy_grid(int max_N, int max_M, int grid, int64_t units, bool sched, int* grid_out,
                 int max_per_cu = 0);
size_t rt_lazy_workspace_bytes(int grid, int max_M);
size_t rt_lazy_lds_bytes(int N, int M);
// the direct method on a sum tree (same mapping and layout as the lazy form)
int rt_launch_dmtree(const rt_class_dev& C, int max_N, int max_M, int grid, int64_t units,
                     hipStream_t stream, int* grid_used);
// builds and uploads the lazy form's rows of a network once (network.cpp)
int rt_lazy_prepare(rtssa_network* net);
// the same plus the workgroup mapping's dependency records (network.cpp)
int rt_group_rows_prepare(rtssa_network* net);
int rt_subwave_slots(int M, int L);
int rt_subwave_lanes(int M);

// single runs (api.cpp), shared by rtssa_simulate and its allocation-free
// variant
int rt_check_method(const rtssa_network* net, const rtssa_options& o, bool want_T,
                    bool want_tie);
int rt_simulate_checks(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                       double t_end, const double* sample_t, int32_t G, uint64_t traj_offset,
                       int64_t R, const double* T_out, const uint32_t* tie_step,
                       const rtssa_options& o, bool may_build_rows);
int rt_run_workspace(const rtssa_network* net, int64_t R, const rtssa_options& o, size_t cap,
                     size_t* bytes, int* lazy_grid);
int rt_simulate_on(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                   double t_end, const double* sample_t, int32_t G, uint64_t seed,
                   uint32_t net_id, uint64_t traj_offset, int64_t R, int32_t* samples,
                   int64_t s_stride_r, int64_t s_stride_g, int64_t s_stride_n, uint32_t* n_out,
                   double* T_out, int32_t* x_final, double* t_last, uint8_t* status,
                   uint64_t* seq_hash, uint32_t* tie_step, const rtssa_options& o, void* wsp,
                   int lazy_grid, hipStream_t stream, rtssa_stats* stats,
                   bool time_kernels = true);
