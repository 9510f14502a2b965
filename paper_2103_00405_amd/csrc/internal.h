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
    rt_net_dev dev{};
};


// Fields the per-firing path reads; passed by value.
struct rt_hot_params {
    double t_end;
    uint32_t key0, key1, net_id, traj_offset;
    uint32_t max_firings;
    int32_t pad;
};

struct rt_sim_params {
    const int32_t* x0;
    int32_t x0_per_traj;
    int32_t G;
    double t_end;
    const double* s;
    uint32_t key0, key1, net_id, traj_offset;
    int64_t R;
    uint32_t max_firings;
    int32_t* samples;
    int64_t ss_r, ss_g, ss_n;
    uint32_t* n_out;
    double* T_out;
    int32_t* x_final;
    double* t_last;
    uint8_t* status;
    unsigned long long* seq_hash;
    uint32_t* tie_step;
    struct rt_ws* ws;
};

// Device workspace: counters written by the kernels, the work-queue head of
// the persistent kernels, and a copy of the launch parameters that rare code
// paths read through a pointer (keeping them out of scalar registers).
struct rt_ws {
    unsigned long long firings, near_ties, clamps, slow_logs;
    unsigned long long status_count[4];
    unsigned long long next_traj;
    unsigned long long pad[7];
    rt_sim_params params;
};

// error reporting and mapping choice (api.cpp)
int rt_fail(int code, const std::string& msg);
int rt_auto_mapping(const rtssa_network* net);
int rt_auto_group_size(int M);

// kernels.hip
int rt_launch_thread(const rtssa_network* net, const rt_sim_params& p, int block, int grid,
                     hipStream_t stream, int* grid_used);
int rt_launch_zero_ws(rt_ws* ws, const rt_sim_params* params, hipStream_t stream);
int rt_launch_score_grad(const double* f, const uint32_t* n, const double* T, int64_t R,
                         int32_t M, int32_t baseline, double* grad, double* se,
                         hipStream_t stream);
int rt_launch_debug_neglog(const uint64_t* m, double* out, uint8_t* slow, int64_t count,
                           int force, hipStream_t stream);
int rt_launch_debug_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                           int64_t count, hipStream_t stream);
int rt_thread_supported(int M, int N);
int rt_launch_group(const rtssa_network* net, const rt_sim_params& p, int L, int grid,
                    hipStream_t stream, int* grid_used);
int rt_group_slots(int M, int L);
size_t rt_group_lds_bytes(int N, int M);
