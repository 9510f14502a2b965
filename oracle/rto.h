/*
 * rto.h -- CPU oracle for the next-reaction random-time stochastic simulation
 * (Liu & Wang, "Parallel implementations of random time algorithm for
 * chemical network stochastic simulations", arXiv:2103.00405).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every array is host memory owned by the caller.
 */
#ifndef RTO_H
#define RTO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RTO_OK = 0, RTO_ABSORBED = 1, RTO_OVERFLOW = 2, RTO_MAX_FIRINGS = 3 };
enum { RTO_SUCCESS = 0, RTO_E_INVALID = -1, RTO_E_HARDCASE = -5 };

/* Mass-action network, reactant/product lists in CSR form (Eq. 1-2).
 * Reaction k consumes react_sigma[e] molecules of react_species[e] for
 * e in [react_ptr[k], react_ptr[k+1]) and produces prod_mult[e] molecules of
 * prod_species[e] for e in [prod_ptr[k], prod_ptr[k+1]).  c[k] is the rate
 * constant c_k. */
typedef struct {
    int32_t N, M;
    const int32_t *react_ptr, *react_species, *react_sigma;
    const int32_t *prod_ptr, *prod_species, *prod_mult;
    const double *c;
} rto_network;

typedef struct {
    uint64_t firings;      /* applied events, summed over trajectories */
    uint64_t near_ties;    /* applied events whose two smallest gaps are within 1e-12 relative */
    uint64_t clamps;       /* applied events whose raw gap was negative and clamped to 0 */
    uint64_t status_count[4];
    int32_t hard_cases;    /* Exp(1) draws where the quad log could not certify rounding */
} rto_stats;

/* One Exp(1) draw E(seed, traj, net, k, n) = RN(-ln u); see rto.c. */
double rto_exp1(uint64_t seed, uint32_t traj, uint32_t net_id, uint32_t k, uint32_t n);
/* -ln(u) rounded to nearest for u = (m+1) 2^-53; returns -1 on a hard case. */
double rto_neglog_u53(uint64_t m);
/* Philox4x32-10 block function. */
void rto_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The selection step of Eq. 25 over v[0..M): *mu = the lowest k among the
 * smallest values (-1 when none is finite), *v1 = that value, *v2 = the
 * second smallest value counted with multiplicity (+inf if none). */
void rto_argmin2(const double* v, int32_t M, int32_t* mu, double* v1, double* v2);
/* The near-tie rule: 1 when RN(d2 - d1) <= RN(1e-12 d1), else 0. */
int rto_near_tie(double d1, double d2);

/* Simulate R trajectories with ids traj_offset .. traj_offset+R-1.
 * x0: [N] when x0_per_traj == 0, else [R][N].
 * samples: [R][G][N] int32 (may be NULL when G == 0).
 * n_out [R][M] uint32, T_out [R][M] double, x_final [R][N] int32,
 * t_last [R] double, status [R] uint8, seq_hash [R] uint64,
 * tie_step [R] uint32 (0xFFFFFFFF when no near-tie).
 * nthreads <= 0 means one thread per online CPU. */
int rto_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                 double t_end, const double* sample_t, int32_t G,
                 uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                 uint64_t max_firings,
                 int32_t* samples, uint32_t* n_out, double* T_out, int32_t* x_final,
                 double* t_last, uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                 int32_t nthreads, rto_stats* stats);

/* rto_simulate with piecewise-constant rate constants (the time-dependent
 * rates of the paper's discussion, Eq. 28): the network's c applies on
 * [0, sched_t[0]), row i of sched_c ([B][M]) from sched_t[i] on; sched_t
 * strictly increasing and > 0. */
int rto_simulate_schedule(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                          double t_end, const double* sample_t, int32_t G,
                          uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                          uint64_t max_firings,
                          int32_t* samples, uint32_t* n_out, double* T_out, int32_t* x_final,
                          double* t_last, uint8_t* status, uint64_t* seq_hash,
                          uint32_t* tie_step, int32_t nthreads, rto_stats* stats,
                          int32_t B, const double* sched_t, const double* sched_c);

/* The lazy form of the same algorithm (section 5's dependency graph, in
 * internal times): a channel's internal time is brought up to date only when
 * its propensity changes or it fires, and the next event is the smallest
 * absolute next firing time.  Same draws, same law, its own rounding; same
 * arrays as rto_simulate. */
int rto_lazy_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                      double t_end, const double* sample_t, int32_t G,
                      uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                      uint64_t max_firings,
                      int32_t* samples, uint32_t* n_out, double* T_out, int32_t* x_final,
                      double* t_last, uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                      int32_t nthreads, rto_stats* stats);

/* rto_lazy_simulate with piecewise-constant rate constants (as
 * rto_simulate_schedule): at a breakpoint every clock runs to it at its old
 * propensity and every channel takes the new rates. */
int rto_lazy_simulate_schedule(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                               double t_end, const double* sample_t, int32_t G,
                               uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                               uint64_t max_firings,
                               int32_t* samples, uint32_t* n_out, double* T_out,
                               int32_t* x_final, double* t_last, uint8_t* status,
                               uint64_t* seq_hash, uint32_t* tie_step, int32_t nthreads,
                               rto_stats* stats, int32_t B, const double* sched_t,
                               const double* sched_c);

/* Gillespie's direct method (section 3, Eq. 17-22) with draws keyed like the
 * GPU library's direct method: one Philox4x32-10 block per firing at counter
 * (firing index, 0xFFFFFFFF, traj, net_id).  Same arrays as rto_simulate
 * without T_out and tie_step (the method has neither). */
int rto_direct_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                        double t_end, const double* sample_t, int32_t G,
                        uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                        uint64_t max_firings,
                        int32_t* samples, uint32_t* n_out, int32_t* x_final,
                        double* t_last, uint8_t* status, uint64_t* seq_hash,
                        int32_t nthreads, rto_stats* stats);

/* The direct method with a_0 and the channel search on a fixed sum tree of
 * fan-out 8 (nodes add their children pairwise; the search scans a node's
 * children in order, taking the first positive child with r <= v_i, else the
 * last positive one, and subtracts the children it passes).  Same draws and
 * arrays as rto_direct_simulate. */
int rto_direct_tree_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                             double t_end, const double* sample_t, int32_t G,
                             uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                             uint64_t max_firings,
                             int32_t* samples, uint32_t* n_out, int32_t* x_final,
                             double* t_last, uint8_t* status, uint64_t* seq_hash,
                             int32_t nthreads, rto_stats* stats);

/* Gillespie direct method with its own SplitMix64 stream: an independent
 * sampler of the same Markov jump law, used only for two-sample law tests. */
int rto_dm_simulate(const rto_network* net, const int32_t* x0, double t_end,
                    const double* sample_t, int32_t G, uint64_t seed, int64_t R,
                    uint64_t max_firings, int32_t* samples, uint32_t* n_out,
                    int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
