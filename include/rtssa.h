/*
 * rtssa.h -- C ABI of the MI355X random-time stochastic simulation library.
 *
 * The library simulates mass-action chemical reaction networks with the next
 * reaction random time algorithm (NRRTA) of Liu & Wang, "Parallel
 * implementations of random time algorithm for chemical network stochastic
 * simulations" (arXiv:2103.00405): section 4, Table 2, on the random
 * time-change representation X(t) = X(0) + sum_k Y_k(T_k(t)) v_k of section 2
 * (Eq. 14-16), with per-channel unit-exponential internal-time gaps (Eq. 23)
 * of which only the fired channel's is refreshed (Eq. 26).
 *
 * Conventions.
 *  - Every function returns an rtssa_status code (0 on success).  On failure
 *    rtssa_last_error() returns a thread-local description.
 *  - "device" pointers are HIP device memory (e.g. torch CUDA tensors);
 *    "host" pointers are ordinary memory.  The caller owns every buffer it
 *    passes; the library owns the handles it returns.
 *  - Work is enqueued on the given hipStream_t (NULL = the default stream)
 *    and is asynchronous unless a function says otherwise.
 *  - Floating point is IEEE binary64 throughout; counts are exact integers.
 *
 * Per-trajectory arithmetic (the contract every mapping and the CPU
 * reference follow bit for bit):
 *   init : t = 0, X = x0, T_k = 0, n_k = 0, P_k = E(k, 0)
 *   a_k  = RN(c_k * RN(h_k(X))), h_k = prod_j C(X_j, sigma_jk) in exact int64
 *          (Eq. 1-2; C(X,2) = X(X-1)/2); inv_k = RN(1 / a_k)
 *   gap_k = +inf if a_k = 0 (frozen channel, Table 2 note), else
 *           max(0, RN(RN(P_k - T_k) * inv_k))
 *   mu   = lowest k with the smallest gap (Eq. 25); Delta = gap_mu
 *   stop (ABSORBED) if Delta = +inf; stop (OK) if t + Delta > t_end
 *   near-tie when RN(d2 - Delta) <= RN(1e-12 * Delta), d2 the second smallest gap
 *   grid points s_g < t + Delta receive X (right-continuous sampling)
 *   stop (OVERFLOW) if X + v_mu leaves [0, 2^31 - 1] (jump not applied)
 *   t += Delta; T_k = fma(a_k, Delta, T_k) for k != mu; T_mu = P_mu;
 *   X += v_mu; n_mu += 1; P_mu = RN(P_mu + E(mu, n_mu)); recompute a, inv
 *   stop (MAX_FIRINGS) once sum_k n_k reaches max_firings
 *   end (OK, ABSORBED): remaining grid points receive X and
 *       T_k = fma(a_k, RN(t_end - t), T_k); after OVERFLOW / MAX_FIRINGS the
 *       remaining grid points receive -1 and T is left at the last event.
 *   E(k, n) = RN(-ln u), correctly rounded, u = ((word >> 11) + 1) 2^-53 with
 *       word the 64-bit half of the Philox4x32-10 block (Salmon et al., SC'11)
 *       at counter (n >> 1, k, traj, net_id) under key (seed_lo, seed_hi):
 *       (w1:w0) for even n, (w3:w2) for odd n.
 *   seq_hash: h = 0xcbf29ce484222325; per applied event h = (h ^ mu) * 0x100000001b3.
 */
#ifndef RTSSA_H
#define RTSSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* rtssa_stream_t; /* same type as hipStream_t */

typedef enum {
    RTSSA_OK = 0,
    RTSSA_E_INVALID = -1,     /* bad argument (shape, range, NULL, ordering) */
    RTSSA_E_UNSUPPORTED = -2, /* molecularity > 2 (the paper's own limit) or size beyond a mapping */
    RTSSA_E_HIP = -3,         /* a HIP runtime call failed */
    RTSSA_E_NOMEM = -4        /* device or host allocation failed */
} rtssa_status;

/* per-trajectory end states; NOT_RUN: the call's sample grid failed the
 * device-side check (see rtssa_simulate) and nothing was simulated */
enum { RTSSA_TRAJ_OK = 0, RTSSA_TRAJ_ABSORBED = 1, RTSSA_TRAJ_OVERFLOW = 2,
       RTSSA_TRAJ_MAX_FIRINGS = 3, RTSSA_TRAJ_NOT_RUN = 255 };

/* kernel mappings (work decomposition of one trajectory) */
enum { RTSSA_MAP_AUTO = 0, RTSSA_MAP_THREAD = 1, RTSSA_MAP_WAVE = 2, RTSSA_MAP_WORKGROUP = 3 };

#define RTSSA_TIE_NONE 0xFFFFFFFFu

typedef struct rtssa_network rtssa_network;

typedef struct {
    uint64_t firings;         /* applied events over all trajectories */
    uint64_t near_ties;       /* applied events with a near-tie (see above) */
    uint64_t clamps;          /* applied events whose raw gap was negative */
    uint64_t slow_logs;       /* Exp(1) draws that needed the accurate log phase */
    uint64_t status_count[4]; /* trajectories per end state */
    double kernel_ms;         /* device time of the simulation launch(es) */
    int32_t mapping;          /* mapping that ran */
    int32_t block;            /* workgroup size that ran */
    int32_t grid;             /* workgroups launched */
    int32_t bad_input;        /* 1: the sample grid failed the device-side check */
} rtssa_stats;

/* Simulation method.  RANDOM_TIME is the paper's next reaction random time
 * algorithm (section 4, Table 2), the library's method.  DIRECT is
 * Gillespie's direct method (section 3, Eq. 17-22), the method the paper
 * compares against: total rate a_0 = sum_k a_k summed in channel order,
 * waiting time RN(RN(-ln u1) / a_0), channel = the first whose running sum
 * reaches RN(u2 a_0); u1 (words 1:0) and u2 (words 3:2) from one
 * Philox4x32-10 block per firing at counter (firing index, 0xFFFFFFFF,
 * trajectory, net_id).  DIRECT runs only in the thread mapping (M, N <= 8)
 * and has no internal times: T_out and tie_step must be NULL.
 * LAZY is the random-time algorithm with the dependency-graph updates of
 * section 5 kept in internal times, for large networks: after a firing of mu
 * only mu and the channels of D(mu) are touched; each runs its internal
 * time from its last update s_k at its old propensity,
 * T_k = fma(a_k, RN(t - s_k), T_k) (mu: T_mu = P_mu, then P_mu += E), takes
 * its new a_k and the absolute next firing time
 * tau_k = t + max(0, RN(RN(P_k - T_k) RN(1 / a_k))) (+inf if a_k = 0); the
 * next event is the smallest tau_k, lowest k on ties; near-ties compare
 * RN(tau_(2) - t) with RN(tau_(1) - t).  Same draws and law as RANDOM_TIME,
 * its own rounding.  One wavefront per trajectory (stats.mapping =
 * RTSSA_MAP_WAVE, block 64) with the tree in LDS; mapping must be AUTO or
 * WAVE.  With a rate schedule, at a breakpoint b every channel runs its
 * clock to b at its old propensity, T_k = fma(a_k, RN(b - s_k), T_k),
 * s_k = b, and takes the new rates and a new tau_k from t = b (a negative gap
 * is clamped and counted as above); nothing fires at b.  E_UNSUPPORTED when
 * the tree does not fit LDS
 * (about 13,000 channels).  The first LAZY run of a network builds its
 * fixed-stride rows (about 270 bytes per channel of device memory, kept
 * until the network is destroyed); that first run must not overlap another
 * call on the same network from a second host thread.  Its channel workspace
 * (44 bytes per channel per resident wavefront) is allocated stream-ordered
 * by the call. */
/* DIRECT_TREE is the direct method with a_0 and the channel search on a
 * fixed sum tree of fan-out 8 over the channels (entries past M are 0; a
 * node adds its children pairwise, ((v0 + v1) + (v2 + v3)) + ((v4 + v5) +
 * (v6 + v7))), run like LAZY with one wavefront per trajectory for large
 * networks: tau = RN(E / a_0) with DIRECT's draws; the search starts at the
 * root with r = RN(u2 a_0) and at each node takes the first child with
 * v_i > 0 and r <= v_i (the last positive child if none), subtracting each
 * child it passes, r = RN(r - v_i).  Same law as DIRECT, its own rounding.
 * As DIRECT: T_out and tie_step must be NULL and no rate schedule; as LAZY:
 * mapping AUTO or WAVE, the same LDS limit and first-run rows. */
enum {
    RTSSA_METHOD_RANDOM_TIME = 0,
    RTSSA_METHOD_DIRECT = 1,
    RTSSA_METHOD_LAZY = 2,
    RTSSA_METHOD_DIRECT_TREE = 3
};

typedef struct {
    uint64_t max_firings;  /* per trajectory; 0 = 10^7; at most 2^32 - 1 */
    int32_t mapping;       /* RTSSA_MAP_*; 0 = chosen from the network size */
    int32_t block;         /* workgroup size; 0 = the mapping's default */
    int32_t grid;          /* workgroups of the persistent grid; 0 = fill the GPU */
    int32_t method;        /* RTSSA_METHOD_*; 0 = random time */
    /* device workspace of at least rtssa_workspace_size() bytes, 256-byte
     * aligned, owned by the caller and not shared with a call in flight;
     * NULL: the call allocates it stream-ordered and frees it after the
     * launch */
    void* workspace;
    uint64_t workspace_bytes;
} rtssa_options;

/* Message for the last failure on this thread (never NULL). */
const char* rtssa_last_error(void);

/* Library version string. */
const char* rtssa_version(void);

/*
 * Compile a network (paper Eq. 1-2, section 2; the paper's Table 4 model file
 * carries the same information).  All arrays are host memory and are copied.
 *   N species, M reactions (N, M >= 0).
 *   Reaction k consumes react_sigma[e] molecules of species react_species[e]
 *   for e in [react_ptr[k], react_ptr[k+1]) and produces prod_mult[e]
 *   molecules of prod_species[e] for e in [prod_ptr[k], prod_ptr[k+1]).
 *   c[k] >= 0 is the rate constant; 0 or within [1e-280, 1e280].
 * Errors: RTSSA_E_INVALID for bad pointers, indices, coefficients < 1,
 * repeated reactant species, non-monotone offsets or bad rates;
 * RTSSA_E_UNSUPPORTED when sum_j sigma_jk > 2 (molecularity limit of the
 * paper's GPU layout, section 5).  Builds the reactant table, the net-change
 * lists v_k and the dependency graph D(mu) = {k : k reads a species that mu
 * changes} (Gibson & Bruck, cited in section 5).
 */
int rtssa_network_create(int32_t N, int32_t M,
                         const int32_t* react_ptr, const int32_t* react_species,
                         const int32_t* react_sigma,
                         const int32_t* prod_ptr, const int32_t* prod_species,
                         const int32_t* prod_mult, const double* c,
                         rtssa_network** out);

/* Free a network handle and its device tables (NULL is ignored). */
int rtssa_network_destroy(rtssa_network* net);

/* Replace the rate constants (host array [M]); same validation as create.
 * Synchronous with respect to the host; do not call while a simulation of
 * this network is in flight. */
int rtssa_network_set_rates(rtssa_network* net, const double* c);

/* Query sizes of a compiled network: N, M, dependency-graph edges, and the
 * mapping the automatic choice selects. Any output pointer may be NULL. */
int rtssa_network_info(const rtssa_network* net, int32_t* N, int32_t* M,
                       int64_t* dep_edges, int32_t* auto_mapping);

/* Piecewise-constant rate constants (the time-dependent rates of the paper's
 * discussion, Eq. 28, solved piece by piece): the network's c applies on
 * [0, times[0]), rates[i*M .. i*M+M-1] from times[i] on.  times: B finite
 * values, > 0, strictly increasing; rates: B x M values, each 0 or within
 * [1e-280, 1e280].  Host arrays, copied.  B = 0 removes the schedule.  When
 * the next firing would fall after a breakpoint (before t_end), every
 * internal time runs to the breakpoint at the old rates
 * (T_k = fma(a_k, b - t, T_k)), t becomes the breakpoint and every a_k and
 * 1/a_k is recomputed with the new rates; no firing, no sample.  A network
 * with a schedule runs with the random-time method in every mapping and in
 * the LAZY form, not in DIRECT or DIRECT_TREE (E_UNSUPPORTED).  Call it only while no launch using
 * the network is in flight; while a batch holds the network it fails
 * with E_INVALID (the batch keeps the schedule's device address). */
int rtssa_network_set_schedule(rtssa_network* net, int32_t B, const double* times,
                               const double* rates);

/*
 * Device workspace, in bytes, of one rtssa_simulate call of this network with
 * R trajectories and these options (opt may be NULL): the run's counters and
 * work-queue heads, plus, for LAZY, one slice of channel records per resident
 * wavefront (about 44 bytes per channel each).  For LAZY, DIRECT_TREE and the
 * random-time sub-wave and workgroup mappings it also builds the network's fixed-stride
 * rows (its jumps and dependency lists, about 256 bytes per channel; for the
 * workgroup mapping also 64 dependency records of 32 bytes per channel) if they
 * are not built yet (synchronous; they are allocated once per network), so
 * that a later call with a caller workspace allocates nothing.  No stream
 * work otherwise.
 */
int rtssa_workspace_size(const rtssa_network* net, int64_t R, const rtssa_options* opt,
                         size_t* bytes);

/*
 * Simulate trajectories traj_offset .. traj_offset + R - 1 of the network on
 * the GPU (the whole hot path of section 4, Table 2, in one launch).
 *   x0        device int32 [N] (x0_per_traj = 0) or [R][N] (x0_per_traj = 1);
 *             counts must be >= 0 (not checked here: the values stay in
 *             device memory; negative counts give meaningless propensities).
 *   t_end     finite, >= 0.
 *   sample_t  device float64 [G], non-decreasing, within [0, t_end]
 *             (may be NULL when G = 0); checked on the device by the call's
 *             first kernel: a grid that fails the check simulates nothing,
 *             every status[r] becomes RTSSA_TRAJ_NOT_RUN, and with stats the
 *             call returns RTSSA_E_INVALID (stats->bad_input = 1).
 *   seed      Philox key; net_id is the fourth counter word.
 *   traj_offset + R <= 2^32.
 * Outputs, all device memory, any of them may be NULL to skip it:
 *   samples   int32, element (r, g, j) at r*s_stride_r + g*s_stride_g + j*s_stride_n
 *   n_out     uint32 [R][M] firings per channel
 *   T_out     float64 [R][M] internal times T_k(t_end) (Eq. 15)
 *   x_final   int32 [R][N]; t_last float64 [R] time of the last applied event
 *   status    uint8 [R] RTSSA_TRAJ_*; seq_hash uint64 [R]
 *   tie_step  uint32 [R] index of the first near-tie event, RTSSA_TIE_NONE if none
 * stats (host, may be NULL): when given, the call waits for the stream and
 * fills it; otherwise the call only enqueues work on the stream and returns
 * without waiting.
 * opt may be NULL (defaults).  With opt->workspace the call allocates
 * nothing and synchronises nothing unless stats is given, so it can be
 * captured into a caller's hipGraph (for LAZY, DIRECT_TREE and the
 * sub-wave and workgroup mappings the network's rows must have been built by
 * rtssa_workspace_size or an earlier run, else RTSSA_E_INVALID); without it
 * a workspace of rtssa_workspace_size() bytes is allocated stream-ordered
 * and freed after the launch.
 */
int rtssa_simulate(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                   double t_end, const double* sample_t, int32_t G,
                   uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                   int32_t* samples, int64_t s_stride_r, int64_t s_stride_g,
                   int64_t s_stride_n,
                   uint32_t* n_out, double* T_out, int32_t* x_final, double* t_last,
                   uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                   const rtssa_options* opt, rtssa_stream_t stream, rtssa_stats* stats);

/* Size of the library's fixed device scratch array (one per GPU). */
#define RTSSA_NOALLOC_SCRATCH_BYTES (4u << 20)

/*
 * rtssa_simulate for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, checks, kernels and results bit for bit, but the run's
 * counters, queue heads, item descriptor and (LAZY) channel records live in a
 * file-scope device array of RTSSA_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends.  The call allocates
 * and frees nothing (no hipMalloc, no events; stats->kernel_ms is 0).
 *   opt->workspace must be NULL.
 *   LAZY, DIRECT_TREE and the sub-wave and workgroup mappings need the network's rows
 *   built first (rtssa_workspace_size or an earlier rtssa_simulate), else
 *   E_INVALID.
 *   LAZY keeps only as many resident wavefronts as their channel records fit
 *   in the array (44 bytes per channel each; same results, fewer trajectories
 *   in flight); a run that does not fit one wavefront's records is rejected
 *   with E_UNSUPPORTED.
 * Every call on a GPU shares that GPU's array (the setup kernel clears what
 * must start at zero): calls that overlap on one GPU -- on two streams, or
 * from two host threads -- race and give wrong results.  Calls on one stream
 * are ordered and safe.
 */
int rtssa_simulate_noalloc(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                           double t_end, const double* sample_t, int32_t G,
                           uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                           int32_t* samples, int64_t s_stride_r, int64_t s_stride_g,
                           int64_t s_stride_n,
                           uint32_t* n_out, double* T_out, int32_t* x_final, double* t_last,
                           uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                           const rtssa_options* opt, rtssa_stream_t stream, rtssa_stats* stats);

/* Device workspace of rtssa_score_grad for R trajectories of M channels. */
int rtssa_score_grad_workspace_size(int64_t R, int32_t M, size_t* bytes);

/*
 * Score-function gradient of E[f(X_T)] with respect to log c_k.  For mass
 * action a_k = c_k h_k (Eq. 1), so the derivative of the path log-likelihood
 * in log c_k is n_k - T_k(t_end), read directly from the internal clocks of
 * Eq. 15.  With baseline = 1 the leave-one-out mean b_r = (sum f - f_r)/(R-1)
 * is subtracted (unbiased); baseline = 0 uses b = 0.
 *   f [R], n [R][M], T [R][M]: device inputs.
 *   grad [M], se [M]: device outputs (se = standard error of the mean of the
 *   per-path terms; se may be NULL).  R >= 1, M >= 1.
 *   workspace: device memory of rtssa_score_grad_workspace_size() bytes
 *   (8-byte aligned), or NULL to allocate it stream-ordered.
 * Deterministic: a fixed partition into blocks and a fixed reduction tree.
 */
int rtssa_score_grad(const double* f, const uint32_t* n, const double* T, int64_t R,
                     int32_t M, int32_t baseline, double* grad, double* se,
                     void* workspace, uint64_t workspace_bytes, rtssa_stream_t stream);

/* ---------------------------------------------------------------------
 * Batches: many independent networks in one launch.
 *
 * Each item is one rtssa_simulate call's worth of arguments (same meaning,
 * same validation).  rtssa_batch_create groups the items into classes by
 * kernel mapping (thread, sub-wavefront lanes per trajectory, workgroup
 * size; taken from the plan file written by rtssa_autotune when plan_path
 * names one, else from the network size), copies their descriptors to the
 * device and owns them; the caller keeps every network, input and output
 * buffer alive and unchanged in address until rtssa_batch_destroy (new rate
 * constants from rtssa_network_set_rates are seen by later runs; a rate
 * schedule cannot be changed meanwhile).  rtssa_batch_run runs
 * every item: with use_graph = 1 the first run captures a hipGraph (one
 * persistent kernel per class on parallel branches) and later runs replay
 * it; with 0 the kernels are enqueued directly.  The results equal those of
 * one rtssa_simulate per item with the same seed (and each item's net_id).
 * stats as in rtssa_simulate (the call then waits for the stream).
 */
typedef struct {
    const rtssa_network* net;
    const int32_t* x0;
    int32_t x0_per_traj;
    int32_t G;
    double t_end;
    const double* sample_t;
    uint32_t net_id;
    int32_t method;        /* RTSSA_METHOD_RANDOM_TIME (0), _LAZY or _DIRECT_TREE */
    uint64_t traj_offset;
    int64_t R;
    int32_t* samples;
    int64_t s_stride_r, s_stride_g, s_stride_n;
    uint32_t* n_out;
    double* T_out;
    int32_t* x_final;
    double* t_last;
    uint8_t* status;
    uint64_t* seq_hash;
    uint32_t* tie_step;
    /* The item's work for scheduling only (0: M x R): within a class the
     * items go to the device queue heaviest first, so that long runs start
     * early; e.g. the firings of a previous run of the same item.  Changes no
     * result.  Negative or non-finite: RTSSA_E_INVALID. */
    double weight;
} rtssa_batch_item;

typedef struct rtssa_batch rtssa_batch;

int rtssa_batch_create(const rtssa_batch_item* items, int32_t count, const rtssa_options* opt,
                       const char* plan_path, rtssa_batch** out);
int rtssa_batch_run(rtssa_batch* batch, uint64_t seed, int32_t use_graph, rtssa_stream_t stream,
                    rtssa_stats* stats);
/* Items may choose their method: RANDOM_TIME items are classed by mapping as
 * above; LAZY and DIRECT_TREE items (each with the same conditions as in
 * rtssa_simulate) form classes of their own, one per method and power-of-two
 * channel range (M <= 64, 65..128, 129..256, ...: each class's LDS tree is
 * sized for its own networks), run one wavefront per trajectory (reported as
 * mapping RTSSA_MAP_WAVE, 64 lanes) and are launched first, largest range
 * first; the lazy form's channel workspace is allocated by
 * rtssa_batch_create.  opt->method must be 0. */
/* cls < 0: *n_items receives the number of classes; else the class's
 * mapping, lanes per trajectory (1 for the thread mapping), items,
 * trajectories and largest channel count. */
int rtssa_batch_info(const rtssa_batch* batch, int32_t cls, int32_t* mapping, int32_t* lanes,
                     int32_t* n_items, int64_t* trajectories, int32_t* max_M);
/* Items of class cls (indices into the creation array, in the class's
 * queue order: heaviest first): *count receives the class's item count and
 * the first min(capacity, count) indices are written to items (may be NULL). */
int rtssa_batch_class_items(const rtssa_batch* batch, int32_t cls, int32_t* items,
                            int32_t capacity, int32_t* count);
int rtssa_batch_destroy(rtssa_batch* batch);

/* Autotuner: for every size class among the items (networks beyond the
 * thread mapping: sub-wavefront classes by lanes per trajectory, workgroup
 * classes by power-of-two channel ranges), time each feasible lane count /
 * workgroup size on a sub-batch of up to `samples` items of the class, run
 * as the batch runs it (one shared persistent grid; outputs not written; at
 * most 4000 firings per trajectory; items with a shared x0 run with more
 * trajectories so that the sub-batch fills the device), and write the
 * fastest, in firings per second, to the plan file plan_path (text lines
 * "wave|workgroup M_lo M_hi L").  Returns the number of classes tuned (>= 0)
 * or a negative error code.  Synchronous; allocates and frees device memory.
 */
int rtssa_autotune(const rtssa_batch_item* items, int32_t count, int32_t samples,
                   const char* plan_path, rtssa_stream_t stream);

/* ---------------------------------------------------------------------
 * Test hooks: the library's own Philox and -ln(u), for checking its
 * arithmetic element by element.  The *_host variants run the same source
 * compiled for the CPU; the device variants launch a kernel.
 */
/* out[i] = RN(-ln((m[i]+1) 2^-53)); force_accurate = 1 skips the fast phase;
 * slow (may be NULL) receives 1 where the accurate phase ran. */
int rtssa_debug_neglog(const uint64_t* m, double* out, uint8_t* slow, int64_t count,
                       int32_t force_accurate, rtssa_stream_t stream);
double rtssa_debug_neglog_host(uint64_t m, int32_t force_accurate, int32_t* slow);
/* The fast phase's double-double approximation yh + yl of -ln u (m < 2^53 - 1). */
void rtssa_debug_neglog_fast_host(uint64_t m, double* yh, double* yl);
/* The selection step (Eq. 25) and the near-tie rule of one mapping, run by
 * the same device functions as the simulation kernels on given values:
 * v device float64 [count][M] (no NaN; +inf allowed); per row r:
 * mu[r] = the lowest k among the smallest values, v1[r] that value,
 * v2[r] the second smallest counted with multiplicity (+inf if none),
 * near[r] = 1 when RN(v2 - v1) <= RN(1e-12 v1).  mu is meaningful only when
 * v1 is finite.  mapping RTSSA_MAP_THREAD: one lane per row, channels in
 * order; RTSSA_MAP_WAVE: groups of lanes = 2..64 lanes of a wavefront, lane l
 * holding channels l + s lanes, reduced by lane exchanges; RTSSA_MAP_WORKGROUP:
 * one workgroup of lanes = 64..1024 threads per row, wavefronts merged through
 * LDS; RTSSA_DEBUG_MAP_WORKGROUP_LDS: the selection of the workgroup kernel
 * that keeps the propensities in LDS (lane minima, then a smallest-value
 * reduction per wavefront and one merge through LDS), whose v2 is exact
 * whenever the near-tie test can hold and otherwise a value no smaller than
 * the true second smallest and out of its reach.  Outputs are device memory:
 * mu int32 [count], v1 and v2 float64 [count], near uint8 [count]. */
#define RTSSA_DEBUG_MAP_WORKGROUP_LDS 4
int rtssa_debug_select(const double* v, int32_t M, int64_t count, int32_t mapping,
                       int32_t lanes, int32_t* mu, double* v1, double* v2, uint8_t* near,
                       rtssa_stream_t stream);
/* out[4i..4i+3] = Philox4x32-10(ctr[4i..4i+3], key) */
int rtssa_debug_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, uint32_t* out,
                       int64_t count, rtssa_stream_t stream);
void rtssa_debug_philox_host(const uint32_t ctr[4], uint32_t key0, uint32_t key1,
                             uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif
