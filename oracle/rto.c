/*
 * rto.c -- CPU oracle for the next-reaction random-time algorithm (NRRTA) of
 * Liu & Wang, arXiv:2103.00405.
 *
 * TEST INFRASTRUCTURE ONLY: this is the plain, slow, obviously-correct
 * reference for the GPU library.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code with the GPU path.
 *
 * What it computes, per trajectory (paper section 4, Table 2, with the
 * internal-time bookkeeping of the random time-change representation,
 * Eq. 14-16, and the per-channel exponential gaps of Eq. 23-26):
 *
 *   state: t, X[N], and per channel k: T_k (internal time elapsed, Eq. 15),
 *          P_k (internal time of the next firing of channel k), n_k (firings).
 *   init : t = 0, X = x0, T_k = 0, n_k = 0, P_k = E(k, 0).
 *   loop : a_k = c_k h_k(X)                          (Eq. 1-2)
 *          gap_k = (P_k - T_k) / a_k  (+inf if a_k = 0, frozen channel)
 *          mu = argmin_k gap_k, Delta = gap_mu       (Eq. 25)
 *          stop if Delta = +inf (absorbed) or t + Delta > t_end
 *          T_k += a_k Delta for k != mu, T_mu = P_mu (Eq. 15 over [t, t+Delta])
 *          X += nu_mu, n_mu += 1, P_mu += E(mu, n_mu) (Eq. 26: only the fired
 *          channel receives a fresh unit-exponential internal gap)
 *   end  : T_k += a_k (t_end - t) for every k.
 *
 * Readings where the paper is silent (all fixed so that a second
 * implementation can reproduce every bit):
 *  - h_k = prod_j C(X_j, sigma_jk); C(X,2) = X(X-1)/2 (Eq. 2 prints X_k for X_j).
 *  - The unfired channels keep their absolute next internal firing time P_k;
 *    their remaining gap is P_k - T_k (Eq. 26 literally says the gap is kept).
 *  - Arithmetic: IEEE binary64, round to nearest even.  h_k is exact in int64
 *    and converted with one rounding; a_k = RN(c_k * h); inv_k = RN(1 / a_k);
 *    gap_k = RN(RN(P_k - T_k) * inv_k), clamped below at 0; T update is one
 *    fused multiply-add; E is RN(-ln u), correctly rounded.
 *  - Ties: the lowest k wins.  A near-tie is counted when
 *    RN(d2 - d1) <= RN(1e-12 * d1), d1 <= d2 the two smallest gaps.
 *  - An event with t + Delta > t_end is not applied.
 *  - Samples: before applying an event at t_new every grid point s_g < t_new
 *    receives the current X (right-continuous path).  At the end every
 *    remaining grid point receives the final X.  After an overflow or the
 *    firing cap the remaining grid points receive -1.
 *  - Overflow: an event that would take a count outside [0, 2^31-1] is not
 *    applied; the trajectory stops with status OVERFLOW.
 *  - E(seed, traj, net, k, n): Philox4x32-10 (Salmon, Moraes, Dror & Shaw,
 *    SC'11), key (seed_lo, seed_hi), counter (n >> 1, k, traj, net); the
 *    64-bit word is (w1:w0) for even n and (w3:w2) for odd n; m = word >> 11,
 *    u = (m + 1) 2^-53 in (0, 1]; E = RN(-ln u), E(u = 1) = +0.
 *  - seq_hash: h = 0xcbf29ce484222325, then h = (h ^ mu) * 0x100000001b3
 *    (mod 2^64) for every applied event.
 */
#include "rto.h"

#include <math.h>
#include <pthread.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define TIE_NONE 0xFFFFFFFFu

/* ---------------------------------------------------------------- Philox */
/* Philox4x32 with 10 rounds, from the published definition: each round
 * multiplies words 0 and 2 by M0 and M1, mixes the high halves with words
 * 1 and 3 and the key, and the key is bumped by the Weyl constants between
 * rounds. */
void rto_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------ Exp(1) draw */
/* RN(-ln u), u = (m+1) 2^-53.  The binary128 logarithm is accurate to a few
 * units in its 113-bit last place; its rounding to binary64 is the correctly
 * rounded result unless the binary128 value sits within 2^-105 (relative) of
 * a binary64 rounding boundary, which is reported as a hard case (-1). */
double rto_neglog_u53(uint64_t m)
{
    double u = (double)(m + 1) * 0x1p-53;          /* exact: m + 1 <= 2^53 */
    if (u == 1.0) return 0.0;
    __float128 q = -logq((__float128)u);
    double d = (double)q;
    __float128 dq = (__float128)d;
    __float128 up = (__float128)nextafter(d, INFINITY);
    __float128 dn = (__float128)nextafter(d, 0.0);
    __float128 mid_up = (dq + up) / 2, mid_dn = (dq + dn) / 2; /* exact */
    __float128 margin = q * 0x1p-105Q;
    if (fabsq(q - mid_up) <= margin || fabsq(q - mid_dn) <= margin) return -1.0;
    return d;
}

double rto_exp1(uint64_t seed, uint32_t traj, uint32_t net_id, uint32_t k, uint32_t n)
{
    uint32_t ctr[4] = { n >> 1, k, traj, net_id };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    rto_philox4x32_10(ctr, key, w);
    uint64_t word = (n & 1u) ? (((uint64_t)w[3] << 32) | w[2])
                             : (((uint64_t)w[1] << 32) | w[0]);
    return rto_neglog_u53(word >> 11);
}

/* ------------------------------------------------------------ propensity */
/* C(x, s) for s in {0, 1, 2}, exact in int64. */
static int64_t choose(int64_t x, int32_t s)
{
    if (s == 0) return 1;
    if (s == 1) return x;
    if (x < 2) return 0;
    return x * (x - 1) / 2;
}

/* a_k = c_k * h_k(X), h_k = prod over reactant entries of C(X_j, sigma_j)
 * (Eq. 1-2); the product has at most two factors (molecularity <= 2).
 * c is the rate constant in force (the network's, or a schedule piece's). */
static double propensity_c(const rto_network* net, const int32_t* X, int k, double c)
{
    int64_t h = 1;
    for (int e = net->react_ptr[k]; e < net->react_ptr[k + 1]; e++)
        h *= choose(X[net->react_species[e]], net->react_sigma[e]);
    return c * (double)h;
}

static double propensity(const rto_network* net, const int32_t* X, int k)
{
    return propensity_c(net, X, k, net->c[k]);
}

/* ------------------------------------------------------------ selection */
/* The selection step of Eq. 25 over M values (the gaps of the eager form,
 * or the absolute next firing times of the lazy form): *mu is the lowest k
 * among the smallest values and *v1 that value; *v2 is the second smallest
 * value counted with multiplicity, so two equal smallest values give
 * *v2 = *v1, and *v2 = +inf when fewer than two values are finite.  When no
 * value is finite (nothing can fire, or M = 0), *mu = -1 and *v1 = +inf.
 * Values are never NaN.  Both path functions below select through this one
 * function. */
void rto_argmin2(const double* v, int32_t M, int32_t* mu, double* v1, double* v2)
{
    int32_t best = -1;
    double d1 = INFINITY, d2 = INFINITY;
    for (int32_t k = 0; k < M; k++) {
        if (v[k] < d1) { d2 = d1; d1 = v[k]; best = k; }
        else if (v[k] < d2) { d2 = v[k]; }
    }
    *mu = best;
    *v1 = d1;
    *v2 = d2;
}

/* The near-tie rule for the two smallest gaps d1 <= d2 (finite d1): they are
 * within 1e-12 relative when RN(d2 - d1) <= RN(1e-12 d1).  Eq. 4 gives ties
 * probability zero; in binary64 a near-tie is where another rounding order
 * could select another channel, so every such event is counted and the first
 * one's firing index reported. */
int rto_near_tie(double d1, double d2)
{
    return d2 - d1 <= 1e-12 * d1;
}

/* ------------------------------------------------------------ one path */
typedef struct {
    const rto_network* net;
    const int32_t* nu_ptr;      /* net change nu_k as (species, delta) lists */
    const int32_t* nu_species;
    const int32_t* nu_delta;
    const int32_t* x0;
    int32_t x0_per_traj;
    double t_end;
    const double* s;
    int32_t G;
    uint64_t seed;
    uint32_t net_id;
    uint64_t traj_offset;
    uint64_t max_firings;
    int32_t *samples, *x_final;
    uint32_t *n_out, *tie_step;
    double *T_out, *t_last;
    uint8_t* status;
    uint64_t* seq_hash;
    int64_t r_begin, r_end;
    int32_t method;             /* 0: random time (Table 2), 1: direct method, 2: lazy form,
                                   3: direct method on a sum tree */
    const int32_t* dep_ptr;     /* D(mu) lists (lazy form) */
    const int32_t* dep_idx;
    int32_t B;                  /* rate breakpoints (0: constant rates) */
    const double* sched_t;      /* [B] breakpoint times */
    const double* sched_c;      /* [B][M] rates from each breakpoint on */
    rto_stats stats;
} job_t;

static void write_sample(job_t* jb, int64_t r, int32_t g, const int32_t* X, int fill_invalid)
{
    int N = jb->net->N;
    int32_t* dst = jb->samples + ((size_t)r * jb->G + g) * N;
    for (int j = 0; j < N; j++) dst[j] = fill_invalid ? -1 : X[j];
}

static void simulate_path(job_t* jb, int64_t r, int32_t* X, double* T, double* P,
                          double* a, double* inv, uint32_t* n, double* gap)
{
    const rto_network* net = jb->net;
    const int N = net->N, M = net->M;
    const uint32_t traj = (uint32_t)(jb->traj_offset + (uint64_t)r);
    const uint64_t seed = jb->seed;
    const uint32_t nid = jb->net_id;

    const int32_t* x0 = jb->x0 + (jb->x0_per_traj ? (size_t)r * N : 0);
    for (int j = 0; j < N; j++) X[j] = x0[j];
    double t = 0.0;
    /* piecewise-constant rates: the network's c before the first breakpoint,
     * row i of sched_c from breakpoint i on */
    const double* crate = net->c;
    int32_t piece = 0;
    double b_next = jb->B > 0 ? jb->sched_t[0] : INFINITY;
    for (int k = 0; k < M; k++) {
        T[k] = 0.0;
        n[k] = 0;
        P[k] = rto_exp1(seed, traj, nid, (uint32_t)k, 0);
        if (P[k] < 0) jb->stats.hard_cases++;
        a[k] = propensity_c(net, X, k, crate[k]);
        inv[k] = a[k] > 0 ? 1.0 / a[k] : 0.0;
    }
    int32_t g = 0;
    uint64_t fired = 0;
    uint8_t st = RTO_OK;
    uint32_t tie = TIE_NONE;
    uint64_t hash = 0xcbf29ce484222325ull;

    for (;;) {
        /* gaps (Eq. 23-24 in internal time), then the selection of Eq. 25:
         * lowest k among the minimal gaps; d2 is the second order statistic */
        for (int k = 0; k < M; k++) {
            if (a[k] == 0.0) {
                gap[k] = INFINITY;
            } else {
                double d = (P[k] - T[k]) * inv[k];
                gap[k] = d < 0.0 ? 0.0 : d;
            }
        }
        int32_t mu;
        double d1, d2;
        rto_argmin2(gap, M, &mu, &d1, &d2);
        double t_new = t + d1;
        /* Eq. 28 with piecewise-constant c_k(t): when the next firing would
         * fall after a rate breakpoint (before t_end), every internal clock
         * runs to the breakpoint at the old rates, the propensities take the
         * new rates, and the gaps are solved again from there */
        if (b_next < jb->t_end && t_new > b_next) {
            double db = b_next - t;
            for (int k = 0; k < M; k++) T[k] = fma(a[k], db, T[k]);
            t = b_next;
            crate = jb->sched_c + (size_t)piece * M;
            piece += 1;
            b_next = piece < jb->B ? jb->sched_t[piece] : INFINITY;
            for (int k = 0; k < M; k++) {
                a[k] = propensity_c(net, X, k, crate[k]);
                inv[k] = a[k] > 0 ? 1.0 / a[k] : 0.0;
            }
            continue;
        }
        if (d1 == INFINITY) { st = RTO_ABSORBED; break; }
        if (t_new > jb->t_end) break;
        if (rto_near_tie(d1, d2)) {
            jb->stats.near_ties++;
            if (tie == TIE_NONE) tie = (uint32_t)fired;
        }
        while (g < jb->G && jb->s[g] < t_new) { write_sample(jb, r, g, X, 0); g++; }
        /* the state jump must stay inside [0, 2^31 - 1] */
        int ok = 1;
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++) {
            int64_t v = (int64_t)X[jb->nu_species[e]] + jb->nu_delta[e];
            if (v < 0 || v > INT32_MAX) ok = 0;
        }
        if (!ok) { st = RTO_OVERFLOW; break; }
        if ((P[mu] - T[mu]) * inv[mu] < 0.0) jb->stats.clamps++;
        /* internal times advance by a_k * Delta (Eq. 15); the fired channel
         * lands exactly on its firing internal time */
        for (int k = 0; k < M; k++)
            if (k != mu) T[k] = fma(a[k], d1, T[k]);
        T[mu] = P[mu];
        t = t_new;
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++)
            X[jb->nu_species[e]] += jb->nu_delta[e];
        n[mu] += 1;
        fired += 1;
        hash = (hash ^ (uint64_t)(uint32_t)mu) * 0x100000001b3ull;
        double E = rto_exp1(seed, traj, nid, (uint32_t)mu, n[mu]);
        if (E < 0) jb->stats.hard_cases++;
        P[mu] = P[mu] + E;
        /* a_k is a pure function of X: recomputing every channel equals
         * recomputing only the channels that read a changed species */
        for (int k = 0; k < M; k++) {
            a[k] = propensity_c(net, X, k, crate[k]);
            inv[k] = a[k] > 0 ? 1.0 / a[k] : 0.0;
        }
        if (fired >= jb->max_firings) { st = RTO_MAX_FIRINGS; break; }
    }

    if (st == RTO_OK || st == RTO_ABSORBED) {
        while (g < jb->G) { write_sample(jb, r, g, X, 0); g++; }
        double dt = jb->t_end - t;
        for (int k = 0; k < M; k++) T[k] = fma(a[k], dt, T[k]);
    } else {
        while (g < jb->G) { write_sample(jb, r, g, X, 1); g++; }
    }

    for (int k = 0; k < M; k++) {
        jb->n_out[(size_t)r * M + k] = n[k];
        jb->T_out[(size_t)r * M + k] = T[k];
    }
    for (int j = 0; j < N; j++) jb->x_final[(size_t)r * N + j] = X[j];
    jb->t_last[r] = t;
    jb->status[r] = st;
    jb->seq_hash[r] = hash;
    jb->tie_step[r] = tie;
    jb->stats.firings += fired;
    jb->stats.status_count[st]++;
}

/* ------------------------------------------------ the lazy form */
/* Section 5 recalls Gibson and Bruck's dependency graph: after a firing only
 * the channels whose propensity reads a species the firing changed get new
 * propensities.  Kept in internal times (Eq. 14-16), that gives a lazy form of
 * the same algorithm: a channel's internal time is brought up to date only
 * when its propensity changes or it fires, and the next event belongs to the
 * channel with the smallest absolute next firing time tau_k (t + gap_k in
 * exact arithmetic).  The draws E(k, n) and the law are those of
 * simulate_path; the rounding differs, so this is a reference of its own.
 *
 *   per channel: T_k is the internal time at time s_k; a_k is the propensity
 *     in force since s_k; tau_k = +inf if a_k = 0, else
 *     s_k + max(0, RN(RN(P_k - T_k) * inv_k)).
 *   event: mu = the lowest k among the smallest tau_k, t_new = tau_mu;
 *     d1 = RN(t_new - t) and d2 = RN(tau_(2) - t) (second smallest tau) feed
 *     the near-tie rule of simulate_path.  Then T_mu = P_mu,
 *     P_mu += E(mu, n_mu), s_mu = t_new; every other k in D(mu):
 *     T_k = fma(a_k, RN(t_new - s_k), T_k), s_k = t_new; every k in D(mu) and
 *     mu get new a_k, inv_k and tau_k (a negative raw gap is clamped to 0
 *     and counted).
 *   end: T_k = fma(a_k, RN(t_stop - s_k), T_k) for every k, with t_stop =
 *     t_end after OK or ABSORBED and the last event's time otherwise.
 *   rate schedule (piecewise-constant c_k(t), as in simulate_path): when the
 *     smallest tau_k lies past the next breakpoint b (b < t_end), every
 *     channel runs its clock to b at its old propensity,
 *     T_k = fma(a_k, RN(b - s_k), T_k), s_k = b, takes the new rates and a new
 *     tau_k from t = b; nothing fires.
 * D(mu) holds the channels with a reactant species whose net change in nu_mu
 * is not zero (build_deps). */
static void lazy_refresh(job_t* jb, const int32_t* X, int k, double t, const double* T,
                         const double* P, double* a, double* inv, double* tau,
                         const double* crate)
{
    a[k] = propensity_c(jb->net, X, k, crate[k]);
    inv[k] = a[k] > 0 ? 1.0 / a[k] : 0.0;
    if (a[k] == 0.0) {
        tau[k] = INFINITY;
        return;
    }
    double gap = (P[k] - T[k]) * inv[k];
    if (gap < 0.0) {
        jb->stats.clamps++;
        gap = 0.0;
    }
    tau[k] = t + gap;
}

static void simulate_path_lazy(job_t* jb, int64_t r, int32_t* X, double* T, double* P,
                               double* a, double* inv, uint32_t* n, double* s_up, double* tau)
{
    const rto_network* net = jb->net;
    const int N = net->N, M = net->M;
    const uint32_t traj = (uint32_t)(jb->traj_offset + (uint64_t)r);
    const uint64_t seed = jb->seed;
    const uint32_t nid = jb->net_id;

    const int32_t* x0 = jb->x0 + (jb->x0_per_traj ? (size_t)r * N : 0);
    for (int j = 0; j < N; j++) X[j] = x0[j];
    double t = 0.0;
    const double* crate = net->c;
    int32_t piece = 0;
    double b_next = jb->B > 0 ? jb->sched_t[0] : INFINITY;
    for (int k = 0; k < M; k++) {
        T[k] = 0.0;
        s_up[k] = 0.0;
        n[k] = 0;
        P[k] = rto_exp1(seed, traj, nid, (uint32_t)k, 0);
        if (P[k] < 0) jb->stats.hard_cases++;
        lazy_refresh(jb, X, k, 0.0, T, P, a, inv, tau, crate);
    }
    int32_t g = 0;
    uint64_t fired = 0;
    uint8_t st = RTO_OK;
    uint32_t tie = TIE_NONE;
    uint64_t hash = 0xcbf29ce484222325ull;

    for (;;) {
        int32_t mu;
        double tau1, tau2;
        rto_argmin2(tau, M, &mu, &tau1, &tau2);
        double t_new = tau1;
        if (b_next < jb->t_end && t_new > b_next) {
            for (int k = 0; k < M; k++) {
                T[k] = fma(a[k], b_next - s_up[k], T[k]);
                s_up[k] = b_next;
            }
            t = b_next;
            crate = jb->sched_c + (size_t)piece * M;
            piece += 1;
            b_next = piece < jb->B ? jb->sched_t[piece] : INFINITY;
            for (int k = 0; k < M; k++) lazy_refresh(jb, X, k, t, T, P, a, inv, tau, crate);
            continue;
        }
        if (tau1 == INFINITY) { st = RTO_ABSORBED; break; }
        if (t_new > jb->t_end) break;
        double d1 = t_new - t, d2 = tau2 - t;
        if (rto_near_tie(d1, d2)) {
            jb->stats.near_ties++;
            if (tie == TIE_NONE) tie = (uint32_t)fired;
        }
        while (g < jb->G && jb->s[g] < t_new) { write_sample(jb, r, g, X, 0); g++; }
        int ok = 1;
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++) {
            int64_t v = (int64_t)X[jb->nu_species[e]] + jb->nu_delta[e];
            if (v < 0 || v > INT32_MAX) ok = 0;
        }
        if (!ok) { st = RTO_OVERFLOW; break; }
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++)
            X[jb->nu_species[e]] += jb->nu_delta[e];
        t = t_new;
        n[mu] += 1;
        fired += 1;
        hash = (hash ^ (uint64_t)(uint32_t)mu) * 0x100000001b3ull;
        /* the fired channel lands on its firing internal time and gets the
         * next one (Eq. 26) */
        T[mu] = P[mu];
        s_up[mu] = t;
        const uint32_t n_mu = n[mu];
        double E_mu = rto_exp1(seed, traj, nid, (uint32_t)mu, n_mu);
        if (E_mu < 0) jb->stats.hard_cases++;
        P[mu] += E_mu;
        lazy_refresh(jb, X, mu, t, T, P, a, inv, tau, crate);
        /* each dependent runs its clock to t at its old propensity (Eq. 15),
         * then takes the new one */
        for (int q = jb->dep_ptr[mu]; q < jb->dep_ptr[mu + 1]; q++) {
            int k = jb->dep_idx[q];
            if (k == mu) continue;
            T[k] = fma(a[k], t - s_up[k], T[k]);
            s_up[k] = t;
            lazy_refresh(jb, X, k, t, T, P, a, inv, tau, crate);
        }
        if (fired >= jb->max_firings) { st = RTO_MAX_FIRINGS; break; }
    }

    int good = st == RTO_OK || st == RTO_ABSORBED;
    double t_stop = good ? jb->t_end : t;
    for (int k = 0; k < M; k++) T[k] = fma(a[k], t_stop - s_up[k], T[k]);
    while (g < jb->G) { write_sample(jb, r, g, X, !good); g++; }
    for (int k = 0; k < M; k++) {
        jb->n_out[(size_t)r * M + k] = n[k];
        jb->T_out[(size_t)r * M + k] = T[k];
    }
    for (int j = 0; j < N; j++) jb->x_final[(size_t)r * N + j] = X[j];
    jb->t_last[r] = t;
    jb->status[r] = st;
    jb->seq_hash[r] = hash;
    jb->tie_step[r] = tie;
    jb->stats.firings += fired;
    jb->stats.status_count[st]++;
}

/* ------------------------------------------------ the direct method */
/* Gillespie's direct method, the comparison method of section 3 and of the
 * discussion (Eq. 17-22): with the total rate a_0 = sum_k a_k (summed in
 * channel order), the waiting time is an Exp(1) draw divided by a_0 (the
 * 1/a_0 that Eq. 22 leaves out), and the firing channel is found by searching
 * the running sums for the first to reach a uniform fraction of a_0.  Both
 * numbers come from one Philox4x32-10 block per firing, at counter
 * (firing index, 0xFFFFFFFF, trajectory, net_id): words 1:0 give the waiting
 * time's u, words 3:2 the search's u, each u = (m + 1) 2^-53 with m the top
 * 53 bits.  The second counter word is never a channel index of the random
 * time draws, so the two methods' streams do not overlap. */
/* The two numbers of one direct-method firing from its Philox block: returns
 * E = RN(-ln u1) (-1 for a hard case) and sets *m2, the search's 53 bits. */
static double direct_draws(const job_t* jb, uint32_t traj, uint64_t fired, uint64_t* m2_out)
{
    const uint32_t key[2] = { (uint32_t)jb->seed, (uint32_t)(jb->seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)fired, 0xFFFFFFFFu, traj, jb->net_id };
    uint32_t w[4];
    rto_philox4x32_10(ctr, key, w);
    uint64_t m1 = ((((uint64_t)w[1] << 32) | w[0]) >> 11);
    uint64_t m2 = ((((uint64_t)w[3] << 32) | w[2]) >> 11);
    *m2_out = m2;
    return rto_neglog_u53(m1);
}

static void simulate_path_direct(job_t* jb, int64_t r, int32_t* X, double* a, uint32_t* n)
{
    const rto_network* net = jb->net;
    const int N = net->N, M = net->M;
    const uint32_t traj = (uint32_t)(jb->traj_offset + (uint64_t)r);

    const int32_t* x0 = jb->x0 + (jb->x0_per_traj ? (size_t)r * N : 0);
    for (int j = 0; j < N; j++) X[j] = x0[j];
    for (int k = 0; k < M; k++) n[k] = 0;
    double t = 0.0;
    int32_t g = 0;
    uint64_t fired = 0;
    uint8_t st = RTO_OK;
    uint64_t hash = 0xcbf29ce484222325ull;

    for (;;) {
        double a0 = 0.0;
        for (int k = 0; k < M; k++) {
            a[k] = propensity(net, X, k);
            a0 += a[k];
        }
        if (a0 == 0.0) { st = RTO_ABSORBED; break; }
        uint64_t m2;
        double E = direct_draws(jb, traj, fired, &m2);
        if (E < 0) jb->stats.hard_cases++;
        double tau = E / a0;
        double t_new = t + tau;
        if (t_new > jb->t_end) break;
        while (g < jb->G && jb->s[g] < t_new) { write_sample(jb, r, g, X, 0); g++; }
        /* the first channel whose running sum reaches u a_0 */
        double target = (double)(m2 + 1) * 0x1p-53 * a0;
        int mu = M - 1;
        double run = 0.0;
        for (int k = 0; k < M; k++) {
            run += a[k];
            if (run >= target) { mu = k; break; }
        }
        int ok = 1;
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++) {
            int64_t v = (int64_t)X[jb->nu_species[e]] + jb->nu_delta[e];
            if (v < 0 || v > INT32_MAX) ok = 0;
        }
        if (!ok) { st = RTO_OVERFLOW; break; }
        t = t_new;
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++)
            X[jb->nu_species[e]] += jb->nu_delta[e];
        n[mu] += 1;
        fired += 1;
        hash = (hash ^ (uint64_t)(uint32_t)mu) * 0x100000001b3ull;
        if (fired >= jb->max_firings) { st = RTO_MAX_FIRINGS; break; }
    }

    int bad = !(st == RTO_OK || st == RTO_ABSORBED);
    while (g < jb->G) { write_sample(jb, r, g, X, bad); g++; }
    for (int k = 0; k < M; k++) jb->n_out[(size_t)r * M + k] = n[k];
    for (int j = 0; j < N; j++) jb->x_final[(size_t)r * N + j] = X[j];
    jb->t_last[r] = t;
    jb->status[r] = st;
    jb->seq_hash[r] = hash;
    jb->stats.firings += fired;
    jb->stats.status_count[st]++;
}

/* ------------------------------------------------ the direct method on a sum tree */
/* The direct method with the total rate and the channel search taken on a
 * fixed tree of fan-out 8 over the channels, the form in which a wavefront
 * sums and searches in parallel.  Level 0 holds a_k (entries past M are 0);
 * a node of level l is the sum of its 8 children of level l - 1 added
 * pairwise, ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)); the top level
 * has one node, a_0.  The waiting time is RN(E / a_0) with E and u2 drawn as
 * in simulate_path_direct.  The search starts at the root with r = RN(u2 a_0)
 * and, at each node, scans its children in order: it takes the first child
 * with v_i > 0 and r <= v_i, or the last child with v_i > 0 if r passes them
 * all, and subtracts each child it passes, r = RN(r - v_i); at level 1 the
 * child taken is the channel.  Same draws as simulate_path_direct, its own
 * rounding. */
#define DT_FAN 8

/* level sizes of the tree over M leaves; returns the top level */
static int dt_levels(int M, int* cnt)
{
    int L = 0;
    cnt[0] = M > 0 ? M : 1;
    while (cnt[L] > 1 || L == 0) {
        cnt[L + 1] = (cnt[L] + DT_FAN - 1) / DT_FAN;
        L++;
    }
    return L;
}

static double dt_node(const double* child, int n, int j)
{
    double v[DT_FAN];
    for (int i = 0; i < DT_FAN; i++) v[i] = j * DT_FAN + i < n ? child[j * DT_FAN + i] : 0.0;
    return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

static void simulate_path_direct_tree(job_t* jb, int64_t r, int32_t* X, double* a, uint32_t* n)
{
    const rto_network* net = jb->net;
    const int N = net->N, M = net->M;
    const uint32_t traj = (uint32_t)(jb->traj_offset + (uint64_t)r);
    int cnt[40];
    const int top = dt_levels(M, cnt);
    double* lev[40];
    for (int l = 1; l <= top; l++) lev[l] = (double*)malloc(sizeof(double) * cnt[l]);

    const int32_t* x0 = jb->x0 + (jb->x0_per_traj ? (size_t)r * N : 0);
    for (int j = 0; j < N; j++) X[j] = x0[j];
    for (int k = 0; k < M; k++) n[k] = 0;
    double t = 0.0;
    int32_t g = 0;
    uint64_t fired = 0;
    uint8_t st = RTO_OK;
    uint64_t hash = 0xcbf29ce484222325ull;

    for (;;) {
        /* every propensity and every node again (the tree is a function of X) */
        for (int k = 0; k < M; k++) a[k] = propensity(net, X, k);
        if (M == 0) a[0] = 0.0;
        for (int l = 1; l <= top; l++) {
            const double* child = l == 1 ? a : lev[l - 1];
            for (int j = 0; j < cnt[l]; j++) lev[l][j] = dt_node(child, cnt[l - 1], j);
        }
        const double a0 = lev[top][0];
        if (a0 == 0.0) { st = RTO_ABSORBED; break; }
        uint64_t m2;
        double E = direct_draws(jb, traj, fired, &m2);
        if (E < 0) jb->stats.hard_cases++;
        double t_new = t + E / a0;
        if (t_new > jb->t_end) break;
        while (g < jb->G && jb->s[g] < t_new) { write_sample(jb, r, g, X, 0); g++; }
        /* the search, from the root down */
        double rem = (double)(m2 + 1) * 0x1p-53 * a0;
        int j = 0;
        for (int l = top; l >= 1; l--) {
            const double* child = l == 1 ? a : lev[l - 1];
            int last = -1;
            for (int i = 0; i < DT_FAN; i++)
                if (j * DT_FAN + i < cnt[l - 1] && child[j * DT_FAN + i] > 0.0) last = i;
            int take = last;
            for (int i = 0; i < last; i++) {
                const double v = child[j * DT_FAN + i];
                if (v > 0.0 && rem <= v) { take = i; break; }
                rem = rem - v;
            }
            j = j * DT_FAN + take;
        }
        const int mu = j;
        int ok = 1;
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++) {
            int64_t v = (int64_t)X[jb->nu_species[e]] + jb->nu_delta[e];
            if (v < 0 || v > INT32_MAX) ok = 0;
        }
        if (!ok) { st = RTO_OVERFLOW; break; }
        t = t_new;
        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++)
            X[jb->nu_species[e]] += jb->nu_delta[e];
        n[mu] += 1;
        fired += 1;
        hash = (hash ^ (uint64_t)(uint32_t)mu) * 0x100000001b3ull;
        if (fired >= jb->max_firings) { st = RTO_MAX_FIRINGS; break; }
    }

    int bad = !(st == RTO_OK || st == RTO_ABSORBED);
    while (g < jb->G) { write_sample(jb, r, g, X, bad); g++; }
    for (int k = 0; k < M; k++) jb->n_out[(size_t)r * M + k] = n[k];
    for (int j2 = 0; j2 < N; j2++) jb->x_final[(size_t)r * N + j2] = X[j2];
    jb->t_last[r] = t;
    jb->status[r] = st;
    jb->seq_hash[r] = hash;
    jb->stats.firings += fired;
    jb->stats.status_count[st]++;
    for (int l = 1; l <= top; l++) free(lev[l]);
}

static void* run_job(void* arg)
{
    job_t* jb = (job_t*)arg;
    int N = jb->net->N, M = jb->net->M;
    int32_t* X = (int32_t*)malloc(sizeof(int32_t) * (N > 0 ? N : 1));
    double* T = (double*)malloc(sizeof(double) * (M > 0 ? M : 1));
    double* P = (double*)malloc(sizeof(double) * (M > 0 ? M : 1));
    double* a = (double*)malloc(sizeof(double) * (M > 0 ? M : 1));
    double* inv = (double*)malloc(sizeof(double) * (M > 0 ? M : 1));
    uint32_t* n = (uint32_t*)malloc(sizeof(uint32_t) * (M > 0 ? M : 1));
    double* s_up = (double*)malloc(sizeof(double) * (M > 0 ? M : 1));
    double* tau = (double*)malloc(sizeof(double) * (M > 0 ? M : 1));
    for (int64_t r = jb->r_begin; r < jb->r_end; r++) {
        if (jb->method == 1) simulate_path_direct(jb, r, X, a, n);
        else if (jb->method == 3) simulate_path_direct_tree(jb, r, X, a, n);
        else if (jb->method == 2) simulate_path_lazy(jb, r, X, T, P, a, inv, n, s_up, tau);
        else simulate_path(jb, r, X, T, P, a, inv, n, tau);
    }
    free(X); free(T); free(P); free(a); free(inv); free(n); free(s_up); free(tau);
    return NULL;
}

/* Net change nu_k = products - reactants as a sparse list without zeros. */
static void build_nu(const rto_network* net, int32_t* ptr, int32_t* sp, int32_t* dl)
{
    int pos = 0;
    for (int k = 0; k < net->M; k++) {
        ptr[k] = pos;
        int start = pos;
        for (int pass = 0; pass < 2; pass++) {
            const int32_t* lp = pass == 0 ? net->react_ptr : net->prod_ptr;
            const int32_t* ls = pass == 0 ? net->react_species : net->prod_species;
            const int32_t* lm = pass == 0 ? net->react_sigma : net->prod_mult;
            for (int e = lp[k]; e < lp[k + 1]; e++) {
                int32_t d = pass == 0 ? -lm[e] : lm[e];
                int found = 0;
                for (int q = start; q < pos; q++)
                    if (sp[q] == ls[e]) { dl[q] += d; found = 1; }
                if (!found) { sp[pos] = ls[e]; dl[pos] = d; pos++; }
            }
        }
        int w = start;
        for (int q = start; q < pos; q++)
            if (dl[q] != 0) { sp[w] = sp[q]; dl[w] = dl[q]; w++; }
        pos = w;
    }
    ptr[net->M] = pos;
}

/* D(mu) for every mu as CSR lists: channel k is in D(mu) when one of its
 * reactant species has a nonzero net change in nu_mu; each k once, in
 * increasing order. */
static void build_deps(const rto_network* net, const int32_t* nu_ptr, const int32_t* nu_sp,
                       int32_t** dptr, int32_t** didx)
{
    const int M = net->M;
    int32_t* ptr = (int32_t*)malloc(sizeof(int32_t) * (M + 1));
    size_t cap = 16, len = 0;
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * cap);
    for (int mu = 0; mu < M; mu++) {
        ptr[mu] = (int32_t)len;
        for (int k = 0; k < M; k++) {
            int reads = 0;
            for (int e = net->react_ptr[k]; e < net->react_ptr[k + 1] && !reads; e++)
                for (int q = nu_ptr[mu]; q < nu_ptr[mu + 1]; q++)
                    if (nu_sp[q] == net->react_species[e]) reads = 1;
            if (!reads) continue;
            if (len == cap) { cap *= 2; idx = (int32_t*)realloc(idx, sizeof(int32_t) * cap); }
            idx[len++] = k;
        }
    }
    ptr[M] = (int32_t)len;
    *dptr = ptr;
    *didx = idx;
}

static int n_threads(int32_t req, int64_t R)
{
    long nt = req > 0 ? req : sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > R) nt = (long)(R > 0 ? R : 1);
    return (int)nt;
}

static int run_all(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                   double t_end, const double* sample_t, int32_t G,
                   uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                   uint64_t max_firings,
                   int32_t* samples, uint32_t* n_out, double* T_out, int32_t* x_final,
                   double* t_last, uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                   int32_t nthreads, rto_stats* stats, int32_t method, int32_t B,
                   const double* sched_t, const double* sched_c)
{
    if (!net || net->N < 0 || net->M < 0 || R < 0 || G < 0) return RTO_E_INVALID;
    if (R == 0) { if (stats) memset(stats, 0, sizeof(*stats)); return RTO_SUCCESS; }
    size_t nnz = (size_t)(net->react_ptr[net->M] + net->prod_ptr[net->M]);
    int32_t* nu_ptr = (int32_t*)malloc(sizeof(int32_t) * (net->M + 1));
    int32_t* nu_sp = (int32_t*)malloc(sizeof(int32_t) * (nnz + 1));
    int32_t* nu_dl = (int32_t*)malloc(sizeof(int32_t) * (nnz + 1));
    build_nu(net, nu_ptr, nu_sp, nu_dl);
    int32_t *dep_ptr = NULL, *dep_idx = NULL;
    if (method == 2) build_deps(net, nu_ptr, nu_sp, &dep_ptr, &dep_idx);

    int nt = n_threads(nthreads, R);
    job_t* jobs = (job_t*)calloc((size_t)nt, sizeof(job_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    for (int i = 0; i < nt; i++) {
        job_t* jb = &jobs[i];
        jb->net = net; jb->nu_ptr = nu_ptr; jb->nu_species = nu_sp; jb->nu_delta = nu_dl;
        jb->x0 = x0; jb->x0_per_traj = x0_per_traj; jb->t_end = t_end; jb->s = sample_t;
        jb->G = G; jb->seed = seed; jb->net_id = net_id; jb->traj_offset = traj_offset;
        jb->max_firings = max_firings; jb->samples = samples; jb->x_final = x_final;
        jb->n_out = n_out; jb->tie_step = tie_step; jb->T_out = T_out; jb->t_last = t_last;
        jb->status = status; jb->seq_hash = seq_hash;
        jb->r_begin = R * i / nt; jb->r_end = R * (i + 1) / nt;
        jb->method = method;
        jb->dep_ptr = dep_ptr; jb->dep_idx = dep_idx;
        jb->B = B; jb->sched_t = sched_t; jb->sched_c = sched_c;
        pthread_create(&th[i], NULL, run_job, jb);
    }
    rto_stats tot;
    memset(&tot, 0, sizeof(tot));
    for (int i = 0; i < nt; i++) {
        pthread_join(th[i], NULL);
        tot.firings += jobs[i].stats.firings;
        tot.near_ties += jobs[i].stats.near_ties;
        tot.clamps += jobs[i].stats.clamps;
        tot.hard_cases += jobs[i].stats.hard_cases;
        for (int q = 0; q < 4; q++) tot.status_count[q] += jobs[i].stats.status_count[q];
    }
    if (stats) *stats = tot;
    free(jobs); free(th); free(nu_ptr); free(nu_sp); free(nu_dl); free(dep_ptr); free(dep_idx);
    return tot.hard_cases ? RTO_E_HARDCASE : RTO_SUCCESS;
}

int rto_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                 double t_end, const double* sample_t, int32_t G,
                 uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                 uint64_t max_firings,
                 int32_t* samples, uint32_t* n_out, double* T_out, int32_t* x_final,
                 double* t_last, uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                 int32_t nthreads, rto_stats* stats)
{
    return run_all(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                   max_firings, samples, n_out, T_out, x_final, t_last, status, seq_hash,
                   tie_step, nthreads, stats, 0, 0, NULL, NULL);
}

int rto_simulate_schedule(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                          double t_end, const double* sample_t, int32_t G,
                          uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                          uint64_t max_firings,
                          int32_t* samples, uint32_t* n_out, double* T_out, int32_t* x_final,
                          double* t_last, uint8_t* status, uint64_t* seq_hash,
                          uint32_t* tie_step, int32_t nthreads, rto_stats* stats,
                          int32_t B, const double* sched_t, const double* sched_c)
{
    if (B < 0 || (B > 0 && (!sched_t || !sched_c))) return RTO_E_INVALID;
    for (int32_t i = 0; i < B; i++)
        if (!(sched_t[i] > (i ? sched_t[i - 1] : 0.0)) || !isfinite(sched_t[i]))
            return RTO_E_INVALID;
    return run_all(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                   max_firings, samples, n_out, T_out, x_final, t_last, status, seq_hash,
                   tie_step, nthreads, stats, 0, B, sched_t, sched_c);
}

int rto_lazy_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                      double t_end, const double* sample_t, int32_t G,
                      uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                      uint64_t max_firings,
                      int32_t* samples, uint32_t* n_out, double* T_out, int32_t* x_final,
                      double* t_last, uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                      int32_t nthreads, rto_stats* stats)
{
    return run_all(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                   max_firings, samples, n_out, T_out, x_final, t_last, status, seq_hash,
                   tie_step, nthreads, stats, 2, 0, NULL, NULL);
}

int rto_lazy_simulate_schedule(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                               double t_end, const double* sample_t, int32_t G,
                               uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                               uint64_t max_firings,
                               int32_t* samples, uint32_t* n_out, double* T_out,
                               int32_t* x_final, double* t_last, uint8_t* status,
                               uint64_t* seq_hash, uint32_t* tie_step, int32_t nthreads,
                               rto_stats* stats, int32_t B, const double* sched_t,
                               const double* sched_c)
{
    if (B < 0 || (B > 0 && (!sched_t || !sched_c))) return RTO_E_INVALID;
    for (int32_t i = 0; i < B; i++)
        if (!(sched_t[i] > (i ? sched_t[i - 1] : 0.0)) || !isfinite(sched_t[i]))
            return RTO_E_INVALID;
    return run_all(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                   max_firings, samples, n_out, T_out, x_final, t_last, status, seq_hash,
                   tie_step, nthreads, stats, 2, B, sched_t, sched_c);
}

int rto_direct_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                        double t_end, const double* sample_t, int32_t G,
                        uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                        uint64_t max_firings,
                        int32_t* samples, uint32_t* n_out, int32_t* x_final,
                        double* t_last, uint8_t* status, uint64_t* seq_hash,
                        int32_t nthreads, rto_stats* stats)
{
    return run_all(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                   max_firings, samples, n_out, NULL, x_final, t_last, status, seq_hash,
                   NULL, nthreads, stats, 1, 0, NULL, NULL);
}

int rto_direct_tree_simulate(const rto_network* net, const int32_t* x0, int32_t x0_per_traj,
                             double t_end, const double* sample_t, int32_t G,
                             uint64_t seed, uint32_t net_id, uint64_t traj_offset, int64_t R,
                             uint64_t max_firings,
                             int32_t* samples, uint32_t* n_out, int32_t* x_final,
                             double* t_last, uint8_t* status, uint64_t* seq_hash,
                             int32_t nthreads, rto_stats* stats)
{
    return run_all(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                   max_firings, samples, n_out, NULL, x_final, t_last, status, seq_hash,
                   NULL, nthreads, stats, 3, 0, NULL, NULL);
}
