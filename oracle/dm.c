/*
 * dm.c -- Gillespie's direct method (the comparison method of paper section 3,
 * Eq. 17-22: exponential waiting time with rate sum_k a_k, then the firing
 * channel chosen with probability a_k / sum a).
 *
 * TEST INFRASTRUCTURE ONLY.  It samples the same Markov jump law as the
 * random-time algorithm with an unrelated random stream (SplitMix64, Steele,
 * Lea & Flood 2014), so two-sample tests between it and the random-time
 * oracle check the law, not the arithmetic.  Plain double arithmetic; no
 * attempt at bit reproducibility against anything else.
 */
#include "rto.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static uint64_t splitmix64_next(uint64_t* s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform on (0, 1] */
static double unif_open0(uint64_t* s) { return ((splitmix64_next(s) >> 11) + 1) * 0x1p-53; }
/* uniform on [0, 1) */
static double unif_open1(uint64_t* s) { return (splitmix64_next(s) >> 11) * 0x1p-53; }

static double prop(const rto_network* net, const int32_t* X, int k)
{
    double h = 1.0;
    for (int e = net->react_ptr[k]; e < net->react_ptr[k + 1]; e++) {
        double x = (double)X[net->react_species[e]];
        if (net->react_sigma[e] == 1) h *= x;
        else h *= x * (x - 1.0) / 2.0;
    }
    return net->c[k] * h;
}

typedef struct {
    const rto_network* net;
    const int32_t* x0;
    double t_end;
    const double* s;
    int32_t G;
    uint64_t seed;
    uint64_t max_firings;
    int32_t* samples;
    uint32_t* n_out;
    int64_t r0, r1;
} dm_job;

static void* dm_run(void* arg)
{
    dm_job* jb = (dm_job*)arg;
    const rto_network* net = jb->net;
    int N = net->N, M = net->M;
    int32_t* X = (int32_t*)malloc(sizeof(int32_t) * (N + 1));
    double* a = (double*)malloc(sizeof(double) * (M + 1));
    for (int64_t r = jb->r0; r < jb->r1; r++) {
        uint64_t st = jb->seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(r + 1));
        splitmix64_next(&st);
        memcpy(X, jb->x0, sizeof(int32_t) * N);
        uint32_t* n = jb->n_out + (size_t)r * M;
        for (int k = 0; k < M; k++) n[k] = 0;
        double t = 0.0;
        int32_t g = 0;
        uint64_t fired = 0;
        for (;;) {
            double a0 = 0.0;
            for (int k = 0; k < M; k++) { a[k] = prop(net, X, k); a0 += a[k]; }
            if (a0 <= 0.0) break;
            double t_new = t + (-log(unif_open0(&st))) / a0;
            if (t_new > jb->t_end) break;
            while (g < jb->G && jb->s[g] < t_new) {
                memcpy(jb->samples + ((size_t)r * jb->G + g) * N, X, sizeof(int32_t) * N);
                g++;
            }
            double target = unif_open1(&st) * a0, acc = 0.0;
            int mu = -1;
            for (int k = 0; k < M; k++) {
                acc += a[k];
                if (a[k] > 0.0) mu = k;
                if (acc > target && a[k] > 0.0) break;
            }
            for (int e = net->react_ptr[mu]; e < net->react_ptr[mu + 1]; e++)
                X[net->react_species[e]] -= net->react_sigma[e];
            for (int e = net->prod_ptr[mu]; e < net->prod_ptr[mu + 1]; e++)
                X[net->prod_species[e]] += net->prod_mult[e];
            n[mu]++;
            t = t_new;
            if (++fired >= jb->max_firings) break;
        }
        while (g < jb->G) {
            memcpy(jb->samples + ((size_t)r * jb->G + g) * N, X, sizeof(int32_t) * N);
            g++;
        }
    }
    free(X);
    free(a);
    return NULL;
}

int rto_dm_simulate(const rto_network* net, const int32_t* x0, double t_end,
                    const double* sample_t, int32_t G, uint64_t seed, int64_t R,
                    uint64_t max_firings, int32_t* samples, uint32_t* n_out,
                    int32_t nthreads)
{
    if (!net || R < 0) return RTO_E_INVALID;
    if (R == 0) return RTO_SUCCESS;
    long nt = nthreads > 0 ? nthreads : sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > R) nt = (long)R;
    dm_job* jobs = (dm_job*)calloc((size_t)nt, sizeof(dm_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    for (long i = 0; i < nt; i++) {
        dm_job* jb = &jobs[i];
        jb->net = net; jb->x0 = x0; jb->t_end = t_end; jb->s = sample_t; jb->G = G;
        jb->seed = seed; jb->max_firings = max_firings; jb->samples = samples;
        jb->n_out = n_out; jb->r0 = R * i / nt; jb->r1 = R * (i + 1) / nt;
        pthread_create(&th[i], NULL, dm_run, jb);
    }
    for (long i = 0; i < nt; i++) pthread_join(th[i], NULL);
    free(jobs);
    free(th);
    return RTO_SUCCESS;
}
