// network.cpp -- host-side network compiler: validation and device tables.
//
// The paper stores the reactant, stoichiometric and update matrices as sparse
// COO lists and limits reactions to two reactant molecules so the tables fit
// on-chip (section 5).  Here a reaction becomes one 8-byte reactant record
// (kind, s0, s1), the net change v_k a short (species, delta) list, and the
// dependency graph D(mu) -- the channels whose propensity reads a species
// that mu changes (Gibson & Bruck, cited in section 5) -- a CSR list.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <set>

#include "internal.h"

static int validate_rate(double c, int k)
{
    if (!(c >= 0.0) || !isfinite(c) || (c != 0.0 && (c < 1e-280 || c > 1e280)))
        return rt_fail(RTSSA_E_INVALID, "rate c[" + std::to_string(k) +
                       "] must be 0 or within [1e-280, 1e280]");
    return RTSSA_OK;
}

static int upload(rtssa_network* n)
{
    // one device allocation; each table 256-byte aligned
    struct part { const void* src; size_t bytes; size_t off; };
    std::vector<part> parts = {
        {n->react.data(), n->react.size() * sizeof(int2), 0},
        {n->c.data(), n->c.size() * sizeof(double), 0},
        {n->nu_ptr.data(), n->nu_ptr.size() * sizeof(int32_t), 0},
        {n->nu_sp.data(), n->nu_sp.size() * sizeof(int32_t), 0},
        {n->nu_dl.data(), n->nu_dl.size() * sizeof(int32_t), 0},
        {n->dep_ptr.data(), n->dep_ptr.size() * sizeof(int32_t), 0},
        {n->dep_idx.data(), n->dep_idx.size() * sizeof(int32_t), 0},
        {n->nu_dense.data(), n->nu_dense.size() * sizeof(int32_t), 0},
    };
    size_t off = 0;
    for (auto& p : parts) {
        p.off = off;
        off += (p.bytes + 255) / 256 * 256 + 256;
    }
    if (hipGetDevice(&n->device) != hipSuccess) return rt_fail(RTSSA_E_HIP, "hipGetDevice failed");
    if (hipMalloc(&n->dev_block, off) != hipSuccess) {
        n->dev_block = nullptr;
        return rt_fail(RTSSA_E_NOMEM, "device allocation of network tables failed");
    }
    char* base = (char*)n->dev_block;
    for (auto& p : parts)
        if (p.bytes && hipMemcpy(base + p.off, p.src, p.bytes, hipMemcpyHostToDevice) != hipSuccess)
            return rt_fail(RTSSA_E_HIP, "copy of network tables failed");
    n->dev.N = n->N;
    n->dev.M = n->M;
    n->dev.react = (const int2*)(base + parts[0].off);
    n->dev.c = (const double*)(base + parts[1].off);
    n->dev.nu_ptr = (const int32_t*)(base + parts[2].off);
    n->dev.nu_sp = (const int32_t*)(base + parts[3].off);
    n->dev.nu_dl = (const int32_t*)(base + parts[4].off);
    n->dev.dep_ptr = (const int32_t*)(base + parts[5].off);
    n->dev.dep_idx = (const int32_t*)(base + parts[6].off);
    n->dev.nu_dense = n->nu_dense.empty() ? nullptr : (const int32_t*)(base + parts[7].off);
    return RTSSA_OK;
}

extern "C" int rtssa_network_create(int32_t N, int32_t M, const int32_t* react_ptr,
                                    const int32_t* react_species, const int32_t* react_sigma,
                                    const int32_t* prod_ptr, const int32_t* prod_species,
                                    const int32_t* prod_mult, const double* c,
                                    rtssa_network** out)
{
    if (!out) return rt_fail(RTSSA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (N < 0 || M < 0 || N > RT_SPECIES_MASK)
        return rt_fail(RTSSA_E_INVALID, "N and M must be >= 0 and N < 2^29");
    if (!react_ptr || !prod_ptr || (M > 0 && !c))
        return rt_fail(RTSSA_E_INVALID, "react_ptr, prod_ptr and c must not be NULL");
    if (react_ptr[0] != 0 || prod_ptr[0] != 0)
        return rt_fail(RTSSA_E_INVALID, "react_ptr[0] and prod_ptr[0] must be 0");
    for (int k = 0; k < M; ++k)
        if (react_ptr[k + 1] < react_ptr[k] || prod_ptr[k + 1] < prod_ptr[k])
            return rt_fail(RTSSA_E_INVALID, "offsets must be non-decreasing");
    if ((react_ptr[M] > 0 && (!react_species || !react_sigma)) ||
        (prod_ptr[M] > 0 && (!prod_species || !prod_mult)))
        return rt_fail(RTSSA_E_INVALID, "species/coefficient arrays must not be NULL");

    rtssa_network* n = new rtssa_network();
    n->N = N;
    n->M = M;
    n->react.resize(std::max(M, 1));
    n->c.assign(std::max(M, 1), 0.0);
    n->nu_ptr.assign(M + 1, 0);
    std::vector<std::vector<int>> readers(N);   // species -> channels reading it
    std::vector<std::vector<std::pair<int, int>>> nu(M);
    for (int k = 0; k < M; ++k) {
        int rc = validate_rate(c[k], k);
        if (rc) { delete n; return rc; }
        n->c[k] = c[k];
        int order = 0, sp[2] = {-1, -1}, sg[2] = {0, 0}, cnt = 0;
        std::map<int, int> delta;
        for (int e = react_ptr[k]; e < react_ptr[k + 1]; ++e) {
            int j = react_species[e], s = react_sigma[e];
            if (j < 0 || j >= N || s < 1) {
                delete n;
                return rt_fail(RTSSA_E_INVALID, "reaction " + std::to_string(k) +
                               ": bad reactant species or coefficient");
            }
            for (int q = 0; q < cnt; ++q)
                if (sp[q] == j) {
                    delete n;
                    return rt_fail(RTSSA_E_INVALID, "reaction " + std::to_string(k) +
                                   ": repeated reactant species (give one entry with its coefficient)");
                }
            order += s;
            if (order > 2) {
                delete n;
                return rt_fail(RTSSA_E_UNSUPPORTED, "reaction " + std::to_string(k) +
                               ": more than two reactant molecules");
            }
            sp[cnt] = j;
            sg[cnt] = s;
            cnt++;
            delta[j] -= s;
        }
        int kind = RT_H_ZERO, s0 = 0, s1 = 0;
        if (cnt == 1 && sg[0] == 1) { kind = RT_H_ONE; s0 = sp[0]; }
        else if (cnt == 1 && sg[0] == 2) { kind = RT_H_PAIR; s0 = sp[0]; }
        else if (cnt == 2) { kind = RT_H_TWO; s0 = sp[0]; s1 = sp[1]; }
        n->react[k] = make_int2(s0 | (kind << 29), s1);
        for (int q = 0; q < cnt; ++q) readers[sp[q]].push_back(k);
        for (int e = prod_ptr[k]; e < prod_ptr[k + 1]; ++e) {
            int j = prod_species[e], m = prod_mult[e];
            if (j < 0 || j >= N || m < 1 || m > (1 << 20)) {
                delete n;
                return rt_fail(RTSSA_E_INVALID, "reaction " + std::to_string(k) +
                               ": bad product species or multiplicity");
            }
            delta[j] += m;
        }
        for (auto& kv : delta)
            if (kv.second != 0) nu[k].push_back(kv);
    }
    if (M == 0) n->react[0] = make_int2(0, 0);
    // net change lists
    for (int k = 0; k < M; ++k) {
        n->nu_ptr[k] = (int)n->nu_sp.size();
        for (auto& kv : nu[k]) { n->nu_sp.push_back(kv.first); n->nu_dl.push_back(kv.second); }
        n->max_nu = std::max<int32_t>(n->max_nu, (int32_t)nu[k].size());
    }
    n->nu_ptr[M] = (int)n->nu_sp.size();
    // one padding entry: kernels may load entry nu_ptr[k] (clamped) for a
    // reaction with an empty list, including the last one
    n->nu_sp.push_back(0);
    n->nu_dl.push_back(0);
    // dependency graph
    n->dep_ptr.assign(M + 1, 0);
    for (int k = 0; k < M; ++k) {
        std::set<int> d;
        for (auto& kv : nu[k])
            for (int r : readers[kv.first]) d.insert(r);
        n->dep_ptr[k] = (int)n->dep_idx.size();
        for (int r : d) n->dep_idx.push_back(r);
        n->max_dep = std::max<int32_t>(n->max_dep, (int32_t)d.size());
    }
    n->dep_ptr[M] = (int)n->dep_idx.size();
    n->dep_idx.push_back(0);                 // padding entry, as for nu_sp
    // dense net change for small networks
    if (M <= RT_THREAD_MAX_M && N <= RT_THREAD_MAX_N && M > 0 && N > 0) {
        n->nu_dense.assign((size_t)M * N, 0);
        for (int k = 0; k < M; ++k)
            for (auto& kv : nu[k]) n->nu_dense[(size_t)k * N + kv.first] = kv.second;
    }
    int rc = upload(n);
    if (rc) { rtssa_network_destroy(n); return rc; }
    *out = n;
    return RTSSA_OK;
}

extern "C" int rtssa_network_destroy(rtssa_network* net)
{
    if (!net) return RTSSA_OK;
    if (net->dev_block || net->sched_block || net->lazy_block || net->group_block) {
        int cur = -1;
        hipGetDevice(&cur);
        if (net->device >= 0 && cur != net->device) hipSetDevice(net->device);
        if (net->dev_block) hipFree(net->dev_block);
        if (net->sched_block) hipFree(net->sched_block);
        if (net->lazy_block) hipFree(net->lazy_block);
        if (net->group_block) hipFree(net->group_block);
        if (cur >= 0 && cur != net->device) hipSetDevice(cur);
    }
    delete net;
    return RTSSA_OK;
}

int rt_lazy_prepare(rtssa_network* net)
{
    if (net->lazy_block) return RTSSA_OK;
    const int M = net->M;
    int S = 1;
    while (S < net->max_nu) S <<= 1;
    if (S > 64) return rt_fail(RTSSA_E_UNSUPPORTED, "a reaction changes more than 64 species");
    const size_t rows = (size_t)std::max(M, 1);
    std::vector<int32_t> touch(rows * 64, -1), more(rows, 0);
    std::vector<int2> nu(rows * S, make_int2(-1, 0));
    for (int mu = 0; mu < M; ++mu) {
        int n_other = 0;
        more[mu] = net->dep_ptr[mu + 1];
        for (int q = net->dep_ptr[mu]; q < net->dep_ptr[mu + 1]; ++q) {
            const int k = net->dep_idx[q];
            if (k == mu) continue;
            if (n_other < 63) touch[(size_t)mu * 64 + 1 + n_other] = k;
            else if (n_other == 63) more[mu] = q;
            ++n_other;
        }
        touch[(size_t)mu * 64] = n_other;
        for (int e = net->nu_ptr[mu]; e < net->nu_ptr[mu + 1]; ++e)
            nu[(size_t)mu * S + (e - net->nu_ptr[mu])] = make_int2(net->nu_sp[e], net->nu_dl[e]);
    }
    const size_t tb = touch.size() * 4, mb = (more.size() * 4 + 255) / 256 * 256;
    const size_t nb = nu.size() * sizeof(int2);
    const size_t moff = (tb + 255) / 256 * 256, noff = moff + mb;
    struct device_guard {
        int prev = -1;
        explicit device_guard(int d)
        {
            if (d >= 0 && hipGetDevice(&prev) == hipSuccess && prev != d) hipSetDevice(d);
            else prev = -1;
        }
        ~device_guard() { if (prev >= 0) hipSetDevice(prev); }
    } guard(net->device);
    void* blk = nullptr;
    if (hipMalloc(&blk, noff + nb) != hipSuccess)
        return rt_fail(RTSSA_E_NOMEM, "device allocation of the lazy form's rows failed");
    if (hipMemcpy(blk, touch.data(), tb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((char*)blk + moff, more.data(), more.size() * 4, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy((char*)blk + noff, nu.data(), nb, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(blk);
        return rt_fail(RTSSA_E_HIP, "copy of the lazy form's rows failed");
    }
    net->lazy_block = blk;
    net->dev.touch = (const int32_t*)blk;
    net->dev.touch_more = (const int32_t*)((char*)blk + moff);
    net->dev.nu_fixed = (const int2*)((char*)blk + noff);
    net->dev.nu_stride = S;
    return RTSSA_OK;
}

// The rates of the dependency records, in record order (c of the record's
// channel, 0 past a row's end).
static void group_record_rates(const rtssa_network* net, std::vector<double>& rc_c)
{
    const int M = net->M;
    rc_c.assign((size_t)std::max(M, 1) * 64, 0.0);
    for (int mu = 0; mu < M; ++mu) {
        double* rowc = rc_c.data() + (size_t)mu * 64;
        rowc[0] = net->c[mu];
        int n_other = 0;
        for (int q = net->dep_ptr[mu]; q < net->dep_ptr[mu + 1]; ++q) {
            const int k = net->dep_idx[q];
            if (k == mu) continue;
            if (n_other < 63) rowc[1 + n_other] = net->c[k];
            ++n_other;
        }
    }
}

int rt_group_rows_prepare(rtssa_network* net)
{
    int rc = rt_lazy_prepare(net);
    if (rc || net->group_block) return rc;
    const int M = net->M;
    const size_t rows = (size_t)std::max(M, 1);
    std::vector<int4> rec(rows * 64, make_int4(-1, 0, 0, 0));
    std::vector<int2> del(rows * 64, make_int2(0, 0));
    std::vector<double> rc_c;
    group_record_rates(net, rc_c);
    for (int mu = 0; mu < M; ++mu) {
        int4* row = rec.data() + (size_t)mu * 64;
        int2* drow = del.data() + (size_t)mu * 64;
        // the change of species j under v_mu (each species once in the list)
        auto change = [&](int j) {
            for (int e = net->nu_ptr[mu]; e < net->nu_ptr[mu + 1]; ++e)
                if (net->nu_sp[e] == j) return net->nu_dl[e];
            return 0;
        };
        auto deltas = [&](int k) {
            const int kind = (int)((uint32_t)net->react[k].x >> 29);
            const int s0 = net->react[k].x & RT_SPECIES_MASK, s1 = net->react[k].y;
            return make_int2(kind != RT_H_ZERO ? change(s0) : 0, kind == RT_H_TWO ? change(s1) : 0);
        };
        row[0] = make_int4(mu, net->react[mu].x, net->react[mu].y, 0);
        drow[0] = deltas(mu);
        int n_other = 0, more = net->dep_ptr[mu + 1];
        for (int q = net->dep_ptr[mu]; q < net->dep_ptr[mu + 1]; ++q) {
            const int k = net->dep_idx[q];
            if (k == mu) continue;
            if (n_other < 63) {
                row[1 + n_other] = make_int4(k, net->react[k].x, net->react[k].y, 0);
                drow[1 + n_other] = deltas(k);
            } else if (n_other == 63) {
                more = q;
            }
            ++n_other;
        }
        row[0].w = n_other;
        row[1].w = more;
    }
    const size_t rb = rec.size() * sizeof(int4), cb = rc_c.size() * sizeof(double);
    const size_t db = del.size() * sizeof(int2);
    const size_t coff = (rb + 255) / 256 * 256, doff = coff + (cb + 255) / 256 * 256;
    struct device_guard {
        int prev = -1;
        explicit device_guard(int d)
        {
            if (d >= 0 && hipGetDevice(&prev) == hipSuccess && prev != d) hipSetDevice(d);
            else prev = -1;
        }
        ~device_guard() { if (prev >= 0) hipSetDevice(prev); }
    } guard(net->device);
    void* blk = nullptr;
    if (hipMalloc(&blk, doff + db) != hipSuccess)
        return rt_fail(RTSSA_E_NOMEM, "device allocation of the dependency records failed");
    if (hipMemcpy(blk, rec.data(), rb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((char*)blk + coff, rc_c.data(), cb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((char*)blk + doff, del.data(), db, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(blk);
        return rt_fail(RTSSA_E_HIP, "copy of the dependency records failed");
    }
    net->group_block = blk;
    net->dev.grow = (const int4*)blk;
    net->dev.growc = (const double*)((char*)blk + coff);
    net->dev.gdel = (const int2*)((char*)blk + doff);
    return RTSSA_OK;
}

extern "C" int rtssa_network_set_rates(rtssa_network* net, const double* c)
{
    if (!net || (!c && net->M > 0)) return rt_fail(RTSSA_E_INVALID, "NULL argument");
    for (int k = 0; k < net->M; ++k) {
        int rc = validate_rate(c[k], k);
        if (rc) return rc;
    }
    for (int k = 0; k < net->M; ++k) net->c[k] = c[k];
    if (net->M > 0 &&
        hipMemcpy((void*)net->dev.c, net->c.data(), sizeof(double) * net->M,
                  hipMemcpyHostToDevice) != hipSuccess)
        return rt_fail(RTSSA_E_HIP, "copy of rates failed");
    if (net->group_block) {
        // the dependency records carry each channel's rate: rewrite those in
        // place (their address may be held by a batch)
        std::vector<double> rc_c;
        group_record_rates(net, rc_c);
        if (hipMemcpy((void*)net->dev.growc, rc_c.data(), rc_c.size() * sizeof(double),
                      hipMemcpyHostToDevice) != hipSuccess)
            return rt_fail(RTSSA_E_HIP, "copy of rates failed");
    }
    return RTSSA_OK;
}

extern "C" int rtssa_network_info(const rtssa_network* net, int32_t* N, int32_t* M,
                                  int64_t* dep_edges, int32_t* auto_mapping)
{
    if (!net) return rt_fail(RTSSA_E_INVALID, "net is NULL");
    if (N) *N = net->N;
    if (M) *M = net->M;
    if (dep_edges) *dep_edges = net->dep_ptr.empty() ? 0 : net->dep_ptr[net->M];
    if (auto_mapping) *auto_mapping = rt_auto_mapping(net);
    return RTSSA_OK;
}

extern "C" int rtssa_network_set_schedule(rtssa_network* net, int32_t B, const double* times,
                                          const double* rates)
{
    if (!net) return rt_fail(RTSSA_E_INVALID, "net is NULL");
    if (net->batch_refs > 0)
        return rt_fail(RTSSA_E_INVALID, "the network is part of a batch; destroy the batch first");
    if (B < 0 || (B > 0 && (!times || (!rates && net->M > 0))))
        return rt_fail(RTSSA_E_INVALID, "bad schedule arguments");
    for (int32_t i = 0; i < B; ++i)
        if (!isfinite(times[i]) || !(times[i] > (i ? times[i - 1] : 0.0)))
            return rt_fail(RTSSA_E_INVALID, "breakpoint times must be finite, > 0 and increasing");
    for (int64_t q = 0; q < (int64_t)B * net->M; ++q) {
        int rc = validate_rate(rates[q], (int)(q % std::max(1, net->M)));
        if (rc) return rc;
    }
    // the schedule lives on the network's device
    struct device_guard {
        int prev = -1;
        explicit device_guard(int d)
        {
            if (d >= 0 && hipGetDevice(&prev) == hipSuccess && prev != d) hipSetDevice(d);
            else prev = -1;
        }
        ~device_guard() { if (prev >= 0) hipSetDevice(prev); }
    } guard(net->device);
    void* blk = nullptr;
    if (B > 0) {
        const size_t tb = (size_t)B * sizeof(double), cb = (size_t)B * net->M * sizeof(double);
        const size_t toff = 0, coff = (tb + 255) / 256 * 256;
        if (hipMalloc(&blk, coff + cb + 256) != hipSuccess)
            return rt_fail(RTSSA_E_NOMEM, "device allocation of the schedule failed");
        if (hipMemcpy((char*)blk + toff, times, tb, hipMemcpyHostToDevice) != hipSuccess ||
            (cb && hipMemcpy((char*)blk + coff, rates, cb, hipMemcpyHostToDevice) != hipSuccess)) {
            hipFree(blk);
            return rt_fail(RTSSA_E_HIP, "copy of the schedule failed");
        }
        net->dev.sched_t = (const double*)((char*)blk + toff);
        net->dev.sched_c = (const double*)((char*)blk + coff);
    } else {
        net->dev.sched_t = nullptr;
        net->dev.sched_c = nullptr;
    }
    if (net->sched_block) hipFree(net->sched_block);
    net->sched_block = blk;
    net->dev.sched_B = B;
    return RTSSA_OK;
}
