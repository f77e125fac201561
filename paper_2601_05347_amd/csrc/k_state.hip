// Device-side state of an index (DevTree): set-up, the plan checks and the
// commits that end a build or a batch update, and the node layout.
//
// Updates never hand a count back to the host: the plan kernels leave the
// sizes of the new directory in a counter array, a one-thread check decides
// whether the update can be applied within the buffers the host reserved,
// and a one-thread commit writes the new leaf count, directory buffer, slot
// bookkeeping and node layout. Every later launch (node levels, queries, the
// next update) reads them from here, so a whole sequence of builds, updates
// and queries can be queued, or captured into a graph, without waiting.
#include "psi_kern.h"
#include "psi_update.h"

namespace psi {

namespace {

// Node layout of a B-ary tree over L leaves, root first: level l of h holds
// ceil(L / B^(h-l)) nodes, levels 0 .. h-1 stored one after the other.
__device__ void set_layout(DevTree* d, uint64_t L, uint32_t B) {
    d->L = L;
    if (L == 0) {
        d->h = 0;
        d->n_inner = 0;
        d->lv[0].off = 0;
        d->lv[0].n = 0;
        d->lv[0].span = 1;
        return;
    }
    uint32_t h = 0;
    for (uint64_t n = L; n > 1 && h + 1 < (uint32_t)MAX_LEVELS; ++h) n = (n + B - 1) / B;
    // level h - u holds ceil(L / B^u) nodes
    uint64_t n = L, off_end = 0;
    for (uint32_t u = 0; u <= h; ++u) {
        d->lv[h - u].n = n;
        if (u > 0) off_end += n;
        n = (n + B - 1) / B;
    }
    uint64_t off = 0, span = 1;
    for (uint32_t l = 0; l <= h; ++l) {
        d->lv[l].off = l < h ? off : 0;
        if (l < h) off += d->lv[l].n;
    }
    for (int l = (int)h; l >= 0; --l) {
        d->lv[l].span = span;
        span *= B;
    }
    d->h = h;
    d->n_inner = off_end;
}

__global__ void k_set_dirs(DevTree* dt, NodeRec* l0, NodeRec* l1, uint64_t* k0, uint64_t* k1, uint32_t* i0,
                           uint32_t* i1) {
    if (threadIdx.x | blockIdx.x) return;
    dt->leaf[0] = l0;
    dt->leaf[1] = l1;
    dt->pkey[0] = k0;
    dt->pkey[1] = k1;
    dt->pid[0] = i0;
    dt->pid[1] = i1;
}

__global__ void k_reset(DevTree* dt, uint32_t B) {
    if (threadIdx.x | blockIdx.x) return;
    dt->cur = 0;
    dt->n_live = 0;
    dt->slot_top = 0;
    dt->n_free = 0;
    dt->next_id = 0;
    dt->sort_top = ~0u;
    set_layout(dt, 0, B);
}

__global__ void k_commit_build(DevTree* dt, uint64_t n, uint64_t L, uint32_t cur, uint32_t next_id, uint32_t B) {
    if (threadIdx.x | blockIdx.x) return;
    dt->cur = cur;
    dt->n_live = n;
    dt->slot_top = L;
    dt->n_free = 0;
    dt->next_id = next_id;
    set_layout(dt, L, B);
}

// Ids of an inserted batch: the batch's keys go to the id table at the next
// free ids, the sorted pairs' ids (positions in the batch) become those ids,
// and new_ids (may be null) receives them in input order. A batch with a
// coordinate out of range, or past the id table's capacity, is rejected
// whole: its new ids read PAD_ID and nothing is written.
__global__ void k_ins_ids(const DevTree* __restrict__ dt, const uint64_t* __restrict__ keys, uint64_t m,
                          uint64_t* __restrict__ idkey, uint64_t id_cap, uint32_t* __restrict__ bi,
                          uint32_t* __restrict__ new_ids, const uint32_t* __restrict__ ctr) {
    const uint32_t base = dt->next_id;
    const bool bad = ctr[9] != 0 || (uint64_t)base + m > id_cap;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        if (bad) {
            if (new_ids) new_ids[e] = PAD_ID;
            continue;
        }
        idkey[base + e] = keys[e];
        bi[e] += base;
        if (new_ids) new_ids[e] = base + (uint32_t)e;
    }
}

// After an insert's plan (runs, pieces, slots to allocate A = ctr[3], slots
// freed F = ctr[5]): decides the outcome ctr[10] -- 0 apply, 1 reject (a
// coordinate out of range, or the new directory, slots or free stack would
// not fit the capacities in cap), 2 the index is empty and the batch becomes
// a fresh tree of ceil(m / phi) leaves. A rejected or fresh-build outcome
// zeroes the run and allocation counts, which turns the leaf-wise kernels that
// follow into no-ops; the 64-bit word at ctr + 12 is zero only for a fresh
// build.
__global__ void k_ins_check(const DevTree* __restrict__ dt, uint32_t* __restrict__ ctr, uint64_t m, uint32_t phi,
                            uint64_t id_cap, Caps cap) {
    if (threadIdx.x | blockIdx.x) return;
    const uint64_t L = dt->L;
    uint32_t outcome = 0;
    if (ctr[9] != 0) {
        outcome = 1;
        atomicOr(cap.err, ERR_RANGE);
    } else if ((uint64_t)dt->next_id + m > id_cap) {
        outcome = 1;
        atomicOr(cap.err, ERR_CAPACITY);
    } else if (L > cap.lgrid) {
        outcome = 1;
        atomicOr(cap.err, ERR_CAPACITY);
    } else if (L == 0) {
        const uint64_t Lb = (m + phi - 1) / phi;
        if (Lb > cap.leaves || Lb > cap.slots) {
            outcome = 1;
            atomicOr(cap.err, ERR_CAPACITY);
        } else {
            outcome = 2;
        }
    } else {
        const uint64_t A = ctr[3], F = ctr[5], nf = dt->n_free;
        const uint64_t take = A < nf ? A : nf;
        const uint64_t Lnew = L - F + A, top = dt->slot_top + (A - take), nf2 = nf - take + F;
        if (F > L || Lnew > cap.leaves || top > cap.slots || nf2 > cap.frees || A > cap.alloc) {
            outcome = 1;
            atomicOr(cap.err, ERR_CAPACITY);
        }
    }
    ctr[10] = outcome;
    *reinterpret_cast<uint64_t*>(ctr + 12) = outcome == 2 ? 0ull : 1ull;
    if (outcome != 0) {
        ctr[1] = 0;
        ctr[3] = 0;
        ctr[4] = 0;
        ctr[5] = 0;
    }
}

__global__ void k_ins_commit(DevTree* dt, const uint32_t* __restrict__ ctr, uint64_t m, uint32_t phi, uint32_t B) {
    if (threadIdx.x | blockIdx.x) return;
    const uint32_t outcome = ctr[10];
    if (outcome == 1) return;
    if (outcome == 2) {
        const uint64_t Lb = (m + phi - 1) / phi;
        dt->cur = 0;
        dt->slot_top = Lb;
        dt->n_free = 0;
        dt->n_live = m;
        dt->next_id += (uint32_t)m;
        set_layout(dt, Lb, B);
        return;
    }
    const uint64_t A = ctr[3], F = ctr[5], nf = dt->n_free;
    const uint64_t take = A < nf ? A : nf;
    dt->slot_top += A - take;
    dt->n_free = nf - take + F;
    if (A > 0) dt->cur ^= 1u;
    dt->n_live += m;
    dt->next_id += (uint32_t)m;
    set_layout(dt, dt->L - F + A, B);
}

// After a delete's plan: if the regrouping of under-full leaves would not fit
// the reserved buffers, it is skipped (the removals stand; leaves may stay
// below the minimum occupancy) and ERR_CAPACITY is latched.
__global__ void k_del_check(const DevTree* __restrict__ dt, uint32_t* __restrict__ ctr, Caps cap) {
    if (threadIdx.x | blockIdx.x) return;
    const uint64_t A = ctr[3], F = ctr[5], nf = dt->n_free;
    if (F == 0) return;
    const uint64_t take = A < nf ? A : nf;
    const uint64_t top = dt->slot_top + (A - take), nf2 = nf - take + F;
    if (ctr[2] > cap.leaves || top > cap.slots || nf2 > cap.frees || A > cap.alloc) {
        atomicOr(cap.err, ERR_CAPACITY);
        ctr[3] = 0;
        ctr[4] = 0;
        ctr[5] = 0;
    }
}

// Rejects the whole delete (ctr[9] = 1: no id is claimed) when the tree has
// more leaves than the launches cover.
__global__ void k_del_precheck(const DevTree* __restrict__ dt, uint32_t* __restrict__ ctr, Caps cap) {
    if (threadIdx.x | blockIdx.x) return;
    if (dt->L > cap.lgrid) {
        ctr[9] = 1;
        atomicOr(cap.err, ERR_CAPACITY);
    }
}

__global__ void k_del_commit(DevTree* dt, const uint32_t* __restrict__ ctr, uint32_t B) {
    if (threadIdx.x | blockIdx.x) return;
    const uint64_t V = ctr[0];
    dt->n_live -= V < dt->n_live ? V : dt->n_live;
    const uint64_t F = ctr[5];
    if (F == 0) return;
    const uint64_t A = ctr[3], nf = dt->n_free;
    const uint64_t take = A < nf ? A : nf;
    dt->slot_top += A - take;
    dt->n_free = nf - take + F;
    dt->cur ^= 1u;
    set_layout(dt, ctr[2], B);
}

// p[i] = v for i < n, only if *gate is nonzero when the kernel runs.
__global__ void k_fill_gated(uint32_t* __restrict__ p, uint64_t n, uint32_t v, const uint32_t* __restrict__ gate) {
    if (*gate == 0) return;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

inline unsigned grid_for(uint64_t n) {
    const uint64_t g = (n + 255) / 256;
    return g < 1 ? 1u : (g > 8192 ? 8192u : (unsigned)g);
}

}  // namespace

void st_set_dirs(hipStream_t st, DevTree* dt, NodeRec* l0, NodeRec* l1, uint64_t* k0, uint64_t* k1, uint32_t* i0,
                 uint32_t* i1) {
    hipLaunchKernelGGL(k_set_dirs, dim3(1), dim3(64), 0, st, dt, l0, l1, k0, k1, i0, i1);
}
void st_reset(hipStream_t st, DevTree* dt, uint32_t B) { hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, dt, B); }
void st_commit_build(hipStream_t st, DevTree* dt, uint64_t n, uint64_t L, uint32_t cur, uint32_t next_id,
                     uint32_t B) {
    hipLaunchKernelGGL(k_commit_build, dim3(1), dim3(64), 0, st, dt, n, L, cur, next_id, B);
}
void st_ins_ids(hipStream_t st, const DevTree* dt, const uint64_t* keys, uint64_t m, uint64_t* idkey, uint64_t id_cap,
                uint32_t* bi, uint32_t* new_ids, const uint32_t* ctr) {
    if (m) hipLaunchKernelGGL(k_ins_ids, dim3(grid_for(m)), dim3(256), 0, st, dt, keys, m, idkey, id_cap, bi, new_ids, ctr);
}
void st_ins_check(hipStream_t st, const DevTree* dt, uint32_t* ctr, uint64_t m, uint32_t phi, uint64_t id_cap,
                  Caps cap) {
    hipLaunchKernelGGL(k_ins_check, dim3(1), dim3(64), 0, st, dt, ctr, m, phi, id_cap, cap);
}
void st_ins_commit(hipStream_t st, DevTree* dt, const uint32_t* ctr, uint64_t m, uint32_t phi, uint32_t B) {
    hipLaunchKernelGGL(k_ins_commit, dim3(1), dim3(64), 0, st, dt, ctr, m, phi, B);
}
void st_del_check(hipStream_t st, const DevTree* dt, uint32_t* ctr, Caps cap) {
    hipLaunchKernelGGL(k_del_check, dim3(1), dim3(64), 0, st, dt, ctr, cap);
}
void st_del_precheck(hipStream_t st, const DevTree* dt, uint32_t* ctr, Caps cap) {
    hipLaunchKernelGGL(k_del_precheck, dim3(1), dim3(64), 0, st, dt, ctr, cap);
}
void st_del_commit(hipStream_t st, DevTree* dt, const uint32_t* ctr, uint32_t B) {
    hipLaunchKernelGGL(k_del_commit, dim3(1), dim3(64), 0, st, dt, ctr, B);
}
void st_fill_gated(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v, const uint32_t* gate) {
    if (n) hipLaunchKernelGGL(k_fill_gated, dim3(grid_for(n)), dim3(256), 0, st, p, n, v, gate);
}

}  // namespace psi
