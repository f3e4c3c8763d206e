// Update maintenance (Section 2.4): counting twins of blocked filters (inserts and
// deletes of tuples), and the propagation of newly inserted tuples from a relation's
// filter toward the root (a parent's rows that now pass insert their own key).
#include <hip/hip_runtime.h>

#include "sj_device.h"
#include "sj_internal.h"

namespace sj {

// ---- counting filters ----------------------------------------------------------
// A counting filter has one 4-bit counter per bit position of the blocked filter it
// twins (same blocks, k, seed and bit pattern): block b's position p is nibble p % 8 of
// word b * B / 8 + p / 8. A bit of the plain filter is set iff its counter is nonzero.
// Counters saturate at 15 and then stay (a saturated counter is never decremented, so
// no deletion can clear a bit another tuple still needs).

__device__ __forceinline__ void cf_step(uint32_t *w, uint32_t nib, int sign) {
    const uint32_t sh = 4u * nib;
    uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const uint32_t c = (old >> sh) & 15u;
        if (c == 15u || (sign < 0 && c == 0u)) return;   // saturated, or nothing to remove
        const uint32_t nw = sign > 0 ? old + (1u << sh) : old - (1u << sh);
        const uint32_t seen = atomicCAS(w, old, nw);
        if (seen == old) return;
        old = seen;
    }
}

__global__ __launch_bounds__(256) void k_cf_update(CfArgs a, int sign) {
    const uint32_t nb = a.nblocks;
    const uint32_t sh = 32u - static_cast<uint32_t>(a.logB);
    const uint32_t wpb = 1u << (a.logB - 3);   // counter words per block
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        if (a.pred) {
            const int32_t v = a.pred[i];
            if (v < a.pred_lo || v >= a.pred_hi) continue;
        }
        const BfKey h = bf_hash(a.keys[i], a.seed, nb);
        uint32_t *blk = a.counts + static_cast<uint64_t>(h.block) * wpb;
        for (int j = 0; j < a.k; ++j) {
            const uint32_t p = (h.g * bf_mult(j)) >> sh;
            cf_step(blk + (p >> 3), p & 7u, sign);
        }
    }
}

// The key count of a device-side length (list sources) replaces a.n.
__global__ __launch_bounds__(256) void k_cf_update_dev(CfArgs a, const uint32_t *n_dev, int sign) {
    a.n = *n_dev;
    const uint32_t nb = a.nblocks;
    const uint32_t sh = 32u - static_cast<uint32_t>(a.logB);
    const uint32_t wpb = 1u << (a.logB - 3);
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const BfKey h = bf_hash(a.keys[i], a.seed, nb);
        uint32_t *blk = a.counts + static_cast<uint64_t>(h.block) * wpb;
        for (int j = 0; j < a.k; ++j) {
            const uint32_t p = (h.g * bf_mult(j)) >> sh;
            cf_step(blk + (p >> 3), p & 7u, sign);
        }
    }
}

__global__ __launch_bounds__(256) void k_cf_probe(CfArgs a, uint8_t *contained, unsigned long long *missing) {
    __shared__ uint64_t s_w[4];
    const uint32_t nb = a.nblocks;
    const uint32_t sh = 32u - static_cast<uint32_t>(a.logB);
    const uint32_t wpb = 1u << (a.logB - 3);
    uint64_t miss = 0;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const BfKey h = bf_hash(a.keys[i], a.seed, nb);
        const uint32_t *blk = a.counts + static_cast<uint64_t>(h.block) * wpb;
        bool ok = true;
        for (int j = 0; j < a.k; ++j) {
            const uint32_t p = (h.g * bf_mult(j)) >> sh;
            ok &= ((blk[p >> 3] >> (4u * (p & 7u))) & 15u) != 0u;
        }
        contained[i] = ok ? 1 : 0;
        miss += ok ? 0 : 1;
    }
    uint64_t tot;
    block_excl_scan<256>(miss, s_w, tot);
    if (threadIdx.x == 0 && tot) atomicAdd(missing, static_cast<unsigned long long>(tot));
}

// Plain filter words from the counters: 8 counter words give one 32-bit filter word.
__global__ __launch_bounds__(256) void k_cf_export(const uint32_t *counts, uint64_t nwords, uint32_t *words) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t w = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        uint32_t bits = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t c = counts[w * 4 + q];
#pragma unroll
            for (int t = 0; t < 8; ++t) bits |= (((c >> (4 * t)) & 15u) != 0u ? 1u : 0u) << (q * 8 + t);
        }
        words[w] = bits;
    }
}

static uint32_t grid_of(uint64_t n) {
    const uint64_t g = (n + 255) / 256;
    return static_cast<uint32_t>(g < 2048 ? (g ? g : 1) : 2048);
}

hipError_t launch_cf_update(const CfArgs &a, const uint32_t *n_dev, uint32_t n_max, int sign, hipStream_t s) {
    if (n_dev) {
        if (n_max == 0) return hipSuccess;
        hipLaunchKernelGGL(k_cf_update_dev, dim3(grid_of(n_max)), dim3(256), 0, s, a, n_dev, sign);
    } else {
        if (a.n == 0) return hipSuccess;
        hipLaunchKernelGGL(k_cf_update, dim3(grid_of(a.n)), dim3(256), 0, s, a, sign);
    }
    return hipGetLastError();
}

hipError_t launch_cf_probe(const CfArgs &a, uint8_t *contained, unsigned long long *missing, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cf_probe, dim3(grid_of(a.n)), dim3(256), 0, s, a, contained, missing);
    return hipGetLastError();
}

hipError_t launch_cf_export(const uint32_t *counts, uint64_t nwords, uint32_t *words, hipStream_t s) {
    if (nwords == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cf_export, dim3(grid_of(nwords)), dim3(256), 0, s, counts, nwords, words);
    return hipGetLastError();
}

// ---- propagation toward the root ---------------------------------------------------
// An exact set of int32 keys: open addressing over 64-bit slots (1 << 32 | key), 0 empty.

__global__ __launch_bounds__(256) void k_set_insert(KeySet set, const int32_t *keys, const uint8_t *skip,
                                                    uint64_t n) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (skip && skip[i]) continue;   // only the keys the filter did not contain
        const uint32_t key = static_cast<uint32_t>(keys[i]);
        const unsigned long long v = (1ull << 32) | key;
        uint32_t slot = fmix32(key * 0x9E3779B1u + 0x7F4A7C15u) & set.mask;
        for (;;) {
            const unsigned long long seen = atomicCAS(reinterpret_cast<unsigned long long *>(set.slots + slot), 0ull, v);
            if (seen == 0ull || seen == v) break;
            slot = (slot + 1) & set.mask;
        }
    }
}

__device__ __forceinline__ bool set_has(const KeySet &set, int32_t k) {
    if (!set.slots) return true;   // no set: every row is a candidate
    const uint32_t key = static_cast<uint32_t>(k);
    const uint64_t v = (1ull << 32) | key;
    uint32_t slot = fmix32(key * 0x9E3779B1u + 0x7F4A7C15u) & set.mask;
    for (;;) {
        const uint64_t s = set.slots[slot];
        if (s == v) return true;
        if (s == 0) return false;
        slot = (slot + 1) & set.mask;
    }
}

// Rows of a relation whose key on `match_col` is in the set, that pass the predicate and
// every filter in `probes`: their key on `out_col` is appended to `out` (order free:
// the keys only go into a filter).
__global__ __launch_bounds__(256) void k_propagate_rows(PropArgs a) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    const uint32_t wpb_shift = static_cast<uint32_t>(a.logB) - 5u;
    for (uint64_t r = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < a.nrows; r += stride) {
        if (a.match_col && !set_has(a.set, a.match_col[r])) continue;
        if (a.pred) {
            const int32_t v = a.pred[r];
            if (v < a.pred_lo || v >= a.pred_hi) continue;
        }
        bool ok = true;
        for (int p = 0; p < a.nprobe && ok; ++p) {
            const uint32_t nb = *a.probe[p].nblocks;
            const BfKey h = bf_hash(a.probe_col[p][r], a.seed, nb);
            ok = bf_test(a.probe[p].words + (static_cast<uint64_t>(h.block) << wpb_shift), h.g, a.k, a.logB);
        }
        if (!ok) continue;
        const uint32_t o = atomicAdd(a.out_n, 1u);
        a.out[o] = a.out_col[r];
    }
}

// New rows of a relation (caller columns): the ones that pass its predicate and its
// children's filters append their parent-edge key.
hipError_t launch_propagate_rows(const PropArgs &a, hipStream_t s) {
    if (a.nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_propagate_rows, dim3(grid_of(a.nrows)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_set_insert(const KeySet &set, const int32_t *keys, const uint8_t *skip, uint64_t n,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_insert, dim3(grid_of(n)), dim3(256), 0, s, set, keys, skip, n);
    return hipGetLastError();
}

}  // namespace sj
