// Device helpers shared by the SieveJoin kernels: hash mixers, the blocked Bloom
// filter's block and bit choice, wave/block scans and the decoupled look-back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sj_internal.h"

namespace sj {

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// MurmurHash3 32-bit finaliser (Austin Appleby, public domain).
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// SplitMix64 output function (Steele, Lea and Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Checksum factor of relation `rel`'s row `rid`: mix64((rel << 32) | rid) | 1.
__device__ __forceinline__ uint64_t chk_factor(uint32_t rel, uint32_t rid) {
    return mix64((static_cast<uint64_t>(rel) << 32) | rid) | 1ull;
}

// ---- blocked Bloom filter ----------------------------------------------------
// A key selects one block of B = 2^logB bits with the high bits of its 32-bit hash
// h = fmix32(key ^ seed) (block = h * nblocks / 2^32) and sets k bits inside it:
// bit i is the top logB bits of g * M_i, g = (h * 0x9E3779B1) ^ ((h * 0x9E3779B1) >> 16).
// Probing a key touches one block only (one 64-byte line for B = 512).

__device__ __forceinline__ uint32_t bf_mult(int i) {
    // odd multipliers, one per bit of the key's pattern (the compiler folds them
    // to immediates in the unrolled loops below)
    switch (i) {
        case 0: return 0x85EBCA77u;
        case 1: return 0xC2B2AE3Du;
        case 2: return 0x27D4EB2Fu;
        case 3: return 0x165667B1u;
        case 4: return 0xD3A2646Du;
        case 5: return 0xFD7046C5u;
        case 6: return 0xB55A4F09u;
        case 7: return 0x2545F491u;
        case 8: return 0x9E6C63D1u;
        case 9: return 0x7FEB352Du;
        case 10: return 0x846CA68Bu;
        default: return 0x68E31DA5u;
    }
}

struct BfKey {
    uint32_t block;
    uint32_t g;
};

__device__ __forceinline__ BfKey bf_hash(int32_t key, uint32_t seed, uint32_t nblocks) {
    uint32_t h = fmix32(static_cast<uint32_t>(key) ^ seed);
    BfKey r;
    r.block = __umulhi(h, nblocks);
    uint32_t g = h * 0x9E3779B1u;
    r.g = g ^ (g >> 16);
    return r;
}

// All k bits of the key's pattern set in the block starting at `blk`?
__device__ __forceinline__ bool bf_test(const uint32_t *__restrict__ blk, uint32_t g, int k, int logB) {
    uint32_t w[kMaxK];
    uint32_t p[kMaxK];
    const uint32_t sh = 32u - static_cast<uint32_t>(logB);
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) {
        if (i < k) {
            p[i] = (g * bf_mult(i)) >> sh;
            w[i] = blk[p[i] >> 5];
        }
    }
    uint32_t ok = 1u;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) {
        if (i < k) ok &= w[i] >> (p[i] & 31u);
    }
    return ok & 1u;
}

// Set the key's k bits; a bit already seen set is not written again.
__device__ __forceinline__ void bf_set(uint32_t *__restrict__ blk, uint32_t g, int k, int logB) {
    uint32_t w[kMaxK];
    uint32_t p[kMaxK];
    const uint32_t sh = 32u - static_cast<uint32_t>(logB);
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) {
        if (i < k) {
            p[i] = (g * bf_mult(i)) >> sh;
            w[i] = blk[p[i] >> 5];
        }
    }
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) {
        if (i < k) {
            const uint32_t m = 1u << (p[i] & 31u);
            if (!(w[i] & m)) atomicOr(blk + (p[i] >> 5), m);
        }
    }
}

// ---- scans -------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// The chip dispatches workgroup b of a launch to XCD b % 8, and each XCD has its own
// L2. For b < n this maps b to a work item so that each XCD takes one contiguous
// range of [0, n) (a bijection on [0, n)): partial cache lines that neighbouring items
// write then meet in one L2 instead of being written back from eight.
constexpr uint32_t kXcds = 8;
__host__ __device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n) {
    const uint32_t per = (n + kXcds - 1) / kXcds;      // items of the larger XCD ranges
    const uint32_t tall = n % kXcds ? n % kXcds : kXcds; // XCDs that take `per` items
    const uint32_t x = b % kXcds, i = b / kXcds;
    return x < tall ? x * per + i : tall * per + (x - tall) * (per - 1) + i;
}

// Order a wave's LDS writes before its later LDS reads by other lanes of the wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a block of BLOCK threads.
// s_wave must hold BLOCK/64 elements. Contains two barriers.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *s_wave, T &total) {
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    T incl = wave_incl_scan(x);
    if (lane == 63) s_wave[wid] = incl;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        T t = s_wave[w];
        if (w < wid) off += t;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return off + incl - x;
}

// ---- decoupled look-back over 32-bit tile counts --------------------------------
// Each tile publishes (flag << 32 | value) in one 64-bit word: flag 1 = the tile's
// own count, flag 2 = inclusive prefix. One atomic word per tile keeps flag and
// value consistent. Called by one thread per tile; returns the tile's exclusive
// prefix. Every spin ends: a tile publishes its own count before it looks back.
__device__ __forceinline__ uint32_t lookback32(uint64_t *status, uint32_t tile, uint32_t agg) {
    constexpr uint64_t kAgg = 1ull << 32, kIncl = 2ull << 32;
    if (tile == 0) {
        __hip_atomic_store(status, kIncl | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    __hip_atomic_store(status + tile, kAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    int64_t j = static_cast<int64_t>(tile) - 1;
    while (true) {
        uint64_t s = __hip_atomic_load(status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t f = static_cast<uint32_t>(s >> 32);
        if (f == 0) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += static_cast<uint32_t>(s);
        if (f == 2) break;
        --j;
    }
    __hip_atomic_store(status + tile, kIncl | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// The same protocol run by a whole wave: each step reads the 64 preceding status
// words at once and stops at the nearest inclusive prefix, so a tile waits for at
// most ceil(distance / 64) rounds instead of one round per predecessor. Called by all
// 64 lanes of one wave; returns the exclusive prefix in every lane.
__device__ __forceinline__ uint32_t lookback32_wave(uint64_t *status, uint32_t tile, uint32_t agg) {
    constexpr uint64_t kAgg = 1ull << 32, kIncl = 2ull << 32;
    const int lane = lane_id();
    if (tile == 0) {
        if (lane == 0) __hip_atomic_store(status, kIncl | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    if (lane == 0) __hip_atomic_store(status + tile, kAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    int64_t j = static_cast<int64_t>(tile) - 1;   // this round reads tiles j, j-1, ..., j-63
    while (true) {
        const int64_t idx = j - lane;
        const uint64_t s =
            idx >= 0 ? __hip_atomic_load(status + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kIncl;
        const uint32_t f = static_cast<uint32_t>(s >> 32);
        const uint64_t incl = __ballot(f == 2);
        const uint64_t empty = __ballot(f == 0);
        const int first = incl ? __ffsll(static_cast<long long>(incl)) - 1 : 64;   // nearest inclusive prefix
        const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);        // lanes 0 .. first
        if (empty & need) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint32_t v = lane <= first ? static_cast<uint32_t>(s) : 0u;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), d, 64));
        excl += v;
        if (first < 64) break;
        j -= 64;
    }
    if (lane == 0)
        __hip_atomic_store(status + tile, kIncl | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

__device__ __forceinline__ uint32_t upper_bound_u64(const uint64_t *a, uint32_t lo, uint32_t hi, uint64_t x) {
    // first i in [lo, hi) with a[i] > x (hi if none)
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] > x)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// The same search by a whole wave (all 64 lanes, the same arguments): each round the
// lanes read 64 evenly spaced pivots of [lo, hi) at once and a ballot keeps the part
// that holds the answer, so a range of m entries takes about log64(m) dependent loads
// instead of log2(m). Every lane returns the answer.
__device__ __forceinline__ uint32_t wave_upper_bound_u64(const uint64_t *a, uint32_t lo, uint32_t hi, uint64_t x) {
    const uint64_t lane = static_cast<uint64_t>(lane_id());
    // invariant: the answer is in [lo, hi], and hi is either the end of the range or an
    // index with a[hi] > x
    while (hi - lo > 64u) {
        const uint64_t step = (static_cast<uint64_t>(hi - lo) + 63u) / 64u;
        const uint64_t idx = lo + lane * step;
        const bool gt = idx < hi ? a[idx] > x : true;
        const uint64_t m = __ballot(gt);
        const uint64_t f = m ? static_cast<uint64_t>(__ffsll(static_cast<unsigned long long>(m)) - 1) : 64u;
        if (f == 0) return lo;
        const uint64_t nhi = lo + f * step;
        const uint32_t nlo = static_cast<uint32_t>(lo + (f - 1) * step + 1);
        hi = nhi < hi ? static_cast<uint32_t>(nhi) : hi;
        lo = nlo;
    }
    const uint64_t idx = lo + lane;
    const bool gt = idx < hi ? a[idx] > x : true;
    const uint64_t m = __ballot(gt);
    return m ? lo + static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(m)) - 1) : hi;
}

// ---- hash index over a bucketed relation's distinct keys ------------------------
// Slot word: ((dir + 1) << 32) | key; 0 marks an empty slot (dir + 1 >= 1).

__device__ __forceinline__ uint32_t slot_hash(int32_t key) {
    return fmix32(static_cast<uint32_t>(key) * 0x9E3779B1u + 0x7F4A7C15u);
}

__device__ __forceinline__ int64_t dir_find(const uint64_t *__restrict__ slots, uint32_t mask, int32_t key) {
    uint32_t s = slot_hash(key) & mask;
    while (true) {
        const uint64_t v = slots[s];
        if (v == 0) return -1;
        if (static_cast<uint32_t>(v) == static_cast<uint32_t>(key)) return static_cast<int64_t>(v >> 32) - 1;
        s = (s + 1) & mask;
    }
}

}  // namespace sj
