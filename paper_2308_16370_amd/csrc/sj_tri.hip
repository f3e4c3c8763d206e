// Directed 3-cycles by intersection.
//
// Section 3.1.3 pairs the sieve with a multi-way (worst-case-optimal) join for the
// cyclic query; this is that enumeration for the 3-cycle root - P - L - root. A result
// tuple (r, p, l) has P.key(p) = x(r), L.key(l) = z(p) and L.close(l) = y(r). For a
// root survivor r the matches are the pairs (p, l) drawn from P's group of x(r) and
// L's group of y(r) that agree on z. The walk takes the smaller group and looks each
// member's z up in the other relation's pair hash, which returns how many rows hold
// that (key, key) pair and the sum of their checksum factors, so one lookup accounts
// for every copy of a repeated pair. The binary plan instead expands every wedge
// (r, p) and then searches L; on power-law edge lists the wedges outnumber the walk
// steps by two orders of magnitude.
//
// Balance: walk lengths per root entry are scanned, and each wave takes equal chunks
// of consecutive walk steps, lane j every 64th step from the j-th (each lane finds its
// entry by binary search over the prefix, then gallops forward), so a hub's long walk
// is split over many waves and the group members a wave reads are consecutive.
#include <hip/hip_runtime.h>

#include "sj_device.h"
#include "sj_internal.h"

namespace sj {

namespace {

constexpr uint64_t kPairEmpty = ~0ull;
constexpr int kTriThreads = 256;

__device__ __forceinline__ uint64_t pair_key(int32_t a, int32_t b) {
    return (static_cast<uint64_t>(static_cast<uint32_t>(a)) << 32) | static_cast<uint32_t>(b);
}

// One 64-bit mix of the pair: the high word picks the table slot, the low word the
// membership bit (4 bits per slot in use).
__device__ __forceinline__ uint64_t pair_mix(uint64_t key) { return mix64(key ^ 0x243F6A8885A308D3ull); }
__device__ __forceinline__ uint32_t pair_slot(uint64_t hm, uint32_t mask) { return static_cast<uint32_t>(hm >> 32) & mask; }
__device__ __forceinline__ uint32_t pair_bit(uint64_t hm, uint32_t mask) {
    return static_cast<uint32_t>(hm) & (4u * mask + 3u);
}

__device__ __forceinline__ bool pair_find(const PairHash &h, uint32_t mask, uint64_t key, uint32_t &c,
                                          uint64_t &ms) {
    const uint64_t hm = pair_mix(key);
    const uint32_t b = pair_bit(hm, mask);
    if (!((h.sig[b >> 5] >> (b & 31u)) & 1u)) return false;   // absent: the table is not read
    uint32_t s = key == kPairEmpty ? h.cap : pair_slot(hm, mask);
    uint4 v;
    while (true) {   // the table is at most half full: an empty slot ends every probe
        v = *reinterpret_cast<const uint4 *>(h.slot + s);
        const uint64_t k = (static_cast<uint64_t>(v.y) << 32) | v.x;
        if (k == key) break;
        if (k == kPairEmpty || s == h.cap) return false;
        s = (s + 1) & mask;
    }
    c = v.z;
    if (c == 0) return false;
    ms = c == 1 ? chk_factor(h.rel, v.w) : h.msum[s];
    return true;
}

__global__ void k_pair_mask(PairHash h, const uint32_t *n_dev) {
    static_assert(sizeof(PairSlot) == 16, "one 16-byte load per slot");
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t n = *n_dev;
    uint32_t c = 16;
    while (c < 2u * n + 1u && c < h.cap) c <<= 1;
    *h.mask = c - 1;
}

__global__ void k_pair_clear(PairHash h) {
    const uint32_t lim = *h.mask + 1u;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const PairSlot empty{kPairEmpty, 0u, 0u};
    for (uint32_t i = t; i < lim; i += gridDim.x * blockDim.x) {
        h.slot[i] = empty;
        h.msum[i] = 0;
        if (i < lim / 8u) h.sig[i] = 0;   // 4 bits per slot: lim / 8 words
    }
    if (t == 0) {
        h.slot[h.cap] = empty;
        h.msum[h.cap] = 0;
    }
}

// One insert per run of equal pairs in adjacent lanes (entries come grouped by their
// first key, so repeated pairs are often neighbours); the run's count and factor sum
// come from a wave prefix sum.
__global__ __launch_bounds__(256) void k_pair_insert(PairHash h, const uint32_t *n_dev, const uint32_t *rid,
                                                     const int32_t *ca, const int32_t *cb, uint32_t rel) {
    const uint32_t n = *n_dev, mask = *h.mask;
    const int lane = lane_id();
    const uint32_t ngroups = (n + 63) / 64;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t g = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; g < ngroups; g += nwaves) {
        const uint32_t e = g * 64 + static_cast<uint32_t>(lane);
        const bool ok = e < n;
        const uint64_t key = ok ? pair_key(ca[e], cb[e]) : 0;
        const uint32_t my_rid = ok ? rid[e] : 0u;
        const uint64_t m = ok ? chk_factor(rel, my_rid) : 0;
        const uint64_t prev = __shfl_up(key, 1, 64);
        int start = (lane == 0 || key != prev) ? lane : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(start, d, 64);
            if (lane >= d && o > start) start = o;
        }
        const uint64_t pre = wave_incl_scan(m);
        const uint64_t before = __shfl(pre, start > 0 ? start - 1 : 0, 64);
        const uint32_t first_rid = __shfl(my_rid, start, 64);
        const uint64_t next = __shfl_down(key, 1, 64);
        const bool tail = ok && (lane == 63 || e + 1 >= n || next != key);
        if (!tail) continue;
        const uint32_t c = static_cast<uint32_t>(lane - start + 1);
        const uint64_t ms = pre - (start > 0 ? before : 0);
        const uint64_t hm = pair_mix(key);
        const uint32_t b = pair_bit(hm, mask);
        if (!((h.sig[b >> 5] >> (b & 31u)) & 1u)) atomicOr(h.sig + (b >> 5), 1u << (b & 31u));
        uint32_t s;
        if (key == kPairEmpty) {
            s = h.cap;
        } else {
            s = pair_slot(hm, mask);
            while (true) {
                const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long *>(&h.slot[s].key),
                                                         static_cast<unsigned long long>(kPairEmpty),
                                                         static_cast<unsigned long long>(key));
                if (old == kPairEmpty || old == key) break;
                s = (s + 1) & mask;
            }
        }
        // the first rows to arrive leave their first row id (read when the pair has one row)
        if (atomicAdd(&h.slot[s].cnt, c) == 0u) h.slot[s].rid = first_rid;
        atomicAdd(reinterpret_cast<unsigned long long *>(h.msum + s), static_cast<unsigned long long>(ms));
    }
}

// Phase 1: each root entry's walk (the smaller of its two groups) and per-tile sums.
__global__ __launch_bounds__(kScanBlock) void k_tri_rows(TriArgs a) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    const uint32_t n = *a.n_root;
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    const uint32_t pmask = *a.P_mask, lmask = *a.L_mask;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t base = tile * kScanTile + threadIdx.x * kScanItems;
        uint64_t sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t e = base + i;
            if (e >= n) continue;
            uint32_t bp = 0, np = 0, bl = 0, nl = 0;
            const int64_t dp = dir_find(a.P_slots, pmask, a.root_x[e]);
            if (dp >= 0) {
                bp = a.P_begin[dp];
                np = a.P_begin[dp + 1] - bp;
            }
            const int64_t dl = dir_find(a.L_slots, lmask, a.root_y[e]);
            if (dl >= 0) {
                bl = a.L_begin[dl];
                nl = a.L_begin[dl + 1] - bl;
            }
            const bool walk_l = nl < np;
            const uint32_t w = walk_l ? nl : np;
            a.w[e] = w | (walk_l ? 0x80000000u : 0u);
            a.beg[e] = walk_l ? bl : bp;
            sum += w;
        }
        uint64_t tot;
        block_excl_scan<kScanBlock>(sum, s_w, tot);
        if (threadIdx.x == 0) a.tile_sums[tile] = tot;
    }
}

// Phase 2 (one block): exclusive scan of the tile sums; the total lands in off[n].
__global__ __launch_bounds__(kScanBlock) void k_tri_tiles(TriArgs a) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    __shared__ uint64_t s_carry;
    const uint32_t n = *a.n_root;
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t t0 = 0; t0 < ntiles; t0 += kScanBlock) {
        const uint32_t t = t0 + threadIdx.x;
        const uint64_t v = t < ntiles ? a.tile_sums[t] : 0;
        uint64_t tot;
        const uint64_t o = block_excl_scan<kScanBlock>(v, s_w, tot);
        if (t < ntiles) a.tile_sums[t] = s_carry + o;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.off[n] = s_carry;
}

// Phase 3: per-entry exclusive prefixes.
__global__ __launch_bounds__(kScanBlock) void k_tri_down(TriArgs a) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    const uint32_t n = *a.n_root;
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t base = tile * kScanTile + threadIdx.x * kScanItems;
        uint64_t w[kScanItems];
        uint64_t sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t e = base + i;
            w[i] = e < n ? (a.w[e] & 0x7FFFFFFFu) : 0;
            sum += w[i];
        }
        uint64_t tot;
        uint64_t o = block_excl_scan<kScanBlock>(sum, s_w, tot) + a.tile_sums[tile];
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t e = base + i;
            if (e < n) a.off[e] = o;
            o += w[i];
        }
    }
}

// The walk: each wave takes chunks of 64 * kTriIters consecutive steps; lane j takes
// steps base + 64 * i + j, so the group members a wave reads are consecutive.
constexpr int kTriIters = 32;
__global__ __launch_bounds__(kTriThreads) void k_tri_count(TriArgs a) {
    __shared__ uint64_t s_c[kTriThreads / 64], s_k[kTriThreads / 64];
    const uint32_t n = *a.n_root;
    const uint64_t total = a.off[n];
    constexpr uint64_t kWaveSteps = 64ull * kTriIters;
    const uint64_t nchunks = (total + kWaveSteps - 1) / kWaveSteps;
    const uint32_t pm = *a.HP.mask, lm = *a.HL.mask;
    const uint32_t lane = static_cast<uint32_t>(lane_id());
    uint64_t cnt = 0, chk = 0;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    for (uint64_t c = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; c < nchunks; c += nwaves) {
        uint64_t w = c * kWaveSteps + lane;
        if (w >= total) continue;
        uint32_t r = upper_bound_u64(a.off, 0, n, w) - 1;
        uint64_t r_lo = a.off[r], r_hi = a.off[r + 1];
        bool loaded = false;
        bool walk_l = false;
        uint32_t beg = 0;
        int32_t x = 0, y = 0;
        uint64_t m1 = 0;
        for (int it = 0; it < kTriIters && w < total; ++it, w += 64) {
            if (w >= r_hi) {
                // gallop from r + 1 to an entry past w, then search: off[r] <= w < off[r + 1]
                uint32_t lo = r + 1, step = 1, hi = lo;
                while (hi < n && a.off[hi + 1] <= w) {
                    lo = hi + 1;
                    hi = min(n - 1, hi + step);
                    step <<= 1;
                }
                r = upper_bound_u64(a.off, lo, hi + 1, w) - 1;
                r_lo = a.off[r];
                r_hi = a.off[r + 1];
                loaded = false;
            }
            if (!loaded) {
                const uint32_t wr = a.w[r];
                walk_l = (wr >> 31) != 0;
                beg = a.beg[r];
                x = a.root_x[r];
                y = a.root_y[r];
                m1 = chk_factor(a.rel_root, a.root_rid[r]);
                loaded = true;
            }
            const uint32_t e = beg + static_cast<uint32_t>(w - r_lo);
            uint32_t hc;
            uint64_t hm, mo;
            bool hit;
            if (!walk_l) {
                mo = chk_factor(a.rel_P, a.P_rid[e]);
                hit = pair_find(a.HL, lm, pair_key(y, a.P_z[e]), hc, hm);
            } else {
                mo = chk_factor(a.rel_L, a.L_rid[e]);
                hit = pair_find(a.HP, pm, pair_key(x, a.L_z[e]), hc, hm);
            }
            if (hit) {
                cnt += hc;
                chk += m1 * mo * hm;
            }
        }
    }
    uint64_t tc, tk;
    block_excl_scan<kTriThreads>(cnt, s_c, tc);
    block_excl_scan<kTriThreads>(chk, s_k, tk);
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = tc;
        a.part[2 * blockIdx.x + 1] = tk;
    }
}

__global__ __launch_bounds__(kTriThreads) void k_tri_final(TriArgs a, uint32_t nblocks) {
    __shared__ uint64_t s_c[kTriThreads / 64], s_k[kTriThreads / 64];
    uint64_t c = 0, k = 0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
        c += a.part[2 * b];
        k += a.part[2 * b + 1];
    }
    uint64_t tc, tk;
    block_excl_scan<kTriThreads>(c, s_c, tc);
    block_excl_scan<kTriThreads>(k, s_k, tk);
    if (threadIdx.x == 0) {
        a.totals[0] = tc;
        a.totals[1] = tk;
    }
}

uint32_t blocks_for(uint64_t items, uint32_t per_block, uint32_t cap) {
    const uint64_t g = (items + per_block - 1) / per_block;
    return g == 0 ? 1u : static_cast<uint32_t>(g < cap ? g : cap);
}

}  // namespace

hipError_t launch_pair_build(const PairHash &h, const uint32_t *n_dev, uint32_t cap_rows, const uint32_t *rid,
                             const int32_t *ca, const int32_t *cb, uint32_t rel, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_mask, dim3(1), dim3(64), 0, s, h, n_dev);
    hipLaunchKernelGGL(k_pair_clear, dim3(blocks_for(uint64_t(h.cap) + 1, 256, kPersistentBlocks)), dim3(256), 0, s, h);
    if (cap_rows > 0)
        hipLaunchKernelGGL(k_pair_insert, dim3(blocks_for(cap_rows, 256, kPersistentBlocks)), dim3(256), 0, s, h,
                           n_dev, rid, ca, cb, rel);
    return hipGetLastError();
}

hipError_t launch_tri_count(const TriArgs &a, hipStream_t s) {
    const uint32_t tiles = blocks_for(a.root_cap, kScanTile, kPersistentBlocks);
    hipLaunchKernelGGL(k_tri_rows, dim3(tiles), dim3(kScanBlock), 0, s, a);
    hipLaunchKernelGGL(k_tri_tiles, dim3(1), dim3(kScanBlock), 0, s, a);
    hipLaunchKernelGGL(k_tri_down, dim3(tiles), dim3(kScanBlock), 0, s, a);
    hipLaunchKernelGGL(k_tri_count, dim3(kTriBlocks), dim3(kTriThreads), 0, s, a);
    hipLaunchKernelGGL(k_tri_final, dim3(1), dim3(kTriThreads), 0, s, a, kTriBlocks);
    return hipGetLastError();
}

}  // namespace sj
