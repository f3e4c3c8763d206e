// Directed 3-cycles and 4-cliques by intersection.
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

// The pair's slot (h.cap for the spare one) and row count, or -1 when it is absent.
__device__ __forceinline__ int64_t pair_slot_of(const PairHash &h, uint32_t mask, uint64_t key, uint32_t &c) {
    const uint64_t hm = pair_mix(key);
    const uint32_t b = pair_bit(hm, mask);
    if (!((h.sig[b >> 5] >> (b & 31u)) & 1u)) return -1;
    uint32_t s = key == kPairEmpty ? h.cap : pair_slot(hm, mask);
    uint4 v;
    while (true) {
        v = *reinterpret_cast<const uint4 *>(h.slot + s);
        const uint64_t k = (static_cast<uint64_t>(v.y) << 32) | v.x;
        if (k == key) break;
        if (k == kPairEmpty || s == h.cap) return -1;
        s = (s + 1) & mask;
    }
    c = v.z;
    return c == 0 ? -1 : static_cast<int64_t>(s);
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
        h.pos[i] = ~0u;
        if (i < lim / 8u) h.sig[i] = 0;   // 4 bits per slot: lim / 8 words
    }
    if (t == 0) {
        h.slot[h.cap] = empty;
        h.msum[h.cap] = 0;
        h.pos[h.cap] = ~0u;
    }
}

// One insert per run of equal pairs in adjacent lanes (entries come sorted by pair, so
// a pair's rows are consecutive); the run's count and factor sum come from a wave
// prefix sum.
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
        // the first rows to arrive leave their first row id (read when the pair has one row);
        // the smallest bucket position among the runs is where the pair's rows start
        if (atomicAdd(&h.slot[s].cnt, c) == 0u) h.slot[s].rid = first_rid;
        atomicMin(h.pos + s, g * 64 + static_cast<uint32_t>(start));
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
    a.lane_cnt[blockIdx.x * blockDim.x + threadIdx.x] = cnt;   // the lane's tuples (hc per match)
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = tc;
        a.part[2 * blockIdx.x + 1] = tk;
        a.block_cnt[blockIdx.x] = tc;
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

// ---- 4-cliques ------------------------------------------------------------------------
// Generic join in the variable order a, b, c, d. For a root entry (a, b) the values c
// come from intersecting ac's group of a with bc's group of b: the walk takes the
// smaller group and looks each member up in the other relation's pair hash, as for
// 3-cycles, and uses the same balanced chunks. For each c found, the values d lie in
// the groups ad(a), bd(b) and cd(c): the smallest is walked and its members are looked
// up in the other two pair hashes. Per tuple of variable values the rows multiply, so
// a match adds the product of the pairs' row counts, and the checksum term is the
// product of the walked rows' factors and the looked-up pairs' factor sums.

__device__ __forceinline__ void k4_range(const K4Group &g, uint32_t mask, int32_t key, uint32_t &b, uint32_t &n) {
    b = 0;
    n = 0;
    const int64_t d = dir_find(g.slots, mask, key);
    if (d >= 0) {
        b = g.begin[d];
        n = g.begin[d + 1] - b;
    }
}

// Phase 1: each root entry's first-level walk (the smaller of ac(a) and bc(b)).
__global__ __launch_bounds__(kScanBlock) void k_k4_rows(K4Args a) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    const uint32_t n = *a.n_root;
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    const uint32_t m_ac = *a.g[0].mask, m_bc = *a.g[2].mask;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t base = tile * kScanTile + threadIdx.x * kScanItems;
        uint64_t sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t e = base + i;
            if (e >= n) continue;
            uint32_t b1, n1, b2, n2;
            k4_range(a.g[0], m_ac, a.root_a[e], b1, n1);
            k4_range(a.g[2], m_bc, a.root_b[e], b2, n2);
            const bool walk_bc = n2 < n1;
            const uint32_t w = walk_bc ? n2 : n1;
            a.w[e] = w | (walk_bc ? 0x80000000u : 0u);
            a.beg[e] = walk_bc ? b2 : b1;
            sum += w;
        }
        uint64_t tot;
        block_excl_scan<kScanBlock>(sum, s_w, tot);
        if (threadIdx.x == 0) a.tile_sums[tile] = tot;
    }
}

// Second level, balanced over the wave. A lane's first-level hit (root entry (a, b) and
// c) names the smallest of the groups ad(a), bd(b), cd(c) to walk, a job of wn members;
// on a power-law graph one hub's group can be thousands of members long, and a lane
// walking it alone holds the other 63 idle. So each first-level round the wave lays its
// jobs end to end (a prefix sum of their lengths) and lane l takes members l, l + 64, ...
// of the concatenation: the job holding member t is the first whose inclusive prefix
// exceeds t (a binary search over the wave's 64 prefixes in LDS). Every member's count
// and checksum terms are products, so regrouping the sums changes nothing.
struct K4Job {
    uint64_t f;                // count: checksum factors of the root row, the walked level-one
                               // row and the level-one pair's rows; write: the two row ids
    int32_t av, bv, cv;
    uint32_t wb, wn;           // the walked group's first entry and member count
    uint32_t c1;               // rows of the level-one pair
    uint32_t l1_pos;           // write: first of those rows in their group (pair-hash order)
    uint8_t W;                 // walked group: 1 (ad), 3 (bd) or 4 (cd)
    uint8_t walk_bc;           // the walked level-one row is bc's (else ac's)
};

// Member e of job jb, whose walked group is W: its d is looked up with (x1, d) in pair
// hash H1 and (x2, d) in H2 (ad walked: bd, cd; bd walked: ad, cd; cd walked: ad, bd).
template <int W>
__device__ __forceinline__ void k4_member_count(const K4Args &a, const K4Job &jb, uint32_t e, uint64_t &cnt,
                                                uint64_t &chk) {
    constexpr int H1 = W == 1 ? 3 : 1, H2 = W == 4 ? 3 : 4;
    const int32_t x1 = H1 == 3 ? jb.bv : jb.av, x2 = H2 == 3 ? jb.bv : jb.cv;
    const K4Group &g = a.g[W];
    const int32_t d = g.other[e];
    uint32_t cA, cB;
    uint64_t sA, sB;
    if (!pair_find(a.h[H1], *a.h[H1].mask, pair_key(x1, d), cA, sA)) return;
    if (!pair_find(a.h[H2], *a.h[H2].mask, pair_key(x2, d), cB, sB)) return;
    cnt += static_cast<uint64_t>(jb.c1) * cA * cB;
    chk += jb.f * chk_factor(g.rel, g.rid[e]) * sA * sB;
}

// The wave's jobs: the job holding member t and t's index in it.
__device__ __forceinline__ uint32_t k4_job_of(const uint64_t *incl, uint64_t t) {
    uint32_t lo = 0, hi = 64;   // first i with incl[i] > t
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (incl[mid] > t)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// The first level of step w (root entry r, member w - r_lo of its walked level-one
// group): whether (a, b, c) closes, and the second-level job if it does. The root
// entry's values and its ad, bd ranges are cached across the lane's steps.
struct K4Cursor {
    uint32_t r;
    uint64_t r_lo, r_hi;
    bool loaded, walk_bc;
    uint32_t beg, ad_b, ad_n, bd_b, bd_n, root_rid;
    int32_t av, bv;
    uint64_t m0;
};

template <bool WRITE_IDS>
__device__ __forceinline__ bool k4_first(const K4Args &a, const uint32_t *gm, const uint32_t *hm, uint32_t n,
                                         uint64_t w, K4Cursor &q, K4Job &jb) {
    if (w >= q.r_hi) {
        uint32_t lo = q.r + 1, step = 1, hi = lo;
        while (hi < n && a.off[hi + 1] <= w) {
            lo = hi + 1;
            hi = min(n - 1, hi + step);
            step <<= 1;
        }
        q.r = upper_bound_u64(a.off, lo, hi + 1, w) - 1;
        q.r_lo = a.off[q.r];
        q.r_hi = a.off[q.r + 1];
        q.loaded = false;
    }
    if (!q.loaded) {
        q.walk_bc = (a.w[q.r] >> 31) != 0;
        q.beg = a.beg[q.r];
        q.av = a.root_a[q.r];
        q.bv = a.root_b[q.r];
        q.root_rid = a.root_rid[q.r];
        q.m0 = WRITE_IDS ? 0 : chk_factor(a.rel_root, q.root_rid);
        k4_range(a.g[1], gm[1], q.av, q.ad_b, q.ad_n);
        k4_range(a.g[3], gm[3], q.bv, q.bd_b, q.bd_n);
        q.loaded = true;
    }
    if (q.ad_n == 0 || q.bd_n == 0) return false;
    const uint32_t e = q.beg + static_cast<uint32_t>(w - q.r_lo);
    // the walked level-one row is ac's (walk over ac(a)) or bc's; the other side's rows
    // come from the pair hash
    const K4Group &g1 = a.g[q.walk_bc ? 2 : 0];
    const int32_t cv = g1.other[e];
    uint32_t c1 = 0;
    int64_t s1;
    uint64_t ms = 0;
    if (WRITE_IDS) {
        s1 = q.walk_bc ? pair_slot_of(a.h[0], hm[0], pair_key(q.av, cv), c1)
                       : pair_slot_of(a.h[2], hm[2], pair_key(q.bv, cv), c1);
    } else {
        const bool hit = q.walk_bc ? pair_find(a.h[0], hm[0], pair_key(q.av, cv), c1, ms)
                                   : pair_find(a.h[2], hm[2], pair_key(q.bv, cv), c1, ms);
        s1 = hit ? 0 : -1;
    }
    if (s1 < 0) return false;
    uint32_t cd_b, cd_n;
    k4_range(a.g[4], gm[4], cv, cd_b, cd_n);
    if (cd_n == 0) return false;
    jb.av = q.av;
    jb.bv = q.bv;
    jb.cv = cv;
    jb.c1 = c1;
    jb.walk_bc = q.walk_bc ? 1 : 0;
    if (q.ad_n <= q.bd_n && q.ad_n <= cd_n) {
        jb.W = 1; jb.wb = q.ad_b; jb.wn = q.ad_n;
    } else if (q.bd_n <= cd_n) {
        jb.W = 3; jb.wb = q.bd_b; jb.wn = q.bd_n;
    } else {
        jb.W = 4; jb.wb = cd_b; jb.wn = cd_n;
    }
    if (WRITE_IDS) {
        jb.f = static_cast<uint64_t>(q.root_rid) | (static_cast<uint64_t>(g1.rid[e]) << 32);
        jb.l1_pos = q.walk_bc ? a.h[0].pos[s1] : a.h[2].pos[s1];
    } else {
        jb.f = q.m0 * chk_factor(g1.rel, g1.rid[e]) * ms;
        jb.l1_pos = 0;
    }
    return true;
}

// One wave's chunk of first-level steps, kTriIters rounds of 64, each round's jobs walked
// by the whole wave. MODE 0: count and checksum (acc0, acc1); MODE 1: the tuples written
// from acc1 (acc0 unused).
template <int MODE>
__device__ __forceinline__ void k4_chunk(const K4Args &a, const CliqueOut *o, const uint32_t *gm, const uint32_t *hm,
                                         uint32_t n, uint64_t total, uint64_t c, K4Job *jobs, uint64_t *incl_s,
                                         uint64_t &acc0, uint64_t &acc1);

__global__ __launch_bounds__(kTriThreads) void k_k4_count(K4Args a) {
    __shared__ uint64_t s_c[kTriThreads / 64], s_k[kTriThreads / 64];
    __shared__ K4Job s_job[kTriThreads / 64][64];
    __shared__ uint64_t s_incl[kTriThreads / 64][64];
    const uint32_t n = *a.n_root;
    const uint64_t total = a.off[n];
    constexpr uint64_t kWaveSteps = 64ull * kTriIters;
    const uint64_t nchunks = (total + kWaveSteps - 1) / kWaveSteps;
    uint32_t gm[5], hm[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        gm[i] = *a.g[i].mask;
        hm[i] = *a.h[i].mask;
    }
    const uint32_t wid = threadIdx.x >> 6;
    uint64_t cnt = 0, chk = 0;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    for (uint64_t c = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; c < nchunks; c += nwaves)
        k4_chunk<0>(a, nullptr, gm, hm, n, total, c, s_job[wid], s_incl[wid], cnt, chk);
    uint64_t tc, tk;
    block_excl_scan<kTriThreads>(cnt, s_c, tc);
    block_excl_scan<kTriThreads>(chk, s_k, tk);
    a.lane_cnt[blockIdx.x * blockDim.x + threadIdx.x] = cnt;   // the lane's tuples (c1 cA cB per match)
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = tc;
        a.part[2 * blockIdx.x + 1] = tk;
        a.block_cnt[blockIdx.x] = tc;
    }
}

// ---- write pass (3-cycles and 4-cliques) ------------------------------------------------
// The count pass gives every lane the same walk steps as the write pass and records each
// lane's and each workgroup's tuple count; the write pass walks again and writes a lane's
// tuples from its offset: the workgroups before it, then the lanes before it. It uses the
// count pass's walk lengths, prefixes and tuple counts (still in the workspace).

template <int NR>
__device__ __forceinline__ void emit_tuple(const CliqueOut &o, uint64_t at, const uint32_t (&rr)[NR]) {
    if (at >= o.capacity) return;
    if (o.proj.n == 0) {
        int32_t *dst = o.out + at * static_cast<uint64_t>(o.nrels);
#pragma unroll
        for (int i = 0; i < NR; ++i) dst[o.role_rel[i]] = static_cast<int32_t>(rr[i]);
    } else {
        int32_t *dst = o.out + at * static_cast<uint64_t>(o.proj.n);
        for (int q = 0; q < o.proj.n; ++q) {
            uint32_t rid = 0;
#pragma unroll
            for (int i = 0; i < NR; ++i)
                if (o.proj.rel[q] == o.role_rel[i]) rid = rr[i];
            dst[q] = o.proj.col[q][rid];
        }
    }
}

__device__ __forceinline__ uint64_t emit_base(const CliqueOut &o, uint64_t *s_tmp) {
    uint64_t before = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += blockDim.x) before += o.block_cnt[b];
    uint64_t blocks_before, t;
    block_excl_scan<kTriThreads>(before, s_tmp, blocks_before);
    const uint64_t lanes_before =
        block_excl_scan<kTriThreads>(o.lane_cnt[blockIdx.x * blockDim.x + threadIdx.x], s_tmp, t);
    return blocks_before + lanes_before;
}

__global__ __launch_bounds__(kTriThreads) void k_tri_emit(TriArgs a, CliqueOut o) {
    __shared__ uint64_t s_tmp[kTriThreads / 64];
    const uint32_t n = *a.n_root;
    const uint64_t total = a.off[n];
    constexpr uint64_t kWaveSteps = 64ull * kTriIters;
    const uint64_t nchunks = (total + kWaveSteps - 1) / kWaveSteps;
    const uint32_t pm = *a.HP.mask, lm = *a.HL.mask;
    const uint32_t lane = static_cast<uint32_t>(lane_id());
    uint64_t cur = emit_base(o, s_tmp);
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    for (uint64_t c = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; c < nchunks; c += nwaves) {
        uint64_t w = c * kWaveSteps + lane;
        if (w >= total) continue;
        uint32_t r = upper_bound_u64(a.off, 0, n, w) - 1;
        uint64_t r_lo = a.off[r], r_hi = a.off[r + 1];
        bool loaded = false, walk_l = false;
        uint32_t beg = 0, rroot = 0;
        int32_t x = 0, y = 0;
        for (int it = 0; it < kTriIters && w < total; ++it, w += 64) {
            if (w >= r_hi) {
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
                walk_l = (a.w[r] >> 31) != 0;
                beg = a.beg[r];
                x = a.root_x[r];
                y = a.root_y[r];
                rroot = a.root_rid[r];
                loaded = true;
            }
            const uint32_t e = beg + static_cast<uint32_t>(w - r_lo);
            uint32_t hc = 0;
            const int64_t sl = walk_l ? pair_slot_of(a.HP, pm, pair_key(x, a.L_z[e]), hc)
                                      : pair_slot_of(a.HL, lm, pair_key(y, a.P_z[e]), hc);
            if (sl < 0) continue;
            const uint32_t mine = walk_l ? a.L_rid[e] : a.P_rid[e];
            const uint32_t p0 = walk_l ? a.HP.pos[sl] : a.HL.pos[sl];
            const uint32_t *orid = walk_l ? a.P_rid : a.L_rid;
            for (uint32_t j = 0; j < hc; ++j) {
                const uint32_t other = orid[p0 + j];
                const uint32_t rr[3] = {rroot, walk_l ? other : mine, walk_l ? mine : other};
                emit_tuple<3>(o, cur++, rr);
            }
        }
    }
}

// The same member in the write pass: every row combination written from `cur`.
template <int W>
__device__ __forceinline__ void k4_member_emit(const K4Args &a, const CliqueOut &o, const K4Job &jb, uint32_t e,
                                               uint64_t &cur) {
    constexpr int H1 = W == 1 ? 3 : 1, H2 = W == 4 ? 3 : 4;
    const int32_t x1 = H1 == 3 ? jb.bv : jb.av, x2 = H2 == 3 ? jb.bv : jb.cv;
    const K4Group &g = a.g[W];
    const int32_t d = g.other[e];
    uint32_t cA = 0, cB = 0;
    const int64_t sA = pair_slot_of(a.h[H1], *a.h[H1].mask, pair_key(x1, d), cA);
    if (sA < 0) return;
    const int64_t sB = pair_slot_of(a.h[H2], *a.h[H2].mask, pair_key(x2, d), cB);
    if (sB < 0) return;
    // roles: 0 root, 1 ac, 2 ad, 3 bc, 4 bd, 5 cd; group / hash index h is role h + 1
    uint32_t rr[6] = {static_cast<uint32_t>(jb.f), 0, 0, 0, 0, 0};
    const uint32_t walked = static_cast<uint32_t>(jb.f >> 32);
    rr[W + 1] = g.rid[e];
    const uint32_t *l1_rid = jb.walk_bc ? a.g[0].rid : a.g[2].rid;
    const uint32_t pA = a.h[H1].pos[sA], pB = a.h[H2].pos[sB];
    for (uint32_t i1 = 0; i1 < jb.c1; ++i1) {
        const uint32_t r1 = l1_rid[jb.l1_pos + i1];
        rr[1] = jb.walk_bc ? r1 : walked;
        rr[3] = jb.walk_bc ? walked : r1;
        for (uint32_t iA = 0; iA < cA; ++iA) {
            rr[H1 + 1] = a.g[H1].rid[pA + iA];
            for (uint32_t iB = 0; iB < cB; ++iB) {
                rr[H2 + 1] = a.g[H2].rid[pB + iB];
                emit_tuple<6>(o, cur++, rr);
            }
        }
    }
}

template <int MODE>
__device__ __forceinline__ void k4_chunk(const K4Args &a, const CliqueOut *o, const uint32_t *gm, const uint32_t *hm,
                                         uint32_t n, uint64_t total, uint64_t c, K4Job *jobs, uint64_t *incl_s,
                                         uint64_t &acc0, uint64_t &acc1) {
    constexpr uint64_t kWaveSteps = 64ull * kTriIters;
    const uint32_t lane = static_cast<uint32_t>(lane_id());
    uint64_t w = c * kWaveSteps + lane;
    K4Cursor q{};
    if (w < total) {
        q.r = upper_bound_u64(a.off, 0, n, w) - 1;
        q.r_lo = a.off[q.r];
        q.r_hi = a.off[q.r + 1];
    }
    for (int it = 0; it < kTriIters; ++it, w += 64) {
        K4Job jb{};
        const bool hit = w < total && k4_first<MODE != 0>(a, gm, hm, n, w, q, jb);
        const uint64_t len = hit ? jb.wn : 0;
        const uint64_t incl = wave_incl_scan(len);
        const uint64_t T = __shfl(incl, 63, 64);
        if (T == 0) continue;   // the same for every lane of the wave
        jobs[lane] = jb;
        incl_s[lane] = incl;
        wave_lds_sync();
        for (uint64_t t = lane; t < T; t += 64) {
            const uint32_t i = k4_job_of(incl_s, t);
            const K4Job &j = jobs[i];
            const uint32_t e = j.wb + static_cast<uint32_t>(t - (incl_s[i] - j.wn));
            if (MODE == 0) {
                if (j.W == 1)
                    k4_member_count<1>(a, j, e, acc0, acc1);
                else if (j.W == 3)
                    k4_member_count<3>(a, j, e, acc0, acc1);
                else
                    k4_member_count<4>(a, j, e, acc0, acc1);
            } else {
                if (j.W == 1)
                    k4_member_emit<1>(a, *o, j, e, acc1);
                else if (j.W == 3)
                    k4_member_emit<3>(a, *o, j, e, acc1);
                else
                    k4_member_emit<4>(a, *o, j, e, acc1);
            }
        }
        wave_lds_sync();   // every lane is done with this round's jobs before they are replaced
    }
}

// The 4-clique write pass: the count pass's walk, balanced the same way (so each lane
// gets the members whose tuples the count pass counted for it), writing every row
// combination of each member from the lane's offset. A member's rows:
// the root row, the walked level-one row, the level-one pair's c1 rows, the walked
// group's row and the two looked-up pairs' rows.
__global__ __launch_bounds__(kTriThreads) void k_k4_emit(K4Args a, CliqueOut o) {
    __shared__ uint64_t s_tmp[kTriThreads / 64];
    __shared__ K4Job s_job[kTriThreads / 64][64];
    __shared__ uint64_t s_incl[kTriThreads / 64][64];
    const uint32_t n = *a.n_root;
    const uint64_t total = a.off[n];
    constexpr uint64_t kWaveSteps = 64ull * kTriIters;
    const uint64_t nchunks = (total + kWaveSteps - 1) / kWaveSteps;
    uint32_t gm[5], hm[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        gm[i] = *a.g[i].mask;
        hm[i] = *a.h[i].mask;
    }
    const uint32_t wid = threadIdx.x >> 6;
    uint64_t unused = 0, cur = emit_base(o, s_tmp);
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    for (uint64_t c = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; c < nchunks; c += nwaves)
        k4_chunk<1>(a, &o, gm, hm, n, total, c, s_job[wid], s_incl[wid], unused, cur);
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

hipError_t launch_k4_count(const K4Args &a, hipStream_t s) {
    TriArgs t{};   // the scan and the final sum read only these fields
    t.n_root = a.n_root;
    t.root_cap = a.root_cap;
    t.w = a.w;
    t.beg = a.beg;
    t.off = a.off;
    t.tile_sums = a.tile_sums;
    t.part = a.part;
    t.totals = a.totals;
    const uint32_t tiles = blocks_for(a.root_cap, kScanTile, kPersistentBlocks);
    hipLaunchKernelGGL(k_k4_rows, dim3(tiles), dim3(kScanBlock), 0, s, a);
    hipLaunchKernelGGL(k_tri_tiles, dim3(1), dim3(kScanBlock), 0, s, t);
    hipLaunchKernelGGL(k_tri_down, dim3(tiles), dim3(kScanBlock), 0, s, t);
    hipLaunchKernelGGL(k_k4_count, dim3(kTriBlocks), dim3(kTriThreads), 0, s, a);
    hipLaunchKernelGGL(k_tri_final, dim3(1), dim3(kTriThreads), 0, s, t, kTriBlocks);
    return hipGetLastError();
}

hipError_t launch_tri_emit(const TriArgs &a, const CliqueOut &o, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_emit, dim3(kTriBlocks), dim3(kTriThreads), 0, s, a, o);
    return hipGetLastError();
}

hipError_t launch_k4_emit(const K4Args &a, const CliqueOut &o, hipStream_t s) {
    hipLaunchKernelGGL(k_k4_emit, dim3(kTriBlocks), dim3(kTriThreads), 0, s, a, o);
    return hipGetLastError();
}

}  // namespace sj
