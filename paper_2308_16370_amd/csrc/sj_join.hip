// Enumeration-phase kernels.
//
// Each sieved non-root relation is regrouped by its parent-edge key ("buckets"):
// a stable LSD radix sort of (key, list index) keeps row ids ascending inside a
// bucket, a head-flag compaction gives the directory of distinct keys, and an
// open-addressed hash index maps a key to its directory entry. Bottom-up over the
// join tree, every entry gets the number of result tuples below it (a product over
// its children of the matching buckets' totals) and the matching checksum weight;
// exclusive prefix sums of both give the exact result size and checksum at the
// root and let each output index be decoded into its row-id tuple directly, with
// no intermediate result materialised.
#include <hip/hip_runtime.h>

#include "sj_device.h"
#include "sj_internal.h"

namespace sj {

static uint32_t grid_for(uint32_t n, uint32_t per_block, uint32_t cap) {
    uint32_t g = (n + per_block - 1) / per_block;
    if (g > cap) g = cap;
    return g ? g : 1;
}

// ================================================================ radix sort
// Keys are u32 bit patterns of int32 join keys (any fixed order groups equal keys);
// values are list indices. Pass p sorts on byte p of the key: bytes 0-3 of the low
// word, then bytes 0-3 of the high word for 2-word keys.

struct KeySrc {
    const int32_t *lo;         // list column of the low key word
    const int32_t *hi;         // list column of the high key word, or nullptr
};

__device__ __forceinline__ uint32_t radix_digit(uint32_t lo, uint32_t hi, int pass) {
    const uint32_t w = pass < 4 ? lo : hi;
    return (w >> ((pass & 3) * kRadixBits)) & (kRadixBins - 1);
}

__global__ __launch_bounds__(kRadixBlock) void k_radix_ghist(KeySrc ks, const uint32_t *n_ptr, uint32_t *ghist) {
    __shared__ uint32_t h[kRadixPasses][kRadixBins];
    const int np = ks.hi ? 8 : 4;
    for (int i = threadIdx.x; i < kRadixPasses * kRadixBins; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = *n_ptr;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const uint32_t lo = static_cast<uint32_t>(ks.lo[e]);
        const uint32_t hi = ks.hi ? static_cast<uint32_t>(ks.hi[e]) : 0u;
        for (int p = 0; p < np; ++p) atomicAdd(&h[p][radix_digit(lo, hi, p)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np * kRadixBins; i += blockDim.x) {
        const uint32_t c = (&h[0][0])[i];
        if (c) atomicAdd(ghist + i, c);
    }
}

// Pass control: ctl[p] = pass p moves data (its digit is not constant); ctl[8 + p] =
// where pass p reads (0: the list, 1: buffer 0, 2: buffer 1); ctl[16] = where the
// sorted data ends up. One thread per pass finds whether a bin holds every key.
// Also sizes the directory's hash index from the entry count (the distinct keys are at
// most that many): the smallest power of two above twice the entries, within the
// index's capacity, so the index is at most half full.
__global__ void k_radix_ctl(const uint32_t *ghist, const uint32_t *n_ptr, int npasses, uint32_t *ctl,
                            uint32_t *slot_mask, uint32_t slot_cap) {
    __shared__ uint32_t s_act[kRadixPasses];
    const uint32_t n = *n_ptr;
    if (threadIdx.x == 0) {
        uint32_t cap = 16;
        while (cap < 2u * n + 1u && cap < slot_cap) cap <<= 1;
        *slot_mask = (cap < slot_cap ? cap : slot_cap) - 1;
    }
    const int p = threadIdx.x >> 5, l = threadIdx.x & 31;   // 32 threads per pass
    uint32_t mx = 0;
    if (p < npasses)
        for (int d = l; d < kRadixBins; d += 32) mx = max(mx, ghist[p * kRadixBins + d]);
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), o, 32)));
    if (l == 0 && p < kRadixPasses) s_act[p] = (p < npasses && n > 1 && mx < n) ? 1u : 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t src = 0;
        for (int q = 0; q < kRadixPasses; ++q) {
            ctl[q] = s_act[q];
            ctl[8 + q] = src;
            if (s_act[q]) src = (src == 1) ? 2u : 1u;
        }
        ctl[16] = src;
    }
}

struct RadixIo {
    const uint32_t *slo, *shi, *sval;   // source (sval nullptr: the list index)
    uint32_t *dlo, *dhi, *dval;
};

__device__ __forceinline__ RadixIo radix_io(const SortScratch &ss, const KeySrc &ks, int pass) {
    const uint32_t src = ss.ctl[8 + pass];
    RadixIo io;
    io.slo = src == 0 ? reinterpret_cast<const uint32_t *>(ks.lo) : ss.klo[src - 1];
    io.shi = src == 0 ? reinterpret_cast<const uint32_t *>(ks.hi) : (ks.hi ? ss.khi[src - 1] : nullptr);
    io.sval = src == 0 ? nullptr : ss.vals[src - 1];
    const int d = (src == 1) ? 1 : 0;
    io.dlo = ss.klo[d];
    io.dhi = ks.hi ? ss.khi[d] : nullptr;
    io.dval = ss.vals[d];
    return io;
}

// Per-tile digit histogram, digit-major: hist[d * ntiles + tile].
__global__ __launch_bounds__(kRadixBlock) void k_radix_hist(int pass, KeySrc ks, SortScratch ss,
                                                            const uint32_t *n_ptr) {
    if (!ss.ctl[pass]) return;
    __shared__ uint32_t h[kRadixBins];
    const uint32_t n = *n_ptr;
    const uint32_t T = radix_tile(n);
    const int items = static_cast<int>(T / kRadixBlock);
    const uint32_t ntiles = (n + T - 1) / T;
    const RadixIo io = radix_io(ss, ks, pass);
    const uint32_t *w = pass < 4 ? io.slo : io.shi;
    const int shift = (pass & 3) * kRadixBits;
    for (uint32_t b = blockIdx.x; b < ntiles; b += gridDim.x) {
        const uint32_t tile = gridDim.x >= ntiles ? xcd_contiguous(b, ntiles) : b;
        h[threadIdx.x] = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kRadixItems; ++i) {
            const uint32_t e = tile * T + i * kRadixBlock + threadIdx.x;
            if (i < items && e < n) atomicAdd(&h[(w[e] >> shift) & (kRadixBins - 1)], 1u);
        }
        __syncthreads();
        ss.hist[threadIdx.x * ntiles + tile] = h[threadIdx.x];
        __syncthreads();
    }
}

// Exclusive scan in place of data[0 .. mul * ceil(n / div)), u32, decoupled look-back
// (div 0: the radix sort's tile for n entries).
__global__ __launch_bounds__(kScanBlock) void k_scan_u32(uint32_t *data, const uint32_t *n_ptr, uint32_t div,
                                                         uint32_t mul, const uint32_t *active, Lookback lb) {
    if (active && !*active) return;
    __shared__ uint32_t s_tile, s_base;
    __shared__ uint32_t s_wave[kScanBlock / 64];
    const uint32_t n = *n_ptr;
    const uint32_t d = div ? div : radix_tile(n);
    const uint32_t len = mul * ((n + d - 1) / d);
    const uint32_t ntiles = (len + kScanTile - 1) / kScanTile;
    while (true) {
        if (threadIdx.x == 0) s_tile = atomicAdd(lb.counter, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint32_t base = tile * kScanTile + threadIdx.x * kScanItems;
        uint32_t x[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            x[i] = (base + i < len) ? data[base + i] : 0u;
            sum += x[i];
        }
        uint32_t tot;
        uint32_t off = block_excl_scan<kScanBlock>(sum, s_wave, tot);
        if (threadIdx.x < 64) {
            const uint32_t b = lookback32_wave(lb.status, tile, tot);
            if (threadIdx.x == 0) s_base = b;
        }
        __syncthreads();
        off += s_base;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < len) data[base + i] = off;
            off += x[i];
        }
        __syncthreads();
    }
}

// Stable scatter of one radix pass. Items are striped (item i of thread t is element
// tile * kRadixTile + i * kRadixBlock + t), processed round by round, so element
// order equals (round, wave, lane) order; a lane's rank among equal digits comes from
// 8 ballots (the lanes sharing its digit), waves are ordered through LDS counts.
__global__ __launch_bounds__(kRadixBlock) void k_radix_scatter(int pass, KeySrc ks, SortScratch ss,
                                                               const uint32_t *n_ptr) {
    if (!ss.ctl[pass]) return;
    constexpr int kWaves = kRadixBlock / 64;
    __shared__ uint32_t s_off[kRadixBins];
    __shared__ uint32_t s_run[kRadixBins];
    __shared__ uint32_t s_cnt[kWaves][kRadixBins];
    const uint32_t n = *n_ptr;
    const uint32_t T = radix_tile(n);
    const int items = static_cast<int>(T / kRadixBlock);
    const uint32_t ntiles = (n + T - 1) / T;
    const RadixIo io = radix_io(ss, ks, pass);
    const int shift = (pass & 3) * kRadixBits;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint32_t b = blockIdx.x; b < ntiles; b += gridDim.x) {
        const uint32_t tile = gridDim.x >= ntiles ? xcd_contiguous(b, ntiles) : b;
        s_off[tid] = ss.hist[tid * ntiles + tile];
        s_run[tid] = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s_cnt[w][tid] = 0;
        __syncthreads();
        for (int i = 0; i < items; ++i) {
            const uint32_t e = tile * T + i * kRadixBlock + tid;
            const bool valid = e < n;
            const uint32_t klo = valid ? io.slo[e] : 0u;
            const uint32_t khi = (valid && io.shi) ? io.shi[e] : 0u;
            const uint32_t val = valid ? (io.sval ? io.sval[e] : e) : 0u;
            const uint32_t d = ((pass < 4 ? klo : khi) >> shift) & (kRadixBins - 1);
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            const uint32_t rank = __popcll(m & lt);
            if (valid && rank == 0) s_cnt[wid][d] = __popcll(m);
            __syncthreads();
            if (valid) {
                uint32_t pos = s_run[d] + rank;
                for (int w = 0; w < wid; ++w) pos += s_cnt[w][d];
                const uint32_t o = s_off[d] + pos;
                io.dlo[o] = klo;
                if (io.dhi) io.dhi[o] = khi;
                io.dval[o] = val;
            }
            __syncthreads();
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                t += s_cnt[w][tid];
                s_cnt[w][tid] = 0;
            }
            s_run[tid] += t;
            __syncthreads();
        }
    }
}

// Gather the list into bucket order.
struct ListRef {
    const uint32_t *rid;
    const int32_t *col[kMaxJCols];
    int ncol;
};

// Gather the list into bucket order, and clear the directory's hash index (sized by
// k_radix_ctl) for k_dir_heads, which fills it.
__global__ void k_gather(ListRef l, const uint32_t *n_ptr, SortScratch ss, Buckets b) {
    const uint32_t n = *n_ptr;
    const uint32_t fin = ss.ctl[16];
    const uint32_t *idx = fin == 0 ? nullptr : ss.vals[fin - 1];
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const uint32_t li = idx ? idx[e] : e;
        b.rid[e] = l.rid[li];
        for (int c = 0; c < l.ncol; ++c) b.col[c][e] = l.col[c][li];
    }
    const uint32_t lim = *b.slot_mask + 1u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < lim; i += gridDim.x * blockDim.x) b.slots[i] = 0;
}

// Directory: ordered compaction of the bucket heads (first entry of each key).
__global__ __launch_bounds__(kSieveBlock) void k_dir_heads(Buckets b, Lookback lb) {
    __shared__ uint32_t s_tile, s_base;
    __shared__ uint32_t s_wave[kSieveBlock / 64];
    const uint32_t n = *b.n;
    const int32_t *keys = b.col[b.key_jcol];
    const uint32_t ntiles = (n + kSieveTile - 1) / kSieveTile;
    while (true) {
        if (threadIdx.x == 0) s_tile = atomicAdd(lb.counter, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint32_t e0 = tile * kSieveTile + threadIdx.x * kSieveItems;
        uint32_t flags = 0;
        int32_t kv[kSieveItems];
        int32_t prev = (e0 > 0 && e0 <= n) ? keys[e0 - 1] : 0;
#pragma unroll
        for (int i = 0; i < kSieveItems; ++i) {
            const uint32_t e = e0 + i;
            kv[i] = e < n ? keys[e] : 0;
            const bool head = e < n && (e == 0 || kv[i] != prev);
            flags |= (head ? 1u : 0u) << i;
            prev = kv[i];
        }
        uint32_t tot;
        const uint32_t off = block_excl_scan<kSieveBlock>(static_cast<uint32_t>(__builtin_popcount(flags)), s_wave, tot);
        if (threadIdx.x < 64) {
            const uint32_t b = lookback32_wave(lb.status, tile, tot);
            if (threadIdx.x == 0) s_base = b;
        }
        __syncthreads();
        uint32_t o = s_base + off;
        const uint32_t mask = *b.slot_mask;
#pragma unroll
        for (int i = 0; i < kSieveItems; ++i) {
            if (flags & (1u << i)) {
                b.dir_begin[o] = e0 + i;
                b.dir_key[o] = kv[i];
                // the key's hash slot (the index was cleared by k_gather and is at most half full)
                const uint64_t val = (static_cast<uint64_t>(o + 1) << 32) | static_cast<uint32_t>(kv[i]);
                uint32_t sl = slot_hash(kv[i]) & mask;
                while (atomicCAS(reinterpret_cast<unsigned long long *>(b.slots + sl), 0ull,
                                 static_cast<unsigned long long>(val)) != 0ull)
                    sl = (sl + 1) & mask;
                ++o;
            }
        }
        if (tile == ntiles - 1 && threadIdx.x == 0) {
            *b.ndir = s_base + tot;
            b.dir_begin[s_base + tot] = n;
        }
        __syncthreads();
    }
}

__global__ void k_dir_mask(Buckets b) {
    if (threadIdx.x != 0) return;
    const uint32_t nd = *b.ndir;
    uint32_t cap = 16;
    while (cap < 2u * nd + 1u) cap <<= 1;
    if (cap > b.slot_cap) cap = b.slot_cap;
    *b.slot_mask = cap - 1;
}

__global__ void k_slots_clear(Buckets b) {
    const uint32_t lim = *b.slot_mask + 1u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < lim; i += gridDim.x * blockDim.x) b.slots[i] = 0;
}

hipError_t launch_build_buckets(const uint32_t *list_rid, const int32_t *const *list_cols, int ncol,
                                const uint32_t *list_count, int key_col, int sec_col, const Buckets &b,
                                const SortScratch &ss, Lookback lb_dir, hipStream_t s) {
    const uint32_t cap = b.cap;
    if (cap == 0) {
        // no rows: an empty directory still needs a valid (cleared) hash index
        hipLaunchKernelGGL(k_dir_mask, dim3(1), dim3(64), 0, s, b);
        hipLaunchKernelGGL(k_slots_clear, dim3(1), dim3(256), 0, s, b);
        return hipGetLastError();
    }
    KeySrc ks;
    ks.lo = list_cols[sec_col >= 0 ? sec_col : key_col];
    ks.hi = sec_col >= 0 ? list_cols[key_col] : nullptr;
    const int npasses = sec_col >= 0 ? 8 : 4;
    const uint32_t tiles = radix_tiles_max(cap);
    const uint32_t tgrid = tiles < kPersistentBlocks ? tiles : kPersistentBlocks;
    // few workgroups: every workgroup adds its histogram to the same 256 x passes counters
    hipLaunchKernelGGL(k_radix_ghist, dim3(grid_for(cap, 256 * 16, 128)), dim3(kRadixBlock), 0, s, ks,
                       list_count, ss.ghist);
    hipLaunchKernelGGL(k_radix_ctl, dim3(1), dim3(256), 0, s, ss.ghist, list_count, npasses, ss.ctl, b.slot_mask,
                       b.slot_cap);
    const uint32_t scan_len_max = kRadixBins * tiles;
    const uint32_t scan_grid = grid_for(scan_len_max, kScanTile, 256);
    for (int p = 0; p < npasses; ++p) {
        hipLaunchKernelGGL(k_radix_hist, dim3(tgrid), dim3(kRadixBlock), 0, s, p, ks, ss, list_count);
        hipLaunchKernelGGL(k_scan_u32, dim3(scan_grid), dim3(kScanBlock), 0, s, ss.hist, list_count, 0u,
                           static_cast<uint32_t>(kRadixBins), ss.ctl + p, ss.lb[p]);
        hipLaunchKernelGGL(k_radix_scatter, dim3(tgrid), dim3(kRadixBlock), 0, s, p, ks, ss, list_count);
    }
    ListRef l;
    l.rid = list_rid;
    l.ncol = ncol;
    for (int c = 0; c < kMaxJCols; ++c) l.col[c] = c < ncol ? list_cols[c] : nullptr;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(cap > b.slot_cap / 2 ? cap : b.slot_cap / 2, 256 * 4, 4096)), dim3(256),
                       0, s, l, list_count, ss, b);
    const uint32_t dgrid = grid_for(cap, kSieveTile, 256);   // each workgroup claims tiles from one counter
    hipLaunchKernelGGL(k_dir_heads, dim3(dgrid), dim3(kSieveBlock), 0, s, b, lb_dir);
    return hipGetLastError();
}

// ================================================================ DP weights
// w(e) = prod over children c of W_c(key_c(e)), v(e) = f(rel, rid(e)) * prod V_c(...),
// with W_c / V_c the totals of the child's bucket for that key (0 if absent).
//
// A thread holds ITEMS entries and looks them up in CH = kDpSlots / ITEMS children at
// once, so every lookup stage (key, hash slot, directory bounds, child prefix weights)
// has up to kDpSlots independent loads in flight and the dependent chain is four stages
// per group of CH children. A relation with one child takes 2 entries per thread; one
// with more children 1 entry of all its children (dp_items): small tiles keep every CU
// busy on the relations of a few hundred thousand entries a sieve leaves. A slot that holds
// another key (rare: the index is at most half full) is resolved by linear probing. A
// thread's entries are kScanBlock apart (entry tile * tile size + i * kScanBlock +
// thread), so the loads of one stage are consecutive across a wave; only the tile's
// total is scanned here.
template <int ITEMS>
__device__ __forceinline__ void dp_entries(const DpArgs &a, const uint32_t *masks, uint32_t base, uint32_t n,
                                           uint64_t *w, uint64_t *v) {
    constexpr int CH = kDpSlots / ITEMS;
    static_assert(kMaxJCols % CH == 0, "child groups tile the child slots");
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = base + i * kScanBlock;
        w[i] = 1;
        v[i] = e < n ? chk_factor(a.rel, a.rid[e]) : 0;
    }
#pragma unroll
    for (int c0 = 0; c0 < kMaxJCols; c0 += CH) {
        if (c0 < a.nchild) {
            int32_t key[CH][ITEMS];
            uint32_t sl[CH][ITEMS];
            uint64_t sv[CH][ITEMS];
            uint32_t lo[CH][ITEMS], hi[CH][ITEMS];
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = c0 + cc;
                const int32_t *col = a.col[a.child_col[c]];
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t e = base + i * kScanBlock;
                    key[cc][i] = (c < a.nchild && e < n) ? col[e] : 0;
                }
            }
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = c0 + cc;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    sl[cc][i] = 0;
                    sv[cc][i] = 0;
                    if (c < a.nchild) {
                        sl[cc][i] = slot_hash(key[cc][i]) & masks[c];
                        sv[cc][i] = a.child[c].slots[sl[cc][i]];
                    }
                }
            }
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = c0 + cc;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    lo[cc][i] = 0;
                    hi[cc][i] = 0;
                    if (c < a.nchild) {
                        while (sv[cc][i] != 0 && static_cast<uint32_t>(sv[cc][i]) != static_cast<uint32_t>(key[cc][i])) {
                            sl[cc][i] = (sl[cc][i] + 1) & masks[c];
                            sv[cc][i] = a.child[c].slots[sl[cc][i]];
                        }
                        const uint32_t d = static_cast<uint32_t>(sv[cc][i] >> 32);   // directory index + 1, 0: absent
                        lo[cc][i] = d ? a.child[c].dir_begin[d - 1] : 0u;
                        hi[cc][i] = d ? a.child[c].dir_begin[d] : 0u;
                    }
                }
            }
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = c0 + cc;
                if (c < a.nchild) {
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) {
                        const uint32_t e = base + i * kScanBlock;
                        if (e < n) {
                            a.blo[c][e] = lo[cc][i];
                            a.bhi[c][e] = hi[cc][i];
                        }
                    }
                }
            }
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = c0 + cc;
                if (c < a.nchild && !(a.skip_mask & (1u << c))) {
                    const uint64_t *cw = a.child[c].cw, *cv = a.child[c].cv;
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) {
                        w[i] *= cw[hi[cc][i]] - cw[lo[cc][i]];
                        v[i] *= cv[hi[cc][i]] - cv[lo[cc][i]];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (base + i * kScanBlock >= n) w[i] = v[i] = 0;
}

// Two launches. Workgroup b of the grid owns a contiguous run of tiles. (1) k_dp_reduce
// writes every entry's weights into cw/cv (not yet scanned) and the run's sums into
// tile_sums[2b], [2b + 1]. (2) k_dp_down adds the sums of the runs before its own (at
// most the grid size of them, read by the whole workgroup) and scans its run tile by
// tile; the last workgroup writes the totals at cw[n], cv[n].
__device__ __forceinline__ void dp_run(uint32_t ntiles, uint32_t &t0, uint32_t &t1) {
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    t0 = min(ntiles, blockIdx.x * per);
    t1 = min(ntiles, t0 + per);
}

template <int ITEMS>
__global__ __launch_bounds__(kScanBlock) void k_dp_reduce(DpArgs a) {
    constexpr uint32_t T = kScanBlock * ITEMS;
    __shared__ uint64_t s_w[kScanBlock / 64], s_v[kScanBlock / 64];
    const uint32_t n = *a.n;
    uint32_t t0, t1;
    dp_run((n + T - 1) / T, t0, t1);
    uint32_t masks[kMaxJCols];
#pragma unroll
    for (int c = 0; c < kMaxJCols; ++c) masks[c] = c < a.nchild ? *a.child[c].slot_mask : 0u;
    uint64_t sw = 0, sv = 0;
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t base = tile * T + threadIdx.x;
        uint64_t w[ITEMS], v[ITEMS];
        dp_entries<ITEMS>(a, masks, base, n, w, v);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (base + i * kScanBlock < n) {
                a.cw[base + i * kScanBlock] = w[i];
                a.cv[base + i * kScanBlock] = v[i];
            }
            sw += w[i];
            sv += v[i];
        }
    }
    uint64_t tw, tv;
    block_excl_scan<kScanBlock>(sw, s_w, tw);
    block_excl_scan<kScanBlock>(sv, s_v, tv);
    if (threadIdx.x == 0) {
        a.tile_sums[2 * blockIdx.x] = tw;
        a.tile_sums[2 * blockIdx.x + 1] = tv;
    }
}

// Per-entry weights into exclusive prefixes, run by run.
template <int ITEMS>
__global__ __launch_bounds__(kScanBlock) void k_dp_down(DpArgs a) {
    constexpr uint32_t T = kScanBlock * ITEMS;
    __shared__ uint64_t s_w[kScanBlock / 64], s_v[kScanBlock / 64];
    const uint32_t n = *a.n;
    uint32_t t0, t1;
    dp_run((n + T - 1) / T, t0, t1);
    uint64_t pw = 0, pv = 0;   // sums of the runs before this one
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kScanBlock) {
        pw += a.tile_sums[2 * b];
        pv += a.tile_sums[2 * b + 1];
    }
    uint64_t cw0, cv0;
    block_excl_scan<kScanBlock>(pw, s_w, cw0);
    block_excl_scan<kScanBlock>(pv, s_v, cv0);
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t base = tile * T + threadIdx.x * ITEMS;
        uint64_t w[ITEMS], v[ITEMS];
        uint64_t sw = 0, sv = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = base + i;
            w[i] = e < n ? a.cw[e] : 0;
            v[i] = e < n ? a.cv[e] : 0;
            sw += w[i];
            sv += v[i];
        }
        uint64_t tw, tv;
        uint64_t ow = block_excl_scan<kScanBlock>(sw, s_w, tw) + cw0;
        uint64_t ov = block_excl_scan<kScanBlock>(sv, s_v, tv) + cv0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = base + i;
            if (e < n) {
                a.cw[e] = ow;
                a.cv[e] = ov;
            }
            ow += w[i];
            ov += v[i];
        }
        cw0 += tw;
        cv0 += tv;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        // every run before this one, and its own: the totals (runs past the last tile are empty)
        a.cw[n] = cw0;
        a.cv[n] = cv0;
        if (a.totals) {
            a.totals[0] = cw0;
            a.totals[1] = cv0;
        }
    }
}

template <int ITEMS>
static void launch_dp_items(const DpArgs &a, hipStream_t s) {
    const uint32_t T = kScanBlock * ITEMS;
    const uint32_t tiles = (a.cap + T - 1) / T;
    const uint32_t g = tiles == 0 ? 1 : (tiles < kPersistentBlocks ? tiles : kPersistentBlocks);
    hipLaunchKernelGGL(k_dp_reduce<ITEMS>, dim3(g), dim3(kScanBlock), 0, s, a);
    hipLaunchKernelGGL(k_dp_down<ITEMS>, dim3(g), dim3(kScanBlock), 0, s, a);
}

hipError_t launch_dp(const DpArgs &a, hipStream_t s) {
    if (a.nchild < 0 || a.nchild > kMaxJCols) return hipErrorInvalidValue;
    switch (dp_items(a.nchild)) {
    case 2: launch_dp_items<2>(a, s); break;
    default: launch_dp_items<1>(a, s); break;
    }
    return hipGetLastError();
}

// ================================================================ materialise
// Output index o decodes into one tuple: the root entry r with cw_root[r] <= o <
// cw_root[r + 1], then, down the tree in preorder, the local index is split over a
// node's children as a mixed-radix number (first child most significant) and
// inside a child's bucket the entry whose prefix range holds it. A thread decodes
// the first index of its chunk and then steps an odometer (last preorder position
// fastest), which visits tuples in the same lexicographic order.

// Odometer state. Every array is indexed by compile-time positions only (the tree's
// shape is a run-time argument, so parent links are followed by per-position tests
// rather than by indexing), which keeps the state in registers.
template <int N>
struct MatState {
    uint32_t e[N];     // current entry of each position
    uint32_t lo[N];    // bucket of each position below its parent's current entry
    uint32_t hi[N];
    uint32_t pe[N];    // current entry of each position's parent
};

template <int N>
__device__ __forceinline__ void set_entry(const MatArgs &a, MatState<N> &st, int x, uint32_t v) {
    st.e[x] = v;
#pragma unroll
    for (int y = 1; y < N; ++y)
        if (y > x && a.parent_pos[y] == x) st.pe[y] = v;
}

// Bucket of position y below its parent's current entry.
template <int N>
__device__ __forceinline__ void find_bucket(const MatArgs &a, MatState<N> &st, int y) {
    st.lo[y] = a.blo[y][st.pe[y]];
    st.hi[y] = a.bhi[y][st.pe[y]];
}

// First entry at or after e (below hi) with a nonzero weight; leaves weigh 1 each.
__device__ __forceinline__ uint32_t first_valid(const MatArgs &a, int y, uint32_t e, uint32_t hi) {
    if (a.is_leaf[y]) return e;
    const uint64_t *cw = a.cw[y];
    while (e < hi && cw[e + 1] == cw[e]) ++e;
    return e;
}

template <int N>
__device__ void mat_decode(const MatArgs &a, MatState<N> &st, uint32_t r, uint64_t L0) {
    uint64_t L[N];
#pragma unroll
    for (int p = 0; p < N; ++p) L[p] = 0;
    set_entry<N>(a, st, 0, r);
    L[0] = L0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        if (p > 0) {
            // the entry of position p inside its bucket that holds local index L[p]
            uint32_t e;
            if (a.is_leaf[p]) {
                e = st.lo[p] + static_cast<uint32_t>(L[p]);
                L[p] = 0;
            } else {
                const uint64_t *cw = a.cw[p];
                const uint64_t base = cw[st.lo[p]];
                e = upper_bound_u64(cw, st.lo[p], st.hi[p] + 1, base + L[p]) - 1;
                L[p] -= cw[e] - base;
            }
            set_entry<N>(a, st, p, e);
        }
        // split L[p] over p's children, last child least significant
#pragma unroll
        for (int c = N - 1; c > p; --c) {
            if (a.parent_pos[c] == p) {
                find_bucket<N>(a, st, c);
                if (a.nchild[p] == 1) {
                    L[c] = L[p];
                } else {
                    const uint64_t W = a.is_leaf[c] ? static_cast<uint64_t>(st.hi[c] - st.lo[c])
                                                    : a.cw[c][st.hi[c]] - a.cw[c][st.lo[c]];
                    L[c] = L[p] % W;
                    L[p] /= W;
                }
            }
        }
    }
}

template <int N>
__device__ __forceinline__ void mat_advance(const MatArgs &a, MatState<N> &st, uint32_t root_n) {
    int changed = -1;
#pragma unroll
    for (int x = N - 1; x >= 1; --x) {
        if (changed < 0) {
            const uint32_t nx = first_valid(a, x, st.e[x] + 1, st.hi[x]);
            if (nx < st.hi[x]) {
                set_entry<N>(a, st, x, nx);
                changed = x;
            }
        }
    }
    if (changed < 0) {
        const uint64_t *cw = a.cw[0];
        uint32_t r = st.e[0] + 1;
        while (r < root_n && cw[r + 1] == cw[r]) ++r;
        set_entry<N>(a, st, 0, r);
        changed = 0;
    }
#pragma unroll
    for (int y = 1; y < N; ++y) {
        if (y > changed) {
            if (a.parent_pos[y] >= changed) find_bucket<N>(a, st, y);
            set_entry<N>(a, st, y, first_valid(a, y, st.lo[y], st.hi[y]));
        }
    }
}

// Whether every table of the factorised materialisation fits its scratch (the same
// answer in every launch that asks).
template <int N>
__device__ bool mat_tables_fit(const MatArgs &a) {
    bool ok = true;
#pragma unroll
    for (int x = 1; x < N; ++x) {
        if (a.tab[x]) {
            // rows are addressed with 32-bit bases, and the table must fit its scratch
            const uint64_t rows = a.cw[x][*a.n_ent[x]];
            if (rows >= (1ull << 32) || rows * static_cast<uint64_t>(a.subtree[x]) > a.tab_words[x]) ok = false;
        }
    }
    return ok;
}

// Blocks of a materialisation whose count is read on the device (a grid-stride loop
// over the output covers the rest).
constexpr uint64_t kMatPersistentBlocks = 4096;
constexpr uint64_t kMatFallbackBlocks = 512;

// Tuples per thread: a thread's C tuples of N entries take at most 16 words of LDS.
template <int N>
constexpr int mat_chunk() {
    return N <= 2 ? 8 : (16 / N > 0 ? 16 / N : 1);
}

// A block owns the outputs [t0, t1) = 256 * C consecutive indices; thread t decodes
// the first index of its chunk and steps the odometer through the rest. The root
// entries covering the block are located once and their prefix weights staged in LDS,
// so each thread's root search runs in LDS. The odometer writes each tuple's entry
// indices into an LDS tile (row pitch C * N + 1 words, so the threads' rows fall in
// distinct banks); a leaf step then needs no memory access. The copy-out turns
// entries into row ids with independent gathers and writes the tile with coalesced
// 16-byte stores.
//
// VAL: the copy-out writes projected values instead of row ids (a.proj.n columns per
// tuple): output column q reads relation a.proj.rel[q]'s entry from the tile, its row
// id, then that row's value in column a.proj.col[q].
template <int N, bool VAL>
__global__ __launch_bounds__(256) void k_materialize(MatArgs a) {
    constexpr int C = mat_chunk<N>();
    constexpr uint32_t ROW = C * N, PITCH = ROW + 1;
    constexpr uint32_t PER = 256u * C;
    constexpr uint32_t WIN = PER + 2;
    __shared__ uint64_t s_cw[WIN];
    __shared__ uint32_t s_out[256 * PITCH];
    __shared__ uint32_t s_r[2];
    __shared__ const uint32_t *s_rid[N];   // row ids of output column q's position
    __shared__ const int32_t *s_pcol[VAL ? kMaxProj : 1];
    __shared__ uint32_t s_prel[VAL ? kMaxProj : 1];
    const uint64_t count = a.count_dev ? *a.count_dev : a.count;
    if (count > a.capacity) return;         // the caller's buffer is too small: write nothing
    if (a.fact && mat_tables_fit<N>(a)) return;   // the factorised launches wrote the output
    const uint32_t root_n = *a.root_n;
    const uint64_t *rcw = a.cw[0];
    if (threadIdx.x == 64) {
#pragma unroll
        for (int x = 0; x < N; ++x) s_rid[a.order[x]] = a.rid[x];
    }
    if constexpr (VAL) {
        if (threadIdx.x < static_cast<uint32_t>(a.proj.n)) {
            s_pcol[threadIdx.x] = a.proj.col[threadIdx.x];
            s_prel[threadIdx.x] = static_cast<uint32_t>(a.proj.rel[threadIdx.x]);
        }
    }
    for (uint64_t blk = blockIdx.x; blk * PER < count; blk += gridDim.x) {
        const uint64_t t0 = blk * PER;
        const uint64_t t1 = (t0 + PER < count) ? t0 + PER : count;
        if (threadIdx.x < 128) {   // wave 0 finds the root entry of t0, wave 1 that of t1 - 1
            const int wv = threadIdx.x >> 6;
            const uint32_t r = wave_upper_bound_u64(rcw, 0, root_n + 1, wv == 0 ? t0 : t1 - 1) - 1;
            if (lane_id() == 0) s_r[wv] = r;
        }
        __syncthreads();
        const uint32_t r0 = s_r[0], r1 = s_r[1];
        const bool in_lds = r1 - r0 + 2 <= WIN;   // zero-weight root entries can widen the range
        if (in_lds)
            for (uint32_t i = threadIdx.x; i < r1 - r0 + 2; i += 256) s_cw[i] = rcw[r0 + i];
        __syncthreads();
        const uint64_t o0 = t0 + static_cast<uint64_t>(threadIdx.x) * C;
        if (o0 < t1) {
            uint32_t r;
            uint64_t L0;
            if (in_lds) {
                r = r0 + upper_bound_u64(s_cw, 0, r1 - r0 + 2, o0) - 1;
                L0 = o0 - s_cw[r - r0];
            } else {
                r = upper_bound_u64(rcw, r0, r1 + 2, o0) - 1;
                L0 = o0 - rcw[r];
            }
            MatState<N> st;
            mat_decode<N>(a, st, r, L0);
            const uint32_t nloc = static_cast<uint32_t>(min(static_cast<uint64_t>(C), t1 - o0));
            uint32_t *row = s_out + threadIdx.x * PITCH;
            for (uint32_t i = 0;;) {
    #pragma unroll
                for (int x = 0; x < N; ++x) row[i * N + a.order[x]] = st.e[x];
                if (++i >= nloc) break;
                mat_advance<N>(a, st, root_n);
            }
        }
        __syncthreads();
        // word w of the block's output is word w % ROW of thread w / ROW's row
        const uint32_t W = VAL ? static_cast<uint32_t>(a.proj.n) : N;   // output words per tuple
        const uint64_t words = (t1 - t0) * W;
        int32_t *dst = a.out + t0 * W;
        for (uint32_t w = threadIdx.x * 4; w < words; w += 256 * 4) {
            int32_t v[4];
    #pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t ww = w + j;
                if constexpr (VAL) {
                    if (ww < words) {
                        const uint32_t t = ww / W, q = ww - t * W, rel = s_prel[q];
                        const uint32_t rid = s_rid[rel][s_out[(t / C) * PITCH + (t % C) * N + rel]];
                        v[j] = s_pcol[q][rid];
                    } else {
                        v[j] = 0;
                    }
                } else {
                    v[j] = ww < words ? static_cast<int32_t>(s_rid[ww % N][s_out[(ww / ROW) * PITCH + ww % ROW]])
                                      : 0;
                }
            }
            if (w + 4 <= words) {
                *reinterpret_cast<int4 *>(dst + w) = make_int4(v[0], v[1], v[2], v[3]);
            } else {
                for (uint32_t j = 0; w + j < words; ++j) dst[w + j] = v[j];
            }
        }
        __syncthreads();   // s_r, s_cw and s_out are reused by the next block of output
    }
}

hipError_t launch_materialize(const MatArgs &a, hipStream_t s) {
    uint32_t per = 0;
    switch (a.nrels) {
#define SJ_MAT_PER(NN) \
    case NN: per = 256u * mat_chunk<NN>(); break;
        SJ_MAT_PER(1) SJ_MAT_PER(2) SJ_MAT_PER(3) SJ_MAT_PER(4) SJ_MAT_PER(5) SJ_MAT_PER(6) SJ_MAT_PER(7)
        SJ_MAT_PER(8) SJ_MAT_PER(9) SJ_MAT_PER(10) SJ_MAT_PER(11) SJ_MAT_PER(12) SJ_MAT_PER(13)
        SJ_MAT_PER(14) SJ_MAT_PER(15) SJ_MAT_PER(16)
#undef SJ_MAT_PER
        default: return hipErrorInvalidValue;
    }
    const uint64_t tuples = a.count_dev ? a.capacity : min(a.count, a.capacity);
    if (tuples == 0) return hipSuccess;
    uint64_t blocks64 = (tuples + per - 1) / per;
    if (a.count_dev && blocks64 > kMatPersistentBlocks) blocks64 = kMatPersistentBlocks;
    // after the factorised launches this decode writes only if a table did not fit:
    // a small grid (the loop over the output covers the rest) keeps its launch short
    if (a.fact && blocks64 > kMatFallbackBlocks) blocks64 = kMatFallbackBlocks;
    if (blocks64 > 0x7fffffffull) return hipErrorInvalidValue;
    const dim3 g(static_cast<uint32_t>(blocks64));
    if (a.proj.n < 0 || a.proj.n > kMaxProj) return hipErrorInvalidValue;
    const bool val = a.proj.n > 0;
    switch (a.nrels) {
#define SJ_MAT_CASE(NN)                                                               \
    case NN:                                                                          \
        if (val)                                                                      \
            hipLaunchKernelGGL((k_materialize<NN, true>), g, dim3(256), 0, s, a);     \
        else                                                                          \
            hipLaunchKernelGGL((k_materialize<NN, false>), g, dim3(256), 0, s, a);    \
        break;
        SJ_MAT_CASE(1) SJ_MAT_CASE(2) SJ_MAT_CASE(3) SJ_MAT_CASE(4) SJ_MAT_CASE(5) SJ_MAT_CASE(6) SJ_MAT_CASE(7)
        SJ_MAT_CASE(8) SJ_MAT_CASE(9) SJ_MAT_CASE(10) SJ_MAT_CASE(11) SJ_MAT_CASE(12) SJ_MAT_CASE(13)
        SJ_MAT_CASE(14) SJ_MAT_CASE(15) SJ_MAT_CASE(16)
#undef SJ_MAT_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ================================================================ factorised materialisation
// The tuples below an entry e of position x are e's row id followed by, for each child
// of x, the tuples below the child's bucket for e, combined as a mixed-radix number
// (last child least significant). They depend on e alone, not on the parent entry that
// reached it, so for each non-root position with children they are written once into a
// table (entry e's rows at rows cw[x][e] .., a row holding the subtree's row ids in
// preorder), deepest positions first. The output, like each table, is then a one-level
// expansion: row o finds its entry e (the last with cw[e] <= o, searched in an LDS
// window of the block's entries), and each child's part of the row is one row of the
// child's table (a row id for a leaf) at the bucket's first prefix weight plus the
// child's digit of o - cw[e]. A wave's lanes take consecutive rows, so the table reads
// and the output writes are contiguous across the wave. Zipf-skewed chains repeat the
// same heavy buckets below many parent entries; their tuples are read from a table
// instead of being decoded again for every parent entry.
//
// A table takes its relation's sort scratch, which the join phase no longer needs.
// Every launch checks that every table fits (the same answer in each); if one does
// not, none is built and launch_materialize decodes the output instead.

constexpr int kExpandC = 4;                         // rows per lane
constexpr uint32_t kExpandPer = 256u * kExpandC;    // rows per block
constexpr uint32_t kExpandWin = kExpandPer + 2;     // entries a block's LDS window holds
static_assert(kExpandPer == 256u * 4u, "the row -> entry scan gives each thread four rows");

// Expansion of position p (the output when OUT, p = 0; else p's table). NCH bounds the
// children of p (LDS arrays); VAL writes projected values instead of row ids.
//
// A block owns kExpandPer consecutive rows. Its entries' prefix weights, row ids and
// children's bucket bases (and bucket weights, for several children) are staged in LDS;
// a row -> entry map of the block is filled by marking each entry's first row and a
// block-wide maximum scan, so a row's entry is one LDS read. Lane l of a wave takes
// rows l, l + 64, l + 128, l + 192 of the wave's 256, and issues the table reads of all
// four before it writes any.
template <int N, int NCH, bool OUT, bool VAL>
__global__ __launch_bounds__(256) void k_mat_expand(MatArgs a, int p) {
    __shared__ uint64_t s_cw[kExpandWin];
    __shared__ uint32_t s_rid[kExpandWin];
    __shared__ uint32_t s_base[NCH][kExpandWin];
    __shared__ uint32_t s_w[NCH > 1 ? NCH : 1][NCH > 1 ? kExpandWin : 1];
    __shared__ uint32_t s_ent[kExpandPer];
    __shared__ uint32_t s_wave[256 / 64];
    __shared__ uint32_t s_r[2];
    __shared__ int s_ok;
    if (threadIdx.x == 0) s_ok = mat_tables_fit<N>(a) ? 1 : 0;
    __syncthreads();
    if (!s_ok) return;
    uint64_t rows;
    if constexpr (OUT) {
        rows = a.count_dev ? *a.count_dev : a.count;
        if (rows > a.capacity) return;      // the caller's buffer is too small: write nothing
    } else {
        rows = a.cw[p][*a.n_ent[p]];
    }
    const uint32_t n_p = *a.n_ent[p];
    const uint64_t *cw = a.cw[p];
    const uint32_t *rid = a.rid[p];
    const uint32_t S = OUT ? 0u : static_cast<uint32_t>(a.subtree[p]);
    uint32_t *tab_p = OUT ? nullptr : a.tab[p];
    // p's children in position order: slot k of the LDS arrays
    int nch = 0;
    int cpos[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k) cpos[k] = N;
#pragma unroll
    for (int c = 1; c < N; ++c) {
        if (c > p && a.parent_pos[c] == p) {
#pragma unroll
            for (int k = 0; k < NCH; ++k)
                if (k == nch) cpos[k] = c;
            ++nch;
        }
    }
    const int lane = lane_id();
    const uint32_t wrow = (threadIdx.x >> 6) * 64u * kExpandC;   // the wave's first row in the block
    for (uint64_t blk = blockIdx.x; blk * kExpandPer < rows; blk += gridDim.x) {
        const uint64_t t0 = blk * kExpandPer;
        const uint64_t t1 = (t0 + kExpandPer < rows) ? t0 + kExpandPer : rows;
        if (threadIdx.x < 128) {   // wave 0 finds the entry of t0, wave 1 that of t1 - 1
            const int wv = threadIdx.x >> 6;
            const uint32_t r = wave_upper_bound_u64(cw, 0, n_p + 1, wv == 0 ? t0 : t1 - 1) - 1;
            if (lane == 0) s_r[wv] = r;
        }
        for (uint32_t j = threadIdx.x; j < kExpandPer; j += 256) s_ent[j] = 0;
        __syncthreads();
        const uint32_t r0 = s_r[0], r1 = s_r[1];
        const uint32_t ne = r1 - r0 + 1;           // entries of the block's rows
        const bool in_lds = ne + 1 <= kExpandWin;  // zero-weight entries can widen the range
        if (in_lds) {
            for (uint32_t i = threadIdx.x; i <= ne; i += 256) {
                const uint64_t c0 = cw[r0 + i];
                s_cw[i] = c0;
                // entry i's first row (later entries of equal start have zero weight before it)
                if (i > 0 && i < ne && c0 < t1) atomicMax(&s_ent[c0 - t0], i);
                if (i < ne) {
                    const uint32_t e = r0 + i;
                    s_rid[i] = rid[e];
#pragma unroll
                    for (int k = 0; k < NCH; ++k) {
                        if (k < nch) {
                            const int c = cpos[k];
                            const uint32_t lo = a.blo[c][e];
                            if (a.is_leaf[c]) {
                                s_base[k][i] = lo;
                                if constexpr (NCH > 1) s_w[k][i] = a.bhi[c][e] - lo;
                            } else {
                                const uint64_t b = a.cw[c][lo];
                                s_base[k][i] = static_cast<uint32_t>(b);
                                if constexpr (NCH > 1) s_w[k][i] = static_cast<uint32_t>(a.cw[c][a.bhi[c][e]] - b);
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // row -> entry: the running maximum of the marks (thread t holds rows 4t .. 4t + 3)
            uint32_t m[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) m[q] = s_ent[threadIdx.x * 4 + q];
#pragma unroll
            for (int q = 1; q < 4; ++q) m[q] = max(m[q], m[q - 1]);
            uint32_t x = m[3];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(x, d, 64);
                if (lane >= d) x = max(x, y);
            }
            if (lane == 63) s_wave[threadIdx.x >> 6] = x;
            uint32_t before = __shfl_up(x, 1, 64);
            if (lane == 0) before = 0;
            __syncthreads();
#pragma unroll
            for (int w = 0; w < 256 / 64; ++w)
                if (w < static_cast<int>(threadIdx.x >> 6)) before = max(before, s_wave[w]);
#pragma unroll
            for (int q = 0; q < 4; ++q) s_ent[threadIdx.x * 4 + q] = max(m[q], before);
        }
        __syncthreads();
        // the lane's rows: entry, local index, and the children's rows
        uint32_t wv[kExpandC][N];
        uint64_t orow[kExpandC];
        bool live[kExpandC];
#pragma unroll
        for (int i = 0; i < kExpandC; ++i) {
            const uint64_t o = t0 + wrow + lane + 64u * i;
            orow[i] = o;
            live[i] = o < t1;
#pragma unroll
            for (int x = 0; x < N; ++x) wv[i][x] = 0;
            if (!live[i]) continue;
            uint64_t L;
            uint32_t base[NCH], wdig[NCH];
            if (in_lds) {
                const uint32_t ei = s_ent[o - t0];
                L = o - s_cw[ei];
                wv[i][0] = s_rid[ei];
#pragma unroll
                for (int k = 0; k < NCH; ++k) {
                    base[k] = s_base[k][ei];
                    wdig[k] = NCH > 1 ? s_w[NCH > 1 ? k : 0][NCH > 1 ? ei : 0] : 0u;
                }
            } else {
                const uint32_t e = upper_bound_u64(cw, r0, r1 + 2, o) - 1;
                L = o - cw[e];
                wv[i][0] = rid[e];
#pragma unroll
                for (int k = 0; k < NCH; ++k) {
                    base[k] = 0;
                    wdig[k] = 0;
                    if (k < nch) {
                        const int c = cpos[k];
                        const uint32_t lo = a.blo[c][e];
                        if (a.is_leaf[c]) {
                            base[k] = lo;
                            wdig[k] = a.bhi[c][e] - lo;
                        } else {
                            const uint64_t b = a.cw[c][lo];
                            base[k] = static_cast<uint32_t>(b);
                            wdig[k] = static_cast<uint32_t>(a.cw[c][a.bhi[c][e]] - b);
                        }
                    }
                }
            }
            // wv[i][x - p] holds position x of p's subtree; the children's digits, last child least significant
#pragma unroll
            for (int k = NCH - 1; k >= 0; --k) {
                if (k < nch) {
                    uint64_t Lc;
                    if (nch == 1) {
                        Lc = L;
                    } else {
                        Lc = L % wdig[k];
                        L /= wdig[k];
                    }
                    const int c = cpos[k];
                    const uint64_t row = static_cast<uint64_t>(base[k]) + Lc;
                    if (a.is_leaf[c]) {
#pragma unroll
                        for (int x = 1; x < N; ++x)
                            if (x == c - p) wv[i][x] = a.rid[c][row];
                    } else {
                        const uint32_t Sc = static_cast<uint32_t>(a.subtree[c]);
                        const uint32_t *src = a.tab[c] + row * Sc;
#pragma unroll
                        for (int x = 1; x < N; ++x)
                            if (x >= c - p && x < c - p + static_cast<int>(Sc)) wv[i][x] = src[x - (c - p)];
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kExpandC; ++i) {
            if (!live[i]) continue;
            const uint64_t o = orow[i];
            if constexpr (OUT) {
                if constexpr (VAL) {
                    const uint32_t W = static_cast<uint32_t>(a.proj.n);
                    int32_t *dst = a.out + o * W;
                    for (uint32_t q = 0; q < W; ++q) {
                        const int rel = a.proj.rel[q];
                        uint32_t r = 0;
#pragma unroll
                        for (int x = 0; x < N; ++x)
                            if (a.order[x] == rel) r = wv[i][x];
                        dst[q] = a.proj.col[q][r];
                    }
                } else {
                    // relation order: output word j is the position holding relation j
                    uint32_t v[N];
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        v[j] = 0;
#pragma unroll
                        for (int x = 0; x < N; ++x)
                            if (a.order[x] == j) v[j] = wv[i][x];
                    }
                    int32_t *dst = a.out + o * N;
                    if constexpr (N % 4 == 0) {
#pragma unroll
                        for (int j = 0; j < N; j += 4)
                            *reinterpret_cast<int4 *>(dst + j) = make_int4(v[j], v[j + 1], v[j + 2], v[j + 3]);
                    } else if constexpr (N % 2 == 0) {
#pragma unroll
                        for (int j = 0; j < N; j += 2) *reinterpret_cast<int2 *>(dst + j) = make_int2(v[j], v[j + 1]);
                    } else {
#pragma unroll
                        for (int j = 0; j < N; ++j) dst[j] = static_cast<int32_t>(v[j]);
                    }
                }
            } else {
                uint32_t *dst = tab_p + o * S;
#pragma unroll
                for (int x = 0; x < N; ++x)
                    if (x < static_cast<int>(S)) dst[x] = wv[i][x];
            }
        }
        __syncthreads();   // s_r, s_ent and the window are reused by the next block of rows
    }
}

bool mat_factorisable(const MatArgs &a) {
    if (a.nrels < 1 || a.nrels > kMatMaxRels) return false;
    for (int x = 0; x < a.nrels; ++x) {
        if (a.nchild[x] > kFactMaxChild) return false;
        if (x > 0 && !a.is_leaf[x] && (!a.tab[x] || a.subtree[x] < 2)) return false;
        if (!a.n_ent[x]) return false;
    }
    return true;
}

template <int N, bool OUT, bool VAL>
static void launch_expand_n(const MatArgs &a, int x, dim3 g, hipStream_t s) {
    if (a.nchild[x] <= 1)
        hipLaunchKernelGGL((k_mat_expand<N, 1, OUT, VAL>), g, dim3(256), 0, s, a, x);
    else
        hipLaunchKernelGGL((k_mat_expand<N, kFactMaxChild, OUT, VAL>), g, dim3(256), 0, s, a, x);
}

template <bool OUT, bool VAL>
static hipError_t launch_expand(const MatArgs &a, int x, uint64_t rows_max, hipStream_t s) {
    if (rows_max == 0) return hipSuccess;
    uint64_t blocks64 = (rows_max + kExpandPer - 1) / kExpandPer;
    if (blocks64 > kMatPersistentBlocks) blocks64 = kMatPersistentBlocks;
    const dim3 g(static_cast<uint32_t>(blocks64));
    switch (a.nrels) {
#define SJ_EXP_CASE(NN) \
    case NN: launch_expand_n<NN, OUT, VAL>(a, x, g, s); break;
        SJ_EXP_CASE(1) SJ_EXP_CASE(2) SJ_EXP_CASE(3) SJ_EXP_CASE(4) SJ_EXP_CASE(5) SJ_EXP_CASE(6) SJ_EXP_CASE(7)
        SJ_EXP_CASE(8) SJ_EXP_CASE(9) SJ_EXP_CASE(10) SJ_EXP_CASE(11) SJ_EXP_CASE(12) SJ_EXP_CASE(13)
        SJ_EXP_CASE(14) SJ_EXP_CASE(15) SJ_EXP_CASE(16)
#undef SJ_EXP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mat_table(const MatArgs &a, int x, hipStream_t s) {
    if (!mat_factorisable(a) || x <= 0 || x >= a.nrels || a.is_leaf[x]) return hipErrorInvalidValue;
    return launch_expand<false, false>(a, x, a.tab_words[x] / static_cast<uint64_t>(a.subtree[x]), s);
}

hipError_t launch_mat_output(const MatArgs &a, hipStream_t s) {
    if (!mat_factorisable(a)) return hipErrorInvalidValue;
    if (a.proj.n < 0 || a.proj.n > kMaxProj) return hipErrorInvalidValue;
    const uint64_t rows = a.count_dev ? a.capacity : min(a.count, a.capacity);
    return a.proj.n > 0 ? launch_expand<true, true>(a, 0, rows, s) : launch_expand<true, false>(a, 0, rows, s);
}

// ================================================================ cyclic joins

__device__ __forceinline__ uint32_t lower_bound_u32(const int32_t *a, uint32_t lo, uint32_t hi, uint32_t x) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (static_cast<uint32_t>(a[mid]) < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t upper_bound_u32(const int32_t *a, uint32_t lo, uint32_t hi, uint32_t x) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (static_cast<uint32_t>(a[mid]) <= x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Entry of position pos in the current prefix.
template <int N>
__device__ __forceinline__ uint32_t entry_at(const MatState<N> &st, int pos) {
    uint32_t e = st.e[0];
#pragma unroll
    for (int q = 1; q < N; ++q)
        if (q == pos) e = st.e[q];
    return e;
}

// The run of L entries matching the current prefix: [r0, r1) (empty if the closing
// values disagree, or a closing edge between two prefix relations fails).
template <int N>
__device__ __forceinline__ void cyc_run(const CycArgs &a, const MatState<N> &st, uint32_t &r0, uint32_t &r1) {
    uint32_t ep = st.e[0];
#pragma unroll
    for (int q = 1; q < N; ++q)
        if (q == a.pos_P) ep = st.e[q];
    const uint32_t lo = a.Lblo[ep], hi = a.Lbhi[ep];
    r0 = r1 = lo;
    if (lo == hi) return;
#pragma unroll
    for (int c = 0; c < kMaxClose; ++c) {
        if (c < a.ninner && a.icol[c][0][entry_at<N>(st, a.ipos[c][0])] != a.icol[c][1][entry_at<N>(st, a.ipos[c][1])])
            return;
    }
    if (a.nclose == 0) {   // no closing edge ends at L: its whole bucket
        r1 = hi;
        return;
    }
    uint32_t val = 0;
    bool agree = true;
#pragma unroll
    for (int c = 0; c < kMaxClose; ++c) {
        if (c < a.nclose) {
            uint32_t eu = st.e[0];
#pragma unroll
            for (int q = 1; q < N; ++q)
                if (q == a.cpos[c]) eu = st.e[q];
            const uint32_t x = static_cast<uint32_t>(a.ccol[c][eu]);
            if (c == 0)
                val = x;
            else if (x != val)
                agree = false;
        }
    }
    if (!agree) return;
    r0 = lower_bound_u32(a.Lclose, lo, hi, val);
    r1 = upper_bound_u32(a.Lclose, r0, hi, val);
}

// One result tuple (the prefix and L's row lrid) at output index o.
template <int N>
__device__ __forceinline__ void cyc_write(const CycArgs &a, const MatState<N> &st, uint32_t lrid, uint64_t o) {
    if (a.m.proj.n == 0) {
        int32_t *dst = a.out + o * a.nrels;
#pragma unroll
        for (int x = 0; x < N; ++x) dst[a.m.order[x]] = static_cast<int32_t>(a.m.rid[x][st.e[x]]);
        dst[a.L_rel] = static_cast<int32_t>(lrid);
    } else {
        const uint32_t W = static_cast<uint32_t>(a.m.proj.n);
        int32_t *dst = a.out + o * W;
        for (uint32_t q = 0; q < W; ++q) {
            const int rel = a.m.proj.rel[q];
            uint32_t rid = lrid;
#pragma unroll
            for (int x = 0; x < N; ++x)
                if (a.m.order[x] == rel) rid = a.m.rid[x][st.e[x]];
            dst[q] = a.m.proj.col[q][rid];
        }
    }
}

template <int N>
__device__ __forceinline__ uint64_t prefix_factor(const CycArgs &a, const MatState<N> &st) {
    uint64_t f = 1;
#pragma unroll
    for (int x = 0; x < N; ++x) f *= chk_factor(static_cast<uint32_t>(a.m.order[x]), a.m.rid[x][st.e[x]]);
    return f;
}

template <int N, bool WRITE>
__global__ __launch_bounds__(256) void k_cyclic(CycArgs a) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.G) return;
    const uint64_t q = a.wpre / a.G, rem = a.wpre % a.G;
    const uint64_t s = q * t + (t < rem ? t : rem);
    const uint64_t e = s + q + (t < rem ? 1 : 0);
    uint64_t cnt = 0, chk = 0;
    if (s < e) {
        const uint32_t root_n = *a.m.root_n;
        const uint32_t r = upper_bound_u64(a.m.cw[0], 0, root_n + 1, s) - 1;
        MatState<N> st;
        mat_decode<N>(a.m, st, r, s - a.m.cw[0][r]);
        uint64_t o = WRITE ? a.off[t] : 0;
        for (uint64_t i = s;;) {
            uint32_t r0, r1;
            cyc_run<N>(a, st, r0, r1);
            if (r1 > r0 && a.nextra > 0) {
                // closing edges at L on other columns: test each entry of the run
                uint32_t xv[kMaxClose];
#pragma unroll
                for (int c = 0; c < kMaxClose; ++c)
                    xv[c] = c < a.nextra ? static_cast<uint32_t>(a.xcol[c][entry_at<N>(st, a.xpos[c])]) : 0u;
                const uint64_t pf = WRITE ? 0 : prefix_factor<N>(a, st);
                for (uint32_t j = r0; j < r1; ++j) {
                    bool ok = true;
#pragma unroll
                    for (int c = 0; c < kMaxClose; ++c)
                        if (c < a.nextra && static_cast<uint32_t>(a.xL[c][j]) != xv[c]) ok = false;
                    if (!ok) continue;
                    if (!WRITE) {
                        ++cnt;
                        chk += pf * chk_factor(static_cast<uint32_t>(a.L_rel), a.Lrid[j]);
                    } else {
                        cyc_write<N>(a, st, a.Lrid[j], o++);
                    }
                }
            } else if (r1 > r0) {
                if (WRITE && a.m.proj.n == 0) {
                    for (uint32_t j = r0; j < r1; ++j, ++o) {
                        int32_t *dst = a.out + o * a.nrels;
#pragma unroll
                        for (int x = 0; x < N; ++x) dst[a.m.order[x]] = static_cast<int32_t>(a.m.rid[x][st.e[x]]);
                        dst[a.L_rel] = static_cast<int32_t>(a.Lrid[j]);
                    }
                } else if (WRITE) {   // projected values
                    const uint32_t W = static_cast<uint32_t>(a.m.proj.n);
                    for (uint32_t j = r0; j < r1; ++j, ++o) {
                        int32_t *dst = a.out + o * W;
                        for (uint32_t q = 0; q < W; ++q) {
                            const int rel = a.m.proj.rel[q];
                            uint32_t rid = a.Lrid[j];
#pragma unroll
                            for (int x = 0; x < N; ++x)
                                if (a.m.order[x] == rel) rid = a.m.rid[x][st.e[x]];
                            dst[q] = a.m.proj.col[q][rid];
                        }
                    }
                } else {
                    cnt += r1 - r0;
                    chk += prefix_factor<N>(a, st) * (a.Lcv[r1] - a.Lcv[r0]);
                }
            }
            if (++i >= e) break;
            mat_advance<N>(a.m, st, root_n);
        }
    }
    if (!WRITE) {
        a.cnt[t] = cnt;
        a.chk[t] = chk;
    }
}

// One block: totals of cnt/chk and the exclusive prefix of cnt.
__global__ __launch_bounds__(1024) void k_cyclic_scan(CycArgs a) {
    __shared__ uint64_t s_w[1024 / 64], s_v[1024 / 64];
    const uint32_t per = (a.G + 1023) / 1024;
    const uint32_t b = threadIdx.x * per, e = min(a.G, b + per);
    uint64_t c = 0, v = 0;
    for (uint32_t i = b; i < e; ++i) {
        c += a.cnt[i];
        v += a.chk[i];
    }
    uint64_t tc, tv;
    uint64_t off = block_excl_scan<1024>(c, s_w, tc);
    block_excl_scan<1024>(v, s_v, tv);
    for (uint32_t i = b; i < e; ++i) {
        a.off[i] = off;
        off += a.cnt[i];
    }
    if (threadIdx.x == 0) {
        a.totals[0] = tc;
        a.totals[1] = tv;
    }
}

template <bool WRITE>
static hipError_t launch_cyclic(const CycArgs &a, hipStream_t s) {
    if (a.G == 0) return hipSuccess;
    const dim3 g((a.G + 255) / 256);
    switch (a.m.nrels) {
#define SJ_CYC_CASE(NN) \
    case NN: hipLaunchKernelGGL((k_cyclic<NN, WRITE>), g, dim3(256), 0, s, a); break;
        SJ_CYC_CASE(1) SJ_CYC_CASE(2) SJ_CYC_CASE(3) SJ_CYC_CASE(4) SJ_CYC_CASE(5) SJ_CYC_CASE(6) SJ_CYC_CASE(7)
#undef SJ_CYC_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cyclic_count(const CycArgs &a, hipStream_t s) {
    if (hipError_t e = launch_cyclic<false>(a, s)) return e;
    if (a.G) hipLaunchKernelGGL(k_cyclic_scan, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cyclic_write(const CycArgs &a, hipStream_t s) { return launch_cyclic<true>(a, s); }

}  // namespace sj
