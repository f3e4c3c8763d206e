// Pruning-phase kernels: workspace clearing, predicate counts, filter sizing, the
// sieve step (probe the incoming filters, write the ordered survivor list) and the
// partitioned filter build.
#include <hip/hip_runtime.h>

#include "sj_device.h"
#include "sj_internal.h"

namespace sj {

// ---- clear a byte range (multiple of 4 bytes, 4-byte aligned) ---------------------
__global__ void k_zero(uint4 *p16, uint64_t n16, uint32_t *tail, uint32_t ntail) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        p16[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_zero(void *p, uint64_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    // p is 256-byte aligned in every use (workspace regions)
    const uint64_t n16 = bytes / 16;
    const uint32_t ntail = static_cast<uint32_t>((bytes - n16 * 16) / 4);
    uint64_t blocks = (n16 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, static_cast<uint4 *>(p), n16,
                       reinterpret_cast<uint32_t *>(static_cast<char *>(p) + n16 * 16), ntail);
    return hipGetLastError();
}

// ---- number of rows passing lo <= v < hi -----------------------------------------
__global__ __launch_bounds__(256) void k_count_pred(const int32_t *__restrict__ col, uint32_t n, int32_t lo,
                                                    int32_t hi, uint32_t *out) {
    __shared__ uint32_t s_w[4];
    uint32_t c = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t v = col[i];
        c += (v >= lo && v < hi) ? 1u : 0u;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    // one atomic per workgroup: atomics on one address serialise device-wide
    if (threadIdx.x == 0) {
        const uint32_t t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (t) atomicAdd(out, t);
    }
}

hipError_t launch_count_pred(const int32_t *col, uint32_t n, int32_t lo, int32_t hi, uint32_t *out,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + 256 * 16 - 1) / (256 * 16);
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(k_count_pred, dim3(blocks), dim3(256), 0, s, col, n, lo, hi, out);
    return hipGetLastError();
}

// ---- inserts into a built filter (Section 2.4) ----

__global__ __launch_bounds__(256) void k_filter_probe(FilterUpdate u) {
    __shared__ uint64_t s_w[4];
    const uint32_t nb = *u.nblocks;
    const uint32_t wpb_shift = static_cast<uint32_t>(u.logB) - 5u;
    uint64_t miss = 0;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < u.n; i += stride) {
        const BfKey h = bf_hash(u.keys[i], u.seed, nb);
        const bool ok = bf_test(u.words + (static_cast<uint64_t>(h.block) << wpb_shift), h.g, u.k, u.logB);
        u.contained[i] = ok ? 1 : 0;
        miss += ok ? 0 : 1;
    }
    uint64_t tot;
    block_excl_scan<256>(miss, s_w, tot);
    if (threadIdx.x == 0 && tot) atomicAdd(u.missing, static_cast<unsigned long long>(tot));
}

// The keys the probe found missing set their bits (a bit already seen set is not written).
__global__ __launch_bounds__(256) void k_filter_set(FilterUpdate u) {
    const uint32_t nb = *u.nblocks;
    const uint32_t wpb_shift = static_cast<uint32_t>(u.logB) - 5u;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < u.n; i += stride) {
        if (u.contained[i]) continue;
        const BfKey h = bf_hash(u.keys[i], u.seed, nb);
        bf_set(u.words + (static_cast<uint64_t>(h.block) << wpb_shift), h.g, u.k, u.logB);
    }
}

hipError_t launch_filter_update(const FilterUpdate &u, bool set, hipStream_t s) {
    if (u.n == 0) return hipSuccess;
    const uint64_t want = (u.n + 255) / 256;
    const uint32_t grid = static_cast<uint32_t>(want < 1024 ? want : 1024);
    hipLaunchKernelGGL(k_filter_probe, dim3(grid), dim3(256), 0, s, u);
    if (set) hipLaunchKernelGGL(k_filter_set, dim3(grid), dim3(256), 0, s, u);
    return hipGetLastError();
}

// ---- the sieve step ------------------------------------------------------------------
// Workgroup b of the grid owns the rows [b * R, (b + 1) * R), R a multiple of
// kProbeTile. k_sieve_step probes every row and records a survivor bit per row; then it
// writes its survivors (row id and join columns, ascending row order) after those of
// workgroups 0 .. b-1, whose count it learns by a decoupled look-back over the grid's
// workgroups (one ticket and one status word per workgroup, so a few hundred atomics
// per launch rather than one per tile). Without a survivor list to write (or as two
// launches, for comparison) it records a survivor count per workgroup and
// k_sieve_compact writes the survivors in a second launch.
//
// A probe touches one filter block: the k words of all items of a batch are loaded
// before any is tested, so a thread keeps many independent loads in flight.
// Zipf-skewed columns repeat a few keys very often: each block keeps a direct-mapped
// LDS cache key -> contains(key) per probed filter (the first kMaxCached of them);
// the filter is read-only during the scan, so a cached answer is exact. A key's slot is
// the top kCacheLog bits of c = key * kCacheMul (odd, so key <-> c is a bijection); the
// entry holds the remaining bits of c and two flags, so one 32-bit store publishes a
// consistent entry and a tag match identifies the key exactly.
#ifndef SJ_MAX_CACHED
#define SJ_MAX_CACHED 1
#endif
#ifndef SJ_CACHE_LOG
#define SJ_CACHE_LOG 13
#endif
#ifndef SJ_PROBE_BATCH
#define SJ_PROBE_BATCH 2
#endif
#ifndef SJ_LDS_BATCH
#define SJ_LDS_BATCH 2
#endif
#ifndef SJ_LIST_BATCH
#define SJ_LIST_BATCH 2
#endif
constexpr int kMaxCached = SJ_MAX_CACHED;
constexpr int kCacheLog = SJ_CACHE_LOG;
constexpr int kProbeBatchMax = SJ_PROBE_BATCH;   // keys per batch of the first probe from memory
constexpr int kLdsBatchMax = SJ_LDS_BATCH;       // ... of the first probe from an LDS filter
constexpr int kListBatchMax = SJ_LIST_BATCH;     // list entries per batch of the later probes
static_assert(kProbeBatchMax >= 1 && kLdsBatchMax >= 1 && kListBatchMax >= 1, "probe batches");
constexpr uint32_t kCacheMul = 0x9E3779B1u;
constexpr uint32_t kCacheOk = 1u, kCacheValid = 2u;
constexpr uint32_t kCacheFlags = (1u << kCacheLog) - 1u;
static_assert(kCacheLog >= 2 && kCacheLog <= 16, "cache entry layout");

__device__ __forceinline__ uint32_t cache_slot(uint32_t c) { return c >> (32 - kCacheLog); }
__device__ __forceinline__ uint32_t cache_tag(uint32_t c) { return c << kCacheLog; }

__device__ __forceinline__ uint32_t sieve_rows_per_group(uint32_t n) {
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    return (per + kProbeTile - 1) / kProbeTile * kProbeTile;
}


// The kSieveItems keys of rows row0 .. row0 + 7 of a column (0 past the end).
__device__ __forceinline__ void load_keys(const int32_t *col, uint32_t row0, uint32_t n, bool full, int32_t *k) {
    if (full) {
        const v4i *src = reinterpret_cast<const v4i *>(col + row0);
        const v4i x0 = __builtin_nontemporal_load(src);
        const v4i x1 = __builtin_nontemporal_load(src + 1);
        k[0] = x0.x; k[1] = x0.y; k[2] = x0.z; k[3] = x0.w;
        k[4] = x1.x; k[5] = x1.y; k[6] = x1.z; k[7] = x1.w;
    } else {
#pragma unroll
        for (int i = 0; i < kSieveItems; ++i) k[i] = row0 + i < n ? col[row0 + i] : 0;
    }
}

// One probe of a batch of keys against a filter in memory, through the LDS answer
// cache of probe slot `cslot` (no cache when cslot < 0). live[ii]: the key needs an
// answer; on return, live[ii] is cleared for keys the filter rejects.
template <int B, int KMAX, bool EXACT>
__device__ __forceinline__ void probe_global(const StepArgs &a, const uint32_t *words, uint32_t nb,
                                             uint32_t *cache, const int32_t *keys, bool *live,
                                             uint32_t wpb_shift, uint32_t sh) {
    uint32_t blk[B], g[B], kc[B];
    uint32_t need = 0;
#pragma unroll
    for (int ii = 0; ii < B; ++ii) {
        kc[ii] = static_cast<uint32_t>(keys[ii]) * kCacheMul;
        blk[ii] = 0;
        g[ii] = 0;
        if (live[ii]) {
            bool hit = false;
            if (cache) {
                const uint32_t e = cache[cache_slot(kc[ii])];
                if ((e & ~kCacheFlags) == cache_tag(kc[ii]) && (e & kCacheValid)) {
                    hit = true;
                    if (!(e & kCacheOk)) live[ii] = false;
                }
            }
            if (!hit) {
                const BfKey h = bf_hash(keys[ii], a.seed, nb);
                blk[ii] = h.block;
                g[ii] = h.g;
                need |= 1u << ii;
            }
        }
    }
    uint32_t w[B][KMAX];
#pragma unroll
    for (int ii = 0; ii < B; ++ii) {
        if (need & (1u << ii)) {
            const uint32_t *b = words + (static_cast<uint64_t>(blk[ii]) << wpb_shift);
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < (EXACT ? KMAX : a.k)) w[ii][j] = b[((g[ii] * bf_mult(j)) >> sh) >> 5];
        }
    }
#pragma unroll
    for (int ii = 0; ii < B; ++ii) {
        if (need & (1u << ii)) {
            uint32_t ok = 1u;
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < (EXACT ? KMAX : a.k)) ok &= w[ii][j] >> (((g[ii] * bf_mult(j)) >> sh) & 31u);
            ok &= 1u;
            if (!ok) live[ii] = false;
            if (cache) cache[cache_slot(kc[ii])] = cache_tag(kc[ii]) | kCacheValid | ok;
        }
    }
}

// Survivors of rows [r0, r_end) (a workgroup's share; survivor bits in a.bits), written
// from output position `base` on in ascending row order.
template <int NCOL>
__device__ __forceinline__ void sieve_write_survivors(const StepArgs &a, uint32_t r0, uint32_t r_end, uint32_t n,
                                                      uint32_t base, uint64_t *s_wave64) {
    const bool list = a.src_rid != nullptr;
    const int tid = threadIdx.x;
    // Four tiles share one block scan: their per-thread survivor counts are packed into
    // 16-bit fields of one 64-bit value (a tile holds fewer than 2^16 rows), so sparse
    // survivors cost a quarter of the barriers.
    constexpr int kGroupTiles = 4;
    static_assert(kProbeTile < (1 << 16), "a tile's survivor count fits 16 bits");
    for (uint32_t g0 = r0; g0 < r_end; g0 += kGroupTiles * kProbeTile) {
        uint32_t fl[kGroupTiles];
        uint64_t packed = 0;
#pragma unroll
        for (int q = 0; q < kGroupTiles; ++q) {
            const uint32_t r = g0 + q * kProbeTile + tid * kSieveItems;
            fl[q] = r < r_end ? a.bits[r >> 3] : 0u;
            packed |= static_cast<uint64_t>(__builtin_popcount(fl[q])) << (16 * q);
        }
        uint64_t ptot;
        const uint64_t pex = block_excl_scan<kProbeBlock>(packed, s_wave64, ptot);
#pragma unroll
        for (int q = 0; q < kGroupTiles; ++q) {
            const uint32_t row0 = g0 + q * kProbeTile + tid * kSieveItems;
            const uint32_t flags = fl[q];
            uint32_t o = base + static_cast<uint32_t>((pex >> (16 * q)) & 0xFFFFu);
            base += static_cast<uint32_t>((ptot >> (16 * q)) & 0xFFFFu);
            if (!flags) continue;
            int32_t v[NCOL][kSieveItems];
            uint32_t rid[kSieveItems];
            if (row0 + kSieveItems <= n) {
#pragma unroll
                for (int c = 0; c < NCOL; ++c) {
                    const v4i *src = reinterpret_cast<const v4i *>(a.col[c] + row0);
                    const v4i x0 = src[0], x1 = src[1];
                    v[c][0] = x0.x; v[c][1] = x0.y; v[c][2] = x0.z; v[c][3] = x0.w;
                    v[c][4] = x1.x; v[c][5] = x1.y; v[c][6] = x1.z; v[c][7] = x1.w;
                }
                if (list) {
                    const v4u *src = reinterpret_cast<const v4u *>(a.src_rid + row0);
                    const v4u r0v = src[0], r1v = src[1];
                    rid[0] = r0v.x; rid[1] = r0v.y; rid[2] = r0v.z; rid[3] = r0v.w;
                    rid[4] = r1v.x; rid[5] = r1v.y; rid[6] = r1v.z; rid[7] = r1v.w;
                } else {
#pragma unroll
                    for (int i = 0; i < kSieveItems; ++i) rid[i] = row0 + i;
                }
            } else {
#pragma unroll
                for (int i = 0; i < kSieveItems; ++i) {
                    const uint32_t r = row0 + i;
                    const bool in = r < n;
#pragma unroll
                    for (int c = 0; c < NCOL; ++c) v[c][i] = in ? a.col[c][r] : 0;
                    rid[i] = in ? (list ? a.src_rid[r] : r) : 0u;
                }
            }
#pragma unroll
            for (int i = 0; i < kSieveItems; ++i) {
                if (flags & (1u << i)) {
                    a.out_rid[o] = rid[i];
#pragma unroll
                    for (int c = 0; c < NCOL; ++c) a.out_col[c][o] = v[c][i];
                    ++o;
                }
            }
        }
    }
}

// A wave's list of live rows: entry = the row's index inside the wave's rows (9 bits)
// plus a dead flag.
constexpr uint16_t kListDead = 0x8000;

// KMAX bounds k; with EXACT, k == KMAX and the per-word guards fold away at compile time
// (k = 2, 4 and 6 have such instances: the per-word checks of a general instance cost
// about a tenth of a scan).
template <int NCOL, int KMAX, bool EXACT, bool FUSED>
__global__ __launch_bounds__(kProbeBlock) void k_sieve_step(StepArgs a) {
    // keys whose k words are in flight together (fewer for k > 8, to stay in registers)
    constexpr int kProbeBatch = KMAX > 8 && kProbeBatchMax > 1 ? kProbeBatchMax / 2 : kProbeBatchMax;
    constexpr int kLdsBatch = KMAX > 8 && kLdsBatchMax > 1 ? kLdsBatchMax / 2 : kLdsBatchMax;
    static_assert(kSieveItems % kProbeBatch == 0 && kSieveItems % kLdsBatch == 0, "batches split a lane's rows");
    constexpr int kWaveRows = 64 * kSieveItems;
    __shared__ uint32_t s_wave[kProbeBlock / 64];
    __shared__ uint32_t s_ticket, s_base;
    __shared__ uint64_t s_wave64[kProbeBlock / 64];
    // FUSED: the rows a workgroup owns follow the order in which workgroups started (a
    // ticket), so every workgroup it waits for below is already running
    if (FUSED && threadIdx.x == 0) s_ticket = atomicAdd(a.lb.counter, 1u);
    __shared__ uint32_t s_cache[kMaxCached > 0 ? kMaxCached : 1][1 << kCacheLog];
    __shared__ uint16_t s_list[kProbeBlock / 64][kWaveRows];
    extern __shared__ v4u s_filter4[];   // [a.lds_words / 4]
    const uint32_t *s_filter = reinterpret_cast<const uint32_t *>(s_filter4);
    for (int i = threadIdx.x; i < kMaxCached * (1 << kCacheLog); i += kProbeBlock) (&s_cache[0][0])[i] = 0;
    const uint32_t wpb_shift = static_cast<uint32_t>(a.logB) - 5u;   // words per block = 1 << wpb_shift
    const uint32_t sh = 32u - static_cast<uint32_t>(a.logB);
    // The smallest probed filter that fits the LDS set aside is copied there. The first
    // probe (that filter, else probe 0 from memory) covers every row; the others are
    // probed from memory for the rows still alive, gathered densely per wave.
    int pl = -1;
    uint32_t nb_l = 0, best = 0xFFFFFFFFu;
    const uint32_t *lsrc = nullptr;
    if (a.lds_words) {
#pragma unroll
        for (int p = 0; p < kMaxProbe; ++p) {
            if (p < a.nprobe) {
                const uint32_t nbp = *a.probe[p].nblocks;
                const uint32_t words = nbp << wpb_shift;
                if (words <= a.lds_words && words < best) {
                    best = words;
                    pl = p;
                    nb_l = nbp;
                    lsrc = a.probe[p].words;
                }
            }
        }
        if (pl >= 0)
            for (uint32_t w = threadIdx.x; w < best / 4; w += kProbeBlock)
                s_filter4[w] = reinterpret_cast<const v4u *>(lsrc)[w];
    }
    const int first = pl >= 0 ? pl : 0;   // the probe that covers every row
    // column each probe reads (selected once: no run-time indexing of the argument block)
    const int32_t *pcol[kMaxProbe];
#pragma unroll
    for (int p = 0; p < kMaxProbe; ++p) {
        pcol[p] = a.col[0];
#pragma unroll
        for (int c = 1; c < NCOL; ++c)
            if (p < a.nprobe && a.probe_col[p] == c) pcol[p] = a.col[c];
    }
    __syncthreads();

    const bool list = a.src_rid != nullptr;
    const uint32_t n = list ? *a.src_count : a.src_rows;
    const uint32_t per = sieve_rows_per_group(n);
    const uint32_t wg = FUSED ? s_ticket : blockIdx.x;
    const uint32_t r_end = min(n, (wg + 1) * per);
    const int tid = threadIdx.x;
    const int lane = lane_id();
    uint16_t *wl = s_list[tid >> 6];
    uint32_t survivors = 0;

    // The first probe's keys of the next tile are loaded while the current tile is
    // probed, so the column's load latency overlaps the probing.
    const int32_t *fcol = pcol[0];
#pragma unroll
    for (int p = 1; p < kMaxProbe; ++p)
        if (p == first) fcol = pcol[p];
    int32_t nxt[kSieveItems];
    {
        const uint32_t t0 = wg * per, row0 = t0 + tid * kSieveItems;
        if (t0 < r_end && a.nprobe > 0) load_keys(fcol, row0, n, row0 + kSieveItems <= n, nxt);
    }

    for (uint32_t t0 = wg * per; t0 < r_end; t0 += kProbeTile) {
        const uint32_t row0 = t0 + tid * kSieveItems;
        const uint32_t wrow0 = t0 + (tid & ~63) * kSieveItems;   // the wave's first row
        const bool full = row0 + kSieveItems <= n;
        int32_t key[kSieveItems];
#pragma unroll
        for (int i = 0; i < kSieveItems; ++i) key[i] = nxt[i];
        {
            const uint32_t t1 = t0 + kProbeTile, row1 = t1 + tid * kSieveItems;
            if (t1 < r_end && a.nprobe > 0) load_keys(fcol, row1, n, row1 + kSieveItems <= n, nxt);
        }

        uint32_t flags = 0;
#pragma unroll
        for (int i = 0; i < kSieveItems; ++i) {
            const uint32_t r = row0 + i;
            bool ok = r < n;
            if (ok && a.pred) {
                const int32_t pv = a.pred[r];
                ok = pv >= a.pred_lo && pv < a.pred_hi;
            }
            flags |= (ok ? 1u : 0u) << i;
        }

        // (1) the first probe, per lane over its rows
        if (a.nprobe > 0 && flags) {
            if (pl >= 0) {
                // the LDS filter: all k words of a batch's keys are read before any is tested
#pragma unroll
                for (int i0 = 0; i0 < kSieveItems; i0 += kLdsBatch) {
                    uint32_t w[kLdsBatch][KMAX], g[kLdsBatch];
#pragma unroll
                    for (int ii = 0; ii < kLdsBatch; ++ii) {
                        const BfKey h = bf_hash(key[i0 + ii], a.seed, nb_l);
                        g[ii] = h.g;
                        const uint32_t *b = s_filter + (h.block << wpb_shift);
#pragma unroll
                        for (int j = 0; j < KMAX; ++j)
                            if (j < (EXACT ? KMAX : a.k)) w[ii][j] = b[((h.g * bf_mult(j)) >> sh) >> 5];
                    }
#pragma unroll
                    for (int ii = 0; ii < kLdsBatch; ++ii) {
                        uint32_t ok = 1u;
#pragma unroll
                        for (int j = 0; j < KMAX; ++j)
                            if (j < (EXACT ? KMAX : a.k)) ok &= w[ii][j] >> (((g[ii] * bf_mult(j)) >> sh) & 31u);
                        if (!(ok & 1u)) flags &= ~(1u << (i0 + ii));
                    }
                }
            } else {
                const uint32_t nb0 = *a.probe[0].nblocks;
#pragma unroll
                for (int i0 = 0; i0 < kSieveItems; i0 += kProbeBatch) {
                    bool live[kProbeBatch];
#pragma unroll
                    for (int ii = 0; ii < kProbeBatch; ++ii) live[ii] = (flags >> (i0 + ii)) & 1u;
                    probe_global<kProbeBatch, KMAX, EXACT>(a, a.probe[0].words, nb0, kMaxCached > 0 ? s_cache[0] : nullptr,
                                                    key + i0, live, wpb_shift, sh);
#pragma unroll
                    for (int ii = 0; ii < kProbeBatch; ++ii)
                        if (!live[ii]) flags &= ~(1u << (i0 + ii));
                }
            }
        }

        // (2) the other probes, over the wave's live rows gathered into a dense list
        if (a.nprobe > 1) {
            const uint32_t cnt = __builtin_popcount(flags);
            const uint32_t incl = wave_incl_scan(cnt);
            const uint32_t total = __shfl(incl, 63, 64);
            {
                uint32_t j = incl - cnt;
#pragma unroll
                for (int i = 0; i < kSieveItems; ++i)
                    if (flags & (1u << i)) wl[j++] = static_cast<uint16_t>(lane * kSieveItems + i);
            }
            wave_lds_sync();
            // a lane keeps its list entries through every probe: the keys of all of them are
            // loaded together (one column-load latency per batch), and an entry's liveness
            // stays in registers from one probe to the next
            constexpr int kLB = NCOL >= 3 ? (kListBatchMax < 2 ? kListBatchMax : 2)
                                          : (KMAX > 8 && kListBatchMax > 1 ? kListBatchMax / 2 : kListBatchMax);   // list batch (registers for NCOL keys each)
            for (uint32_t e0 = lane; e0 < total; e0 += 64u * kLB) {
                bool live[kLB], live0[kLB];
                uint16_t ent[kLB];
#pragma unroll
                for (int ii = 0; ii < kLB; ++ii) {
                    const uint32_t e = e0 + ii * 64u;
                    ent[ii] = e < total ? wl[e] : kListDead;
                    live[ii] = !(ent[ii] & kListDead);
                    live0[ii] = live[ii];
                }
                int32_t keys[NCOL][kLB];
#pragma unroll
                for (int c = 0; c < NCOL; ++c)
#pragma unroll
                    for (int ii = 0; ii < kLB; ++ii)
                        keys[c][ii] = live[ii] ? a.col[c][wrow0 + (ent[ii] & (kWaveRows - 1))] : 0;
#pragma unroll
                for (int p = 0; p < kMaxProbe; ++p) {
                    if (p < a.nprobe && p != first) {
                        int32_t pk[kLB];
#pragma unroll
                        for (int ii = 0; ii < kLB; ++ii) {
                            pk[ii] = keys[0][ii];
#pragma unroll
                            for (int c = 1; c < NCOL; ++c)
                                if (a.probe_col[p] == c) pk[ii] = keys[c][ii];
                        }
                        probe_global<kLB, KMAX, EXACT>(a, a.probe[p].words, *a.probe[p].nblocks,
                                                (p < kMaxCached) ? s_cache[p < kMaxCached ? p : 0] : nullptr,
                                                pk, live, wpb_shift, sh);
                    }
                }
#pragma unroll
                for (int ii = 0; ii < kLB; ++ii) {
                    const uint32_t e = e0 + ii * 64u;
                    if (e < total && live0[ii] && !live[ii]) wl[e] = ent[ii] | kListDead;
                }
            }
            wave_lds_sync();
            {
                uint32_t j = incl - cnt;
#pragma unroll
                for (int i = 0; i < kSieveItems; ++i)
                    if (flags & (1u << i))
                        if (wl[j++] & kListDead) flags &= ~(1u << i);
            }
            wave_lds_sync();
        }

        if (row0 < n) a.bits[row0 >> 3] = static_cast<uint8_t>(flags);
        survivors += __builtin_popcount(flags);
    }
    uint32_t tot;
    block_excl_scan<kProbeBlock>(survivors, s_wave, tot);
    if (!FUSED) {
        if (tid == 0) a.counts[blockIdx.x] = tot;
        return;
    }
    // the survivors of the workgroups before this one (decoupled look-back over the
    // tickets), then this workgroup's survivors from the bits it wrote
    if (tid < 64) {
        const uint32_t b = lookback32_wave(a.lb.status, wg, tot);
        if (tid == 0) s_base = b;
    }
    __syncthreads();
    const uint32_t base = s_base;
    if (wg == gridDim.x - 1 && tid == 0) *a.out_count = base + tot;
    sieve_write_survivors<NCOL>(a, wg * per, r_end, n, base, s_wave64);
}


// Survivors of workgroup b's rows, written after those of workgroups 0 .. b-1.
template <int NCOL>
__global__ __launch_bounds__(kProbeBlock) void k_sieve_compact(StepArgs a) {
    __shared__ uint32_t s_wave[kProbeBlock / 64];
    __shared__ uint64_t s_wave64[kProbeBlock / 64];
    const bool list = a.src_rid != nullptr;
    const uint32_t n = list ? *a.src_count : a.src_rows;
    const uint32_t per = sieve_rows_per_group(n);
    const int tid = threadIdx.x;
    uint32_t before = 0;
    for (uint32_t g = tid; g < blockIdx.x; g += kProbeBlock) before += a.counts[g];
    uint32_t tot;
    block_excl_scan<kProbeBlock>(before, s_wave, tot);
    if (blockIdx.x == gridDim.x - 1 && tid == 0) *a.out_count = tot + a.counts[blockIdx.x];
    sieve_write_survivors<NCOL>(a, blockIdx.x * per, min(n, (blockIdx.x + 1) * per), n, tot, s_wave64);
}

template <int KMAX, bool EXACT, bool FUSED>
static hipError_t launch_probe_k(const StepArgs &a, hipStream_t s) {
    if (a.grid == 0 || a.grid > kProbeGridMax) return hipErrorInvalidValue;
    const dim3 g(a.grid), b(kProbeBlock);
    const size_t lds = 4ull * a.lds_words;
    switch (a.ncol) {
#define SJ_PROBE_CASE(NC) \
    case NC: hipLaunchKernelGGL((k_sieve_step<NC, KMAX, EXACT, FUSED>), g, b, lds, s, a); break;
        SJ_PROBE_CASE(1) SJ_PROBE_CASE(2) SJ_PROBE_CASE(3) SJ_PROBE_CASE(4)
        SJ_PROBE_CASE(5) SJ_PROBE_CASE(6) SJ_PROBE_CASE(7) SJ_PROBE_CASE(8)
#undef SJ_PROBE_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool FUSED>
static hipError_t launch_probe_any(const StepArgs &a, hipStream_t s) {
    switch (a.k) {
    case 2: return launch_probe_k<2, true, FUSED>(a, s);
    case 4: return launch_probe_k<4, true, FUSED>(a, s);
    case 6: return launch_probe_k<6, true, FUSED>(a, s);
    default: return a.k <= 8 ? launch_probe_k<8, false, FUSED>(a, s) : launch_probe_k<kMaxK, false, FUSED>(a, s);
    }
}

hipError_t launch_sieve_probe(const StepArgs &a, uint32_t max_rows, hipStream_t s) {
    if (max_rows == 0) return hipSuccess;
    return launch_probe_any<false>(a, s);
}

hipError_t launch_sieve_fused(const StepArgs &a, uint32_t max_rows, hipStream_t s) {
    if (max_rows == 0) return hipSuccess;
    if (!a.out_rid || !a.lb.status || !a.lb.counter) return hipErrorInvalidValue;
    return launch_probe_any<true>(a, s);
}

hipError_t launch_sieve_compact(const StepArgs &a, uint32_t max_rows, hipStream_t s) {
    if (max_rows == 0 || !a.out_rid) return hipSuccess;
    if (a.grid == 0 || a.grid > kProbeGridMax) return hipErrorInvalidValue;
    const dim3 g(a.grid), b(kProbeBlock);
    switch (a.ncol) {
#define SJ_COMPACT_CASE(NC) \
    case NC: hipLaunchKernelGGL((k_sieve_compact<NC>), g, b, 0, s, a); break;
        SJ_COMPACT_CASE(1) SJ_COMPACT_CASE(2) SJ_COMPACT_CASE(3) SJ_COMPACT_CASE(4)
        SJ_COMPACT_CASE(5) SJ_COMPACT_CASE(6) SJ_COMPACT_CASE(7) SJ_COMPACT_CASE(8)
#undef SJ_COMPACT_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- partitioned filter build ----------------------------------------------------------
// Global atomics serialise at the device's atomic units (about 2.7e10 per second on
// MI355X whatever the footprint), so a filter is built by region: a region is a run of
// consecutive blocks small enough for one workgroup's LDS. (1) every tile counts its
// keys per region; (2) an exclusive scan over (region, tile) gives each tile its slice
// of every region's bucket; (3) each kept key is scattered into its region's bucket;
// (4) one workgroup per region rehashes its bucket's keys, sets their bits with LDS
// atomics and writes the region out with plain coalesced stores, which also clears
// the bits no key sets.

__device__ __forceinline__ bool bfb_take(const BuildArgs &a, uint32_t e, int32_t &key) {
    if (a.pred) {
        const int32_t pv = a.pred[e];
        if (pv < a.pred_lo || pv >= a.pred_hi) return false;
    }
    key = a.keys[e];
    return true;
}

struct BfbShape {
    uint32_t n, nb, nreg, tile, ntiles;
    uint32_t rshift;           // a region is 2^rshift blocks
};

__device__ __forceinline__ BfbShape bfb_shape(const BuildArgs &a) {
    BfbShape s;
    s.n = a.n_dev ? *a.n_dev : a.n;
    const uint64_t nkeys = a.nkeys_dev ? *a.nkeys_dev : s.n;
    // the filter is sized for the keys it receives: ceil(bits_per_key * nkeys / B) blocks
    const uint64_t B = 1ull << a.logB;
    uint64_t nb = (nkeys * a.bits_per_key + B - 1) / B;
    s.nb = nb ? static_cast<uint32_t>(nb) : 1u;
    // the largest region unless that leaves fewer than kRegionsTarget regions
    s.rshift = 31u - static_cast<uint32_t>(__builtin_clz(a.region_blocks));
    while (s.rshift > kRegionMinShift && (s.nb >> s.rshift) < kRegionsTarget) --s.rshift;
    s.nreg = (s.nb + (1u << s.rshift) - 1) >> s.rshift;
    s.tile = build_tile_of(s.n);
    s.ntiles = (s.n + s.tile - 1) / s.tile;
    return s;
}

// (1) Per-tile region counts. A key repeated inside a tile is staged once: a
// direct-mapped LDS cache of the tile's keys drops repeats (Zipf heavy hitters would
// otherwise pile millions of identical entries into one region). The cache is updated
// by exchange, so copies of one key that arrive together in a wave are ordered by the
// exchanges and only the first is kept. Which copies are kept is recorded in a bitmap
// (bit e: element e is staged) that the scatter pass follows, so both passes agree.
constexpr int kDedupLog = 13;
constexpr uint32_t kDedupMul = 0x9E3779B1u;

constexpr int kBuildBatch = 8;   // elements per thread whose loads are issued together

__host__ __device__ constexpr uint32_t inv_odd32(uint32_t a) {
    uint32_t x = a;                       // Newton's iteration for the inverse mod 2^32
    for (int i = 0; i < 5; ++i) x *= 2u - a * x;
    return x;
}
static_assert(kDedupMul * inv_odd32(kDedupMul) == 1u, "multiplier inverse");

__device__ __forceinline__ uint32_t dedup_slot(uint32_t key) { return (key * kDedupMul) >> (32 - kDedupLog); }
// An empty slot s holds a key whose own slot is s ^ 1, which no key looked up in s equals.
__device__ __forceinline__ uint32_t dedup_empty(uint32_t s) {
    return ((s ^ 1u) << (32 - kDedupLog)) * inv_odd32(kDedupMul);
}

__global__ __launch_bounds__(kBuildBlock) void k_bfb_hist(BuildArgs a) {
    extern __shared__ uint32_t s_hist[];   // [nreg]
    __shared__ uint32_t s_seen[1 << kDedupLog];
    const BfbShape sh = bfb_shape(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.nblocks = sh.nb;
    for (uint32_t b = blockIdx.x; b < sh.ntiles; b += gridDim.x) {
        // one tile per workgroup when the grid covers the tiles (it does up to kBuildMaxTiles)
        const uint32_t tile = gridDim.x >= sh.ntiles ? xcd_contiguous(b, sh.ntiles) : b;
        for (uint32_t r = threadIdx.x; r < sh.nreg; r += kBuildBlock) s_hist[r] = 0;
        for (uint32_t i = threadIdx.x; i < (1u << kDedupLog); i += kBuildBlock) s_seen[i] = dedup_empty(i);
        __syncthreads();
        const uint32_t t0 = tile * sh.tile;
        for (uint32_t j0 = 0; j0 < sh.tile; j0 += kBuildBlock * kBuildBatch) {
            int32_t key[kBuildBatch];
            bool take[kBuildBatch];
#pragma unroll
            for (int u = 0; u < kBuildBatch; ++u) {
                const uint32_t e = t0 + j0 + u * kBuildBlock + threadIdx.x;
                take[u] = e < sh.n;
                key[u] = take[u] ? a.keys[e] : 0;
                if (take[u] && a.pred) {
                    const int32_t pv = a.pred[e];
                    take[u] = pv >= a.pred_lo && pv < a.pred_hi;
                }
            }
#pragma unroll
            for (int u = 0; u < kBuildBatch; ++u) {
                bool keep = false;
                if (take[u]) {
                    const uint32_t kk = static_cast<uint32_t>(key[u]);
                    keep = atomicExch(&s_seen[dedup_slot(kk)], kk) != kk;
                    if (keep) {
                        const BfKey h = bf_hash(key[u], a.seed, sh.nb);
                        atomicAdd(&s_hist[h.block >> sh.rshift], 1u);
                    }
                }
                const uint64_t m = __ballot(keep);
                if (lane_id() == 0) a.keep[(t0 + j0 + u * kBuildBlock + threadIdx.x) >> 6] = m;
            }
        }
        __syncthreads();
        for (uint32_t r = threadIdx.x; r < sh.nreg; r += kBuildBlock) a.hist[r * sh.ntiles + tile] = s_hist[r];
        __syncthreads();
    }
}

// Exclusive scan in place of hist[0 .. nreg * ntiles) (decoupled look-back); the
// grand total (the number of staged keys) goes to *total_dev.
__global__ __launch_bounds__(kScanBlock) void k_bfb_scan(BuildArgs a) {
    __shared__ uint32_t s_tile, s_base;
    __shared__ uint32_t s_wave[kScanBlock / 64];
    const BfbShape sh = bfb_shape(a);
    const uint32_t len = sh.nreg * sh.ntiles;
    const uint32_t ntiles = (len + kScanTile - 1) / kScanTile;
    while (true) {
        if (threadIdx.x == 0) s_tile = atomicAdd(a.lb.counter, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint32_t base = tile * kScanTile + threadIdx.x * kScanItems;
        uint32_t x[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            x[i] = (base + i < len) ? a.hist[base + i] : 0u;
            sum += x[i];
        }
        uint32_t tot;
        uint32_t off = block_excl_scan<kScanBlock>(sum, s_wave, tot);
        if (threadIdx.x < 64) {
            const uint32_t b = lookback32_wave(a.lb.status, tile, tot);
            if (threadIdx.x == 0) s_base = b;
        }
        __syncthreads();
        if (tile == ntiles - 1 && threadIdx.x == 0) *a.total_dev = s_base + tot;
        off += s_base;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < len) a.hist[base + i] = off;
            off += x[i];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBuildBlock) void k_bfb_scatter(BuildArgs a) {
    extern __shared__ uint32_t s_off[];    // [nreg]
    const BfbShape sh = bfb_shape(a);
    for (uint32_t b = blockIdx.x; b < sh.ntiles; b += gridDim.x) {
        // one tile per workgroup when the grid covers the tiles (it does up to kBuildMaxTiles)
        const uint32_t tile = gridDim.x >= sh.ntiles ? xcd_contiguous(b, sh.ntiles) : b;
        for (uint32_t r = threadIdx.x; r < sh.nreg; r += kBuildBlock) s_off[r] = a.hist[r * sh.ntiles + tile];
        __syncthreads();
        const uint32_t t0 = tile * sh.tile;
        for (uint32_t j0 = 0; j0 < sh.tile; j0 += kBuildBlock * kBuildBatch) {
            int32_t key[kBuildBatch];
            bool take[kBuildBatch];
#pragma unroll
            for (int u = 0; u < kBuildBatch; ++u) {
                const uint32_t e = t0 + j0 + u * kBuildBlock + threadIdx.x;
                const uint64_t m = a.keep[e >> 6];
                take[u] = e < sh.n && ((m >> (e & 63)) & 1ull);
                key[u] = take[u] ? a.keys[e] : 0;
            }
#pragma unroll
            for (int u = 0; u < kBuildBatch; ++u) {
                if (take[u]) {
                    const BfKey h = bf_hash(key[u], a.seed, sh.nb);
                    const uint32_t pos = atomicAdd(&s_off[h.block >> sh.rshift], 1u);
                    a.stage[pos] = static_cast<uint32_t>(key[u]);
                }
            }
        }
        __syncthreads();
    }
}

// KMAX bounds k; with EXACT, k == KMAX (instances for k = 2, 4 and 6, as for the probes).
template <int KMAX, bool EXACT>
__global__ __launch_bounds__(kRegionThreads) void k_bfb_region(BuildArgs a) {
    extern __shared__ uint32_t s_words[];  // [region_blocks * words per block]
    const BfbShape sh = bfb_shape(a);
    const uint32_t wpb_shift = static_cast<uint32_t>(a.logB) - 5u;
    const uint32_t hs = 32u - static_cast<uint32_t>(a.logB);
    const uint32_t total = *a.total_dev;
    constexpr int U = 4;
    for (uint32_t r = blockIdx.x; r < sh.nreg; r += gridDim.x) {
        const uint32_t b0 = r << sh.rshift;
        const uint32_t nbr = min(1u << sh.rshift, sh.nb - b0);
        const uint32_t nw = nbr << wpb_shift;
        for (uint32_t i = threadIdx.x; i < nw; i += kRegionThreads) s_words[i] = 0;
        __syncthreads();
        const uint32_t beg = sh.ntiles ? a.hist[r * sh.ntiles] : 0u;
        const uint32_t end = (r + 1 < sh.nreg && sh.ntiles) ? a.hist[(r + 1) * sh.ntiles] : total;
        for (uint32_t e0 = beg + threadIdx.x; e0 < end; e0 += kRegionThreads * U) {
            uint32_t bb[U], gg[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t e = e0 + u * kRegionThreads;
                // the staged key's block (inside this region) and second hash word, recomputed
                const BfKey h = bf_hash(static_cast<int32_t>(e < end ? a.stage[e] : 0u), a.seed, sh.nb);
                bb[u] = e < end ? h.block - b0 : 0xFFFFFFFFu;
                gg[u] = h.g;
            }
            // read every word the batch touches first, then OR only the bits still clear:
            // heavy-hitter keys staged by many tiles find their bits set and cost no atomic
            uint32_t w[U][KMAX];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (bb[u] != 0xFFFFFFFFu) {
                    const uint32_t *wb = s_words + (bb[u] << wpb_shift);
#pragma unroll
                    for (int j = 0; j < KMAX; ++j)
                        if (j < (EXACT ? KMAX : a.k)) w[u][j] = wb[((gg[u] * bf_mult(j)) >> hs) >> 5];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (bb[u] != 0xFFFFFFFFu) {
                    uint32_t *wb = s_words + (bb[u] << wpb_shift);
#pragma unroll
                    for (int j = 0; j < KMAX; ++j) {
                        if (j < (EXACT ? KMAX : a.k)) {
                            const uint32_t p = (gg[u] * bf_mult(j)) >> hs;
                            const uint32_t bit = 1u << (p & 31u);
                            if (!(w[u][j] & bit)) atomicOr(wb + (p >> 5), bit);
                        }
                    }
                }
            }
        }
        __syncthreads();
        uint32_t *dst = a.words + (static_cast<uint64_t>(b0) << wpb_shift);
        for (uint32_t i = threadIdx.x; i < nw; i += kRegionThreads) dst[i] = s_words[i];
        __syncthreads();
    }
}

hipError_t launch_filter_build_stage(const BuildArgs &a, int stage, hipStream_t s) {
    const uint32_t ntiles_max = min(kBuildMaxTiles, (a.n_max + kBuildTileMin - 1) / kBuildTileMin);
    const uint32_t nreg_max = region_count_cap(a.nblocks_max, a.region_blocks);
    const size_t lds_hist = 4ull * (nreg_max ? nreg_max : 1);
    const size_t lds_region = 4ull * a.region_blocks * (1u << (a.logB - 5));
    const uint32_t tgrid = ntiles_max == 0 ? 1 : (ntiles_max < 2048 ? ntiles_max : 2048);
    switch (stage) {
        case 0:
            hipLaunchKernelGGL(k_bfb_hist, dim3(tgrid), dim3(kBuildBlock), lds_hist, s, a);
            break;
        case 1: {
            // every workgroup claims at least one tile from a single counter: size the grid to the work
            const uint32_t scan_tiles = (nreg_max * ntiles_max + kScanTile - 1) / kScanTile;
            const uint32_t sgrid = scan_tiles == 0 ? 1 : (scan_tiles < 256 ? scan_tiles : 256);
            hipLaunchKernelGGL(k_bfb_scan, dim3(sgrid), dim3(kScanBlock), 0, s, a);
            break;
        }
        case 2:
            hipLaunchKernelGGL(k_bfb_scatter, dim3(tgrid), dim3(kBuildBlock), lds_hist, s, a);
            break;
        case 3: {
            const uint32_t rgrid = nreg_max == 0 ? 1 : (nreg_max < 2048 ? nreg_max : 2048);
            switch (a.k) {
            case 2: hipLaunchKernelGGL((k_bfb_region<2, true>), dim3(rgrid), dim3(kRegionThreads), lds_region, s, a); break;
            case 4: hipLaunchKernelGGL((k_bfb_region<4, true>), dim3(rgrid), dim3(kRegionThreads), lds_region, s, a); break;
            case 6: hipLaunchKernelGGL((k_bfb_region<6, true>), dim3(rgrid), dim3(kRegionThreads), lds_region, s, a); break;
            default: hipLaunchKernelGGL((k_bfb_region<kMaxK, false>), dim3(rgrid), dim3(kRegionThreads), lds_region, s, a); break;
            }
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sj
