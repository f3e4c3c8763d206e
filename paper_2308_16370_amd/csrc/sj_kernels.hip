// Pruning-phase kernels: workspace clearing, predicate counts, filter sizing and
// the fused sieve step (probe incoming filters, build outgoing filters, write the
// ordered survivor list).
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
__global__ void k_count_pred(const int32_t *__restrict__ col, uint32_t n, int32_t lo, int32_t hi,
                             uint32_t *out) {
    uint32_t c = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t v = col[i];
        c += (v >= lo && v < hi) ? 1u : 0u;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

hipError_t launch_count_pred(const int32_t *col, uint32_t n, int32_t lo, int32_t hi, uint32_t *out,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + 256 * 16 - 1) / (256 * 16);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_count_pred, dim3(blocks), dim3(256), 0, s, col, n, lo, hi, out);
    return hipGetLastError();
}

// ---- filter sizes: nblocks = max(1, ceil(bits_per_key * eligible / B)) --------------
__global__ void k_size_filters(SizeArgs a) {
    const int f = threadIdx.x;
    if (f >= a.nfilters) return;
    const uint64_t n = a.elig[f] ? *a.elig[f] : a.rows[f];
    uint64_t nb = (n * a.bits_per_key + a.block_bits - 1) / a.block_bits;
    if (nb == 0) nb = 1;
    *a.nblocks[f] = static_cast<uint32_t>(nb);
}

hipError_t launch_size_filters(const SizeArgs &a, hipStream_t s) {
    if (a.nfilters == 0) return hipSuccess;
    hipLaunchKernelGGL(k_size_filters, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ---- the fused sieve step ----------------------------------------------------------
// Persistent blocks take tiles of kSieveTile consecutive rows in order. Thread t of a
// tile owns rows [t * kSieveItems, (t + 1) * kSieveItems) of it, so a thread's
// survivors are contiguous in row order and one block-wide exclusive scan of the
// per-thread counts plus the tile's look-back prefix places every survivor.
template <int NCOL>
__global__ __launch_bounds__(kSieveBlock) void k_sieve_step(StepArgs a) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_base;
    __shared__ uint32_t s_wave[kSieveBlock / 64];

    const bool list = a.src_rid != nullptr;
    const uint32_t n = list ? *a.src_count : a.src_rows;
    const uint32_t ntiles = (n + kSieveTile - 1) / kSieveTile;
    const int tid = threadIdx.x;

    uint32_t pnb[kMaxProbe], bnb[kMaxBuild];
#pragma unroll
    for (int p = 0; p < kMaxProbe; ++p) pnb[p] = (p < a.nprobe) ? *a.probe[p].nblocks : 0u;
#pragma unroll
    for (int b = 0; b < kMaxBuild; ++b) bnb[b] = (b < a.nbuild) ? *a.build[b].nblocks : 0u;
    const uint32_t wpb_shift = static_cast<uint32_t>(a.logB) - 5u;   // words per block = 1 << wpb_shift

    while (true) {
        if (tid == 0) s_tile = atomicAdd(a.lb.counter, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint32_t row0 = tile * kSieveTile + tid * kSieveItems;

        int32_t v[NCOL][kSieveItems];
        uint32_t rid[kSieveItems];
        bool full = row0 + kSieveItems <= n;
        if (full) {
#pragma unroll
            for (int c = 0; c < NCOL; ++c) {
                const v4i *src = reinterpret_cast<const v4i *>(a.col[c] + row0);
                const v4i x0 = __builtin_nontemporal_load(src);
                const v4i x1 = __builtin_nontemporal_load(src + 1);
                v[c][0] = x0.x; v[c][1] = x0.y; v[c][2] = x0.z; v[c][3] = x0.w;
                v[c][4] = x1.x; v[c][5] = x1.y; v[c][6] = x1.z; v[c][7] = x1.w;
            }
            if (list) {
                const v4u *src = reinterpret_cast<const v4u *>(a.src_rid + row0);
                const v4u r0 = __builtin_nontemporal_load(src);
                const v4u r1 = __builtin_nontemporal_load(src + 1);
                rid[0] = r0.x; rid[1] = r0.y; rid[2] = r0.z; rid[3] = r0.w;
                rid[4] = r1.x; rid[5] = r1.y; rid[6] = r1.z; rid[7] = r1.w;
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

        uint32_t flags = 0;
#pragma unroll
        for (int i = 0; i < kSieveItems; ++i) {
            const uint32_t r = row0 + i;
            bool ok = r < n;
            if (ok && a.pred) {
                const int32_t pv = a.pred[r];
                ok = pv >= a.pred_lo && pv < a.pred_hi;
            }
#pragma unroll
            for (int p = 0; p < kMaxProbe; ++p) {
                if (p < a.nprobe && ok) {
                    int32_t key = v[0][i];
#pragma unroll
                    for (int c = 1; c < NCOL; ++c)
                        if (a.probe_col[p] == c) key = v[c][i];
                    const BfKey h = bf_hash(key, a.seed, pnb[p]);
                    ok = bf_test(a.probe[p].words + (static_cast<uint64_t>(h.block) << wpb_shift), h.g, a.k, a.logB);
                }
            }
            if (ok) {
#pragma unroll
                for (int b = 0; b < kMaxBuild; ++b) {
                    if (b < a.nbuild) {
                        int32_t key = v[0][i];
#pragma unroll
                        for (int c = 1; c < NCOL; ++c)
                            if (a.build_col[b] == c) key = v[c][i];
                        const BfKey h = bf_hash(key, a.seed, bnb[b]);
                        bf_set(a.build[b].words + (static_cast<uint64_t>(h.block) << wpb_shift), h.g, a.k, a.logB);
                    }
                }
            }
            flags |= (ok ? 1u : 0u) << i;
        }

        if (a.out_rid) {
            const uint32_t cnt = __builtin_popcount(flags);
            uint32_t tot;
            const uint32_t off = block_excl_scan<kSieveBlock>(cnt, s_wave, tot);
            if (tid == 0) s_base = lookback32(a.lb.status, tile, tot);
            __syncthreads();
            uint32_t o = s_base + off;
            if (tile == ntiles - 1 && tid == 0) *a.out_count = s_base + tot;
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
        __syncthreads();   // s_tile / s_base / s_wave are rewritten by the next tile
    }
}

hipError_t launch_sieve_step(const StepArgs &a, uint32_t max_rows, hipStream_t s) {
    if (max_rows == 0) return hipSuccess;
    uint32_t tiles = (max_rows + kSieveTile - 1) / kSieveTile;
    uint32_t blocks = tiles < kPersistentBlocks ? tiles : kPersistentBlocks;
    switch (a.ncol) {
        case 1: hipLaunchKernelGGL(k_sieve_step<1>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_sieve_step<2>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_sieve_step<3>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_sieve_step<4>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        case 5: hipLaunchKernelGGL(k_sieve_step<5>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        case 6: hipLaunchKernelGGL(k_sieve_step<6>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        case 7: hipLaunchKernelGGL(k_sieve_step<7>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_sieve_step<8>, dim3(blocks), dim3(kSieveBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sj
