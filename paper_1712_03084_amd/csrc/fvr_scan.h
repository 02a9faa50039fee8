// Exclusive scan building blocks: the two-launch scan of the marching-cubes
// block totals, and the bin-offset scan of the splat, folded into tile_list
// and tile_order (so it costs no launches of its own).
//
// The input of n items of C interleaved int32 components is cut into tiles
// of kScanTile items; a 256-thread block reduces one tile to its totals
// (scan_tile_sum), and later a 256-thread block scans one tile on top of the
// totals of the tiles before it (scan_tile_down).
#pragma once

#include "fvr_common.h"

namespace fvr {

constexpr int kScanBlock = 256;
constexpr int kScanIpt = 8;  // consecutive items per thread
constexpr int kScanTile = kScanBlock * kScanIpt;

__host__ __device__ inline int scan_tiles(int n) { return (n + kScanTile - 1) / kScanTile; }

// Inclusive scan of one int across a 64-lane wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// partial[tile * C + c] = sum of component c over the tile's items.
// Called by all kScanBlock threads of a block.
template <int C>
__device__ __forceinline__ void scan_tile_sum(const int32_t *__restrict__ in, int n, int tile,
                                              int32_t *__restrict__ partial) {
    __shared__ int red[C][kScanBlock / 64];
    const int base = tile * kScanTile + threadIdx.x * kScanIpt;
    int s[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0;
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        const int i = base + j;
        if (i < n) {
#pragma unroll
            for (int c = 0; c < C; ++c) s[c] += in[(size_t)i * C + c];
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        int v = s[c];
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane == 0) red[c][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < C) {
        int t = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) t += red[threadIdx.x][w];
        partial[tile * C + threadIdx.x] = t;
    }
}

// out[i * C + c] = sum over items before i (all tiles); the last tile also
// writes out[n * C + c] = total (and totals[c], if not null).  partial holds
// the totals of tiles 0 .. tile - 1 (scan_tile_sum, in an earlier kernel).
// Called by all kScanBlock threads of a block.
template <int C>
__device__ __forceinline__ void scan_tile_down(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                               int n, const int32_t *__restrict__ partial, int tile,
                                               int ntiles, int32_t *totals = nullptr) {
    __shared__ int wsum[C][kScanBlock / 64];
    __shared__ int bsum[C][kScanBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // the totals of the earlier tiles, loaded in parallel and reduced
    // (a serial loop would wait on one load after another)
    int pb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) pb[c] = 0;
    for (int b = threadIdx.x; b < tile; b += blockDim.x) {
#pragma unroll
        for (int c = 0; c < C; ++c) pb[c] += partial[b * C + c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) pb[c] += __shfl_xor(pb[c], d, 64);
        if (lane == 0) bsum[c][wid] = pb[c];
    }
    const int base = tile * kScanTile + threadIdx.x * kScanIpt;
    int v[kScanIpt][C], s[C], incl[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0;
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        const int i = base + j;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            v[j][c] = i < n ? in[(size_t)i * C + c] : 0;
            s[c] += v[j][c];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        incl[c] = wave_incl_scan(s[c]);
        if (lane == 63) wsum[c][wid] = incl[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        int run = incl[c] - s[c];
        for (int w = 0; w < kScanBlock / 64; ++w) run += bsum[c][w];
        for (int w = 0; w < wid; ++w) run += wsum[c][w];
#pragma unroll
        for (int j = 0; j < kScanIpt; ++j) {
            const int i = base + j;
            if (i < n) out[(size_t)i * C + c] = run;
            run += v[j][c];
        }
        if (tile == ntiles - 1 && threadIdx.x == blockDim.x - 1) {
            out[(size_t)n * C + c] = run;
            if (totals) totals[c] = run;
        }
    }
}

}  // namespace fvr
