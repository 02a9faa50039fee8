// Iso-level, marching cubes with prefix-sum compaction, and the small
// utility kernels (fill, status reset, scan) for gfx950.
//
// Iso-level (Sec. III-B): L = mean of A at the input sample locations,
// sampled trilinearly between voxel centres; per-thread compensated double
// sums, a fixed reduction tree per block and one block that reduces the block
// partials in a fixed order, so L is deterministic.  This is the only double
// precision arithmetic on the GPU.
//
// Marching cubes (end of Sec. III-B) without a dense per-cell output:
//   mc_classify (when the row ranges of A are known) settles the blocks of
//               1024 grid points whose cells lie on one side of the level and
//               lists the others; the kernels below then run persistent
//               blocks over that list
//   mc_count    each thread owns 4 consecutive grid points q (linear order):
//               the 3 grid edges leaving q that cross the level (vertices),
//               the case of the cell with lower corner q, its triangle count
//               and whether it is active; block totals -> blk_counts
//               and, for blocks the surface passes, one code byte per point
//               (the case, or the edge bits on the upper borders)
//   scan        exclusive scan of the block totals: over the listed blocks
//               in one block when there is a list, else over all blocks in
//               two launches (folding it into the neighbouring kernels with
//               group totals kept by atomics measured slower: 117 us against
//               79 us for the four marching-cubes stages at 256^3)
//   mc_generate from the codes (blocks without vertices or active cells exit
//               at once), block-scan, write each vertex at its global rank
//               (vertex order = (linear index, axis)), record the vertex id of
//               every crossing edge, and compact the active cells
//               (linear index, case, first triangle)
//   mc_triangles one thread per active cell emits its table triangles
#include <algorithm>

#include "fvr_common.h"
#include "fvr_scan.h"

namespace fvr {

__constant__ uint8_t c_mc_count[256];
__constant__ int8_t c_mc_edges[256 * kMcRow];

// The classification kernels copy the triangle counts into LDS: a lookup is
// then an LDS read, so it never waits for the field loads still in flight.
__device__ __forceinline__ void mc_count_table(uint8_t *t) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) t[i] = c_mc_count[i];
    __syncthreads();
}

constexpr int kMcThreads = 256;
constexpr int kMcPpt = 4;                       // grid points per thread
constexpr int kMcPerBlock = kMcThreads * kMcPpt;
constexpr int kLevelThreads = 256;
constexpr int kLevelPpt = 4;

// ---------------------------------------------------------------------------
// Utilities
// ---------------------------------------------------------------------------
__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void prep_kernel(DevStatus *st, int32_t *bins, int nbins) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        st->flags = 0;
        st->rejected = 0;
        st->mc_total[0] = st->mc_total[1] = st->mc_total[2] = 0;
        st->n_used = 0;
        st->level = 0.0;
        st->wmax_bits = 0;
        st->wnmax_bits = 0;
        st->tile_ticket = 0;
        st->n_busy = 0;
        st->mc_active = 0;
        st->n_zplanes = 0;
        st->fe_points = 0;
    }
    if (bins && i < nbins) bins[i] = 0;
}

// The status block copied by one small kernel into the context's pinned,
// device-accessible host copy: the stores go straight to host memory and are
// visible once the stream has been synchronized.  Cheaper at the end of a
// frame than a device-to-host copy (about 4 us per frame on the proxy frame).
__global__ void status_publish_kernel(const DevStatus *__restrict__ st, uint32_t *__restrict__ dst) {
    static_assert(sizeof(DevStatus) % 4 == 0, "status words");
    const uint32_t *src = reinterpret_cast<const uint32_t *>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(DevStatus) / 4); i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_status_publish(const DevStatus *st, DevStatus *host, hipStream_t s) {
    status_publish_kernel<<<1, 64, 0, s>>>(st, reinterpret_cast<uint32_t *>(host));
    return hipGetLastError();
}

hipError_t launch_prep(DevStatus *st, int32_t *bins, int nbins, hipStream_t s) {
    const int blocks = nbins > 0 ? (nbins + 255) / 256 : 1;
    prep_kernel<<<dim3(blocks), dim3(256), 0, s>>>(st, bins, nbins);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    fill_i32_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(p, n, v);
    return hipGetLastError();
}

// Exclusive scan of n items of C interleaved components in two kernels:
//   scan_reduce  block b sums scan tile b -> partial[b]
//   scan_down    block b adds partial[0..b) and scans its tile; the last
//                block also writes the totals.
template <int C>
__global__ void __launch_bounds__(kScanBlock)
scan_reduce_kernel(const int32_t *__restrict__ in, int n, int32_t *__restrict__ partial) {
    scan_tile_sum<C>(in, n, blockIdx.x, partial);
}

template <int C>
__global__ void __launch_bounds__(kScanBlock)
scan_down_kernel(const int32_t *__restrict__ in, int32_t *__restrict__ out, int n,
                 const int32_t *__restrict__ partial, int32_t *totals) {
    scan_tile_down<C>(in, out, n, partial, blockIdx.x, gridDim.x, totals);
}

// Offsets of the blocks in the marching-cubes list, in one block: the other
// blocks have zero totals, so the exclusive scan over all nb blocks reduces
// to a scan of the listed blocks in block order.  A bitmap of the listed
// blocks gives each its rank in that order (popcounts of the words before
// it), the listed totals are scanned in rank order, and each listed block
// gets its offsets; out[3 nb + c] and st->mc_total receive the totals.  More
// than kListCap listed blocks (a surface through most of the grid): a plain
// scan over all nb blocks in the same block.
constexpr int kListThreads = 1024;
constexpr int kListCap = 4096;
static_assert(kListCap % kListThreads == 0, "whole entries per thread");

__global__ void __launch_bounds__(kListThreads)
mc_list_scan_kernel(const int32_t *__restrict__ list, const int32_t *__restrict__ cnt, int nb,
                    int32_t *__restrict__ out, DevStatus *st) {
    extern __shared__ __attribute__((aligned(16))) int lsm[];
    const int nw = (nb + 31) >> 5;          // bitmap words
    unsigned *bits = reinterpret_cast<unsigned *>(lsm);
    int *wbase = lsm + nw;                  // listed blocks before each word
    int4 *srt = reinterpret_cast<int4 *>(lsm + ((2 * nw + 3) & ~3));  // (block, counts) in block order
    __shared__ int wsum[3][kListThreads / 64];
    const int n = st->mc_active;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (n <= kListCap) {
        // this thread's entries i = threadIdx.x + kListThreads u and their
        // totals, loaded once: the totals' loads are in flight while the
        // bitmap is built and ranked
        constexpr int kPer = kListCap / kListThreads;
        int4 e[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = (int)threadIdx.x + kListThreads * u;
            e[u].x = i < n ? list[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (e[u].x >= 0) e[u] = make_int4(e[u].x, cnt[3 * e[u].x], cnt[3 * e[u].x + 1], cnt[3 * e[u].x + 2]);
        for (int w = threadIdx.x; w < nw; w += kListThreads) bits[w] = 0u;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (e[u].x >= 0) atomicOr(&bits[e[u].x >> 5], 1u << (e[u].x & 31));
        __syncthreads();
        // exclusive scan of the words' popcounts: thread t owns words [t S, (t+1) S)
        const int S = (nw + kListThreads - 1) / kListThreads;
        const int w0 = min((int)threadIdx.x * S, nw), w1 = min(w0 + S, nw);
        int sp = 0;
        for (int w = w0; w < w1; ++w) sp += __popc(bits[w]);
        int incl = wave_incl_scan(sp);
        if (lane == 63) wsum[0][wid] = incl;
        __syncthreads();
        int run = incl - sp;
        for (int v = 0; v < wid; ++v) run += wsum[0][v];
        for (int w = w0; w < w1; ++w) {
            wbase[w] = run;
            run += __popc(bits[w]);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (e[u].x >= 0) {
                const int b = e[u].x;
                srt[wbase[b >> 5] + __popc(bits[b >> 5] & ((1u << (b & 31)) - 1u))] = e[u];
            }
        __syncthreads();
        // exclusive scan of the listed totals in block order
        const int T = (n + kListThreads - 1) / kListThreads;
        const int r0 = min((int)threadIdx.x * T, n), r1 = min(r0 + T, n);
        int s3[3] = {0, 0, 0};
        for (int r = r0; r < r1; ++r) {
            s3[0] += srt[r].y;
            s3[1] += srt[r].z;
            s3[2] += srt[r].w;
        }
        int inc3[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            inc3[c] = wave_incl_scan(s3[c]);
            if (lane == 63) wsum[c][wid] = inc3[c];
        }
        __syncthreads();
        int run3[3], tot[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            run3[c] = inc3[c] - s3[c];
            tot[c] = 0;
            for (int v = 0; v < kListThreads / 64; ++v) {
                if (v < wid) run3[c] += wsum[c][v];
                tot[c] += wsum[c][v];
            }
        }
        for (int r = r0; r < r1; ++r) {
            const int4 e = srt[r];
            out[3 * e.x + 0] = run3[0];
            out[3 * e.x + 1] = run3[1];
            out[3 * e.x + 2] = run3[2];
            run3[0] += e.y;
            run3[1] += e.z;
            run3[2] += e.w;
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                out[3 * nb + c] = tot[c];
                st->mc_total[c] = tot[c];
            }
        }
        return;
    }
    // many listed blocks: a scan over every block, thread t owning a contiguous range
    const int S = (nb + kListThreads - 1) / kListThreads;
    const int b0 = min((int)threadIdx.x * S, nb), b1 = min(b0 + S, nb);
    int s3[3] = {0, 0, 0};
    for (int b = b0; b < b1; ++b) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s3[c] += cnt[3 * b + c];
    }
    int inc3[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        inc3[c] = wave_incl_scan(s3[c]);
        if (lane == 63) wsum[c][wid] = inc3[c];
    }
    __syncthreads();
    int run3[3], tot[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        run3[c] = inc3[c] - s3[c];
        tot[c] = 0;
        for (int v = 0; v < kListThreads / 64; ++v) {
            if (v < wid) run3[c] += wsum[c][v];
            tot[c] += wsum[c][v];
        }
    }
    for (int b = b0; b < b1; ++b) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int v = cnt[3 * b + c];
            out[3 * b + c] = run3[c];
            run3[c] += v;
        }
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            out[3 * nb + c] = tot[c];
            st->mc_total[c] = tot[c];
        }
    }
}

static size_t mc_list_scan_lds(int nb) {
    const int nw = (nb + 31) >> 5;
    return (size_t)((2 * nw + 3) & ~3) * sizeof(int) + (size_t)kListCap * sizeof(int4);
}

hipError_t launch_mc_list_scan(const int32_t *list, const int32_t *cnt, int nb, int32_t *out,
                               DevStatus *st, hipStream_t s) {
    const size_t lds = mc_list_scan_lds(nb);
    if (lds > (size_t)kLdsPerWorkgroup - 2048) return hipErrorInvalidValue;
    mc_list_scan_kernel<<<dim3(1), dim3(kListThreads), lds, s>>>(list, cnt, nb, out, st);
    return hipGetLastError();
}

hipError_t mc_configure() { return raise_dynamic_lds((const void *)mc_list_scan_kernel); }

int scan_partials(int n) { return scan_tiles(n); }

hipError_t launch_scan(const int32_t *in, int32_t *out, int n, int C, int32_t *partial,
                       int32_t *totals, hipStream_t s) {
    const int nb = n > 0 ? scan_partials(n) : 1;
    if (C == 3) {
        scan_reduce_kernel<3><<<nb, kScanBlock, 0, s>>>(in, n, partial);
        scan_down_kernel<3><<<nb, kScanBlock, 0, s>>>(in, out, n, partial, totals);
    } else if (C == 1) {
        scan_reduce_kernel<1><<<nb, kScanBlock, 0, s>>>(in, n, partial);
        scan_down_kernel<1><<<nb, kScanBlock, 0, s>>>(in, out, n, partial, totals);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Iso-level
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sample_trilinear(const float *__restrict__ A, const Grid &g,
                                                  float x, float y, float z) {
    const float X[3] = {x, y, z};
    int b[3];
    float t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = __fsub_rn(__fdiv_rn(__fsub_rn(X[a], g.bmin[a]), g.h[a]), 0.5f);
        // points inside the box have u in [-1/2, N - 1/2]; the clamp keeps the
        // conversion defined for any input (NaN goes to -1)
        int bb = (int)floorf(fminf(fmaxf(u, -1.0f), (float)g.n[a]));
        bb = min(max(bb, 0), g.n[a] - 2);
        b[a] = bb;
        t[a] = fminf(fmaxf(u - (float)bb, 0.0f), 1.0f);
    }
    const size_t sx = 1, sy = g.n[0], sz = (size_t)g.n[0] * g.n[1];
    const size_t o = b[0] + sy * b[1] + sz * b[2];
    const float c00 = A[o] + t[0] * (A[o + sx] - A[o]);
    const float c10 = A[o + sy] + t[0] * (A[o + sy + sx] - A[o + sy]);
    const float c01 = A[o + sz] + t[0] * (A[o + sz + sx] - A[o + sz]);
    const float c11 = A[o + sz + sy] + t[0] * (A[o + sz + sy + sx] - A[o + sz + sy]);
    const float c0 = c00 + t[1] * (c10 - c00);
    const float c1 = c01 + t[1] * (c11 - c01);
    return c0 + t[2] * (c1 - c0);
}

__global__ void __launch_bounds__(kLevelThreads)
level_partial_kernel(const float *__restrict__ pts, int m, const float *__restrict__ A, Grid g,
                     double *__restrict__ psum, int32_t *__restrict__ pcnt) {
    __shared__ double ssum[kLevelThreads];
    __shared__ int scnt[kLevelThreads];
    double sum = 0.0, comp = 0.0;
    int cnt = 0;
    const int base = blockIdx.x * kLevelThreads * kLevelPpt;
    // all of a thread's samples are gathered before any is summed, so their
    // loads overlap: positions from clamped indices, then the 8 corners of
    // every position (the sampler keeps any input inside the grid); points
    // past the end or outside the box are then skipped in order
    float v[kLevelPpt];
    bool acc[kLevelPpt];
#pragma unroll
    for (int j = 0; j < kLevelPpt; ++j) {
        const int i = base + j * kLevelThreads + threadIdx.x;
        const int ic = min(i, m - 1);
        const float x = pts[3 * ic], y = pts[3 * ic + 1], z = pts[3 * ic + 2];
        // NaN coordinates fail the comparisons too
        acc[j] = i < m && x >= g.bmin[0] && x <= g.bmax[0] && y >= g.bmin[1] && y <= g.bmax[1] &&
                 z >= g.bmin[2] && z <= g.bmax[2];
        v[j] = sample_trilinear(A, g, x, y, z);
    }
#pragma unroll
    for (int j = 0; j < kLevelPpt; ++j) {
        if (!acc[j]) continue;
        const double vj = (double)v[j];
        const double s = sum + vj;
        comp += fabs(sum) >= fabs(vj) ? (sum - s) + vj : (vj - s) + sum;
        sum = s;
        ++cnt;
    }
    ssum[threadIdx.x] = sum + comp;
    scnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = kLevelThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
            scnt[threadIdx.x] += scnt[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        psum[blockIdx.x] = ssum[0];
        pcnt[blockIdx.x] = scnt[0];
    }
}

// Sum and count over the nb block partials (compensated, in a fixed order,
// so every caller gets the same bits).  Called by all kLevelThreads threads
// of a block; each gets the totals.
__device__ __forceinline__ void level_reduce(const double *__restrict__ psum, const int32_t *__restrict__ pcnt,
                                             int nb, double &total, int &count) {
    __shared__ double ssum[kLevelThreads];
    __shared__ int scnt[kLevelThreads];
    double sum = 0.0, comp = 0.0;
    int cnt = 0;
    // partials kB at a time: loads from clamped indices go out together, the
    // ones past the end count as zero; the summation order is fixed
    constexpr int kB = 4;
    for (int b0 = 0; b0 < nb; b0 += kB * kLevelThreads) {
        double pv[kB];
        int pc[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int i = min(b0 + u * kLevelThreads + (int)threadIdx.x, nb - 1);
            pv[u] = psum[i];
            pc[u] = pcnt[i];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (b0 + u * kLevelThreads + (int)threadIdx.x >= nb) break;
            const double v = pv[u];
            const double s = sum + v;
            comp += fabs(sum) >= fabs(v) ? (sum - s) + v : (v - s) + sum;
            sum = s;
            cnt += pc[u];
        }
    }
    ssum[threadIdx.x] = sum + comp;
    scnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = kLevelThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
            scnt[threadIdx.x] += scnt[threadIdx.x + w];
        }
        __syncthreads();
    }
    total = ssum[0];
    count = scnt[0];
}

// L = sum / count (0 when no sample was accepted), kept in fp64 in the
// status block and as the float the classification compares against.
__device__ __forceinline__ float level_publish(double total, int count, DevStatus *st, float *level_f32) {
    const double L = count > 0 ? total / (double)count : 0.0;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->n_used = count;
        st->level = L;
        *level_f32 = (float)L;
    }
    return (float)L;
}

__global__ void __launch_bounds__(kLevelThreads)
level_final_kernel(const double *__restrict__ psum, const int32_t *__restrict__ pcnt, int nb,
                   DevStatus *st, float *level_f32) {
    double total;
    int count;
    level_reduce(psum, pcnt, nb, total, count);
    level_publish(total, count, st, level_f32);
}

int level_blocks(int m) { return (m + kLevelThreads * kLevelPpt - 1) / (kLevelThreads * kLevelPpt); }

hipError_t launch_level(const float *pts, int m, const float *A, const Grid &g, double *psum,
                        int32_t *pcnt, DevStatus *st, float *level_f32, bool final, hipStream_t s) {
    const int nb = level_blocks(m);
    if (nb > 0) {
        level_partial_kernel<<<dim3(nb), dim3(kLevelThreads), 0, s>>>(pts, m, A, g, psum, pcnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (final) level_final_kernel<<<1, kLevelThreads, 0, s>>>(psum, pcnt, nb, st, level_f32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Marching cubes
// ---------------------------------------------------------------------------
hipError_t mc_upload_table(const uint8_t *counts, const int8_t *edges) {
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_mc_count), counts, 256);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_mc_edges), edges, 256 * kMcRow);
}

int mc_blocks(const Grid &g) {
    const int64_t n = (int64_t)g.n[0] * g.n[1] * g.n[2];
    return (int)((n + kMcPerBlock - 1) / kMcPerBlock);
}

// Edge bits (bit a: grid edge (q, q + e_a) crosses the level) and the case of
// the cell with lower corner q (-1 when q is on the upper border).
__device__ __forceinline__ void mc_point(const float *__restrict__ A, const Grid &g, int qx, int qy,
                                         int qz, size_t l, float L, int &ebits, int &cs) {
    const size_t sy = g.n[0], sz = (size_t)g.n[0] * g.n[1];
    const bool in0 = A[l] > L;
    const bool hx = qx + 1 < g.n[0], hy = qy + 1 < g.n[1], hz = qz + 1 < g.n[2];
    ebits = 0;
    cs = -1;
    if (hx && hy && hz) {
        cs = in0 ? 1 : 0;
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            const size_t o = l + (k & 1) + ((k >> 1) & 1) * sy + ((k >> 2) & 1) * sz;
            cs |= (A[o] > L ? 1 : 0) << k;
        }
        ebits = (((cs >> 1) & 1) != (cs & 1) ? 1 : 0) | (((cs >> 2) & 1) != (cs & 1) ? 2 : 0) |
                (((cs >> 4) & 1) != (cs & 1) ? 4 : 0);
    } else {
        if (hx && ((A[l + 1] > L) != in0)) ebits |= 1;
        if (hy && ((A[l + sy] > L) != in0)) ebits |= 2;
        if (hz && ((A[l + sz] > L) != in0)) ebits |= 4;
    }
}

// Edge bits and cell cases of the 4 consecutive grid points (qx..qx+3, qy, qz)
// of one row (Nx % 4 == 0, qx % 4 == 0), from the 4 rows (y or y+1) x (z or
// z+1) loaded as one float4 plus the fifth value each.  a0[i] = A(qx+i, qy, qz),
// a1[a][i] = A at the far end of point i's edge along axis a (for vertices).
__device__ __forceinline__ void mc_quad(const float *__restrict__ A, const Grid &g, int qx, int qy,
                                        int qz, size_t l, float L, int eb[4], int cs[4],
                                        float a0[4], float a1[3][4]) {
    const size_t sy = g.n[0], sz = (size_t)g.n[0] * g.n[1];
    const bool hy = qy + 1 < g.n[1], hz = qz + 1 < g.n[2], hx4 = qx + 4 < g.n[0];
    float r[4][5];  // rows (dy, dz) = (0,0), (1,0), (0,1), (1,1)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool have = (k & 1 ? hy : true) && (k & 2 ? hz : true);
        const size_t o = l + (k & 1 ? sy : 0) + (k & 2 ? sz : 0);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        float e = 0.f;
        if (have) {
            v = *reinterpret_cast<const float4 *>(A + o);
            if (hx4) e = A[o + 4];
        }
        r[k][0] = v.x;
        r[k][1] = v.y;
        r[k][2] = v.z;
        r[k][3] = v.w;
        r[k][4] = e;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool hx = qx + i + 1 < g.n[0];
        a0[i] = r[0][i];
        a1[0][i] = r[0][i + 1];
        a1[1][i] = r[1][i];
        a1[2][i] = r[2][i];
        const bool in0 = r[0][i] > L;
        eb[i] = (hx && ((r[0][i + 1] > L) != in0) ? 1 : 0) | (hy && ((r[1][i] > L) != in0) ? 2 : 0) |
                (hz && ((r[2][i] > L) != in0) ? 4 : 0);
        cs[i] = -1;
        if (hx && hy && hz) {
            cs[i] = (in0 ? 1 : 0) | (r[0][i + 1] > L ? 2 : 0) | (r[1][i] > L ? 4 : 0) |
                    (r[1][i + 1] > L ? 8 : 0) | (r[2][i] > L ? 16 : 0) | (r[2][i + 1] > L ? 32 : 0) |
                    (r[3][i] > L ? 64 : 0) | (r[3][i + 1] > L ? 128 : 0);
        }
    }
}

__device__ __forceinline__ int block_sum(int v, int *red) {
    // 256 threads = 4 waves
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wid] = v;
    __syncthreads();
    const int t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}

// Blocks of the marching cubes whose cells' corner rows lie all above the
// level or all at or below it have no crossing edge and no active cell: one
// thread per block settles them from the per-row ranges of A (zero totals,
// the open-surface flag when above: every row has points on the x borders)
// and appends the others to `list` (st->mc_active entries, in no particular
// order).  The rows r0 .. r1 of a block's points and their cells' corners
// lie in rows r0 .. r1 + 1 and the same rows of the next plane (r + Ny).
// With the level's block partials given (psum not null), every block
// reduces them itself and block 0 publishes the level (the work of
// level_final_kernel, with the same bits); else the level is *level_f32.
__global__ void __launch_bounds__(kLevelThreads)
mc_classify_kernel(float *__restrict__ level_f32, const double *__restrict__ psum,
                   const int32_t *__restrict__ pcnt, int lnb, const float2 *__restrict__ rowmm, Grid g,
                   int nb, int32_t *__restrict__ blk_counts, int32_t *__restrict__ list, DevStatus *st) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    float L;
    if (psum) {
        double total;
        int count;
        level_reduce(psum, pcnt, lnb, total, count);
        L = level_publish(total, count, st, level_f32);
    } else {
        L = *level_f32;
    }
    bool active = false, inside = false;
    if (b < nb) {
        const size_t n = (size_t)g.n[0] * g.n[1] * g.n[2];
        const unsigned nrows = (unsigned)g.n[1] * g.n[2];
        const unsigned b0 = (unsigned)b * (unsigned)kMcPerBlock;
        const unsigned r0 = b0 / (unsigned)g.n[0];
        const unsigned r1 = (unsigned)((min((size_t)b0 + kMcPerBlock, n) - 1) / (unsigned)g.n[0]);
        const unsigned span = r1 - r0 + 2;
        float mn = INFINITY, mx = -INFINITY;
        for (unsigned i = 0; i < 2 * span; ++i) {
            const unsigned r = i < span ? r0 + i : r0 + (i - span) + (unsigned)g.n[1];
            if (r < nrows) {
                const float2 v = rowmm[r];
                mn = fminf(mn, v.x);
                mx = fmaxf(mx, v.y);
            }
        }
        if (mn > L || mx <= L) {
            blk_counts[3 * b + 0] = 0;
            blk_counts[3 * b + 1] = 0;
            blk_counts[3 * b + 2] = 0;
            inside = mn > L;
        } else {
            active = true;
        }
    }
    if (__ballot(inside) && lane == 0) atomicOr(&st->flags, kFlagOpen);
    // one list append per block: every block appends to the one counter at
    // about the same time, and fewer returning atomics queue on it than with
    // one per wave
    __shared__ int wcnt[kLevelThreads / 64], bbase;
    const unsigned long long m = __ballot(active);
    const int wid = threadIdx.x >> 6;
    if (lane == 0) wcnt[wid] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kLevelThreads / 64; ++w) tot += wcnt[w];
        bbase = tot ? atomicAdd(&st->mc_active, tot) : 0;
    }
    __syncthreads();
    if (active) {
        int base = bbase;
        for (int w = 0; w < wid; ++w) base += wcnt[w];
        list[base + __popcll(m & ((1ull << lane) - 1ull))] = b;
    }
}

// Classification of the blocks in `list` (st->mc_active of them; persistent
// blocks stride over the list), or of block blockIdx.x when list is null.
__global__ void __launch_bounds__(kMcThreads)
mc_count_kernel(const float *__restrict__ A, const float *__restrict__ level_f32,
                const int32_t *__restrict__ list, Grid g, int32_t *__restrict__ blk_counts,
                uint32_t *__restrict__ codes, uint8_t *__restrict__ cases_out, DevStatus *st) {
    __shared__ int red[4];
    __shared__ uint8_t s_ntri[256];
    const float L = *level_f32;
    const size_t n = (size_t)g.n[0] * g.n[1] * g.n[2];
    const int nblk = list ? st->mc_active : (int)gridDim.x;
    // this block's first list entry, loaded together with the list length
    // (the list has room for every block, so the entry exists; it is used
    // only when it is below the length)
    const unsigned first = list ? (unsigned)list[blockIdx.x] : (unsigned)blockIdx.x;
    if ((int)blockIdx.x >= nblk) return;
    mc_count_table(s_ntri);
    for (int it = blockIdx.x; it < nblk; it += gridDim.x) {
    const unsigned blk = it == (int)blockIdx.x ? first : (list ? (unsigned)list[it] : (unsigned)it);
    uint32_t code4 = 0;  // the 4 point codes, byte i for point l0 + i
    const unsigned l0u = blk * (unsigned)kMcPerBlock + threadIdx.x * (unsigned)kMcPpt;
    const size_t l0 = l0u;
    int nv = 0, nt = 0, na = 0;
    bool open = false;
    if (l0 < n) {
        const unsigned ru = l0u / (unsigned)g.n[0];
        int qx = (int)(l0u - ru * (unsigned)g.n[0]);
        int qz = (int)(ru / (unsigned)g.n[1]);
        int qy = (int)(ru - (unsigned)qz * (unsigned)g.n[1]);
        if ((g.n[0] & 3) == 0 && ((uintptr_t)A & 15) == 0) {
            // the 4 points share a row: vector loads of the 4 neighbouring rows
            int eb[4], cs[4];
            float a0[4], a1[3][4];
            mc_quad(A, g, qx, qy, qz, l0, L, eb, cs, a0, a1);
            const bool yzb = qy == 0 || qz == 0 || qy == g.n[1] - 1 || qz == g.n[2] - 1;
#pragma unroll
            for (int i = 0; i < kMcPpt; ++i) {
                nv += __popc(eb[i]);
                code4 |= (uint32_t)(cs[i] >= 0 ? cs[i] : eb[i]) << (8 * i);
                if (cs[i] >= 0) {
                    const int c = (int)s_ntri[cs[i]];
                    nt += c;
                    na += c > 0;
                    if (cases_out)
                        cases_out[qx + i + (size_t)(g.n[0] - 1) * (qy + (size_t)(g.n[1] - 1) * qz)] =
                            (uint8_t)cs[i];
                }
                const bool border = yzb || qx + i == 0 || qx + i == g.n[0] - 1;
                if (border && a0[i] > L) open = true;
            }
        } else {
#pragma unroll
            for (int i = 0; i < kMcPpt; ++i) {
                const size_t l = l0 + i;
                if (l < n) {
                    int eb, cs;
                    mc_point(A, g, qx, qy, qz, l, L, eb, cs);
                    nv += __popc(eb);
                    code4 |= (uint32_t)(cs >= 0 ? cs : eb) << (8 * i);
                    if (cs >= 0) {
                        const int c = (int)s_ntri[cs];
                        nt += c;
                        na += c > 0;
                        if (cases_out)
                            cases_out[qx + (size_t)(g.n[0] - 1) * (qy + (size_t)(g.n[1] - 1) * qz)] =
                                (uint8_t)cs;
                    }
                    const bool border = qx == 0 || qy == 0 || qz == 0 || qx == g.n[0] - 1 ||
                                        qy == g.n[1] - 1 || qz == g.n[2] - 1;
                    if (border && A[l] > L) open = true;
                }
                if (++qx == g.n[0]) {
                    qx = 0;
                    if (++qy == g.n[1]) {
                        qy = 0;
                        ++qz;
                    }
                }
            }
        }
    }
    if (__ballot(open) && (threadIdx.x & 63) == 0) atomicOr(&st->flags, kFlagOpen);
    nv = block_sum(nv, red);
    nt = block_sum(nt, red);
    na = block_sum(na, red);
    if (threadIdx.x == 0) {
        blk_counts[3 * blk + 0] = nv;
        blk_counts[3 * blk + 1] = nt;
        blk_counts[3 * blk + 2] = na;
    }
    // codes only where the surface passes: mc_generate skips the other blocks
    if (nv > 0 || na > 0) codes[l0 / 4] = code4;
    }
}

// Exclusive block scan of three counters (256 threads).
__device__ __forceinline__ void block_excl_scan3(int v[3], int *red /* [3][4] */) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        incl[c] = v[c];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl[c], d, 64);
            if (lane >= d) incl[c] += u;
        }
        if (lane == 63) red[c * 4 + wid] = incl[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int off = 0;
        for (int w = 0; w < wid; ++w) off += red[c * 4 + w];
        v[c] = off + incl[c] - v[c];
    }
    __syncthreads();
}

__device__ __forceinline__ bool mesh_fits(const DevStatus *st, const MeshCaps &caps) {
    return st->mc_total[0] <= caps.vertices && st->mc_total[1] <= caps.triangles &&
           st->mc_total[2] <= caps.cells && !(caps.check_invalid && (st->flags & kFlagInvalid));
}

// Derivative of A along axis b at grid point q (linear index l) by central
// differences, one-sided on the grid's outer layer (physical units).
__device__ __forceinline__ float grad_axis(const float *__restrict__ A, const Grid &g, size_t l,
                                           const int q[3], int b, float aq) {
    const size_t step = b == 0 ? 1 : b == 1 ? (size_t)g.n[0] : (size_t)g.n[0] * g.n[1];
    const bool lo = q[b] == 0, hi = q[b] == g.n[b] - 1;
    const float ap = hi ? aq : A[l + step];
    const float am = lo ? aq : A[l - step];
    return (ap - am) / ((lo || hi ? 1.0f : 2.0f) * g.h[b]);
}

// Output normal of the vertex on grid edge (q0, q0 + e_a) at parameter t:
// -grad A (A is larger inside), the gradients of the two ends interpolated
// linearly with t, normalised (zero where the interpolated gradient is).
__device__ void edge_normal(const float *__restrict__ A, const Grid &g, size_t l0, const int q0[3], int a,
                            size_t step, float a0, float a1, float t, float nv[3]) {
    const int q1[3] = {q0[0] + (a == 0), q0[1] + (a == 1), q0[2] + (a == 2)};
    float len2 = 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const float g0 = grad_axis(A, g, l0, q0, b, a0);
        const float g1 = grad_axis(A, g, l0 + step, q1, b, a1);
        nv[b] = -fmaf(t, g1 - g0, g0);
        len2 = fmaf(nv[b], nv[b], len2);
    }
    const float inv = len2 > 0.0f ? 1.0f / sqrtf(len2) : 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b) nv[b] *= inv;
}

__global__ void __launch_bounds__(kMcThreads)
mc_generate_kernel(const float *__restrict__ A, const float *__restrict__ level_f32, Grid g,
                   const int32_t *__restrict__ list, const int32_t *__restrict__ blk_counts,
                   const int32_t *__restrict__ blk_off, const uint32_t *__restrict__ codes,
                   float *__restrict__ verts, float *__restrict__ nrms, int32_t *__restrict__ vidx,
                   int4 *__restrict__ cells, const DevStatus *st, MeshCaps caps,
                   uint32_t *__restrict__ host_status) {
    __shared__ int red[12];
    __shared__ uint8_t s_ntri[256];
    __shared__ uint2 elist[3 * kMcPerBlock];  // the block's crossing edges, by vertex rank
    // The status block is final here (the mesh kernels only read it): block 0
    // copies it to the host (as status_publish_kernel does), and the stores'
    // latency hides behind the mesh work instead of costing a launch.
    if (host_status && blockIdx.x == 0) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(st);
        for (int i = threadIdx.x; i < (int)(sizeof(DevStatus) / 4); i += blockDim.x) host_status[i] = src[i];
    }
    // this block's first list entry, loaded together with the status (the
    // list has room for every block; the entry is used only below the length)
    const unsigned first = list ? (unsigned)list[blockIdx.x] : (unsigned)blockIdx.x;
    if (!mesh_fits(st, caps)) return;
    // the blocks in `list` (persistent blocks stride over it), or block
    // blockIdx.x when list is null
    const int nblk = list ? st->mc_active : (int)gridDim.x;
    const size_t n = (size_t)g.n[0] * g.n[1] * g.n[2];
    bool have_table = false;
    for (int it = blockIdx.x; it < nblk; it += gridDim.x) {
    const unsigned blk = it == (int)blockIdx.x ? first : (list ? (unsigned)list[it] : (unsigned)it);
    // the block's totals, offsets and codes in one round of loads.  A block
    // without vertices and active cells has nothing to write (and mc_count
    // stored no codes for it: the codes loaded then are stale and unused).
    const int bv = blk_counts[3 * blk], ba = blk_counts[3 * blk + 2];
    int vbase = blk_off[3 * blk + 0], tbase = blk_off[3 * blk + 1], abase = blk_off[3 * blk + 2];
    const unsigned l0u = blk * (unsigned)kMcPerBlock + threadIdx.x * (unsigned)kMcPpt;
    const size_t l0 = l0u;
    const uint32_t code_ld = l0 < n ? codes[l0u / 4] : 0u;
    if (bv == 0 && ba == 0) continue;
    if (!have_table) {
        mc_count_table(s_ntri);
        have_table = true;
    }
    const float L = *level_f32;
    int eb[kMcPpt], cs[kMcPpt];
    int cnt[3] = {0, 0, 0};
    int qx = 0, qy = 0, qz = 0;
    uint32_t code4 = 0;
    if (l0 < n) {
        const unsigned ru = l0u / (unsigned)g.n[0];
        qx = (int)(l0u - ru * (unsigned)g.n[0]);
        qz = (int)(ru / (unsigned)g.n[1]);
        qy = (int)(ru - (unsigned)qz * (unsigned)g.n[1]);
        code4 = code_ld;
    }
    {
        int x = qx, y = qy, z = qz;
#pragma unroll
        for (int i = 0; i < kMcPpt; ++i) {
            const int code = (int)((code4 >> (8 * i)) & 255u);
            eb[i] = 0;
            cs[i] = -1;
            if (l0 + i < n) {
                if (x + 1 < g.n[0] && y + 1 < g.n[1] && z + 1 < g.n[2]) {
                    // the case holds the corners at q and q + e_a
                    cs[i] = code;
                    eb[i] = ((code ^ (code >> 1)) & 1) | (((code ^ (code >> 2)) & 1) << 1) |
                            (((code ^ (code >> 4)) & 1) << 2);
                } else {
                    eb[i] = code & 7;
                }
            }
            if (++x == g.n[0]) {
                x = 0;
                if (++y == g.n[1]) {
                    y = 0;
                    ++z;
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kMcPpt; ++i) {
        cnt[0] += __popc(eb[i]);
        if (cs[i] >= 0) {
            const int c = (int)s_ntri[cs[i]];
            cnt[1] += c;
            cnt[2] += c > 0;
        }
    }
    const int vblk = vbase;  // the block's first vertex
    block_excl_scan3(cnt, red);
    tbase += cnt[1];
    abase += cnt[2];
    // this thread's crossing edges into the block's edge list, at their
    // vertex ranks within the block (order: linear index, axis)
    int k = cnt[0];
    int x = qx, y = qy, z = qz;
    for (int i = 0; i < kMcPpt; ++i) {
        const size_t l = l0 + i;
        if (l >= n) break;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if ((eb[i] >> a) & 1)
                elist[k++] = make_uint2((unsigned)l, (unsigned)x | ((unsigned)y << 10) | ((unsigned)z << 20) |
                                                         ((unsigned)a << 30));
        if (cs[i] >= 0) {
            const int c = (int)s_ntri[cs[i]];
            if (c > 0) {
                cells[abase] = make_int4((int)l, cs[i], tbase, 0);
                ++abase;
                tbase += c;
            }
        }
        if (++x == g.n[0]) {
            x = 0;
            if (++y == g.n[1]) {
                y = 0;
                ++z;
            }
        }
    }
    __syncthreads();
    // one vertex per thread (a listed block has a few dozen): the position
    // on its edge, its normal, and its id at the edge's slot
    for (int e = threadIdx.x; e < bv; e += blockDim.x) {
        const uint2 en = elist[e];
        const size_t l = en.x;
        const int ex = (int)(en.y & 1023u), ey = (int)((en.y >> 10) & 1023u), ez = (int)((en.y >> 20) & 1023u);
        const int a = (int)(en.y >> 30);
        const int vid = vblk + e;
        const size_t step = a == 0 ? 1 : a == 1 ? (size_t)g.n[0] : (size_t)g.n[0] * g.n[1];
        const float a0 = A[l], a1 = A[l + step];
        const float t = (L - a0) / (a1 - a0);
        float p[3] = {fmaf((float)ex + 0.5f, g.h[0], g.bmin[0]), fmaf((float)ey + 0.5f, g.h[1], g.bmin[1]),
                      fmaf((float)ez + 0.5f, g.h[2], g.bmin[2])};
        p[a] += t * g.h[a];
        verts[3 * (size_t)vid + 0] = p[0];
        verts[3 * (size_t)vid + 1] = p[1];
        verts[3 * (size_t)vid + 2] = p[2];
        if (nrms) {
            const int q0[3] = {ex, ey, ez};
            float nv[3];
            edge_normal(A, g, l, q0, a, step, a0, a1, t, nv);
            nrms[3 * (size_t)vid + 0] = nv[0];
            nrms[3 * (size_t)vid + 1] = nv[1];
            nrms[3 * (size_t)vid + 2] = nv[2];
        }
        vidx[3 * l + a] = vid;
    }
}
}

__global__ void __launch_bounds__(256)
mc_triangles_kernel(const int4 *__restrict__ cells, const int32_t *__restrict__ vidx, Grid g,
                    int32_t *__restrict__ tris, const DevStatus *st, MeshCaps caps) {
    if (!mesh_fits(st, caps)) return;
    const int n_cells = st->mc_total[2];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_cells; i += gridDim.x * blockDim.x) {
    const int4 c = cells[i];
    const size_t l = (size_t)(unsigned)c.x;
    const int cs = c.y;
    const size_t sy = g.n[0], sz = (size_t)g.n[0] * g.n[1];
    const int nt = c_mc_count[cs];
    for (int t = 0; t < nt; ++t) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int e = c_mc_edges[cs * kMcRow + 3 * t + j];
            const int axis = e >> 2, r = e & 3;
            // offsets of the edge's low corner on the two other axes (x<y<z order)
            const int o0 = axis == 0 ? 1 : 0, o1 = axis == 2 ? 1 : 2;
            int off[3] = {0, 0, 0};
            off[o0] = r & 1;
            off[o1] = r >> 1;
            const size_t lq = l + off[0] + off[1] * sy + off[2] * sz;
            tris[3 * ((size_t)c.z + t) + j] = vidx[3 * lq + axis];
        }
    }
    }
}

// Persistent grid of the list-driven marching-cubes kernels: the blocks
// the surface passes are a few percent of all (a 256^3 grid has 16k).
constexpr int kMcPersist = 2048;

hipError_t launch_mc_classify(float *level_f32, const double *psum, const int32_t *pcnt, int lnb,
                              const float2 *rowmm, const Grid &g, int32_t *blk_counts, int32_t *list,
                              DevStatus *st, hipStream_t s) {
    const int nb = mc_blocks(g);
    mc_classify_kernel<<<dim3((nb + kLevelThreads - 1) / kLevelThreads), dim3(kLevelThreads), 0, s>>>(
        level_f32, psum, pcnt, lnb, rowmm, g, nb, blk_counts, list, st);
    return hipGetLastError();
}

static int mc_grid(const Grid &g, const int32_t *list) {
    return list ? std::min(mc_blocks(g), kMcPersist) : mc_blocks(g);
}

hipError_t launch_mc_count(const float *A, const float *level_f32, const int32_t *list, const Grid &g,
                           int32_t *blk_counts, uint32_t *codes, uint8_t *cases_out, DevStatus *st,
                           hipStream_t s) {
    mc_count_kernel<<<dim3(mc_grid(g, list)), dim3(kMcThreads), 0, s>>>(A, level_f32, list, g, blk_counts,
                                                                        codes, cases_out, st);
    return hipGetLastError();
}

hipError_t launch_mc_generate(const float *A, const float *level_f32, const int32_t *list, const Grid &g,
                              const int32_t *blk_counts, const int32_t *blk_offsets,
                              const uint32_t *codes, float *verts, float *normals, int32_t *vidx,
                              int4 *cells, const DevStatus *st, MeshCaps caps, DevStatus *host_status,
                              hipStream_t s) {
    mc_generate_kernel<<<dim3(mc_grid(g, list)), dim3(kMcThreads), 0, s>>>(
        A, level_f32, g, list, blk_counts, blk_offsets, codes, verts, normals, vidx, cells, st, caps,
        reinterpret_cast<uint32_t *>(host_status));
    return hipGetLastError();
}

hipError_t launch_mc_triangles(const int4 *cells, const int32_t *vidx, const Grid &g, int32_t *tris,
                               const DevStatus *st, MeshCaps caps, hipStream_t s) {
    // a grid-stride loop over the active cells: blocks beyond the count only
    // read the status and exit, so the grid stays moderate
    const long long want = (caps.cells + 255) / 256;
    const int blocks = (int)std::max(1LL, std::min(want, 1024LL));
    mc_triangles_kernel<<<dim3(blocks), dim3(256), 0, s>>>(cells, vidx, g, tris, st, caps);
    return hipGetLastError();
}

}  // namespace fvr
