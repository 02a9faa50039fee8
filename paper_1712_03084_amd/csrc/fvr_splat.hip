// Weighted Gaussian splat (eqs. (1)-(2), Sec. III-B) fused with the forward
// real FFT along x, for gfx950.
//
// Each point spreads its weighted normal W N over the 4^3 voxels around it
// with g(.; sigma1) and its weight W with g(.; sigma2):
//   S_c(q) = sum_i g(|X_i - p(q)|; sigma1) W_i N_ic,  D(q) = sum_i g(|X_i - p(q)|; sigma2) W_i
// and V = S / D (0 where D = 0); w = W / d(q) of eq. (1) depends on the point
// only through W, so 1/d(q) factors out of the sum.  g is separable, so per
// point the kernel evaluates 4 factors per axis and Gaussian, not 64.
//
// Data flow (no global atomics on the field, no V round trip through HBM):
//   bin_count   validate, reject points outside the bbox, key = (y, z) row of
//               the footprint origin, histogram with a per-bin arrival rank
//   scan        bin offsets
//   bin_scatter packed 32-byte records (x, y, z, W | W N) in bin order
//   tile_list   tiles of ty x tz full x-rows that some point reaches, and
//               their occupancy flags (the later passes skip the others)
//   splat_fft_x persistent blocks claim the busy tiles: a tile gathers the
//               points of the (ty+3) x (tz+3) bins whose footprints reach it,
//               accumulates S and D in LDS, forms V, runs the real FFT of
//               every x-row in LDS and writes the three half-spectrum planes
//               (the x component times j w_x).
#include <algorithm>

#include "fvr_common.h"
#include "fvr_fft_engine.h"
#include "fvr_scan.h"

namespace fvr {

constexpr int kSplatThreads = 512;
constexpr int kSplatMaxPlane = 2048;  // voxels per channel plane of a tile, at most
constexpr int kMaxBins = 128;   // (ty+3)(tz+3) footprint-origin bins per tile, at most
constexpr int kChunkPts = 8;    // consecutive points of a bin per splat work item
constexpr int kUnitBits = 48;   // a term is below 2^48 units; a run of kChunkPts below 2^51

// Footprint origin floor((x - bmin)/h - 1/2) in float32, each operation
// correctly rounded (no contraction), so every implementation that follows
// this formula picks the same voxels.
__device__ __forceinline__ float voxel_coord(float x, float bmin, float h) {
    return __fsub_rn(__fdiv_rn(__fsub_rn(x, bmin), h), 0.5f);
}

// Exact, order-independent fixed-point accumulation in f64 registers.
// A run accumulator holds kBias + x, where x is an integer count of the
// tile's unit.  A run adds at most kChunkPts = 8 terms t with |t| < 2^48
// units, so before each addition |x| <= 7 * 2^48 and |x + t| < 2^51: the
// exact value kBias + x + t lies in [2^52, 2^53], where the representable
// doubles are exactly the integers.  A term t = g s is added with one fused
// multiply-add, which rounds kBias + x + t once to the nearest integer.  The
// factor s is given an odd 53-bit significand (lowest bit set: a relative
// change of 2^-53): g = a 2^i, s = b 2^j with a, b odd and b >= 2^52, so if
// t = ab 2^(i+j) were an odd multiple of 1/2, i + j = -1 and |t| >= 2^51.
// For |t| < 2^48 the sum is therefore never halfway between two integers:
// the result is kBias + x + nearest(t) whatever x is.  Every
// term is therefore rounded on its own, and the sums are exact integers,
// independent of the order of the points (bit-reproducible).
constexpr double kBias = 6755399441055744.0;  // 1.5 * 2^52
constexpr int kBiasHi = 0x43380000;           // high word of kBias; its low word is 0

__device__ __forceinline__ double odd_significand(double x) {
    return __hiloint2double(__double2hiint(x), __double2loint(x) | 1);
}

// The integer x of a run accumulator kBias + x as a two's-complement int64:
// the low words agree, and the high word differs by kBias's alone.
__device__ __forceinline__ unsigned long long run_value(double a) {
    const unsigned lo = (unsigned)__double2loint(a);
    const unsigned hi = (unsigned)(__double2hiint(a) - kBiasHi);
    return ((unsigned long long)hi << 32) | lo;
}

// Exponent e of the frame's fixed-point scale for a maximum mx >= 0:
// mx < (1 - 2^-10) 2^e.  A term's Gaussian factors are products of rounded
// exponentials (a few float32 ulps above 1 at most), so the headroom keeps
// every term below 2^E_t units.
__device__ __forceinline__ int unit_exp(float mx) {
    int e;
    const float fr = frexpf(mx, &e);
    return fr >= 1.0f - 0x1p-10f ? e + 1 : e;
}

// Nearest voxel centre of x (the non-weighted splat): the cell containing
// the point, floor((x - bmin)/h) in float32 with each operation correctly
// rounded, clamped to the grid.
__device__ __forceinline__ int nearest_voxel(float x, float bmin, float h, int n) {
    const int i = (int)floorf(__fdiv_rn(__fsub_rn(x, bmin), h));
    return min(max(i, 0), n - 1);
}

// An int64 to float via double: hi 2^32 + lo is exact in double while |x| <
// 2^53 and is then rounded once (a few instructions against the long
// integer sequence of a direct int64 to float conversion).
__device__ __forceinline__ float i64_to_float(long long x) {
    const double hi = (double)(int)(x >> 32), lo = (double)(unsigned)(x & 0xffffffffll);
    return (float)fma(hi, 4294967296.0, lo);
}

__device__ __forceinline__ bool finite3(float a, float b, float c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// 1024 points per block: the block's groups of equal bin share one atomic
// (61k atomics for the 700k-point proxy frame, 126k with 256-point blocks)
constexpr int kBinThreads = 1024;

__global__ void __launch_bounds__(kBinThreads)
bin_count_kernel(const float *__restrict__ pts, const float *__restrict__ nrm,
                 const float *__restrict__ w, int m, Grid g, int nearest, int32_t *__restrict__ bin_count,
                 int32_t *__restrict__ key, int32_t *__restrict__ rank, uint2 *__restrict__ blk_max,
                 DevStatus *st) {
    constexpr int kHash = 2 * kBinThreads;  // power of two, twice the block: probing always ends
    static_assert(kHash == 1 << 11, "hash width");
    __shared__ int hkey[kHash], hcnt[kHash], hbase[kHash];             // bins
    __shared__ int gkey[kHash], gcnt[kHash], goff[kHash], gbin[kHash];  // (bin, i0_x) pairs
    // cleared first: the stores overlap the loads of the points
    for (int t = threadIdx.x; t < kHash; t += blockDim.x) {
        hkey[t] = -1;
        hcnt[t] = 0;
        gkey[t] = -1;
        gcnt[t] = 0;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool bad = false, rej = false;
    int k = -1, kx = 0;  // bin, and the footprint x origin i0_x + 1
    float wmax = 0.0f, wnmax = 0.0f;
    if (i < m) {
        const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        const float nx = nrm[3 * i], ny = nrm[3 * i + 1], nz = nrm[3 * i + 2];
        const float wi = w ? w[i] : 1.0f;
        bad = !(finite3(x, y, z) && finite3(nx, ny, nz) && isfinite(wi) && wi >= 0.0f);
        if (!bad) {
            const bool acc = x >= g.bmin[0] && x <= g.bmax[0] && y >= g.bmin[1] &&
                             y <= g.bmax[1] && z >= g.bmin[2] && z <= g.bmax[2];
            if (acc) {
                // the nearest-voxel splat sums unweighted normals: W = 1 there
                const float wu = nearest ? 1.0f : wi;
                wmax = wu;
                wnmax = wu * fmaxf(fabsf(nx), fmaxf(fabsf(ny), fabsf(nz)));
                int ix, iy, iz;
                if (nearest) {
                    ix = nearest_voxel(x, g.bmin[0], g.h[0], g.n[0]);
                    iy = nearest_voxel(y, g.bmin[1], g.h[1], g.n[1]);
                    iz = nearest_voxel(z, g.bmin[2], g.h[2], g.n[2]);
                } else {
                    ix = (int)floorf(voxel_coord(x, g.bmin[0], g.h[0]));
                    iy = (int)floorf(voxel_coord(y, g.bmin[1], g.h[1]));
                    iz = (int)floorf(voxel_coord(z, g.bmin[2], g.h[2]));
                    ix = min(max(ix, -1), g.n[0] - 1);
                    iy = min(max(iy, -1), g.n[1] - 1);
                    iz = min(max(iz, -1), g.n[2] - 1);
                }
                k = (iz + 1) * (g.n[1] + 1) + (iy + 1);
                kx = ix + 1;
            } else {
                rej = true;
            }
        }
    }
    // Block-aggregated histogram whose ranks group a bin's points by i0_x.
    // Points arrive in capture (scanline) order, so a block holds few
    // distinct bins, and the points of one bin and i0_x reach the same 4^3
    // voxels: placed next to each other, the splat sums them in registers
    // before one LDS atomic per voxel (a proxy frame's runs grow from 1.4 to
    // 2.3 points).  Each point claims its (bin, i0_x) pair in one LDS hash
    // table (its offset within the block's points of the pair); a thread per
    // distinct pair places the pair within the block's share of its bin in a
    // second table (offset within the bin); a thread per distinct bin adds
    // the block's count with a single global atomic - the global traffic of
    // a plain per-bin histogram - and a point's rank is the sum of the three
    // offsets.
    __syncthreads();
    const int nxk = g.n[0] + 1;
    const int k2 = k >= 0 ? k * nxk + kx : -1;  // < 513^3 < 2^31
    auto probe = [](int *keys, int key) {
        unsigned h = ((unsigned)key * 2654435761u) >> (32 - 11);  // log2(kHash) bits
        for (;;) {
            const int prev = atomicCAS(&keys[h], -1, key);
            if (prev == -1 || prev == key) return (int)h;
            h = (h + 1) & (kHash - 1);
        }
    };
    // the lanes of a wave mostly hold distinct pairs, so their table
    // atomics rarely meet on one address
    int gslot = 0, myoff = 0;
    if (k2 >= 0) {
        gslot = probe(gkey, k2);
        myoff = atomicAdd(&gcnt[gslot], 1);
        gbin[gslot] = k;  // every point of the pair stores the same bin
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kHash; t += blockDim.x) {
        if (gkey[t] >= 0) {
            const int slot = probe(hkey, gbin[t]);
            gbin[t] = slot;
            goff[t] = atomicAdd(&hcnt[slot], gcnt[t]);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kHash; t += blockDim.x) {
        const int kk = hkey[t];
        if (kk >= 0) hbase[t] = atomicAdd(&bin_count[kk], hcnt[t]);
    }
    __syncthreads();
    const int myrank = k2 >= 0 ? hbase[gbin[gslot]] + goff[gslot] + myoff : 0;
    if (i < m) {
        key[i] = k;
        if (k >= 0) rank[i] = myrank;
    }
    const unsigned long long brej = __ballot(rej), bbad = __ballot(bad);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        wmax = fmaxf(wmax, __shfl_xor(wmax, d, 64));
        wnmax = fmaxf(wnmax, __shfl_xor(wnmax, d, 64));
    }
    __shared__ float red[2][kBinThreads / 64];
    const int wid = threadIdx.x >> 6;
    if (lane == 0) {
        if (brej) atomicAdd(&st->rejected, (uint32_t)__popcll(brej));
        if (bbad) atomicOr(&st->flags, kFlagInvalid);
        red[0][wid] = wmax;
        red[1][wid] = wnmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the block's maxima; tile_order reduces them (atomics of every block on
        // one status word would serialise in one L2 channel); non-negative
        // floats order like their bit patterns
        float bw = 0.0f, bn = 0.0f;
        for (int w = 0; w < kBinThreads / 64; ++w) {
            bw = fmaxf(bw, red[0][w]);
            bn = fmaxf(bn, red[1][w]);
        }
        blk_max[blockIdx.x] = make_uint2(__float_as_uint(bw), __float_as_uint(bn));
    }
}

// Record of a binned point: (f_x, f_y, f_z, W), (W N_x, W N_y, W N_z, i0_x),
// W and W N_c in the frame's fixed-point scale (below 2^kUnitBits),
// with i0 = floor(v) the footprint origin chosen by the float32 formula for
// v = (X - bmin)/h - 1/2 above, and f = v - i0 the point's offset from that
// origin's centre in voxels, evaluated in f64 (h = (bmax - bmin)/N in f64)
// and rounded once to float32.  A float32 v carries an absolute error of up
// to 2^-16 voxels at N = 512, which the Gaussians would turn into relative
// errors of order 1e-5 in V; the f64 offset keeps only float32's own relative
// rounding of f.  The (i0_y, i0_z) pair is the record's bin; i0_x travels as
// integer bits.
__global__ void __launch_bounds__(256)
bin_scatter_kernel(const float *__restrict__ pts, const float *__restrict__ nrm,
                   const float *__restrict__ w, int m, Grid g, const int32_t *__restrict__ key,
                   const int32_t *__restrict__ rank, const int32_t *__restrict__ bin_off,
                   const DevStatus *__restrict__ st, int nearest, float4 *__restrict__ rec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int k = key[i];
    if (k < 0) return;
    const int pos = bin_off[k] + rank[i];
    // W and W N_c in the frame's fixed-point scale: the largest becomes
    // < 2^kUnitBits (ldexp scales exactly, whatever the exponent)
    const int sw = kUnitBits - unit_exp(__uint_as_float(st->wmax_bits));
    const int sn = kUnitBits - unit_exp(__uint_as_float(st->wnmax_bits));
    if (nearest) {
        // one unit per point and its normal as given, at its nearest voxel
        const float x = pts[3 * i];
        rec[2 * pos] = make_float4(0.0f, 0.0f, 0.0f, ldexpf(1.0f, sw));
        rec[2 * pos + 1] = make_float4(ldexpf(nrm[3 * i], sn), ldexpf(nrm[3 * i + 1], sn),
                                       ldexpf(nrm[3 * i + 2], sn),
                                       __int_as_float(nearest_voxel(x, g.bmin[0], g.h[0], g.n[0])));
        return;
    }
    const float wi = w ? w[i] : 1.0f;
    float f[3];
    int ix = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float x = pts[3 * i + a];
        const float fl = floorf(voxel_coord(x, g.bmin[a], g.h[a]));
        const double h64 = ((double)g.bmax[a] - (double)g.bmin[a]) / (double)g.n[a];
        f[a] = (float)(((double)x - (double)g.bmin[a]) / h64 - 0.5 - (double)fl);
        if (a == 0) ix = (int)fl;
    }
    rec[2 * pos] = make_float4(f[0], f[1], f[2], ldexpf(wi, sw));
    rec[2 * pos + 1] = make_float4(ldexpf(wi * nrm[3 * i], sn), ldexpf(wi * nrm[3 * i + 1], sn),
                                   ldexpf(wi * nrm[3 * i + 2], sn), __int_as_float(ix));
}

// Forward transform along x of the tile's ncx complex rows of length
// N = 16 P in LDS (split complex: row j's real parts at S[2 N j + e], its
// imaginary parts N floats later), for the register-pencil lengths.  Four
// steps on N = P x 16: lane n2 of a row takes x[16 n1 + n2] over n1, a
// length-P DFT, and the twiddles w_N^(n2 k1); the values go through the
// exchange area X (pitch P + 1: both of its accesses are conflict-free);
// lane k1 then takes a length-16 DFT over n2, giving X[k1 + P k2].  All
// index arithmetic is shifts and masks; the transformed rows replace the
// input in S.  Synchronises on entry and on return.
template <int P>
__device__ __forceinline__ void splat_rows_fft16(float *__restrict__ S, float2 *__restrict__ X, int ncx,
                                                 const float2 *__restrict__ twl) {
    constexpr int N = 16 * P;
    __syncthreads();
    for (int i = threadIdx.x; i < ncx * 16; i += blockDim.x) {
        const int j = i >> 4, n2 = i & 15;
        const float *re = S + 2 * N * j, *im = re + N;
        float2 v[P];
#pragma unroll
        for (int n1 = 0; n1 < P; ++n1) v[n1] = make_float2(re[16 * n1 + n2], im[16 * n1 + n2]);
        if constexpr (P > 1) Dft<P>::run(v, -1);
        float2 *x = X + (16 * j + n2) * (P + 1);
        x[0] = v[0];
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) x[k1] = cmul(v[k1], twl[n2 * k1]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ncx * P; i += blockDim.x) {
        const int j = i / P, k1 = i % P;
        float2 v[16];
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) v[n2] = X[(16 * j + n2) * (P + 1) + k1];
        Dft<16>::run(v, -1);
        float *re = S + 2 * N * j, *im = re + N;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            re[k1 + P * k2] = v[k2].x;
            im[k1 + P * k2] = v[k2].y;
        }
    }
    __syncthreads();
}

// Accumulation is in 64-bit fixed point with integer LDS atomics (gfx950's
// LDS float atomics run ~30x slower than its integer ones, and integer sums
// do not depend on the order of the additions).  The unit of a tile is
// 2^(e - E_t), where (1 - 2^-10) 2^e bounds the frame's largest |W N_c| (or
// W) and
// E_t = min(48, 62 - ceil(log2 N_t)) for the N_t points of the tile's bins:
// every term is below 2^E_t units, a run of at most kChunkPts terms below
// 2^51, and no voxel sum can exceed 2^62.  Each term is rounded to the unit
// on its own (f64 run sums above), so a term's error is at most half a unit,
// 2^-49 of the frame's largest term while N_t <= 2^14.  The sums are exact, hence independent
// of the order of the additions: the splat is bit-reproducible.
// V = (sigma2/sigma1) (S unit_S) / (D unit_D); the tile's 2^E_t cancels.
// Work decomposition: the candidate points of a tile come in bins of equal
// footprint origin (i0_y, i0_z), and all points of one bin reach the same
// in-tile rows.  The block enumerates (bin, chunk of up to kChunkPts
// consecutive points, row) items - only rows that exist in the tile.  Per
// point an item spends 6 exponentials on its 4 x-voxels of the row: the
// (y, z) factor of each Gaussian and, per Gaussian, the x factor at the first
// centre and its ratio to the next (the later x factors follow by products).
template <bool kNearest>
__global__ void __launch_bounds__(kSplatThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
splat_fft_x_kernel(const float4 *__restrict__ rec, const int32_t *__restrict__ bin_off, Grid g,
                   SplatConsts sc, FftAxis ax, DevStatus *__restrict__ st,
                   const int32_t *__restrict__ list, void *__restrict__ spec,
                   float *__restrict__ v_out) {
    extern __shared__ unsigned long long acc[];
    __shared__ int b_start[kMaxBins], b_pre[kMaxBins + 1], b_rows[kMaxBins], b_ny[kMaxBins];
    __shared__ int b_cnt[kMaxBins];
    __shared__ int b_qy[kMaxBins], b_qz[kMaxBins], b_iy[kMaxBins], b_iz[kMaxBins];
    __shared__ unsigned b_mrows[kMaxBins], b_mny[kMaxBins];

    __shared__ int s_tile, s_npts;
    const int Nx = g.n[0], Ny = g.n[1], Nz = g.n[2];
    const int TY = sc.ty, TZ = sc.tz, R = TY * TZ;
    const int nbusy = st->n_busy;
    const int plane = R * Nx;  // voxels per channel plane
    // int64 accumulator rows hold x = -2 .. Nx + 2 (voxel x at x + 2): a
    // footprint reaches x = i0_x - 1 .. i0_x + 2 with i0_x in [-1, Nx - 1], so
    // a flush needs no bounds test; contributions to the pad voxels are
    // dropped.  The pitch Nx + 5 is odd: with Nx a multiple of the bank count,
    // an even pitch would put a voxel's bank on x alone, and the points of a
    // tile cluster in x (the surface crossings).
    const int P = Nx + 5, aplane = R * P;
    const int H = g.H, Hp = g.Hp;
    const size_t pl = (size_t)Nz * Ny * Hp;
    float2 *twl = reinterpret_cast<float2 *>(acc + 4 * aplane);
    load_twiddles(twl, ax);
    // the records carry W and W N_c scaled by 2^(kUnitBits - e) (e from the
    // frame maxima); a tile scales its terms by a further 2^(E_t - kUnitBits)
    const int eS = unit_exp(__uint_as_float(st->wnmax_bits));
    const int eD = unit_exp(__uint_as_float(st->wmax_bits));
    const float k1 = exp2f(2.0f * sc.e1[0]), k2 = exp2f(2.0f * sc.e2[0]);

    // Persistent blocks claim the busy tiles from a ticket counter; block b
    // starts with tile b of the list without a counter round trip, and the
    // counter hands out the tickets from gridDim.x on.
    bool first_tile = true;
    for (;;) {
    if (threadIdx.x == 0)
        s_tile = first_tile ? (int)blockIdx.x : (int)gridDim.x + (int)atomicAdd(&st->tile_ticket, 1);
    first_tile = false;
    __syncthreads();
    const int ticket = s_tile;
    if (ticket >= nbusy) break;
    const int tile = list[ticket];
    const int by = tile % sc.tiles_y, bz = tile / sc.tiles_y;
    const int y0 = by * TY, z0 = bz * TZ;

    // bins of origin rows (iy, iz) whose rows i + fp_lo .. i + fp_hi overlap
    // the tile (4-row footprints: iy in [y0-2, y0+TY], clipped to [-1, N-1];
    // nearest voxels: the tile's own rows)
    const int flo = sc.fp_lo, fhi = sc.fp_hi;
    const int iz_lo = max(z0 - fhi, -1), iz_hi = min(z0 + TZ - 1 - flo, Nz - 1);
    const int iy_lo = max(y0 - fhi, -1), iy_hi = min(y0 + TY - 1 - flo, Ny - 1);
    const int nby = iy_hi - iy_lo + 1, nbins = nby * (iz_hi - iz_lo + 1);
    for (int t = threadIdx.x; t < nbins; t += blockDim.x) {
        const int iy = iy_lo + t % nby, iz = iz_lo + t / nby;
        const int kb = (iz + 1) * (Ny + 1) + (iy + 1);
        const int qy0 = max(iy + flo, y0), qy1 = min(min(iy + fhi, y0 + TY - 1), Ny - 1);
        const int qz0 = max(iz + flo, z0), qz1 = min(min(iz + fhi, z0 + TZ - 1), Nz - 1);
        const int ny = max(qy1 - qy0 + 1, 0), nz = max(qz1 - qz0 + 1, 0);
        const int cnt = bin_off[kb + 1] - bin_off[kb];
        const int nchunk = (cnt + kChunkPts - 1) / kChunkPts;
        b_start[t] = bin_off[kb];
        b_cnt[t] = cnt;
        b_rows[t] = ny * nz;
        b_ny[t] = max(ny, 1);
        b_qy[t] = qy0;
        b_qz[t] = qz0;
        b_iy[t] = iy;
        b_iz[t] = iz;
        b_mrows[t] = div_magic(max(ny * nz, 1));
        b_mny[t] = div_magic(max(ny, 1));
        b_pre[t + 1] = nchunk * ny * nz;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // inclusive prefix of the bins' item counts (nbins <= 128: two per
        // lane), and the tile's point count N_t
        const int l = threadIdx.x;
        const int v0 = 2 * l < nbins ? b_pre[2 * l + 1] : 0;
        const int v1 = 2 * l + 1 < nbins ? b_pre[2 * l + 2] : 0;
        int npts = (2 * l < nbins ? b_cnt[2 * l] : 0) + (2 * l + 1 < nbins ? b_cnt[2 * l + 1] : 0);
        int incl = v0 + v1;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl, d, 64);
            if (l >= d) incl += u;
            npts += __shfl_xor(npts, d, 64);
        }
        const int excl = incl - v0 - v1;
        if (2 * l < nbins) b_pre[2 * l + 1] = excl + v0;
        if (2 * l + 1 < nbins) b_pre[2 * l + 2] = excl + v0 + v1;
        if (l == 0) {
            b_pre[0] = 0;
            s_npts = npts;
        }
    }
    __syncthreads();
    const int total = b_pre[nbins];
    // the tile's exponent E_t: N_t terms of at most 2^E_t units stay below 2^62
    const int e_t = min(kUnitBits, 62 - (32 - __clz(max(s_npts - 1, 0))));
    const float qt = ldexpf(1.0f, e_t - kUnitBits);
    if (total == 0) {  // not in the busy list; kept for safety
        __syncthreads();
        continue;
    }
    for (int i = threadIdx.x; i < 4 * aplane; i += blockDim.x) acc[i] = 0ull;
    __syncthreads();

    // item of this thread's k-th iteration, or -1 when it has no more.  The
    // threads take consecutive items, so neighbouring lanes mostly hold the
    // rows of one chunk: they read the same records and add into different
    // accumulator rows.  (Lanes owning far-apart ranges of the item list
    // measured 106.6 against 103 us on the proxy frame.)
    auto item = [&](int k) -> int {
        const int j = k * (int)blockDim.x + threadIdx.x;
        return j < total ? j : -1;
    };

    // A lane's items increase monotonically, so it keeps the decode parameters
    // of its current bin in registers and reads the bin tables only when it
    // moves to a later bin.  (An LDS read in the steady-state loop would wait
    // for the previous item's queued atomics: LDS operations retire in order.)
    struct BinState {
        int b, lo, hi, start, cnt, rows, ny, qy0, qz0, iy, iz;
        unsigned mrows, mny;
    };
    auto enter_bin = [&](BinState &st, int b) {
        st.b = b;
        st.lo = b_pre[b];
        st.hi = b_pre[b + 1];
        st.start = b_start[b];
        st.cnt = b_cnt[b];
        st.rows = b_rows[b];
        st.ny = b_ny[b];
        st.qy0 = b_qy[b];
        st.qz0 = b_qz[b];
        st.iy = b_iy[b];
        st.iz = b_iz[b];
        st.mrows = b_mrows[b];
        st.mny = b_mny[b];
    };
    BinState bs;
    int j = item(0), k = 0;
    if (j >= 0) {
        int lo = 0, hi = nbins - 1;  // last bin with b_pre[bin] <= j
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b_pre[mid] <= j) lo = mid; else hi = mid - 1;
        }
        enter_bin(bs, lo);
    }
    // decode item jj (in bin bs, advancing it as needed): its chunk of points
    // [p, p + len) and its row (qy, qz)
    auto decode = [&](int jj, int &p, int &len, int &qy, int &qz, int &iy, int &iz) {
        while (jj >= bs.hi) enter_bin(bs, bs.b + 1);
        const int local = jj - bs.lo;
        const int ci = udiv(local, bs.rows, bs.mrows);
        const int r = local - ci * bs.rows;
        const int rzi = udiv(r, bs.ny, bs.mny);
        p = bs.start + ci * kChunkPts;
        len = min(kChunkPts, bs.cnt - ci * kChunkPts);
        qz = bs.qz0 + rzi;
        qy = bs.qy0 + (r - rzi * bs.ny);
        iy = bs.iy;
        iz = bs.iz;
    };

    // Points of one chunk that share a footprint cell (consecutive equal i0_x;
    // capture order keeps neighbouring samples together) are summed in f64
    // run accumulators (exact integers, see odd_significand) and reach LDS as
    // one atomic per voxel and channel when the cell changes.
    double run[4][4];
    int run_ix = 0, run_row = 0;
    auto flush = [&]() {
        const int l = run_row * P + run_ix + 1;  // voxel x = run_ix - 1 in the padded row
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int ox = 0; ox < 4; ++ox) {
                if (kNearest && ox != 1) continue;  // the point's own voxel x = run_ix only
                atomicAdd(&acc[c * aplane + l + ox], run_value(run[ox][c]));
                run[ox][c] = kBias;
            }
    };
#pragma unroll
    for (int ox = 0; ox < 4; ++ox)
#pragma unroll
        for (int c = 0; c < 4; ++c) run[ox][c] = kBias;

    while (j >= 0) {
        int p, len, qy, qz, iy, iz;
        decode(j, p, len, qy, qz, iy, iz);
        const int row = (qz - z0) * TY + (qy - y0);
        float4 r0 = rec[2 * p], r1 = rec[2 * p + 1];
        run_ix = __float_as_int(r1.w);
        run_row = row;
        for (int t = 0; t < len; ++t) {
            float4 n0 = r0, n1 = r1;
            if (t + 1 < len) {  // prefetch the chunk's next record
                n0 = rec[2 * (p + t + 1)];
                n1 = rec[2 * (p + t + 1) + 1];
            }
            const int ix = __float_as_int(r1.w);
            if (ix != run_ix) {
                flush();
                run_ix = ix;
            }
            if (kNearest) {
                // the non-weighted splat: the normal and one count, at the
                // point's nearest voxel (run slot ox = 1 is voxel x = i0_x);
                // adding an odd-significand s below 2^48 rounds as g s does
                run[1][0] += odd_significand((double)r1.x);
                run[1][1] += odd_significand((double)r1.y);
                run[1][2] += odd_significand((double)r1.z);
                run[1][3] += odd_significand((double)r0.w);
                r0 = n0;
                r1 = n1;
                continue;
            }
            // offsets of this row's centre from the point, in voxels
            const float dy = r0.y + (float)(iy - qy);
            const float dz = r0.z + (float)(iz - qz);
            const float a1 = __builtin_amdgcn_exp2f(sc.e1[1] * dy * dy + sc.e1[2] * dz * dz) * qt;
            const float a2 = __builtin_amdgcn_exp2f(sc.e2[1] * dy * dy + sc.e2[2] * dz * dz) * qt;
            const double sx = odd_significand((double)(a1 * r1.x));
            const double sy = odd_significand((double)(a1 * r1.y));
            const double sz = odd_significand((double)(a1 * r1.z));
            const double sd = odd_significand((double)(a2 * r0.w));
            // x factors at the 4 centres ox - 1, offsets d = fx + 1 - ox:
            // 2^(e (d-1)^2) = 2^(e d^2) 2^(e (1 - 2d)), and that ratio gains 2^(2e) per step
            const float d0 = r0.x + 1.0f;
            float g1 = __builtin_amdgcn_exp2f(sc.e1[0] * d0 * d0);
            float g2 = __builtin_amdgcn_exp2f(sc.e2[0] * d0 * d0);
            float h1 = __builtin_amdgcn_exp2f(sc.e1[0] * (1.0f - 2.0f * d0));
            float h2 = __builtin_amdgcn_exp2f(sc.e2[0] * (1.0f - 2.0f * d0));
#pragma unroll
            for (int ox = 0; ox < 4; ++ox) {
                const double G1 = (double)g1, G2 = (double)g2;
                run[ox][0] = fma(G1, sx, run[ox][0]);
                run[ox][1] = fma(G1, sy, run[ox][1]);
                run[ox][2] = fma(G1, sz, run[ox][2]);
                run[ox][3] = fma(G2, sd, run[ox][3]);
                if (ox < 3) {
                    g1 *= h1;
                    g2 *= h2;
                    h1 *= k1;
                    h2 *= k2;
                }
            }
            r0 = n0;
            r1 = n1;
        }
        flush();
        j = item(++k);
    }
    __syncthreads();

    // V = (sigma2/sigma1) 2^(eS - eD) S / D, 0 where D = 0; converted in
    // registers first, then written as float planes over the front of the
    // accumulator buffer (the float rows overlap int64 slots still unread by
    // other threads, hence the barrier in between)
    constexpr int kVpt = kSplatMaxPlane / kSplatThreads;
    float vv[kVpt][3];
    const float ratio = sc.vscale * ldexpf(1.0f, eS - eD);
#pragma unroll
    for (int t = 0; t < kVpt; ++t) {
        const int l = threadIdx.x + t * blockDim.x;
        vv[t][0] = vv[t][1] = vv[t][2] = 0.f;
        if (l < plane) {
            const int row = l / Nx, la = l + 5 * row + 2;  // padded accumulator index
            const long long d = (long long)acc[3 * aplane + la];
            if (d > 0) {
                // the sums to float through double (two 32-bit conversions, a
                // scale and an add; exact below 2^53, one rounding to float),
                // and v_rcp_f32 (about 1 ulp) in place of a divide
                const float inv = ratio * __builtin_amdgcn_rcpf(i64_to_float(d));
                vv[t][0] = i64_to_float((long long)acc[la]) * inv;
                vv[t][1] = i64_to_float((long long)acc[aplane + la]) * inv;
                vv[t][2] = i64_to_float((long long)acc[2 * aplane + la]) * inv;
            }
        }
    }
    __syncthreads();
    float *S = reinterpret_cast<float *>(acc);
    const size_t n = (size_t)Nx * Ny * Nz;
#pragma unroll
    for (int t = 0; t < kVpt; ++t) {
        const int l = threadIdx.x + t * blockDim.x;
        if (l < plane) {
            S[l] = vv[t][0];
            S[plane + l] = vv[t][1];
            S[2 * plane + l] = vv[t][2];
            if (v_out) {
                const int row = l / Nx, qx = l - row * Nx;
                const int qy = y0 + row % TY, qz = z0 + row / TY;
                if (qy < Ny && qz < Nz) {
                    const size_t o = qx + (size_t)Nx * (qy + (size_t)Ny * qz);
                    v_out[o] = vv[t][0];
                    v_out[n + o] = vv[t][1];
                    v_out[2 * n + o] = vv[t][2];
                }
            }
        }
    }
    __syncthreads();

    // Real FFT along x: real rows (2j, 2j+1) of the flat (channel, row) order
    // - always the same channel since R is even - form complex row j.
    const int ncx = 3 * R / 2;
    // the exchange area of the pencil lengths follows the rows (it fits in the
    // accumulator's space: 24 R Nx + 192 R bytes against 32 R (Nx + 5))
    float2 *xa = reinterpret_cast<float2 *>(S + 3 * plane);
    switch (Nx) {
        case 256: splat_rows_fft16<16>(S, xa, ncx, twl); break;
        case 128: splat_rows_fft16<8>(S, xa, ncx, twl); break;
        case 64: splat_rows_fft16<4>(S, xa, ncx, twl); break;
        case 32: splat_rows_fft16<2>(S, xa, ncx, twl); break;
        case 16: splat_rows_fft16<1>(S, xa, ncx, twl); break;
        default:
            // at most 1.5 kSplatMaxPlane elements over kSplatThreads threads
            fft_rows<false, (3 * kSplatMaxPlane / 2 + kSplatThreads - 1) / kSplatThreads>(RowsS{S, 2 * Nx, Nx},
                                                                                          ncx, ax, twl, -1);
    }

    // Unpack X_a[k] = (Z[k] + conj Z[N-k]) / 2, X_b[k] = (Z[k] - conj Z[N-k]) / 2i,
    // k = 0..Nx/2, and store; the x component is multiplied by j w_x.
    const unsigned mH = div_magic(H);
    for (int i = threadIdx.x; i < ncx * H; i += blockDim.x) {
        const int jr = udiv(i, H, mH), kx = i - jr * H;
        const float *re = S + 2 * jr * Nx, *im = re + Nx;
        const int km = kx == 0 ? 0 : Nx - kx;
        const float zr = re[kx], zi = im[kx];
        const float mr = re[km], mi = im[km];
        float2 xa = make_float2(0.5f * (zr + mr), 0.5f * (zi - mi));
        float2 xb = make_float2(0.5f * (zi + mi), 0.5f * (mr - zr));
        const int ra = (2 * jr) % R, c = (2 * jr) / R;
        if (c == 0) {
            const float wx = deriv_w(kx, Nx, g.wstep[0]);
            xa = make_float2(-wx * xa.y, wx * xa.x);
            xb = make_float2(-wx * xb.y, wx * xb.x);
        }
        const int ya = y0 + ra % TY, za = z0 + ra / TY;
        const int yb = y0 + (ra + 1) % TY, zb = z0 + (ra + 1) / TY;
        const size_t ia = c * pl + ((size_t)za * Ny + ya) * Hp + kx;
        const size_t ib = c * pl + ((size_t)zb * Ny + yb) * Hp + kx;
        if (g.spec_st == kSpecF32) {
            if (ya < Ny && za < Nz) spec_st<kSpecF32>(spec, ia, xa);
            if (yb < Ny && zb < Nz) spec_st<kSpecF32>(spec, ib, xb);
        } else {
            // the reduced storages keep the x share of the inverse's 1/n
            const float sx = g.fscale[0];
            xa = make_float2(xa.x * sx, xa.y * sx);
            xb = make_float2(xb.x * sx, xb.y * sx);
            if (g.spec_st == kSpecBF16) {
                if (ya < Ny && za < Nz) spec_st<kSpecBF16>(spec, ia, xa);
                if (yb < Ny && zb < Nz) spec_st<kSpecBF16>(spec, ib, xb);
            } else {
                if (ya < Ny && za < Nz) spec_st<kSpecF16>(spec, ia, xa);
                if (yb < Ny && zb < Nz) spec_st<kSpecF16>(spec, ib, xb);
            }
        }
    }
    __syncthreads();  // LDS is reused by the next tile
    }
}

static int g_splat_blocks = 256;

hipError_t splat_configure() {
    hipError_t e = raise_dynamic_lds((const void *)splat_fft_x_kernel<false>);
    if (e == hipSuccess) e = raise_dynamic_lds((const void *)splat_fft_x_kernel<true>);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // two persistent blocks per CU (each takes under half the LDS), so one
    // block's setup and epilogue overlap the other's accumulation
    if (e == hipSuccess && cus > 0) g_splat_blocks = 2 * cus;
    return e;
}

int splat_blocks() { return g_splat_blocks; }

int splat_max_plane() { return kSplatMaxPlane; }

size_t splat_lds_bytes(const Grid &g, const SplatConsts &sc) {
    return (size_t)4 * sc.ty * sc.tz * (g.n[0] + 5) * sizeof(unsigned long long) +
           g.n[0] * sizeof(float2);
}

int bin_count_blocks(int m) { return m > 0 ? (m + kBinThreads - 1) / kBinThreads : 0; }

hipError_t launch_bin_count(const float *pts, const float *nrm, const float *w, int m,
                            const Grid &g, int nearest, int32_t *bin_count, int32_t *key, int32_t *rank,
                            uint2 *blk_max, DevStatus *st, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    bin_count_kernel<<<dim3(bin_count_blocks(m)), dim3(kBinThreads), 0, s>>>(pts, nrm, w, m, g, nearest,
                                                                     bin_count, key, rank, blk_max, st);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const float *pts, const float *nrm, const float *w, int m,
                              const Grid &g, const int32_t *key, const int32_t *rank,
                              const int32_t *bin_off, const DevStatus *st, int nearest, float4 *rec,
                              hipStream_t s) {
    if (m <= 0) return hipSuccess;
    bin_scatter_kernel<<<dim3((m + 255) / 256), dim3(256), 0, s>>>(pts, nrm, w, m, g, key, rank,
                                                                   bin_off, st, nearest, rec);
    return hipGetLastError();
}

constexpr int kTileLanes = 8;  // lanes per tile in tile_list

// Per splat tile (kTileLanes lanes): the point-rows that fall into it (each point of
// bin (iy, iz) adds one item row per tile row within its footprint rows
// iy - 1 .. iy + 2, iz - 1 .. iz + 2).  Busy tiles get occ = 1 and an entry
// (tile, cost) in `pend`, in no particular order.  Block b < nscan also sums
// scan tile b of the bin counts into partial[b] (first half of the bin scan).
constexpr int kTileListThreads = 256;

__global__ void __launch_bounds__(kTileListThreads)
tile_list_kernel(const int32_t *__restrict__ bin_count, int nbins, int nscan,
                 int32_t *__restrict__ partial, Grid g, SplatConsts sc, int ntiles,
                 uint8_t *__restrict__ occ, int2 *__restrict__ pend, DevStatus *st) {
    if ((int)blockIdx.x < nscan) scan_tile_sum<1>(bin_count, nbins, blockIdx.x, partial);
    // kTileLanes lanes per tile, lane r on the tile's origin rows iz_lo + r,
    // iz_lo + r + kTileLanes, ...; their sums meet by shuffles
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = gt / kTileLanes, r = gt % kTileLanes;
    long long cost = 0;
    if (tile < ntiles) {
        const int Ny = g.n[1], Nz = g.n[2];
        const int y0 = (tile % sc.tiles_y) * sc.ty, z0 = (tile / sc.tiles_y) * sc.tz;
        const int y1 = min(y0 + sc.ty, Ny) - 1, z1 = min(z0 + sc.tz, Nz) - 1;  // last tile rows
        // origin rows i whose rows i + lo .. i + hi meet the tile
        const int lo = sc.fp_lo, hi = sc.fp_hi;
        const int iz_lo = max(z0 - hi, -1), iz_hi = min(z0 + sc.tz - 1 - lo, Nz - 1);
        const int iy_lo = max(y0 - hi, -1), iy_hi = min(y0 + sc.ty - 1 - lo, Ny - 1);
        // the loads of a bin row are independent: unrolled, they are in flight together
        for (int iz = iz_lo + r; iz <= iz_hi; iz += kTileLanes) {
            const int nz = min(iz + hi, z1) - max(iz + lo, z0) + 1;
            const int row = (iz + 1) * (Ny + 1) + 1;
            long long sum = 0;
#pragma unroll 8
            for (int iy = iy_lo; iy <= iy_hi; ++iy)
                sum += (long long)bin_count[row + iy] * max(min(iy + hi, y1) - max(iy + lo, y0) + 1, 0);
            cost += max(nz, 0) * sum;
        }
    }
#pragma unroll
    for (int d = kTileLanes / 2; d > 0; d >>= 1) cost += __shfl_xor(cost, d, kTileLanes);
    if (tile < ntiles && r == 0) occ[tile] = cost > 0 ? 1 : 0;
    const bool busy = tile < ntiles && r == 0 && cost > 0;
    // one list append per block (every block appends to the one counter:
    // fewer atomics queue on it than with one per wave)
    __shared__ int wcnt[kTileListThreads / 64], bbase;
    const unsigned long long b = __ballot(busy);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) wcnt[wid] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kTileListThreads / 64; ++w) tot += wcnt[w];
        bbase = tot ? atomicAdd(&st->n_busy, tot) : 0;
    }
    __syncthreads();
    if (busy) {
        int base = bbase;
        for (int w = 0; w < wid; ++w) base += wcnt[w];
        pend[base + __popcll(b & ((1ull << lane) - 1ull))] = make_int2(tile, (int)min(cost, 0x7fffffffLL));
    }
}

// Busy tiles in decreasing cost (64 logarithmic cost classes, a counting
// sort in one block), so the persistent splat blocks take the longest tiles
// first and finish together.
constexpr int kTileClasses = 64;

__device__ __forceinline__ int tile_class(int cost) {
    const int msb = 31 - __clz(cost);
    return 2 * msb + (msb > 0 ? (cost >> (msb - 1)) & 1 : 0);
}

// Blocks 0 .. nscan - 1 finish the bin scan (scan tile b on top of the
// partial sums of tile_list); block nscan reduces the weight maxima and sorts
// the busy tiles.
__global__ void __launch_bounds__(256)
tile_order_kernel(const int32_t *__restrict__ bin_count, int32_t *__restrict__ bin_off, int nbins,
                  int nscan, const int32_t *__restrict__ partial, const int2 *__restrict__ pend,
                  int32_t *__restrict__ list, const uint2 *__restrict__ blk_max, int nblk,
                  DevStatus *st) {
    if ((int)blockIdx.x < nscan) {
        scan_tile_down<1>(bin_count, bin_off, nbins, partial, blockIdx.x, nscan);
        return;
    }
    __shared__ int hist[kTileClasses], cursor[kTileClasses];
    __shared__ unsigned wmax[kScanBlock / 64], wnmax[kScanBlock / 64];
    // Loads go out kBatch at a time with clamped indices (a duplicate does not
    // change a maximum or a count that the index check excludes), so each
    // batch costs one memory round trip.  The first batch of busy tiles goes
    // out with the block maxima, and when it holds them all (the usual case)
    // the scatter below reuses it.
    constexpr int kBatch = 8;
    constexpr int kOne = kBatch * kScanBlock;
    const int n = st->n_busy;
    int2 e0[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) e0[u] = pend[max(min(u * kScanBlock + (int)threadIdx.x, n - 1), 0)];
    // the frame's largest W and W |N_c| (fixed-point units of the splat)
    unsigned mw = 0, mn = 0;
    for (int b0 = 0; b0 < nblk; b0 += kOne) {
        uint2 v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) v[u] = blk_max[min(b0 + u * kScanBlock + (int)threadIdx.x, nblk - 1)];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            mw = max(mw, v[u].x);
            mn = max(mn, v[u].y);
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        mw = max(mw, (unsigned)__shfl_xor((int)mw, d, 64));
        mn = max(mn, (unsigned)__shfl_xor((int)mn, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        wmax[threadIdx.x >> 6] = mw;
        wnmax[threadIdx.x >> 6] = mn;
    }
    if (threadIdx.x < kTileClasses) hist[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
        if (u * kScanBlock + (int)threadIdx.x < n) atomicAdd(&hist[tile_class(e0[u].y)], 1);
    for (int b0 = kOne; b0 < n; b0 += kOne) {
        int2 e[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) e[u] = pend[min(b0 + u * kScanBlock + (int)threadIdx.x, n - 1)];
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (b0 + u * kScanBlock + (int)threadIdx.x < n) atomicAdd(&hist[tile_class(e[u].y)], 1);
    }
    __syncthreads();
    if (threadIdx.x < kTileClasses) {
        // classes in decreasing order: the start of class c is the count of classes above it
        const int c = threadIdx.x;
        int above = 0;
        for (int k = c + 1; k < kTileClasses; ++k) above += hist[k];
        cursor[c] = above;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
        if (u * kScanBlock + (int)threadIdx.x < n) list[atomicAdd(&cursor[tile_class(e0[u].y)], 1)] = e0[u].x;
    for (int b0 = kOne; b0 < n; b0 += kOne) {
        int2 e[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) e[u] = pend[min(b0 + u * kScanBlock + (int)threadIdx.x, n - 1)];
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (b0 + u * kScanBlock + (int)threadIdx.x < n) list[atomicAdd(&cursor[tile_class(e[u].y)], 1)] = e[u].x;
    }
    if (threadIdx.x == 0) {
        unsigned a = 0, b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a = max(a, wmax[w]);
            b = max(b, wnmax[w]);
        }
        st->wmax_bits = a;
        st->wnmax_bits = b;
    }
}

hipError_t launch_tile_list(const int32_t *bin_count, int32_t *bin_off, int nbins, int32_t *partial,
                            const Grid &g, const SplatConsts &sc, uint8_t *occ, int2 *pend,
                            int32_t *list, const uint2 *blk_max, int m, DevStatus *st, hipStream_t s) {
    const int ntiles = sc.tiles_y * ((g.n[2] + sc.tz - 1) / sc.tz);
    const int nscan = scan_tiles(nbins);
    const int blocks = std::max((ntiles * kTileLanes + kTileListThreads - 1) / kTileListThreads, nscan);
    tile_list_kernel<<<dim3(blocks), dim3(kTileListThreads), 0, s>>>(bin_count, nbins, nscan, partial, g, sc, ntiles,
                                                       occ, pend, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    tile_order_kernel<<<dim3(nscan + 1), dim3(kScanBlock), 0, s>>>(bin_count, bin_off, nbins, nscan, partial,
                                                                 pend, list, blk_max, bin_count_blocks(m), st);
    return hipGetLastError();
}

int bin_scan_tiles(int nbins) { return scan_tiles(nbins); }

hipError_t launch_splat_fft_x(const float4 *rec, const int32_t *bin_off, const Grid &g,
                              const SplatConsts &sc, const FftAxis &ax, DevStatus *st,
                              const int32_t *list, void *spec, float *v_out, hipStream_t s) {
    const int tiles = sc.tiles_y * ((g.n[2] + sc.tz - 1) / sc.tz);
    const int blocks = tiles < g_splat_blocks ? tiles : g_splat_blocks;
    const size_t lds = splat_lds_bytes(g, sc);
    if (sc.nearest)
        splat_fft_x_kernel<true><<<dim3(blocks), dim3(kSplatThreads), lds, s>>>(
            rec, bin_off, g, sc, ax, st, list, spec, v_out);
    else
        splat_fft_x_kernel<false><<<dim3(blocks), dim3(kSplatThreads), lds, s>>>(
            rec, bin_off, g, sc, ax, st, list, spec, v_out);
    return hipGetLastError();
}

}  // namespace fvr
