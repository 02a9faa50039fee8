// Internal declarations shared by the host runtime and the HIP kernels of the
// gfx950 FT-reconstruction library.  Not part of the public ABI (include/fvr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvr {

constexpr int kMaxDim = 512;
constexpr int kMaxStages = 8;
constexpr int kMcMaxTris = 5;         // triangles per marching-cubes case, at most
constexpr int kMcRow = 3 * kMcMaxTris;
constexpr int kLdsPerWorkgroup = 160 * 1024;  // gfx950: 160 KiB of LDS per workgroup

// Allow a kernel all LDS beyond its static allocation as dynamic LDS.
inline hipError_t raise_dynamic_lds(const void *kernel) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, kernel);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kLdsPerWorkgroup - (int)a.sharedSizeBytes);
}

// One axis of the 3D FFT: length n = prod(radix[0..nstages)), radices from
// {2, 3, 4, 5, 8}; tw[t] = exp(-2 pi i t / n) for t < n, float32 values
// rounded from a double-precision table.
struct FftAxis {
    int n;
    int nstages;
    // radix of stage s in bits [4s, 4s + 4): a packed word, since a dynamically
    // indexed array in a kernel argument is copied to per-lane scratch memory
    unsigned radices;
    const float2 *tw;
};

// Grid geometry in float32, shared by every stage.
struct Grid {
    int n[3];          // Nx, Ny, Nz
    int H;             // Nx/2 + 1: length of a half-spectrum row
    int Hp;            // row pitch of the spectrum planes: H rounded up to 16 (128-byte rows)
    int ty, tz;        // splat tile rows along y and z (full x rows per tile)
    int tiles_y;       // ceil(Ny / ty)
    float bmin[3];
    float bmax[3];
    float h[3];        // (bmax - bmin) / N, float32
    float wstep[3];    // 2 pi / extent: angular frequency of wavenumber 1
    // Spectrum storage: kSpecF32 (complex64), kSpecBF16 or kSpecF16 (two
    // 16-bit floats per bin).  The reduced forms split the 1/n of the
    // inverse over the forward passes (each stores its output times
    // 1/N_axis), which keeps FP16 clear of overflow.
    int spec_st;
    float fscale[3];   // factor on the stored output of the x, y and z forward passes
    float iscale;      // factor on A after the inverse (1/n for complex64, else 1)
};
constexpr int kSpecF32 = 0, kSpecBF16 = 1, kSpecF16 = 2;
inline size_t spec_elem_bytes(int st) { return st == kSpecF32 ? 8 : 4;}

// Load and store of one spectrum bin of storage `ST` at element index i.
#if defined(__HIPCC__)
template <int ST>
__device__ __forceinline__ float2 spec_unpack(unsigned u) {
    if constexpr (ST == kSpecBF16) {
        return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
    } else {
        const _Float16 lo = __builtin_bit_cast(_Float16, (unsigned short)(u & 0xffffu));
        const _Float16 hi = __builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
        return make_float2((float)lo, (float)hi);
    }
}
// round to nearest even (finite inputs)
__device__ __forceinline__ unsigned bf16_bits(float x) {
    const unsigned b = __float_as_uint(x);
    return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
}
template <int ST>
__device__ __forceinline__ unsigned spec_pack(float2 v) {
    if constexpr (ST == kSpecBF16) {
        return bf16_bits(v.x) | (bf16_bits(v.y) << 16);
    } else {
        const unsigned lo = __builtin_bit_cast(unsigned short, (_Float16)v.x);
        const unsigned hi = __builtin_bit_cast(unsigned short, (_Float16)v.y);
        return lo | (hi << 16);
    }
}
template <int ST>
__device__ __forceinline__ float2 spec_ld(const void *base, size_t i) {
    if constexpr (ST == kSpecF32) return static_cast<const float2 *>(base)[i];
    else return spec_unpack<ST>(static_cast<const unsigned *>(base)[i]);
}
template <int ST>
__device__ __forceinline__ void spec_st(void *base, size_t i, float2 v) {
    if constexpr (ST == kSpecF32) static_cast<float2 *>(base)[i] = v;
    else static_cast<unsigned *>(base)[i] = spec_pack<ST>(v);
}
#endif

// Splat-specific constants.  Gaussian weights are evaluated per axis as
// exp2(e1[a] * d^2) with d the point-to-centre offset in voxels of axis a:
// e1[a] = -h_a^2 / sigma1^2 * log2(e), e2[a] the same with sigma2.
struct SplatConsts {
    float e1[3];
    float e2[3];
    float vscale;      // sigma2 / sigma1: the ratio of the two 1/sigma prefactors (1: nearest)
    int ty, tz;        // tile rows along y and z (full x rows per tile)
    int tiles_y;       // ceil(Ny / ty)
    int nearest;       // 1: the non-weighted splat (each point to its nearest voxel)
    int fp_lo, fp_hi;  // rows a point of origin row i reaches: i + fp_lo .. i + fp_hi
};

// Device-side status block, read back once per frame.
struct DevStatus {
    uint32_t flags;       // bit 0: invalid input value; bit 1: open surface; bit 2: 16-bit spectrum overflow
    uint32_t rejected;    // points outside the bbox
    int32_t mc_total[3];  // vertices, triangles, active cells
    int32_t n_used;       // points that entered the level average
    double level;
    uint32_t wmax_bits;   // float bits of max W over accepted points (W >= 0)
    uint32_t wnmax_bits;  // float bits of max W |N_c| over accepted points
    int32_t tile_ticket;  // next entry of the busy-tile list to claim (persistent splat blocks)
    int32_t n_busy;       // splat tiles that some point reaches
    int32_t mc_active;    // marching-cubes blocks left for the classification (mc_classify)
    int32_t n_zplanes;    // z planes some splat tile reaches (read by the z pass)
    int32_t fe_points;    // points the depth front end produced
};
constexpr uint32_t kFlagInvalid = 1u;
constexpr uint32_t kFlagOpen = 2u;
constexpr uint32_t kFlagRange = 4u;

// ---------------------------------------------------------------------------
// Launch wrappers (each enqueues on `s` and returns the launch error)
// ---------------------------------------------------------------------------

// Fill `n` int32 with `v`.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

// Reset the status block and zero `nbins` bin counters in one launch.
hipError_t launch_prep(DevStatus *st, int32_t *bins, int nbins, hipStream_t s);
// Device statics (fvr_static.hip): twiddle tables of every supported length
// and the scratch array of the allocation-free entry point, one copy per GPU.
// statics_init looks their addresses up once per device (device current).
hipError_t statics_init(int device);
int twiddle_offset(int n);                               // -1 if n is unsupported
const float2 *statics_twiddles(int device, int n);       // nullptr before statics_init
unsigned char *statics_scratch(int device);              // FVR_NOALLOC_SCRATCH_BYTES

// Copy of the status block into pinned host memory (hipHostMalloc) by a kernel.
hipError_t launch_status_publish(const DevStatus *st, DevStatus *host, hipStream_t s);

// Exclusive scan of `n` items of `C` interleaved int32 components (C = 1 or 3):
// out[i*C + c] = sum_{j<i} in[j*C + c]; out[n*C + c] = total; totals[c] = total.
// `partial` is scratch of scan_partials(n) * C ints.
int scan_partials(int n);
hipError_t launch_scan(const int32_t *in, int32_t *out, int n, int C, int32_t *partial,
                       int32_t *totals, hipStream_t s);

// Splat, stage 1: validate and bin points by the (y, z) row of their
// footprint origin.  key[i] = -1 for rejected points.
int bin_count_blocks(int m);
// blk_max: per bin_count block, the bits of its largest W and W |N_c|
// (reduced by tile_order into st->wmax_bits, st->wnmax_bits)
hipError_t launch_bin_count(const float *pts, const float *nrm, const float *w, int m,
                            const Grid &g, int nearest, int32_t *bin_count, int32_t *key, int32_t *rank,
                            uint2 *blk_max, DevStatus *st, hipStream_t s);
// Splat, stage 2: scatter packed records (fractional voxel offsets, W, W N,
// x footprint origin) into bin order.
hipError_t launch_bin_scatter(const float *pts, const float *nrm, const float *w, int m,
                              const Grid &g, const int32_t *key, const int32_t *rank,
                              const int32_t *bin_off, const DevStatus *st, int nearest, float4 *rec,
                              hipStream_t s);
// Splat, stage 3 fused with the forward real FFT along x: each block owns
// ty x tz full x-rows, accumulates S_x, S_y, S_z and D in LDS (64-bit fixed
// point, scaled per frame from st->wmax_bits / wnmax_bits), forms
// V = S/D, transforms along x and writes three half-spectrum planes
// (the x-component already multiplied by j w_x).  v_out (optional) receives V.
// Tiles no point reaches are skipped: occ[tile] = 0 and their spectrum rows
// are left unwritten (they are zero); occupied tiles set occ[tile] = 1.
// Busy splat tiles: occ[tile] = 1 when some point's footprint reaches the
// tile (0 otherwise), and the indices of those tiles in list[0, st->n_busy),
// in decreasing order of work; pend is scratch of one int2 per tile.  The
// same two launches scan the bin counts into bin_off (nbins + 1 ints, the
// last the total); partial is scratch of bin_scan_tiles(nbins) ints.
int bin_scan_tiles(int nbins);
hipError_t launch_tile_list(const int32_t *bin_count, int32_t *bin_off, int nbins, int32_t *partial,
                            const Grid &g, const SplatConsts &sc, uint8_t *occ, int2 *pend,
                            int32_t *list, const uint2 *blk_max, int m, DevStatus *st, hipStream_t s);
hipError_t launch_splat_fft_x(const float4 *rec, const int32_t *bin_off, const Grid &g,
                              const SplatConsts &sc, const FftAxis &ax, DevStatus *st,
                              const int32_t *list, void *spec, float *v_out, hipStream_t s);
int splat_blocks();
// Voxels of one channel plane of a splat tile (tile rows x Nx), at most.
int splat_max_plane();
size_t splat_lds_bytes(const Grid &g, const SplatConsts &sc);

// Forward y transform of the three planes, combining the x and y
// derivative terms: plane0 <- F_y(plane0) + j w_y F_y(plane1); plane2 <- F_y(plane2).
// Rows of unoccupied tiles are read as zero; a z plane with no occupied tile
// is neither read nor written and gets zocc[z] = 0 (1 otherwise).
hipError_t launch_fft_y_fwd(void *spec, const uint8_t *occ, uint8_t *zocc, DevStatus *st,
                            const Grid &g, const FftAxis &ax, hipStream_t s);
// Forward z transform of planes 0 and 2, the spectral solve, inverse z:
// plane0 <- F_z^-1[(F_z plane0 + j w_z F_z plane2) / |w|^2], DC -> 0.
// Planes with zocc[z] = 0 are read as zero.
hipError_t launch_fft_z_solve(void *spec, const uint8_t *zocc, const Grid &g, const FftAxis &az,
                              hipStream_t s);
// Inverse y transform of plane 0.
hipError_t launch_fft_y_inv(void *spec, const Grid &g, const FftAxis &ay, hipStream_t s);
// Both inverse passes below in one kernel (one block per z plane; the plane
// does not go back to HBM between them), for Nx = Ny = 256: fft_yx_fused(g).
// rowmm[z Ny + y] receives (min, max) of A over the row.
bool fft_yx_fused(const Grid &g);
hipError_t launch_fft_yx_inv(const void *spec, float *A, float2 *rowmm, DevStatus *st, const Grid &g,
                             const FftAxis &ay, hipStream_t s);
// Inverse real FFT along x of plane 0, scaled by g.iscale -> A (Nz, Ny, Nx);
// rowmm[z Ny + y] receives (min, max) of A over the row, as the fused pass
// writes it.  With a 16-bit spectrum storage both inverse kernels set
// kFlagRange in st when they write a non-finite value (an overflowed store
// upstream).
hipError_t launch_fft_x_c2r(const void *spec, float *A, float2 *rowmm, DevStatus *st, const Grid &g,
                            const FftAxis &ax, hipStream_t s);

// Iso-level: per-block double partial sums of trilinear A at accepted points,
// then (final) one block reduces them in a fixed order into st->level,
// st->n_used and *level_f32 (the level rounded to float for the
// marching-cubes comparisons).  Without final the partials are left for
// launch_mc_classify to reduce.
hipError_t launch_level(const float *pts, int m, const float *A, const Grid &g,
                        double *partial_sum, int32_t *partial_cnt, DevStatus *st,
                        float *level_f32, bool final, hipStream_t s);
int level_blocks(int m);

// Marching cubes.
hipError_t mc_upload_table(const uint8_t *counts, const int8_t *edges);
int mc_blocks(const Grid &g);
// From rowmm, the (min, max) of A per row (z Ny + y): blocks whose cells'
// corner rows lie all above or all at/below the level are settled without
// reading A (zero totals); the others go to list (st->mc_active entries).
// With partial_sum not null it also finishes the level from the lnb
// partials launch_level left (same result as its final step); else it reads
// *level_f32.
hipError_t launch_mc_classify(float *level_f32, const double *partial_sum, const int32_t *partial_cnt,
                              int lnb, const float2 *rowmm, const Grid &g, int32_t *blk_counts,
                              int32_t *list, DevStatus *st, hipStream_t s);
// Exclusive scan of the totals of the nb marching-cubes blocks when only the
// blocks in list (st->mc_active of them) can be nonzero: out[3 b + c] for the
// listed blocks (the others are not written), out[3 nb + c] and
// st->mc_total[c] the totals.  One launch.
hipError_t launch_mc_list_scan(const int32_t *list, const int32_t *cnt, int nb, int32_t *out,
                               DevStatus *st, hipStream_t s);
hipError_t mc_configure();
// list: the blocks mc_classify left (null: every block).
hipError_t launch_mc_count(const float *A, const float *level_f32, const int32_t *list, const Grid &g,
                           int32_t *blk_counts, uint32_t *codes, uint8_t *cases_out, DevStatus *st,
                           hipStream_t s);
// The mesh kernels read the totals of the count scan from `st`; they write
// nothing when a total exceeds its capacity (vertices, triangles, active
// cells) or the frame was flagged invalid.
struct MeshCaps {
    long long vertices, triangles, cells;
    int check_invalid;
};
hipError_t launch_mc_generate(const float *A, const float *level_f32, const int32_t *list, const Grid &g,
                              const int32_t *blk_counts, const int32_t *blk_offsets,
                              const uint32_t *codes, float *verts, float *normals, int32_t *vidx,
                              int4 *cells, const DevStatus *st, MeshCaps caps, DevStatus *host_status,
                              hipStream_t s);
// (host_status, if not null: pinned host memory that receives a copy of the
// final status block, as launch_status_publish would write it)
hipError_t launch_mc_triangles(const int4 *cells, const int32_t *vidx, const Grid &g, int32_t *tris,
                               const DevStatus *st, MeshCaps caps, hipStream_t s);

// Raise the dynamic-LDS limit of the kernels that stage tiles above 64 KiB.
hipError_t splat_configure();
hipError_t fft_configure();

// Host-side marching-cubes table generation (library's own generator).
void mc_generate_table(uint8_t counts[256], int8_t edges[256 * kMcRow]);

}  // namespace fvr

namespace fvr {
// Depth front end (Sec. III-A): depth maps to oriented, weighted points.
constexpr int kFeMaxViews = 16;
struct FeCams {
    float c[kFeMaxViews][16];  // per view: fx fy cx cy, R (3x3 row-major, camera to world), t
};
struct FeParams {
    int views, height, width, radius;
    float tau;  // largest depth difference inside a triangle
};
hipError_t launch_fe_pixels(const float *depth, const FeParams &fp, const FeCams &cams, int32_t *rowcnt,
                            float *dense, int32_t *flag, hipStream_t s);
hipError_t launch_fe_scatter(const float *dense, const int32_t *flag, const int32_t *off, int n,
                             const DevStatus *st, long long cap, float *pts, float *nrm, float *w,
                             hipStream_t s);
}  // namespace fvr
