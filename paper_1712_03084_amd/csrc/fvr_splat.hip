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
//   splat_fft_x one block per tile of ty x tz full x-rows: gathers the points
//               of the (ty+3) x (tz+3) rows of bins whose footprints reach
//               the tile, accumulates S and D with LDS float atomics, forms V,
//               runs the real FFT of every x-row in LDS and writes the three
//               half-spectrum planes, the x component times j w_x.
#include "fvr_common.h"
#include "fvr_fft_engine.h"

namespace fvr {

constexpr int kSplatThreads = 256;
constexpr int kMaxSegs = 16;

// Footprint origin floor((x - bmin)/h - 1/2) in float32, each operation
// correctly rounded (no contraction), so every implementation that follows
// this formula picks the same voxels.
__device__ __forceinline__ float voxel_coord(float x, float bmin, float h) {
    return __fsub_rn(__fdiv_rn(__fsub_rn(x, bmin), h), 0.5f);
}

__device__ __forceinline__ bool finite3(float a, float b, float c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

__global__ void __launch_bounds__(256)
bin_count_kernel(const float *__restrict__ pts, const float *__restrict__ nrm,
                 const float *__restrict__ w, int m, Grid g, int32_t *__restrict__ bin_count,
                 int32_t *__restrict__ key, int32_t *__restrict__ rank, DevStatus *st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false, rej = false;
    if (i < m) {
        const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        const float wi = w ? w[i] : 1.0f;
        bad = !(finite3(x, y, z) && finite3(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]) &&
                isfinite(wi) && wi >= 0.0f);
        int k = -1;
        if (!bad) {
            const bool acc = x >= g.bmin[0] && x <= g.bmax[0] && y >= g.bmin[1] &&
                             y <= g.bmax[1] && z >= g.bmin[2] && z <= g.bmax[2];
            if (acc) {
                int iy = (int)floorf(voxel_coord(y, g.bmin[1], g.h[1]));
                int iz = (int)floorf(voxel_coord(z, g.bmin[2], g.h[2]));
                iy = min(max(iy, -1), g.n[1] - 1);
                iz = min(max(iz, -1), g.n[2] - 1);
                k = (iz + 1) * (g.n[1] + 1) + (iy + 1);
                rank[i] = atomicAdd(&bin_count[k], 1);
            } else {
                rej = true;
            }
        }
        key[i] = k;
    }
    const unsigned long long brej = __ballot(rej), bbad = __ballot(bad);
    if ((threadIdx.x & 63) == 0) {
        if (brej) atomicAdd(&st->rejected, (uint32_t)__popcll(brej));
        if (bbad) atomicOr(&st->flags, kFlagInvalid);
    }
}

__global__ void __launch_bounds__(256)
bin_scatter_kernel(const float *__restrict__ pts, const float *__restrict__ nrm,
                   const float *__restrict__ w, int m, const int32_t *__restrict__ key,
                   const int32_t *__restrict__ rank, const int32_t *__restrict__ bin_off,
                   float4 *__restrict__ rec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int k = key[i];
    if (k < 0) return;
    const int pos = bin_off[k] + rank[i];
    const float wi = w ? w[i] : 1.0f;
    rec[2 * pos] = make_float4(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], wi);
    rec[2 * pos + 1] = make_float4(wi * nrm[3 * i], wi * nrm[3 * i + 1], wi * nrm[3 * i + 2], 0.0f);
}

__global__ void __launch_bounds__(kSplatThreads)
splat_fft_x_kernel(const float4 *__restrict__ rec, const int32_t *__restrict__ bin_off, Grid g,
                   SplatConsts sc, FftAxis ax, float2 *__restrict__ spec, float *__restrict__ v_out) {
    extern __shared__ float smem[];
    __shared__ int seg_start[kMaxSegs];
    __shared__ int seg_pre[kMaxSegs + 1];

    const int Nx = g.n[0], Ny = g.n[1], Nz = g.n[2];
    const int TY = sc.ty, TZ = sc.tz, R = TY * TZ;
    const int by = blockIdx.x % sc.tiles_y, bz = blockIdx.x / sc.tiles_y;
    const int y0 = by * TY, z0 = bz * TZ;
    const int plane = R * Nx;            // floats per channel plane
    float *S = smem;                     // 3 planes: S_x, S_y, S_z, then D
    float *D = smem + 3 * plane;

    for (int i = threadIdx.x; i < 4 * plane; i += blockDim.x) smem[i] = 0.0f;

    // candidate points: bins of footprint origins (iy, iz) whose 4-row
    // footprints overlap the tile, i.e. iy in [y0-2, y0+TY], iz in [z0-2, z0+TZ]
    const int iz_lo = max(z0 - 2, -1), iz_hi = min(z0 + TZ, Nz - 1);
    const int iy_lo = max(y0 - 2, -1), iy_hi = min(y0 + TY, Ny - 1);
    const int nseg = iz_hi - iz_lo + 1;
    if (threadIdx.x < nseg) {
        const int iz = iz_lo + threadIdx.x;
        const int k0 = (iz + 1) * (Ny + 1) + (iy_lo + 1);
        const int k1 = (iz + 1) * (Ny + 1) + (iy_hi + 1) + 1;
        seg_start[threadIdx.x] = bin_off[k0];
        seg_pre[threadIdx.x + 1] = bin_off[k1] - bin_off[k0];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        seg_pre[0] = 0;
        for (int s = 0; s < nseg; ++s) seg_pre[s + 1] += seg_pre[s];
    }
    __syncthreads();
    const int total = seg_pre[nseg];

    for (int j = threadIdx.x; j < total; j += blockDim.x) {
        int s = 0;
        while (seg_pre[s + 1] <= j) ++s;
        const int p = seg_start[s] + (j - seg_pre[s]);
        const float4 r0 = rec[2 * p], r1 = rec[2 * p + 1];
        const float X[3] = {r0.x, r0.y, r0.z};
        float v[3];
        int i0[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = voxel_coord(X[a], g.bmin[a], g.h[a]);
            i0[a] = (int)floorf(v[a]);
        }
        float wx1[4], wx2[4], wy1[4], wy2[4], wz1[4], wz2[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const float dx = v[0] - (float)(i0[0] + o - 1);
            const float dy = v[1] - (float)(i0[1] + o - 1);
            const float dz = v[2] - (float)(i0[2] + o - 1);
            wx1[o] = __builtin_amdgcn_exp2f(sc.e1[0] * dx * dx);
            wx2[o] = __builtin_amdgcn_exp2f(sc.e2[0] * dx * dx);
            wy1[o] = __builtin_amdgcn_exp2f(sc.e1[1] * dy * dy);
            wy2[o] = __builtin_amdgcn_exp2f(sc.e2[1] * dy * dy);
            wz1[o] = __builtin_amdgcn_exp2f(sc.e1[2] * dz * dz);
            wz2[o] = __builtin_amdgcn_exp2f(sc.e2[2] * dz * dz);
        }
#pragma unroll
        for (int oz = 0; oz < 4; ++oz) {
            const int qz = i0[2] + oz - 1;
            if (qz < z0 || qz >= z0 + TZ || qz >= Nz) continue;
#pragma unroll
            for (int oy = 0; oy < 4; ++oy) {
                const int qy = i0[1] + oy - 1;
                if (qy < y0 || qy >= y0 + TY || qy >= Ny) continue;
                const int row = (qz - z0) * TY + (qy - y0);
                const float a1 = wy1[oy] * wz1[oz], a2 = wy2[oy] * wz2[oz];
#pragma unroll
                for (int ox = 0; ox < 4; ++ox) {
                    const int qx = i0[0] + ox - 1;
                    if (qx < 0 || qx >= Nx) continue;
                    const int l = row * Nx + qx;
                    const float g1 = wx1[ox] * a1;
                    atomicAdd(&S[l], g1 * r1.x);
                    atomicAdd(&S[plane + l], g1 * r1.y);
                    atomicAdd(&S[2 * plane + l], g1 * r1.z);
                    atomicAdd(&D[l], wx2[ox] * a2 * r0.w);
                }
            }
        }
    }
    __syncthreads();

    // V = (sigma2/sigma1) S' / D' (the Gaussians' 1/sigma prefactors), 0 where D = 0
    for (int l = threadIdx.x; l < plane; l += blockDim.x) {
        const float d = D[l];
        const float inv = d > 0.0f ? sc.vscale / d : 0.0f;
        const float vx = S[l] * inv, vy = S[plane + l] * inv, vz = S[2 * plane + l] * inv;
        S[l] = vx;
        S[plane + l] = vy;
        S[2 * plane + l] = vz;
        if (v_out) {
            const int row = l / Nx, qx = l - row * Nx;
            const int qy = y0 + row % TY, qz = z0 + row / TY;
            if (qy < Ny && qz < Nz) {
                const size_t n = (size_t)Nx * Ny * Nz;
                const size_t o = qx + (size_t)Nx * (qy + (size_t)Ny * qz);
                v_out[o] = vx;
                v_out[n + o] = vy;
                v_out[2 * n + o] = vz;
            }
        }
    }
    __syncthreads();

    // Real FFT along x: real rows (2j, 2j+1) of the flat (channel, row) order
    // - always the same channel since R is even - form complex row j.
    const int ncx = 3 * R / 2;
    fft_rows<false>(RowsS{S, 2 * Nx, Nx}, ncx, ax, -1);

    // Unpack X_a[k] = (Z[k] + conj Z[N-k]) / 2, X_b[k] = (Z[k] - conj Z[N-k]) / 2i,
    // k = 0..Nx/2, and store; the x component is multiplied by j w_x.
    const int H = g.H;
    const unsigned mH = div_magic(H);
    const size_t pl = (size_t)Nz * Ny * H;
    for (int i = threadIdx.x; i < ncx * H; i += blockDim.x) {
        const int jr = udiv(i, H, mH), k = i - jr * H;
        const float *re = S + 2 * jr * Nx, *im = re + Nx;
        const int km = k == 0 ? 0 : Nx - k;
        const float zr = re[k == Nx ? 0 : k], zi = im[k == Nx ? 0 : k];
        const float mr = re[km], mi = im[km];
        float2 xa = make_float2(0.5f * (zr + mr), 0.5f * (zi - mi));
        float2 xb = make_float2(0.5f * (zi + mi), 0.5f * (mr - zr));
        const int ra = (2 * jr) % R, c = (2 * jr) / R;
        if (c == 0) {
            const float wx = deriv_w(k, Nx, g.wstep[0]);
            xa = make_float2(-wx * xa.y, wx * xa.x);
            xb = make_float2(-wx * xb.y, wx * xb.x);
        }
        const int ya = y0 + ra % TY, za = z0 + ra / TY;
        const int yb = y0 + (ra + 1) % TY, zb = z0 + (ra + 1) / TY;
        if (ya < Ny && za < Nz) spec[c * pl + ((size_t)za * Ny + ya) * H + k] = xa;
        if (yb < Ny && zb < Nz) spec[c * pl + ((size_t)zb * Ny + yb) * H + k] = xb;
    }
}

hipError_t splat_configure() {
    return hipFuncSetAttribute((const void *)splat_fft_x_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
}

size_t splat_lds_bytes(const Grid &g, const SplatConsts &sc) {
    return (size_t)4 * sc.ty * sc.tz * g.n[0] * sizeof(float);
}

hipError_t launch_bin_count(const float *pts, const float *nrm, const float *w, int m,
                            const Grid &g, int32_t *bin_count, int32_t *key, int32_t *rank,
                            DevStatus *st, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    bin_count_kernel<<<dim3((m + 255) / 256), dim3(256), 0, s>>>(pts, nrm, w, m, g, bin_count, key,
                                                                 rank, st);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const float *pts, const float *nrm, const float *w, int m,
                              const int32_t *key, const int32_t *rank, const int32_t *bin_off,
                              float4 *rec, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    bin_scatter_kernel<<<dim3((m + 255) / 256), dim3(256), 0, s>>>(pts, nrm, w, m, key, rank,
                                                                   bin_off, rec);
    return hipGetLastError();
}

hipError_t launch_splat_fft_x(const float4 *rec, const int32_t *bin_off, const Grid &g,
                              const SplatConsts &sc, const FftAxis &ax, float2 *spec,
                              float *v_out, hipStream_t s) {
    const int tiles = sc.tiles_y * ((g.n[2] + sc.tz - 1) / sc.tz);
    const size_t lds = splat_lds_bytes(g, sc);
    splat_fft_x_kernel<<<dim3(tiles), dim3(kSplatThreads), lds, s>>>(rec, bin_off, g, sc, ax, spec,
                                                                     v_out);
    return hipGetLastError();
}

}  // namespace fvr
