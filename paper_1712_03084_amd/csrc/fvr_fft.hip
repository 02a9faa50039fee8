// Strided FFT passes of the spectral integration (Sec. III-B) on gfx950.
//
// Spectra are three half-spectrum planes of shape (Nz, Ny, H), H = Nx/2 + 1,
// kx fastest, each bin complex64 or two packed 16-bit floats (bf16 / fp16;
// every pass computes in float32).  The forward x transform (with the x derivative
// factor) is fused into the splat kernel; these passes finish the transform
// along y and z, apply the integration filter, and invert:
//
//   fft_y_fwd   P0 <- F_y P0 + j w_y F_y P1          (x and y derivative terms)
//               P2 <- F_y P2
//   fft_z_solve P0 <- F_z^-1 [ (F_z P0 + j w_z F_z P2) / |w|^2 ],  DC -> 0
//   fft_y_inv   P0 <- F_y^-1 P0
//   fft_x_c2r   A  <- F_x^-1 P0 / (Nx Ny Nz)          (real output)
//   fft_yx_inv  both of the above in one kernel per z plane (Nx = Ny = 256
//               or 128), with each row's range of A as a by-product
//
// By linearity this equals the paper's per-component transform, filter and
// inverse followed by the sum of the X, Y and Z components.
//
// y and z passes: a block owns kChunk consecutive kx columns of one plane
// line (fixed z for y, fixed ky for z) and the whole transformed axis, staged
// in LDS as [axis][kChunk] so each global row access is kChunk contiguous
// complex values.
#include "fvr_common.h"
#include "fvr_fft_engine.h"

namespace fvr {

constexpr int kChunk = 16;
constexpr int kPassThreads = 256;
constexpr int kC2rRows = 16;   // real rows per C2R block (pairs -> 8 complex rows)
constexpr int kBatch = 8;      // 16-byte global loads kept in flight per thread

__device__ __forceinline__ int nchunks(int H) { return (H + kChunk - 1) / kChunk; }

// Pencil tiles.  A tile is [len][kChunk] complex values of one spectrum
// plane, element (t, c) at bin t * stride + kx0 + c of src (zero for
// kx0 + c >= H); rows start on 64-byte boundaries (stride and kx0 are
// multiples of 16), so a thread moves two adjacent bins per access: 16 bytes
// of complex64 or 8 bytes of two packed 16-bit complex values.  prefetch()
// issues all of a thread's loads of one tile (PF = len * kChunk / 2 /
// kPassThreads of them) into registers, as stored; commit() widens them to
// float32 in LDS.  Issuing the loads of two or three tiles before the first
// commit keeps one memory round trip per block.  Rows t with keep[t] == 0
// (keep non-null) are known to be zero and are not read.
template <int ST> struct PairOf { typedef uint2 T; };
template <> struct PairOf<kSpecF32> { typedef float4 T; };
template <int ST> using PairT = typename PairOf<ST>::T;
template <int ST> constexpr size_t kBinBytes = ST == kSpecF32 ? 8 : 4;

// address of bin i of a spectrum array of storage ST
template <int ST>
__device__ __forceinline__ char *bin_at(void *spec, size_t i) {
    return static_cast<char *>(spec) + i * kBinBytes<ST>;
}

template <int ST, int PF>
__device__ __forceinline__ void prefetch(PairT<ST> (&v)[PF], const char *__restrict__ src, size_t stride, int len,
                                         int kx0, int H, const uint8_t *keep) {
    const int tot2 = len * (kChunk / 2);
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int i = u * kPassThreads + threadIdx.x;
        const int t = i / (kChunk / 2), c = 2 * (i % (kChunk / 2));
        PairT<ST> w = {};
        if (i < tot2 && kx0 + c < H && (!keep || keep[t]))
            w = *reinterpret_cast<const PairT<ST> *>(src + (t * stride + kx0 + c) * kBinBytes<ST>);
        if (kx0 + c + 1 >= H) {  // the pair's second bin is row padding
            if constexpr (ST == kSpecF32) {
                w.z = 0.f;
                w.w = 0.f;
            } else {
                w.y = 0u;
            }
        }
        v[u] = w;
    }
}

template <int ST, int PF>
__device__ __forceinline__ void commit(float2 *dst, const PairT<ST> (&v)[PF], int len) {
    const int tot2 = len * (kChunk / 2);
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int i = u * kPassThreads + threadIdx.x;
        if (i >= tot2) continue;
        if constexpr (ST == kSpecF32) {
            reinterpret_cast<float4 *>(dst)[i] = v[u];
        } else {
            const float2 a = spec_unpack<ST>(v[u].x), b = spec_unpack<ST>(v[u].y);
            reinterpret_cast<float4 *>(dst)[i] = make_float4(a.x, a.y, b.x, b.y);
        }
    }
}

// Writes a tile back; the 16-bit storages store it times `scale`.
template <int ST>
__device__ __forceinline__ void store_pencils(char *__restrict__ dstg, const float2 *src, size_t stride, int len,
                                              int kx0, int H, float scale) {
    const int tot2 = len * (kChunk / 2);
    for (int i = threadIdx.x; i < tot2; i += kPassThreads) {
        const int t = i / (kChunk / 2), c = 2 * (i % (kChunk / 2));
        const float4 v = reinterpret_cast<const float4 *>(src)[i];
        char *d = dstg + (t * stride + kx0 + c) * kBinBytes<ST>;
        if constexpr (ST == kSpecF32) {
            if (kx0 + c + 1 < H)
                *reinterpret_cast<float4 *>(d) = v;
            else if (kx0 + c < H)
                *reinterpret_cast<float2 *>(d) = make_float2(v.x, v.y);
        } else {
            const unsigned pa = spec_pack<ST>(make_float2(v.x * scale, v.y * scale));
            const unsigned pb = spec_pack<ST>(make_float2(v.z * scale, v.w * scale));
            if (kx0 + c + 1 < H)
                *reinterpret_cast<uint2 *>(d) = make_uint2(pa, pb);
            else if (kx0 + c < H)
                *reinterpret_cast<unsigned *>(d) = pa;
        }
    }
}

template <int ST, int PF>
__global__ void __launch_bounds__(kPassThreads)
fft_y_fwd_kernel(void *__restrict__ spec, const uint8_t *__restrict__ occ, uint8_t *__restrict__ zocc,
                 DevStatus *__restrict__ st, Grid g, FftAxis ay) {
    extern __shared__ __attribute__((aligned(16))) float2 lds[];
    __shared__ uint8_t keep[kMaxDim];
    __shared__ int any;
    const int Ny = g.n[1], H = g.H, Hp = g.Hp;
    const size_t plane = (size_t)g.n[2] * Ny * Hp;
    const int nch = nchunks(H);
    const int chunk = blockIdx.x % nch, z = blockIdx.x / nch;
    const int k0 = chunk * kChunk;
    // rows of this z plane that the splat wrote (their tile holds a point)
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const uint8_t *orow = occ + (size_t)(z / g.tz) * g.tiles_y;
    for (int y = threadIdx.x; y < Ny; y += blockDim.x) {
        const uint8_t o = orow[y / g.ty];
        keep[y] = o;
        if (o) any = 1;
    }
    __syncthreads();
    if (chunk == 0 && threadIdx.x == 0) {
        zocc[z] = any ? 1 : 0;
        if (any) atomicAdd(&st->n_zplanes, 1);  // planes the later passes read
    }
    if (!any) return;  // an all-zero plane stays zero through the y transform
    float2 *A = lds, *B = lds + Ny * kChunk, *tw = lds + 2 * Ny * kChunk;
    const int tot = Ny * kChunk;
    const size_t zoff = (size_t)z * Ny * Hp;
    const float sy = ST == kSpecF32 ? 1.0f : g.fscale[1];  // the y share of the inverse's 1/n
    PairT<ST> va[PF], vb[PF], vc[PF];
    prefetch<ST, PF>(va, bin_at<ST>(spec, zoff), Hp, Ny, k0, H, keep);
    prefetch<ST, PF>(vb, bin_at<ST>(spec, plane + zoff), Hp, Ny, k0, H, keep);
    load_twiddles(tw, ay);
    commit<ST, PF>(A, va, Ny);
    commit<ST, PF>(B, vb, Ny);
    prefetch<ST, PF>(vc, bin_at<ST>(spec, 2 * plane + zoff), Hp, Ny, k0, H, keep);  // in flight during the transforms
    __syncthreads();
    fft_rows<true>(RowsC{A, 1, kChunk}, kChunk, ay, tw, -1);
    fft_rows<true>(RowsC{B, 1, kChunk}, kChunk, ay, tw, -1);
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int ky = i / kChunk;
        const float w = deriv_w(ky, Ny, g.wstep[1]);
        const float2 b = B[i];
        A[i] = make_float2(A[i].x - w * b.y, A[i].y + w * b.x);
    }
    __syncthreads();
    store_pencils<ST>(bin_at<ST>(spec, zoff), A, Hp, Ny, k0, H, sy);
    commit<ST, PF>(B, vc, Ny);
    __syncthreads();
    fft_rows<true>(RowsC{B, 1, kChunk}, kChunk, ay, tw, -1);
    store_pencils<ST>(bin_at<ST>(spec, 2 * plane + zoff), B, Hp, Ny, k0, H, sy);
}

template <int ST, int PF>
__global__ void __launch_bounds__(kPassThreads)
fft_z_solve_kernel(void *__restrict__ spec, const uint8_t *__restrict__ zocc, Grid g, FftAxis az) {
    extern __shared__ __attribute__((aligned(16))) float2 lds[];
    __shared__ uint8_t keep[kMaxDim];
    const int Ny = g.n[1], Nz = g.n[2], H = g.H, Hp = g.Hp;
    for (int z = threadIdx.x; z < Nz; z += blockDim.x) keep[z] = zocc[z];
    __syncthreads();
    const size_t plane = (size_t)Nz * Ny * Hp;
    const size_t zstride = (size_t)Ny * Hp;
    const int nch = nchunks(H);
    const int chunk = blockIdx.x % nch, ky = blockIdx.x / nch;
    const int k0 = chunk * kChunk;
    float2 *A = lds, *B = lds + Nz * kChunk, *tw = lds + 2 * Nz * kChunk;
    const int tot = Nz * kChunk;
    const size_t yoff = (size_t)ky * Hp;
    PairT<ST> va[PF], vb[PF];
    prefetch<ST, PF>(va, bin_at<ST>(spec, yoff), zstride, Nz, k0, H, keep);
    prefetch<ST, PF>(vb, bin_at<ST>(spec, 2 * plane + yoff), zstride, Nz, k0, H, keep);
    load_twiddles(tw, az);
    commit<ST, PF>(A, va, Nz);
    commit<ST, PF>(B, vb, Nz);
    __syncthreads();
    fft_rows<true>(RowsC{A, 1, kChunk}, kChunk, az, tw, -1);
    fft_rows<true>(RowsC{B, 1, kChunk}, kChunk, az, tw, -1);
    const float wy = (float)kappa(ky, Ny) * g.wstep[1];
    const float sz = ST == kSpecF32 ? 1.0f : g.fscale[2];  // the z share of the inverse's 1/n
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int kz = i / kChunk, c = i % kChunk, kx = k0 + c;
        const float wx = (float)kappa(kx, g.n[0]) * g.wstep[0];
        const float wzf = (float)kappa(kz, Nz) * g.wstep[2];
        const float w2 = wx * wx + wy * wy + wzf * wzf;
        const float inv = w2 > 0.f ? sz / w2 : 0.0f;
        const float wz = deriv_w(kz, Nz, g.wstep[2]);
        const float2 b = B[i];
        const float2 a = A[i];
        A[i] = make_float2((a.x - wz * b.y) * inv, (a.y + wz * b.x) * inv);
    }
    __syncthreads();
    fft_rows<true>(RowsC{A, 1, kChunk}, kChunk, az, tw, +1);
    store_pencils<ST>(bin_at<ST>(spec, yoff), A, zstride, Nz, k0, H, 1.0f);
}

template <int ST, int PF>
__global__ void __launch_bounds__(kPassThreads)
fft_y_inv_kernel(void *__restrict__ spec, Grid g, FftAxis ay) {
    extern __shared__ __attribute__((aligned(16))) float2 lds[];
    const int Ny = g.n[1], H = g.H, Hp = g.Hp;
    const int nch = nchunks(H);
    const int chunk = blockIdx.x % nch, z = blockIdx.x / nch;
    const int k0 = chunk * kChunk;
    const size_t zoff = (size_t)z * Ny * Hp;
    float2 *tw = lds + Ny * kChunk;
    PairT<ST> va[PF];
    prefetch<ST, PF>(va, bin_at<ST>(spec, zoff), Hp, Ny, k0, H, nullptr);
    load_twiddles(tw, ay);
    commit<ST, PF>(lds, va, Ny);
    __syncthreads();
    fft_rows<true>(RowsC{lds, 1, kChunk}, kChunk, ay, tw, +1);
    store_pencils<ST>(bin_at<ST>(spec, zoff), lds, Hp, Ny, k0, H, 1.0f);
}

// Inverse real transform along x.  Two real rows a, b (consecutive linear
// rows) are recovered together from one complex transform of
// Z[k] = X_a[k] + i X_b[k], with X[k] for k > Nx/2 taken as conj(X[Nx-k])
// (Hermitian symmetry of a real row's spectrum); the imaginary parts of the
// k = 0 and k = Nx/2 bins are dropped, as a real row's spectrum has none.
// A 16-bit storage that overflowed leaves a non-finite value in A: the pass
// flags it (kFlagRange).
template <int ST>
__global__ void __launch_bounds__(kPassThreads)
fft_x_c2r_kernel(const void *__restrict__ spec, float *__restrict__ A, float2 *__restrict__ rowmm,
                 DevStatus *__restrict__ st, Grid g, FftAxis ax, float scale) {
    extern __shared__ __attribute__((aligned(16))) float2 lds[];
    const int Nx = g.n[0], Hp = g.Hp;
    const int nrows = g.n[1] * g.n[2];
    const int row0 = blockIdx.x * kC2rRows;
    const int ncx = kC2rRows / 2;
    const int tot = ncx * Nx;
    float2 *tw = lds + tot;
    load_twiddles(tw, ax);
    const unsigned mN = div_magic(Nx);
    for (int base = 0; base < tot; base += kBatch * kPassThreads) {
        float2 xa[kBatch], xb[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int i = base + u * kPassThreads + threadIdx.x;
            const int jr = udiv(i, Nx, mN), k = i - jr * Nx;
            const int ra = row0 + 2 * jr;
            xa[u] = xb[u] = make_float2(0.f, 0.f);
            if (i < tot && ra < nrows) {
                const int kk = k > Nx / 2 ? Nx - k : k;
                xa[u] = spec_ld<ST>(spec, (size_t)ra * Hp + kk);
                xb[u] = spec_ld<ST>(spec, (size_t)(ra + 1) * Hp + kk);
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int i = base + u * kPassThreads + threadIdx.x;
            if (i >= tot) continue;
            const int jr = udiv(i, Nx, mN), k = i - jr * Nx;
            float2 a = xa[u], b = xb[u];
            if (k > Nx / 2) {
                a.y = -a.y;
                b.y = -b.y;
            }
            if (k == 0 || 2 * k == Nx) {
                a.y = 0.f;
                b.y = 0.f;
            }
            lds[i] = make_float2(a.x - b.y, a.y + b.x);
        }
    }
    __syncthreads();
    fft_rows<false>(RowsC{lds, Nx, 1}, ncx, ax, tw, +1);
    bool bad = false;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int jr = udiv(i, Nx, mN), k = i - jr * Nx;
        const int ra = row0 + 2 * jr;
        if (ra < nrows) {
            const float2 z = lds[i];
            A[(size_t)ra * Nx + k] = z.x * scale;
            A[(size_t)(ra + 1) * Nx + k] = z.y * scale;
            if constexpr (ST != kSpecF32) bad |= !__builtin_isfinite(z.x) || !__builtin_isfinite(z.y);
        }
    }
    if constexpr (ST != kSpecF32)
        if (bad) atomicOr(&st->flags, kFlagRange);
    // (min, max) of each real row as stored, one wave per complex row
    const int lane = threadIdx.x & 63;
    for (int jr = threadIdx.x >> 6; jr < ncx; jr += blockDim.x >> 6) {
        const int ra = row0 + 2 * jr;
        if (ra >= nrows) break;  // uniform across the wave
        float4 mm = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
        for (int k = lane; k < Nx; k += 64) {
            const float2 z = lds[jr * Nx + k];
            const float va = z.x * scale, vb = z.y * scale;
            mm = make_float4(fminf(mm.x, va), fmaxf(mm.y, va), fminf(mm.z, vb), fmaxf(mm.w, vb));
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            mm.x = fminf(mm.x, __shfl_xor(mm.x, d, 64));
            mm.y = fmaxf(mm.y, __shfl_xor(mm.y, d, 64));
            mm.z = fminf(mm.z, __shfl_xor(mm.z, d, 64));
            mm.w = fmaxf(mm.w, __shfl_xor(mm.w, d, 64));
        }
        if (lane == 0) {
            rowmm[ra] = make_float2(mm.x, mm.y);
            rowmm[ra + 1] = make_float2(mm.z, mm.w);
        }
    }
}

// ---------------------------------------------------------------------------
// Register pencils, for transform lengths N = N1 N2 with N2 dividing N1
// (16, 32, 64, 128, 256).  A block of 16 N2 threads transforms the 16 columns
// of one chunk; thread (c, t) = (tid % 16, tid / 16) holds N1 elements of
// column c in registers:
//   input    x[n1] = row t + N2 n1, read straight from the spectrum (for a
//            fixed register the 16 lanes of a row read 128 contiguous bytes)
//   step 1   N1-point DFT over n1, then the twiddle w_N^(t k1)
//   LDS      one exchange: thread t takes k1 = t + N2 q (q < Q = N1 / N2)
//   step 2   N2-point DFTs over n2
//   output   x[q N2 + k2] = X[k1 + N1 k2] = row t + N2 (q + Q k2)
// The output rows of thread t have the input form t + N2 m again
// (m = q + Q k2), so an inverse transform starts from the registers after a
// register permutation.
// Raw buffer access to the spectrum allocation (three planes, below 2 GiB at
// 512^3): 32-bit byte offsets from one 128-bit resource instead of a 64-bit
// address per element, and the hardware's range check does the masking - a
// load past the range returns zero and a store past it is dropped - so rows
// known to be zero and idle lanes need neither a branch nor a memory access.
// (Word 3 of the resource: the raw 32-bit-element format of gfx9-family GPUs.)
constexpr unsigned kOob = 0xFFFFFFF0u;  // an offset past any spectrum allocation

// One spectrum plane behind a buffer resource, storage ST (kB bytes per bin).
template <int ST>
struct SpecBuf {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    static constexpr unsigned kB = ST == kSpecF32 ? 8u : 4u;
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ SpecBuf(const void *base, unsigned bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000)) {}
    __device__ __forceinline__ float2 load(unsigned off) const {
        if constexpr (ST == kSpecF32)
            return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        else
            return spec_unpack<ST>(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    __device__ __forceinline__ void store(unsigned off, float2 v) const {
        if constexpr (ST == kSpecF32)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(spec_pack<ST>(v), r, off, 0, 0);
    }
};

// byte address of plane p of a spectrum array with bins of kB bytes
template <int ST>
__device__ __forceinline__ const char *plane_base(const void *spec, size_t plane, int p) {
    return static_cast<const char *>(spec) + (size_t)p * plane * SpecBuf<ST>::kB;
}

template <int N1, int N2>
struct Pencil {
    static constexpr int N = N1 * N2, Q = N1 / N2, THREADS = 16 * N2;
    // LDS stride of one k1 group: 16 columns per n2 plus 16 padding values,
    // so the four row groups of a wave's read fall in alternate bank halves
    static constexpr int KS = 16 * N2 + 16;
    static constexpr int EX = N1 * KS;
    static_assert(N1 % N2 == 0, "N2 must divide N1");

    __device__ __forceinline__ static int in_row(int t, int n1) { return t + N2 * n1; }
    __device__ __forceinline__ static int out_row(int t, int i) {
        return t + N2 * (i / N2 + Q * (i % N2));
    }

    // Transform the block's columns; `tw` holds w_N^m = exp(-2 pi i m / N),
    // m < N; `ex` is free for reuse when this returns.  FACTORED (N1 = 16):
    // w^(t k1) = w^(t (k1 mod 4)) w^(4 t (k1 div 4)) from 6 table entries
    // instead of 15 (fewer registers held, one more rounding).
    template <int DIR, bool FACTORED = false>
    __device__ __forceinline__ static void run(float2 (&x)[N1], float2 *ex, const float2 *tw, int c,
                                               int t) {
        Dft<N1>::run(x, DIR);
        if constexpr (FACTORED) {
            static_assert(N1 == 16, "factored twiddles for 16 registers");
            float2 lo[4], hi[4];
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                lo[k] = tw[t * k];
                hi[k] = tw[4 * t * k];
            }
#pragma unroll
            for (int k1 = 1; k1 < N1; ++k1) {
                const int a = k1 & 3, b = k1 >> 2;
                float2 w = a == 0 ? hi[b] : b == 0 ? lo[a] : cmul(lo[a], hi[b]);
                if (DIR > 0) w.y = -w.y;
                x[k1] = cmul(x[k1], w);
            }
        } else {
#pragma unroll
            for (int k1 = 1; k1 < N1; ++k1) {
                float2 w = tw[t * k1];
                if (DIR > 0) w.y = -w.y;
                x[k1] = cmul(x[k1], w);
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) ex[k1 * KS + t * 16 + c] = x[k1];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2) x[q * N2 + n2] = ex[(t + N2 * q) * KS + n2 * 16 + c];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) Dft<N2>::run(x + q * N2, DIR);
    }

    // Output register q N2 + k2 becomes input register q + Q k2.
    __device__ __forceinline__ static void to_input(float2 (&x)[N1]) {
        float2 y[N1];
#pragma unroll
        for (int i = 0; i < N1; ++i) y[i / N2 + Q * (i % N2)] = x[i];
#pragma unroll
        for (int i = 0; i < N1; ++i) x[i] = y[i];
    }
};

template <int N1, int N2, int ST>
__global__ void __launch_bounds__(16 * N2)
pen_y_fwd_kernel(void *__restrict__ spec, const uint8_t *__restrict__ occ,
                 uint8_t *__restrict__ zocc, DevStatus *__restrict__ st, Grid g,
                 const float2 *__restrict__ twg) {
    using Pn = Pencil<N1, N2>;
    constexpr int N = Pn::N;  // = Ny
    __shared__ float2 ex[Pn::EX];
    __shared__ float2 tw[N];
    __shared__ uint8_t keep[N];
    __shared__ int any;
    const int H = g.H, Hp = g.Hp;
    const size_t plane = (size_t)g.n[2] * N * Hp;
    const int nch = nchunks(H);
    const int chunk = blockIdx.x % nch, z = blockIdx.x / nch;
    const int k0 = chunk * kChunk;
    const int c = threadIdx.x & 15, t = threadIdx.x >> 4;
    // rows of this z plane that the splat wrote (their tile holds a point)
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const uint8_t *orow = occ + (size_t)(z / g.tz) * g.tiles_y;
    for (int y = threadIdx.x; y < N; y += Pn::THREADS) {
        const uint8_t o = orow[y / g.ty];
        keep[y] = o;
        if (o) any = 1;
    }
    for (int i = threadIdx.x; i < N; i += Pn::THREADS) tw[i] = twg[i];
    __syncthreads();
    if (chunk == 0 && threadIdx.x == 0) {
        zocc[z] = any ? 1 : 0;
        if (any) atomicAdd(&st->n_zplanes, 1);  // planes the later passes read
    }
    if (!any) return;  // an all-zero plane stays zero through the y transform
    const bool col = k0 + c < H;
    // byte offsets: rows of tiles that no point reaches (and idle lanes) get
    // an offset past the range and read as zero
    // one resource per plane, so the same offsets serve all three
    using SB = SpecBuf<ST>;
    const unsigned plb = (unsigned)(plane * SB::kB);
    const SB s0(spec, plb), s1(plane_base<ST>(spec, plane, 1), plb), s2(plane_base<ST>(spec, plane, 2), plb);
    const unsigned o0 = (unsigned)(((size_t)z * N * Hp + k0 + c) * SB::kB);
    const unsigned rowb = (unsigned)Hp * SB::kB;
    // the reduced storages keep their share of the inverse's 1/n here
    const float sy = ST == kSpecF32 ? 1.0f : g.fscale[1];
    unsigned ro[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
        const int r = Pn::in_row(t, n1);
        ro[n1] = (col && keep[r]) ? o0 + (unsigned)r * rowb : kOob;
    }
    float2 a[N1], b[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
        a[n1] = s0.load(ro[n1]);
        b[n1] = s1.load(ro[n1]);
    }
    Pn::template run<-1>(a, ex, tw, c, t);
    Pn::template run<-1>(b, ex, tw, c, t);
    // P0 <- F_y P0 + j w_y F_y P1
    const unsigned so = col ? o0 : kOob;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const int r = Pn::out_row(t, i);
        const float w = deriv_w(r, N, g.wstep[1]);
        float2 v = make_float2(a[i].x - w * b[i].y, a[i].y + w * b[i].x);
        if (ST != kSpecF32) v = make_float2(v.x * sy, v.y * sy);
        s0.store(col ? so + (unsigned)r * rowb : kOob, v);
    }
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) b[n1] = s2.load(ro[n1]);
    Pn::template run<-1>(b, ex, tw, c, t);
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        float2 v = b[i];
        if (ST != kSpecF32) v = make_float2(v.x * sy, v.y * sy);
        s2.store(col ? so + (unsigned)Pn::out_row(t, i) * rowb : kOob, v);
    }
}

// Chunks of 16 columns leave the last column alone when H = 16 m + 1 (Nx a
// multiple of 32): a block for it would transform 15 columns of zeros.  The
// z pass then gives that column (kx = Nx/2) of kNyqLines ky lines to each of
// its first `nyqb` blocks, line kNyqLines b + c in the place of column c,
// and the other blocks the m full chunks of every line.  Each column gets
// the same arithmetic either way.  (The column's loads are 8 bytes per
// 128-byte line, so a few lines per block spread them over many CUs.  For
// the y pass, whose lines would be whole z planes apart, the chunk layout
// measured faster.)
constexpr int kNyqLines = 4;
static int nyquist_blocks(int H, int lines) {
    return (H > kChunk && (H - 1) % kChunk == 0) ? (lines + kNyqLines - 1) / kNyqLines : 0;
}

template <int N1, int N2, int ST>
__global__ void __launch_bounds__(16 * N2)
pen_z_solve_kernel(void *__restrict__ spec, const uint8_t *__restrict__ zocc, Grid g,
                   const float2 *__restrict__ twg, int nyqb) {
    using Pn = Pencil<N1, N2>;
    constexpr int N = Pn::N;  // = Nz
    __shared__ float2 ex[Pn::EX];
    __shared__ float2 tw[N];
    __shared__ uint8_t keep[N];
    const int Ny = g.n[1], H = g.H, Hp = g.Hp;
    for (int i = threadIdx.x; i < N; i += Pn::THREADS) {
        keep[i] = zocc[i];
        tw[i] = twg[i];
    }
    __syncthreads();
    // planes 0 and 2 through raw buffer resources: 32-bit byte offsets, and
    // z planes that stay zero (and idle lanes) read as zero without a load
    const size_t plane = (size_t)N * Ny * Hp;
    using SB = SpecBuf<ST>;
    const unsigned plb = (unsigned)(plane * SB::kB);
    const SB s0(spec, plb), s2(plane_base<ST>(spec, plane, 2), plb);
    const unsigned zsb = (unsigned)Ny * Hp * SB::kB;
    const int c = threadIdx.x & 15, t = threadIdx.x >> 4;
    int kx, ky;  // this thread's column
    bool col;
    if ((int)blockIdx.x < nyqb) {
        // column Nx/2 of line ky = kNyqLines b + c
        kx = H - 1;
        ky = kNyqLines * (int)blockIdx.x + c;
        col = c < kNyqLines && ky < Ny;
        if (!col) ky = 0;
    } else {
        const int b = (int)blockIdx.x - nyqb;
        const int nch = nyqb ? (H - 1) / kChunk : nchunks(H);
        kx = (b % nch) * kChunk + c;
        ky = b / nch;
        col = kx < H;
    }
    const unsigned o0 = (unsigned)(((size_t)ky * Hp + kx) * SB::kB);
    float2 a[N1], b[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
        const int r = Pn::in_row(t, n1);
        const unsigned o = (col && keep[r]) ? o0 + (unsigned)r * zsb : kOob;
        a[n1] = s0.load(o);
        b[n1] = s2.load(o);
    }
    Pn::template run<-1>(a, ex, tw, c, t);
    Pn::template run<-1>(b, ex, tw, c, t);
    // (F_z P0 + j w_z F_z P2) / |w|^2, zero at the DC bin
    const float wx = (float)kappa(kx, g.n[0]) * g.wstep[0];
    const float wy = (float)kappa(ky, Ny) * g.wstep[1];
    const float wxy = wx * wx + wy * wy;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const int kz = Pn::out_row(t, i);
        const float wzf = (float)kappa(kz, N) * g.wstep[2];
        const float w2 = wxy + wzf * wzf;
        // v_rcp_f32 (about 1 ulp) in place of a correctly rounded divide
        float inv = w2 > 0.f ? __builtin_amdgcn_rcpf(w2) : 0.0f;
        if (ST != kSpecF32) inv *= g.fscale[2];  // the z share of the inverse's 1/n
        const float wz = deriv_w(kz, N, g.wstep[2]);
        a[i] = make_float2((a[i].x - wz * b[i].y) * inv, (a[i].y + wz * b[i].x) * inv);
    }
    Pn::to_input(a);
    Pn::template run<+1>(a, ex, tw, c, t);
#pragma unroll
    for (int i = 0; i < N1; ++i) s0.store(col ? o0 + (unsigned)Pn::out_row(t, i) * zsb : kOob, a[i]);
}

template <int N1, int N2, int ST>
__global__ void __launch_bounds__(16 * N2)
pen_y_inv_kernel(void *__restrict__ spec, Grid g, const float2 *__restrict__ twg) {
    using Pn = Pencil<N1, N2>;
    constexpr int N = Pn::N;  // = Ny
    __shared__ float2 ex[Pn::EX];
    __shared__ float2 tw[N];
    for (int i = threadIdx.x; i < N; i += Pn::THREADS) tw[i] = twg[i];
    __syncthreads();
    const int H = g.H, Hp = g.Hp;
    const int nch = nchunks(H);
    const int chunk = blockIdx.x % nch, z = blockIdx.x / nch;
    const int k0 = chunk * kChunk;
    const int c = threadIdx.x & 15, t = threadIdx.x >> 4;
    const bool col = k0 + c < H;
    const size_t p = (size_t)z * N * Hp + k0 + c;
    float2 a[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1)
        a[n1] = col ? spec_ld<ST>(spec, p + (size_t)Pn::in_row(t, n1) * Hp) : make_float2(0.f, 0.f);
    Pn::template run<+1>(a, ex, tw, c, t);
#pragma unroll
    for (int i = 0; i < N1; ++i)
        if (col) spec_st<ST>(spec, p + (size_t)Pn::out_row(t, i) * Hp, a[i]);
}

// Inverse real transform along x for pencil lengths: a block takes 32 real
// rows (a, b) = (row0 + 2c, row0 + 2c + 1), c < 16, packed as complex rows
// Z_c[k] = X_a[k] + i X_b[k] (X[k] = conj X[N-k] above N/2; the imaginary
// parts of bins 0 and N/2 dropped), transforms the 16 columns as a pencil and
// writes Re -> row a, Im -> row b.  Spectra are read once each (both Z[k] and
// Z[N-k] come from the pair at k) and the real rows leave through LDS as
// 16-byte stores.
template <int N1, int N2, int ST>
__global__ void __launch_bounds__(16 * N2)
pen_x_c2r_kernel(const void *__restrict__ spec, float *__restrict__ A, float2 *__restrict__ rowmm,
                 DevStatus *__restrict__ st, Grid g, const float2 *__restrict__ twg, float scale) {
    using Pn = Pencil<N1, N2>;
    constexpr int N = Pn::N;  // = Nx
    constexpr int ZP = N + 1;       // LDS pitch of a packed complex row (float2)
    constexpr int OP = N + 4;       // LDS pitch of a real output row (float)
    constexpr int BUF = Pn::EX > 16 * ZP ? Pn::EX : 16 * ZP;
    static_assert(BUF * 2 >= 32 * OP, "output staging fits the buffer");
    __shared__ __attribute__((aligned(16))) float2 buf[BUF];
    __shared__ float2 tw[N];
    for (int i = threadIdx.x; i < N; i += Pn::THREADS) tw[i] = twg[i];
    const int Hp = g.Hp, H = N / 2 + 1;
    const int nrows = g.n[1] * g.n[2];
    const int row0 = blockIdx.x * 32;
    for (int i = threadIdx.x; i < 16 * H; i += Pn::THREADS) {
        const int c = i / H, k = i - c * H;
        const int ra = row0 + 2 * c;
        float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
        if (ra < nrows) {
            a = spec_ld<ST>(spec, (size_t)ra * Hp + k);
            b = spec_ld<ST>(spec, (size_t)(ra + 1) * Hp + k);
        }
        if (k == 0 || k == N / 2) {
            a.y = 0.f;
            b.y = 0.f;
        }
        buf[c * ZP + k] = make_float2(a.x - b.y, a.y + b.x);
        if (k > 0 && k < N / 2) buf[c * ZP + N - k] = make_float2(a.x + b.y, b.x - a.y);
    }
    __syncthreads();
    const int c = threadIdx.x & 15, t = threadIdx.x >> 4;
    float2 x[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) x[n1] = buf[c * ZP + Pn::in_row(t, n1)];
    __syncthreads();  // buf becomes the exchange buffer
    Pn::template run<+1>(x, buf, tw, c, t);
    float *ob = reinterpret_cast<float *>(buf);
    bool bad = false;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const int k = Pn::out_row(t, i);
        ob[(2 * c) * OP + k] = x[i].x * scale;
        ob[(2 * c + 1) * OP + k] = x[i].y * scale;
        if constexpr (ST != kSpecF32) bad |= !__builtin_isfinite(x[i].x) || !__builtin_isfinite(x[i].y);
    }
    if constexpr (ST != kSpecF32)
        if (bad) atomicOr(&st->flags, kFlagRange);
    __syncthreads();
    constexpr int Q4 = N / 4;  // float4 per real row
    // a row's Q4 float4 lie on consecutive lanes of one wave (Q4 divides 64
    // and the thread count): their (min, max) reduces over those lanes
    static_assert(64 % Q4 == 0 && Pn::THREADS % 64 == 0, "rows within a wave");
    for (int i = threadIdx.x; i < 32 * Q4; i += Pn::THREADS) {
        const int r = i / Q4, q = i - r * Q4;
        const float4 v = *reinterpret_cast<const float4 *>(ob + r * OP + 4 * q);
        if (row0 + r < nrows) *reinterpret_cast<float4 *>(A + (size_t)(row0 + r) * N + 4 * q) = v;
        float mn = fminf(fminf(v.x, v.y), fminf(v.z, v.w)), mx = fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w));
#pragma unroll
        for (int d = Q4 / 2; d > 0; d >>= 1) {
            mn = fminf(mn, __shfl_xor(mn, d, 64));
            mx = fmaxf(mx, __shfl_xor(mx, d, 64));
        }
        if (q == 0 && row0 + r < nrows) rowmm[row0 + r] = make_float2(mn, mx);
    }
}

// Pencil factorisation of a transform length, or 0 when it has none.
// Inverse y transform and inverse real x transform of one z plane in one
// block, for Nx = Ny = 256: the plane's y-inverse spectrum stays on chip
// (registers, then LDS) instead of making a round trip through HBM between
// two passes.  1024 threads in 4 groups of 256; group q runs the y pencil on
// column chunks q and q + 4 (kx < 128).  The kx = 0 and kx = 128 columns are
// spectra of real sequences along y (Hermitian in ky), so they share one
// transform: Z = X_0 + i X_128 gives x_0 = Re, x_128 = Im.  Then, for each
// half of the rows, the y-inverse rows go to LDS, each group packs 16 pairs
// of real rows as complex rows (as the c2r pass does), transforms them along
// x and the real rows leave through LDS as 16-byte stores.
constexpr int kYx = 256;
constexpr int kYxThreads = 1024;
constexpr int kYxYP = kYx / 2 + 1;  // LDS pitch of a y-inverse row (complex)
constexpr int kYxOP = kYx + 4;      // LDS pitch of a real output row (float)
using PenYx = Pencil<16, 16>;
constexpr int kYxBuf = 4 * PenYx::EX;  // float2: four exchange buffers
static_assert(kYxBuf >= (kYx / 2) * kYxYP, "half plane of y-inverse rows fits");
static_assert(2 * kYxBuf >= (kYx / 2) * kYxOP, "half plane of output rows fits");

template <int ST>
__global__ void __launch_bounds__(kYxThreads)
yx_inv256_kernel(const void *__restrict__ spec, float *__restrict__ A, float2 *__restrict__ rowmm,
                 DevStatus *__restrict__ st, Grid g, const float2 *__restrict__ twg, float scale) {
    using Pn = PenYx;
    constexpr int N = kYx;
    extern __shared__ __attribute__((aligned(16))) float2 smem[];
    float2 *buf = smem;            // exchange buffers / y-inverse rows / output rows
    float2 *tw = smem + kYxBuf;    // w_256^m (the same table serves x and y)
    float2 *nyq = tw + N;          // the Nyquist column kx = 128
    const int grp = threadIdx.x >> 8, lt = threadIdx.x & 255;
    const int c = lt & 15, t = lt >> 4;
    const int z = blockIdx.x, Hp = g.Hp;
    const size_t P = (size_t)z * N * Hp;  // the plane's first bin
    float2 *ex = buf + grp * Pn::EX;
    if (threadIdx.x < N) {
        tw[threadIdx.x] = twg[threadIdx.x];
        nyq[threadIdx.x] = spec_ld<ST>(spec, P + (size_t)threadIdx.x * Hp + N / 2);
    }

    // y-inverse of chunks grp and grp + 4 (columns 16 ch + c)
    // uniform row bases plus one 32-bit lane offset (in_row(t, n1) = t + 16 n1);
    // the first chunk's loads go first, so its transform can start while the
    // second chunk is still in flight
    float2 a[2][16];
    const unsigned lo = (unsigned)t * Hp + 16u * grp + c;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) a[h][n1] = spec_ld<ST>(spec, P + (size_t)(16 * n1) * Hp + lo + 64u * h);
    __syncthreads();  // twiddles and the Nyquist column
    if (grp == 0 && c == 0) {
        // column 0 carries the Nyquist column in its imaginary part
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const float2 w = nyq[Pn::in_row(t, n1)];
            a[0][n1] = make_float2(a[0][n1].x - w.y, a[0][n1].y + w.x);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) Pn::template run<+1, true>(a[h], ex, tw, c, t);
    // finish both transforms before the row writes (interleaving them raises
    // the register peak past 128 and spills)
    __builtin_amdgcn_sched_barrier(0);

    float *O = reinterpret_cast<float *>(buf);
    // out_row(t, i) = t + 16 i: row y lies in half y / 128 = i / 8, at
    // y - 128 half = out_row(t, i mod 8).  The loop body handles a[.][0..7];
    // the second half's values move down at its end.  Column 0 keeps the
    // pair (x_0, x_128) of the two real columns as one complex value.
    static_assert(Pn::Q == 1, "output row t + 16 i");
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        __syncthreads();  // exchange buffers (or the previous half's output rows) free
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kx = 16 * (grp + 4 * h) + c;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                buf[Pn::out_row(t, i) * kYxYP + kx] = a[h][i];
                a[h][i] = a[h][i + 8];
            }
        }
        __syncthreads();
        // group grp packs real rows (2p, 2p + 1), p = 16 grp + c, as
        // Z[k] = X_a[k] + i X_b[k] over the full length (X[N-k] = conj X[k]);
        // bins 0 and N/2 of a real row are real, both read from column 0
        const int ra = 2 * (16 * grp + c), rb = ra + 1;
        float2 x[16];
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const int k = Pn::in_row(t, n1);
            const int kk = k <= N / 2 ? k : N - k;
            const int col = kk == N / 2 ? 0 : kk;
            float2 xa = buf[ra * kYxYP + col], xb = buf[rb * kYxYP + col];
            if (kk == 0) {
                xa.y = 0.f;
                xb.y = 0.f;
            } else if (kk == N / 2) {
                xa = make_float2(xa.y, 0.f);
                xb = make_float2(xb.y, 0.f);
            }
            x[n1] = k <= N / 2 ? make_float2(xa.x - xb.y, xa.y + xb.x)
                               : make_float2(xa.x + xb.y, xb.x - xa.y);
        }
        __syncthreads();  // the rows are read: buf becomes the exchange buffers
        Pn::template run<+1, true>(x, ex, tw, c, t);
        // every group is past the exchange (run ends with a block barrier)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = Pn::out_row(t, i);
            O[ra * kYxOP + k] = x[i].x * scale;
            O[rb * kYxOP + k] = x[i].y * scale;
        }
        __syncthreads();
        // 128 rows of 64 float4, 16 lanes per row (4 float4 each): the row's
        // (min, max) as stored reduces over its 16 lanes
        constexpr int Q4 = N / 4;
        static_assert(kYxThreads / 16 * 2 == 128 && Q4 == 64, "two row passes of 64 rows");
        float *dst = A + ((size_t)z * N + 128 * half) * N;
        // the lane from the exec mask and the wave index as a scalar: no
        // thread index needs to stay live into this loop
        const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int l16 = lane & 15;
        bool bad = false;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int r = 4 * wave + (lane >> 4) + 64 * v;
            float mn = INFINITY, mx = -INFINITY;
#pragma unroll
            for (int u = 0; u < Q4 / 16; ++u) {
                const int q = l16 + 16 * u;
                const float4 e = *reinterpret_cast<const float4 *>(O + r * kYxOP + 4 * q);
                *reinterpret_cast<float4 *>(dst + (unsigned)(r * N + 4 * q)) = e;
                mn = fminf(mn, fminf(fminf(e.x, e.y), fminf(e.z, e.w)));
                mx = fmaxf(mx, fmaxf(fmaxf(e.x, e.y), fmaxf(e.z, e.w)));
                if constexpr (ST != kSpecF32)
                    bad |= !__builtin_isfinite(e.x) || !__builtin_isfinite(e.y) || !__builtin_isfinite(e.z) ||
                           !__builtin_isfinite(e.w);
            }
#pragma unroll
            for (int d = 8; d > 0; d >>= 1) {
                mn = fminf(mn, __shfl_xor(mn, d, 16));
                mx = fmaxf(mx, __shfl_xor(mx, d, 16));
            }
            if (l16 == 0) rowmm[(size_t)z * N + 128 * half + r] = make_float2(mn, mx);
        }
        if constexpr (ST != kSpecF32)
            if (bad) atomicOr(&st->flags, kFlagRange);
    }
}

size_t yx_inv256_lds() { return (size_t)(kYxBuf + 2 * kYx) * sizeof(float2); }

// Both inverse passes for Nx = Ny = 128: two 512-thread blocks per z plane,
// block (z, h) writing rows y = 64 h .. 64 h + 63 of A (two blocks per plane
// keep the whole chip busy at 128 planes; each runs the plane's y inverse,
// a few MB of extra reads at 128^3).  Four groups of 128 threads run the
// 16 x 8 register pencil along y on column chunks kx = 16 q + c (kx < 64);
// the kx = 0 and kx = 64 columns share one transform (Z = X_0 + i X_64, as in
// the 256 kernel).  The half's y-inverse rows go to LDS, pairs of real rows
// are packed as complex rows and transformed along x with the same pencil,
// and the rows leave through LDS as 16-byte stores with their (min, max).
constexpr int kYh = 128;
constexpr int kYhThreads = 512;
using PenYh = Pencil<16, 8>;
constexpr int kYhYP = kYh / 2 + 1;     // LDS pitch of a y-inverse row (complex)
constexpr int kYhOP = kYh + 4;         // LDS pitch of a real output row (float)
constexpr int kYhBuf = 4 * PenYh::EX;  // float2: four exchange buffers
static_assert(kYhBuf >= (kYh / 2) * kYhYP, "half plane of y-inverse rows fits");
static_assert(2 * kYhBuf >= (kYh / 2) * kYhOP, "half plane of output rows fits");
static_assert(PenYh::THREADS * 4 == kYhThreads, "four groups");

template <int ST>
__global__ void __launch_bounds__(kYhThreads)
yx_inv128_kernel(const void *__restrict__ spec, float *__restrict__ A, float2 *__restrict__ rowmm,
                 DevStatus *__restrict__ st, Grid g, const float2 *__restrict__ twg, float scale) {
    using Pn = PenYh;
    constexpr int N = kYh;
    extern __shared__ __attribute__((aligned(16))) float2 smem[];
    float2 *buf = smem;           // exchange buffers / y-inverse rows / output rows
    float2 *tw = smem + kYhBuf;   // w_128^m (the same table serves x and y)
    float2 *nyq = tw + N;         // the Nyquist column kx = 64
    const int grp = threadIdx.x >> 7, lt = threadIdx.x & 127;
    const int c = lt & 15, t = lt >> 4;
    const int z = blockIdx.x >> 1, h = blockIdx.x & 1, Hp = g.Hp;
    const size_t P = (size_t)z * N * Hp;  // the plane's first bin
    float2 *ex = buf + grp * Pn::EX;
    if (threadIdx.x < N) {
        tw[threadIdx.x] = twg[threadIdx.x];
        nyq[threadIdx.x] = spec_ld<ST>(spec, P + (size_t)threadIdx.x * Hp + N / 2);
    }
    const int kx = 16 * grp + c;
    float2 a[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) a[n1] = spec_ld<ST>(spec, P + (size_t)Pn::in_row(t, n1) * Hp + kx);
    __syncthreads();  // twiddles and the Nyquist column
    if (kx == 0) {
        // column 0 carries the Nyquist column in its imaginary part
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const float2 w = nyq[Pn::in_row(t, n1)];
            a[n1] = make_float2(a[n1].x - w.y, a[n1].y + w.x);
        }
    }
    Pn::template run<+1>(a, ex, tw, c, t);
    // this half's y-inverse rows to LDS (the exchange buffers are free)
    float2 *Y = buf;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = Pn::out_row(t, i);
        if ((r >> 6) == h) {
            const int rr = r & 63;
            if (kx == 0) {
                Y[rr * kYhYP] = make_float2(a[i].x, 0.f);
                Y[rr * kYhYP + N / 2] = make_float2(a[i].y, 0.f);
            } else {
                Y[rr * kYhYP + kx] = a[i];
            }
        }
    }
    __syncthreads();
    // groups 0 and 1 pack real rows (2p, 2p + 1), p = 16 grp + c, of the half
    // as Z[k] = X_a[k] + i X_b[k] over the full length; groups 2 and 3 run the
    // transform on zeros (its barriers are the block's)
    const int p = 16 * grp + c, ra = 2 * p, rb = ra + 1;
    float2 x[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
        x[n1] = make_float2(0.f, 0.f);
        if (p < 32) {
            const int k = Pn::in_row(t, n1);
            const int kk = k <= N / 2 ? k : N - k;
            float2 xa = Y[ra * kYhYP + kk], xb = Y[rb * kYhYP + kk];
            if (kk == 0 || kk == N / 2) {
                xa.y = 0.f;
                xb.y = 0.f;
            }
            x[n1] = k <= N / 2 ? make_float2(xa.x - xb.y, xa.y + xb.x) : make_float2(xa.x + xb.y, xb.x - xa.y);
        }
    }
    __syncthreads();  // the rows are read: buf becomes the exchange buffers
    Pn::template run<+1>(x, ex, tw, c, t);
    float *O = reinterpret_cast<float *>(buf);
    bool bad = false;
    if (p < 32) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = Pn::out_row(t, i);
            O[ra * kYhOP + k] = x[i].x * scale;
            O[rb * kYhOP + k] = x[i].y * scale;
            if constexpr (ST != kSpecF32) bad |= !__builtin_isfinite(x[i].x) || !__builtin_isfinite(x[i].y);
        }
    }
    if constexpr (ST != kSpecF32)
        if (bad) atomicOr(&st->flags, kFlagRange);
    __syncthreads();
    // 64 rows of 32 float4: 32 lanes per row, two rows per wave; each row's
    // (min, max) reduces over its lanes
    constexpr int Q4 = N / 4;
    static_assert((64 * Q4) % kYhThreads == 0 && Q4 == 32, "whole rows per wave");
    float *dst = A + ((size_t)z * N + 64 * h) * N;
#pragma unroll
    for (int i = threadIdx.x; i < 64 * Q4; i += kYhThreads) {
        const int r = i / Q4, q = i - r * Q4;
        const float4 v = *reinterpret_cast<const float4 *>(O + r * kYhOP + 4 * q);
        *reinterpret_cast<float4 *>(dst + (size_t)r * N + 4 * q) = v;
        float mn = fminf(fminf(v.x, v.y), fminf(v.z, v.w)), mx = fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w));
#pragma unroll
        for (int d = 16; d > 0; d >>= 1) {
            mn = fminf(mn, __shfl_xor(mn, d, 32));
            mx = fmaxf(mx, __shfl_xor(mx, d, 32));
        }
        if (q == 0) rowmm[(size_t)z * N + 64 * h + r] = make_float2(mn, mx);
    }
}

size_t yx_inv128_lds() { return (size_t)(kYhBuf + 2 * kYh) * sizeof(float2); }

static int pencil_code(int n) {
    switch (n) {
        case 16: return 44;
        case 32: return 84;
        case 64: return 88;
        case 128: return 168;
        case 256: return 1616;
        default: return 0;
    }
}

#define FVR_PEN_SWITCH(code, KERNEL, ARGS, GRID)                                          \
    switch (code) {                                                                       \
        case 44: KERNEL<4, 4><<<GRID, 64, 0, s>>> ARGS; break;                          \
        case 84: KERNEL<8, 4><<<GRID, 64, 0, s>>> ARGS; break;                          \
        case 88: KERNEL<8, 8><<<GRID, 128, 0, s>>> ARGS; break;                         \
        case 168: KERNEL<16, 8><<<GRID, 128, 0, s>>> ARGS; break;                       \
        default: KERNEL<16, 16><<<GRID, 256, 0, s>>> ARGS; break;                       \
    }

#define FVR_PEN_SWITCH3(code, KERNEL, ST, ARGS, GRID)                                     \
    switch (code) {                                                                       \
        case 44: KERNEL<4, 4, ST><<<GRID, 64, 0, s>>> ARGS; break;                      \
        case 84: KERNEL<8, 4, ST><<<GRID, 64, 0, s>>> ARGS; break;                      \
        case 88: KERNEL<8, 8, ST><<<GRID, 128, 0, s>>> ARGS; break;                     \
        case 168: KERNEL<16, 8, ST><<<GRID, 128, 0, s>>> ARGS; break;                   \
        default: KERNEL<16, 16, ST><<<GRID, 256, 0, s>>> ARGS; break;                   \
    }

// Per-thread prefetch depth for a pencil length: len * kChunk / 2 / 256 16-byte loads.
static int prefetch_depth(int len) {
    const int need = (len * (kChunk / 2) + kPassThreads - 1) / kPassThreads;
    return need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
}

#define FVR_PF_SWITCH(len, KERNEL, ST, ARGS, ...)                                         \
    switch (prefetch_depth(len)) {                                                        \
        case 2: KERNEL<ST, 2><<<__VA_ARGS__>>> ARGS; break;                              \
        case 4: KERNEL<ST, 4><<<__VA_ARGS__>>> ARGS; break;                              \
        case 8: KERNEL<ST, 8><<<__VA_ARGS__>>> ARGS; break;                              \
        default: KERNEL<ST, 16><<<__VA_ARGS__>>> ARGS; break;                            \
    }
// Stockham kernels instantiated for the spectrum storage of the grid.
#define FVR_PF_ST(len, KERNEL, ARGS, ...)                                                 \
    switch (g.spec_st) {                                                                  \
        case kSpecBF16: { FVR_PF_SWITCH(len, KERNEL, kSpecBF16, ARGS, __VA_ARGS__) } break; \
        case kSpecF16: { FVR_PF_SWITCH(len, KERNEL, kSpecF16, ARGS, __VA_ARGS__) } break;   \
        default: { FVR_PF_SWITCH(len, KERNEL, kSpecF32, ARGS, __VA_ARGS__) } break;         \
    }

template <int ST>
static hipError_t configure_stockham() {
    const void *k[] = {(const void *)fft_y_fwd_kernel<ST, 2>,   (const void *)fft_y_fwd_kernel<ST, 4>,
                       (const void *)fft_y_fwd_kernel<ST, 8>,   (const void *)fft_y_fwd_kernel<ST, 16>,
                       (const void *)fft_z_solve_kernel<ST, 2>, (const void *)fft_z_solve_kernel<ST, 4>,
                       (const void *)fft_z_solve_kernel<ST, 8>, (const void *)fft_z_solve_kernel<ST, 16>,
                       (const void *)fft_y_inv_kernel<ST, 2>,   (const void *)fft_y_inv_kernel<ST, 4>,
                       (const void *)fft_y_inv_kernel<ST, 8>,   (const void *)fft_y_inv_kernel<ST, 16>,
                       (const void *)fft_x_c2r_kernel<ST>};
    for (const void *f : k) {
        hipError_t e = raise_dynamic_lds(f);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fft_configure() {
    hipError_t e = configure_stockham<kSpecF32>();
    if (e == hipSuccess) e = configure_stockham<kSpecBF16>();
    if (e == hipSuccess) e = configure_stockham<kSpecF16>();
    if (e != hipSuccess) return e;
    const void *k[] = {(const void *)yx_inv256_kernel<kSpecF32>,
                       (const void *)yx_inv256_kernel<kSpecBF16>, (const void *)yx_inv256_kernel<kSpecF16>,
                       (const void *)yx_inv128_kernel<kSpecF32>, (const void *)yx_inv128_kernel<kSpecBF16>,
                       (const void *)yx_inv128_kernel<kSpecF16>};
    for (const void *f : k) {
        e = raise_dynamic_lds(f);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// pencil buffers plus the twiddle table
static size_t pass_lds(int n, int bufs) { return ((size_t)bufs * n * kChunk + n) * sizeof(float2); }

// Pencil kernels instantiated for the spectrum storage of the grid.
#define FVR_PEN_ST(code, KERNEL, ARGS, GRID)                                                  \
    switch (g.spec_st) {                                                                      \
        case kSpecBF16: { FVR_PEN_SWITCH3(code, KERNEL, kSpecBF16, ARGS, GRID) } break;       \
        case kSpecF16: { FVR_PEN_SWITCH3(code, KERNEL, kSpecF16, ARGS, GRID) } break;         \
        default: { FVR_PEN_SWITCH3(code, KERNEL, kSpecF32, ARGS, GRID) } break;               \
    }

hipError_t launch_fft_y_fwd(void *spec, const uint8_t *occ, uint8_t *zocc, DevStatus *st,
                            const Grid &g, const FftAxis &ax, hipStream_t s) {
    const int nch = (g.H + kChunk - 1) / kChunk;
    if (const int pc = pencil_code(g.n[1])) {
        FVR_PEN_ST(pc, pen_y_fwd_kernel, (spec, occ, zocc, st, g, ax.tw), dim3(nch * g.n[2]))
        return hipGetLastError();
    }
    FVR_PF_ST(g.n[1], fft_y_fwd_kernel, (spec, occ, zocc, st, g, ax), dim3(nch * g.n[2]), dim3(kPassThreads),
              pass_lds(g.n[1], 2), s)
    return hipGetLastError();
}

hipError_t launch_fft_z_solve(void *spec, const uint8_t *zocc, const Grid &g, const FftAxis &ax,
                              hipStream_t s) {
    const int nch = (g.H + kChunk - 1) / kChunk;
    if (const int pc = pencil_code(g.n[2])) {
        const int nyqb = nyquist_blocks(g.H, g.n[1]);
        const int blocks = nyqb ? nyqb + (g.H - 1) / kChunk * g.n[1] : nch * g.n[1];
        FVR_PEN_ST(pc, pen_z_solve_kernel, (spec, zocc, g, ax.tw, nyqb), dim3(blocks))
        return hipGetLastError();
    }
    FVR_PF_ST(g.n[2], fft_z_solve_kernel, (spec, zocc, g, ax), dim3(nch * g.n[1]), dim3(kPassThreads),
              pass_lds(g.n[2], 2), s)
    return hipGetLastError();
}

hipError_t launch_fft_y_inv(void *spec, const Grid &g, const FftAxis &ax, hipStream_t s) {
    const int nch = (g.H + kChunk - 1) / kChunk;
    if (const int pc = pencil_code(g.n[1])) {
        FVR_PEN_ST(pc, pen_y_inv_kernel, (spec, g, ax.tw), dim3(nch * g.n[2]))
        return hipGetLastError();
    }
    FVR_PF_ST(g.n[1], fft_y_inv_kernel, (spec, g, ax), dim3(nch * g.n[2]), dim3(kPassThreads), pass_lds(g.n[1], 1),
              s)
    return hipGetLastError();
}

bool fft_yx_fused(const Grid &g) {
    return (g.n[0] == kYx && g.n[1] == kYx) || (g.n[0] == kYh && g.n[1] == kYh);
}

hipError_t launch_fft_yx_inv(const void *spec, float *A, float2 *rowmm, DevStatus *st, const Grid &g,
                             const FftAxis &ay, hipStream_t s) {
    if (!fft_yx_fused(g)) return hipErrorInvalidValue;
    const float scale = g.spec_st == kSpecF32 ? 1.0f / ((float)g.n[0] * (float)g.n[1] * (float)g.n[2]) : g.iscale;
    if (g.n[0] == kYh) {
        const dim3 grid(2 * g.n[2]), blk(kYhThreads);
        switch (g.spec_st) {
            case kSpecBF16:
                yx_inv128_kernel<kSpecBF16><<<grid, blk, yx_inv128_lds(), s>>>(spec, A, rowmm, st, g, ay.tw, scale);
                break;
            case kSpecF16:
                yx_inv128_kernel<kSpecF16><<<grid, blk, yx_inv128_lds(), s>>>(spec, A, rowmm, st, g, ay.tw, scale);
                break;
            default:
                yx_inv128_kernel<kSpecF32><<<grid, blk, yx_inv128_lds(), s>>>(spec, A, rowmm, st, g, ay.tw, scale);
        }
        return hipGetLastError();
    }
    switch (g.spec_st) {
        case kSpecBF16:
            yx_inv256_kernel<kSpecBF16><<<dim3(g.n[2]), dim3(kYxThreads), yx_inv256_lds(), s>>>(spec, A, rowmm, st, g,
                                                                                           ay.tw, scale);
            break;
        case kSpecF16:
            yx_inv256_kernel<kSpecF16><<<dim3(g.n[2]), dim3(kYxThreads), yx_inv256_lds(), s>>>(spec, A, rowmm, st, g,
                                                                                          ay.tw, scale);
            break;
        default:
            yx_inv256_kernel<kSpecF32><<<dim3(g.n[2]), dim3(kYxThreads), yx_inv256_lds(), s>>>(spec, A, rowmm, st, g,
                                                                                          ay.tw, scale);
    }
    return hipGetLastError();
}

hipError_t launch_fft_x_c2r(const void *spec, float *A, float2 *rowmm, DevStatus *st, const Grid &g,
                            const FftAxis &ax, hipStream_t s) {
    const int nrows = g.n[1] * g.n[2];
    const float scale = g.spec_st == kSpecF32 ? 1.0f / ((float)g.n[0] * (float)g.n[1] * (float)g.n[2]) : g.iscale;
    if (const int pc = pencil_code(g.n[0])) {
        FVR_PEN_ST(pc, pen_x_c2r_kernel, (spec, A, rowmm, st, g, ax.tw, scale), dim3((nrows + 31) / 32))
        return hipGetLastError();
    }
    const dim3 grid((nrows + kC2rRows - 1) / kC2rRows), blk(kPassThreads);
    const size_t lds = ((size_t)(kC2rRows / 2) * g.n[0] + g.n[0]) * sizeof(float2);
    switch (g.spec_st) {
        case kSpecBF16:
            fft_x_c2r_kernel<kSpecBF16><<<grid, blk, lds, s>>>(spec, A, rowmm, st, g, ax, scale);
            break;
        case kSpecF16:
            fft_x_c2r_kernel<kSpecF16><<<grid, blk, lds, s>>>(spec, A, rowmm, st, g, ax, scale);
            break;
        default:
            fft_x_c2r_kernel<kSpecF32><<<grid, blk, lds, s>>>(spec, A, rowmm, st, g, ax, scale);
    }
    return hipGetLastError();
}

}  // namespace fvr
