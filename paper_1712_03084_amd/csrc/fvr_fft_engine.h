// In-LDS batched complex FFT for gfx950 (device code).
//
// A block transforms `nrows` independent complex rows of length n held in
// LDS, in place, with a mixed-radix Stockham schedule (radix 2, 3, 4, 5, 8).
// Each stage: every thread loads its butterflies' R inputs into registers,
// applies the twiddles and an R-point DFT, the block synchronises, then every
// thread stores its R outputs to their auto-sorted positions.  Holding all
// butterflies of a stage in registers makes the in-place update safe; the
// caller guarantees nrows * n <= blockDim.x * EPT (kFftEpt by default).
//
// Stage with radix R, running product ns of earlier radices, nb = n / R:
//   butterfly j of a row reads  x[j + r nb], r < R
//   twiddles     x_r *= exp(dir 2 pi i r k / (ns R)),  k = j mod ns
//   R-point DFT with root exp(dir 2 pi i / R)
//   writes       y[(j - k) R + k + r ns]
// dir = -1 is the forward transform, +1 the unnormalised inverse.
#pragma once

#include <hip/hip_runtime.h>

#include "fvr_common.h"

namespace fvr {

constexpr int kFftEpt = 32;  // complex elements per thread per stage, at most

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// (dir * i) * a
__device__ __forceinline__ float2 mul_i(float2 a, int dir) {
    return dir < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <int R> struct Dft;

template <> struct Dft<2> {
    __device__ __forceinline__ static void run(float2 *a, int) {
        const float2 t = a[1];
        a[1] = csub(a[0], t);
        a[0] = cadd(a[0], t);
    }
};

template <> struct Dft<3> {
    __device__ __forceinline__ static void run(float2 *a, int dir) {
        const float c = 0.5f, s = 0.86602540378443865f;  // cos(pi/3), sin(pi/3)
        const float2 sum = cadd(a[1], a[2]);
        const float2 t = csub(a[0], cscale(sum, c));
        const float2 d = cscale(mul_i(csub(a[1], a[2]), dir), s);
        a[0] = cadd(a[0], sum);
        a[1] = cadd(t, d);
        a[2] = csub(t, d);
    }
};

template <> struct Dft<4> {
    __device__ __forceinline__ static void run(float2 *a, int dir) {
        const float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        const float2 t2 = cadd(a[1], a[3]), t3 = mul_i(csub(a[1], a[3]), dir);
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    }
};

template <> struct Dft<5> {
    __device__ __forceinline__ static void run(float2 *a, int dir) {
        // cos and sin of 2 pi / 5 and 4 pi / 5
        const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
        const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
        const float2 b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
        const float2 d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
        const float2 t1 = cadd(a[0], cadd(cscale(b1, c1), cscale(b2, c2)));
        const float2 t2 = cadd(a[0], cadd(cscale(b1, c2), cscale(b2, c1)));
        const float2 u1 = mul_i(cadd(cscale(d1, s1), cscale(d2, s2)), dir);
        const float2 u2 = mul_i(csub(cscale(d1, s2), cscale(d2, s1)), dir);
        a[0] = cadd(a[0], cadd(b1, b2));
        a[1] = cadd(t1, u1);
        a[4] = csub(t1, u1);
        a[2] = cadd(t2, u2);
        a[3] = csub(t2, u2);
    }
};

template <> struct Dft<8> {
    __device__ __forceinline__ static void run(float2 *a, int dir) {
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4>::run(e, dir);
        Dft<4>::run(o, dir);
        const float r = 0.70710678118654752f;  // sqrt(1/2)
        // o[k] *= exp(dir 2 pi i k / 8)
        o[1] = cscale(cadd(o[1], mul_i(o[1], dir)), r);
        o[2] = mul_i(o[2], dir);
        o[3] = cscale(csub(mul_i(o[3], dir), o[3]), r);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = cadd(e[k], o[k]);
            a[k + 4] = csub(e[k], o[k]);
        }
    }
};

template <> struct Dft<16> {
    // 16 = 4 x 4: DFT over n1 of x[4 n1 + n2], twiddle w16^(n2 k1), DFT over n2;
    // output k1 + 4 k2 in natural order
    __device__ __forceinline__ static void run(float2 *a, int dir) {
        const float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f;  // cos, sin of pi/8
        const float r = 0.70710678118654752f;
        float2 y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            float2 b[4] = {a[n2], a[4 + n2], a[8 + n2], a[12 + n2]};
            Dft<4>::run(b, dir);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = b[k1];
        }
        // w16^m = (cos(2 pi m / 16), dir sin(2 pi m / 16)) for m = n2 k1 in {1, 2, 3, 4, 6, 9}
        y[1][1] = cmul(y[1][1], make_float2(c1, dir * s1));
        y[1][2] = cmul(y[1][2], make_float2(r, dir * r));
        y[1][3] = cmul(y[1][3], make_float2(s1, dir * c1));
        y[2][1] = cmul(y[2][1], make_float2(r, dir * r));
        y[2][2] = mul_i(y[2][2], dir);
        y[2][3] = cmul(y[2][3], make_float2(-r, dir * r));
        y[3][1] = cmul(y[3][1], make_float2(s1, dir * c1));
        y[3][2] = cmul(y[3][2], make_float2(-r, dir * r));
        y[3][3] = cmul(y[3][3], make_float2(-c1, -dir * s1));
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 b[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            Dft<4>::run(b, dir);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = b[k2];
        }
    }
};

// floor(x / d) for x < 2^16, d < 2^16 via a multiply-high: m = ceil(2^32 / d).
__device__ __forceinline__ unsigned div_magic(unsigned d) { return d == 1 ? 0u : 0xFFFFFFFFu / d + 1u; }
__device__ __forceinline__ int udiv(int x, int d, unsigned m) {
    return d == 1 ? x : (int)__umulhi((unsigned)x, m);
}

// LDS row accessors.
// Interleaved complex: element (r, e) at p[r * rs + e * es] (float2 units).
struct RowsC {
    float2 *p;
    int rs, es;
    __device__ __forceinline__ float2 ld(int r, int e) const { return p[r * rs + e * es]; }
    __device__ __forceinline__ void st(int r, int e, float2 v) const { p[r * rs + e * es] = v; }
};
// Split complex: real part at p[r * rs + e], imaginary part `im` floats later.
struct RowsS {
    float *p;
    int rs, im;
    __device__ __forceinline__ float2 ld(int r, int e) const {
        return make_float2(p[r * rs + e], p[r * rs + e + im]);
    }
    __device__ __forceinline__ void st(int r, int e, float2 v) const {
        p[r * rs + e] = v.x;
        p[r * rs + e + im] = v.y;
    }
};

// ROW_FASTEST: consecutive threads take consecutive rows (rows interleaved in
// LDS, e.g. columns of a y or z pencil tile); otherwise consecutive threads
// take consecutive butterflies of one row (rows contiguous in LDS).  EPT bounds
// the elements per thread (nrows * n <= blockDim.x * EPT); the registers held
// per thread scale with it.
template <int R, bool ROW_FASTEST, int EPT, class Acc>
__device__ __forceinline__ void fft_stage(const Acc &acc, int nrows, int n, int ns,
                                          const float2 *__restrict__ tw, int dir) {
    constexpr int MAXB = (EPT + R - 1) / R;
    const int nb = n / R;
    const int total = nrows * nb;
    const int stride = n / (ns * R);
    const unsigned m_nb = div_magic(nb), m_ns = div_magic(ns), m_rows = div_magic(nrows);
    const int T = blockDim.x;
    float2 v[MAXB][R];
    int rowv[MAXB], basev[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * T;
        rowv[i] = -1;
        if (b < total) {
            int row, j;
            if (ROW_FASTEST) {
                j = udiv(b, nrows, m_rows);
                row = b - j * nrows;
            } else {
                row = udiv(b, nb, m_nb);
                j = b - row * nb;
            }
            const int k = j - udiv(j, ns, m_ns) * ns;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = acc.ld(row, j + r * nb);
            if (k != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[r * k * stride];
                    if (dir > 0) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            Dft<R>::run(v[i], dir);
            rowv[i] = row;
            basev[i] = (j - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        if (rowv[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) acc.st(rowv[i], basev[i] + r * ns, v[i][r]);
        }
    }
    __syncthreads();
}

// Transform all rows.  The caller has synchronised after filling the rows
// (and `tw`, normally an LDS copy of ax.tw); the rows are synchronised again
// on return.
// Inlined into the kernel, so that the axis description (a kernel argument)
// is never addressed through memory.
template <bool ROW_FASTEST, int EPT = kFftEpt, class Acc>
__device__ __forceinline__ void fft_rows(const Acc &acc, int nrows, const FftAxis &ax, const float2 *tw,
                                         int dir) {
    int ns = 1;
    for (int s = 0; s < ax.nstages; ++s) {
        const int R = (ax.radices >> (4 * s)) & 15u;
        switch (R) {
            case 8: fft_stage<8, ROW_FASTEST, EPT>(acc, nrows, ax.n, ns, tw, dir); break;
            case 4: fft_stage<4, ROW_FASTEST, EPT>(acc, nrows, ax.n, ns, tw, dir); break;
            case 2: fft_stage<2, ROW_FASTEST, EPT>(acc, nrows, ax.n, ns, tw, dir); break;
            case 3: fft_stage<3, ROW_FASTEST, EPT>(acc, nrows, ax.n, ns, tw, dir); break;
            default: fft_stage<5, ROW_FASTEST, EPT>(acc, nrows, ax.n, ns, tw, dir); break;
        }
        ns *= R;
    }
}

// Copy an axis's twiddle table (n <= 512 entries) into LDS; the caller
// synchronises before use.
__device__ __forceinline__ void load_twiddles(float2 *dst, const FftAxis &ax) {
    for (int i = threadIdx.x; i < ax.n; i += blockDim.x) dst[i] = ax.tw[i];
}

// Signed wavenumber of DFT bin k of length n (the Nyquist bin n/2 maps to -n/2).
__device__ __forceinline__ int kappa(int k, int n) { return k < n / 2 ? k : k - n; }
// Derivative factor w_a: zero on the Nyquist bin.
__device__ __forceinline__ float deriv_w(int k, int n, float wstep) {
    return (2 * k == n) ? 0.0f : (float)kappa(k, n) * wstep;
}

}  // namespace fvr
