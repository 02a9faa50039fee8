// Front end of the path (Sec. III-A) for gfx950: K depth maps to the raw
// oriented, confidence-weighted points X_k(u), N_k(u), W_k(u) the splat
// consumes, so that a frame crosses the host link as depth maps (about
// 0.9 MB per view) instead of 28-byte points.
//
// Per foreground pixel u (depth D > 0 and finite) of view k:
//   X^loc = ((u_x - c_x) D / f_x, (u_y - c_y) D / f_y, D)   (inverse projection)
//   N^loc = mean of the unit normals of the kept triangles that have u as a
//           vertex.  The organized triangulation splits each 2 x 2 pixel quad
//           along the diagonal whose ends differ less in depth (the (0,0)-(1,1)
//           diagonal on a tie) and keeps a triangle when its three pixels are
//           foreground and no two of its depths differ by more than tau (the
//           step-discontinuity constraint).  A triangle's normal is taken with
//           the winding that faces the camera: its pixels project to a
//           triangle of fixed image orientation, so (p2 - p0) x (p1 - p0) in
//           the vertex order below always points towards the camera.
//   W1 = max(<-X^loc / |X^loc|, N^loc>, 0)
//   W2 = foreground pixels in the (2r+1)^2 square around u (pixels outside
//        the image count as background) / (2r+1)^2
//   W = W1 W2; X = R X^loc + t, N = R N^loc in world coordinates.
// Pixels with no kept triangle give no point.  Points come out view by view
// in raster order (compaction by an exclusive scan of per-pixel flags).
#include "fvr_common.h"

namespace fvr {

namespace {

constexpr int kFeThreads = 256;

__device__ __forceinline__ bool foreground(float d) { return d > 0.0f && d <= 3.0e38f; }

// foreground pixels of row `row` in columns u - r .. u + r
__global__ void __launch_bounds__(kFeThreads)
fe_rowcount_kernel(const float *__restrict__ depth, int n, int width, int r, int32_t *__restrict__ rowcnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int u = i % width;
    const float *d = depth + (size_t)(i - u);
    int c = 0;
    for (int x = max(u - r, 0); x <= min(u + r, width - 1); ++x) c += foreground(d[x]) ? 1 : 0;
    rowcnt[i] = c;
}

struct P3 {
    float x, y, z;
};

__device__ __forceinline__ P3 sub3(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ P3 cross3(P3 a, P3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__global__ void __launch_bounds__(kFeThreads)
fe_pixel_kernel(const float *__restrict__ depth, const int32_t *__restrict__ rowcnt, FeParams fp, FeCams cams,
                float *__restrict__ dense, int32_t *__restrict__ flag) {
    const int H = fp.height, W = fp.width;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= fp.views * H * W) return;
    const int k = i / (H * W), rem = i - k * H * W;
    const int v = rem / W, u = rem - v * W;
    const float *Dk = depth + (size_t)k * H * W;
    flag[i] = 0;
    if (!foreground(Dk[rem])) return;
    const float *c = cams.c[k];
    const float fx = c[0], fy = c[1], cx = c[2], cy = c[3];
    // 3 x 3 neighbourhood (background outside the image)
    float nd[3][3];
    P3 np[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int x = u + dx - 1, y = v + dy - 1;
            const float d = (x >= 0 && x < W && y >= 0 && y < H) ? Dk[y * W + x] : 0.0f;
            nd[dy][dx] = foreground(d) ? d : 0.0f;
            np[dy][dx] = {((float)x - cx) * d / fx, ((float)y - cy) * d / fy, d};
        }
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    int cnt = 0;
    auto tri = [&](int ay, int ax, int by, int bx, int cy_, int cx_) {
        // the pixel (1, 1) must be one of the three corners
        if (!((ay == 1 && ax == 1) || (by == 1 && bx == 1) || (cy_ == 1 && cx_ == 1))) return;
        const float d0 = nd[ay][ax], d1 = nd[by][bx], d2 = nd[cy_][cx_];
        if (d0 == 0.0f || d1 == 0.0f || d2 == 0.0f) return;
        if (fabsf(d0 - d1) > fp.tau || fabsf(d0 - d2) > fp.tau || fabsf(d1 - d2) > fp.tau) return;
        const P3 p0 = np[ay][ax], p1 = np[by][bx], p2 = np[cy_][cx_];
        const P3 n = cross3(sub3(p2, p0), sub3(p1, p0));
        const float len = sqrtf(n.x * n.x + n.y * n.y + n.z * n.z);
        if (!(len > 0.0f)) return;
        sx += n.x / len;
        sy += n.y / len;
        sz += n.z / len;
        ++cnt;
    };
    // the four quads around the pixel: top-left corner (qy, qx) in the 3 x 3 window
#pragma unroll
    for (int qy = 0; qy < 2; ++qy)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx) {
            // corners a = (qy, qx), b = (qy, qx+1), c = (qy+1, qx), d = (qy+1, qx+1)
            const float da = nd[qy][qx], db = nd[qy][qx + 1], dc = nd[qy + 1][qx], dd = nd[qy + 1][qx + 1];
            if (fabsf(da - dd) <= fabsf(db - dc)) {
                tri(qy, qx, qy, qx + 1, qy + 1, qx + 1);      // (a, b, d)
                tri(qy, qx, qy + 1, qx + 1, qy + 1, qx);      // (a, d, c)
            } else {
                tri(qy, qx, qy, qx + 1, qy + 1, qx);          // (a, b, c)
                tri(qy, qx + 1, qy + 1, qx + 1, qy + 1, qx);  // (b, d, c)
            }
        }
    if (cnt == 0) return;
    const float inv = 1.0f / (float)cnt;
    const P3 N = {sx * inv, sy * inv, sz * inv};
    const P3 X = np[1][1];
    const float xl = sqrtf(X.x * X.x + X.y * X.y + X.z * X.z);
    const float w1 = fmaxf(-(X.x * N.x + X.y * N.y + X.z * N.z) / xl, 0.0f);
    int box = 0;
    for (int y = max(v - fp.radius, 0); y <= min(v + fp.radius, H - 1); ++y)
        box += rowcnt[(size_t)k * H * W + (size_t)y * W + u];
    const float side = (float)(2 * fp.radius + 1);
    const float w2 = (float)box / (side * side);
    const float *R = c + 4, *t = c + 13;
    float *o = dense + 7 * (size_t)i;
    o[0] = R[0] * X.x + R[1] * X.y + R[2] * X.z + t[0];
    o[1] = R[3] * X.x + R[4] * X.y + R[5] * X.z + t[1];
    o[2] = R[6] * X.x + R[7] * X.y + R[8] * X.z + t[2];
    o[3] = R[0] * N.x + R[1] * N.y + R[2] * N.z;
    o[4] = R[3] * N.x + R[4] * N.y + R[5] * N.z;
    o[5] = R[6] * N.x + R[7] * N.y + R[8] * N.z;
    o[6] = w1 * w2;
    flag[i] = 1;
}

// Flagged pixels to the point arrays at their scan offsets; nothing is
// written when the total exceeds the capacity.
__global__ void __launch_bounds__(kFeThreads)
fe_scatter_kernel(const float *__restrict__ dense, const int32_t *__restrict__ flag,
                  const int32_t *__restrict__ off, int n, const DevStatus *__restrict__ st, long long cap,
                  float *__restrict__ pts, float *__restrict__ nrm, float *__restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i] || (long long)st->fe_points > cap) return;
    const size_t j = (size_t)off[i];
    const float *o = dense + 7 * (size_t)i;
    pts[3 * j] = o[0];
    pts[3 * j + 1] = o[1];
    pts[3 * j + 2] = o[2];
    nrm[3 * j] = o[3];
    nrm[3 * j + 1] = o[4];
    nrm[3 * j + 2] = o[5];
    w[j] = o[6];
}

}  // namespace

hipError_t launch_fe_pixels(const float *depth, const FeParams &fp, const FeCams &cams, int32_t *rowcnt,
                            float *dense, int32_t *flag, hipStream_t s) {
    const int n = fp.views * fp.height * fp.width;
    const int blocks = (n + kFeThreads - 1) / kFeThreads;
    fe_rowcount_kernel<<<dim3(blocks), dim3(kFeThreads), 0, s>>>(depth, n, fp.width, fp.radius, rowcnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    fe_pixel_kernel<<<dim3(blocks), dim3(kFeThreads), 0, s>>>(depth, rowcnt, fp, cams, dense, flag);
    return hipGetLastError();
}

hipError_t launch_fe_scatter(const float *dense, const int32_t *flag, const int32_t *off, int n,
                             const DevStatus *st, long long cap, float *pts, float *nrm, float *w,
                             hipStream_t s) {
    const int blocks = (n + kFeThreads - 1) / kFeThreads;
    fe_scatter_kernel<<<dim3(blocks), dim3(kFeThreads), 0, s>>>(dense, flag, off, n, st, cap, pts, nrm, w);
    return hipGetLastError();
}

}  // namespace fvr
