/*
 * FP64 CPU oracle for the volumetric Fourier-transform reconstruction
 * (Alexiadis et al., Sec. III-B).  TEST INFRASTRUCTURE ONLY: the tests, the
 * package's smoke check and the benchmark's CPU-baseline leg are its only
 * callers.  The GPU library never links or calls it, and this file shares no
 * code, header or table with the GPU library.
 *
 * Plain loops, slow and literal.  Every accumulation is in double precision;
 * float inputs are promoted.  The one place float32 arithmetic is used on
 * purpose is the choice of each point's 4^3 splat footprint (an integer
 * decided by floating point), which follows the same float32 formula the
 * GPU kernel uses so both sides pick the same voxels.
 *
 * Conventions (Sec. III-B; readings where the paper is silent are marked R):
 *   grid q in [0,Nx) x [0,Ny) x [0,Nz), linear index l = qx + Nx (qy + Ny qz)
 *   R: voxel centre p(q)_a = bmin_a + (q_a + 1/2) h_a,  h_a = (bmax_a - bmin_a) / N_a
 *   R: a point is accepted iff bmin <= X <= bmax componentwise
 *   sigma1 = half the voxel diagonal, sigma2^2 = 3/2 sigma1^2   (text after eq. 2)
 *   g(x; s) = exp(-x^2 / s^2) / s                               (text after eq. 1)
 *   R: footprint = 4 voxel centres per axis nearest the point:
 *      floor(u) - 1 .. floor(u) + 2 with u = (X - bmin)/h - 1/2; voxels off
 *      the grid are dropped
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Float32 footprint origin: u = (x - bmin) / h - 0.5 in float32, h computed
 * as (bmax - bmin) / N in float32.  Returns floor(u). */
static int footprint_origin_f32(float x, float bmin, float bmax, int n)
{
    volatile float h = (bmax - bmin) / (float)n;
    volatile float d = x - bmin;
    volatile float u = d / h;
    volatile float v = u - 0.5f;
    return (int)floorf(v);
}

static int point_accepted(const float *x, const float *bbox)
{
    for (int a = 0; a < 3; ++a)
        if (!(x[a] >= bbox[a] && x[a] <= bbox[a + 3]))
            return 0;
    return 1;
}

/*
 * Weighted Gaussian splat, eqs. (1)-(2).
 *   S_c(q) = sum_i g(|X_i - p(q)|; sigma1) W_i N_ic
 *   D(q)   = sum_i g(|X_i - p(q)|; sigma2) W_i
 *   V_c(q) = S_c(q) / D(q), or 0 where D(q) = 0.
 * Since w_k(u,q) = W_k(u) / d(q) depends on the point only through W, the
 * 1/d(q) factor of eq. (1) comes out of the sum, which gives V = S / D.
 * weights == NULL means every W_i = 1.
 * Outputs are (Nz, Ny, Nx) arrays, x fastest; S and V hold 3 such arrays
 * (component-major).  Returns the number of rejected (outside-bbox) points.
 * nthreads > 1 splits the voxel planes among OpenMP threads without
 * changing any sum (see the loop).
 */
int64_t oracle_splat(const float *points, const float *normals, const float *weights,
                     int64_t m, const int32_t *dims, const float *bbox,
                     double *S, double *D, double *V, int nthreads)
{
    const int Nx = dims[0], Ny = dims[1], Nz = dims[2];
    const int64_t n = (int64_t)Nx * Ny * Nz;
    double h[3];
    for (int a = 0; a < 3; ++a)
        h[a] = ((double)bbox[a + 3] - (double)bbox[a]) / (double)dims[a];
    const double sigma1 = 0.5 * sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    const double sigma2 = sigma1 * sqrt(1.5);

    memset(S, 0, sizeof(double) * 3 * n);
    memset(D, 0, sizeof(double) * n);
    int64_t rejected = 0;
    for (int64_t i = 0; i < m; ++i)
        if (!point_accepted(points + 3 * i, bbox)) ++rejected;

    /* With several threads, thread t owns the voxel planes z in
     * [z0(t), z1(t)) and visits every point in input order, adding only to
     * its own planes: each voxel still receives its terms in input order, so
     * the sums are those of the single-threaded loop, bit for bit. */
    if (nthreads < 1) nthreads = 1;
    if (nthreads > Nz) nthreads = Nz;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
    for (int t = 0; t < nthreads; ++t) {
        const int z0 = (int)((int64_t)Nz * t / nthreads), z1 = (int)((int64_t)Nz * (t + 1) / nthreads);
        for (int64_t i = 0; i < m; ++i) {
            const float *X = points + 3 * i;
            if (!point_accepted(X, bbox)) continue;
            const double W = weights ? (double)weights[i] : 1.0;
            int i0[3];
            for (int a = 0; a < 3; ++a)
                i0[a] = footprint_origin_f32(X[a], bbox[a], bbox[a + 3], dims[a]);
            if (i0[2] + 2 < z0 || i0[2] - 1 >= z1) continue;
            for (int oz = -1; oz <= 2; ++oz) {
                const int qz = i0[2] + oz;
                if (qz < 0 || qz >= Nz || qz < z0 || qz >= z1) continue;
                for (int oy = -1; oy <= 2; ++oy) {
                    const int qy = i0[1] + oy;
                    if (qy < 0 || qy >= Ny) continue;
                    for (int ox = -1; ox <= 2; ++ox) {
                        const int qx = i0[0] + ox;
                        if (qx < 0 || qx >= Nx) continue;
                        const double px = (double)bbox[0] + (qx + 0.5) * h[0];
                        const double py = (double)bbox[1] + (qy + 0.5) * h[1];
                        const double pz = (double)bbox[2] + (qz + 0.5) * h[2];
                        const double dx = (double)X[0] - px;
                        const double dy = (double)X[1] - py;
                        const double dz = (double)X[2] - pz;
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        const double g1 = exp(-r2 / (sigma1 * sigma1)) / sigma1;
                        const double g2 = exp(-r2 / (sigma2 * sigma2)) / sigma2;
                        const int64_t l = qx + (int64_t)Nx * (qy + (int64_t)Ny * qz);
                        for (int c = 0; c < 3; ++c)
                            S[c * n + l] += g1 * W * (double)normals[3 * i + c];
                        D[l] += g2 * W;
                    }
                }
            }
        }
    }
    for (int64_t l = 0; l < n; ++l)
        for (int c = 0; c < 3; ++c)
            V[c * n + l] = D[l] > 0.0 ? S[c * n + l] / D[l] : 0.0;
    return rejected;
}

/* Nearest voxel centre of x: the grid cell containing the point,
 * floor((x - bmin) / h) in float32 (h = (bmax - bmin) / N in float32), clamped
 * to the grid - the same float32 formula as the GPU kernel, since floating
 * point decides an integer here. */
static int nearest_voxel_f32(float x, float bmin, float bmax, int n)
{
    volatile float h = (bmax - bmin) / (float)n;
    volatile float d = x - bmin;
    volatile float u = d / h;
    int i = (int)floorf(u);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    return i;
}

/*
 * Non-weighted splat, the simplest version of Sec. III-B: each accepted
 * sample is assigned ("clamped") to its nearest voxel, and the vector field
 * is the sum of the normals assigned to a voxel divided by their number;
 * V = 0 where no sample lands.  Weights play no part.  S holds the sums
 * (3 arrays), cnt the counts; returns the number of rejected points.
 */
int64_t oracle_splat_nearest(const float *points, const float *normals, int64_t m,
                             const int32_t *dims, const float *bbox, double *S, int64_t *cnt,
                             double *V)
{
    const int Nx = dims[0], Ny = dims[1], Nz = dims[2];
    const int64_t n = (int64_t)Nx * Ny * Nz;
    memset(S, 0, sizeof(double) * 3 * n);
    memset(cnt, 0, sizeof(int64_t) * n);
    int64_t rejected = 0;
    for (int64_t i = 0; i < m; ++i) {
        const float *X = points + 3 * i;
        if (!point_accepted(X, bbox)) { ++rejected; continue; }
        const int qx = nearest_voxel_f32(X[0], bbox[0], bbox[3], Nx);
        const int qy = nearest_voxel_f32(X[1], bbox[1], bbox[4], Ny);
        const int qz = nearest_voxel_f32(X[2], bbox[2], bbox[5], Nz);
        const int64_t l = qx + (int64_t)Nx * (qy + (int64_t)Ny * qz);
        for (int c = 0; c < 3; ++c) S[c * n + l] += (double)normals[3 * i + c];
        cnt[l] += 1;
    }
    for (int64_t l = 0; l < n; ++l)
        for (int c = 0; c < 3; ++c)
            V[c * n + l] = cnt[l] > 0 ? S[c * n + l] / (double)cnt[l] : 0.0;
    return rejected;
}

/*
 * Iso-level L: mean of A at the input sample locations (text before the
 * CUDA remark closing Sec. III-B).  R: A is sampled by trilinear
 * interpolation between voxel centres, the cell clamped to the grid and the
 * local coordinates clamped to [0,1]; only accepted points count; the mean
 * is unweighted; the sum is compensated (Neumaier).
 * Returns L and writes the number of points used.  No points gives L = 0.
 */
double oracle_level(const double *A, const int32_t *dims, const float *bbox,
                    const float *points, int64_t m, int64_t *n_used)
{
    const int N[3] = {dims[0], dims[1], dims[2]};
    double h[3];
    for (int a = 0; a < 3; ++a)
        h[a] = ((double)bbox[a + 3] - (double)bbox[a]) / (double)dims[a];
    double sum = 0.0, comp = 0.0;
    int64_t used = 0;
    for (int64_t i = 0; i < m; ++i) {
        const float *X = points + 3 * i;
        if (!point_accepted(X, bbox)) continue;
        int b[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            const double u = ((double)X[a] - (double)bbox[a]) / h[a] - 0.5;
            int bb = (int)floor(u);
            if (bb < 0) bb = 0;
            if (bb > N[a] - 2) bb = N[a] - 2;
            double tt = u - bb;
            if (tt < 0.0) tt = 0.0;
            if (tt > 1.0) tt = 1.0;
            b[a] = bb;
            t[a] = tt;
        }
        double val = 0.0;
        for (int k = 0; k < 8; ++k) {
            const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
            const double wgt = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) *
                               (oz ? t[2] : 1.0 - t[2]);
            const int64_t l = (b[0] + ox) + (int64_t)N[0] * ((b[1] + oy) + (int64_t)N[1] * (b[2] + oz));
            val += wgt * A[l];
        }
        /* Neumaier summation */
        const double s = sum + val;
        if (fabs(sum) >= fabs(val)) comp += (sum - s) + val;
        else comp += (val - s) + sum;
        sum = s;
        ++used;
    }
    *n_used = used;
    return used ? (sum + comp) / (double)used : 0.0;
}

/*
 * Marching cubes (the extraction step closing Sec. III-B) with a welded,
 * indexed output.
 *   cell c: 0 <= c_a <= N_a - 2; corner k at offset (k&1, (k>>1)&1, (k>>2)&1)
 *   inside(q) <=> A(q) > level;  case(c) = sum_k inside(c + off_k) 2^k
 *   cube edge id = 4 axis + b_lo + 2 b_hi (b_lo, b_hi: the offset bits of the
 *   two other axes, in x<y<z order); the edge starts at its low corner.
 *   Each grid edge (q, q + e_a) whose ends differ in inside() carries one
 *   vertex p(q) + t h_a e_a, t = (level - A(q)) / (A(q + e_a) - A(q)).
 *   Vertices are numbered in (l(q), a) order; triangles in (l(c), table) order.
 * tri_count[256] and tri_edges[256 * 15] come from the oracle's own table
 * generator (the rule is documented there).
 * Output sizes are checked against the capacities; the required counts are
 * always written.  Returns 0, or -1 if a capacity is too small.  nthreads > 1
 * spreads the z planes over OpenMP threads; the output is the same.
 * normals (optional, V x 3): the unit vertex normals -grad A described at
 * mc_plane_vertices (Sec. III-B lists normals among the mesh outputs).
 */
/* dA/dx_b at grid point q by central differences, one-sided on the grid's
 * outer layer (reading of the normals the extraction outputs). */
static double grad_axis(const double *A, const int32_t *dims, const double *h, const int q[3], int b)
{
    const int64_t stride[3] = {1, dims[0], (int64_t)dims[0] * dims[1]};
    const int64_t l = q[0] + stride[1] * q[1] + stride[2] * q[2];
    const int lo = q[b] == 0, hi = q[b] == dims[b] - 1;
    const double ap = hi ? A[l] : A[l + stride[b]];
    const double am = lo ? A[l] : A[l - stride[b]];
    return (ap - am) / ((lo || hi ? 1.0 : 2.0) * h[b]);
}

/* Vertices whose grid point lies in plane qz, in (l, axis) order; writes
 * ids from `first` (and positions, if they fit) when vid is not NULL.
 * Normals (optional): -grad A, the gradients at the edge's two grid points
 * interpolated linearly with t, normalised (zero where that is zero). */
static int64_t mc_plane_vertices(const double *A, const int32_t *dims, const float *bbox,
                                 const double *h, double level, int qz, int64_t first,
                                 int32_t *vid, double *verts, int64_t vert_cap, double *normals)
{
    const int Nx = dims[0], Ny = dims[1];
    int64_t nv = first;
    for (int qy = 0; qy < Ny; ++qy)
        for (int qx = 0; qx < Nx; ++qx) {
            const int64_t l = qx + (int64_t)Nx * (qy + (int64_t)Ny * qz);
            const int q[3] = {qx, qy, qz};
            const int64_t stride[3] = {1, Nx, (int64_t)Nx * Ny};
            for (int a = 0; a < 3; ++a) {
                if (vid) vid[3 * l + a] = -1;
                if (q[a] + 1 >= dims[a]) continue;
                const double a0 = A[l], a1 = A[l + stride[a]];
                if ((a0 > level) == (a1 > level)) continue;
                if (vid) {
                    if (nv < vert_cap) {
                        const double t = (level - a0) / (a1 - a0);
                        for (int b = 0; b < 3; ++b) {
                            double p = (double)bbox[b] + (q[b] + 0.5) * h[b];
                            if (b == a) p += t * h[a];
                            verts[3 * nv + b] = p;
                        }
                        if (normals) {
                            int q1[3] = {qx, qy, qz};
                            q1[a] += 1;
                            double g[3], len2 = 0.0;
                            for (int b = 0; b < 3; ++b) {
                                const double g0 = grad_axis(A, dims, h, q, b);
                                const double g1 = grad_axis(A, dims, h, q1, b);
                                g[b] = -((1.0 - t) * g0 + t * g1);
                                len2 += g[b] * g[b];
                            }
                            const double len = sqrt(len2);
                            for (int b = 0; b < 3; ++b) normals[3 * nv + b] = len > 0.0 ? g[b] / len : 0.0;
                        }
                    }
                    vid[3 * l + a] = (int32_t)nv;
                }
                ++nv;
            }
        }
    return nv - first;
}

/* Triangles of the cells in plane cz, in (l(c), table) order.  With fill,
 * writes the case bytes (if cases is not NULL) and the triangles from
 * `first` (if they fit); otherwise only counts. */
static int64_t mc_plane_triangles(const double *A, const int32_t *dims, double level, int cz,
                                  const uint8_t *tri_count, const int8_t *tri_edges,
                                  const int32_t *vid, int fill, int64_t first, int32_t *tris,
                                  int64_t tri_cap, uint8_t *cases)
{
    const int Nx = dims[0], Ny = dims[1];
    int64_t nt = first;
    for (int cy = 0; cy < Ny - 1; ++cy)
        for (int cx = 0; cx < Nx - 1; ++cx) {
            int cs = 0;
            for (int k = 0; k < 8; ++k) {
                const int64_t l = (cx + (k & 1)) + (int64_t)Nx * ((cy + ((k >> 1) & 1)) +
                                                                (int64_t)Ny * (cz + ((k >> 2) & 1)));
                if (A[l] > level) cs |= 1 << k;
            }
            if (!fill) {
                nt += tri_count[cs];
                continue;
            }
            if (cases)
                cases[cx + (int64_t)(Nx - 1) * (cy + (int64_t)(Ny - 1) * cz)] = (uint8_t)cs;
            for (int t = 0; t < tri_count[cs]; ++t) {
                for (int j = 0; j < 3; ++j) {
                    const int e = tri_edges[cs * 15 + 3 * t + j];
                    const int axis = e / 4, r = e % 4;
                    int off[3] = {0, 0, 0};
                    int o = 0;
                    for (int b = 0; b < 3; ++b) {
                        if (b == axis) continue;
                        off[b] = o == 0 ? (r & 1) : ((r >> 1) & 1);
                        ++o;
                    }
                    const int64_t l = (cx + off[0]) + (int64_t)Nx * ((cy + off[1]) +
                                                                   (int64_t)Ny * (cz + off[2]));
                    if (tris && nt < tri_cap) tris[3 * nt + j] = vid[3 * l + axis];
                }
                ++nt;
            }
        }
    return nt - first;
}

int oracle_marching_cubes(const double *A, const int32_t *dims, const float *bbox,
                          double level, const uint8_t *tri_count, const int8_t *tri_edges,
                          double *verts, int64_t vert_cap, int32_t *tris, int64_t tri_cap,
                          uint8_t *cases, int64_t *n_verts, int64_t *n_tris, int nthreads,
                          double *normals)
{
    const int Nx = dims[0], Ny = dims[1], Nz = dims[2];
    const int64_t n = (int64_t)Nx * Ny * Nz;
    double h[3];
    for (int a = 0; a < 3; ++a)
        h[a] = ((double)bbox[a + 3] - (double)bbox[a]) / (double)dims[a];
    int32_t *vid = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n);
    int64_t *vfirst = (int64_t *)malloc(sizeof(int64_t) * ((size_t)Nz + 1));
    int64_t *tfirst = (int64_t *)malloc(sizeof(int64_t) * ((size_t)Nz + 1));
    if (!vid || !vfirst || !tfirst) {
        free(vid);
        free(vfirst);
        free(tfirst);
        return -2;
    }
    if (nthreads < 1) nthreads = 1;

    /* Vertices on active grid edges, in (l, axis) order: each z plane is
     * counted, the counts are prefix-summed in plane order, and each plane
     * numbers its vertices from its offset - the numbering of one loop over
     * l, whatever the number of threads. */
    vfirst[0] = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int qz = 0; qz < Nz; ++qz)
        vfirst[qz + 1] = mc_plane_vertices(A, dims, bbox, h, level, qz, 0, NULL, NULL, 0, NULL);
    for (int qz = 0; qz < Nz; ++qz) vfirst[qz + 1] += vfirst[qz];
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int qz = 0; qz < Nz; ++qz)
        mc_plane_vertices(A, dims, bbox, h, level, qz, vfirst[qz], vid, verts, vert_cap, normals);

    /* Triangles, cell by cell in (l(c), table) order, the same way per plane
     * of cells. */
    tfirst[0] = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int cz = 0; cz < Nz - 1; ++cz)
        tfirst[cz + 1] = mc_plane_triangles(A, dims, level, cz, tri_count, tri_edges, vid, 0, 0, NULL,
                                            0, NULL);
    for (int cz = 0; cz < Nz - 1; ++cz) tfirst[cz + 1] += tfirst[cz];
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int cz = 0; cz < Nz - 1; ++cz)
        mc_plane_triangles(A, dims, level, cz, tri_count, tri_edges, vid, 1, tfirst[cz], tris, tri_cap,
                           cases);
    const int64_t nv = vfirst[Nz], nt = tfirst[Nz - 1];
    free(vid);
    free(vfirst);
    free(tfirst);
    *n_verts = nv;
    *n_tris = nt;
    return (nv > vert_cap || nt > tri_cap) ? -1 : 0;
}
