/* Drives the oracle's C functions on a small ragged grid under AddressSanitizer
 * and UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py).  Points
 * include some outside the bbox and a zero weight; marching cubes runs once
 * with too small a capacity and once in full.  argv[1] names a binary file
 * with the marching-cubes table (256 counts, then 256 x 15 edge ids).
 * Prints "ok" and returns 0 when every result passes its checks. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_splat(const float *points, const float *normals, const float *weights, int64_t m,
                     const int32_t *dims, const float *bbox, double *S, double *D, double *V, int nthreads);
int64_t oracle_splat_nearest(const float *points, const float *normals, int64_t m, const int32_t *dims,
                             const float *bbox, double *S, int64_t *cnt, double *V);
double oracle_level(const double *A, const int32_t *dims, const float *bbox, const float *points, int64_t m,
                    int64_t *n_used);
int oracle_marching_cubes(const double *A, const int32_t *dims, const float *bbox, double level,
                          const uint8_t *tri_count, const int8_t *tri_edges, double *verts, int64_t vert_cap,
                          int32_t *tris, int64_t tri_cap, uint8_t *cases, int64_t *n_verts, int64_t *n_tris,
                          int nthreads, double *normals);

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static double uniform(void) {  /* xorshift64*, in [0, 1) */
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return (double)((rng * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

#define FAIL(...) do { fprintf(stderr, __VA_ARGS__); fputc('\n', stderr); return 1; } while (0)

int main(int argc, char **argv) {
    if (argc < 2) FAIL("usage: oracle_driver TABLE");
    uint8_t counts[256];
    int8_t edges[256 * 15];
    FILE *f = fopen(argv[1], "rb");
    if (!f || fread(counts, 1, 256, f) != 256 || fread(edges, 1, sizeof edges, f) != sizeof edges)
        FAIL("cannot read the table");
    fclose(f);

    const int32_t dims[3] = {12, 10, 8};
    const float bbox[6] = {-1.2f, -1.0f, -0.8f, 1.2f, 1.0f, 0.8f};
    const int64_t m = 400, n = (int64_t)dims[0] * dims[1] * dims[2];
    float *p = malloc(sizeof(float) * 3 * m), *nr = malloc(sizeof(float) * 3 * m), *w = malloc(sizeof(float) * m);
    for (int64_t i = 0; i < m; ++i) {
        /* a sphere of radius 0.6 with outward normals; every 37th point outside the box */
        double d[3], s = 0;
        for (int a = 0; a < 3; ++a) { d[a] = 2 * uniform() - 1; s += d[a] * d[a]; }
        s = sqrt(s) + 1e-12;
        for (int a = 0; a < 3; ++a) {
            p[3 * i + a] = (float)(0.6 * d[a] / s);
            nr[3 * i + a] = (float)(d[a] / s);
        }
        if (i % 37 == 0) p[3 * i] = 2.0f;
        w[i] = i % 53 == 0 ? 0.0f : (float)(0.05 + uniform());
    }
    double *S = malloc(sizeof(double) * 3 * n), *D = malloc(sizeof(double) * n), *V = malloc(sizeof(double) * 3 * n);
    double *V2 = malloc(sizeof(double) * 3 * n);
    const int64_t rej = oracle_splat(p, nr, w, m, dims, bbox, S, D, V, 1);
    const int64_t rej2 = oracle_splat(p, nr, w, m, dims, bbox, S, D, V2, 2);
    if (rej != 11 || rej2 != rej) FAIL("rejected %lld / %lld, expected 11", (long long)rej, (long long)rej2);
    if (memcmp(V, V2, sizeof(double) * 3 * n)) FAIL("splat differs between 1 and 2 threads");
    double vmax = 0;
    for (int64_t i = 0; i < 3 * n; ++i) {
        if (!isfinite(V[i])) FAIL("non-finite V");
        vmax = fmax(vmax, fabs(V[i]));
    }
    if (!(vmax > 0)) FAIL("V is zero");

    int64_t *cnt = malloc(sizeof(int64_t) * n);
    const int64_t rejn = oracle_splat_nearest(p, nr, m, dims, bbox, S, cnt, V2);
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += cnt[i];
    if (rejn != rej || total != m - rej) FAIL("nearest splat counts %lld + %lld", (long long)total, (long long)rejn);

    /* A = 0.6 - |x| on the voxel centres: inside the sphere is above 0 */
    double *A = malloc(sizeof(double) * n);
    for (int z = 0; z < dims[2]; ++z)
        for (int y = 0; y < dims[1]; ++y)
            for (int x = 0; x < dims[0]; ++x) {
                const int q[3] = {x, y, z};
                double r2 = 0;
                for (int a = 0; a < 3; ++a) {
                    const double h = ((double)bbox[a + 3] - bbox[a]) / dims[a];
                    const double c = bbox[a] + (q[a] + 0.5) * h;
                    r2 += c * c;
                }
                A[x + (int64_t)dims[0] * (y + (int64_t)dims[1] * z)] = 0.6 - sqrt(r2);
            }
    int64_t used = 0;
    const double L = oracle_level(A, dims, bbox, p, m, &used);
    if (used != m - rej || !(fabs(L) < 0.2)) FAIL("level %g from %lld points", L, (long long)used);

    uint8_t *cases = malloc((size_t)(dims[0] - 1) * (dims[1] - 1) * (dims[2] - 1));
    int64_t nv = 0, nt = 0;
    double vsmall[3 * 4];
    int32_t tsmall[3 * 4];
    int rc = oracle_marching_cubes(A, dims, bbox, L, counts, (const int8_t *)edges, vsmall, 4, tsmall, 4, cases,
                                   &nv, &nt, 1, NULL);
    if (nv <= 4 || nt <= 4) FAIL("mesh too small: %lld vertices, %lld triangles", (long long)nv, (long long)nt);
    (void)rc;
    double *verts = malloc(sizeof(double) * 3 * nv), *nrm = malloc(sizeof(double) * 3 * nv);
    int32_t *tris = malloc(sizeof(int32_t) * 3 * nt);
    int64_t nv2 = 0, nt2 = 0;
    rc = oracle_marching_cubes(A, dims, bbox, L, counts, (const int8_t *)edges, verts, nv, tris, nt, cases, &nv2,
                               &nt2, 2, nrm);
    if (rc != 0 || nv2 != nv || nt2 != nt) FAIL("full mesh rc %d", rc);
    for (int64_t i = 0; i < 3 * nt; ++i)
        if (tris[i] < 0 || tris[i] >= nv) FAIL("triangle index out of range");
    /* closed: every undirected edge in exactly two triangles (sum over edges of 2 = 3 nt) */
    if ((3 * nt) % 2) FAIL("odd edge count");

    free(p); free(nr); free(w); free(S); free(D); free(V); free(V2); free(cnt); free(A); free(cases);
    free(verts); free(nrm); free(tris);
    printf("ok %lld vertices %lld triangles L %.6f\n", (long long)nv, (long long)nt, L);
    return 0;
}
