// Host runtime and C ABI of the gfx950 FT-reconstruction library.
//
// A context owns, per device: a plan cache keyed by grid dims (radix
// schedule and float32 twiddle tables rounded from double), grow-only device
// scratch, a pinned status block, and optional per-kernel HIP-event timing.
// fvr_reconstruct enqueues the stages of Sec. III-B on the context's stream:
//   reset -> bin_count -> tile_list/tile_order (+ bin scan) -> bin_scatter ->
//   splat+fft_x -> fft_y -> fft_z+solve -> fft_y_inv + fft_x_c2r (or the
//   fused fft_yx_inv) -> level -> [mc_classify] -> mc_count -> scan ->
//   mc_generate -> mc_triangles -> one device->host read of the status
//   (mesh counts, flags, level) at the end.
#include <algorithm>
#include <array>
#include <chrono>
#include <deque>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fvr.h"
#include "fvr_common.h"

using namespace fvr;

namespace {

enum KernelId {
    K_PREP, K_BIN_COUNT, K_TILE_LIST, K_BIN_SCATTER, K_SPLAT_FFT_X, K_FFT_Y_FWD,
    K_FFT_Z_SOLVE, K_FFT_Y_INV, K_FFT_X_C2R, K_FFT_YX_INV, K_LEVEL, K_MC_CLASSIFY, K_MC_COUNT, K_MC_SCAN,
    K_MC_GENERATE, K_MC_TRIANGLES, K_COUNT
};
const char *kKernelNames[K_COUNT] = {
    "prep", "bin_count", "tile_list", "bin_scatter", "splat_fft_x", "fft_y_fwd",
    "fft_z_solve", "fft_y_inv", "fft_x_c2r", "fft_yx_inv", "level", "mc_classify", "mc_count", "mc_scan",
    "mc_generate", "mc_triangles"};

thread_local std::string g_error;

// A scratch buffer of the context: memory it owns (p, cap, grown on demand),
// or, during an allocation-free call, a slice of the device's static scratch
// array; `view` is the memory the current call uses.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    void *view = nullptr;
    uint64_t epoch = 0;  // allocation-free call that carved `view` (0: owned memory)
    size_t bytes = 0;    // size of that slice
};

struct Plan {
    int dims[3];
    FftAxis ax[3];
    SplatConsts sc;
    uint64_t tune_gen = 0;  // tuning table generation the plan was built from
};

// Radix schedule: as many 8s as possible, then a 4 or 2, then 3s and 5s
// (at most kMaxStages; false if n has another factor or needs more stages).
bool factor(int n, int rad[kMaxStages], int &ns) {
    ns = 0;
    int a = 0;
    while (n % 2 == 0) { n /= 2; ++a; }
    auto push = [&](int r) {
        if (ns == kMaxStages) return false;
        rad[ns++] = r;
        return true;
    };
    while (a >= 3) { if (!push(8)) return false; a -= 3; }
    if (a == 2 && !push(4)) return false;
    if (a == 1 && !push(2)) return false;
    while (n % 3 == 0) { n /= 3; if (!push(3)) return false; }
    while (n % 5 == 0) { n /= 5; if (!push(5)) return false; }
    return n == 1;
}

// Tuned plan parameters per grid shape (fvr_set_tuning), shared by every
// context and batch of the process so that all paths compute the same bits.
struct Tuning {
    int radices[3][kMaxStages];
    int nstages[3];  // 0: the default schedule for that axis
    int splat_ty, splat_tz;  // 0: the default splat tile
};
std::mutex g_tune_mutex;
std::map<std::array<int, 3>, Tuning> g_tuning;
uint64_t g_tune_gen = 1;

}  // namespace

struct fvr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::map<std::array<int, 3>, Plan> plans;
    // allocation-free calls carve their buffers from the static scratch
    unsigned char *arena = nullptr;  // non-null during such a call
    size_t arena_off = 0;
    size_t arena_cap = FVR_NOALLOC_SCRATCH_BYTES;
    uint64_t arena_epoch = 0;
    uint64_t scratch_gen = 0;  // bumped whenever an owned buffer moves
    DevBuf bin_count, bin_off, key, rank, rec, spec, field, vidx, cells, mc_cnt, mc_off, mc_codes,
        lvl_sum, lvl_cnt, status, level_f32, scan_part, occ, zocc, tiles, tile_pend, blk_max, rowmm, mc_list,
        fe_rowcnt, fe_dense, fe_flag, fe_off;
    DevStatus *host_status = nullptr;
    fvr_stats last{};  // sizes of the last call; the counters come from host_status
    uint32_t timing_mask = 0;  // bit k: time kernel k
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<int> ev_kid;
    size_t ev_used = 0;
    double t_ms[K_COUNT] = {0};
    int64_t t_n[K_COUNT] = {0};
};

namespace {

const char *const kRangeMsg = "a 16-bit spectrum value overflowed: use float32 storage";

fvr_status fail(fvr_ctx *c, fvr_status s, const std::string &msg) {
    if (c) c->err = msg;
    g_error = msg;
    return s;
}

fvr_status hip_fail(fvr_ctx *c, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? FVR_E_NOMEM : FVR_E_DEVICE, m);
}

#define HIP_TRY(c, expr, what)                              \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail((c), e_, (what)); \
    } while (0)

hipError_t ensure(DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (bytes <= b.cap) return hipSuccess;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.cap = bytes;
    return e;
}

// Makes `bytes` of buffer b available to the current call: the context's
// own memory (grown with hipMalloc), or, in an allocation-free call, a
// 256-byte aligned slice of the static scratch (the same slice when the
// buffer is asked for again within the call).  Overflowing the static
// scratch reports hipErrorOutOfMemory without allocating.
hipError_t get(fvr_ctx *c, DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (!c->arena) {
        void *before = b.p;
        hipError_t e = ensure(b, bytes);
        if (e == hipSuccess) b.view = b.p;
        if (b.p != before) ++c->scratch_gen;  // captured graphs hold the old address
        b.epoch = 0;
        return e;
    }
    if (b.epoch == c->arena_epoch && b.bytes >= bytes) return hipSuccess;
    const size_t off = (c->arena_off + 255) & ~(size_t)255;
    if (off > c->arena_cap || bytes > c->arena_cap - off) return hipErrorOutOfMemory;
    b.view = c->arena + off;
    b.epoch = c->arena_epoch;
    b.bytes = bytes;
    c->arena_off = off + bytes;
    return hipSuccess;
}

template <class T> T *P(DevBuf &b) { return static_cast<T *>(b.view); }

// RAII launch timer: records a HIP event before and after the launch when
// timing is on; the pairs are read after the next synchronisation.
struct Timed {
    fvr_ctx *c;
    int kid;
    size_t idx = (size_t)-1;
    Timed(fvr_ctx *ctx, int k) : c(ctx), kid(k) {
        if (!((c->timing_mask >> k) & 1u)) return;
        if (c->ev_used == c->ev.size()) {
            // timing-only events: no system-scope fence (and cache write-back)
            // at each record; they are read after a stream synchronisation
            hipEvent_t a, b;
            if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return;
            if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
                (void)hipEventDestroy(a);
                return;
            }
            c->ev.push_back({a, b});
            c->ev_kid.push_back(k);
        }
        idx = c->ev_used++;
        c->ev_kid[idx] = k;
        (void)hipEventRecord(c->ev[idx].first, c->stream);
    }
    ~Timed() {
        if (idx != (size_t)-1) (void)hipEventRecord(c->ev[idx].second, c->stream);
    }
};

void collect_timing(fvr_ctx *c) {
    for (size_t i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[i].first, c->ev[i].second) == hipSuccess) {
            c->t_ms[c->ev_kid[i]] += ms;
            c->t_n[c->ev_kid[i]] += 1;
        }
    }
    c->ev_used = 0;
}

fvr_status sync(fvr_ctx *c) {
    HIP_TRY(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (c->ev_used) collect_timing(c);
    return FVR_OK;
}

fvr_status check_grid(fvr_ctx *c, const int32_t dims[3], const float bbox[6]) {
    if (!dims || !bbox) return fail(c, FVR_E_INVALID, "dims or bbox is NULL");
    for (int a = 0; a < 3; ++a) {
        const int n = dims[a];
        if (n < 8 || (n & 1)) return fail(c, FVR_E_INVALID, "grid dims must be even and >= 8");
        if (n > kMaxDim) return fail(c, FVR_E_UNSUPPORTED, "grid dim above 512");
        int r[kMaxStages], ns;
        if (!factor(n, r, ns)) return fail(c, FVR_E_UNSUPPORTED, "grid dim must be 2^a 3^b 5^c");
        if (!std::isfinite(bbox[a]) || !std::isfinite(bbox[a + 3]) || !(bbox[a + 3] > bbox[a]))
            return fail(c, FVR_E_INVALID, "bbox must be finite with max > min");
        const float h = (bbox[a + 3] - bbox[a]) / (float)n;
        if (!(h > 0.f) || !std::isfinite(h)) return fail(c, FVR_E_INVALID, "bbox extent too small");
    }
    return FVR_OK;
}

// Marching cubes alone has no transform-size constraint: any dims >= 2 whose
// 3 n edge slots fit int32 indexing.
fvr_status check_extract_grid(fvr_ctx *c, const int32_t dims[3], const float bbox[6]) {
    if (!dims || !bbox) return fail(c, FVR_E_INVALID, "dims or bbox is NULL");
    int64_t n = 1;
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < 2) return fail(c, FVR_E_INVALID, "grid dims must be >= 2");
        n *= dims[a];
        if (!std::isfinite(bbox[a]) || !std::isfinite(bbox[a + 3]) || !(bbox[a + 3] > bbox[a]))
            return fail(c, FVR_E_INVALID, "bbox must be finite with max > min");
    }
    if (3 * n > 0x7fffffff) return fail(c, FVR_E_UNSUPPORTED, "grid too large for int32 indexing");
    return FVR_OK;
}

Grid make_grid(const int32_t dims[3], const float bbox[6]) {
    Grid g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = dims[a];
        g.bmin[a] = bbox[a];
        g.bmax[a] = bbox[a + 3];
        volatile float ext = bbox[a + 3] - bbox[a];
        volatile float h = ext / (float)dims[a];
        g.h[a] = h;
        g.wstep[a] = (float)(2.0 * M_PI / ((double)bbox[a + 3] - (double)bbox[a]));
    }
    g.H = dims[0] / 2 + 1;
    g.Hp = (g.H + 15) / 16 * 16;
    g.ty = g.tz = 1;  // splat tiling, filled in from the plan where it matters
    g.tiles_y = dims[1];
    g.spec_st = kSpecF32;
    g.fscale[0] = g.fscale[1] = g.fscale[2] = 1.0f;
    g.iscale = 1.0f / ((float)dims[0] * (float)dims[1] * (float)dims[2]);
    return g;
}

// The grid of a frame, with its spectrum storage.  The reduced storages
// store each forward pass's output times 1/N_axis (powers of two: exact
// scalings), and take the angular frequencies in units of 1/h_x: the
// derivative multiplies by h_x w and the solve divides by h_x^2 |w|^2, so
// the spectrum holds A / h_x and the last inverse pass multiplies by h_x.
// Without that, the solve's 1/|w|^2 would carry a factor h^2 (the square of
// the bbox's length unit) into every stored value, and FP16 would keep
// most of them as subnormals.
Grid frame_grid(const fvr_frame *f) {
    Grid g = make_grid(f->dims, f->bbox);
    if (f->options & (FVR_STORAGE_BF16 | FVR_STORAGE_FP16)) {
        g.spec_st = (f->options & FVR_STORAGE_BF16) ? kSpecBF16 : kSpecF16;
        const double hx = ((double)f->bbox[3] - (double)f->bbox[0]) / (double)f->dims[0];
        for (int a = 0; a < 3; ++a) {
            g.fscale[a] = 1.0f / (float)f->dims[a];
            g.wstep[a] = (float)(2.0 * M_PI * hx / ((double)f->bbox[a + 3] - (double)f->bbox[a]));
        }
        g.iscale = (float)hx;
    }
    return g;
}

// Default splat tile: ty x tz full x-rows.  Four rows (2 x 2) up to
// Nx = 128 and eight (2 x 4) above, within the kernel's plane bound (R Nx <=
// 2048; Nx <= 512 keeps 4 rows in bound).  Measured on the human proxy at
// 128^3: 59 us for the splat with 2 x 2 tiles against 112 us with 4 x 4
// (smaller tiles balance the persistent blocks better); at 256^3 2 x 4
// (104 us) beats 2 x 2 (126 us); the autotuner picks the same row counts
// on the {96, 128, 160, 192}^3 frames of the batched workload.
void default_splat_tile(int nx, int &ty, int &tz) {
    int R = nx <= 128 ? 4 : 8;
    while (R > 4 && R * nx > splat_max_plane()) R /= 2;
    tz = R >= 8 ? 4 : 2;
    ty = R / tz;
}

// Radix schedules, twiddles (the device's static table: nothing to allocate)
// and splat tiling of a grid shape.
fvr_status build_plan(fvr_ctx *c, const int32_t dims[3], Plan &np) {
    std::memcpy(np.dims, dims, sizeof(np.dims));
    Tuning tu{};
    bool tuned = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        auto it = g_tuning.find({dims[0], dims[1], dims[2]});
        if (it != g_tuning.end()) {
            tu = it->second;
            tuned = true;
        }
        np.tune_gen = g_tune_gen;
    }
    for (int a = 0; a < 3; ++a) {
        int r[kMaxStages], ns;
        if (!factor(dims[a], r, ns)) return fail(c, FVR_E_UNSUPPORTED, "grid dim must be 2^a 3^b 5^c");
        if (tuned && tu.nstages[a] > 0) {  // a tuned radix order (validated when it was set)
            ns = tu.nstages[a];
            for (int k = 0; k < ns; ++k) r[k] = tu.radices[a][k];
        }
        np.ax[a].n = dims[a];
        np.ax[a].nstages = ns;
        np.ax[a].radices = 0;
        for (int k = 0; k < ns; ++k) np.ax[a].radices |= (unsigned)r[k] << (4 * k);
        np.ax[a].tw = statics_twiddles(c->device, dims[a]);
        if (!np.ax[a].tw) return fail(c, FVR_E_DEVICE, "twiddle table missing for this length");
    }
    default_splat_tile(dims[0], np.sc.ty, np.sc.tz);
    if (tuned && tu.splat_ty > 0) {
        np.sc.ty = tu.splat_ty;
        np.sc.tz = tu.splat_tz;
    }
    np.sc.tiles_y = (dims[1] + np.sc.ty - 1) / np.sc.ty;
    return FVR_OK;
}

// A splat tile of ty x tz full x-rows fits the kernel: an even number of rows
// (the x transform pairs rows of one channel), at most kSplatMaxPlane voxels
// per channel, at most 128 footprint bins.
bool splat_tile_ok(int nx, int ty, int tz) {
    const int R = ty * tz;
    return ty >= 1 && tz >= 1 && R % 2 == 0 && R * nx <= splat_max_plane() && (ty + 3) * (tz + 3) <= 128;
}

// Frame-dependent splat constants: the Gaussians' exponents (the bbox may
// change between calls) and the splat variant.
void plan_geometry(Plan *p, const fvr_frame *f) {
    const int32_t *dims = f->dims;
    const float *bbox = f->bbox;
    double h[3], s1sq = 0.0;
    for (int a = 0; a < 3; ++a) {
        h[a] = ((double)bbox[a + 3] - (double)bbox[a]) / (double)dims[a];
        s1sq += 0.25 * h[a] * h[a];
    }
    const double s2sq = 1.5 * s1sq;
    const double log2e = 1.4426950408889634;
    for (int a = 0; a < 3; ++a) {
        p->sc.e1[a] = (float)(-h[a] * h[a] / s1sq * log2e);
        p->sc.e2[a] = (float)(-h[a] * h[a] / s2sq * log2e);
    }
    const bool nearest = (f->options & FVR_SPLAT_NEAREST) != 0;
    p->sc.nearest = nearest ? 1 : 0;
    p->sc.fp_lo = nearest ? 0 : -1;
    p->sc.fp_hi = nearest ? 0 : 2;
    // V = S / D carries the ratio sigma2/sigma1 of the two 1/sigma factors;
    // the nearest-voxel splat is a plain mean
    p->sc.vscale = nearest ? 1.0f : (float)std::sqrt(1.5);
}

fvr_status get_plan(fvr_ctx *c, const fvr_frame *f, Plan **out) {
    const int32_t *dims = f->dims;
    const std::array<int, 3> key = {dims[0], dims[1], dims[2]};
    auto it = c->plans.find(key);
    Plan *p;
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        gen = g_tune_gen;
    }
    if (it != c->plans.end() && it->second.tune_gen != gen) {  // the tuning changed
        c->plans.erase(it);
        it = c->plans.end();
    }
    if (it == c->plans.end()) {
        Plan np;
        fvr_status r = build_plan(c, dims, np);
        if (r != FVR_OK) return r;
        p = &(c->plans[key] = np);
    } else {
        p = &it->second;
    }
    plan_geometry(p, f);
    *out = p;
    return FVR_OK;
}

// The frame's host-side fields: point count, required pointers, grid, bbox.
fvr_status check_frame_fields(fvr_ctx *c, const fvr_frame *f) {
    if (!f) return fail(c, FVR_E_INVALID, "frame is NULL");
    if (f->n_points < 0) return fail(c, FVR_E_INVALID, "n_points < 0");
    // the kernels index coordinates as 3 i in 32-bit integers
    if (f->n_points > FVR_MAX_POINTS) return fail(c, FVR_E_INVALID, "n_points above FVR_MAX_POINTS");
    if (f->n_points > 0 && (!f->points || !f->normals))
        return fail(c, FVR_E_INVALID, "points or normals is NULL");
    if (f->options & ~(FVR_SPLAT_NEAREST | FVR_STORAGE_BF16 | FVR_STORAGE_FP16))
        return fail(c, FVR_E_INVALID, "unknown frame option bits");
    if ((f->options & FVR_STORAGE_BF16) && (f->options & FVR_STORAGE_FP16))
        return fail(c, FVR_E_INVALID, "FVR_STORAGE_BF16 and FVR_STORAGE_FP16 together");
    fvr_status r = check_grid(c, f->dims, f->bbox);
    if (r != FVR_OK) return r;
    return FVR_OK;
}

fvr_status check_frame(fvr_ctx *c, const fvr_frame *f) {
    if (!c) return fail(nullptr, FVR_E_INVALID, "context is NULL");
    return check_frame_fields(c, f);
}

// A scratch request of the current call; in an allocation-free call a
// request beyond the static scratch is refused with FVR_E_NOMEM.
#define GET(c, buf, bytes, what)                                                              \
    do {                                                                                      \
        hipError_t e_ = get((c), (buf), (bytes));                                             \
        if (e_ == hipErrorOutOfMemory && (c)->arena)                                          \
            return fail((c), FVR_E_NOMEM,                                                     \
                        std::string("the frame needs more than the FVR_NOALLOC_SCRATCH_BYTES " \
                                    "of static scratch (at ") + (what) + ")");                \
        if (e_ != hipSuccess) return hip_fail((c), e_, (what));                               \
    } while (0)

// Scratch of stages 1-5 (status, binning, splat, transforms) for m points.
fvr_status field_bufs(fvr_ctx *c, const Grid &g, const Plan *p, int m) {
    const int ntiles = p->sc.tiles_y * ((g.n[2] + p->sc.tz - 1) / p->sc.tz);
    const int nbins = (g.n[2] + 1) * (g.n[1] + 1);
    const size_t nspec = (size_t)g.n[2] * g.n[1] * g.Hp;
    GET(c, c->status, sizeof(DevStatus), "status");
    GET(c, c->bin_count, sizeof(int32_t) * nbins, "bins");
    GET(c, c->bin_off, sizeof(int32_t) * (nbins + 1), "bin offsets");
    GET(c, c->key, sizeof(int32_t) * (size_t)m, "keys");
    GET(c, c->rank, sizeof(int32_t) * (size_t)m, "ranks");
    GET(c, c->rec, sizeof(float4) * 2 * (size_t)m, "records");
    GET(c, c->spec, spec_elem_bytes(g.spec_st) * 3 * nspec, "spectra");
    GET(c, c->occ, (size_t)ntiles, "tile occupancy");
    GET(c, c->tiles, sizeof(int32_t) * (size_t)ntiles, "tile list");
    GET(c, c->tile_pend, sizeof(int2) * (size_t)ntiles, "tile costs");
    GET(c, c->blk_max, sizeof(uint2) * (size_t)std::max(1, bin_count_blocks(m)), "block maxima");
    GET(c, c->zocc, (size_t)g.n[2], "plane occupancy");
    // sized for both scans of the frame before anything is enqueued
    const int scan_items = std::max(bin_scan_tiles(nbins), 3 * scan_partials(mc_blocks(g)));
    GET(c, c->scan_part, sizeof(int32_t) * (size_t)scan_items, "scan scratch");
    GET(c, c->rowmm, sizeof(float2) * (size_t)g.n[1] * g.n[2], "row ranges");
    return FVR_OK;
}

// Scratch of the iso-level (stage 6) for m points.
fvr_status level_bufs(fvr_ctx *c, int m) {
    const int nb = level_blocks(m);
    GET(c, c->lvl_sum, sizeof(double) * (size_t)nb, "level partials");
    GET(c, c->lvl_cnt, sizeof(int32_t) * (size_t)nb, "level counts");
    GET(c, c->level_f32, sizeof(float), "level");
    return FVR_OK;
}

// Marching cubes never writes more active cells than triangles (every active
// cell emits at least one) or than the grid has cells.
MeshCaps mesh_caps(const Grid &g, const fvr_mesh *mesh, bool check_invalid) {
    const long long ncell_max = (long long)(g.n[0] - 1) * (g.n[1] - 1) * (g.n[2] - 1);
    MeshCaps caps;
    caps.vertices = mesh->vertices ? mesh->vertex_capacity : 0;
    caps.triangles = mesh->triangles ? mesh->triangle_capacity : 0;
    caps.cells = std::max(0LL, std::min((long long)caps.triangles, ncell_max));
    caps.check_invalid = check_invalid ? 1 : 0;
    return caps;
}

// Scratch of stages 7-9 (marching cubes), with the block list of the fused path.
fvr_status mc_bufs(fvr_ctx *c, const Grid &g, const MeshCaps &caps, bool with_list) {
    const int nb = mc_blocks(g);
    const size_t n = (size_t)g.n[0] * g.n[1] * g.n[2];
    GET(c, c->mc_cnt, sizeof(int32_t) * 3 * (size_t)nb, "mc counts");
    GET(c, c->mc_off, sizeof(int32_t) * 3 * ((size_t)nb + 1), "mc offsets");
    GET(c, c->vidx, sizeof(int32_t) * 3 * n, "vertex ids");
    GET(c, c->mc_codes, (size_t)nb * 1024, "point codes");
    GET(c, c->scan_part, sizeof(int32_t) * 3 * (size_t)scan_partials(nb), "scan scratch");
    if (with_list) GET(c, c->mc_list, sizeof(int32_t) * (size_t)nb, "mc block list");
    GET(c, c->cells, sizeof(int4) * (size_t)std::max(1LL, caps.cells), "active cells");
    return FVR_OK;
}

// Stages 1-4 (and optionally 5): status reset, binning, splat + x FFT and,
// unless splat_only, the remaining transform passes into `field`.
fvr_status run_field(fvr_ctx *c, const fvr_frame *f, Plan *p, const Grid &g0, float *field,
                     float *v_out, bool splat_only) {
    Grid g = g0;
    g.ty = p->sc.ty;
    g.tz = p->sc.tz;
    g.tiles_y = p->sc.tiles_y;
    const int m = (int)f->n_points;
    const int nbins = (g.n[2] + 1) * (g.n[1] + 1);
    fvr_status r = field_bufs(c, g, p, m);
    if (r != FVR_OK) return r;
    c->last = fvr_stats{};
    c->last.tiles = p->sc.tiles_y * ((g.n[2] + p->sc.tz - 1) / p->sc.tz);
    c->last.planes = g.n[2];
    DevStatus *st = P<DevStatus>(c->status);
    hipStream_t s = c->stream;
    { Timed t(c, K_PREP); HIP_TRY(c, launch_prep(st, P<int32_t>(c->bin_count), nbins, s), "prep"); }
    { Timed t(c, K_BIN_COUNT);
      HIP_TRY(c, launch_bin_count(f->points, f->normals, f->weights, m, g, p->sc.nearest, P<int32_t>(c->bin_count),
                                  P<int32_t>(c->key), P<int32_t>(c->rank), P<uint2>(c->blk_max), st, s),
              "bin_count"); }
    { Timed t(c, K_TILE_LIST);
      HIP_TRY(c, launch_tile_list(P<int32_t>(c->bin_count), P<int32_t>(c->bin_off), nbins,
                                  P<int32_t>(c->scan_part), g, p->sc, P<uint8_t>(c->occ),
                                  P<int2>(c->tile_pend), P<int32_t>(c->tiles), P<uint2>(c->blk_max), m, st, s),
              "tile_list"); }
    { Timed t(c, K_BIN_SCATTER);
      HIP_TRY(c, launch_bin_scatter(f->points, f->normals, f->weights, m, g, P<int32_t>(c->key),
                                    P<int32_t>(c->rank), P<int32_t>(c->bin_off), st, p->sc.nearest,
                                    P<float4>(c->rec), s),
              "bin_scatter"); }
    { Timed t(c, K_SPLAT_FFT_X);
      HIP_TRY(c, launch_splat_fft_x(P<float4>(c->rec), P<int32_t>(c->bin_off), g, p->sc, p->ax[0],
                                    st, P<int32_t>(c->tiles), P<void>(c->spec), v_out, s), "splat_fft_x"); }
    if (splat_only) return FVR_OK;
    void *sp = P<void>(c->spec);
    { Timed t(c, K_FFT_Y_FWD);
      HIP_TRY(c, launch_fft_y_fwd(sp, P<uint8_t>(c->occ), P<uint8_t>(c->zocc), st, g, p->ax[1], s), "fft_y_fwd"); }
    { Timed t(c, K_FFT_Z_SOLVE);
      HIP_TRY(c, launch_fft_z_solve(sp, P<uint8_t>(c->zocc), g, p->ax[2], s), "fft_z_solve"); }
    if (fft_yx_fused(g)) {
        Timed t(c, K_FFT_YX_INV);
        HIP_TRY(c, launch_fft_yx_inv(sp, field, P<float2>(c->rowmm), st, g, p->ax[1], s), "fft_yx_inv");
    } else {
        { Timed t(c, K_FFT_Y_INV); HIP_TRY(c, launch_fft_y_inv(sp, g, p->ax[1], s), "fft_y_inv"); }
        { Timed t(c, K_FFT_X_C2R); HIP_TRY(c, launch_fft_x_c2r(sp, field, P<float2>(c->rowmm), st, g, p->ax[0], s), "fft_x_c2r"); }
    }
    return FVR_OK;
}

// final = false leaves the block partials for the classification of the
// marching-cubes blocks to reduce (run_mc with rowmm).
fvr_status run_level(fvr_ctx *c, const fvr_frame *f, const Grid &g, const float *field, bool final = true) {
    const int m = (int)f->n_points;
    fvr_status r = level_bufs(c, m);
    if (r != FVR_OK) return r;
    { Timed t(c, K_LEVEL);
      HIP_TRY(c, launch_level(f->points, m, field, g, P<double>(c->lvl_sum), P<int32_t>(c->lvl_cnt),
                              P<DevStatus>(c->status), P<float>(c->level_f32), final, c->stream),
              "level"); }
    return FVR_OK;
}

// Marching cubes on `field` at the level in c->level_f32; status block must
// already be reset.  Fills mesh counts; writes arrays only if they fit.
// With rowmm, level_nb > 0 says the level's level_nb block partials are still to
// be reduced (run_level with final = false); the classification does it.
// Marching cubes enqueued; block 0 of mc_generate copies the final status
// block to host_dst (pinned host memory).
fvr_status enqueue_mc(fvr_ctx *c, const Grid &g, const float *field, const float2 *rowmm,
                      const fvr_mesh *mesh, uint8_t *cases_out, bool check_invalid, int level_nb,
                      DevStatus *host_dst) {
    const int nb = mc_blocks(g);
    const MeshCaps caps = mesh_caps(g, mesh, check_invalid);
    fvr_status r0 = mc_bufs(c, g, caps, rowmm != nullptr);
    if (r0 != FVR_OK) return r0;
    c->last.mc_blocks = nb;
    c->last.mc_blocks_listed = rowmm ? -1 : nb;  // -1: read from the status block
    DevStatus *st = P<DevStatus>(c->status);
    hipStream_t s = c->stream;
    int32_t *list = nullptr;
    if (rowmm) {
        list = P<int32_t>(c->mc_list);
        Timed t(c, K_MC_CLASSIFY);
        HIP_TRY(c, launch_mc_classify(P<float>(c->level_f32), level_nb > 0 ? P<double>(c->lvl_sum) : nullptr,
                                      P<int32_t>(c->lvl_cnt), level_nb, rowmm, g, P<int32_t>(c->mc_cnt),
                                      list, st, s), "mc_classify");
    }
    { Timed t(c, K_MC_COUNT);
      HIP_TRY(c, launch_mc_count(field, P<float>(c->level_f32), list, g, P<int32_t>(c->mc_cnt),
                                 P<uint32_t>(c->mc_codes), cases_out, st, s), "mc_count"); }
    { Timed t(c, K_MC_SCAN);
      if (list) {
          HIP_TRY(c, launch_mc_list_scan(list, P<int32_t>(c->mc_cnt), nb, P<int32_t>(c->mc_off), st, s),
                  "mc_scan");
      } else {
          HIP_TRY(c, launch_scan(P<int32_t>(c->mc_cnt), P<int32_t>(c->mc_off), nb, 3,
                                 P<int32_t>(c->scan_part), st->mc_total, s), "mc_scan");
      } }
    // Generation follows without a host round trip: the kernels check the
    // totals against the capacities themselves and write nothing on a shortfall.
    { Timed t(c, K_MC_GENERATE);
      HIP_TRY(c, launch_mc_generate(field, P<float>(c->level_f32), list, g, P<int32_t>(c->mc_cnt),
                                    P<int32_t>(c->mc_off), P<uint32_t>(c->mc_codes), mesh->vertices,
                                    mesh->normals, P<int32_t>(c->vidx), P<int4>(c->cells), st, caps,
                                    host_dst, s),
              "mc_generate"); }
    { Timed t(c, K_MC_TRIANGLES);
      HIP_TRY(c, launch_mc_triangles(P<int4>(c->cells), P<int32_t>(c->vidx), g, mesh->triangles, st,
                                     caps, s), "mc_triangles"); }
    return FVR_OK;
}

// The mesh counts, flags and errors of a finished frame from its status block.
fvr_status finish_mesh(fvr_ctx *c, const DevStatus &hs, fvr_mesh *mesh, bool check_invalid) {
    if (check_invalid && (hs.flags & kFlagInvalid))
        return fail(c, FVR_E_INVALID, "non-finite point, normal or weight, or a negative weight");
    if (hs.flags & kFlagRange) return fail(c, FVR_E_RANGE, kRangeMsg);
    mesh->n_vertices = hs.mc_total[0];
    mesh->n_triangles = hs.mc_total[1];
    mesh->n_rejected = hs.rejected;
    mesh->flags = (hs.flags & kFlagOpen) ? FVR_FLAG_OPEN_SURFACE : 0u;
    if (hs.mc_total[0] > mesh->vertex_capacity || hs.mc_total[1] > mesh->triangle_capacity)
        return fail(c, FVR_E_CAPACITY, "mesh output capacity too small");
    if (hs.mc_total[0] > 0 && !mesh->vertices) return fail(c, FVR_E_INVALID, "vertices is NULL");
    if (hs.mc_total[1] > 0 && !mesh->triangles) return fail(c, FVR_E_INVALID, "triangles is NULL");
    return FVR_OK;
}

// Marching cubes on `field` at the level in c->level_f32 (status block
// already reset), waited for; fills the mesh counts.
fvr_status run_mc(fvr_ctx *c, const Grid &g, const float *field, const float2 *rowmm, fvr_mesh *mesh,
                  uint8_t *cases_out, bool check_invalid, int level_nb = 0) {
    fvr_status r = enqueue_mc(c, g, field, rowmm, mesh, cases_out, check_invalid, level_nb, c->host_status);
    if (r != FVR_OK) return r;
    if ((r = sync(c)) != FVR_OK) return r;
    const DevStatus hs = *c->host_status;
    return finish_mesh(c, hs, mesh, check_invalid);
}

// All stages of one frame enqueued on c's stream (plan and scratch ready);
// the final status block goes to host_dst.
fvr_status enqueue_reconstruct(fvr_ctx *c, const fvr_frame *f, Plan *p, const fvr_mesh *mesh,
                               DevStatus *host_dst) {
    const Grid g = frame_grid(f);
    fvr_status r;
    GET(c, c->field, sizeof(float) * (size_t)g.n[0] * g.n[1] * g.n[2], "field");
    if ((r = run_field(c, f, p, g, P<float>(c->field), nullptr, false)) != FVR_OK) return r;
    // the last inverse pass left each row's range of A: blocks of cells
    // entirely on one side of the level skip the field, and their
    // classification also finishes the level
    const int level_nb = level_blocks((int)f->n_points);
    if ((r = run_level(c, f, g, P<float>(c->field), level_nb == 0)) != FVR_OK) return r;
    return enqueue_mc(c, g, P<float>(c->field), P<float2>(c->rowmm), mesh, nullptr, true, level_nb, host_dst);
}

// Every device buffer a context owns.
std::vector<DevBuf *> ctx_bufs(fvr_ctx *c) {
    return {&c->bin_count, &c->bin_off, &c->key, &c->rank, &c->rec, &c->spec, &c->field,
            &c->vidx, &c->cells, &c->mc_cnt, &c->mc_off, &c->mc_codes, &c->lvl_sum, &c->lvl_cnt,
            &c->status, &c->level_f32, &c->scan_part, &c->occ, &c->zocc, &c->tiles, &c->tile_pend,
            &c->blk_max, &c->rowmm, &c->mc_list, &c->fe_rowcnt, &c->fe_dense, &c->fe_flag, &c->fe_off};
}

size_t ctx_bytes(fvr_ctx *c) {
    size_t t = 0;
    for (DevBuf *b : ctx_bufs(c)) t += b->cap;
    return t;
}

// Every scratch buffer of one frame, requested before anything is enqueued.
fvr_status frame_bufs(fvr_ctx *c, const fvr_frame *f, const Plan *p, const fvr_mesh *mesh) {
    const Grid g = frame_grid(f);
    const int m = (int)f->n_points;
    GET(c, c->field, sizeof(float) * (size_t)g.n[0] * g.n[1] * g.n[2], "field");
    fvr_status r;
    if ((r = field_bufs(c, g, p, m)) != FVR_OK) return r;
    if ((r = level_bufs(c, m)) != FVR_OK) return r;
    return mc_bufs(c, g, mesh_caps(g, mesh, true), true);
}

}  // namespace

extern "C" {

fvr_status fvr_create(int device, void *hip_stream, fvr_ctx **out) {
    if (!out) return fail(nullptr, FVR_E_INVALID, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return fail(nullptr, FVR_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(nullptr, FVR_E_INVALID, "device index out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    // twiddle tables and static scratch of this device (looked up once)
    e = statics_init(device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "device statics");
    fvr_ctx *c = new fvr_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    uint8_t counts[256];
    int8_t edges[256 * kMcRow];
    try {
        mc_generate_table(counts, edges);
    } catch (const std::exception &ex) {
        delete c;
        return fail(nullptr, FVR_E_DEVICE, std::string("mc table: ") + ex.what());
    }
    e = mc_upload_table(counts, edges);
    if (e == hipSuccess) e = splat_configure();
    if (e == hipSuccess) e = fft_configure();
    if (e == hipSuccess) e = mc_configure();
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->host_status, sizeof(DevStatus));
    if (e != hipSuccess) {
        fvr_status s = hip_fail(nullptr, e, "context setup");
        delete c;
        return s;
    }
    *out = c;
    return FVR_OK;
}

void fvr_destroy(fvr_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (DevBuf *b : ctx_bufs(c))
        if (b->p) (void)hipFree(b->p);
    for (auto &pr : c->ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (c->host_status) (void)hipHostFree(c->host_status);
    delete c;
}

fvr_status fvr_set_stream(fvr_ctx *c, void *hip_stream) {
    if (!c) return fail(nullptr, FVR_E_INVALID, "context is NULL");
    c->stream = (hipStream_t)hip_stream;
    return FVR_OK;
}

fvr_status fvr_reconstruct(fvr_ctx *c, const fvr_frame *f, fvr_mesh *mesh) {
    fvr_status r = check_frame(c, f);
    if (r != FVR_OK) return r;
    if (!mesh) return fail(c, FVR_E_INVALID, "mesh is NULL");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    Plan *p;
    if ((r = get_plan(c, f, &p)) != FVR_OK) return r;
    if ((r = enqueue_reconstruct(c, f, p, mesh, c->host_status)) != FVR_OK) return r;
    if ((r = sync(c)) != FVR_OK) return r;
    const DevStatus hs = *c->host_status;
    r = finish_mesh(c, hs, mesh, true);
    mesh->level = hs.level;
    return r;
}

fvr_status fvr_reconstruct_noalloc(fvr_ctx *c, const fvr_frame *f, fvr_mesh *mesh) {
    fvr_status r = check_frame(c, f);
    if (r != FVR_OK) return r;
    if (!mesh) return fail(c, FVR_E_INVALID, "mesh is NULL");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    unsigned char *arena = statics_scratch(c->device);
    if (!arena) return fail(c, FVR_E_DEVICE, "static scratch not set up on this device");
    // the plan lives on the stack (no plan-cache insertion), its twiddles in
    // the device's static table
    Plan plan;
    if ((r = build_plan(c, f->dims, plan)) != FVR_OK) return r;
    plan_geometry(&plan, f);
    // arena mode for this call: every scratch buffer is a slice of the static
    // array; timing events (created on first use) are off
    struct ArenaCall {
        fvr_ctx *c;
        uint32_t mask;
        ArenaCall(fvr_ctx *ctx, unsigned char *a) : c(ctx), mask(ctx->timing_mask) {
            c->arena = a;
            c->arena_off = 0;
            ++c->arena_epoch;
            c->timing_mask = 0;
        }
        ~ArenaCall() {
            c->arena = nullptr;
            c->timing_mask = mask;
        }
    } call(c, arena);
    // carve every buffer of the path before anything is enqueued, so a frame
    // beyond the static scratch is refused without side effects
    if ((r = frame_bufs(c, f, &plan, mesh)) != FVR_OK) return r;
    // the same stages as fvr_reconstruct on the carved buffers
    if ((r = enqueue_reconstruct(c, f, &plan, mesh, c->host_status)) != FVR_OK) return r;
    if ((r = sync(c)) != FVR_OK) return r;
    const DevStatus hs = *c->host_status;
    r = finish_mesh(c, hs, mesh, true);
    mesh->level = hs.level;
    return r;
}

fvr_status fvr_indicator(fvr_ctx *c, const fvr_frame *f, float *field_out, double *level_out) {
    fvr_status r = check_frame(c, f);
    if (r != FVR_OK) return r;
    if (!field_out) return fail(c, FVR_E_INVALID, "field_out is NULL");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    Plan *p;
    if ((r = get_plan(c, f, &p)) != FVR_OK) return r;
    const Grid g = frame_grid(f);
    // the transform writes into the context's field first: on invalid input
    // the caller's buffer stays untouched
    GET(c, c->field, sizeof(float) * (size_t)g.n[0] * g.n[1] * g.n[2], "field");
    if ((r = run_field(c, f, p, g, P<float>(c->field), nullptr, false)) != FVR_OK) return r;
    if ((r = run_level(c, f, g, P<float>(c->field))) != FVR_OK) return r;
    HIP_TRY(c, launch_status_publish(P<DevStatus>(c->status), c->host_status, c->stream),
            "status readback");
    if ((r = sync(c)) != FVR_OK) return r;
    if (c->host_status->flags & kFlagInvalid)
        return fail(c, FVR_E_INVALID, "non-finite point, normal or weight, or a negative weight");
    if (c->host_status->flags & kFlagRange) return fail(c, FVR_E_RANGE, kRangeMsg);
    HIP_TRY(c, hipMemcpyAsync(field_out, P<float>(c->field), sizeof(float) * (size_t)g.n[0] * g.n[1] * g.n[2],
                              hipMemcpyDeviceToDevice, c->stream), "field copy");
    if ((r = sync(c)) != FVR_OK) return r;
    if (level_out) *level_out = c->host_status->level;
    return FVR_OK;
}

fvr_status fvr_extract(fvr_ctx *c, const float *field, const int32_t dims[3], const float bbox[6],
                       float level, fvr_mesh *mesh, uint8_t *cases_out) {
    if (!c) return fail(nullptr, FVR_E_INVALID, "context is NULL");
    fvr_status r = check_extract_grid(c, dims, bbox);
    if (r != FVR_OK) return r;
    if (!field || !mesh) return fail(c, FVR_E_INVALID, "field or mesh is NULL");
    if (!std::isfinite(level)) return fail(c, FVR_E_INVALID, "level is not finite");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    const Grid g = make_grid(dims, bbox);
    GET(c, c->status, sizeof(DevStatus), "status");
    GET(c, c->level_f32, sizeof(float), "level");
    { Timed t(c, K_PREP); HIP_TRY(c, launch_prep(P<DevStatus>(c->status), nullptr, 0, c->stream), "prep"); }
    HIP_TRY(c, hipMemcpyAsync(P<float>(c->level_f32), &level, sizeof(float), hipMemcpyHostToDevice, c->stream),
            "level upload");
    r = run_mc(c, g, field, nullptr, mesh, cases_out, false);
    mesh->level = level;
    mesh->n_rejected = 0;
    return r;
}

fvr_status fvr_debug_splat(fvr_ctx *c, const fvr_frame *f, float *v_out) {
    fvr_status r = check_frame(c, f);
    if (r != FVR_OK) return r;
    if (!v_out) return fail(c, FVR_E_INVALID, "v_out is NULL");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    Plan *p;
    if ((r = get_plan(c, f, &p)) != FVR_OK) return r;
    const Grid g = frame_grid(f);
    // the splat writes V only on tiles that some point reaches
    HIP_TRY(c, launch_fill_i32(reinterpret_cast<int32_t *>(v_out), 3 * (int64_t)g.n[0] * g.n[1] * g.n[2], 0,
                               c->stream), "clear v_out");
    if ((r = run_field(c, f, p, g, nullptr, v_out, true)) != FVR_OK) return r;
    HIP_TRY(c, launch_status_publish(P<DevStatus>(c->status), c->host_status, c->stream),
            "status readback");
    if ((r = sync(c)) != FVR_OK) return r;
    if (c->host_status->flags & kFlagInvalid)
        return fail(c, FVR_E_INVALID, "non-finite point, normal or weight, or a negative weight");
    return FVR_OK;
}

}  // extern "C"

// A batch runs several frames as one unit of device work: frame i goes to
// slot i mod S, each slot a context of its own (scratch, status block and a
// stream of default priority), so frames of different slots overlap on the
// device.  The whole batch - a fork from the caller's stream to the slot
// streams, every frame's stages, a join - is captured once into a HIP graph
// and launched as one; a later batch with the same frames, outputs and
// scratch addresses replays the instantiated graph without capturing.
struct fvr_batch {
    int device = 0;
    hipStream_t origin = nullptr;
    hipStream_t own_origin = nullptr;  // made by the batch when the caller gave none
    std::vector<fvr_ctx *> slots;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    DevStatus *host_st = nullptr;  // pinned, one status block per frame
    int host_cap = 0;
    int use_graph = 1;
    std::string err;
    struct Cached {
        std::vector<unsigned char> key;
        hipGraphExec_t exec;
    };
    std::vector<Cached> graphs;  // most recent last
};

namespace {

constexpr size_t kMaxCachedGraphs = 8;

fvr_status bfail(fvr_batch *b, fvr_status s, const std::string &msg) {
    if (b) b->err = msg;
    g_error = msg;
    return s;
}

fvr_status bhip(fvr_batch *b, hipError_t e, const char *what) {
    return bfail(b, e == hipErrorOutOfMemory ? FVR_E_NOMEM : FVR_E_DEVICE,
                 std::string(what) + ": " + hipGetErrorString(e));
}

void drop_graphs(fvr_batch *b) {
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

// Everything a captured graph depends on: the frames and outputs, the
// status array, and the scratch generation of every slot.
std::vector<unsigned char> batch_key(const fvr_batch *b, const fvr_frame *frames, const fvr_mesh *meshes,
                                     int n) {
    std::vector<unsigned char> k;
    auto put = [&](const void *p, size_t len) {
        const unsigned char *q = static_cast<const unsigned char *>(p);
        k.insert(k.end(), q, q + len);
    };
    put(&n, sizeof(n));
    put(&b->host_st, sizeof(b->host_st));
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        put(&g_tune_gen, sizeof(g_tune_gen));
    }
    for (fvr_ctx *c : b->slots) put(&c->scratch_gen, sizeof(c->scratch_gen));
    for (int i = 0; i < n; ++i) {
        put(&frames[i], sizeof(fvr_frame));
        put(&meshes[i].vertices, sizeof(meshes[i].vertices));
        put(&meshes[i].normals, sizeof(meshes[i].normals));
        put(&meshes[i].triangles, sizeof(meshes[i].triangles));
        put(&meshes[i].vertex_capacity, sizeof(int64_t));
        put(&meshes[i].triangle_capacity, sizeof(int64_t));
    }
    return k;
}

// Fork, every frame's stages on its slot's stream, join.
fvr_status batch_enqueue(fvr_batch *b, const fvr_frame *frames, fvr_mesh *meshes, int n,
                         std::vector<Plan> &plans) {
    const int S = (int)b->slots.size();
    hipError_t e = hipEventRecord(b->fork, b->origin);
    if (e != hipSuccess) return bhip(b, e, "batch fork");
    for (int k = 0; k < S && k < n; ++k)
        if ((e = hipStreamWaitEvent(b->slots[k]->stream, b->fork, 0)) != hipSuccess) return bhip(b, e, "batch fork");
    for (int i = 0; i < n; ++i) {
        fvr_ctx *c = b->slots[i % S];
        fvr_status r = enqueue_reconstruct(c, &frames[i], &plans[i], &meshes[i], b->host_st + i);
        if (r != FVR_OK) return bfail(b, r, c->err);
    }
    for (int k = 0; k < S && k < n; ++k) {
        if ((e = hipEventRecord(b->join[k], b->slots[k]->stream)) != hipSuccess) return bhip(b, e, "batch join");
        if ((e = hipStreamWaitEvent(b->origin, b->join[k], 0)) != hipSuccess) return bhip(b, e, "batch join");
    }
    return FVR_OK;
}

}  // namespace

extern "C" {

fvr_status fvr_batch_create(int device, void *hip_stream, int slots, fvr_batch **out) {
    if (!out) return bfail(nullptr, FVR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 64) return bfail(nullptr, FVR_E_INVALID, "slots must be in 1..64");
    fvr_batch *b = new fvr_batch();
    b->device = device;
    b->origin = (hipStream_t)hip_stream;
    for (int k = 0; k < slots; ++k) {
        fvr_ctx *c = nullptr;
        fvr_status r = fvr_create(device, nullptr, &c);
        hipStream_t st = nullptr;
        hipError_t e = r == FVR_OK ? hipStreamCreateWithFlags(&st, hipStreamNonBlocking) : hipSuccess;
        hipEvent_t ev = nullptr;
        if (r == FVR_OK && e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (r != FVR_OK || e != hipSuccess) {
            if (st) (void)hipStreamDestroy(st);
            if (c) fvr_destroy(c);
            fvr_batch_destroy(b);
            return r != FVR_OK ? r : bhip(nullptr, e, "batch stream");
        }
        c->stream = st;
        b->slots.push_back(c);
        b->join.push_back(ev);
    }
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    // the null stream cannot be captured: without a caller stream the batch
    // forks from a stream of its own
    if (e == hipSuccess && !b->origin) {
        e = hipStreamCreateWithFlags(&b->own_origin, hipStreamNonBlocking);
        b->origin = b->own_origin;
    }
    if (e != hipSuccess) {
        fvr_batch_destroy(b);
        return bhip(nullptr, e, "batch event");
    }
    *out = b;
    return FVR_OK;
}

void fvr_batch_destroy(fvr_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    for (fvr_ctx *c : b->slots) (void)hipStreamSynchronize(c->stream);
    drop_graphs(b);
    for (fvr_ctx *c : b->slots) {
        hipStream_t st = c->stream;
        fvr_destroy(c);
        if (st) (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : b->join) (void)hipEventDestroy(ev);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->host_st) (void)hipHostFree(b->host_st);
    if (b->own_origin) (void)hipStreamDestroy(b->own_origin);
    delete b;
}

fvr_status fvr_batch_set_stream(fvr_batch *b, void *hip_stream) {
    if (!b) return bfail(nullptr, FVR_E_INVALID, "batch is NULL");
    b->origin = hip_stream ? (hipStream_t)hip_stream : b->own_origin;
    if (!b->origin) {
        hipError_t e = hipStreamCreateWithFlags(&b->own_origin, hipStreamNonBlocking);
        if (e != hipSuccess) return bhip(b, e, "batch stream");
        b->origin = b->own_origin;
    }
    drop_graphs(b);
    return FVR_OK;
}

fvr_status fvr_batch_use_graph(fvr_batch *b, int enable) {
    if (!b) return bfail(nullptr, FVR_E_INVALID, "batch is NULL");
    b->use_graph = enable ? 1 : 0;
    return FVR_OK;
}

fvr_status fvr_batch_reconstruct(fvr_batch *b, const fvr_frame *frames, fvr_mesh *meshes, int n) {
    if (!b) return bfail(nullptr, FVR_E_INVALID, "batch is NULL");
    if (n < 0 || (n > 0 && (!frames || !meshes))) return bfail(b, FVR_E_INVALID, "frames or meshes is NULL");
    if (n == 0) return FVR_OK;
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return bhip(b, e, "hipSetDevice");
    const int S = (int)b->slots.size();
    // host checks, plans and every slot's scratch, all before any enqueue;
    // each frame keeps its own copy of the plan (frames of one shape may
    // differ in bbox and splat)
    std::vector<Plan> plans((size_t)n);
    for (int i = 0; i < n; ++i) {
        fvr_ctx *c = b->slots[i % S];
        Plan *pp = nullptr;
        fvr_status r = check_frame(c, &frames[i]);
        if (r == FVR_OK) r = get_plan(c, &frames[i], &pp);
        if (r == FVR_OK) {
            plans[i] = *pp;
            r = frame_bufs(c, &frames[i], &plans[i], &meshes[i]);
        }
        if (r != FVR_OK) return bfail(b, r, std::string("frame ") + std::to_string(i) + ": " + c->err);
    }
    if (n > b->host_cap) {
        drop_graphs(b);
        if (b->host_st) (void)hipHostFree(b->host_st);
        b->host_st = nullptr;
        b->host_cap = 0;
        if ((e = hipHostMalloc((void **)&b->host_st, sizeof(DevStatus) * (size_t)n)) != hipSuccess)
            return bhip(b, e, "batch status blocks");
        b->host_cap = n;
    }
    if (b->use_graph) {
        std::vector<unsigned char> key = batch_key(b, frames, meshes, n);
        hipGraphExec_t exec = nullptr;
        for (size_t k = 0; k < b->graphs.size(); ++k)
            if (b->graphs[k].key == key) {
                exec = b->graphs[k].exec;
                std::rotate(b->graphs.begin() + k, b->graphs.begin() + k + 1, b->graphs.end());
                break;
            }
        if (!exec) {
            if ((e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return bhip(b, e, "hipStreamBeginCapture");
            fvr_status r = batch_enqueue(b, frames, meshes, n, plans);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(b->origin, &graph);
            if (r != FVR_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return r;
            }
            if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return bhip(b, e, "hipGraphInstantiate");
            if (b->graphs.size() == kMaxCachedGraphs) {
                (void)hipGraphExecDestroy(b->graphs.front().exec);
                b->graphs.erase(b->graphs.begin());
            }
            b->graphs.push_back({std::move(key), exec});
        }
        if ((e = hipGraphLaunch(exec, b->origin)) != hipSuccess) return bhip(b, e, "hipGraphLaunch");
    } else {
        fvr_status r = batch_enqueue(b, frames, meshes, n, plans);
        if (r != FVR_OK) return r;
    }
    if ((e = hipStreamSynchronize(b->origin)) != hipSuccess) return bhip(b, e, "hipStreamSynchronize");
    // per-frame results; the first error is returned, every mesh is filled
    fvr_status first = FVR_OK;
    for (int i = 0; i < n; ++i) {
        fvr_ctx *c = b->slots[i % S];
        const DevStatus hs = b->host_st[i];
        fvr_status r = finish_mesh(c, hs, &meshes[i], true);
        meshes[i].level = hs.level;
        if (r != FVR_OK && first == FVR_OK) {
            first = r;
            b->err = std::string("frame ") + std::to_string(i) + ": " + c->err;
        }
    }
    if (first != FVR_OK) g_error = b->err;
    return first;
}

const char *fvr_batch_last_error(const fvr_batch *b) { return b ? b->err.c_str() : g_error.c_str(); }

}  // extern "C"

// A serving loop with continuous batching.  Requests (host arrays in, host
// mesh out) queue in arrival order; a request is admitted when a slot is
// free and the device memory the slots would then hold stays within the
// budget.  An admitted request's upload runs on a shared copy stream, its
// stages on the slot's stream (so uploads overlap other slots' compute, and
// frames of different slots overlap each other), and its mesh comes back in
// exactly its size once the counts are known.  Completions are harvested by
// fvr_server_poll, which also admits the waiting requests as slots and
// memory free up.
struct fvr_server {
    int device = 0;
    size_t budget = 0;
    hipStream_t copy = nullptr;
    fvr_ctx *measure = nullptr;  // sizes a frame's scratch (arena arithmetic only)
    struct Slot {
        fvr_ctx *c = nullptr;
        int state = 0;  // 0 free, 1 computing, 2 copying the mesh back
        fvr_request req{};
        uint64_t ticket = 0;
        double t_submit = 0.0, t_admit = 0.0;
        DevBuf d_in, d_verts, d_tris, d_nrm;
        float *h_in = nullptr;
        size_t h_in_cap = 0;
        unsigned char *h_out = nullptr;  // pinned mesh staging
        size_t h_out_cap = 0;
        hipEvent_t h2d = nullptr, done = nullptr;
        fvr_mesh mesh{};
        DevStatus st{};
        fvr_status status = FVR_OK;
    };
    std::vector<Slot> slots;
    struct Pending {
        fvr_request req;
        uint64_t ticket;
        double t_submit;
        size_t scratch;  // the frame's scratch bytes
    };
    std::deque<Pending> pending;
    std::deque<fvr_result> results;
    uint64_t next_ticket = 1;
    int64_t admitted = 0, completed = 0, rejected = 0, max_in_flight = 0;
    std::string err;
};

namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

fvr_status sfail(fvr_server *v, fvr_status st, const std::string &msg) {
    if (v) v->err = msg;
    g_error = msg;
    return st;
}

// Bytes a request needs on the device: its scratch plus inputs and mesh.
size_t io_bytes(const fvr_request &r) {
    const size_t m = (size_t)std::max<int64_t>(r.n_points, 0);
    const size_t v = (size_t)std::max<int64_t>(r.vertex_capacity, 1);
    return align256(28 * m) + align256(12 * v) + align256(12 * (size_t)std::max<int64_t>(r.triangle_capacity, 1)) +
           (r.normals_out ? align256(12 * v) : 0);
}

size_t slot_bytes(fvr_server::Slot &s) {
    return ctx_bytes(s.c) + s.d_in.cap + s.d_verts.cap + s.d_tris.cap + s.d_nrm.cap;
}

// Device bytes slot k would hold after taking a frame of `scratch` + `io`
// bytes (its buffers only grow).
size_t slot_bytes_after(fvr_server::Slot &s, size_t scratch, size_t io) {
    return std::max(ctx_bytes(s.c), scratch) + std::max(s.d_in.cap + s.d_verts.cap + s.d_tris.cap + s.d_nrm.cap, io);
}

// The scratch bytes of a frame: the allocation-free carving arithmetic over
// a dummy base (no memory is touched).
fvr_status frame_scratch_bytes(fvr_server *v, const fvr_frame *f, const fvr_mesh *mesh, size_t *out) {
    fvr_ctx *c = v->measure;
    Plan plan;
    fvr_status r = build_plan(c, f->dims, plan);
    if (r != FVR_OK) return r;
    plan_geometry(&plan, f);
    c->arena = reinterpret_cast<unsigned char *>((uintptr_t)4096);
    c->arena_cap = (size_t)1 << 50;
    c->arena_off = 0;
    ++c->arena_epoch;
    r = frame_bufs(c, f, &plan, mesh);
    c->arena = nullptr;
    c->arena_cap = FVR_NOALLOC_SCRATCH_BYTES;
    *out = c->arena_off;
    return r;
}

fvr_frame device_frame(const fvr_request &q, const float *d_in) {
    fvr_frame f{};
    const size_t m = (size_t)q.n_points;
    f.points = d_in;
    f.normals = d_in + 3 * m;
    f.weights = q.weights ? d_in + 6 * m : nullptr;
    f.n_points = q.n_points;
    std::memcpy(f.dims, q.dims, sizeof(f.dims));
    std::memcpy(f.bbox, q.bbox, sizeof(f.bbox));
    f.options = q.options;
    return f;
}

void push_result(fvr_server *v, const fvr_server::Slot &s, fvr_status st, const std::string &msg) {
    fvr_result r{};
    r.ticket = s.ticket;
    r.status = st;
    r.n_vertices = s.mesh.n_vertices;
    r.n_triangles = s.mesh.n_triangles;
    r.level = s.mesh.level;
    r.n_rejected = s.mesh.n_rejected;
    r.flags = s.mesh.flags;
    r.user = s.req.user;
    r.submit_ms = s.t_submit;
    r.admit_ms = s.t_admit;
    r.done_ms = now_ms();
    std::snprintf(r.error, sizeof(r.error), "%s", msg.c_str());
    v->results.push_back(r);
}

// Upload, enqueue and start one request on slot k.
fvr_status launch_on(fvr_server *v, int k, const fvr_server::Pending &pd) {
    fvr_server::Slot &s = v->slots[k];
    fvr_ctx *c = s.c;
    const fvr_request &q = pd.req;
    const size_t m = (size_t)q.n_points;
    const size_t in_floats = (q.weights ? 7 : 6) * m;
    HIP_TRY(c, ensure(s.d_in, sizeof(float) * std::max<size_t>(in_floats, 1)), "server inputs");
    HIP_TRY(c, ensure(s.d_verts, 12 * (size_t)std::max<int64_t>(q.vertex_capacity, 1)), "server vertices");
    HIP_TRY(c, ensure(s.d_tris, 12 * (size_t)std::max<int64_t>(q.triangle_capacity, 1)), "server triangles");
    if (q.normals_out) HIP_TRY(c, ensure(s.d_nrm, 12 * (size_t)std::max<int64_t>(q.vertex_capacity, 1)), "server normals");
    float *din = static_cast<float *>(s.d_in.p);
    // inputs: straight from the caller's memory when it is pinned, else
    // through the slot's pinned staging
    const float *src[3] = {q.points, q.normals, q.weights};
    const size_t len[3] = {3 * m, 3 * m, q.weights ? m : 0};
    if (!(q.flags & FVR_REQUEST_PINNED) && in_floats > 0) {
        if (s.h_in_cap < in_floats) {
            if (s.h_in) (void)hipHostFree(s.h_in);
            s.h_in = nullptr;
            s.h_in_cap = 0;
            HIP_TRY(c, hipHostMalloc((void **)&s.h_in, sizeof(float) * in_floats), "server staging");
            s.h_in_cap = in_floats;
        }
        size_t o = 0;
        for (int a = 0; a < 3; ++a) {
            if (len[a]) std::memcpy(s.h_in + o, src[a], sizeof(float) * len[a]);
            src[a] = s.h_in + o;
            o += len[a];
        }
    }
    size_t o = 0;
    for (int a = 0; a < 3; ++a) {
        if (len[a])
            HIP_TRY(c, hipMemcpyAsync(din + o, src[a], sizeof(float) * len[a], hipMemcpyHostToDevice, v->copy),
                    "server upload");
        o += len[a];
    }
    HIP_TRY(c, hipEventRecord(s.h2d, v->copy), "server upload event");
    HIP_TRY(c, hipStreamWaitEvent(c->stream, s.h2d, 0), "server upload wait");
    fvr_frame f = device_frame(q, din);
    s.mesh = fvr_mesh{};
    s.mesh.vertices = static_cast<float *>(s.d_verts.p);
    s.mesh.triangles = static_cast<int32_t *>(s.d_tris.p);
    s.mesh.normals = q.normals_out ? static_cast<float *>(s.d_nrm.p) : nullptr;
    s.mesh.vertex_capacity = q.vertex_capacity;
    s.mesh.triangle_capacity = q.triangle_capacity;
    Plan *p = nullptr;
    fvr_status r = get_plan(c, &f, &p);
    if (r == FVR_OK) r = enqueue_reconstruct(c, &f, p, &s.mesh, c->host_status);
    if (r != FVR_OK) return r;
    HIP_TRY(c, hipEventRecord(s.done, c->stream), "server event");
    s.req = q;
    s.ticket = pd.ticket;
    s.t_submit = pd.t_submit;
    s.t_admit = now_ms();
    s.state = 1;
    ++v->admitted;
    return FVR_OK;
}

// Admit waiting requests in arrival order while a slot is free and the
// slots' device memory stays within the budget; a request that cannot fit
// even with every other slot idle is refused.
void admit(fvr_server *v) {
    while (!v->pending.empty()) {
        const fvr_server::Pending &pd = v->pending.front();
        const size_t io = io_bytes(pd.req);
        size_t held = 0;
        int busy = 0;
        for (auto &sl : v->slots) {
            held += slot_bytes(sl);
            busy += sl.state != 0;
        }
        // the free slot that grows least (one already large enough if any)
        int best = -1;
        size_t best_total = 0;
        for (int k = 0; k < (int)v->slots.size(); ++k) {
            fvr_server::Slot &sl = v->slots[k];
            if (sl.state != 0) continue;
            const size_t total = held - slot_bytes(sl) + slot_bytes_after(sl, pd.scratch, io);
            if (best < 0 || total < best_total) {
                best = k;
                best_total = total;
            }
        }
        if (best < 0) return;  // every slot busy
        if (best_total > v->budget) {
            if (busy) return;  // memory frees up as slots finish
            fvr_server::Slot tmp;
            tmp.ticket = pd.ticket;
            tmp.req = pd.req;
            tmp.t_submit = pd.t_submit;
            tmp.t_admit = now_ms();
            push_result(v, tmp, FVR_E_NOMEM, "frame does not fit the server's device-memory budget");
            ++v->rejected;
            v->pending.pop_front();
            continue;
        }
        fvr_status r = launch_on(v, best, pd);
        if (r != FVR_OK) {
            fvr_server::Slot &sl = v->slots[best];
            sl.ticket = pd.ticket;
            sl.req = pd.req;
            sl.t_submit = pd.t_submit;
            push_result(v, sl, r, sl.c->err);
            (void)hipStreamSynchronize(sl.c->stream);
            sl.state = 0;
            ++v->rejected;
        }
        v->pending.pop_front();
        int in_flight = 0;
        for (auto &sl : v->slots) in_flight += sl.state != 0;
        v->max_in_flight = std::max<int64_t>(v->max_in_flight, in_flight);
    }
}

// Advance the slots whose device work finished: counts known -> copy the
// mesh back in its exact size; copy done -> result, slot free.
void harvest(fvr_server *v) {
    for (auto &s : v->slots) {
        if (s.state == 0) continue;
        if (hipEventQuery(s.done) != hipSuccess) continue;
        fvr_ctx *c = s.c;
        if (s.state == 1) {
            s.st = *c->host_status;
            s.status = finish_mesh(c, s.st, &s.mesh, true);
            s.mesh.level = s.st.level;
            if (s.status != FVR_OK) {
                push_result(v, s, s.status, c->err);
                s.state = 0;
                ++v->completed;
                continue;
            }
            const size_t nv = (size_t)s.mesh.n_vertices, nt = (size_t)s.mesh.n_triangles;
            const size_t need = 12 * nv + 12 * nt + (s.req.normals_out ? 12 * nv : 0);
            if (s.h_out_cap < need) {
                if (s.h_out) (void)hipHostFree(s.h_out);
                s.h_out = nullptr;
                s.h_out_cap = 0;
                if (hipHostMalloc((void **)&s.h_out, std::max<size_t>(need, 256)) != hipSuccess) {
                    push_result(v, s, FVR_E_NOMEM, "pinned mesh staging");
                    s.state = 0;
                    ++v->completed;
                    continue;
                }
                s.h_out_cap = std::max<size_t>(need, 256);
            }
            hipError_t e = hipSuccess;
            if (nv) e = hipMemcpyAsync(s.h_out, s.d_verts.p, 12 * nv, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess && nt)
                e = hipMemcpyAsync(s.h_out + 12 * nv, s.d_tris.p, 12 * nt, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess && nv && s.req.normals_out)
                e = hipMemcpyAsync(s.h_out + 12 * (nv + nt), s.d_nrm.p, 12 * nv, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipEventRecord(s.done, c->stream);
            if (e != hipSuccess) {
                push_result(v, s, FVR_E_DEVICE, hipGetErrorString(e));
                s.state = 0;
                ++v->completed;
                continue;
            }
            s.state = 2;
            continue;
        }
        // state 2: the mesh is in pinned memory
        const size_t nv = (size_t)s.mesh.n_vertices, nt = (size_t)s.mesh.n_triangles;
        if (nv) std::memcpy(s.req.vertices, s.h_out, 12 * nv);
        if (nt) std::memcpy(s.req.triangles, s.h_out + 12 * nv, 12 * nt);
        if (nv && s.req.normals_out) std::memcpy(s.req.normals_out, s.h_out + 12 * (nv + nt), 12 * nv);
        push_result(v, s, FVR_OK, "");
        s.state = 0;
        ++v->completed;
    }
}

}  // namespace

extern "C" {

fvr_status fvr_server_create(int device, int slots, size_t hbm_budget, fvr_server **out) {
    if (!out) return sfail(nullptr, FVR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 64) return sfail(nullptr, FVR_E_INVALID, "slots must be in 1..64");
    fvr_server *v = new fvr_server();
    v->device = device;
    v->budget = hbm_budget;
    fvr_status r = fvr_create(device, nullptr, &v->measure);
    hipError_t e = r == FVR_OK ? hipStreamCreateWithFlags(&v->copy, hipStreamNonBlocking) : hipSuccess;
    for (int k = 0; k < slots && r == FVR_OK && e == hipSuccess; ++k) {
        fvr_server::Slot sl;
        r = fvr_create(device, nullptr, &sl.c);
        hipStream_t st = nullptr;
        if (r == FVR_OK) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (r == FVR_OK && e == hipSuccess) e = hipEventCreateWithFlags(&sl.h2d, hipEventDisableTiming);
        if (r == FVR_OK && e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (sl.c) sl.c->stream = st;
        v->slots.push_back(sl);
    }
    if (r != FVR_OK || e != hipSuccess) {
        fvr_server_destroy(v);
        return r != FVR_OK ? r : sfail(nullptr, FVR_E_DEVICE, std::string("server setup: ") + hipGetErrorString(e));
    }
    *out = v;
    return FVR_OK;
}

void fvr_server_destroy(fvr_server *v) {
    if (!v) return;
    (void)hipSetDevice(v->device);
    for (auto &s : v->slots) {
        if (!s.c) continue;
        hipStream_t st = s.c->stream;
        if (st) (void)hipStreamSynchronize(st);
        for (DevBuf *b : {&s.d_in, &s.d_verts, &s.d_tris, &s.d_nrm})
            if (b->p) (void)hipFree(b->p);
        if (s.h_in) (void)hipHostFree(s.h_in);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.h2d) (void)hipEventDestroy(s.h2d);
        if (s.done) (void)hipEventDestroy(s.done);
        fvr_destroy(s.c);
        if (st) (void)hipStreamDestroy(st);
    }
    if (v->copy) {
        (void)hipStreamSynchronize(v->copy);
        (void)hipStreamDestroy(v->copy);
    }
    if (v->measure) fvr_destroy(v->measure);
    delete v;
}

fvr_status fvr_server_submit(fvr_server *v, const fvr_request *q, uint64_t *ticket) {
    if (!v || !q) return sfail(v, FVR_E_INVALID, "server or request is NULL");
    fvr_frame f{};
    f.points = q->points;
    f.normals = q->normals;
    f.weights = q->weights;
    f.n_points = q->n_points;
    std::memcpy(f.dims, q->dims, sizeof(f.dims));
    std::memcpy(f.bbox, q->bbox, sizeof(f.bbox));
    f.options = q->options;
    fvr_status r = check_frame_fields(v->measure, &f);
    if (r != FVR_OK) return sfail(v, r, v->measure->err);
    if (q->vertex_capacity < 0 || q->triangle_capacity < 0 || !q->vertices || !q->triangles)
        return sfail(v, FVR_E_INVALID, "mesh outputs are NULL or capacities negative");
    if (q->flags & ~FVR_REQUEST_PINNED) return sfail(v, FVR_E_INVALID, "unknown request flag bits");
    HIP_TRY(v->measure, hipSetDevice(v->device), "hipSetDevice");
    fvr_mesh mm{};
    mm.vertices = q->vertices;
    mm.triangles = q->triangles;
    mm.vertex_capacity = q->vertex_capacity;
    mm.triangle_capacity = q->triangle_capacity;
    fvr_server::Pending pd{*q, v->next_ticket++, now_ms(), 0};
    if ((r = frame_scratch_bytes(v, &f, &mm, &pd.scratch)) != FVR_OK) return sfail(v, r, v->measure->err);
    if (ticket) *ticket = pd.ticket;
    v->pending.push_back(pd);
    admit(v);
    return FVR_OK;
}

fvr_status fvr_server_poll(fvr_server *v, fvr_result *out, int max_results, int *n_out) {
    if (!v || !n_out || (max_results > 0 && !out)) return sfail(v, FVR_E_INVALID, "bad poll arguments");
    *n_out = 0;
    hipError_t e = hipSetDevice(v->device);
    if (e != hipSuccess) return sfail(v, FVR_E_DEVICE, hipGetErrorString(e));
    harvest(v);
    admit(v);
    harvest(v);  // a copy-back may already have finished
    int n = 0;
    while (n < max_results && !v->results.empty()) {
        out[n++] = v->results.front();
        v->results.pop_front();
    }
    *n_out = n;
    return FVR_OK;
}

fvr_status fvr_server_info(const fvr_server *v, fvr_server_stats *out) {
    if (!v || !out) return sfail(nullptr, FVR_E_INVALID, "server or out is NULL");
    fvr_server_stats st{};
    st.pending = (int64_t)v->pending.size();
    for (const auto &s : v->slots) st.in_flight += s.state != 0;
    st.results_waiting = (int64_t)v->results.size();
    st.admitted = v->admitted;
    st.completed = v->completed;
    st.refused = v->rejected;
    st.max_in_flight = v->max_in_flight;
    fvr_server *w = const_cast<fvr_server *>(v);
    for (auto &s : w->slots) st.device_bytes += slot_bytes(s);
    st.budget = v->budget;
    *out = st;
    return FVR_OK;
}

const char *fvr_server_last_error(const fvr_server *v) { return v ? v->err.c_str() : g_error.c_str(); }

fvr_status fvr_depth_to_points(fvr_ctx *c, const fvr_depth_views *dv, float *points, float *normals,
                               float *weights, int64_t capacity, int64_t *n_points) {
    if (!c) return fail(nullptr, FVR_E_INVALID, "context is NULL");
    if (!dv || !n_points) return fail(c, FVR_E_INVALID, "views or n_points is NULL");
    *n_points = 0;
    if (!dv->depth || !dv->cameras) return fail(c, FVR_E_INVALID, "depth or cameras is NULL");
    if (dv->views < 1 || dv->views > kFeMaxViews) return fail(c, FVR_E_INVALID, "views must be 1..16");
    if (dv->height < 2 || dv->width < 2 || (int64_t)dv->height * dv->width > (1 << 24))
        return fail(c, FVR_E_INVALID, "depth maps must be at least 2 x 2 and at most 2^24 pixels");
    const int64_t npix = (int64_t)dv->views * dv->height * dv->width;
    if (npix > FVR_MAX_POINTS) return fail(c, FVR_E_INVALID, "too many pixels");
    if (!(dv->step_threshold >= 0.0f) || !std::isfinite(dv->step_threshold))
        return fail(c, FVR_E_INVALID, "step_threshold must be finite and >= 0");
    if (dv->box_radius < 0 || dv->box_radius > 1000) return fail(c, FVR_E_INVALID, "box_radius must be 0..1000");
    if (capacity < 0 || (capacity > 0 && (!points || !normals || !weights)))
        return fail(c, FVR_E_INVALID, "output arrays are NULL");
    FeCams cams{};
    for (int k = 0; k < dv->views; ++k)
        for (int j = 0; j < 16; ++j) {
            const float x = dv->cameras[16 * k + j];
            if (!std::isfinite(x)) return fail(c, FVR_E_INVALID, "camera parameters must be finite");
            cams.c[k][j] = x;
        }
    for (int k = 0; k < dv->views; ++k)
        if (cams.c[k][0] == 0.0f || cams.c[k][1] == 0.0f) return fail(c, FVR_E_INVALID, "zero focal length");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    const int n = (int)npix;
    GET(c, c->status, sizeof(DevStatus), "status");
    GET(c, c->fe_rowcnt, sizeof(int32_t) * (size_t)n, "front-end row counts");
    GET(c, c->fe_dense, sizeof(float) * 7 * (size_t)n, "front-end pixels");
    GET(c, c->fe_flag, sizeof(int32_t) * (size_t)n, "front-end flags");
    GET(c, c->fe_off, sizeof(int32_t) * ((size_t)n + 1), "front-end offsets");
    GET(c, c->scan_part, sizeof(int32_t) * (size_t)scan_partials(n), "scan scratch");
    FeParams fp{dv->views, dv->height, dv->width, dv->box_radius, dv->step_threshold};
    DevStatus *st = P<DevStatus>(c->status);
    hipStream_t s = c->stream;
    HIP_TRY(c, launch_prep(st, nullptr, 0, s), "prep");
    HIP_TRY(c, launch_fe_pixels(dv->depth, fp, cams, P<int32_t>(c->fe_rowcnt), P<float>(c->fe_dense),
                                P<int32_t>(c->fe_flag), s), "front end");
    HIP_TRY(c, launch_scan(P<int32_t>(c->fe_flag), P<int32_t>(c->fe_off), n, 1, P<int32_t>(c->scan_part),
                           &st->fe_points, s), "front-end scan");
    HIP_TRY(c, launch_fe_scatter(P<float>(c->fe_dense), P<int32_t>(c->fe_flag), P<int32_t>(c->fe_off), n, st,
                                 capacity, points, normals, weights, s), "front-end scatter");
    HIP_TRY(c, launch_status_publish(st, c->host_status, s), "status readback");
    fvr_status r = sync(c);
    if (r != FVR_OK) return r;
    *n_points = c->host_status->fe_points;
    if (*n_points > capacity) return fail(c, FVR_E_CAPACITY, "point output capacity too small");
    return FVR_OK;
}

fvr_status fvr_last_stats(const fvr_ctx *c, fvr_stats *out) {
    if (!c || !out) return fail(nullptr, FVR_E_INVALID, "context or out is NULL");
    *out = c->last;
    const DevStatus &h = *c->host_status;
    out->busy_tiles = h.n_busy;
    out->nonzero_planes = h.n_zplanes;
    if (out->mc_blocks_listed < 0) out->mc_blocks_listed = h.mc_active;
    out->points_used = h.n_used;
    out->points_rejected = h.rejected;
    return FVR_OK;
}

fvr_status fvr_set_tuning(const int32_t dims[3], const fvr_tuning *t) {
    if (!dims) return fail(nullptr, FVR_E_INVALID, "dims is NULL");
    const float unit_box[6] = {0.f, 0.f, 0.f, 1.f, 1.f, 1.f};
    fvr_status r = check_grid(nullptr, dims, unit_box);
    if (r != FVR_OK) return r;
    const std::array<int, 3> key = {dims[0], dims[1], dims[2]};
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    ++g_tune_gen;
    if (!t) {
        g_tuning.erase(key);
        return FVR_OK;
    }
    Tuning tu{};
    for (int a = 0; a < 3; ++a) {
        const int ns = t->nstages[a];
        if (ns < 0 || ns > kMaxStages) return fail(nullptr, FVR_E_INVALID, "nstages out of range");
        int prod = 1;
        for (int k = 0; k < ns; ++k) {
            const int rad = t->radices[a][k];
            if (rad != 2 && rad != 3 && rad != 4 && rad != 5 && rad != 8)
                return fail(nullptr, FVR_E_INVALID, "radix must be 2, 3, 4, 5 or 8");
            prod *= rad;
            tu.radices[a][k] = rad;
        }
        if (ns > 0 && prod != dims[a]) return fail(nullptr, FVR_E_INVALID, "radices do not multiply to the dim");
        tu.nstages[a] = ns;
    }
    if (t->splat_ty || t->splat_tz) {
        if (!splat_tile_ok(dims[0], t->splat_ty, t->splat_tz))
            return fail(nullptr, FVR_E_INVALID, "splat tile does not fit the kernel");
        tu.splat_ty = t->splat_ty;
        tu.splat_tz = t->splat_tz;
    }
    g_tuning[key] = tu;
    return FVR_OK;
}

fvr_status fvr_get_tuning(const int32_t dims[3], fvr_tuning *t) {
    if (!dims || !t) return fail(nullptr, FVR_E_INVALID, "dims or out is NULL");
    const float unit_box[6] = {0.f, 0.f, 0.f, 1.f, 1.f, 1.f};
    fvr_status r = check_grid(nullptr, dims, unit_box);
    if (r != FVR_OK) return r;
    // the plan's parameters: tuned where set, the defaults otherwise
    std::memset(t, 0, sizeof(*t));
    for (int a = 0; a < 3; ++a) {
        int rr[kMaxStages], ns;
        factor(dims[a], rr, ns);
        t->nstages[a] = ns;
        for (int k = 0; k < ns; ++k) t->radices[a][k] = rr[k];
    }
    default_splat_tile(dims[0], t->splat_ty, t->splat_tz);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tuning.find({dims[0], dims[1], dims[2]});
    if (it != g_tuning.end()) {
        const Tuning &tu = it->second;
        for (int a = 0; a < 3; ++a)
            if (tu.nstages[a] > 0) {
                t->nstages[a] = tu.nstages[a];
                for (int k = 0; k < tu.nstages[a]; ++k) t->radices[a][k] = tu.radices[a][k];
            }
        if (tu.splat_ty > 0) {
            t->splat_ty = tu.splat_ty;
            t->splat_tz = tu.splat_tz;
        }
    }
    return FVR_OK;
}

fvr_status fvr_check_frame(const fvr_frame *frame) {
    return check_frame_fields(nullptr, frame);
}

fvr_status fvr_check_grid(const int32_t dims[3], const float bbox[6]) {
    return check_grid(nullptr, dims, bbox);
}

fvr_status fvr_mc_table(uint8_t counts[256], int8_t edges[256 * 15]) {
    if (!counts || !edges) return fail(nullptr, FVR_E_INVALID, "NULL output");
    try {
        mc_generate_table(counts, edges);
    } catch (const std::exception &ex) {
        return fail(nullptr, FVR_E_DEVICE, std::string("mc table: ") + ex.what());
    }
    return FVR_OK;
}

fvr_status fvr_timing_enable(fvr_ctx *c, int enable) {
    if (!c) return fail(nullptr, FVR_E_INVALID, "context is NULL");
    c->timing_mask = enable ? (1u << K_COUNT) - 1u : 0u;
    return FVR_OK;
}

fvr_status fvr_timing_select(fvr_ctx *c, uint32_t mask) {
    if (!c) return fail(nullptr, FVR_E_INVALID, "context is NULL");
    c->timing_mask = mask & ((1u << K_COUNT) - 1u);
    return FVR_OK;
}

fvr_status fvr_timing_reset(fvr_ctx *c) {
    if (!c) return fail(nullptr, FVR_E_INVALID, "context is NULL");
    for (int i = 0; i < K_COUNT; ++i) {
        c->t_ms[i] = 0.0;
        c->t_n[i] = 0;
    }
    return FVR_OK;
}

int fvr_timing_count(void) { return K_COUNT; }

const char *fvr_timing_name(int i) { return (i >= 0 && i < K_COUNT) ? kKernelNames[i] : nullptr; }

fvr_status fvr_timing_get(const fvr_ctx *c, int i, double *total_ms, int64_t *launches) {
    if (!c || i < 0 || i >= K_COUNT) return fail(nullptr, FVR_E_INVALID, "bad context or index");
    if (total_ms) *total_ms = c->t_ms[i];
    if (launches) *launches = c->t_n[i];
    return FVR_OK;
}

const char *fvr_status_string(fvr_status s) {
    switch (s) {
        case FVR_OK: return "ok";
        case FVR_E_INVALID: return "invalid argument";
        case FVR_E_UNSUPPORTED: return "unsupported grid";
        case FVR_E_NOMEM: return "out of device memory";
        case FVR_E_CAPACITY: return "output capacity too small";
        case FVR_E_DEVICE: return "device error";
        case FVR_E_RANGE: return "16-bit spectrum overflow";
        default: break;
    }
    return "unknown status";
}

const char *fvr_last_error(const fvr_ctx *c) { return c ? c->err.c_str() : g_error.c_str(); }

}  // extern "C"
