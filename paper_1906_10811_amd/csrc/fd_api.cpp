// fd_api.cpp -- host side of libfd: descriptors, workspace layout, sparse
// tables, and the time loops of fd_forward / fd_adjoint / fd_gradient.
//
// The time loop runs on the host and enqueues one fused step kernel per time
// step (the thesis keeps the time loop on the host and offloads the space
// loop, Section 3.3.2 "TimeFunction"; the two time levels the update needs
// rotate through two buffers, the n = 2 case of its t_k = (time + k) mod n
// rotation, with the new level written over the oldest one in place).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fd.h"
#include "fd_api_internal.h"
#include "fd_internal.h"

using namespace fd;

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string t_err;
}

int fdi_fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

extern "C" const char *fd_last_error(void) { return t_err.c_str(); }

#define HIPCHK(x)                                                                       \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess)                                                           \
            return fdi_fail(FD_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e_));       \
    } while (0)

#define API_GUARD_BEGIN try {
#define API_GUARD_END                                                                   \
    }                                                                                   \
    catch (const std::bad_alloc &) {                                                    \
        return fdi_fail(FD_ERR_NOMEM, "host allocation failed");                        \
    }                                                                                   \
    catch (...) {                                                                       \
        return fdi_fail(FD_ERR_STATE, "internal error");                                \
    }

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int round_up(int v, int a) { return (v + a - 1) / a * a; }

}  // namespace

// Maximal-order central second-derivative weights, radius r:
// c_j = 2 (-1)^(j+1) (r!)^2 / (j^2 (r-j)! (r+j)!), c_0 = -2 sum c_j.
// All factorials up to 16! are exact in double.
void fdi_second_derivative_weights(int r, double *c) {
    auto fact = [](int n) {
        double f = 1.0;
        for (int i = 2; i <= n; ++i) f *= i;
        return f;
    };
    double sum = 0.0;
    for (int j = 1; j <= r; ++j) {
        const double sgn = (j % 2 == 1) ? 1.0 : -1.0;
        c[j] = 2.0 * sgn * fact(r) * fact(r) / ((double)j * j * fact(r - j) * fact(r + j));
        sum += c[j];
    }
    c[0] = -2.0 * sum;
}

// ----------------------------------------------------------- grid plumbing
bool fdi_check_desc(const fd_grid_desc *d) {
    if (!d) return fdi_fail(FD_ERR_ARG, "null descriptor"), false;
    if (d->ndim != 2 && d->ndim != 3) return fdi_fail(FD_ERR_ARG, "ndim must be 2 or 3"), false;
    for (int a = 0; a < d->ndim; ++a) {
        if (d->shape[a] < 2) return fdi_fail(FD_ERR_ARG, "shape[%d] < 2", a), false;
        if (!(d->spacing[a] > 0.0) || !std::isfinite(d->spacing[a]))
            return fdi_fail(FD_ERR_ARG, "spacing[%d] must be > 0", a), false;
        if (!std::isfinite(d->origin[a])) return fdi_fail(FD_ERR_ARG, "origin[%d]", a), false;
    }
    if (d->space_order < 2 || d->space_order > 2 * kMaxR || d->space_order % 2)
        return fdi_fail(FD_ERR_ARG, "space_order must be even, 2..16"), false;
    if (d->nbl < 0) return fdi_fail(FD_ERR_ARG, "nbl < 0"), false;
    if (d->storage < 0 || d->storage > 4) return fdi_fail(FD_ERR_ARG, "storage"), false;
    if ((d->storage == FD_STORE_F16_DIFF || d->storage == FD_STORE_BF16_DIFF) && d->ndim != 3)
        return fdi_fail(FD_ERR_ARG, "the difference storages are 3D only"), false;
    if (d->amp_scale < 0.f || !std::isfinite(d->amp_scale)) return fdi_fail(FD_ERR_ARG, "amp_scale"), false;
    if (d->max_src < 0 || d->max_rec < 0 || d->zchunk < 0) return fdi_fail(FD_ERR_ARG, "capacities"), false;
    if (d->tile_x != 0 && d->tile_x != 32 && d->tile_x != 64 && d->tile_x != 96)
        return fdi_fail(FD_ERR_ARG, "tile_x must be 0, 32, 64 or 96"), false;
    if (d->sinc_radius < 0 || d->sinc_radius > kMaxSincR)
        return fdi_fail(FD_ERR_ARG, "sinc_radius must be 0..%d", kMaxSincR), false;
    if (!std::isfinite(d->sinc_beta)) return fdi_fail(FD_ERR_ARG, "sinc_beta"), false;
    if (d->time_block < 0 || d->time_block > 2) return fdi_fail(FD_ERR_ARG, "time_block must be 0, 1 or 2"), false;
    if (d->param_storage != FD_PARAM_F32 && d->param_storage != FD_PARAM_Q16)
        return fdi_fail(FD_ERR_ARG, "param_storage must be FD_PARAM_F32 or FD_PARAM_Q16"), false;
    if (d->param_storage == FD_PARAM_Q16 && d->ndim != 3)
        return fdi_fail(FD_ERR_ARG, "the 16-bit p code is 3D only"), false;
    if (d->time_block == 2 && !(d->ndim == 3 && d->storage == FD_STORE_F32 && d->space_order <= 2 * kT2MaxR &&
                                d->param_storage == FD_PARAM_F32))
        return fdi_fail(FD_ERR_ARG, "time_block 2 needs a 3D float32 grid of space order <= %d with float32 p",
                        2 * kT2MaxR),
               false;
    long long pts = 1;
    for (int a = 0; a < d->ndim; ++a) pts *= (long long)d->shape[a] + 2LL * d->nbl;
    if (pts > (1LL << 34)) return fdi_fail(FD_ERR_ARG, "grid too large"), false;
    return true;
}

Layout fdi_layout(const fd_grid_desc *d) {
    Layout L{};
    const int r = d->space_order / 2;
    L.ndim = d->ndim;
    L.r = r;
    L.nx = d->shape[0] + 2 * d->nbl;
    if (d->ndim == 3) {
        L.ny = d->shape[1] + 2 * d->nbl;
        L.nz = d->shape[2] + 2 * d->nbl;
        L.yh = r;
    } else {
        L.ny = 1;
        L.nz = d->shape[1] + 2 * d->nbl;
        L.yh = 0;
    }
    L.pitch = round_up(kXOff + round_up(L.nx, 4) + 8, 64);
    L.nya = L.ny + 2 * L.yh;
    L.nza = L.nz + 2 * r;
    L.plane = (long long)L.pitch * L.nya;
    L.elems = L.plane * L.nza;
    return L;
}

namespace {

struct SparseDev {   // device tables of one side (sources or receivers)
    int cap = 0;     // points
    long long *idx = nullptr;
    float *w = nullptr;
    int *plane_ptr = nullptr;
    int4 *corner = nullptr;
    int *ent_src = nullptr;
    float *ent_w = nullptr;
    size_t stage_off = 0;    // offset of this side's area in the host staging buffer
};

struct WsPlan {
    size_t vel, p, uA, uB, uC, uD, damp, misc, total;
    size_t t2pp, t2corner;   // extended source tables of the two-level step (0 when unused)
    size_t stage_t2;         // their host staging area
    size_t src[6], rec[6];   // idx, w, plane_ptr, corner, ent_src, ent_w
    size_t field_bytes;
    int cap_src, cap_rec;
    size_t stage_bytes, stage_damp, stage_src, stage_rec, stage_side_bytes_src, stage_side_bytes_rec;
};

constexpr int kNPart = 512;   // misfit partial sums
constexpr int kFoldEvery = 32;   // adjoint steps per float32 partial gradient sum

size_t side_bytes(int cap, int nc, size_t nptr, size_t off[6], size_t base) {
    size_t o = base;
    off[0] = o; o = align_up(o + sizeof(long long) * (size_t)cap * nc, 256);
    off[1] = o; o = align_up(o + sizeof(float) * (size_t)cap * nc, 256);
    off[2] = o; o = align_up(o + sizeof(int) * nptr, 256);
    off[3] = o; o = align_up(o + sizeof(int4) * (size_t)cap * nc, 256);
    off[4] = o; o = align_up(o + sizeof(int) * (size_t)cap * nc, 256);
    off[5] = o; o = align_up(o + sizeof(float) * (size_t)cap * nc, 256);
    return o - base;
}

// Grid points one sparse point touches: the 2^d cell corners, or (2r)^d
// windowed-sinc nodes.
int sparse_nodes(const fd_grid_desc *d) {
    if (d->sinc_radius == 0) return 1 << d->ndim;
    int n = 1;
    for (int a = 0; a < d->ndim; ++a) n *= 2 * d->sinc_radius;
    return n;
}

// Width of the 3D step tiles in float4 columns: 16 (64 x 16 points) or 8
// (32 x 32).  The 32 x 32 shape stages 2r halo rows per 32 rows instead of
// per 16, but each row of its x halo is one more cache-line request.
// Measured (336^3 and 280^3, every even order): 64 x 16 is faster up to so 8
// (by 3-11 %), 32 x 32 from so 14 on (by 4-16 %, 25 % in 16-bit at 280^3);
// at so 10 and 12 the 32 x 32 shape wins only where 64-point rows leave many
// lanes idle (280 = 4.375 x 64: +2 %, 16-bit +4-6 %; 336 = 5.25 x 64: -3 %).
// A ragged last x column of at most 32 points fills a 64 x 16 tile's lanes
// to half or less; the mixed shape gives that column 32 x 32 tiles instead.
// Measured, float32 (against 64 x 16 everywhere): 280^3 +7 % at so 4, +9 %
// at so 8, +10 % at so 12 (also 10 % above 32 x 32 tiles there), 336^3
// +1 %, 592^3 +2.5 %.  With 16-bit fields a 32-point row is half a cache
// line and the mixed shape lost 7-10 %, so 16-bit grids keep 64 x 16.
constexpr double kTileNarrowGain = 0.06;   // lane-use margin that selects 32 x 32 at so 10, 12

bool mixed_fits(const Layout &L) { return L.nx > 64 && L.nx % 64 != 0 && L.nx % 64 <= 32; }

// Whether fd_forward runs two leapfrog levels per launch (k_step3d_t2).
// Its recomputed ring grows with the radius: 16 % of a 64 x 16 tile at
// radius 1, 69 % at radius 4.  Measured (float32, 400 steps), two levels
// against one step per launch: so 2 on 336^3 427 vs 386 Gpts/s and on 280^3
// 408 vs 365; so 4 401 vs 383 and 340 vs 360; so 6 349 vs 378 and 295 vs
// 354; so 8 313 vs 372 and 267 vs 347.  So the automatic choice takes two
// levels at space order 2 and one step elsewhere.
bool t2_enabled(const fd_grid_desc *d) {
    const bool avail = d->ndim == 3 && d->storage == FD_STORE_F32 && d->space_order <= 2 * kT2MaxR &&
                       d->param_storage == FD_PARAM_F32;
    return avail && (d->time_block == 2 || (d->time_block == 0 && d->space_order == 2));
}

// 16-bit value-and-difference storage, and the element type of a storage.
inline bool diff_storage(const fd_grid_desc *d) {
    return d->storage == FD_STORE_F16_DIFF || d->storage == FD_STORE_BF16_DIFF;
}
inline Store elem_store(int storage) {
    return storage == FD_STORE_F32 ? Store::F32
           : (storage == FD_STORE_F16 || storage == FD_STORE_F16_DIFF) ? Store::F16
                                                                        : Store::BF16;
}

// Tiles of the two-level step: 64 x 16 whatever the one-step shape.
inline int t2_ntx(const Layout &L) { return (L.nx + 63) / 64; }
inline int t2_nty(const Layout &L) { return (L.ny + 15) / 16; }

// Tile shape code of a grid (16, 8 or kShapeMixed; 2D grids: 16).
int tile_shape(const fd_grid_desc *d, const Layout &L) {
    if (L.ndim != 3) return 16;
    if (d->tile_x == 64) return 16;
    if (d->tile_x == 32) return 8;
    if (L.r >= 7) return 8;   // no mixed kernel at so 14, 16
    if (d->tile_x == 96) return mixed_fits(L) ? kShapeMixed : 16;
    if (d->storage == FD_STORE_F32 && mixed_fits(L)) return kShapeMixed;
    auto used = [&](int tw4) {   // fraction of tile lanes that hold a grid point
        const double tx = tile3_x(tw4), ty = tile3_y(tw4);
        return (double)L.nx * L.ny / (std::ceil(L.nx / tx) * tx * std::ceil(L.ny / ty) * ty);
    };
    return L.r >= 5 && used(8) > used(16) + kTileNarrowGain ? 8 : 16;
}

struct TileGrid {
    int ntx, nty, nstrip;   // 64 x 16 (or single-shape) tiles per axis; 32 x 32 tiles of the last column
    int tiles() const { return ntx * nty + nstrip; }
};

// Tiles of the step kernels' xy (3D) or x (2D) decomposition; the injection
// tables keep one plane-pointer row per tile.
TileGrid tile_grid(const Layout &L, int shape) {
    TileGrid t{};
    if (L.ndim != 3) {
        t.ntx = (L.nx + kTileX - 1) / kTileX;
        t.nty = 1;
    } else if (shape == kShapeMixed) {
        t.ntx = L.nx / 64;
        t.nty = (L.ny + 15) / 16;
        t.nstrip = (L.ny + 31) / 32;
    } else {
        t.ntx = (L.nx + tile3_x(shape) - 1) / tile3_x(shape);
        t.nty = (L.ny + tile3_y(shape) - 1) / tile3_y(shape);
    }
    return t;
}

WsPlan plan(const fd_grid_desc *d, const Layout &L) {
    WsPlan w{};
    const size_t esz = d->storage == FD_STORE_F32 ? 4 : 2;
    const int nc = sparse_nodes(d);
    const size_t nptr = (size_t)tile_grid(L, tile_shape(d, L)).tiles() * (L.nz + 1);
    w.cap_src = d->max_src ? d->max_src : 64;
    w.cap_rec = d->max_rec ? d->max_rec : 4096;
    w.field_bytes = align_up((size_t)L.elems * esz, 256);
    const size_t f32 = align_up((size_t)L.elems * 4, 256);
    size_t o = 0;
    w.vel = o; o += f32;
    w.p = o; o += d->param_storage == FD_PARAM_Q16 ? align_up((size_t)L.elems * 2, 256) : f32;
    w.uA = o; o += w.field_bytes;
    w.uB = o; o += w.field_bytes;
    const bool t2 = t2_enabled(d);
    w.uC = o; if (t2 || diff_storage(d)) o += w.field_bytes;   // (the difference field)
    w.uD = o; if (t2) o += w.field_bytes;
    w.damp = o; o = align_up(o + sizeof(float) * (size_t)(L.nx + L.ny + L.nz), 256);
    w.misc = o; o = align_up(o + sizeof(double) * kNPart + 256, 256);
    o += side_bytes(w.cap_src, nc, nptr, w.src, o);
    o += side_bytes(w.cap_rec, nc, nptr, w.rec, o);
    // two-level step: per 64 x 16 tile, the source grid points of the tile
    // grown by its ring (a point lies in at most 4 grown tiles)
    const size_t t2ptr = t2 ? (size_t)t2_ntx(L) * t2_nty(L) * (L.nz + 1) : 0;
    const size_t t2cor = t2 ? (size_t)4 * w.cap_src * nc : 0;
    w.t2pp = o; o = align_up(o + sizeof(int) * t2ptr, 256);
    w.t2corner = o; o = align_up(o + sizeof(int4) * t2cor, 256);
    w.total = o;
    // host staging mirrors the uploaded regions
    size_t s = 0;
    w.stage_damp = s; s = align_up(s + sizeof(float) * (size_t)(L.nx + L.ny + L.nz), 256);
    w.stage_src = s;
    w.stage_side_bytes_src = w.src[5] + align_up(sizeof(float) * (size_t)w.cap_src * nc, 256) - w.src[0];
    s += w.stage_side_bytes_src;
    w.stage_rec = s;
    w.stage_side_bytes_rec = w.rec[5] + align_up(sizeof(float) * (size_t)w.cap_rec * nc, 256) - w.rec[0];
    s += w.stage_side_bytes_rec;
    w.stage_t2 = s;
    s += w.total - w.t2pp;
    w.stage_bytes = s;
    return w;
}

}  // namespace

struct fd_grid {
    fd_grid_desc d;
    int device;
    Layout L;
    Store st;
    float amp;
    int nc;
    double c[kMaxR + 1];
    double cell;           // prod(h)
    char *ws;
    size_t ws_bytes;
    WsPlan wp;
    float *vel, *p, *damp;
    uint16_t *pq;          // FD_PARAM_Q16: the codes of p (p is then null)
    float pq_base, pq_step;
    void *uA, *uB;
    double *partials;
    unsigned *vmax_bits;   // [0] max, [1] min of v (bits)
    SparseDev sd[2];       // 0 = sources, 1 = receivers
    std::vector<double> cached_xyz[2];
    int cached_n[2];
    int ncorner[2];        // injection corners in the current tables
    double vmax, vmin, dt_crit, sigma_max;
    double dt_cached;
    char *stage;
    hipEvent_t stage_ev;
    bool stage_pending;
    int ntx, nty;
    int shape3;              // 3D tile shape code (16, 8 or kShapeMixed)
    int nstrip;              // mixed shape: 32 x 32 tiles of the last x column
    int ntz[3], zchunk[3];   // per step mode (kPlain, kBracket, kImage)
    hipStream_t last_stream;   // stream of the latest enqueued work
    bool has_last_stream;
    bool auto_amp;             // F16 storage with the scale chosen per dt
    // forward state: u^n in cur, u^{n-1} in prev (two of uA..uD); rows of
    // the traces sampled so far in the current run
    void *cur, *prev;
    int rows_done;
    // two-level step
    bool t2;
    void *uC, *uD;
    bool diff;               // 16-bit value and difference: the difference lives in uC
    int t2_ntz, t2_zchunk;
    int *t2_pp;
    int4 *t2_corner;
    int t2_ncorner;
};

namespace {

// ------------------------------------------------------------- staging
int stage_acquire(fd_grid *g) {
    if (g->stage_pending) {
        HIPCHK(hipEventSynchronize(g->stage_ev));
        g->stage_pending = false;
    }
    return FD_OK;
}

int stage_release(fd_grid *g, hipStream_t s) {
    HIPCHK(hipEventRecord(g->stage_ev, s));
    g->stage_pending = true;
    return FD_OK;
}

inline void note_stream(fd_grid *g, hipStream_t s) {
    g->last_stream = s;
    g->has_last_stream = true;
}

// Damping tables sigma_a(i) dt / 2 = damp_max (d_a/nbl)^2 dt / 2 and p = dt^2 v^2.
// F16 storage without a caller scale: the stored field is 2^k u with 2^k
// about prod(h) / (dt^2 v_max^2), the inverse of what a unit source puts in
// its cell in one step, so near-source values sit near 1 and the far field
// stays in half precision's normal range (>= 6.1e-5) down to 1e-4 of that.
int ensure_dt(fd_grid *g, double dt, hipStream_t s) {
    if (g->dt_cached == dt) return FD_OK;
    if (g->auto_amp)
        g->amp = (float)std::exp2(std::round(std::log2(g->cell / (dt * dt * g->vmax * g->vmax))));
    const Layout &L = g->L;
    int rc = stage_acquire(g);
    if (rc) return rc;
    float *tab = (float *)(g->stage + g->wp.stage_damp);
    const int n[3] = {L.nx, L.ny, L.nz};
    const int phys[3] = {g->d.shape[0], g->d.ndim == 3 ? g->d.shape[1] : 1,
                         g->d.ndim == 3 ? g->d.shape[2] : g->d.shape[1]};
    int o = 0;
    for (int a = 0; a < 3; ++a) {
        const bool has_layer = !(a == 1 && g->d.ndim == 2) && g->d.nbl > 0;
        for (int i = 0; i < n[a]; ++i) {
            double v = 0.0;
            if (has_layer) {
                const int nbl = g->d.nbl;
                const int dist = std::max(0, std::max(nbl - i, i - (nbl + phys[a] - 1)));
                const double q = (double)dist / nbl;
                v = g->sigma_max * q * q * dt / 2.0;
            }
            tab[o++] = (float)v;
        }
    }
    HIPCHK(hipMemcpyAsync(g->damp, tab, sizeof(float) * o, hipMemcpyHostToDevice, s));
    rc = stage_release(g, s);
    if (rc) return rc;
    if (g->pq) {
        // p0 = dt^2 v_min^2 and dp = (dt^2 v_max^2 - p0) / 65535 as the
        // float32 values the step decodes with
        const double dt2 = dt * dt;
        const double pmin = dt2 * g->vmin * g->vmin, pmax = dt2 * g->vmax * g->vmax;
        g->pq_base = (float)pmin;
        g->pq_step = (float)((pmax - pmin) / 65535.0);
        HIPCHK(launch_make_pq(L, g->vel, dt, g->pq_base, g->pq_step, g->pq, s));
    } else {
        HIPCHK(launch_make_p(L, g->vel, dt, g->p, s));
    }
    g->dt_cached = dt;
    return FD_OK;
}

constexpr double kPi = 3.14159265358979323846;

// Modified Bessel function I0 by its power series sum_k ((x/2)^k / k!)^2
// (all terms positive; x <= ~40 here).
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500 && term > 1e-18 * sum; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
    }
    return sum;
}

// Interpolation weights of one point along one axis at fractional grid
// position t (0 <= t <= n-1): multilinear (2 nodes, cell n-2 for a point on
// the last line) or Kaiser-windowed sinc of half-width r (2r nodes from
// floor(t) - r + 1; Hicks 2002).
struct AxisWeights {
    int k0, n;
    double w[2 * kMaxSincR];
};

void axis_weights(double t, int n, int r, double beta, AxisWeights &o) {
    if (r == 0) {
        int k = (int)std::floor(t);
        if (k >= n - 1) k = n - 2;
        const double p = t - k;
        o.k0 = k;
        o.n = 2;
        o.w[0] = 1.0 - p;
        o.w[1] = p;
        return;
    }
    const double b = beta > 0.0 ? beta : kPi * r / 2.0;
    const double i0b = bessel_i0(b);
    o.k0 = (int)std::floor(t) - r + 1;
    o.n = 2 * r;
    for (int i = 0; i < o.n; ++i) {
        const double d = (double)(o.k0 + i) - t;   // signed distance in cells
        double sinc;
        if (d == std::round(d))
            sinc = d == 0.0 ? 1.0 : 0.0;            // exact at the integers
        else
            sinc = std::sin(kPi * d) / (kPi * d);
        const double u = 1.0 - (d / r) * (d / r);
        o.w[i] = u >= 0.0 ? sinc * bessel_i0(b * std::sqrt(u)) / i0b : 0.0;
    }
}

// Sparse tables of one side from host coordinates: the weights of the nodes
// each point touches (tensor product of axis_weights; nodes outside the
// padded grid dropped), pitched offsets for sampling (a dropped node points
// at the zero column with weight 0), and the per-tile, per-plane CSR of the
// distinct non-zero-weight nodes for injection.
int ensure_side(fd_grid *g, int side, int npts, const double *xyz, hipStream_t s) {
    const int ndim = g->d.ndim;
    const int cap = side == 0 ? g->wp.cap_src : g->wp.cap_rec;
    if (npts < 0) return fdi_fail(FD_ERR_ARG, "%s count must be >= 0", side ? "receiver" : "source");
    if (npts > cap)
        return fdi_fail(FD_ERR_ARG, "%d %s exceed the grid's capacity %d", npts,
                        side ? "receivers" : "sources", cap);
    if (npts > 0 && !xyz) return fdi_fail(FD_ERR_ARG, "null coordinates");
    std::vector<double> key;   // (no points: empty tables, nothing injected or sampled)
    if (npts > 0) key.assign(xyz, xyz + (size_t)npts * ndim);
    if (g->cached_n[side] == npts && g->cached_xyz[side] == key) return FD_OK;

    const Layout &L = g->L;
    const int nc = g->nc;
    const int padded[3] = {L.nx, ndim == 3 ? L.ny : L.nz, L.nz};
    const long long zcol = L.offset((L.nx + 3) & ~3, 0, 0);
    std::vector<long long> idx((size_t)npts * nc);
    std::vector<float> w((size_t)npts * nc);
    struct Ent { int tile, z, y, x, pt; float w; };
    std::vector<Ent> ents;
    ents.reserve((size_t)npts * nc);
    AxisWeights aw[3];
    for (int p = 0; p < npts; ++p) {
        for (int a = 0; a < ndim; ++a) {
            const double t = (xyz[(size_t)p * ndim + a] - g->d.origin[a]) / g->d.spacing[a];
            if (!(t >= 0.0 && t <= (double)(g->d.shape[a] - 1)))
                return fdi_fail(FD_ERR_ARG, "%s %d outside the grid along axis %d",
                                side ? "receiver" : "source", p, a);
            axis_weights(t, g->d.shape[a], g->d.sinc_radius, g->d.sinc_beta, aw[a]);
        }
        const int per = aw[0].n;   // nodes per axis
        for (int c = 0; c < nc; ++c) {
            int ix[3] = {0, 0, 0};
            double wt = 1.0;
            bool inside = true;
            int rem = c;
            for (int a = 0; a < ndim; ++a) {
                const int k = rem % per;
                rem /= per;
                ix[a] = aw[a].k0 + k + g->d.nbl;
                wt *= aw[a].w[k];
                if (ix[a] < 0 || ix[a] >= padded[a]) inside = false;
            }
            const size_t slot = (size_t)p * nc + c;
            if (!inside) {
                idx[slot] = zcol;
                w[slot] = 0.f;
                continue;
            }
            int x = ix[0], y = 0, z = 0;
            if (ndim == 3) { y = ix[1]; z = ix[2]; } else { z = ix[1]; }
            idx[slot] = L.offset(x, y, z);
            w[slot] = (float)wt;
            int tile;
            if (ndim != 3)
                tile = x / kTileX;
            else if (g->shape3 == kShapeMixed)
                tile = x < g->ntx * 64 ? (y / 16) * g->ntx + x / 64 : g->ntx * g->nty + y / 32;
            else
                tile = (y / tile3_y(g->shape3)) * g->ntx + x / tile3_x(g->shape3);
            if ((float)wt != 0.f) ents.push_back({tile, z, y, x, p, (float)wt});
        }
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Ent &a, const Ent &b) {
        if (a.tile != b.tile) return a.tile < b.tile;
        if (a.z != b.z) return a.z < b.z;
        if (a.y != b.y) return a.y < b.y;
        if (a.x != b.x) return a.x < b.x;
        return a.pt < b.pt;
    });
    // distinct grid points (corners) and their contributing entries
    std::vector<int4> corners;
    std::vector<long long> ckey;   // tile * (nz + 1) + z of each corner
    std::vector<int> esrc;
    std::vector<float> ew;
    for (size_t i = 0; i < ents.size();) {
        size_t j = i;
        const int beg = (int)esrc.size();
        while (j < ents.size() && ents[j].tile == ents[i].tile && ents[j].z == ents[i].z &&
               ents[j].y == ents[i].y && ents[j].x == ents[i].x) {
            esrc.push_back(ents[j].pt);
            ew.push_back(ents[j].w);
            ++j;
        }
        corners.push_back(make_int4(ents[i].x, ents[i].y, beg, (int)esrc.size()));
        ckey.push_back((long long)ents[i].tile * (L.nz + 1) + ents[i].z);
        i = j;
    }
    // plane pointers of every tile: pptr[k] = first corner with key >= k
    const size_t nptr = (size_t)(g->ntx * g->nty + g->nstrip) * (L.nz + 1);
    std::vector<int> pptr(nptr, 0);
    {
        size_t c = 0;
        for (size_t k = 0; k < nptr; ++k) {
            while (c < ckey.size() && ckey[c] < (long long)k) ++c;
            pptr[k] = (int)c;
        }
    }

    int rc = stage_acquire(g);
    if (rc) return rc;
    const size_t *off = side == 0 ? g->wp.src : g->wp.rec;
    char *st = g->stage + (side == 0 ? g->wp.stage_src : g->wp.stage_rec);
    const size_t base = off[0];
    if (!idx.empty()) {
        memcpy(st + (off[0] - base), idx.data(), sizeof(long long) * idx.size());
        memcpy(st + (off[1] - base), w.data(), sizeof(float) * w.size());
    }
    memcpy(st + (off[2] - base), pptr.data(), sizeof(int) * pptr.size());
    if (!corners.empty()) {
        memcpy(st + (off[3] - base), corners.data(), sizeof(int4) * corners.size());
        memcpy(st + (off[4] - base), esrc.data(), sizeof(int) * esrc.size());
        memcpy(st + (off[5] - base), ew.data(), sizeof(float) * ew.size());
    }
    // upload the used part of each table (the capacities can be large for
    // windowed-sinc points)
    const size_t used[6] = {sizeof(long long) * idx.size(), sizeof(float) * w.size(), sizeof(int) * pptr.size(),
                            sizeof(int4) * corners.size(), sizeof(int) * esrc.size(), sizeof(float) * ew.size()};
    for (int k = 0; k < 6; ++k)
        if (used[k]) HIPCHK(hipMemcpyAsync(g->ws + off[k], st + (off[k] - base), used[k], hipMemcpyHostToDevice, s));
    if (side == 0 && g->t2) {
        // Extended tables of the two-level step: for each 64 x 16 tile, the
        // source grid points inside the tile grown by the ring its level-1
        // region covers (R rows in y, R rounded up to whole float4 groups in
        // x), per plane, in (tile, z, y, x) order; the entries are those of
        // the point's corner above.
        const int r = L.r, hx = 4 * ((r + 3) / 4);
        const int ntx2 = t2_ntx(L), nty2 = t2_nty(L);
        struct Ext { int tile, z, y, x, corner; };
        std::vector<Ext> ext;
        ext.reserve(corners.size() * 4);
        for (size_t c = 0; c < corners.size(); ++c) {
            const int x = corners[c].x, y = corners[c].y;
            const int z = (int)(ckey[c] % (L.nz + 1));
            for (int ty = std::max(0, y / 16 - 1); ty <= std::min(nty2 - 1, y / 16 + 1); ++ty)
                for (int tx = std::max(0, x / 64 - 1); tx <= std::min(ntx2 - 1, x / 64 + 1); ++tx)
                    if (x >= 64 * tx - hx && x < 64 * tx + 64 + hx && y >= 16 * ty - r && y < 16 * ty + 16 + r)
                        ext.push_back({ty * ntx2 + tx, z, y, x, (int)c});
        }
        std::sort(ext.begin(), ext.end(), [](const Ext &a, const Ext &b) {
            if (a.tile != b.tile) return a.tile < b.tile;
            if (a.z != b.z) return a.z < b.z;
            if (a.y != b.y) return a.y < b.y;
            return a.x < b.x;
        });
        const size_t nptr2 = (size_t)ntx2 * nty2 * (L.nz + 1);
        int *pp2 = (int *)(g->stage + g->wp.stage_t2);
        int4 *cor2 = (int4 *)(g->stage + g->wp.stage_t2 + (g->wp.t2corner - g->wp.t2pp));
        size_t e = 0;
        for (size_t k = 0; k < nptr2; ++k) {
            while (e < ext.size() && (long long)ext[e].tile * (L.nz + 1) + ext[e].z < (long long)k) ++e;
            pp2[k] = (int)e;
        }
        for (size_t i = 0; i < ext.size(); ++i) cor2[i] = corners[ext[i].corner];
        HIPCHK(hipMemcpyAsync(g->t2_pp, pp2, sizeof(int) * nptr2, hipMemcpyHostToDevice, s));
        if (!ext.empty())
            HIPCHK(hipMemcpyAsync(g->t2_corner, cor2, sizeof(int4) * ext.size(), hipMemcpyHostToDevice, s));
        g->t2_ncorner = (int)ext.size();
    }
    rc = stage_release(g, s);
    if (rc) return rc;
    g->cached_xyz[side] = std::move(key);
    g->cached_n[side] = npts;
    g->ncorner[side] = (int)corners.size();
    return FD_OK;
}

StepArgs base_args(const fd_grid *g) {
    StepArgs a{};
    a.L = g->L;
    a.p = g->p;
    a.pq = g->pq;
    a.pq_base = g->pq_base;
    a.pq_step = g->pq_step;
    a.damp = g->damp;
    const double *h = g->d.spacing;
    const double hx2 = h[0] * h[0];
    const double hz2 = (g->d.ndim == 3 ? h[2] * h[2] : h[1] * h[1]);
    const double hy2 = g->d.ndim == 3 ? h[1] * h[1] : 0.0;
    // c_j / h^2 rounded once to float32; the centre weight is then -2 times
    // the sum of the rounded neighbour weights (c_0 = -2 sum c_j exactly),
    // so the float32 operator still maps a constant field to zero.  With
    // the centre weight rounded on its own instead, that residual is about
    // 1e-7 |w0| u per step and doubles the error against the oracle at so
    // 8 and 12.
    double wsum = 0.0;
    for (int j = 0; j <= kMaxR; ++j) {
        const bool in = j >= 1 && j <= g->L.r;
        a.wx[j] = in ? (float)(g->c[j] / hx2) : 0.f;
        a.wz[j] = in ? (float)(g->c[j] / hz2) : 0.f;
        a.wy[j] = (in && g->d.ndim == 3) ? (float)(g->c[j] / hy2) : 0.f;
        wsum += (double)a.wx[j] + (double)a.wy[j] + (double)a.wz[j];
    }
    a.w0 = (float)(-2.0 * wsum);
    a.ntx = g->ntx;
    a.nty = g->nty;
    a.shape3 = g->shape3;
    a.nstrip = g->nstrip;
    // The new level is the next step's centre field.  A 16-bit field of up to
    // kCachedField bytes is stored with ordinary stores, so that it can still
    // sit in the memory-side cache (256 MB) when the next step reads it:
    // measured +4 % (336^3, 106 MB) and +3 % (280^3, 64 MB) in bfloat16, but
    // -12 % at 592^3 (507 MB); in float32 ordinary stores lost 20 % at 336^3
    // and 7 % at 280^3 (the written lines crowd out of L2 the neighbour rows
    // that the halo loads expect there).
    a.out_cached = (g->st != Store::F32 && g->wp.field_bytes <= kCachedField) ? 1 : 0;
    a.ntz = g->ntz[kPlain];
    a.zchunk = g->zchunk[kPlain];
    return a;
}

Inject make_inject(const fd_grid *g, int side, const float *vals, float scale) {
    const SparseDev &d = g->sd[side];
    Inject in{};
    in.plane_ptr = d.plane_ptr;
    in.corner = d.corner;
    in.src = d.ent_src;
    in.w = d.ent_w;
    in.vals = (g->ncorner[side] > 0) ? vals : nullptr;
    in.scale = scale;
    return in;
}

Sample make_sample(const fd_grid *g, int side, int npts, float *out, float scale) {
    const SparseDev &d = g->sd[side];
    Sample s{};
    s.npts = npts;
    s.nc = g->nc;
    s.lpp = 1;
    while (s.lpp < g->nc && s.lpp < 64) s.lpp *= 2;
    s.idx = d.idx;
    s.w = d.w;
    s.out = out;
    s.scale = scale;
    return s;
}

inline int samp_blocks(const Sample &s) { return sample_blocks(s); }

int check_dt(const fd_grid *g, double dt, int nt) {
    if (nt < 0) return fdi_fail(FD_ERR_ARG, "nt < 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fdi_fail(FD_ERR_ARG, "dt must be > 0");
    if (dt >= g->dt_crit)
        return fdi_fail(FD_ERR_UNSTABLE, "dt %.6g s >= stability limit %.6g s", dt, g->dt_crit);
    return FD_OK;
}

// empty_ok: a forward or adjoint run may have no sources (an initial-value
// problem) or no receivers (only the final state wanted)
int check_shot(const fd_grid *g, const fd_shot *sh, bool empty_ok = false) {
    if (!sh) return fdi_fail(FD_ERR_ARG, "null shot");
    if (sh->nsrc < 0 || sh->nrec < 0) return fdi_fail(FD_ERR_ARG, "nsrc and nrec must be >= 0");
    if (!empty_ok && (sh->nsrc < 1 || sh->nrec < 1)) return fdi_fail(FD_ERR_ARG, "nsrc and nrec must be >= 1");
    (void)g;
    return FD_OK;
}

}  // namespace

// ------------------------------------------------------------ public calls
extern "C" int fd_grid_workspace_bytes(const fd_grid_desc *desc, size_t *bytes) {
    API_GUARD_BEGIN
    if (!bytes) return fdi_fail(FD_ERR_ARG, "null output");
    if (!fdi_check_desc(desc)) return FD_ERR_ARG;
    const Layout L = fdi_layout(desc);
    *bytes = plan(desc, L).total;
    return FD_OK;
    API_GUARD_END
}

extern "C" int fd_grid_create(const fd_grid_desc *desc, void *workspace, size_t ws_bytes,
                              const float *vp_dev, void *stream, fd_grid **out) {
    API_GUARD_BEGIN
    if (!out) return fdi_fail(FD_ERR_ARG, "null output handle");
    *out = nullptr;
    if (!fdi_check_desc(desc)) return FD_ERR_ARG;
    if (!workspace || !vp_dev) return fdi_fail(FD_ERR_ARG, "null workspace or velocity");
    if ((uintptr_t)workspace % 256) return fdi_fail(FD_ERR_ARG, "workspace must be 256-byte aligned");
    const Layout L = fdi_layout(desc);
    const WsPlan wp = plan(desc, L);
    if (ws_bytes < wp.total)
        return fdi_fail(FD_ERR_NOMEM, "workspace %zu bytes < required %zu", ws_bytes, wp.total);
    hipStream_t s = (hipStream_t)stream;

    fd_grid *g = new fd_grid();
    g->d = *desc;
    HIPCHK(hipGetDevice(&g->device));
    g->L = L;
    g->st = elem_store(desc->storage);
    g->diff = diff_storage(desc);
    g->amp = (desc->storage != FD_STORE_F32 && desc->amp_scale > 0.f) ? desc->amp_scale : 1.f;
    g->auto_amp = g->st == Store::F16 && !(desc->amp_scale > 0.f);
    g->nc = sparse_nodes(desc);
    fdi_second_derivative_weights(L.r, g->c);
    g->cell = 1.0;
    for (int a = 0; a < desc->ndim; ++a) g->cell *= desc->spacing[a];
    g->ws = (char *)workspace;
    g->ws_bytes = ws_bytes;
    g->wp = wp;
    g->vel = (float *)(g->ws + wp.vel);
    const bool q16 = desc->param_storage == FD_PARAM_Q16;
    g->p = q16 ? nullptr : (float *)(g->ws + wp.p);
    g->pq = q16 ? (uint16_t *)(g->ws + wp.p) : nullptr;
    g->uA = g->ws + wp.uA;
    g->uB = g->ws + wp.uB;
    g->t2 = t2_enabled(desc);
    g->uC = g->ws + wp.uC;
    g->uD = g->ws + wp.uD;
    g->t2_pp = (int *)(g->ws + wp.t2pp);
    g->t2_corner = (int4 *)(g->ws + wp.t2corner);
    g->t2_ncorner = 0;
    g->cur = g->uA;
    g->prev = g->uB;
    g->rows_done = 0;
    g->damp = (float *)(g->ws + wp.damp);
    g->partials = (double *)(g->ws + wp.misc);
    g->vmax_bits = (unsigned *)(g->ws + wp.misc + sizeof(double) * kNPart);
    for (int side = 0; side < 2; ++side) {
        const size_t *o = side == 0 ? wp.src : wp.rec;
        SparseDev &d = g->sd[side];
        d.cap = side == 0 ? wp.cap_src : wp.cap_rec;
        d.idx = (long long *)(g->ws + o[0]);
        d.w = (float *)(g->ws + o[1]);
        d.plane_ptr = (int *)(g->ws + o[2]);
        d.corner = (int4 *)(g->ws + o[3]);
        d.ent_src = (int *)(g->ws + o[4]);
        d.ent_w = (float *)(g->ws + o[5]);
        g->cached_n[side] = -1;
        g->ncorner[side] = 0;
    }
    g->dt_cached = -1.0;
    g->has_last_stream = false;
    g->stage = nullptr;
    g->stage_pending = false;
    auto cleanup = [&](int rc) {
        if (g->stage) (void)hipHostFree(g->stage);
        (void)hipEventDestroy(g->stage_ev);
        delete g;
        return rc;
    };
    if (hipEventCreateWithFlags(&g->stage_ev, hipEventDisableTiming) != hipSuccess) {
        delete g;
        return fdi_fail(FD_ERR_DEVICE, "hipEventCreate failed");
    }
    if (hipHostMalloc((void **)&g->stage, wp.stage_bytes, hipHostMallocDefault) != hipSuccess)
        return cleanup(fdi_fail(FD_ERR_NOMEM, "pinned staging allocation failed"));

    // launch geometry of each step mode (the gradient modes differ in
    // register use, hence occupancy, hence chunking)
    g->shape3 = tile_shape(desc, L);
    {
        const TileGrid tg = tile_grid(L, g->shape3);
        g->ntx = tg.ntx;
        g->nty = tg.nty;
        g->nstrip = tg.nstrip;
    }
    for (int m = 0; m < 3; ++m) {
        if (desc->ndim == 2) {
            g->zchunk[m] = kTile2Z;
            g->ntz[m] = (L.nz + kTile2Z - 1) / kTile2Z;
            continue;
        }
        int zc = desc->zchunk;
        if (zc <= 0) {
            // One balanced round of workgroups: k workgroups on every CU
            // (2 <= k <= min(3, occupancy)), with the number of z chunks per
            // xy tile that fills k * CUs slots best, so no second, partly
            // filled round trails the first.  On a tie, k = 2 for float32
            // fields and k = 3 for 16-bit ones: measured on 336^3, so 4..16,
            // k = 2 wins by 0.5-5 % in float32 and k = 3 by 6-13 % in 16-bit
            // (more concurrent columns thrash the per-XCD L2 that serves the
            // halo reads; with half the bytes per point, 16-bit columns fit
            // one more).  On 280^3 (90 tiles) the fill decides: k = 3 fills
            // 94 % of the slots, k = 2 only 88 %.
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess ||
                cus <= 0)
                cus = 256;
            // (the forward slot runs the difference step under the difference storages)
            const int mk = (m == kPlain && g->diff) ? (int)kDiff : m;
            const int occ = std::max(1, step_blocks_per_cu(3, L.r, g->st, mk, g->shape3, g->pq != nullptr));
            const int tiles = std::max(1, g->ntx * g->nty + g->nstrip);
            const int kmax = std::min(occ, 3), prefer = g->st == Store::F32 ? 2 : 3;
            int nzc = 1;
            double best = -1.0;
            for (int k = std::min(2, kmax); k <= kmax; ++k) {
                const int n = std::max(1, std::min(L.nz, k * cus / tiles));
                const double fill = std::min(1.0, (double)n * tiles / ((double)k * cus));
                const double score = fill - (k == prefer ? 0.0 : 0.02);
                if (score > best) {
                    best = score;
                    nzc = n;
                }
            }
            // Wide xy planes give long chunks (592^3: 370 tiles, k = 3, two
            // chunks of 296 planes); measured against chunks of 64 planes
            // there, one round of long chunks is as fast in float32 and 3 %
            // faster in bfloat16.
            zc = (L.nz + nzc - 1) / nzc;
        }
        g->zchunk[m] = std::min(std::min(zc, L.nz), kMaxChunk);
        g->ntz[m] = (L.nz + g->zchunk[m] - 1) / g->zchunk[m];
    }
    if (g->t2) {
        // two-level step: one balanced round of workgroups as above, at the
        // kernel's own occupancy; each z chunk recomputes R level-1 planes at
        // either end (shared with the neighbouring chunks), so chunks stay
        // long
        int zc = desc->zchunk;
        if (zc <= 0) {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess ||
                cus <= 0)
                cus = 256;
            const int occ = std::max(1, step_t2_blocks_per_cu(L.r));
            const int tiles = t2_ntx(L) * t2_nty(L);
            const int nzc = std::max(1, std::min(L.nz, occ * cus / tiles));
            zc = (L.nz + nzc - 1) / nzc;
        }
        g->t2_zchunk = std::min(std::min(zc, L.nz), kMaxChunk);
        g->t2_ntz = (L.nz + g->t2_zchunk - 1) / g->t2_zchunk;
    }

    // zero every field (halos included), fill velocity, find v_max
    hipError_t e = hipSuccess;
    if ((e = launch_zero_field(L, g->uA, g->st, s)) != hipSuccess ||
        (e = launch_zero_field(L, g->uB, g->st, s)) != hipSuccess ||
        ((g->t2 || g->diff) && (e = launch_zero_field(L, g->uC, g->st, s)) != hipSuccess) ||
        (g->t2 && (e = launch_zero_field(L, g->uD, g->st, s)) != hipSuccess) ||
        (e = launch_zero_field(L, g->vel, Store::F32, s)) != hipSuccess ||
        (e = (g->pq ? launch_zero_field(L, g->pq, Store::F16, s) : launch_zero_field(L, g->p, Store::F32, s))) !=
            hipSuccess)
        return cleanup(fdi_fail(FD_ERR_DEVICE, "zero fill: %s", hipGetErrorString(e)));
    const int phys[3] = {desc->shape[0], desc->ndim == 3 ? desc->shape[1] : 1,
                         desc->ndim == 3 ? desc->shape[2] : desc->shape[1]};
    if ((e = launch_fill_velocity(L, vp_dev, desc->vp_padded, desc->nbl, phys, g->vel, s)) != hipSuccess ||
        (e = hipMemsetAsync(g->vmax_bits, 0, sizeof(unsigned), s)) != hipSuccess ||
        (e = hipMemsetD32Async((hipDeviceptr_t)(g->vmax_bits + 1), 0x7F800000u, 1, s)) != hipSuccess ||
        (e = launch_vrange(L, g->vel, g->vmax_bits, s)) != hipSuccess)
        return cleanup(fdi_fail(FD_ERR_DEVICE, "velocity setup: %s", hipGetErrorString(e)));
    unsigned bits[2] = {0, 0};
    if ((e = hipMemcpyAsync(bits, g->vmax_bits, sizeof bits, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return cleanup(fdi_fail(FD_ERR_DEVICE, "velocity readback: %s", hipGetErrorString(e)));
    float vmax, vmin;
    memcpy(&vmax, &bits[0], sizeof vmax);
    memcpy(&vmin, &bits[1], sizeof vmin);
    if (!(vmax > 0.f) || !std::isfinite(vmax))
        return cleanup(fdi_fail(FD_ERR_ARG, "velocity must be finite and > 0 everywhere"));
    g->vmax = vmax;
    g->vmin = vmin;
    // von Neumann limit: dt_crit = 1 / (v_max sqrt(sum_{j odd} c_j * sum_a h_a^-2))
    double s_odd = 0.0;
    for (int j = 1; j <= L.r; j += 2) s_odd += g->c[j];
    double ih2 = 0.0;
    for (int a = 0; a < desc->ndim; ++a) ih2 += 1.0 / (desc->spacing[a] * desc->spacing[a]);
    g->dt_crit = 1.0 / (g->vmax * std::sqrt(s_odd * ih2));
    double hmin = desc->spacing[0];
    for (int a = 1; a < desc->ndim; ++a) hmin = std::min(hmin, desc->spacing[a]);
    if (desc->nbl == 0)
        g->sigma_max = 0.0;
    else if (desc->damp_max > 0.0)
        g->sigma_max = desc->damp_max;
    else
        g->sigma_max = 3.0 * g->vmax * std::log(1000.0) / (2.0 * desc->nbl * hmin);
    *out = g;
    return FD_OK;
    API_GUARD_END
}

extern "C" int fd_grid_destroy(fd_grid *g) {
    API_GUARD_BEGIN
    if (!g) return FD_OK;
    DeviceGuard dg(g->device);
    if (g->stage_pending) (void)hipEventSynchronize(g->stage_ev);
    if (g->has_last_stream) (void)hipStreamSynchronize(g->last_stream);
    if (g->stage) (void)hipHostFree(g->stage);
    (void)hipEventDestroy(g->stage_ev);
    delete g;
    return FD_OK;
    API_GUARD_END
}

extern "C" int fd_grid_get_info(const fd_grid *g, fd_grid_info *info) {
    if (!g || !info) return fdi_fail(FD_ERR_ARG, "null argument");
    memset(info, 0, sizeof *info);
    info->ndim = g->d.ndim;
    info->padded[0] = g->L.nx;
    if (g->d.ndim == 3) {
        info->padded[1] = g->L.ny;
        info->padded[2] = g->L.nz;
    } else {
        info->padded[1] = g->L.nz;
    }
    info->padded_points = (long long)g->L.nx * g->L.ny * g->L.nz;
    info->vmax = g->vmax;
    info->critical_dt = g->dt_crit;
    info->damp_max = g->sigma_max;
    info->field_bytes = g->wp.field_bytes;
    const int tw4 = g->shape3 == kShapeMixed ? 16 : g->shape3;
    info->tile[0] = g->d.ndim == 3 ? tile3_x(tw4) : kTileX;
    info->tile[1] = g->d.ndim == 3 ? tile3_y(tw4) : kTile2Z;
    info->tile_strip = g->nstrip > 0 ? g->L.nx - 64 * g->ntx : 0;
    info->zchunk = g->zchunk[kPlain];
    info->time_block = g->t2 ? 2 : 1;
    info->param_storage = g->d.param_storage;
    info->param_base = g->pq && g->dt_cached > 0.0 ? g->pq_base : 0.0;
    info->param_step = g->pq && g->dt_cached > 0.0 ? g->pq_step : 0.0;
    return FD_OK;
}

// Enqueue forward steps n0 .. n1-1 of an nt-step run continuing from the
// grid's state (u^n0 in g->cur, u^{n0-1} in g->prev; a run can be advanced
// in chunks).  Trace row n-1 samples u^n: the one-step kernel samples its
// centre field in the launch that starts from it; the two-level kernel
// samples both its input levels (rows n-1 and n-2) in the launch that starts
// from level n.  g->rows_done counts the rows sampled so far; before a
// one-step launch overwrites u^{n-1} in place, a row left to it is sampled
// first, and the last chunk samples what remains.  If ckpt is given, (u^c,
// u^{c-1}) is copied to ckpt[2*(c/K)], ckpt[2*(c/K)+1] before step c for
// every multiple c of K (one step per launch then).
int fdi_forward_steps(fd_grid *g, const fd_shot *sh, int nt, int n0, int n1, float *rec_out,
                      void **ckpt, int K, hipStream_t s) {
    note_stream(g, s);
    StepArgs a = base_args(g);
    const float inj_scale = (float)(g->amp / g->cell);
    const float smp_scale = 1.f / g->amp;
    auto row = [&](int r) -> float * {
        return (rec_out && r >= 0 && r < nt && r >= g->rows_done) ? rec_out + (size_t)r * sh->nrec : nullptr;
    };
    const bool t2 = g->t2 && !ckpt;
    int n = n0;
    while (n < n1) {
        if (t2 && n + 2 <= n1) {
            // two levels: u^{n+1} and u^{n+2} into the pair not holding u^n, u^{n-1}
            void *fa = nullptr, *fb = nullptr;
            void *bufs[4] = {g->uA, g->uB, g->uC, g->uD};
            for (void *b : bufs)
                if (b != g->cur && b != g->prev) (fa ? fb : fa) = b;
            StepArgs t = a;
            t.u = g->cur;
            t.prev = g->prev;
            t.out = fb;    // u^{n+1}
            t.out2 = fa;   // u^{n+2}
            t.ntx = t2_ntx(g->L);
            t.nty = t2_nty(g->L);
            t.ntz = g->t2_ntz;
            t.zchunk = g->t2_zchunk;
            const SparseDev &d = g->sd[0];
            const bool any = g->ncorner[0] > 0;
            t.inj = Inject{g->t2_pp, g->t2_corner, d.ent_src, d.ent_w,
                           any ? sh->src_wavelet + (size_t)n * sh->nsrc : nullptr, inj_scale};
            t.inj2 = Inject{g->t2_pp, g->t2_corner, d.ent_src, d.ent_w,
                            any ? sh->src_wavelet + (size_t)(n + 1) * sh->nsrc : nullptr, inj_scale};
            t.smp = make_sample(g, 1, sh->nrec, row(n - 1), smp_scale);
            t.nsamp_blocks = samp_blocks(t.smp);
            t.smp2 = make_sample(g, 1, sh->nrec, row(n - 2), smp_scale);
            t.nsamp_blocks2 = samp_blocks(t.smp2);
            HIPCHK(launch_step_t2(t, s));
            g->rows_done = std::max(g->rows_done, std::min(n, nt));
            g->prev = fb;
            g->cur = fa;
            n += 2;
            continue;
        }
        if (ckpt && n % K == 0) {
            HIPCHK(hipMemcpyAsync(ckpt[2 * (n / K)], g->cur, g->wp.field_bytes, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(ckpt[2 * (n / K) + 1], g->prev, g->wp.field_bytes, hipMemcpyDeviceToDevice, s));
        }
        if (float *r2 = row(n - 2)) {   // u^{n-1} is about to be overwritten
            Sample sm = make_sample(g, 1, sh->nrec, r2, smp_scale);
            HIPCHK(launch_sample(sm, g->prev, g->st, s));
        }
        a.u = g->cur;
        a.prev = g->diff ? g->uC : g->prev;   // the difference, or u^{n-1}
        a.out = g->prev;
        a.out2 = g->diff ? g->uC : nullptr;   // the new difference, in place
        a.inj = make_inject(g, 0, sh->src_wavelet + (size_t)n * sh->nsrc, inj_scale);
        a.smp = make_sample(g, 1, sh->nrec, row(n - 1), smp_scale);
        a.nsamp_blocks = samp_blocks(a.smp);
        HIPCHK(launch_step(a, g->st, g->diff ? kDiff : kPlain, s));
        g->rows_done = std::max(g->rows_done, std::min(n, nt));
        std::swap(g->cur, g->prev);
        ++n;
    }
    if (n1 == nt && nt >= 1) {
        if (float *r2 = row(nt - 2)) {
            Sample sm = make_sample(g, 1, sh->nrec, r2, smp_scale);
            HIPCHK(launch_sample(sm, g->prev, g->st, s));
        }
        if (float *r1 = row(nt - 1)) {
            Sample sm = make_sample(g, 1, sh->nrec, r1, smp_scale);
            HIPCHK(launch_sample(sm, g->cur, g->st, s));
        }
        g->rows_done = nt;
    }
    return FD_OK;
}

// Validate a forward run and make the grid's tables current for it.
int fdi_forward_prepare(fd_grid *g, const fd_shot *sh, int nt, double dt, hipStream_t s) {
    int rc;
    if (!g) return fdi_fail(FD_ERR_ARG, "null grid");
    if ((rc = check_shot(g, sh, true))) return rc;
    if ((rc = check_dt(g, dt, nt))) return rc;
    if (nt > 0 && sh->nsrc > 0 && !sh->src_wavelet) return fdi_fail(FD_ERR_ARG, "null wavelet");
    if ((rc = ensure_dt(g, dt, s))) return rc;
    if ((rc = ensure_side(g, 0, sh->nsrc, sh->src_xyz, s))) return rc;
    if ((rc = ensure_side(g, 1, sh->nrec, sh->rec_xyz, s))) return rc;
    return FD_OK;
}

// Zero initial state (u^0 = u^{-1} = 0) in uA, uB, and a new run's rows.
int fdi_forward_zero_state(fd_grid *g, hipStream_t s) {
    HIPCHK(launch_zero_field(g->L, g->uA, g->st, s));
    HIPCHK(launch_zero_field(g->L, g->uB, g->st, s));
    if (g->diff) HIPCHK(launch_zero_field(g->L, g->uC, g->st, s));
    g->cur = g->uA;
    g->prev = g->uB;
    g->rows_done = 0;
    return FD_OK;
}

int fdi_grid_device(const fd_grid *g) { return g->device; }

extern "C" int fd_forward(fd_grid *g, const fd_shot *sh, int nt, double dt, float *rec_out,
                          const fd_fwd_opts *opts, void *stream) {
    API_GUARD_BEGIN
    if (!g) return fdi_fail(FD_ERR_ARG, "null grid");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = fdi_forward_prepare(g, sh, nt, dt, s))) return rc;
    if (nt > 0 && sh->nrec > 0 && !rec_out) return fdi_fail(FD_ERR_ARG, "null receiver output");
    const Layout &L = g->L;
    if (opts && opts->u0) HIPCHK(launch_dense_to_field(L, opts->u0, g->uA, g->st, g->amp, s));
    else HIPCHK(launch_zero_field(L, g->uA, g->st, s));
    if (opts && opts->u_prev && !g->diff) HIPCHK(launch_dense_to_field(L, opts->u_prev, g->uB, g->st, g->amp, s));
    else HIPCHK(launch_zero_field(L, g->uB, g->st, s));
    if (g->diff) {   // the difference u^0 - u^{-1}, rounded once
        if (opts && (opts->u0 || opts->u_prev))
            HIPCHK(launch_dense_diff_to_field(L, opts->u0, opts->u_prev, g->uC, g->st, g->amp, s));
        else
            HIPCHK(launch_zero_field(L, g->uC, g->st, s));
    }
    g->cur = g->uA;
    g->prev = g->uB;
    g->rows_done = 0;
    if ((rc = fdi_forward_steps(g, sh, nt, 0, nt, rec_out, nullptr, 1, s))) return rc;
    if (opts && opts->save_u) HIPCHK(launch_field_to_dense(L, g->cur, opts->save_u, g->st, 1.f / g->amp, s));
    if (opts && opts->save_u_prev) {
        if (g->diff)
            HIPCHK(launch_field_diff_to_dense(L, g->cur, g->uC, opts->save_u_prev, g->st, 1.f / g->amp, s));
        else
            HIPCHK(launch_field_to_dense(L, g->prev, opts->save_u_prev, g->st, 1.f / g->amp, s));
    }
    return FD_OK;
    API_GUARD_END
}

extern "C" int fd_adjoint(fd_grid *g, const fd_shot *sh, int nt, double dt,
                          const float *residual, float *src_adj, void *stream) {
    API_GUARD_BEGIN
    if (!g) return fdi_fail(FD_ERR_ARG, "null grid");
    int rc;
    if ((rc = check_shot(g, sh, true))) return rc;
    if ((rc = check_dt(g, dt, nt))) return rc;
    if (nt > 0 && ((sh->nrec > 0 && !residual) || (sh->nsrc > 0 && !src_adj)))
        return fdi_fail(FD_ERR_ARG, "null residual or output");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ensure_dt(g, dt, s))) return rc;
    if ((rc = ensure_side(g, 0, sh->nsrc, sh->src_xyz, s))) return rc;
    if ((rc = ensure_side(g, 1, sh->nrec, sh->rec_xyz, s))) return rc;
    const Layout &L = g->L;
    note_stream(g, s);
    HIPCHK(launch_zero_field(L, g->uA, g->st, s));
    HIPCHK(launch_zero_field(L, g->uB, g->st, s));
    StepArgs a = base_args(g);
    void *A = g->uA, *B = g->uB;   // lambda^k, lambda^{k+1}
    // 16-bit storage keeps amp_adj * lambda.  lambda is of order v^2 r, not
    // dt^2 v^2 w / prod(h) like the forward field, so the forward's scale
    // times dt^2 / prod(h) (rounded to a power of two, exact) keeps the
    // stored adjoint field in range; float32 storage is not scaled.
    const double amp_adj = g->st == Store::F32 ? 1.0
                                               : std::exp2(std::round(std::log2((double)g->amp * dt * dt / g->cell)));
    const float inj_scale = (float)(amp_adj / (dt * dt));
    const float smp_scale = (float)(dt * dt / (g->cell * amp_adj));
    for (int k = nt; k >= 1; --k) {
        a.u = A;
        a.prev = B;
        a.out = B;
        a.inj = make_inject(g, 1, residual + (size_t)(k - 1) * sh->nrec, inj_scale);
        a.smp = make_sample(g, 0, sh->nsrc, k <= nt - 1 ? src_adj + (size_t)k * sh->nsrc : nullptr, smp_scale);
        a.nsamp_blocks = samp_blocks(a.smp);
        HIPCHK(launch_step(a, g->st, kPlain, s));
        std::swap(A, B);
    }
    if (nt >= 1) {
        Sample sm = make_sample(g, 0, sh->nsrc, src_adj, smp_scale);
        HIPCHK(launch_sample(sm, A, g->st, s));
    }
    return FD_OK;
    API_GUARD_END
}

namespace {
// Gradient workspace.  Fixed interval K: 2 checkpoint fields every K steps,
// the two rotating fields of the segment recompute and K imaging brackets.
// Binomial (K = number of snapshot slots): K+1 snapshot pairs, the state
// pair, the output field of the bracket step and one bracket.  Both: the
// float64 accumulator and the float32 partial sum (pitched), traces and
// residual.
struct GradPlan {
    size_t ckpt, rot, br, grad, gpart, rec, resid, total;
    int ncp, nseg, K, nbr;   // checkpoint pairs (binomial: snapshot slots + 1), fixed-interval segments
    bool binomial;
};
GradPlan grad_plan(const fd_grid *g, int nt, int nrec, int K, int flags) {
    GradPlan p{};
    p.K = K;
    p.binomial = (flags & FD_GRAD_BINOMIAL) != 0;
    // fixed interval: segments of K steps; no checkpoint is stored for the
    // last segment, whose brackets the forward pass writes directly
    p.nseg = p.binomial ? 0 : (K >= nt ? 1 : (nt + K - 1) / K);
    p.ncp = p.binomial ? std::min(K, nt) + 1 : p.nseg - 1;
    p.nbr = p.binomial ? 2 : std::min(K, nt);   // binomial: output field + bracket
    const size_t fb = g->wp.field_bytes;
    size_t o = 0;
    p.ckpt = o; o += fb * 2 * (size_t)p.ncp;
    // two working fields for the resident and binomial schedules (the fixed
    // interval recomputes each segment in its checkpoint's fields)
    p.rot = o;
    if (p.binomial || K >= nt) o += fb * 2;
    p.br = o; o += fb * (size_t)p.nbr;
    p.grad = o; o = align_up(o + sizeof(double) * (size_t)g->L.elems, 256);
    p.gpart = o; o = align_up(o + sizeof(float) * (size_t)g->L.elems, 256);
    p.rec = o; o = align_up(o + sizeof(float) * (size_t)nt * nrec, 256);
    p.resid = o; o = align_up(o + sizeof(float) * (size_t)nt * nrec, 256);
    p.total = o;
    return p;
}
}  // namespace

extern "C" int fd_gradient_workspace_bytes(const fd_grid *g, int nt, int nrec, int K, int flags, size_t *bytes) {
    API_GUARD_BEGIN
    if (!g || !bytes) return fdi_fail(FD_ERR_ARG, "null argument");
    if (nt < 1 || nrec < 1 || K < ((flags & FD_GRAD_BINOMIAL) ? 0 : 1))
        return fdi_fail(FD_ERR_ARG, "nt, nrec >= 1; checkpoint_every >= 1 (>= 0 snapshot slots when binomial)");
    *bytes = grad_plan(g, nt, nrec, K, flags).total;
    return FD_OK;
    API_GUARD_END
}

extern "C" int fd_gradient(fd_grid *g, const fd_shot *sh, int nt, double dt, const float *d_obs,
                           int K, int flags, void *workspace, size_t ws_bytes, double *misfit,
                           double *grad_m, float *rec_out, float *src_adj, void *stream) {
    API_GUARD_BEGIN
    if (!g) return fdi_fail(FD_ERR_ARG, "null grid");
    int rc;
    if ((rc = check_shot(g, sh))) return rc;
    if ((rc = check_dt(g, dt, nt))) return rc;
    if (nt < 1 || K < ((flags & FD_GRAD_BINOMIAL) ? 0 : 1))
        return fdi_fail(FD_ERR_ARG, "nt >= 1; checkpoint_every >= 1 (>= 0 snapshot slots when binomial)");
    if (flags & ~(FD_GRAD_RESIDUAL_GIVEN | FD_GRAD_BINOMIAL | FD_GRAD_VELOCITY))
        return fdi_fail(FD_ERR_ARG, "unknown fd_gradient flag");
    if (g->st != Store::F32) return fdi_fail(FD_ERR_ARG, "fd_gradient needs float32 storage");
    if (g->pq) return fdi_fail(FD_ERR_ARG, "fd_gradient needs float32 p (FD_PARAM_F32)");
    if (!d_obs || !misfit || !grad_m || !workspace || !sh->src_wavelet)
        return fdi_fail(FD_ERR_ARG, "null pointer argument");
    if ((uintptr_t)workspace % 256) return fdi_fail(FD_ERR_ARG, "workspace must be 256-byte aligned");
    const GradPlan gp = grad_plan(g, nt, sh->nrec, K, flags);
    if (ws_bytes < gp.total) return fdi_fail(FD_ERR_NOMEM, "gradient workspace %zu < %zu", ws_bytes, gp.total);
    std::vector<fd_ckpt_action> plan;
    if (gp.binomial && (rc = fdi_checkpoint_plan(nt, K, &plan, nullptr))) return rc;
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ensure_dt(g, dt, s))) return rc;
    if ((rc = ensure_side(g, 0, sh->nsrc, sh->src_xyz, s))) return rc;
    if ((rc = ensure_side(g, 1, sh->nrec, sh->rec_xyz, s))) return rc;
    note_stream(g, s);
    const Layout &L = g->L;
    char *ws = (char *)workspace;
    const size_t fb = g->wp.field_bytes;
    std::vector<void *> ck((size_t)2 * gp.ncp);
    for (int i = 0; i < 2 * gp.ncp; ++i) ck[i] = ws + gp.ckpt + fb * (size_t)i;
    void *rotA = ws + gp.rot, *rotB = ws + gp.rot + fb;   // (not allocated for the fixed interval, which does not use them)
    std::vector<float *> br(gp.nbr);
    for (int i = 0; i < gp.nbr; ++i) br[i] = (float *)(ws + gp.br + fb * (size_t)i);
    double *gacc = (double *)(ws + gp.grad);
    float *gpart = (float *)(ws + gp.gpart);
    float *recb = (float *)(ws + gp.rec);
    float *resid = (float *)(ws + gp.resid);
    const long long nres = (long long)nt * sh->nrec;
    const int given = (flags & FD_GRAD_RESIDUAL_GIVEN) ? 1 : 0;

    StepArgs a = base_args(g);
    const float fwd_inj = (float)(1.0 / g->cell);
    const float adj_inj = (float)(1.0 / (dt * dt));
    const float adj_smp = (float)(dt * dt / g->cell);
    void *LA = g->uA, *LB = g->uB;   // lambda^k, lambda^{k+1}
    // forward step n with the imaging bracket of level n into `brf`
    auto bracket_step = [&](int n, void *u, void *prev, void *out, float *brf, float *rec_row) -> int {
        a.u = u;
        a.prev = prev;
        a.out = out;
        a.inj = make_inject(g, 0, sh->src_wavelet + (size_t)n * sh->nsrc, fwd_inj);
        a.smp = make_sample(g, 1, sh->nrec, rec_row, 1.f);
        a.nsamp_blocks = samp_blocks(a.smp);
        a.img = Imaging{};
        a.img.br_out = brf;
        a.ntz = g->ntz[kBracket];
        a.zchunk = g->zchunk[kBracket];
        HIPCHK(launch_step(a, g->st, kBracket, s));
        return FD_OK;
    };
    // adjoint step k: lambda^{k-1} from lambda^k, lambda^{k+1}, residual row
    // k-1, and grad -= lambda^{k-1} * bracket of level k-1.  The products
    // are summed in float32 and folded into the float64 gradient after every
    // kFoldEvery adjoint steps of the reverse sweep (the same steps for every
    // schedule, so the result does not depend on the schedule).
    int adj_done = 0;
    auto adjoint_step = [&](int k, const float *brf) -> int {
        a.u = LA;
        a.prev = LB;
        a.out = LB;
        a.inj = make_inject(g, 1, resid + (size_t)(k - 1) * sh->nrec, adj_inj);
        a.smp = make_sample(g, 0, sh->nsrc, (src_adj && k <= nt - 1) ? src_adj + (size_t)k * sh->nsrc : nullptr,
                            adj_smp);
        a.nsamp_blocks = samp_blocks(a.smp);
        a.img = Imaging{};
        a.img.br_in = brf;
        a.img.gpart = gpart;
        a.ntz = g->ntz[kImage];
        a.zchunk = g->zchunk[kImage];
        HIPCHK(launch_step(a, g->st, kImage, s));
        std::swap(LA, LB);
        if (++adj_done % kFoldEvery == 0) HIPCHK(launch_fold_f64(L, gacc, gpart, s));
        return FD_OK;
    };
    HIPCHK(launch_zero_f64(gacc, L.elems, s));
    HIPCHK(launch_zero_field(L, gpart, Store::F32, s));

    if (!gp.binomial && K >= nt) {
        // Every bracket fits the workspace: the forward pass itself writes
        // the bracket of each level (no checkpoint, no recompute), then the
        // residual, then the whole adjoint sweep.
        void *A = rotA, *B = rotB;   // u^n, u^{n-1}
        HIPCHK(launch_zero_field(L, A, g->st, s));
        HIPCHK(launch_zero_field(L, B, g->st, s));
        for (int n = 0; n < nt; ++n) {
            if ((rc = bracket_step(n, A, B, B, br[n], n >= 1 ? recb + (size_t)(n - 1) * sh->nrec : nullptr)))
                return rc;
            std::swap(A, B);
        }
        Sample sm = make_sample(g, 1, sh->nrec, recb + (size_t)(nt - 1) * sh->nrec, 1.f);
        HIPCHK(launch_sample(sm, A, g->st, s));
        HIPCHK(launch_misfit(recb, d_obs, nres, given, resid, g->partials, kNPart, misfit, s));
        HIPCHK(launch_zero_field(L, g->uA, g->st, s));
        HIPCHK(launch_zero_field(L, g->uB, g->st, s));
        for (int k = nt; k >= 1; --k)
            if ((rc = adjoint_step(k, br[k - 1]))) return rc;
    } else if (!gp.binomial) {
        // 1. forward with checkpoints of (u^c, u^{c-1}) every K steps.  The
        //    steps of the last segment write their imaging brackets as they
        //    go: the sweep below would otherwise recompute exactly these
        //    steps first (the bracket mode's u is bitwise the plain mode's).
        const int clast = (gp.nseg - 1) * K;
        if ((rc = fdi_forward_zero_state(g, s))) return rc;
        if ((rc = fdi_forward_steps(g, sh, nt, 0, clast, recb, ck.data(), K, s))) return rc;
        {
            void *A = g->cur, *B = g->prev;   // u^n, u^{n-1}, as the chunked forward leaves them
            for (int n = clast; n < nt; ++n) {
                if ((rc = bracket_step(n, A, B, B, br[n - clast], recb + (size_t)(n - 1) * sh->nrec))) return rc;
                std::swap(A, B);
            }
            Sample sm = make_sample(g, 1, sh->nrec, recb + (size_t)(nt - 1) * sh->nrec, 1.f);
            HIPCHK(launch_sample(sm, A, g->st, s));
        }
        // 2. residual and misfit (FP64)
        HIPCHK(launch_misfit(recb, d_obs, nres, given, resid, g->partials, kNPart, misfit, s));
        // 3. adjoint sweep over segments, last to first.  Each earlier
        //    segment is recomputed from its checkpoint, writing the imaging
        //    bracket of every time level; the adjoint steps read one bracket
        //    per point.
        HIPCHK(launch_zero_field(L, g->uA, g->st, s));
        HIPCHK(launch_zero_field(L, g->uB, g->st, s));
        for (int seg = gp.nseg - 1; seg >= 0; --seg) {
            const int c = seg * K;
            const int e = std::min(c + K, nt);
            if (c != clast) {
                // each checkpoint serves one recompute: step in its own fields
                void *A = ck[2 * seg], *B = ck[2 * seg + 1];   // u^n, u^{n-1}
                for (int n = c; n < e; ++n) {
                    if ((rc = bracket_step(n, A, B, B, br[n - c], nullptr))) return rc;
                    std::swap(A, B);
                }
            }
            for (int k = e; k >= c + 1; --k)
                if ((rc = adjoint_step(k, br[k - 1 - c]))) return rc;
        }
    } else {
        // Binomial schedule over a pool of fields (the checkpoint pairs and
        // the two rotating fields) with reference counts instead of copies:
        // a snapshot slot references the two fields of the state it saved,
        // RESTORE makes those fields the current state, and a step whose
        // in-place target is referenced by a slot writes a free field
        // instead.  The pool always holds one: the slots reference at most
        // 2 (slots + 1) of its 2 (slots + 1) + 2 fields, and when a step needs
        // a free field at most one of the current two is unreferenced.
        // YOUTURN takes one bracket step out of place and the adjoint step
        // that consumes it.  The first sweep samples the receivers; the first
        // YOUTURN (level nt-1) completes the traces and forms the residual.
        const int npool = 2 * gp.ncp + 2;
        std::vector<void *> pool(npool);
        for (int i = 0; i < 2 * gp.ncp; ++i) pool[i] = ck[i];
        pool[2 * gp.ncp] = rotA;
        pool[2 * gp.ncp + 1] = rotB;
        std::vector<int> ref(npool, 0);
        std::vector<int> slot_u(gp.ncp, -1), slot_p(gp.ncp, -1);
        float *out_f = br[0], *brf = br[1];
        int cu = 0, cp = 1;   // pool fields of (u^n, u^{n-1})
        // Every pool field is zeroed once: a step writes only the grid points
        // of its output, so the zero halo that realises the zero extension
        // must already be there in whichever field it writes.  So is the
        // out-of-place output of the bracket step, which the last trace row
        // samples (a windowed-sinc node outside the grid reads its zero
        // column with weight 0, and 0 times a stale NaN is NaN), and the
        // bracket field.
        for (int i = 0; i < npool; ++i) HIPCHK(launch_zero_field(L, pool[i], g->st, s));
        HIPCHK(launch_zero_field(L, out_f, g->st, s));
        HIPCHK(launch_zero_field(L, brf, Store::F32, s));
        HIPCHK(launch_zero_field(L, g->uA, g->st, s));
        HIPCHK(launch_zero_field(L, g->uB, g->st, s));
        slot_u[0] = cu;
        slot_p[0] = cp;
        ref[cu] = ref[cp] = 1;
        auto free_field = [&]() -> int {
            for (int i = 0; i < npool; ++i)
                if (ref[i] == 0 && i != cu && i != cp) return i;
            return -1;
        };
        for (const fd_ckpt_action &act : plan) {
            switch (act.kind) {
                case FD_ACT_STORE: {
                    if (act.slot < 0 || act.slot >= gp.ncp) return fdi_fail(FD_ERR_STATE, "bad schedule slot");
                    if (slot_u[act.slot] >= 0) {
                        --ref[slot_u[act.slot]];
                        --ref[slot_p[act.slot]];
                    }
                    slot_u[act.slot] = cu;
                    slot_p[act.slot] = cp;
                    ++ref[cu];
                    ++ref[cp];
                    break;
                }
                case FD_ACT_RESTORE:
                    if (act.slot < 0 || act.slot >= gp.ncp || slot_u[act.slot] < 0)
                        return fdi_fail(FD_ERR_STATE, "bad schedule slot");
                    cu = slot_u[act.slot];
                    cp = slot_p[act.slot];
                    break;
                case FD_ACT_ADVANCE:
                    for (int n = act.step; n < act.step + act.count; ++n) {
                        const int out = ref[cp] == 0 ? cp : free_field();
                        if (out < 0) return fdi_fail(FD_ERR_STATE, "checkpoint pool exhausted");
                        a.u = pool[cu];
                        a.prev = pool[cp];
                        a.out = pool[out];
                        a.inj = make_inject(g, 0, sh->src_wavelet + (size_t)n * sh->nsrc, fwd_inj);
                        a.smp = make_sample(g, 1, sh->nrec,
                                            (act.first && n >= 1) ? recb + (size_t)(n - 1) * sh->nrec : nullptr, 1.f);
                        a.nsamp_blocks = samp_blocks(a.smp);
                        a.img = Imaging{};
                        a.ntz = g->ntz[kPlain];
                        a.zchunk = g->zchunk[kPlain];
                        HIPCHK(launch_step(a, g->st, kPlain, s));
                        cp = cu;
                        cu = out;
                    }
                    break;
                case FD_ACT_YOUTURN: {
                    const int n = act.step;
                    if ((rc = bracket_step(n, pool[cu], pool[cp], out_f, brf,
                                           (act.first && n >= 1) ? recb + (size_t)(n - 1) * sh->nrec : nullptr)))
                        return rc;
                    if (act.first) {   // n == nt-1: last trace row, then the residual
                        Sample sm = make_sample(g, 1, sh->nrec, recb + (size_t)(nt - 1) * sh->nrec, 1.f);
                        HIPCHK(launch_sample(sm, out_f, g->st, s));
                        HIPCHK(launch_misfit(recb, d_obs, nres, given, resid, g->partials, kNPart, misfit, s));
                    }
                    if ((rc = adjoint_step(n + 1, brf))) return rc;
                    break;
                }
                default:
                    return fdi_fail(FD_ERR_STATE, "bad schedule action");
            }
        }
    }
    if (adj_done % kFoldEvery) HIPCHK(launch_fold_f64(L, gacc, gpart, s));
    HIPCHK(launch_field_to_dense_f64(L, gacc, (flags & FD_GRAD_VELOCITY) ? g->vel : nullptr, grad_m, s));
    if (src_adj) {
        Sample sm = make_sample(g, 0, sh->nsrc, src_adj, adj_smp);
        HIPCHK(launch_sample(sm, LA, g->st, s));
    }
    if (rec_out)
        HIPCHK(hipMemcpyAsync(rec_out, recb, sizeof(float) * (size_t)nres, hipMemcpyDeviceToDevice, s));
    return FD_OK;
    API_GUARD_END
}
