// fd_internal.h -- device layout and kernel-launch interface shared by the
// host side of libfd (fd_api.cpp, fd_serve.cpp) and its kernels
// (fd_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fd {

constexpr int kMaxR = 8;          // space order 16
constexpr int kMaxSincR = 8;      // windowed-sinc half-width of sparse points
constexpr int kXOff = 64;         // elements before x = 0 in every row (>= kMaxR, 128-B aligned)
constexpr int kTileX = 64;        // x points per 2D tile (16 lanes x 4 points)
constexpr int kTile2Z = 64;       // z rows per 2D tile
constexpr int kBlock = 256;       // threads per workgroup
constexpr int kMaxChunk = 512;    // z planes per 3D workgroup at most
// Largest field whose new time level a step stores with ordinary stores
// rather than non-temporal ones (16-bit 3D fields, 2D diffusion fields): a
// field this small can still sit in the 256 MB memory-side cache when the
// next step reads it.
constexpr size_t kCachedField = size_t(128) << 20;
// Bytes of the static device scratch behind fd_diffusion_run_noalloc (two
// pitched float32 fields: a 2500 x 2500 grid at every space order).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;

// 3D step tiles have tw4 float4 columns per row: 16 (64 x 16 points) or 8
// (32 x 32 points); either way one point quad per lane of a workgroup.  A
// grid's tile shape code is 16 or 8 (every tile so), or kShapeMixed: 64 x 16
// tiles over the whole 64-point x columns and 32 x 32 tiles for the last
// column, when it is at most 32 points wide.
constexpr int kShapeMixed = 0;
inline int tile3_x(int tw4) { return 4 * tw4; }
inline int tile3_y(int tw4) { return kBlock / tw4; }

// Pitched device layout of one field: rows of `pitch` elements, x = 0 at
// element kXOff; `yh` zero rows above and below each plane (r in 3D, 0 in
// 2D); r zero planes before and after the grid.  Halo cells are zeroed once
// and never written, which realises the zero extension of the Laplacian.
struct Layout {
    int ndim;
    int r;
    int nx, ny, nz;       // padded data extents; ny == 1 in 2D (axis 1 of a 2D grid is z)
    int yh;               // y halo rows
    int pitch;            // elements per row
    int nya;              // rows per plane = ny + 2 yh
    int nza;              // planes = nz + 2 r
    long long plane;      // elements per plane = pitch * nya
    long long elems;      // elements per field = plane * nza

    __host__ __device__ long long offset(int x, int y, int z) const {
        return ((long long)(z + r) * nya + (y + yh)) * (long long)pitch + kXOff + x;
    }
};

// Per-tile, per-plane CSR of the grid points that receive a point-source
// term in a step.  The tiles are those of the step kernels (64 x 16 or
// 32 x 32 in xy for 3D, 64 in x for 2D), numbered tile = ty * ntx + tx; in
// the mixed 3D shape the 32 x 32 tiles of the last x column follow, as
// ntx * nty + y / 32.  Corner k lies at
// (x, y) of plane z inside tile t with
//   plane_ptr[t * (nz + 1) + z] <= k < plane_ptr[t * (nz + 1) + z + 1];
// each grid point appears at most once, and its value is
// sum_{e = beg..end-1} w[e] * vals[src[e]].
struct Inject {
    const int *plane_ptr;   // [tiles][nz + 1]
    const int4 *corner;     // (x, y, beg, end)
    const int *src;         // entry -> index into vals
    const float *w;         // entry -> interpolation weight
    const float *vals;      // this step's row of values, nullptr = no injection
    float scale;            // multiplies every value
};

// Sampling of the centre field at sparse points by extra workgroups: `lpp`
// lanes (a power of two, at most 64) share one point.
struct Sample {
    int npts;
    int nc;                 // nodes per point (2^ndim corners or (2r)^ndim sinc nodes)
    int lpp;                // lanes per point
    const long long *idx;   // [npts][nc] element offsets in the pitched layout
    const float *w;         // [npts][nc]
    float *out;             // row of npts outputs, nullptr = no sampling
    float scale;
};

// Workgroups that sample the points of `s` (0 when it samples nothing).
inline int sample_blocks(const Sample &s) {
    if (!s.out || s.npts <= 0) return 0;
    const int per = kBlock / s.lpp;
    return (s.npts + per - 1) / per;
}

// Gradient support (float32 storage).  A recompute step (kBracket) also
// writes, for time n, the imaging bracket
//   br^n = (u^{n+1} - 2 u^n + u^{n-1}) + s (u^{n+1} - u^{n-1}),  s = sigma dt/2,
// from the three levels it holds in registers; an adjoint step (kImage)
// then accumulates grad -= lam^n * br^n for its new value lam^n into a
// float32 partial sum, which the host folds into the float64 gradient every
// few steps.  br and the partial sum use the pitched field layout.
struct Imaging {
    float *br_out;          // kBracket: bracket of the step's time level
    const float *br_in;     // kImage: bracket of the step's time level
    float *gpart;           // kImage: float32 partial sum, folded into float64 by the host loop
};

// kDiff (16-bit 3D storage only): the grid keeps u^n and the difference
// delta = u^n - u^{n-1}; `prev` is the difference field (read at the point),
// `out` receives u^{n+1} and `out2` the new difference (in place of `prev`).
enum StepMode { kPlain = 0, kBracket = 1, kImage = 2, kDiff = 3 };

struct StepArgs {
    Layout L;
    const void *u;          // centre field (read, with halo)
    const void *prev;       // previous field (read)
    void *out;              // new field (may alias prev: in-place update)
    const float *p;         // dt^2 v^2, pitched FP32 (null when pq is set)
    const uint16_t *pq;     // 16-bit code of p, pitched: p = fma(code, pq_step, pq_base)
    float pq_base, pq_step;
    const float *damp;      // sigma dt/2 per index: [nx] x, then [ny] y, then [nz] z
    float w0;               // centre weight sum_a c_0 / h_a^2
    float wx[kMaxR + 1];    // c_j / h_x^2
    float wy[kMaxR + 1];
    float wz[kMaxR + 1];
    int ntx, nty, ntz;      // tiles per axis (3D mixed shape: of the 64 x 16 tiles; ntz counts z chunks)
    int shape3;             // 3D tile shape code: 16, 8 or kShapeMixed
    int nstrip;             // mixed shape: 32 x 32 tiles of the last x column (else 0)
    int out_cached;         // 3D: store u^{n+1} with an ordinary store, not a non-temporal one
    int zchunk;             // planes per 3D workgroup
    int nsamp_blocks;       // trailing workgroups that sample instead of stepping
    Inject inj;
    Sample smp;
    Imaging img;
    // two-level step (k_step3d_t2): u^{n+2} goes to out2 (out receives
    // u^{n+1}); inj2 holds the second level's source row (both levels read
    // the extended tables of inj); smp2 samples the previous field in
    // nsamp_blocks2 workgroups after the nsamp_blocks that sample u
    void *out2;
    Inject inj2;
    Sample smp2;
    int nsamp_blocks2;
};

enum class Store { F32 = 0, F16 = 1, BF16 = 2 };

// Resident workgroups per CU of a step kernel (0 if unknown).
int step_blocks_per_cu(int ndim, int r, Store st, int mode, int shape3, bool pq);

// Launchers (fd_kernels.hip).  Each returns the hipError_t of the launch.
// launch_step reads p from a.pq when that is set (3D, kPlain and kDiff).
hipError_t launch_step(const StepArgs &a, Store st, int mode, hipStream_t s);
// Two leapfrog levels in one launch (3D, float32, radius <= kT2MaxR): 64 x
// 16 tiles (a.ntx, a.nty), a.ntz z chunks of a.zchunk planes; a.inj points
// at the extended per-tile source tables (the grid points within the tile
// grown by R in y and by R rounded up to 4 in x).
constexpr int kT2MaxR = 4;
hipError_t launch_step_t2(const StepArgs &a, hipStream_t s);
int step_t2_blocks_per_cu(int r);
hipError_t launch_sample(const Sample &smp, const void *field, Store st, hipStream_t s);
hipError_t launch_fill_velocity(const Layout &L, const float *vp, int vp_padded, int nbl,
                                const int *phys, float *vel, hipStream_t s);
// out_bits[0] = bits of max v, out_bits[1] = bits of min v over the grid
// points (positive floats order as their bits); the caller sets them to 0
// and to the bits of +inf first.
hipError_t launch_vrange(const Layout &L, const float *vel, unsigned *out_bits, hipStream_t s);
hipError_t launch_make_p(const Layout &L, const float *vel, double dt, float *p, hipStream_t s);
// code = nearest integer in [0, 65535] to (dt^2 v^2 - base) / step, float64
hipError_t launch_make_pq(const Layout &L, const float *vel, double dt, double base, double step,
                          uint16_t *pq, hipStream_t s);
hipError_t launch_zero_field(const Layout &L, void *f, Store st, hipStream_t s);
hipError_t launch_dense_to_field(const Layout &L, const float *dense, void *f, Store st,
                                 float scale, hipStream_t s);
hipError_t launch_field_to_dense(const Layout &L, const void *f, float *dense, Store st,
                                 float scale, hipStream_t s);
// Difference storage: d = round(scale * (a - b)) from two dense fields, and
// dense = (u - d) / scale from the stored value and difference (16-bit).
hipError_t launch_dense_diff_to_field(const Layout &L, const float *a, const float *b, void *d, Store st,
                                      float scale, hipStream_t s);
hipError_t launch_field_diff_to_dense(const Layout &L, const void *u, const void *d, float *dense, Store st,
                                      float scale, hipStream_t s);
// One explicit diffusion step, 2D: out = u + w0 u + sum_j wx_j (..) + wz_j (..)
// (weights already multiplied by nu dt).
hipError_t launch_diffuse2d(const Layout &L, const float *u, float *out, float w0, const float *wx,
                            const float *wz, hipStream_t s);
// Temporally blocked variant: nlev (1 .. diffuse2d_max_levels(r)) steps per launch.
int diffuse2d_max_levels(int r);
hipError_t launch_diffuse2d_tb(const Layout &L, const float *u, float *out, float w0, const float *wx,
                               const float *wz, int nlev, hipStream_t s);
// Address of the static scratch (kStaticScratchBytes) on `device`, which
// must be the current device; resolved with hipGetSymbolAddress on the
// first call per device and kept.
hipError_t static_scratch(int device, void **ptr);
hipError_t launch_misfit(const float *rec, const float *obs, long long n, int residual_given,
                         float *resid, double *partials, int npart, double *out, hipStream_t s);
hipError_t launch_zero_f64(double *p, long long n, hipStream_t s);
// acc += part; part = 0 over the grid rows of two pitched fields of layout L
// (float64 and float32); halo and pad cells are not touched.
hipError_t launch_fold_f64(const Layout &L, double *acc, float *part, hipStream_t s);
// Dense copy of a pitched float64 field; with vel (pitched float32
// velocity, nullable) each value is multiplied by -2 / v^3 in float64.
hipError_t launch_field_to_dense_f64(const Layout &L, const double *f, const float *vel, double *dense,
                                     hipStream_t s);

}  // namespace fd
