// fd_diffusion.cpp -- the thesis's benchmark problem (Section 5.1.2): 2D
// diffusion, first order in time, on the pitched 2D layout of libfd.  A
// host time loop enqueues one tiled step kernel per time step, ping-ponging
// between two workspace fields (the new level cannot overwrite the old one:
// every point of u^n is read by its neighbours' updates).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/fd.h"
#include "fd_api_internal.h"
#include "fd_internal.h"

using namespace fd;

namespace {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool to_grid_desc(const fd_diffusion_desc *d, fd_grid_desc *g) {
    if (!d) return fdi_fail(FD_ERR_ARG, "null descriptor"), false;
    if (!(d->nu > 0.0) || !std::isfinite(d->nu)) return fdi_fail(FD_ERR_ARG, "nu must be > 0"), false;
    if (d->time_block < 0) return fdi_fail(FD_ERR_ARG, "time_block must be >= 0"), false;
    memset(g, 0, sizeof *g);
    g->ndim = 2;
    g->shape[0] = d->shape[0];
    g->shape[1] = d->shape[1];
    g->spacing[0] = d->spacing[0];
    g->spacing[1] = d->spacing[1];
    g->space_order = d->space_order;
    g->storage = FD_STORE_F32;
    return fdi_check_desc(g);
}

// nu dt above this is unstable: 1 / (2 sum_{j odd} c_j (hx^-2 + hy^-2))
double nu_dt_limit(const fd_diffusion_desc *d, int r) {
    double c[kMaxR + 1];
    fdi_second_derivative_weights(r, c);
    double s_odd = 0.0;
    for (int j = 1; j <= r; j += 2) s_odd += c[j];
    const double hx2 = d->spacing[0] * d->spacing[0], hy2 = d->spacing[1] * d->spacing[1];
    return 1.0 / (2.0 * s_odd * (1.0 / hx2 + 1.0 / hy2));
}

}  // namespace

extern "C" int fd_diffusion_dt_limit(const fd_diffusion_desc *desc, double *dt_max) {
    fd_grid_desc g;
    if (!dt_max) return fdi_fail(FD_ERR_ARG, "null output");
    if (!to_grid_desc(desc, &g)) return FD_ERR_ARG;
    *dt_max = nu_dt_limit(desc, desc->space_order / 2) / desc->nu;
    return FD_OK;
}

extern "C" int fd_diffusion_workspace_bytes(const fd_diffusion_desc *desc, size_t *bytes) {
    fd_grid_desc g;
    if (!bytes) return fdi_fail(FD_ERR_ARG, "null output");
    if (!to_grid_desc(desc, &g)) return FD_ERR_ARG;
    const Layout L = fdi_layout(&g);
    *bytes = 2 * align_up(sizeof(float) * (size_t)L.elems, 256);
    return FD_OK;
}

namespace {
int run_diffusion(const fd_diffusion_desc *desc, void *workspace, size_t ws_bytes, const float *u0,
                  float *u_out, int nt, double dt, void *stream) {
    fd_grid_desc g;
    if (!to_grid_desc(desc, &g)) return FD_ERR_ARG;
    if (!workspace || !u0 || !u_out) return fdi_fail(FD_ERR_ARG, "null pointer argument");
    if ((uintptr_t)workspace % 256) return fdi_fail(FD_ERR_ARG, "workspace must be 256-byte aligned");
    if (nt < 0 || !(dt > 0.0) || !std::isfinite(dt)) return fdi_fail(FD_ERR_ARG, "nt >= 0 and dt > 0");
    const Layout L = fdi_layout(&g);
    const size_t fb = align_up(sizeof(float) * (size_t)L.elems, 256);
    if (ws_bytes < 2 * fb) return fdi_fail(FD_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, 2 * fb);
    double c[kMaxR + 1];
    fdi_second_derivative_weights(L.r, c);
    const double hx2 = desc->spacing[0] * desc->spacing[0], hy2 = desc->spacing[1] * desc->spacing[1];
    const double limit = nu_dt_limit(desc, L.r);
    if (desc->nu * dt > limit)
        return fdi_fail(FD_ERR_UNSTABLE, "nu dt %.6g exceeds the explicit limit %.6g", desc->nu * dt, limit);
    hipStream_t s = (hipStream_t)stream;
    float *A = (float *)workspace, *B = (float *)((char *)workspace + fb);
    const double k = desc->nu * dt;
    float wx[kMaxR + 1], wz[kMaxR + 1];
    for (int j = 0; j <= kMaxR; ++j) {
        wx[j] = (j >= 1 && j <= L.r) ? (float)(k * c[j] / hx2) : 0.f;
        wz[j] = (j >= 1 && j <= L.r) ? (float)(k * c[j] / hy2) : 0.f;
    }
    const float w0 = (float)(k * (c[0] / hx2 + c[0] / hy2));
    hipError_t e;
    if ((e = launch_zero_field(L, A, Store::F32, s)) != hipSuccess ||
        (e = launch_zero_field(L, B, Store::F32, s)) != hipSuccess ||
        (e = launch_dense_to_field(L, u0, A, Store::F32, 1.f, s)) != hipSuccess)
        return fdi_fail(FD_ERR_DEVICE, "diffusion setup: %s", hipGetErrorString(e));
    // temporal blocking: each launch advances up to `per` levels from a tile
    // staged with an r*per halo (the thesis's OPS tiling / YASK wave-front
    // tiling idea, Section 2.2 and 2.3.1, in LDS)
    // Automatic choice (measured on 2500^2 and 10000^2 for every radius and
    // level count): 8 levels at radius 1 and 2, 4 at radius 4; at the other
    // radii the redundant halo levels cost more than the HBM traffic they
    // save, and one step per launch is faster.
    int per = diffuse2d_max_levels(L.r);
    if (desc->time_block > 0) per = std::min(per, desc->time_block);
    else per = (L.r == 1 || L.r == 2) ? 8 : L.r == 4 ? 4 : 1;
    for (int n = 0; n < nt;) {
        const int lev = std::min(per, nt - n);
        if (per <= 1)
            e = launch_diffuse2d(L, A, B, w0, wx, wz, s);
        else
            e = launch_diffuse2d_tb(L, A, B, w0, wx, wz, lev, s);
        if (e != hipSuccess) return fdi_fail(FD_ERR_DEVICE, "diffusion step: %s", hipGetErrorString(e));
        std::swap(A, B);
        n += lev;
    }
    if ((e = launch_field_to_dense(L, A, u_out, Store::F32, 1.f, s)) != hipSuccess)
        return fdi_fail(FD_ERR_DEVICE, "diffusion readback: %s", hipGetErrorString(e));
    return FD_OK;
}
}  // namespace

extern "C" int fd_diffusion_run(const fd_diffusion_desc *desc, void *workspace, size_t ws_bytes,
                                const float *u0, float *u_out, int nt, double dt, void *stream) {
    return run_diffusion(desc, workspace, ws_bytes, u0, u_out, nt, dt, stream);
}

extern "C" int fd_diffusion_run_noalloc(const fd_diffusion_desc *desc, const float *u0, float *u_out, int nt,
                                        double dt, void *stream) {
    fd_grid_desc g;
    if (!to_grid_desc(desc, &g)) return FD_ERR_ARG;
    const Layout L = fdi_layout(&g);
    const size_t need = 2 * align_up(sizeof(float) * (size_t)L.elems, 256);
    if (need > kStaticScratchBytes)
        return fdi_fail(FD_ERR_NOMEM, "grid needs %zu scratch bytes, above the static maximum of %zu", need,
                        kStaticScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fdi_fail(FD_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    void *ws = nullptr;
    if ((e = static_scratch(dev, &ws)) != hipSuccess)
        return fdi_fail(FD_ERR_DEVICE, "static scratch of device %d: %s", dev, hipGetErrorString(e));
    return run_diffusion(desc, ws, kStaticScratchBytes, u0, u_out, nt, dt, stream);
}
