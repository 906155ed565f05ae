// fd_kernels.hip -- gfx950 kernels of libfd.
//
// The hot loop is the per-step space loop of an explicit finite-difference
// stepper (the thesis launches one data-parallel loop per time step from a
// host time loop, Section 3.3.3 "Parallel loop invocation"); here one launch
// of k_step3d / k_step2d performs the whole step:
//
//   lap  = w0 u + sum_j wx_j (u_{x+j} + u_{x-j}) + wy_j (..) + wz_j (..)
//   s    = sigma dt / 2                     (per-axis tables, 0 off the layer)
//   unew = (2u - (1 - s) uprev + p (lap + src)) / (1 + s),  p = dt^2 v^2
//
// with the point-source term `src` added by the thread that owns the point
// and the receiver sampling of the centre field done by extra workgroups of
// the same launch.  All weights are precomputed on the host (no division in
// the inner loop: the lesson of the aggressive-DSE kernel of Section 5.1.5).
//
// 3D: 2.5D blocking.  A workgroup owns a 64 x 16 or a 32 x 32 xy tile and
// marches a chunk of z planes.  Each lane keeps 4 consecutive x points and a register queue
// of the 2r+1 z values of its column; the current xy plane (tile + r halo) is
// staged through LDS (double-buffered, one barrier per plane) for the x and y
// neighbours.  Loads of plane z+1 are issued before plane z is computed.
// Arithmetic is FP32 whatever the storage type.  No MFMA: the update is a
// star stencil, not a contraction, and is bound by HBM bandwidth.  The 3D
// step's device code is in fd_step3d.h, its instantiations in the
// fd_step3d_*.hip units (one per storage type and form).
#include "fd_step3d.h"

#include <stdint.h>

#include <mutex>
#include <type_traits>

// Device scratch of the allocation-free diffusion entry point: a fixed
// array in the code object, one copy per GPU, reached from host code only
// through the address hipGetSymbolAddress returns for the current device
// (see fd::static_scratch); the name itself is not a device address there.
static __device__ __align__(256) unsigned char scratch[fd::kStaticScratchBytes];

namespace fd {
namespace {

// ------------------------------------------------------ 3D two-level step
// Temporal blocking of the 2.5D march (the wave-front tiling of Section
// 2.3.1 and the tiling of Section 2.2, done in registers and LDS): from u^n
// and u^{n-1} a workgroup computes level 1, u^{n+1}, on its 64 x 16 tile
// grown by a ring of R points (the ring belongs to the neighbour tiles and
// is recomputed here, so that no workgroup waits for another), and level 2,
// u^{n+2}, on its tile, R planes behind level 1 in the z march.  It writes
// u^{n+1} and u^{n+2} of its tile: per point and two steps HBM carries u^n,
// u^{n-1} and p in and two fields out, 10 bytes per point-step instead of
// 16.  The outputs go to a second pair of fields (u^n and u^{n-1} are read
// as the neighbours' ring until the launch ends).  Each level is the same
// sequence of float32 operations as the one-step kernel's, so two levels
// here give bitwise the fields of two one-step launches.
template <int R>
struct T2Shape {
    static constexpr int TW = 16, TY = 16;                   // tile: 16 float4 columns x 16 rows
    static constexpr int HX4 = (R + 3) / 4;                  // float4 columns of an R-point ring in x
    static constexpr int W1 = TW + 2 * HX4, H1 = TY + 2 * R;    // level-1 region E1 (float4 x rows)
    static constexpr int W2 = W1 + 2 * HX4, H2 = H1 + 2 * R;    // staged u^n plane E2
    static constexpr int N1 = W1 * H1, N2 = W2 * H2;
    static constexpr int NR1 = N1 - TW * TY;                 // ring groups of E1
    static constexpr int NR1L = TY * 2 * HX4;                // ... of which in the tile's rows
    static constexpr int NS = 1 + (NR1 + kBlock - 1) / kBlock;  // level-1 groups per lane (0: own)
    static constexpr int NR2 = N2 - N1;                      // ring groups of E2 (u^n only)
    static constexpr int NR2L = H1 * 2 * HX4;
    static constexpr int HP2 = (NR2 + kBlock - 1) / kBlock;
    static constexpr int NQ = 2 * R + 1;
    static constexpr int kMaxPl = kMaxChunk + 2 * R;         // level-1 planes of a chunk
    // LDS, in float4 (at radius 4 just under the 80 KB that lets two
    // workgroups share a CU); the level-1 source terms of a plane are
    // scattered into the staging buffer the next plane will use, idle then
    static constexpr int kU = 0;                             // [2][N2] staged u^n planes
    static constexpr int kV = kU + 2 * N2;                   // [R + 1][N1] ring of u^{n+1} planes
    static constexpr int kP = kV + (R + 1) * N1;             // [R + 1][NR2] parked E2 ring of u^n
    static constexpr int kS2 = kP + (R + 1) * NR2;           // [kBlock] level-2 source terms
    static constexpr int kDz = kS2 + kBlock;                 // float [kMaxPl] z damping of level-1 planes
    static constexpr int kPp = kDz + kMaxPl / 4;             // int [kMaxPl + 1] source plane pointers
    static constexpr int kSize = kPp + (kMaxPl + 1 + 3) / 4;
};

// Ring group h of a region W x H (float4 x rows) around an inner block of
// IW x IH starting at (HX, RY): the RY rows above (full width), then HX
// columns left and right of each inner row, then the RY rows below.
template <int W, int H, int IW, int IH, int HX, int RY>
__device__ inline void ring_pos(int h, int &cx, int &cy) {
    if (h < RY * W) {
        cy = h / W;
        cx = h - cy * W;
    } else if (h < RY * W + IH * 2 * HX) {
        const int j = h - RY * W;
        const int row = j / (2 * HX), c = j - row * (2 * HX);
        cy = RY + row;
        cx = c < HX ? c : IW + c;
    } else {
        const int j = h - RY * W - IH * 2 * HX;
        cy = RY + IH + j / W;
        cx = j - (j / W) * W;
    }
}

template <int R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_step3d_t2(const StepArgs a) {
    using K = T2Shape<R>;
    constexpr int TW = K::TW, TY = K::TY, HX4 = K::HX4, W1 = K::W1, W2 = K::W2, N1 = K::N1, N2 = K::N2;
    constexpr int NS = K::NS, HP2 = K::HP2, NQ = K::NQ;
    __shared__ float4 smem[K::kSize];
    const int ntile = (int)gridDim.x - a.nsamp_blocks - a.nsamp_blocks2;
    if ((int)blockIdx.x >= ntile) {
        const int b = (int)blockIdx.x - ntile;
        if (b < a.nsamp_blocks)
            sample_block<Store::F32>(a.smp, a.u, b);
        else
            sample_block<Store::F32>(a.smp2, a.prev, b - a.nsamp_blocks);
        return;
    }
    const int t = xcd_remap((int)blockIdx.x, ntile);
    const int tiles = a.ntx * a.nty;
    const int tid = t % tiles, bz = t / tiles;
    const int x0 = (tid % a.ntx) * 4 * TW, y0 = (tid / a.ntx) * TY;
    const Layout L = a.L;
    const int c0 = bz * a.zchunk, c1 = min(c0 + a.zchunk, L.nz);
    const int zl0 = c0 - R;                  // level-1 plane of the first iteration
    const int npl = c1 - c0 + 2 * R;         // iterations: level-1 planes [c0 - R, c1 + R)
    const int lane = (int)threadIdx.x;
    const long long plane = L.plane;
    const long long zcol = L.offset((L.nx + 3) & ~3, 0, 0);   // zero in every row of every plane
    const float *__restrict__ U = (const float *)a.u;
    const float *Pv = (const float *)a.prev;
    const float *__restrict__ Pp = a.p;
    float *O1 = (float *)a.out;
    float *O2 = (float *)a.out2;

    float4 *stg = smem + K::kU;
    float4 *ring = smem + K::kV;
    float4 *park = smem + K::kP;
    float4 *s_src2 = smem + K::kS2;
    float *s_dz = reinterpret_cast<float *>(smem + K::kDz);
    int *s_pp = reinterpret_cast<int *>(smem + K::kPp);
    // per-plane tables of the chunk's level-1 planes (z damping; source plane
    // pointers, which give no sources outside the grid)
    const int *tile_pp = a.inj.plane_ptr + (long long)tid * (L.nz + 1);
    for (int i = lane; i <= npl; i += kBlock) {
        const int z = zl0 + i;
        if (i < npl) s_dz[i] = (z >= 0 && z < L.nz) ? a.damp[L.nx + L.ny + z] : 0.f;
        s_pp[i] = a.inj.vals ? tile_pp[min(max(z, 0), L.nz)] : 0;
    }
    s_src2[lane] = make_float4(0.f, 0.f, 0.f, 0.f);

    // level-1 groups of this lane: slot 0 its own tile group, slots 1.. ring
    // groups of E1; grid coordinates, E1 and E2 indices, validity
    const int tx = lane % TW, ty = lane / TW;
    int e1i[NS], e2i[NS], gxs[NS];
    bool in1[NS];
    long long off[NS];
    float sxy[NS][4];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        int cx = HX4 + tx, cy = R + ty;
        bool used = true;
        if (k > 0) {
            const int h = lane + (k - 1) * kBlock;
            used = h < K::NR1;
            ring_pos<W1, K::H1, TW, TY, HX4, R>(used ? h : 0, cx, cy);
        }
        const int gx = x0 - 4 * HX4 + 4 * cx, gy = y0 - R + cy;
        in1[k] = used && gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny;
        e1i[k] = used ? cy * W1 + cx : -1;
        e2i[k] = (cy + R) * W2 + cx + HX4;
        gxs[k] = gx;
        off[k] = in1[k] ? L.offset(gx, gy, 0) : zcol;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            sxy[k][i] = in1[k] ? a.damp[min(gx + i, L.nx - 1)] + a.damp[L.nx + gy] : 0.f;
    }
    // the E2 ring of u^n (staged for level 1's x and y neighbours only)
    int h2i[HP2];
    long long hoff[HP2];
#pragma unroll
    for (int k = 0; k < HP2; ++k) {
        const int h = lane + k * kBlock;
        int cx = 0, cy = 0;
        ring_pos<W2, K::H2, W1, K::H1, HX4, R>(h < K::NR2 ? h : 0, cx, cy);
        const int gx = x0 - 8 * HX4 + 4 * cx, gy = y0 - 2 * R + cy;
        const bool ok = h < K::NR2 && gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny;
        h2i[k] = h < K::NR2 ? cy * W2 + cx : -1;
        hoff[k] = ok ? L.offset(gx, gy, 0) : zcol;
    }
    const bool act = in1[0];                      // the lane's tile group is inside the grid
    const int nvalid = L.nx - gxs[0];

    auto zclamp = [&](int z) { return min(max(z, -R), L.nz + R - 1); };
    // z queues: q[k][j] = u^n of slot k at plane zl - R + j; w[j] = u^{n+1}
    // of slot 0 at plane zl - 2R + j; pq[j] = p of slot 0 at plane zl - R + j
    float4 q[NS][NQ], w[NQ], pq[R + 1];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) q[k][j] = Elem<Store::F32>::ld4(U + off[k] + (long long)zclamp(c0 - 2 * R + j) * plane);
#pragma unroll
    for (int j = 0; j < NQ; ++j) w[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    // The E2 ring of plane z belongs to neighbour tiles, which fetch plane z
    // as their queue front R planes before this tile stages it; it is loaded
    // with this tile's own fronts (plane zl + R), when the neighbours' fetch
    // can serve it from L2, and parked in LDS slot (iteration + R) mod (R+1)
    // until staged.  The first R planes are parked here.
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
        for (int k = 0; k < HP2; ++k)
            if (h2i[k] >= 0)
                park[j * K::NR2 + k * kBlock + lane] = Elem<Store::F32>::ld4(U + hoff[k] + (long long)zclamp(zl0 + j) * plane);
#pragma unroll
    for (int j = 0; j <= R; ++j) pq[j] = make_float4(0.f, 0.f, 0.f, 0.f);

    struct Pre {
        float4 front[NS], mv[NS], pv[NS], h2[HP2];
    };
    // u^{n-1} and p use ordinary loads: the ring's values are read by the
    // neighbour tiles in the same plane step, and their fetch should find
    // the line in L2 (non-temporal loads here doubled the bytes read).
    auto issue = [&](Pre &r, int it) __attribute__((always_inline)) {
        it = min(it, npl - 1);   // past the chunk: a harmless in-bounds reload
        const int zl = zl0 + it;
        const long long fo = (long long)zclamp(zl + R) * plane, zo = (long long)zclamp(zl) * plane;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            r.front[k] = Elem<Store::F32>::ld4(U + off[k] + fo);
            r.mv[k] = Elem<Store::F32>::ld4(Pv + off[k] + zo);
            r.pv[k] = Elem<Store::F32>::ld4(Pp + off[k] + zo);
        }
#pragma unroll
        for (int k = 0; k < HP2; ++k) r.h2[k] = Elem<Store::F32>::ld4(U + hoff[k] + fo);
    };

    // The Laplacian of one group: x neighbours from an LDS row (the group's
    // own value xc in the middle), y neighbours j rows up and down, z from
    // the queue; the same fused multiply-adds in the same order as the
    // one-step kernel.
    auto laplace = [&](const float4 *row, int rowpitch, const float4 &xc, const float4 *zq, float lap[4])
        __attribute__((always_inline)) {
        float xs[4 * (2 * HX4 + 1)];
#pragma unroll
        for (int c = -HX4; c <= HX4; ++c) {
            const float4 v = (c == 0) ? xc : row[c];
            xs[4 * (c + HX4) + 0] = v.x;
            xs[4 * (c + HX4) + 1] = v.y;
            xs[4 * (c + HX4) + 2] = v.z;
            xs[4 * (c + HX4) + 3] = v.w;
        }
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const float4 yp = row[j * rowpitch], ym = row[-j * rowpitch];
            const float4 zp = zq[R + j], zm = zq[R - j];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float xsum = xs[4 * HX4 + i + j] + xs[4 * HX4 + i - j];
                lap[i] = j == 1 ? a.wx[1] * xsum : __builtin_fmaf(a.wx[j], xsum, lap[i]);
                lap[i] = __builtin_fmaf(a.wy[j], comp(yp, i) + comp(ym, i), lap[i]);
                lap[i] = __builtin_fmaf(a.wz[j], comp(zp, i) + comp(zm, i), lap[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) lap[i] = __builtin_fmaf(a.w0, xs[4 * HX4 + i], lap[i]);
    };

    auto body = [&](int it, const Pre &cur, Pre &nxt) __attribute__((always_inline)) {
        const int zl = zl0 + it;
        float4 *st = stg + (it & 1) * N2;
        float *s_src1 = reinterpret_cast<float *>(stg + ((it + 1) & 1) * N2);   // idle this plane
        float4 *park_w = park + ((it + R) % (R + 1)) * K::NR2 + lane;
        const float4 *park_r = park + (it % (R + 1)) * K::NR2 + lane;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            q[k][2 * R] = cur.front[k];
            if (e1i[k] >= 0) st[e2i[k]] = q[k][R];
        }
#pragma unroll
        for (int k = 0; k < HP2; ++k) {
            if (h2i[k] >= 0) {
                park_w[k * kBlock] = cur.h2[k];
                st[h2i[k]] = park_r[k * kBlock];
            }
        }
        issue(nxt, it + 1);
        // sources: level 1 at plane zl (the extended tables, row n), level 2
        // at plane zl - R (the tile's points of the same tables, row n + 1)
        const bool lev2 = it >= 2 * R;
        const int e0 = __builtin_amdgcn_readfirstlane(s_pp[it]);
        const int e1 = __builtin_amdgcn_readfirstlane(s_pp[it + 1]);
        const int f0 = lev2 ? __builtin_amdgcn_readfirstlane(s_pp[it - R]) : 0;
        const int f1 = lev2 ? __builtin_amdgcn_readfirstlane(s_pp[it - R + 1]) : 0;
        if (e0 < e1) {
            // The buffer held the previous plane's staged values: every wave
            // is past reading them, then it is cleared.  (On such a plane
            // the barrier at its end keeps the next plane's staging from
            // overwriting the terms before they are read.)
            __syncthreads();
            for (int i = lane; i < N1; i += kBlock) reinterpret_cast<float4 *>(s_src1)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            __syncthreads();
            for (int e = e0 + lane; e < e1; e += kBlock) {
                const int4 c = a.inj.corner[e];
                float v = 0.f;
                for (int k = c.z; k < c.w; ++k) v = __builtin_fmaf(a.inj.w[k], a.inj.vals[a.inj.src[k]], v);
                s_src1[(c.y - (y0 - R)) * (4 * W1) + (c.x - (x0 - 4 * HX4))] = v * a.inj.scale;
            }
        }
        if (f0 < f1) {
            for (int e = f0 + lane; e < f1; e += kBlock) {
                const int4 c = a.inj.corner[e];
                if (c.x >= x0 && c.x < x0 + 4 * TW && c.y >= y0 && c.y < y0 + TY) {
                    float v = 0.f;
                    for (int k = c.z; k < c.w; ++k) v = __builtin_fmaf(a.inj2.w[k], a.inj2.vals[a.inj2.src[k]], v);
                    reinterpret_cast<float *>(s_src2)[(c.y - y0) * (4 * TW) + (c.x - x0)] = v * a.inj2.scale;
                }
            }
        }
        __syncthreads();
        // level 1 on every slot of the lane, zero outside the grid
        const bool in_z = zl >= 0 && zl < L.nz;
        const float sz1 = s_dz[it];
        float4 *rw = ring + (it % (R + 1)) * N1;
        float4 v1[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            v1[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (k == 0 || e1i[k] >= 0) {
                float lap[4];
                laplace(st + e2i[k], W2, q[k][R], q[k], lap);
                float4 src4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (e0 < e1 && e1i[k] >= 0) src4 = reinterpret_cast<const float4 *>(s_src1)[e1i[k]];
                const float src[4] = {src4.x, src4.y, src4.z, src4.w};
                float un[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float u1 = update_point(comp(q[k][R], i), comp(cur.mv[k], i), comp(cur.pv[k], i), lap[i],
                                                  src[i], sxy[k][i] + sz1);
                    un[i] = (in_z && in1[k] && gxs[k] + i < L.nx) ? u1 : 0.f;
                }
                asm volatile("" ::"v"(un[0]), "v"(un[1]), "v"(un[2]), "v"(un[3]));
                v1[k] = make_float4(un[0], un[1], un[2], un[3]);
            }
            if (e1i[k] >= 0) rw[e1i[k]] = v1[k];
        }
        w[2 * R] = v1[0];
        pq[R] = cur.pv[0];
        // u^{n+1} of the tile, for the planes of this chunk
        if (act && zl >= c0 && zl < c1) {
            const long long o = off[0] + (long long)zl * plane;
            if (nvalid >= 4) {
                st4nt_f32(O1 + o, v1[0]);
            } else {
                const float rv[3] = {v1[0].x, v1[0].y, v1[0].z};
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (i < nvalid) O1[o + i] = rv[i];
            }
        }
        // level 2 at plane zl - R: x and y neighbours from the u^{n+1} plane
        // written R iterations ago, z from the lane's queue, u^n from the
        // bottom of its u^n queue
        if (lev2) {
            float4 src4 = make_float4(0.f, 0.f, 0.f, 0.f);
            if (f0 < f1) {
                src4 = s_src2[lane];
                s_src2[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            if (act) {
                const float4 *rr = ring + ((it - R) % (R + 1)) * N1 + e1i[0];
                float lap[4];
                laplace(rr, W1, w[R], w, lap);
                const float src[4] = {src4.x, src4.y, src4.z, src4.w};
                const float sz2 = s_dz[it - R];
                float un[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    un[i] = update_point(comp(w[R], i), comp(q[0][0], i), comp(pq[0], i), lap[i], src[i],
                                         sxy[0][i] + sz2);
                asm volatile("" ::"v"(un[0]), "v"(un[1]), "v"(un[2]), "v"(un[3]));
                const long long o = off[0] + (long long)(zl - R) * plane;
                if (nvalid >= 4) {
                    st4nt_f32(O2 + o, make_float4(un[0], un[1], un[2], un[3]));
                } else {
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        if (i < nvalid) O2[o + i] = un[i];
                }
            }
        }
        if (e0 < e1 || f0 < f1) __syncthreads();   // read (and level 2's cleared) before the buffers are reused
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) q[k][j] = q[k][j + 1];
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) w[j] = w[j + 1];
#pragma unroll
        for (int j = 0; j < R; ++j) pq[j] = pq[j + 1];
    };

    __syncthreads();   // staged tables and cleared source buffers, before the first plane
    Pre p0, p1;
    issue(p0, 0);
    int it = 0;
    for (; it + 2 <= npl; it += 2) {
        body(it, p0, p1);
        body(it + 1, p1, p0);
    }
    if (it < npl) body(it, p0, p1);
}

// ------------------------------------------------------------------ 2D step
// Grid axes (x, z); tile 64 x 64 staged whole in LDS with an r halo; each
// lane computes 4 x points in each of 4 rows.
template <int R, Store S, int MODE>
__global__ __launch_bounds__(kBlock) void k_step2d(const StepArgs a) {
    using E = Elem<S>;
    using T = typename E::T;
    constexpr int HX4 = (R + 3) / 4;
    constexpr int W4 = 16 + 2 * HX4;
    constexpr int LH = kTile2Z + 2 * R;
    __shared__ float4 lds[LH * W4];

    const Layout L = a.L;
    const int ntile = (int)gridDim.x - a.nsamp_blocks;   // tiles first, then sampling
    if ((int)blockIdx.x >= ntile) {
        sample_block<S>(a.smp, a.u, (int)blockIdx.x - ntile);
        return;
    }
    const int t = xcd_remap((int)blockIdx.x, ntile);
    const int bx = t % a.ntx, bz = t / a.ntx;
    const int x0 = bx * kTileX, z0 = bz * kTile2Z;
    const int z1 = min(z0 + kTile2Z, L.nz);
    const int lane = (int)threadIdx.x;
    __shared__ float s_dz[kTile2Z];
    __shared__ int s_pp[kTile2Z + 1];
    const int *tile_pp = a.inj.plane_ptr + (long long)bx * (L.nz + 1);
    for (int i = lane; i <= z1 - z0; i += kBlock) {
        if (i < z1 - z0) s_dz[i] = a.damp[L.nx + L.ny + z0 + i];
        s_pp[i] = a.inj.vals ? tile_pp[z0 + i] : 0;
    }
    const T *U = (const T *)a.u;
    const long long zcol = L.offset((L.nx + 3) & ~3, 0, 0);   // zero in every row

    for (int i = lane; i < LH * W4; i += kBlock) {
        const int lr = i / W4, c = i - lr * W4;
        const int gz = z0 - R + lr, gx = x0 - 4 * HX4 + 4 * c;
        const bool ok = gz >= 0 && gz < L.nz && gx >= 0 && gx < L.nx;
        lds[i] = E::ld4(U + (ok ? L.offset(gx, 0, gz) : zcol));
    }
    __syncthreads();

    const int tx = lane & 15, tz = lane >> 4;
    const int x = x0 + 4 * tx;
    if (x >= L.nx) return;
    const int nvalid = L.nx - x;
    float sx[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) sx[i] = a.damp[min(x + i, L.nx - 1)];
    const T *Pv = (const T *)a.prev;
    T *O = (T *)a.out;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int z = z0 + tz * 4 + rr;
        if (z >= L.nz) break;
        const float4 *row = lds + (R + tz * 4 + rr) * W4 + HX4 + tx;
        float xs[4 * (2 * HX4 + 1)];
#pragma unroll
        for (int c = -HX4; c <= HX4; ++c) {
            const float4 v = row[c];
            xs[4 * (c + HX4) + 0] = v.x;
            xs[4 * (c + HX4) + 1] = v.y;
            xs[4 * (c + HX4) + 2] = v.z;
            xs[4 * (c + HX4) + 3] = v.w;
        }
        float lap[4];
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const float4 zp = row[j * W4], zm = row[-j * W4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float t = lap_term2(a.wx[j], xs[4 * HX4 + i + j] + xs[4 * HX4 + i - j], a.wz[j],
                                          comp(zp, i) + comp(zm, i));
                lap[i] = j == 1 ? t : lap[i] + t;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) lap[i] = __builtin_fmaf(a.w0, xs[4 * HX4 + i], lap[i]);
        float src[4] = {0.f, 0.f, 0.f, 0.f};
        const int e0 = s_pp[z - z0], e1 = s_pp[z - z0 + 1];
        if (e0 < e1) gather_sources(a.inj, e0, e1, x, src[0], src[1], src[2], src[3]);
        const long long off = L.offset(x, 0, z);
        const float4 pc = ld4nt_f32(a.p + off);
        const float4 mc = E::ld4nt(Pv + off);
        const float4 cc = row[0];
        const float sz = s_dz[z - z0];
        float un[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            un[i] = update_point(comp(cc, i), comp(mc, i), comp(pc, i), lap[i], src[i], sx[i] + sz);
        if constexpr (S != Store::F32)   // round to float32, then to 16 bits (no fused conversion)
            asm volatile("" : "+v"(un[0]), "+v"(un[1]), "+v"(un[2]), "+v"(un[3]));
        if (nvalid >= 4) {
            E::st4nt(O + off, make_float4(un[0], un[1], un[2], un[3]));
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < nvalid) E::st(O + off + i, un[i]);
        }
        if constexpr (MODE != kPlain) {
            float sv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) sv[i] = sx[i] + sz;
            grad_epilogue<MODE>(a.img, off, nvalid, un, cc, mc, sv);
        }
    }
}

// ------------------------------------------------------- 2D diffusion step
// The thesis's benchmark operator: one forward-Euler step of u_t = nu Lap u.
// Tile 64 x 64 staged in LDS with an r halo; each lane updates 4 x points in
// each of 4 rows.  Weights carry nu dt (hoisted on the host, no division).
struct DiffArgs {
    Layout L;
    const float *u;
    float *out;
    float w0;
    float wx[kMaxR + 1];
    float wz[kMaxR + 1];
    int ntx, ntz;
    int out_cached;   // ordinary stores of the new level (small fields), else non-temporal
};

template <int R>
__global__ __launch_bounds__(kBlock) void k_diffuse2d(const DiffArgs a) {
    constexpr int HX4 = (R + 3) / 4;
    constexpr int W4 = 16 + 2 * HX4;
    constexpr int LH = kTile2Z + 2 * R;
    __shared__ float4 lds[LH * W4];
    const Layout L = a.L;
    const int t = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int bx = t % a.ntx, bz = t / a.ntx;
    const int x0 = bx * kTileX, z0 = bz * kTile2Z;
    const int lane = (int)threadIdx.x;
    const long long zcol = L.offset((L.nx + 3) & ~3, 0, 0);
    for (int i = lane; i < LH * W4; i += kBlock) {
        const int lr = i / W4, c = i - lr * W4;
        const int gz = z0 - R + lr, gx = x0 - 4 * HX4 + 4 * c;
        const bool ok = gz >= 0 && gz < L.nz && gx >= 0 && gx < L.nx;
        lds[i] = *reinterpret_cast<const float4 *>(a.u + (ok ? L.offset(gx, 0, gz) : zcol));
    }
    __syncthreads();
    const int tx = lane & 15, tz = lane >> 4;
    const int x = x0 + 4 * tx;
    if (x >= L.nx) return;
    const int nvalid = L.nx - x;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int z = z0 + tz * 4 + rr;
        if (z >= L.nz) break;
        const float4 *row = lds + (R + tz * 4 + rr) * W4 + HX4 + tx;
        float xs[4 * (2 * HX4 + 1)];
#pragma unroll
        for (int c = -HX4; c <= HX4; ++c) {
            const float4 v = row[c];
            xs[4 * (c + HX4) + 0] = v.x;
            xs[4 * (c + HX4) + 1] = v.y;
            xs[4 * (c + HX4) + 2] = v.z;
            xs[4 * (c + HX4) + 3] = v.w;
        }
        float un[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) un[i] = a.w0 * xs[4 * HX4 + i];
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const float4 zp = row[j * W4], zm = row[-j * W4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float acc = a.wx[j] * (xs[4 * HX4 + i + j] + xs[4 * HX4 + i - j]);
                acc += a.wz[j] * (comp(zp, i) + comp(zm, i));
                un[i] += acc;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) un[i] += xs[4 * HX4 + i];
        const long long off = L.offset(x, 0, z);
        if (nvalid >= 4) {
            const float4 r4 = make_float4(un[0], un[1], un[2], un[3]);
            if (a.out_cached)
                *reinterpret_cast<float4 *>(a.out + off) = r4;
            else
                st4nt_f32(a.out + off, r4);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < nvalid) a.out[off + i] = un[i];
        }
    }
}

// Temporally blocked diffusion: one launch advances `nlev` (<= 16/R) levels.
// A workgroup stages its 64 x 64 output tile plus an H = R*nlev halo in z and
// an H rounded up to a multiple of 4 in x (zero outside the grid; the
// rounding keeps every staged row and the written tile on 16-byte
// boundaries at odd H) in one LDS buffer and updates it in place level by
// level on the shrinking region that stays exact: level t is computed on
// rows and 4-point groups at least R*t from the staged border (rounded out
// to whole groups; the rounding margin holds values that nothing exact
// reads).  Between levels each lane keeps its new values in registers
// across a barrier, so one buffer suffices.  HBM traffic: 8 B per point per
// launch, i.e. 8/nlev B per point and step.
constexpr int kTbHalo = 16;                        // R * levels per launch, at most
constexpr int kTbRows = kTile2Z + 2 * kTbHalo;     // 96 staged rows
constexpr int kTbPadX = 4;                         // zero floats left/right of a staged row
constexpr int kTbW4 = (kTileX + 2 * kTbHalo + 2 * kTbPadX) / 4;   // float4 per staged row
constexpr int kTbPerLane = (kTbRows * kTbW4 + kBlock - 1) / kBlock;   // staged float4 groups per lane

// The LDS buffer (40 KB) allows four workgroups, i.e. four waves per SIMD.
// At radii 3, 5 and 7 the compiler's own allocation (137-154 VGPRs) allows
// only three, so those radii are held to four waves per SIMD (97-101 VGPRs,
// no spills: 5-15 % faster); at the other radii the default allocation
// already fits four waves, and the same bound made radius 2 slower.

template <int R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((R & 1) && R > 1 ? 4 : 1))) void k_diffuse2d_tb(const DiffArgs a, int nlev) {
    __shared__ float4 lds[kTbRows * kTbW4];
    const Layout L = a.L;
    const int t0 = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int bx = t0 % a.ntx, bz = t0 / a.ntx;
    const int H = R * nlev;                       // staged halo of this launch in z
    const int Hx = (H + 3) & ~3;                  // and in x, whole float4 groups
    const int x0 = bx * kTileX - Hx, z0 = bz * kTile2Z - H;   // grid coords of staged (0, 0)
    const int rows = kTile2Z + 2 * H;
    const int g4 = kTbW4;                         // staged float4 per row: the full LDS row, so every
                                                  // neighbour group a level reads holds grid data or zero
    const int lane = (int)threadIdx.x;
    // stage level 0; float4 column c covers grid x = x0 - 4 + 4c (a float4
    // load when that is 16-B aligned in the grid, else element by element)
    for (int i = lane; i < rows * g4; i += kBlock) {
        const int lr = i / g4, c = i - lr * g4;
        const int gz = z0 + lr, gx = x0 - kTbPadX + 4 * c;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gz >= 0 && gz < L.nz && gx + 3 >= 0 && gx < L.nx) {
            if (gx >= 0 && (gx & 3) == 0) {
                v = *reinterpret_cast<const float4 *>(a.u + L.offset(gx, 0, gz));
            } else {
                float e[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int xx = gx + k;
                    e[k] = (xx >= 0 && xx < L.nx) ? a.u[L.offset(xx, 0, gz)] : 0.f;
                }
                v = make_float4(e[0], e[1], e[2], e[3]);
            }
        }
        lds[lr * kTbW4 + c] = v;
    }
    __syncthreads();
    const float *ldsf = reinterpret_cast<const float *>(lds);
    // Each lane owns fixed float4 groups of the staged tile (row-major with
    // the constant row stride, so the index split is a multiply-shift); a
    // level updates the groups inside its exact region.  Neighbours are read
    // as whole float4 groups: x from the 2 ceil(R/4) + 1 groups of the row,
    // z from the groups j rows up and down (conflict-free 16-byte LDS reads).
    constexpr int HX4 = (R + 3) / 4;
    for (int t = 1; t <= nlev; ++t) {
        // level t region: rows [R t, rows - R t), float4 columns [c0, c1)
        const int r0 = R * t, r1 = rows - R * t;
        const int c0 = 1 + (R * t) / 4;                        // first float4 column (pad column is 0)
        const int c1 = 1 + (kTileX + 2 * Hx - R * t + 3) / 4;  // one past the last
        float4 res[kTbPerLane];
#pragma unroll
        for (int k = 0; k < kTbPerLane; ++k) {
            const int gidx = lane + k * kBlock;
            const int lr = gidx / kTbW4, c = gidx - lr * kTbW4;
            res[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (lr >= r0 && lr < r1 && c >= c0 && c < c1) {
                const float4 *row = lds + lr * kTbW4 + c;
                float xs[4 * (2 * HX4 + 1)];
#pragma unroll
                for (int q = -HX4; q <= HX4; ++q) {
                    const float4 v = row[q];
                    xs[4 * (q + HX4) + 0] = v.x;
                    xs[4 * (q + HX4) + 1] = v.y;
                    xs[4 * (q + HX4) + 2] = v.z;
                    xs[4 * (q + HX4) + 3] = v.w;
                }
                float un[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) un[i] = a.w0 * xs[4 * HX4 + i];
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    const float4 zp = row[j * kTbW4], zm = row[-j * kTbW4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float acc = a.wx[j] * (xs[4 * HX4 + i + j] + xs[4 * HX4 + i - j]);
                        acc += a.wz[j] * (comp(zp, i) + comp(zm, i));
                        un[i] += acc;
                    }
                }
                const int gz = z0 + lr;
                const int gx = x0 - kTbPadX + 4 * c;
                float o[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool in = gz >= 0 && gz < L.nz && gx + i >= 0 && gx + i < L.nx;
                    o[i] = in ? un[i] + xs[4 * HX4 + i] : 0.f;   // the field is zero outside the grid
                }
                res[k] = make_float4(o[0], o[1], o[2], o[3]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kTbPerLane; ++k) {
            const int gidx = lane + k * kBlock;
            const int lr = gidx / kTbW4, c = gidx - lr * kTbW4;
            if (lr >= r0 && lr < r1 && c >= c0 && c < c1) lds[lr * kTbW4 + c] = res[k];
        }
        __syncthreads();
    }
    // write the 64 x 64 tile
    for (int i = lane; i < kTile2Z * (kTileX / 4); i += kBlock) {
        const int lr = i / (kTileX / 4), cq = i - lr * (kTileX / 4);
        const int gz = z0 + H + lr, gx = x0 + Hx + 4 * cq;
        if (gz >= L.nz || gx >= L.nx) continue;
        const int c = (kTbPadX + Hx) / 4 + cq;         // float4 column of the written group
        const float *src = ldsf + ((H + lr) * kTbW4 + c) * 4;
        const int nvalid = L.nx - gx;
        const long long off = L.offset(gx, 0, gz);
        if (nvalid >= 4) {
            const float4 r4 = lds[(H + lr) * kTbW4 + c];
            if (a.out_cached)
                *reinterpret_cast<float4 *>(a.out + off) = r4;
            else
                st4nt_f32(a.out + off, r4);
        } else {
            for (int k = 0; k < nvalid; ++k) a.out[off + k] = src[k];
        }
    }
}

template <int... Rs>
struct DiffTable {
    static void (*get(int r))(const DiffArgs) {
        void (*f)(const DiffArgs) = nullptr;
        ((r == Rs ? (f = k_diffuse2d<Rs>, 0) : 0), ...);
        return f;
    }
    static void (*get_tb(int r))(const DiffArgs, int) {
        void (*f)(const DiffArgs, int) = nullptr;
        ((r == Rs ? (f = k_diffuse2d_tb<Rs>, 0) : 0), ...);
        return f;
    }
};

template <Store S>
__global__ void k_sample(const Sample s, const void *field) {
    sample_block<S>(s, field, (int)blockIdx.x);
}

// --------------------------------------------------------------- utilities
__global__ void k_fill_velocity(const Layout L, const float *vp, int vp_padded, int nbl,
                                int px, int py, int pz, float *vel) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        float v;
        if (vp_padded) {
            v = vp[i];
        } else {
            const int ix = min(max(x - nbl, 0), px - 1);
            const int iz = min(max(z - nbl, 0), pz - 1);
            if (L.ndim == 3) {
                const int iy = min(max(y - nbl, 0), py - 1);
                v = vp[((long long)iz * py + iy) * px + ix];
            } else {
                v = vp[(long long)iz * px + ix];
            }
        }
        vel[L.offset(x, y, z)] = v;
    }
}

__global__ void k_vrange(const Layout L, const float *vel, unsigned *out) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    float m = 0.f, lo = __uint_as_float(0x7F800000u);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        const float v = vel[L.offset(x, y, z)];
        // NaN or non-positive velocities poison the maximum on purpose
        m = (v > 0.f) ? fmaxf(m, v) : __uint_as_float(0x7F800000u);
        if (!(v > 0.f)) break;
        lo = fminf(lo, v);
    }
    // positive floats order as their bit patterns
    atomicMax(out, __float_as_uint(m));
    atomicMin(out + 1, __float_as_uint(lo));
}

__global__ void k_make_p(const Layout L, const float *vel, double dt2, float *p) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        const long long o = L.offset(x, y, z);
        const double v = (double)vel[o];
        p[o] = (float)(dt2 * v * v);
    }
}

// The 16-bit code of p: the nearest integer in [0, 65535] to (p - base) /
// step with p = dt^2 v^2, all in float64 (base and step are the float32
// values the step's decode uses, so the code is the nearest one for that
// decode).  Each operation rounds on its own (no contraction), as the
// definition states.
__global__ void k_make_pq(const Layout L, const float *vel, double dt2, double base, double step,
                          uint16_t *pq) {
#pragma clang fp contract(off)
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        const long long o = L.offset(x, y, z);
        const double v = (double)vel[o];
        const double p = dt2 * v * v;
        const double c = step > 0.0 ? rint((p - base) / step) : 0.0;
        pq[o] = (uint16_t)fmin(fmax(c, 0.0), 65535.0);
    }
}

template <typename T>
__global__ void k_zero(T *f, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        f[i] = T(0);
}

template <Store S>
__global__ void k_dense_to_field(const Layout L, const float *dense, void *f, float scale) {
    using E = Elem<S>;
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        E::st((typename E::T *)f + L.offset(x, y, z), dense[i] * scale);
    }
}

template <Store S>
__global__ void k_field_to_dense(const Layout L, const void *f, float *dense, float scale) {
    using E = Elem<S>;
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        dense[i] = E::ld((const typename E::T *)f + L.offset(x, y, z)) * scale;
    }
}

// Misfit: residual and per-block FP64 partial sums of r^2/2 (fixed order),
// then a single workgroup folds the partials in index order.
__global__ void k_misfit_partial(const float *rec, const float *obs, long long n, int given,
                                 float *resid, double *partials) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const float r = given ? obs[i] : rec[i] - obs[i];
        if (resid) resid[i] = r;
        acc += 0.5 * (double)r * (double)r;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void k_misfit_final(const double *partials, int npart, double *out) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < npart; i += kBlock) acc += partials[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// ------------------------------------------------------------ dispatch tables
template <Store S, int MODE, int... Rs>
struct Table2 {
    static StepFn get(int r) {
        StepFn f = nullptr;
        ((r == Rs ? (f = k_step2d<Rs, S, MODE>, 0) : 0), ...);
        return f;
    }
};

template <Store S, int MODE>
using Tab2 = Table2<S, MODE, 1, 2, 3, 4, 5, 6, 7, 8>;

// The gradient modes exist for float32 storage and p only, the difference
// storage for 16-bit 3D fields only, the 16-bit p codes in 3D only (kPlain
// and kDiff); the 3D kernels come from the storage type's own unit.
StepFn pick_step(int ndim, int r, Store st, int mode, int tw4, bool pq) {
    if (ndim == 3) {
        if (pq && mode != kPlain && mode != kDiff) return nullptr;
        if ((mode == kBracket || mode == kImage) && st != Store::F32) return nullptr;
        if (mode == kDiff && st == Store::F32) return nullptr;
        switch (st) {
            case Store::F32: return step3d_kernel_f32(r, mode, tw4, pq);
            case Store::F16: return mode == kDiff ? step3d_kernel_f16_diff(r, tw4, pq) : step3d_kernel_f16(r, tw4, pq);
            case Store::BF16:
                return mode == kDiff ? step3d_kernel_bf16_diff(r, tw4, pq) : step3d_kernel_bf16(r, tw4, pq);
        }
        return nullptr;
    }
    if (pq || mode == kDiff) return nullptr;
    if (mode == kBracket) return st == Store::F32 ? Tab2<Store::F32, kBracket>::get(r) : nullptr;
    if (mode == kImage) return st == Store::F32 ? Tab2<Store::F32, kImage>::get(r) : nullptr;
    switch (st) {
        case Store::F32: return Tab2<Store::F32, kPlain>::get(r);
        case Store::F16: return Tab2<Store::F16, kPlain>::get(r);
        case Store::BF16: return Tab2<Store::BF16, kPlain>::get(r);
    }
    return nullptr;
}

inline int grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

hipError_t launch_step_t2(const StepArgs &a, hipStream_t s) {
    void (*f)(const StepArgs) = nullptr;
    switch (a.L.r) {
        case 1: f = k_step3d_t2<1>; break;
        case 2: f = k_step3d_t2<2>; break;
        case 3: f = k_step3d_t2<3>; break;
        case 4: f = k_step3d_t2<4>; break;
        default: return hipErrorInvalidValue;
    }
    if (a.L.ndim != 3) return hipErrorInvalidValue;
    const int blocks = a.ntx * a.nty * a.ntz + a.nsamp_blocks + a.nsamp_blocks2;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int step_t2_blocks_per_cu(int r) {
    const void *f = r == 1 ? reinterpret_cast<const void *>(k_step3d_t2<1>)
                    : r == 2 ? reinterpret_cast<const void *>(k_step3d_t2<2>)
                    : r == 3 ? reinterpret_cast<const void *>(k_step3d_t2<3>)
                    : r == 4 ? reinterpret_cast<const void *>(k_step3d_t2<4>)
                             : nullptr;
    if (!f) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, 0) != hipSuccess) return 0;
    return n;
}

hipError_t launch_step(const StepArgs &a, Store st, int mode, hipStream_t s) {
    StepFn f = pick_step(a.L.ndim, a.L.r, st, mode, a.shape3, a.pq != nullptr);
    if (!f) return hipErrorInvalidValue;
    const int tiles = (a.ntx * a.nty + (a.L.ndim == 3 ? a.nstrip : 0)) * a.ntz;
    const int blocks = tiles + a.nsamp_blocks;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int step_blocks_per_cu(int ndim, int r, Store st, int mode, int tw4, bool pq) {
    StepFn f = pick_step(ndim, r, st, mode, tw4, pq);
    if (!f) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(f), kBlock, 0) !=
        hipSuccess)
        return 0;
    return n;
}

hipError_t launch_sample(const Sample &smp, const void *field, Store st, hipStream_t s) {
    if (!smp.out || smp.npts <= 0) return hipSuccess;
    const int blocks = sample_blocks(smp);
    switch (st) {
        case Store::F32: hipLaunchKernelGGL(k_sample<Store::F32>, dim3(blocks), dim3(kBlock), 0, s, smp, field); break;
        case Store::F16: hipLaunchKernelGGL(k_sample<Store::F16>, dim3(blocks), dim3(kBlock), 0, s, smp, field); break;
        case Store::BF16: hipLaunchKernelGGL(k_sample<Store::BF16>, dim3(blocks), dim3(kBlock), 0, s, smp, field); break;
    }
    return hipGetLastError();
}

hipError_t launch_fill_velocity(const Layout &L, const float *vp, int vp_padded, int nbl,
                                const int *phys, float *vel, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_fill_velocity, dim3(grid_for(n)), dim3(kBlock), 0, s, L, vp, vp_padded,
                       nbl, phys[0], phys[1], phys[2], vel);
    return hipGetLastError();
}

hipError_t launch_vrange(const Layout &L, const float *vel, unsigned *out_bits, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_vrange, dim3(grid_for(n)), dim3(kBlock), 0, s, L, vel, out_bits);
    return hipGetLastError();
}

hipError_t launch_make_p(const Layout &L, const float *vel, double dt, float *p, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_make_p, dim3(grid_for(n)), dim3(kBlock), 0, s, L, vel, dt * dt, p);
    return hipGetLastError();
}

hipError_t launch_make_pq(const Layout &L, const float *vel, double dt, double base, double step,
                          uint16_t *pq, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_make_pq, dim3(grid_for(n)), dim3(kBlock), 0, s, L, vel, dt * dt, base, step, pq);
    return hipGetLastError();
}

hipError_t launch_zero_field(const Layout &L, void *f, Store st, hipStream_t s) {
    if (st == Store::F32)
        hipLaunchKernelGGL(k_zero<float>, dim3(grid_for(L.elems)), dim3(kBlock), 0, s, (float *)f, L.elems);
    else
        hipLaunchKernelGGL(k_zero<uint16_t>, dim3(grid_for(L.elems)), dim3(kBlock), 0, s, (uint16_t *)f, L.elems);
    return hipGetLastError();
}

// acc += part, part = 0, over the grid rows of the two pitched fields (x in
// [0, round4(nx)): the cells past nx are zero in both, so they stay zero);
// the zero halo and pad are left alone.
__global__ void k_fold_f64(double *acc, float *part, const Layout L) {
    const int g4 = (L.nx + 3) / 4;   // float4 groups per row
    const long long n = (long long)g4 * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long row = i / g4;
        const int gx = (int)(i - row * g4);
        const long long off = L.offset(4 * gx, (int)(row % L.ny), (int)(row / L.ny));   // a multiple of 4
        const float4 p = *reinterpret_cast<const float4 *>(part + off);
        double2 *a = reinterpret_cast<double2 *>(acc + off);
        double2 a0 = a[0], a1 = a[1];
        a0.x += p.x;
        a0.y += p.y;
        a1.x += p.z;
        a1.y += p.w;
        a[0] = a0;
        a[1] = a1;
        *reinterpret_cast<float4 *>(part + off) = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

hipError_t launch_fold_f64(const Layout &L, double *acc, float *part, hipStream_t s) {
    const long long n = (long long)((L.nx + 3) / 4) * L.ny * L.nz;
    hipLaunchKernelGGL(k_fold_f64, dim3(grid_for(n)), dim3(kBlock), 0, s, acc, part, L);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double *p, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_dense_to_field(const Layout &L, const float *dense, void *f, Store st,
                                 float scale, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    const dim3 g(grid_for(n)), b(kBlock);
    switch (st) {
        case Store::F32: hipLaunchKernelGGL(k_dense_to_field<Store::F32>, g, b, 0, s, L, dense, f, scale); break;
        case Store::F16: hipLaunchKernelGGL(k_dense_to_field<Store::F16>, g, b, 0, s, L, dense, f, scale); break;
        case Store::BF16: hipLaunchKernelGGL(k_dense_to_field<Store::BF16>, g, b, 0, s, L, dense, f, scale); break;
    }
    return hipGetLastError();
}

hipError_t launch_field_to_dense(const Layout &L, const void *f, float *dense, Store st,
                                 float scale, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    const dim3 g(grid_for(n)), b(kBlock);
    switch (st) {
        case Store::F32: hipLaunchKernelGGL(k_field_to_dense<Store::F32>, g, b, 0, s, L, f, dense, scale); break;
        case Store::F16: hipLaunchKernelGGL(k_field_to_dense<Store::F16>, g, b, 0, s, L, f, dense, scale); break;
        case Store::BF16: hipLaunchKernelGGL(k_field_to_dense<Store::BF16>, g, b, 0, s, L, f, dense, scale); break;
    }
    return hipGetLastError();
}

namespace {
template <Store S>
__global__ void k_dense_diff_to_field(const Layout L, const float *a, const float *b, void *d, float scale) {
    using E = Elem<S>;
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        E::st((typename E::T *)d + L.offset(x, y, z), ((a ? a[i] : 0.f) - (b ? b[i] : 0.f)) * scale);
    }
}

template <Store S>
__global__ void k_field_diff_to_dense(const Layout L, const void *u, const void *d, float *dense, float scale) {
    using E = Elem<S>;
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        const long long o = L.offset(x, y, z);
        dense[i] = (E::ld((const typename E::T *)u + o) - E::ld((const typename E::T *)d + o)) * scale;
    }
}
}  // namespace

hipError_t launch_dense_diff_to_field(const Layout &L, const float *a, const float *b, void *d, Store st,
                                      float scale, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    const dim3 g(grid_for(n)), bl(kBlock);
    if (st == Store::F16)
        hipLaunchKernelGGL(k_dense_diff_to_field<Store::F16>, g, bl, 0, s, L, a, b, d, scale);
    else if (st == Store::BF16)
        hipLaunchKernelGGL(k_dense_diff_to_field<Store::BF16>, g, bl, 0, s, L, a, b, d, scale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_field_diff_to_dense(const Layout &L, const void *u, const void *d, float *dense, Store st,
                                      float scale, hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    const dim3 g(grid_for(n)), bl(kBlock);
    if (st == Store::F16)
        hipLaunchKernelGGL(k_field_diff_to_dense<Store::F16>, g, bl, 0, s, L, u, d, dense, scale);
    else if (st == Store::BF16)
        hipLaunchKernelGGL(k_field_diff_to_dense<Store::BF16>, g, bl, 0, s, L, u, d, dense, scale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

namespace {
// dense = f, or with a velocity field the chain rule from m = 1/v^2 to v:
// dense = f * dm/dv = f * (-2 / v^3), in float64.
__global__ void k_field_to_dense_f64(const Layout L, const double *f, const float *vel, double *dense) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % L.nx);
        const int y = (int)((i / L.nx) % L.ny);
        const int z = (int)(i / ((long long)L.nx * L.ny));
        const long long o = L.offset(x, y, z);
        double g = f[o];
        if (vel) {
            const double v = (double)vel[o];
            g *= -2.0 / (v * v * v);
        }
        dense[i] = g;
    }
}
}  // namespace

hipError_t launch_field_to_dense_f64(const Layout &L, const double *f, const float *vel, double *dense,
                                     hipStream_t s) {
    const long long n = (long long)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_field_to_dense_f64, dim3(grid_for(n)), dim3(kBlock), 0, s, L, f, vel, dense);
    return hipGetLastError();
}

hipError_t launch_diffuse2d(const Layout &L, const float *u, float *out, float w0, const float *wx,
                            const float *wz, hipStream_t s) {
    auto f = DiffTable<1, 2, 3, 4, 5, 6, 7, 8>::get(L.r);
    if (!f || L.ndim != 2) return hipErrorInvalidValue;
    DiffArgs a{};
    a.L = L;
    a.u = u;
    a.out = out;
    a.w0 = w0;
    for (int j = 0; j <= kMaxR; ++j) {
        a.wx[j] = wx[j];
        a.wz[j] = wz[j];
    }
    a.ntx = (L.nx + kTileX - 1) / kTileX;
    a.ntz = (L.nz + kTile2Z - 1) / kTile2Z;
    a.out_cached = (size_t)L.elems * sizeof(float) <= kCachedField;
    hipLaunchKernelGGL(f, dim3(a.ntx * a.ntz), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int diffuse2d_max_levels(int r) { return kTbHalo / r; }

hipError_t launch_diffuse2d_tb(const Layout &L, const float *u, float *out, float w0, const float *wx,
                               const float *wz, int nlev, hipStream_t s) {
    auto f = DiffTable<1, 2, 3, 4, 5, 6, 7, 8>::get_tb(L.r);
    if (!f || L.ndim != 2 || nlev < 1 || L.r * nlev > kTbHalo) return hipErrorInvalidValue;
    DiffArgs a{};
    a.L = L;
    a.u = u;
    a.out = out;
    a.w0 = w0;
    for (int j = 0; j <= kMaxR; ++j) {
        a.wx[j] = wx[j];
        a.wz[j] = wz[j];
    }
    a.ntx = (L.nx + kTileX - 1) / kTileX;
    a.ntz = (L.nz + kTile2Z - 1) / kTile2Z;
    a.out_cached = (size_t)L.elems * sizeof(float) <= kCachedField;
    hipLaunchKernelGGL(f, dim3(a.ntx * a.ntz), dim3(kBlock), 0, s, a, nlev);
    return hipGetLastError();
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t static_scratch(int device, void **ptr) {
    if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_misfit(const float *rec, const float *obs, long long n, int residual_given,
                         float *resid, double *partials, int npart, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_misfit_partial, dim3(npart), dim3(kBlock), 0, s, rec, obs, n,
                       residual_given, resid, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_misfit_final, dim3(1), dim3(kBlock), 0, s, partials, npart, out);
    return hipGetLastError();
}

}  // namespace fd
