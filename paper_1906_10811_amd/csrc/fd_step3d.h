// fd_step3d.h -- device code of the 3D step, shared by the translation
// units of libfd's kernels.
//
// The step kernel k_step3d<R, S, MODE, SHAPE, PQ> is instantiated for every
// radius, storage type, step mode, tile shape and form of p; the
// instantiations of one storage type and form live in a translation unit of
// their own (fd_step3d_f32.hip; fd_step3d_f16.hip, fd_step3d_bf16.hip and
// their _diff forms) so that they compile in parallel, and each exports a
// lookup of its kernels.  The helpers below (storage types, sampling,
// source scatter, the update) are also used by the other kernels of
// fd_kernels.hip.  Everything device-side has internal linkage: each unit
// compiles its own copy of what it uses.
#ifndef FD_STEP3D_H
#define FD_STEP3D_H

#include "fd_internal.h"

#include <stdint.h>

#include <type_traits>

namespace fd {

using StepFn = void (*)(const StepArgs);

// The 3D step kernels of one storage type (and, for 16-bit fields, one
// storage form: two levels or value plus difference) for radius r, step
// mode, tile shape code (16, 8 or kShapeMixed = 0) and p in float32 or as
// 16-bit codes; null where that combination is not built.
StepFn step3d_kernel_f32(int r, int mode, int shape, bool pq);
StepFn step3d_kernel_f16(int r, int shape, bool pq);
StepFn step3d_kernel_f16_diff(int r, int shape, bool pq);
StepFn step3d_kernel_bf16(int r, int shape, bool pq);
StepFn step3d_kernel_bf16_diff(int r, int shape, bool pq);

namespace {

// ------------------------------------------------------------ storage types
// ld4/st4 move 4 consecutive points.  The *nt forms carry the non-temporal
// hint: u^{n-1}, dt^2 v^2 and u^{n+1} are each touched once per step, so
// streaming them past the caches leaves L2 to the centre field, whose
// planes are re-read as halo by the neighbouring tiles.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ inline float4 ld4nt_f32(const float *p) {
    const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
    return make_float4(t.x, t.y, t.z, t.w);
}
__device__ inline void st4nt_f32(float *p, float4 v) {
    const f32x4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<f32x4 *>(p));
}
__device__ inline uint2 ld2nt_u32(const uint16_t *p) {
    const u32x2 t = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
    return make_uint2(t.x, t.y);
}
__device__ inline void st2nt_u32(uint16_t *p, uint2 v) {
    const u32x2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<u32x2 *>(p));
}

template <Store S> struct Elem;

template <> struct Elem<Store::F32> {
    using T = float;
    using Raw = float4;   // 4 points as loaded (converted to float4 only where used)
    __device__ static float4 ld4(const T *p) { return *reinterpret_cast<const float4 *>(p); }
    __device__ static float4 ld4nt(const T *p) { return ld4nt_f32(p); }
    __device__ static Raw ld4raw(const T *p) { return ld4(p); }
    __device__ static Raw ld4ntraw(const T *p) { return ld4nt(p); }
    __device__ static float4 cvt(const Raw &r) { return r; }
    __device__ static void st4nt(T *p, float4 v) { st4nt_f32(p, v); }
    __device__ static void st4(T *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }
    __device__ static float ld(const T *p) { return *p; }
    __device__ static void st(T *p, float v) { *p = v; }
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ inline float h2f(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
__device__ inline uint16_t f2h(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
// bfloat16: the upper half of the float32 pattern; float32 -> bfloat16
// rounds to nearest even in hardware (v_cvt_pk_bf16_f32 converts a pair).
__device__ inline float b2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline uint16_t f2b(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <typename Cvt> struct Elem16 {
    using T = uint16_t;
    __device__ static float4 unpack(uint2 v) {
        return make_float4(Cvt::to_f(v.x & 0xFFFF), Cvt::to_f(v.x >> 16), Cvt::to_f(v.y & 0xFFFF),
                           Cvt::to_f(v.y >> 16));
    }
    __device__ static uint2 pack(float4 v) { return make_uint2(Cvt::pack2(v.x, v.y), Cvt::pack2(v.z, v.w)); }
    using Raw = uint2;
    __device__ static float4 ld4(const T *p) { return unpack(*reinterpret_cast<const uint2 *>(p)); }
    __device__ static float4 ld4nt(const T *p) { return unpack(ld2nt_u32(p)); }
    // Raw loads keep the 16-bit pairs in registers; the unpack happens where
    // the values are used, so a prefetch issued planes ahead does not wait
    // for its data at the load.
    __device__ static Raw ld4raw(const T *p) { return *reinterpret_cast<const uint2 *>(p); }
    __device__ static Raw ld4ntraw(const T *p) { return ld2nt_u32(p); }
    __device__ static float4 cvt(const Raw &r) { return unpack(r); }
    __device__ static void st4nt(T *p, float4 v) { st2nt_u32(p, pack(v)); }
    __device__ static void st4(T *p, float4 v) { *reinterpret_cast<uint2 *>(p) = pack(v); }
    __device__ static float ld(const T *p) { return Cvt::to_f(*p); }
    __device__ static void st(T *p, float v) { *p = Cvt::from_f(v); }
};
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
struct CvtF16 {
    __device__ static float to_f(uint32_t h) { return h2f((uint16_t)h); }
    __device__ static uint16_t from_f(float f) { return f2h(f); }
    // one v_cvt_pk_f16_f32 (round to nearest even, as the single conversion)
    // instead of two conversions and an or
    __device__ static uint32_t pack2(float a, float b) {
        const f32x2 v = {a, b};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
    }
};
struct CvtBF16 {
    __device__ static float to_f(uint32_t b) { return b2f((uint16_t)b); }
    __device__ static uint16_t from_f(float f) { return f2b(f); }
    __device__ static uint32_t pack2(float a, float b) {
        const f32x2 v = {a, b};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
    }
};
template <> struct Elem<Store::F16> : Elem16<CvtF16> {};
template <> struct Elem<Store::BF16> : Elem16<CvtBF16> {};

__device__ inline float comp(const float4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// p = dt^2 v^2 of 4 points: float32 as stored, or the 16-bit codes c of
// the quantised form, p = fma(c, step, base) in float32.
__device__ inline float4 param4(const float4 &v, float, float) { return v; }
__device__ inline float4 param4(const uint2 &c, float base, float step) {
    return make_float4(__builtin_fmaf((float)(c.x & 0xFFFFu), step, base),
                       __builtin_fmaf((float)(c.x >> 16), step, base),
                       __builtin_fmaf((float)(c.y & 0xFFFFu), step, base),
                       __builtin_fmaf((float)(c.y >> 16), step, base));
}

// Workgroups are dealt to the 8 XCDs round-robin by hardware id.  Renumber
// so that each XCD runs one contiguous range of logical tiles: x-neighbour
// and y-neighbour tiles then share an L2, which serves their halo reads.
__device__ inline int xcd_remap(int h, int G) {
    constexpr int X = 8;
    const int xcd = h % X, k = h / X;
    const int per = G / X, rem = G % X;
    return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

template <Store S>
__device__ void sample_block(const Sample &s, const void *field, int blk) {
    using E = Elem<S>;
    // s.lpp lanes share a point: each sums a strided share of its nodes, then
    // the group reduces with xor shuffles (fixed order: deterministic).
    const int lane = (int)threadIdx.x;
    const int i = blk * (kBlock / s.lpp) + lane / s.lpp;
    const int sub = lane & (s.lpp - 1);
    const typename E::T *f = (const typename E::T *)field;
    float v = 0.f;
    if (i < s.npts) {
        const long long b = (long long)i * s.nc;
        for (int c = sub; c < s.nc; c += s.lpp) v = __builtin_fmaf(s.w[b + c], E::ld(f + s.idx[b + c]), v);
    }
    for (int o = s.lpp >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (i < s.npts && sub == 0) s.out[i] = v * s.scale;
}

// Source terms of one plane of a 3D tile (TX points per row): the tile's
// corners [e0, e1) of the plane are spread over the workgroup; each lane sums
// the weighted values of its corners into the tile-shaped LDS buffer (a grid
// point occurs once per plane, so no two lanes write one cell).
template <int TX>
__device__ inline void scatter_sources(const Inject &inj, int e0, int e1, int x0, int y0, float *s_src) {
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) {
        const int4 c = inj.corner[e];
        float v = 0.f;
        for (int k = c.z; k < c.w; ++k) v = __builtin_fmaf(inj.w[k], inj.vals[inj.src[k]], v);
        s_src[(c.y - y0) * TX + (c.x - x0)] = v * inj.scale;
    }
}

// Source term of the points (x..x+3) of one 2D row from the row's corners
// [e0, e1) in the tile (the lanes of a row walk the same short list).
__device__ inline void gather_sources(const Inject &inj, int e0, int e1, int x, float &s0, float &s1,
                                      float &s2, float &s3) {
    for (int e = e0; e < e1; ++e) {
        const int4 c = inj.corner[e];
        const int d = c.x - x;
        if ((unsigned)d < 4u) {
            float v = 0.f;
            for (int k = c.z; k < c.w; ++k) v = __builtin_fmaf(inj.w[k], inj.vals[inj.src[k]], v);
            v *= inj.scale;
            s0 += d == 0 ? v : 0.f;
            s1 += d == 1 ? v : 0.f;
            s2 += d == 2 ? v : 0.f;
            s3 += d == 3 ? v : 0.f;
        }
    }
}

// The update and the Laplacian are written with explicit fused multiply-adds
// so that every kernel instantiation (plain, bracket, imaging; any storage)
// rounds them identically: a state recomputed by one step mode is bitwise
// the state another mode computed, which checkpoint recomputation relies on.
//
// With alpha = 1/(1+s) and (1-s)/(1+s) = 2 alpha - 1 the centred update
// alpha [2c - (1-s) m + p (lap + src)] is m + alpha [2 (c - m) + p (lap + src)]:
// no beta, and c - m is exact where the two levels are close.  The hardware
// reciprocal of 1 is exactly 1 (checked, as for every power of two), so
// outside the damping layer alpha is 1 with no select.
__device__ inline float update_point(float c, float m, float p, float lap, float src, float s) {
    const float alpha = __builtin_amdgcn_rcpf(1.f + s);
    return __builtin_fmaf(alpha, __builtin_fmaf(p, lap + src, 2.f * (c - m)), m);
}

// The same update for the difference storage: with u^{n-1} = u^n - d,
// u^{n+1} - u^n = [(1 - s) d + p (lap + src)] / (1 + s)
//               = alpha [2 d + p (lap + src)] - d,
// computed directly (no cancellation of the two levels).
__device__ inline float update_diff(float d, float p, float lap, float src, float s) {
    const float alpha = __builtin_amdgcn_rcpf(1.f + s);
    return __builtin_fmaf(alpha, __builtin_fmaf(p, lap + src, 2.f * d), -d);
}

// One radius-j term of the 2D Laplacian at a point: the weights times the
// sums of the two neighbours at distance j along each axis.
__device__ inline float lap_term2(float wx, float xs, float wz, float zs) {
    return __builtin_fmaf(wz, zs, wx * xs);
}

// g -= lam * br for the lane's 4 points into the float32 partial sum (the
// host folds it into the float64 gradient every few adjoint steps); gv is
// the partial sum's current value at those points.
__device__ inline void image_accumulate(float *g, int nvalid, const float un[4], const float4 &br,
                                        const float4 &gv) {
    float4 v;
    v.x = __builtin_fmaf(-un[0], br.x, gv.x);
    v.y = __builtin_fmaf(-un[1], br.y, gv.y);
    v.z = __builtin_fmaf(-un[2], br.z, gv.z);
    v.w = __builtin_fmaf(-un[3], br.w, gv.w);
    if (nvalid >= 4) {
        st4nt_f32(g, v);
    } else {
        const float r[3] = {v.x, v.y, v.z};
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (i < nvalid) g[i] = r[i];
    }
}

// Gradient epilogues of a step (float32 fields, pitched offset `off` of the
// first of 4 points, nvalid of them inside the grid).
template <int MODE>
__device__ inline void grad_epilogue(const Imaging &img, long long off, int nvalid, const float un[4],
                                     const float4 &c, const float4 &m, const float s[4]) {
    if constexpr (MODE == kBracket) {
        float b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float u1 = un[i], u0 = comp(c, i), um = comp(m, i);
            b[i] = __builtin_fmaf(s[i], u1 - um, (u1 - 2.f * u0) + um);
        }
        if (nvalid >= 4) {
            st4nt_f32(img.br_out + off, make_float4(b[0], b[1], b[2], b[3]));
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < nvalid) img.br_out[off + i] = b[i];
        }
    } else if constexpr (MODE == kImage) {
        image_accumulate(img.gpart + off, nvalid, un, ld4nt_f32(img.br_in + off), ld4nt_f32(img.gpart + off));
    }
}

// ------------------------------------------------------------------ 3D step
// f(integral_constant<I>) for I = B .. E-1, unrolled at compile time.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Shared memory of a 3D step workgroup with tiles of TW float4 columns,
// carved from one buffer (offsets in float4) so that a launch that mixes
// tile shapes reserves only the larger layout.
template <int R, int TW>
struct Smem3 {
    static constexpr int TY = kBlock / TW, HX4 = (R + 3) / 4, W4 = TW + 2 * HX4, LH = TY + 2 * R;
    static constexpr int NH = 2 * R * TW + 2 * TY * HX4;     // halo items of a plane
    static constexpr int kLds = 0;                           // [2][LH * W4] staged planes
    static constexpr int kRing = kLds + 2 * LH * W4;         // [(R + 1) * NH] halo ring
    static constexpr int kSrc = kRing + (R + 1) * NH;        // [kBlock] source terms of a plane
    static constexpr int kDz = kSrc + kBlock;                // float [kMaxChunk] z damping
    static constexpr int kPp = kDz + kMaxChunk / 4;          // int [kMaxChunk + 1] plane pointers
    static constexpr int kSize = kPp + (kMaxChunk + 1 + 3) / 4;
};

// One workgroup's step: the xy tile at (x0, y0) of TW float4 columns per
// row (16: 64 x 16 points, 8: 32 x 32) and z chunk bz; tid is the tile's
// row in the source plane-pointer table.
template <int R, Store S, int MODE, int TW, bool PQ>
__device__ __forceinline__ void step3d_tile(const StepArgs &a, float4 *smem, int x0, int y0, int bz, int tid) {
    static_assert(!PQ || MODE == kPlain || MODE == kDiff, "the gradient modes read float32 p");
    using E = Elem<S>;
    using T = typename E::T;
    using SM = Smem3<R, TW>;
    constexpr int TX = 4 * TW;                // x points per tile
    constexpr int TY = kBlock / TW;           // y rows per tile
    constexpr int HX4 = (R + 3) / 4;          // float4 halo columns per side
    constexpr int W4 = TW + 2 * HX4;          // float4 per LDS row
    constexpr int LH = TY + 2 * R;            // LDS rows
    float4 (*lds)[LH * W4] = reinterpret_cast<float4 (*)[LH * W4]>(smem + SM::kLds);

    const Layout L = a.L;
    const int z0 = bz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, L.nz);
    // Odd chunks march downwards: two adjacent chunks then read the warm-up
    // planes around their common boundary at about the same time (both at
    // their start, or both at their end), while the first read is still
    // cached.  Measured: 0.5 % fewer fetched bytes, 0.5-1 % faster.
    const int dir = (bz & 1) ? -1 : 1;
    const int len = z1 - z0;
    const int zs = dir > 0 ? z0 : z1 - 1;   // first plane of the march

    const int lane = (int)threadIdx.x;
    // Per-plane tables of this chunk (damping along z, source CSR pointers)
    // are staged in LDS so that the plane loop issues no uniform global load:
    // a vector-memory wait for one would also drain the prefetched planes.
    float *s_dz = reinterpret_cast<float *>(smem + SM::kDz);
    int *s_pp = reinterpret_cast<int *>(smem + SM::kPp);
    const int *tile_pp = a.inj.plane_ptr + (long long)tid * (L.nz + 1);
    for (int i = lane; i <= z1 - z0; i += kBlock) {
        if (i < z1 - z0) s_dz[i] = a.damp[L.nx + L.ny + z0 + i];
        s_pp[i] = a.inj.vals ? tile_pp[z0 + i] : 0;
    }
    // Source terms of the current plane, scattered by the workgroup (one
    // float4 per lane; a lane clears its cells after reading them).
    static_assert(TY * TX / 4 == kBlock, "one float4 of source terms per lane");
    float4 *s_src4 = smem + SM::kSrc;
    s_src4[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int tx = lane % TW, ty = lane / TW;
    const int x = x0 + 4 * tx, y = y0 + ty;
    const bool active = (y < L.ny) && (x < L.nx);
    // Masked lanes and halo items read a column that is zero in every row of
    // every plane (x in [round4(nx), round4(nx)+8) is never written), so all
    // loads are unconditional and no select waits on a load.
    const long long zcol = L.offset((L.nx + 3) & ~3, 0, 0);
    const long long base = active ? L.offset(x, y, 0) : zcol;
    const long long plane = L.plane;

    const T *__restrict__ U = (const T *)a.u;
    const T *Pv = (const T *)a.prev;
    T *O = (T *)a.out;
    const float *__restrict__ Pp = a.p;
    const uint16_t *__restrict__ Pq = a.pq;

    // Halo items of the staged plane: 2r rows above/below the tile (TW float4
    // each) and HX4 float4 columns left/right of each tile row.
    constexpr int NYH = 2 * R * TW;
    constexpr int NXH = 2 * TY * HX4;
    constexpr int NH = NYH + NXH;
    constexpr int HPT = (NH + kBlock - 1) / kBlock;
    long long hoff[HPT];
    int hl[HPT];
    bool hok[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int i = lane + k * kBlock;
        hl[k] = -1;
        hok[k] = false;
        hoff[k] = zcol;
        if (i < NYH) {
            const int hr = i / TW, hc = i % TW;
            const int ly = hr < R ? hr : TY + hr;
            const int gy = y0 + ly - R, gx = x0 + 4 * hc;
            hl[k] = ly * W4 + HX4 + hc;
            hok[k] = (gy >= 0) && (gy < L.ny) && (gx < L.nx);
            hoff[k] = hok[k] ? L.offset(gx, gy, 0) : zcol;
        } else if (i < NH) {
            const int j = i - NYH;
            const int side = j / (TY * HX4);
            const int rem = j - side * (TY * HX4);
            const int row = rem / HX4, c = rem - row * HX4;
            const int gy = y0 + row;
            const int gx = side == 0 ? x0 - 4 * HX4 + 4 * c : x0 + TX + 4 * c;
            hl[k] = (R + row) * W4 + (side == 0 ? c : HX4 + TW + c);
            hok[k] = (gy < L.ny) && (gx >= 0) && (gx < L.nx);
            hoff[k] = hok[k] ? L.offset(gx, gy, 0) : zcol;
        }
    }

    float sxy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int xi = min(x + i, L.nx - 1);
        sxy[i] = active ? a.damp[xi] + a.damp[L.nx + y] : 0.f;
    }
    // The z queue: logical entry k (0 = plane z-R .. 2R = plane z+R) of the
    // body with rotation ROT lives in q[(k + ROT) % NQP], NQP >= 2R+1 slots
    // rounded up to a multiple of 3.  With a rotating queue the plane loop
    // is unrolled NQP times and the rotation advances one per plane, so the
    // queue never moves (the new front takes a free slot); otherwise ROT
    // stays 0 and the entries shift down after each plane, 2R float4 moves.
    // Measured: at so 14 (NQ = 15) rotating is 3.7 % faster; 16-bit fields
    // at so 10, 12 and 16 gain 1-6 % with a padded queue (at so 4 and 6
    // they lose up to 1.3 %), float32 ones -1.1 to +0.5 %; at so 8 the
    // nine-fold loop fetched 2.6 % more bytes
    // from HBM and ran 1.7 % slower (the step is HBM-bound there); in the
    // imaging mode it needs registers that cost a workgroup per CU.
    constexpr int NQ = 2 * R + 1;
    constexpr bool kRot = MODE != kImage && (R == 1 || R == 7 || (S != Store::F32 && R >= 5));
    constexpr int NQP = kRot ? (NQ + 2) / 3 * 3 : NQ;
    constexpr int UNR = kRot ? NQP : 3;
    float4 q[NQP];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) q[k] = E::ld4(U + base + (long long)(zs + dir * (k - R)) * plane);

    // Halo ring: each lane keeps the halo items it loads in R+1 LDS slots.
    // A halo row of plane z belongs to a neighbour tile, which streams plane
    // z as its queue front R planes before this tile stages plane z; loading
    // the halo at that same time lets the neighbour's fetch serve it from L2.
    constexpr int kRing = R + 1;
    static_assert(NH == SM::NH, "halo layout");
    float4 *ring = smem + SM::kRing;
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < HPT; ++k)
            if (hl[k] >= 0) ring[i * NH + lane + k * kBlock] = E::ld4(U + hoff[k] + (long long)(zs + dir * i) * plane);

    // Loads for plane z: the queue front u(z+R), the halo of plane z+R,
    // dt^2 v^2 and u^{n-1}.  Three register sets rotate so that the loads of
    // plane z+2 are in flight while plane z is computed (two planes ahead);
    // the loop is unrolled by three so the rotation needs no register moves,
    // which would otherwise wait for the loads they move.  (A fourth set,
    // three planes ahead, measured 1-2.5 % slower.)
    using Raw = typename E::Raw;
    struct PlaneRegs {
        Raw front, mv;
        std::conditional_t<PQ, uint2, float4> pv;   // p as stored
        Raw hv[HPT];      // halo of plane z+R
        float4 br, gp;    // imaging step: bracket and partial gradient of plane z
    };
    auto issue = [&](PlaneRegs &r, int st) __attribute__((always_inline)) {
        st = min(st, len - 1);   // past the chunk: a harmless in-bounds reload
        const long long zo = (long long)(zs + dir * st) * plane;
        const long long fo = zo + (long long)(dir * R) * plane;   // the queue front, R planes ahead
        r.front = E::ld4raw(U + base + fo);
#pragma unroll
        for (int k = 0; k < HPT; ++k) r.hv[k] = E::ld4raw(U + hoff[k] + fo);
        if constexpr (PQ)
            r.pv = ld2nt_u32(Pq + base + zo);
        else
            r.pv = ld4nt_f32(Pp + base + zo);
        r.mv = E::ld4ntraw(Pv + base + zo);
        if constexpr (MODE == kImage) {
            r.br = ld4nt_f32(a.img.br_in + base + zo);
            r.gp = ld4nt_f32(a.img.gpart + base + zo);
        }
    };
    auto body = [&](auto rot, int st, const PlaneRegs &cur, PlaneRegs &ahead) __attribute__((always_inline)) {
        constexpr int ROT = kRot ? decltype(rot)::value : 0;
#define QQ(k) q[((k) + ROT) % NQP]
        const int z = zs + dir * st;
        float4 *buf = lds[st & 1];
        QQ(2 * R) = E::cvt(cur.front);
        buf[(R + ty) * W4 + HX4 + tx] = QQ(R);
        // park the halo of plane z+R (fetched with the front of the same
        // plane) and stage the halo of plane z parked R planes ago
        float4 *ring_w = ring + ((st + R) % kRing) * NH + lane;
        const float4 *ring_r = ring + (st % kRing) * NH + lane;
#pragma unroll
        for (int k = 0; k < HPT; ++k) {
            if (hl[k] >= 0) {
                ring_w[k * kBlock] = E::cvt(cur.hv[k]);
                buf[hl[k]] = ring_r[k * kBlock];
            }
        }
        issue(ahead, st + 2);
        // tables in LDS are block-uniform: the branches below are uniform
        const int e0 = __builtin_amdgcn_readfirstlane(s_pp[z - z0]);
        const int e1 = __builtin_amdgcn_readfirstlane(s_pp[z - z0 + 1]);
        if (e0 < e1) scatter_sources<TX>(a.inj, e0, e1, x0, y0, reinterpret_cast<float *>(s_src4));
        __syncthreads();
        float4 src4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e0 < e1) {
            src4 = s_src4[lane];
            s_src4[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
            __syncthreads();   // cleared before any lane scatters the next plane
        }

        if (active) {
            const float4 mvf = E::cvt(cur.mv);
            const float4 pv = param4(cur.pv, a.pq_base, a.pq_step);
            // x neighbours: 2*HX4+1 float4 chunks of the lane's LDS row
            float xs[4 * (2 * HX4 + 1)];
            const float4 *row = buf + (R + ty) * W4 + HX4 + tx;
#pragma unroll
            for (int c = -HX4; c <= HX4; ++c) {
                const float4 v = (c == 0) ? QQ(R) : row[c];
                xs[4 * (c + HX4) + 0] = v.x;
                xs[4 * (c + HX4) + 1] = v.y;
                xs[4 * (c + HX4) + 2] = v.z;
                xs[4 * (c + HX4) + 3] = v.w;
            }
            // per radius j one fused multiply-add per axis on the sum of the
            // two neighbours, the centre term last (the sum then builds up
            // from the small neighbour terms before the large centre one
            // cancels it)
            float lap[4];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                const float4 yp = row[j * W4], ym = row[-j * W4];
                const float4 zp = QQ(R + j), zm = QQ(R - j);
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
            const float src[4] = {src4.x, src4.y, src4.z, src4.w};
            const float sz = s_dz[z - z0];
            float un[4];
            [[maybe_unused]] typename E::Raw draw;   // kDiff: the new difference as stored
            if constexpr (MODE == kDiff) {
                // value and difference: mvf is d = u^n - u^{n-1}; the new
                // difference is rounded to 16 bits first, and u^{n+1} is u^n
                // plus that stored difference, so the stored pair stays
                // consistent
                static_assert(S != Store::F32, "difference storage is 16-bit");
                float4 d4;
                d4.x = update_diff(mvf.x, pv.x, lap[0], src[0], sxy[0] + sz);
                d4.y = update_diff(mvf.y, pv.y, lap[1], src[1], sxy[1] + sz);
                d4.z = update_diff(mvf.z, pv.z, lap[2], src[2], sxy[2] + sz);
                d4.w = update_diff(mvf.w, pv.w, lap[3], src[3], sxy[3] + sz);
                asm volatile("" : "+v"(d4.x), "+v"(d4.y), "+v"(d4.z), "+v"(d4.w));
                draw = E::pack(d4);
                const float4 ds = E::cvt(draw);
#pragma unroll
                for (int i = 0; i < 4; ++i) un[i] = comp(QQ(R), i) + comp(ds, i);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    un[i] = update_point(comp(QQ(R), i), comp(mvf, i), comp(pv, i), lap[i], src[i],
                                         sxy[i] + sz);
            }
            const long long off = base + (long long)z * plane;
            float4 r4 = make_float4(un[0], un[1], un[2], un[3]);
            // All four results are computed here, before the ragged-edge
            // branch: otherwise the compiler sinks the fourth point's
            // Laplacian into the full-width store path and re-reads its LDS
            // neighbours one at a time there, serialising LDS latency.  For
            // 16-bit storage the values also pass through as opaque float32
            // values, so that each is rounded to float32 and then to 16 bits
            // as written; otherwise the compiler may fuse a point's last
            // multiply into its conversion (one rounding instead of two),
            // point by point as code generation decides.
            if constexpr (S == Store::F32)
                asm volatile("" ::"v"(r4.x), "v"(r4.y), "v"(r4.z), "v"(r4.w));
            else
                asm volatile("" : "+v"(r4.x), "+v"(r4.y), "+v"(r4.z), "+v"(r4.w));
            const int nvalid = L.nx - x;
            if (nvalid >= 4) {
                // (float32 fields always stream the new level past the caches)
                if (S != Store::F32 && a.out_cached)
                    E::st4(O + off, r4);
                else
                    E::st4nt(O + off, r4);
            } else {
                const float rv[3] = {r4.x, r4.y, r4.z};
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (i < nvalid) E::st(O + off + i, rv[i]);
            }
            if constexpr (MODE == kDiff) {
                T *D = (T *)a.out2;
                if (nvalid >= 4) {
                    if (a.out_cached)
                        *reinterpret_cast<typename E::Raw *>(D + off) = draw;
                    else
                        st2nt_u32(D + off, draw);
                } else {
                    const float4 ds = E::cvt(draw);
                    const float dv[3] = {ds.x, ds.y, ds.z};
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        if (i < nvalid) E::st(D + off + i, dv[i]);
                }
            }
            if constexpr (MODE == kBracket) {
                float sv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) sv[i] = sxy[i] + sz;
                grad_epilogue<MODE>(a.img, off, nvalid, un, QQ(R), mvf, sv);
            } else if constexpr (MODE == kImage) {
                image_accumulate(a.img.gpart + off, nvalid, un, cur.br, cur.gp);
            }
        }
        if constexpr (!kRot) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) q[k] = q[k + 1];
        }
#undef QQ
    };

    __syncthreads();   // staged tables and the cleared source tile, before the first plane
    PlaneRegs s0, s1, s2;
    auto set = [&](auto I) -> PlaneRegs & {   // register set I mod 3
        constexpr int k = decltype(I)::value % 3;
        if constexpr (k == 0) return s0;
        else if constexpr (k == 1) return s1;
        else return s2;
    };
    issue(s0, 0);
    issue(s1, 1);
    int st = 0;
    // body i of an unrolled group computes from set i mod 3 and issues into
    // set (i + 2) mod 3; UNR is a multiple of 3, so each group starts from
    // the same sets (and, when the queue rotates, from rotation 0)
    for (; st + UNR <= len; st += UNR)
        static_for<0, UNR>([&](auto I) {
            constexpr int i = decltype(I)::value;
            body(I, st + i, set(I), set(std::integral_constant<int, i + 2>{}));
        });
    static_for<0, UNR - 1>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (st + i < len) body(I, st + i, set(I), set(std::integral_constant<int, i + 2>{}));
    });
}

// The 3D step.  SHAPE 16 or 8: every tile has that many float4 columns.
// SHAPE 0: 64 x 16 tiles over the ntx whole 64-point columns and, beside
// them, nstrip 32 x 32 tiles for the last, narrower x column (at most 32
// points), which a 64-point tile would fill to half or less.  Tiles are
// numbered x fastest, then y, then the strip, then z chunk.  PQ: p is read
// as 16-bit codes (a.pq) instead of float32.
template <int R, Store S, int MODE, int SHAPE, bool PQ>
__global__ __launch_bounds__(kBlock) void k_step3d(const StepArgs a) {
    constexpr int kSmem = SHAPE == 16 ? Smem3<R, 16>::kSize
                          : SHAPE == 8 ? Smem3<R, 8>::kSize
                                       : (Smem3<R, 16>::kSize > Smem3<R, 8>::kSize ? Smem3<R, 16>::kSize
                                                                                 : Smem3<R, 8>::kSize);
    __shared__ float4 smem[kSmem];
    // Tile workgroups come first in dispatch order (renumbered per XCD); the
    // sampling workgroups trail them and take free slots, so they never
    // displace a tile into a second round.
    const int ntile = (int)gridDim.x - a.nsamp_blocks;
    if ((int)blockIdx.x >= ntile) {
        sample_block<S>(a.smp, a.u, (int)blockIdx.x - ntile);
        return;
    }
    const int t = xcd_remap((int)blockIdx.x, ntile);
    const int nmain = a.ntx * a.nty;
    const int tiles = nmain + a.nstrip;
    const int u = t % tiles, bz = t / tiles;
    if constexpr (SHAPE == 0) {
        if (u < nmain)
            step3d_tile<R, S, MODE, 16, PQ>(a, smem, (u % a.ntx) * 64, (u / a.ntx) * 16, bz, u);
        else
            step3d_tile<R, S, MODE, 8, PQ>(a, smem, a.ntx * 64, (u - nmain) * 32, bz, u);
    } else {
        step3d_tile<R, S, MODE, SHAPE, PQ>(a, smem, (u % a.ntx) * 4 * SHAPE, (u / a.ntx) * (kBlock / SHAPE), bz,
                                           u);
    }
}

// Kernel lookup of one storage type and step mode over the radii Rs.
template <Store S, int MODE, int... Rs>
struct Step3dTable {
    template <bool PQ>
    static StepFn get(int r, int shape) {
        StepFn f = nullptr;
        if (shape == 16) ((r == Rs ? (f = k_step3d<Rs, S, MODE, 16, PQ>, 0) : 0), ...);
        if (shape == 8) ((r == Rs ? (f = k_step3d<Rs, S, MODE, 8, PQ>, 0) : 0), ...);
        // (radii 7 and 8 always run 32 x 32 tiles: no mixed kernel)
        if (shape == 0) ((r == Rs ? (f = k_step3d<Rs, S, MODE, (Rs <= 6 ? 0 : 8), PQ>, 0) : 0), ...);
        return f;
    }
};

// (p codes: kPlain and kDiff only)
template <Store S, int MODE>
StepFn step3d_get(int r, int shape, bool pq) {
    using Tb = Step3dTable<S, MODE, 1, 2, 3, 4, 5, 6, 7, 8>;
    if constexpr (MODE == kPlain || MODE == kDiff)
        return pq ? Tb::template get<true>(r, shape) : Tb::template get<false>(r, shape);
    else
        return pq ? nullptr : Tb::template get<false>(r, shape);
}

}  // namespace
}  // namespace fd

#endif
