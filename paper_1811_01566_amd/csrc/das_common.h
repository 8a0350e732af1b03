// Shared device machinery of the DAS kernels (forward gather, forward-mode
// derivative w.r.t. the speed of sound, adjoint scatter): tile geometry,
// per-transmit and per-channel window bases, window-local fixed-point delays
// and RF staging.  See das.hip for the design.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "ff.h"
#include "wf_internal.h"

namespace wf {
namespace {

constexpr float kQScale = 8388608.0f;  // 2^23
constexpr float kHiQuant = 32768.0f;   // 2^15: grid of the exact "hi" parts

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------

// Distance (samples) from pixel to element: dx = X - x_e, z2 = Z^2.
__device__ __forceinline__ ff dist_ff(ff dx, ff z2) { return ff_sqrt(ff_add(ff_sqr(dx), z2)); }

// round((v - base) * 2^23) for a window-local value v - base >= 0.
__device__ __forceinline__ uint32_t to_q(ff v, int base) {
    ff s = two_sum(v.hi, -(float)base);
    float lo = s.lo + v.lo;
    float h = fmaxf(rintf(s.hi * kQScale), 0.0f);
    float l = rintf(lo * kQScale);
    return (uint32_t)h + (uint32_t)(int)l;
}

// Window-local distance round((sqrt(dx^2 + z2) - base) * 2^23), dx and z2
// float-float.  The square root is the hardware estimate s plus one Newton
// correction; s - base is exact (base is an integer at most s), so the
// correction is rounded separately and added as an integer.
__device__ __forceinline__ uint32_t dist_q(ff dx, ff z2, int base) {
    const ff r2 = ff_add(ff_sqr(dx), z2);
    const float s = __builtin_amdgcn_sqrtf(r2.hi);
    const ff p = two_prod(s, s);
    const float r = ((r2.hi - p.hi) - p.lo) + r2.lo;
    const float corr = r * (0.5f * __builtin_amdgcn_rcpf(fmaxf(s, 1e-30f)));
    const float h = fmaxf((s - (float)base) * kQScale, 0.0f);
    return (uint32_t)h + (uint32_t)(int)rintf(corr * kQScale);
}

// Window-local distance, as dist_q, from a lateral offset dx = dxh + dxl
// whose hi part lies on a grid 2^-g coarse enough that the channel and pixel
// hi parts add exactly (host-chosen g), so forming dx costs two adds, and
// with the base pre-scaled: bq = base * 2^23 (exact).  r^2 = dxh^2 + z2 is
// formed with one TwoProd and one TwoSum (the dxl^2 term, < 2^-24, is
// dropped); s - base is exact, so (s - base) 2^23 is one fused multiply-add.
__device__ __forceinline__ uint32_t dist_q_grid(float dxh, float dxl, ff z2, float bq) {
    const ff p = two_prod(dxh, dxh);
    const float cross = (dxh + dxh) * dxl;
    const ff r2 = two_sum(p.hi, z2.hi);
    const float lo = r2.lo + (p.lo + (cross + z2.lo));
    const float s = __builtin_amdgcn_sqrtf(r2.hi);
    const ff sp = two_prod(s, s);
    const float res = ((r2.hi - sp.hi) - sp.lo) + lo;  // r^2 - s^2
    const float corr = res * ((0.5f * kQScale) * __builtin_amdgcn_rcpf(fmaxf(s, 1e-30f)));
    const float h = fmaxf(fmaf(s, kQScale, -bq), 0.0f);
    return (uint32_t)h + (uint32_t)(int)rintf(corr);
}

typedef float v2f __attribute__((ext_vector_type(2)));

// Hides where a value came from: the difference of two converted int16
// samples then stays one float subtract, where the optimiser would rewrite
// it as an integer subtract plus a second convert.
__device__ __forceinline__ void opaque(float& x) { asm("" : "+v"(x)); }
__device__ __forceinline__ void opaque_u(uint32_t& x) { asm("" : "+v"(x)); }

// Byte address of window entry (u >> 23) at byte offset `off`: one shift
// and one shift-add (the compiler would otherwise emit shift, mask, add).
__device__ __forceinline__ uint32_t entry_addr(uint32_t u, uint32_t off) {
    const uint32_t idx = u >> kQBits;
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, 3, %2" : "=v"(r) : "v"(idx), "s"(off));
    return r;
}

// Smallest distance (samples) from an element at (xe, 0) to the rectangle
// [xlo, xhi] x [zlo, zhi]; plain float, used only for window bases that
// carry a one-sample margin.
__device__ __forceinline__ float rect_min_dist(float xe, float xlo, float xhi, float zlo,
                                               float zhi) {
    float dx = fmaxf(0.0f, fmaxf(xlo - xe, xe - xhi));
    float dz = fminf(fmaxf(0.0f, zlo), zhi);
    return sqrtf(dx * dx + dz * dz);
}

// Raw RF of one staged group (8 samples + the next one), held in registers
// between the load and the LDS commit so that the load latency hides behind
// the previous transmit's arithmetic.  Loads go through a raw buffer
// resource spanning one transmit's records: a byte offset at or beyond its
// size (kOffNone) returns zeros, so groups outside the record need neither a
// branch nor a zero fill.
typedef unsigned v4u __attribute__((ext_vector_type(4)));
constexpr uint32_t kOffNone = 0x80000000u;  // beyond any record buffer (< 2 GiB)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rf_rsrc(const void* base, uint32_t bytes) {
    // raw buffer (stride 0), 32-bit data format: out-of-range dwords read 0
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

template <typename RT>
struct RawGroup;

template <>
struct RawGroup<int16_t> {
    v4u q;
    int nx;
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        nx = (int)(short)__builtin_amdgcn_raw_buffer_load_b16(r, off + 16u, 0, 0);
    }
    __device__ __forceinline__ void get(float v[9]) const {
        const int w[4] = {(int)q.x, (int)q.y, (int)q.z, (int)q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = (float)((w[i] << 16) >> 16);
            v[2 * i + 1] = (float)(w[i] >> 16);
        }
        v[8] = (float)nx;
    }
};

template <>
struct RawGroup<__half> {
    v4u q;
    unsigned nx;
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        nx = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, off + 16u, 0, 0);
    }
    __device__ __forceinline__ void get(float v[9]) const {
        const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            __half_raw lo, hi;
            lo.x = (unsigned short)(w[i] & 0xFFFFu);
            hi.x = (unsigned short)(w[i] >> 16);
            v[2 * i] = __half2float(__half(lo));
            v[2 * i + 1] = __half2float(__half(hi));
        }
        __half_raw n;
        n.x = (unsigned short)(nx & 0xFFFFu);
        v[8] = __half2float(__half(n));
    }
};

template <>
struct RawGroup<float> {
    v4u a, b;
    unsigned nx;
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        b = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
        nx = __builtin_amdgcn_raw_buffer_load_b32(r, off + 32u, 0, 0);
    }
    __device__ __forceinline__ void get(float v[9]) const {
        v[0] = __uint_as_float(a.x); v[1] = __uint_as_float(a.y);
        v[2] = __uint_as_float(a.z); v[3] = __uint_as_float(a.w);
        v[4] = __uint_as_float(b.x); v[5] = __uint_as_float(b.y);
        v[6] = __uint_as_float(b.z); v[7] = __uint_as_float(b.w);
        v[8] = __uint_as_float(nx);
    }
};

// ---------------------------------------------------------------------------
// tile, per-transmit tables, pixels, delays
// ---------------------------------------------------------------------------

struct TileGeom {
    int iz0, ix0;            // first row / column of the tile
    float zlo, zhi, xlo, xhi;  // tile rectangle in samples (float)
};

// tile index -> rows [iz0, iz0 + TZ), columns [ix0, ix0 + TXW); a tile holds
// NT * PX pixels (NT threads per workgroup, PX pixels per thread)
template <int NT, int PX>
__device__ __forceinline__ TileGeom tile_geom(const DasArgs& a, int tile) {
    if (a.xcd_order) {
        // workgroups are dealt to the 8 XCDs round-robin: give XCD k the
        // contiguous tile range [k n/8, (k+1) n/8) so its L2 sees a narrow
        // band of the image (and of the RF)
        const int per = (a.ntz * a.ntx) >> 3;
        tile = (tile & 7) * per + (tile >> 3);
    }
    const int tzi = tile % a.ntz;
    const int txi = tile / a.ntz;
    const int TZ = 1 << a.tz_log2;
    const int TXW = (NT * PX) >> a.tz_log2;
    TileGeom g;
    g.iz0 = tzi * TZ;
    g.ix0 = txi * TXW;
    const int iz1 = min(g.iz0 + TZ, a.nz) - 1;
    const int ix1 = min(g.ix0 + TXW, a.nx) - 1;
    const float za = a.Z0.x + (float)g.iz0 * a.dZ.x, zb = a.Z0.x + (float)iz1 * a.dZ.x;
    const float xa = a.x0f + (float)g.ix0 * a.dxf, xb = a.x0f + (float)ix1 * a.dxf;
    g.zlo = fminf(za, zb);
    g.zhi = fmaxf(za, zb);
    g.xlo = fminf(xa, xb);
    g.xhi = fmaxf(xa, xb);
    return g;
}

// Per-transmit LDS tables of a tile, built by the whole workgroup:
//   m_tab[t] = (window base a_t, PWI column step, PWI tile base hi, lo) and
//   q_tab[t] = PWI (Az.hi, Az.lo, Ax.hi, Ax.lo) * 2^23 | STAI (DX.hi, DX.lo, xe, 0).
template <int MODE, int NT, int PX>
__device__ __forceinline__ void tx_tables(const DasArgs& a, const TileGeom& g, int4* m_tab,
                                          float4* q_tab) {
    const int TZ = 1 << a.tz_log2;
    const int TXW = (NT * PX) >> a.tz_log2;
    const int iz1 = min(g.iz0 + TZ, a.nz) - 1;
    const int ix1 = min(g.ix0 + TXW, a.nx) - 1;
    const float kstep = (float)(NT >> a.tz_log2);  // columns between a lane's pixels
    for (int t = threadIdx.x; t < a.T; t += NT) {
        const TxConst tc = a.tx_tab[t];
        int at, dq = 0;
        float2 pb = make_float2(0.0f, 0.0f);
        float4 q;
        if (MODE == 1) {
            const float c0 = tc.v0.x, az = tc.v0.z, ax = tc.v1.x;
            const float m00 = c0 + (float)g.iz0 * az + (float)g.ix0 * ax;
            const float m10 = c0 + (float)iz1 * az + (float)g.ix0 * ax;
            const float m01 = c0 + (float)g.iz0 * az + (float)ix1 * ax;
            const float m11 = c0 + (float)iz1 * az + (float)ix1 * ax;
            at = (int)floorf(fminf(fminf(m00, m10), fminf(m01, m11))) - 1;
            ff base = ff_make(tc.v0.x, tc.v0.y);
            base = ff_add(base, ff_mul_f(ff_make(tc.v0.z, tc.v0.w), (float)g.iz0));
            base = ff_add(base, ff_mul_f(ff_make(tc.v1.x, tc.v1.y), (float)g.ix0));
            base = ff_add_f(base, -(float)at);
            const float bh = rintf(base.hi * kHiQuant) * (1.0f / kHiQuant);
            const float bl = (base.hi - bh) + base.lo;
            pb = make_float2(bh * kQScale, bl * kQScale);
            q = make_float4(tc.v0.z * kQScale, tc.v0.w * kQScale, tc.v1.x * kQScale,
                            tc.v1.y * kQScale);
            // a lane's pixels are kstep columns apart: the delay grows by the
            // same Q9.23 step (rounded once; <= 1.5 units of error)
            dq = (int)rintf(fmaf(kstep, q.z, kstep * q.w));
        } else {
            at = (int)floorf(rect_min_dist(tc.v0.z, g.xlo, g.xhi, g.zlo, g.zhi) + a.O.x) - 1;
            q = tc.v0;
        }
        m_tab[t] = make_int4(at, dq, __float_as_int(pb.x), __float_as_int(pb.y));
        q_tab[t] = q;
    }
}

// The pixels of one lane: pixel k is q = k * NT + thread index of the tile
// (column-major inside the tile).
template <int PX>
struct PixelSet {
    float qz[PX], qx[PX];   // tile-local indices (exact in float)
    ff zp[PX], z2[PX];
    float xh[PX], xl[PX];   // lateral offset of the pixel from column 0, hi on the 2^-g grid
    bool valid[PX];
    int iz[PX], ix[PX];
};

// Pixel q = k NT + thread of the tile.  With WF_DAS_PATCH_LANES, each group
// of 16 lanes covers a 4 x 4 pixel patch (a wave: 16 deep x 4 wide, or 8 x 8
// in 8-deep tiles) instead of 16 consecutive rows of one column: the window
// entries one 16-lane group reads then span about 3 (dz + dx) samples
// instead of 15 dz, which keeps them in distinct LDS banks.  Pixel k of a
// lane stays k NT / TZ columns right of pixel 0 (the PWI transmit delay
// relies on it), and every pixel keeps its own accumulation order, so the
// output does not depend on the mapping.
#ifndef WF_DAS_PATCH_LANES
#define WF_DAS_PATCH_LANES 1
#endif

// The adjoint scatters with LDS atomics and passes PATCH = false: down one
// column the window entries rise with depth (both times of flight grow with
// z), so the lanes of a wave mostly hit distinct addresses, where a 4 x 4
// patch would pile several lanes onto each entry.
template <int NT, int PX, bool PATCH = (WF_DAS_PATCH_LANES != 0)>
__device__ __forceinline__ void pixel_set(const DasArgs& a, const TileGeom& g,
                                          PixelSet<PX>& p) {
    const int TZ = 1 << a.tz_log2;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int q = k * NT + (int)threadIdx.x;
        int qzi, qxi;
        if (PATCH) {
            const int l = q & 63, w = q >> 6;
            const int wz_log2 = a.tz_log2 >= 4 ? 4 : 3;  // wave slot 16 x 4 or 8 x 8
            const int lz = wz_log2 == 4 ? ((l & 3) | ((l >> 4) << 2))
                                        : ((l & 3) | (((l >> 4) & 1) << 2));
            const int lx = wz_log2 == 4 ? ((l >> 2) & 3) : (((l >> 2) & 3) | ((l >> 5) << 2));
            const int nzs_log2 = a.tz_log2 - wz_log2;  // wave slots down a tile column
            qzi = ((w & ((1 << nzs_log2) - 1)) << wz_log2) + lz;
            qxi = ((w >> nzs_log2) << (6 - wz_log2)) + lx;
        } else {
            qzi = q & (TZ - 1);
            qxi = q >> a.tz_log2;
        }
        const int iz = g.iz0 + qzi, ix = g.ix0 + qxi;
        p.iz[k] = iz;
        p.ix[k] = ix;
        p.valid[k] = (iz < a.nz) && (ix < a.nx);
        p.qz[k] = (float)qzi;
        p.qx[k] = (float)qxi;
        p.zp[k] = ff_add(ff_make(a.Z0.x, a.Z0.y), ff_mul_f(ff_make(a.dZ.x, a.dZ.y), (float)iz));
        p.z2[k] = ff_sqr(p.zp[k]);
        const ff ixdx = ff_mul_f(ff_make(a.dX.x, a.dX.y), (float)ix);
        p.xh[k] = rintf(ixdx.hi * a.dxq) * a.inv_dxq;
        p.xl[k] = (ixdx.hi - p.xh[k]) + ixdx.lo;
    }
}

// Channel bases of a chunk (threads first_thread .. + kChunk - 1): b_tab[j] = integer base of
// the receive delay over the tile, b_tab[kChunk + j] = 1 if the receive
// aperture of channel c0 + j reaches the tile (one sample of margin).
__device__ __forceinline__ void chunk_tables(const DasArgs& a, const TileGeom& g, int c0,
                                             int* b_tab, int first_thread = 0) {
    // this thread's channel of the chunk; threads outside
    // [first_thread, first_thread + kChunk) have none
    const int tid = (int)threadIdx.x - first_thread;
    if (tid >= 0 && tid < kChunk) {
        const int c = c0 + tid;
        int b = 0, act = 0;
        if (c < a.C) {
            const float xe = a.ch_tab[c].z;
            b = (int)floorf(rect_min_dist(xe, g.xlo, g.xhi, g.zlo, g.zhi)) - 1;
            const float dxm = fmaxf(0.0f, fmaxf(g.xlo - xe, xe - g.xhi));
            act = !(a.fnum2 > 0.0f) || (a.fnum2 * dxm <= g.zhi + 1.0f);
        }
        b_tab[tid] = b;
        b_tab[kChunk + tid] = act;
    }
}

// Window-local receive delays (Q9.23) of a chunk for this lane's pixels;
// apodised channels and pixels outside the grid point into the zero pad.
template <int PX>
__device__ __forceinline__ void rx_delays(const DasArgs& a, const PixelSet<PX>& p, int c0,
                                          const int* bj, uint32_t rq[PX][kChunk]) {
    const uint32_t masked = (uint32_t)a.nst << kQBits;
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
        const int c = c0 + j;
        if (c < a.C) {
            const ChConst cc = a.ch_tab[c];
            const float bq = (float)bj[j] * kQScale;
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const float dxh = cc.x + p.xh[k];  // exact: both on the 2^-g grid
                const float dxl = cc.y + p.xl[k];
                const bool on = p.valid[k] &&
                                !(a.fnum2 > 0.0f && a.fnum2 * fabsf(dxh + dxl) > p.zp[k].hi);
                const uint32_t q = min(dist_q_grid(dxh, dxl, p.z2[k], bq), a.rxspan_q);
                rq[k][j] = on ? q : masked;
            }
        } else {
#pragma unroll
            for (int k = 0; k < PX; ++k) rq[k][j] = masked;
        }
    }
}

// Window-local transmit delays (Q9.23) of transmit t for this lane's pixels.
template <int MODE, int PX>
__device__ __forceinline__ void tx_delays(const DasArgs& a, const PixelSet<PX>& p, int4 m,
                                          float4 q, int at, uint32_t tq[PX]) {
    if (MODE == 1) {
        // exact: every term is a multiple of 2^8 below 2^32
        const float s = fmaf(p.qz[0], q.x, fmaf(p.qx[0], q.z, __int_as_float(m.z)));
        const float l = fmaf(p.qz[0], q.y, fmaf(p.qx[0], q.w, __int_as_float(m.w)));
        const uint32_t q0 = (uint32_t)fmaxf(s, 0.0f) + (uint32_t)(int)rintf(l);
        const int dq = __builtin_amdgcn_readfirstlane(m.y);
#pragma unroll
        for (int k = 0; k < PX; ++k) tq[k] = min(q0 + (uint32_t)(k * dq), a.txspan_q);
    } else {
        if (a.O.x == 0.0f && a.O.y == 0.0f) {  // t0 = 0: window-local distance
            const float bq = (float)at * kQScale;
#pragma unroll
            for (int k = 0; k < PX; ++k)
                tq[k] = min(dist_q_grid(q.x + p.xh[k], q.y + p.xl[k], p.z2[k], bq), a.txspan_q);
        } else {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const ff d = ff_add(ff_make(q.x + p.xh[k], 0.0f), ff_make(q.y + p.xl[k], 0.0f));
                const ff v = ff_add(dist_ff(d, p.z2[k]), ff_make(a.O.x, a.O.y));
                tq[k] = min(to_q(v, at), a.txspan_q);
            }
        }
    }
}

}  // namespace
}  // namespace wf
