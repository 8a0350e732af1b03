// Delay-and-Sum kernels for gfx950: delay geometry (K1) and the LDS-staged
// gather / linear-interpolate / accumulate (K2), for synthetic transmit
// aperture (STAI) and plane-wave (PWI) imaging (WaveFlow, Sec. II-B).
//
// K2 design (one workgroup = 256 lanes = one tile of 256*PX pixels):
//  * Delays are split into a window base and a window-local part.  For a
//    tile, transmit t gets an integer base a_t <= min over the tile of its
//    transmit delay, channel c a base b_c <= min of its receive delay; the
//    RF window of the pair (t, c) then starts at sample a_t + b_c and the
//    local delays are small (< 512 samples), stored as unsigned Q9.23
//    fixed point.  Their integer sum is exact, its top 9 bits index the
//    LDS window and its 23 low bits are, verbatim, the mantissa of the
//    float 1 + frac.
//  * Local delays are formed in float-float FP32 (ff.h) and rounded once,
//    so the fractional sample index carries ~1e-7 samples of error where a
//    plain FP32 time of flight near sample 2000 would carry ~1e-4.
//  * Each window entry holds the pair (2 r[n] - r[n+1], r[n+1] - r[n]), so
//    one 8-byte LDS read and one FMA give the interpolated sample:
//    (2 r0 - r1) + (1 + frac)(r1 - r0) = r0 + frac (r1 - r0).  Entries
//    outside 0 <= n <= S-2 are zero, so the inner loop has no bounds test.
//  * Receive apodisation and pixels outside the grid point the receive
//    delay into a zero pad behind the staged window: masked pairs cost the
//    same instructions and add exactly 0.
//  * Loop nest: channel chunks of 16 (receive delays in registers) x all
//    transmits (transmit delays recomputed per chunk; the PWI transmit
//    delay is linear in the pixel indices and is evaluated exactly from a
//    per-tile float-float base) x 16 channels x PX pixels.
//  * Accumulation is FP32, in a fixed order per pixel: results are bitwise
//    reproducible run to run.
#pragma clang fp contract(off)

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "ff.h"
#include "wf_internal.h"

namespace wf {
namespace {

constexpr float kQScale = 8388608.0f;  // 2^23
constexpr float kHiQuant = 32768.0f;   // 2^15: grid of the exact "hi" parts

// ---------------------------------------------------------------------------
// RF sample loaders: 8 consecutive samples from a 16-byte aligned address.
// ---------------------------------------------------------------------------
template <typename RT>
struct RfLoad;

template <>
struct RfLoad<int16_t> {
    static __device__ __forceinline__ void load8(const int16_t* p, float v[8]) {
        const int4 q = *reinterpret_cast<const int4*>(p);
        const int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = (float)((w[i] << 16) >> 16);
            v[2 * i + 1] = (float)(w[i] >> 16);
        }
    }
    static __device__ __forceinline__ float load1(const int16_t* p) { return (float)*p; }
};

template <>
struct RfLoad<__half> {
    static __device__ __forceinline__ void load8(const __half* p, float v[8]) {
        const int4 q = *reinterpret_cast<const int4*>(p);
        const int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            __half_raw lo, hi;
            lo.x = (unsigned short)(w[i] & 0xFFFF);
            hi.x = (unsigned short)((unsigned)w[i] >> 16);
            v[2 * i] = __half2float(__half(lo));
            v[2 * i + 1] = __half2float(__half(hi));
        }
    }
    static __device__ __forceinline__ float load1(const __half* p) { return __half2float(*p); }
};

template <>
struct RfLoad<float> {
    static __device__ __forceinline__ void load8(const float* p, float v[8]) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        const float4 b = *reinterpret_cast<const float4*>(p + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
    static __device__ __forceinline__ float load1(const float* p) { return *p; }
};

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

// Smallest distance (samples) from an element at (xe, 0) to the rectangle
// [xlo, xhi] x [zlo, zhi]; plain float, used only for window bases that
// carry a one-sample margin.
__device__ __forceinline__ float rect_min_dist(float xe, float xlo, float xhi, float zlo,
                                               float zhi) {
    float dx = fmaxf(0.0f, fmaxf(xlo - xe, xe - xhi));
    float dz = fminf(fmaxf(0.0f, zlo), zhi);
    return sqrtf(dx * dx + dz * dz);
}

// ---------------------------------------------------------------------------
// K2: gather / interpolate / accumulate
// ---------------------------------------------------------------------------
template <int MODE, typename RT, int PX>
__global__ void __launch_bounds__(kThreads) das_kernel(const DasArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int slot = a.slot;
    float2* win = reinterpret_cast<float2*>(smem);
    const size_t win_bytes = (size_t)kChunk * slot * sizeof(float2);
    int* a_tab = reinterpret_cast<int*>(smem + win_bytes);
    float2* p_tab = reinterpret_cast<float2*>(smem + win_bytes + ((a.T * 4 + 15) & ~15));
    int* b_tab = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(p_tab) + a.T * 8);

    const int frame = blockIdx.y;
    const int tile = blockIdx.x;
    const int tzi = tile % a.ntz;
    const int txi = tile / a.ntz;
    const int TZ = 1 << a.tz_log2;
    const int TXW = (kThreads * PX) >> a.tz_log2;
    const int iz0 = tzi * TZ;
    const int ix0 = txi * TXW;
    const int iz1 = min(iz0 + TZ, a.nz) - 1;
    const int ix1 = min(ix0 + TXW, a.nx) - 1;

    // tile rectangle in samples (float), for the window bases
    const float za = a.Z0.x + (float)iz0 * a.dZ.x, zb = a.Z0.x + (float)iz1 * a.dZ.x;
    const float xa = a.x0f + (float)ix0 * a.dxf, xb = a.x0f + (float)ix1 * a.dxf;
    const float zlo = fminf(za, zb), zhi = fmaxf(za, zb);
    const float xlo = fminf(xa, xb), xhi = fmaxf(xa, xb);

    // ---- per-transmit window bases for this tile --------------------------
    for (int t = tid; t < a.T; t += kThreads) {
        const TxConst tc = a.tx_tab[t];
        int at;
        if (MODE == 1) {
            const float c0 = tc.v0.x, az = tc.v0.z, ax = tc.v1.x;
            const float m00 = c0 + (float)iz0 * az + (float)ix0 * ax;
            const float m10 = c0 + (float)iz1 * az + (float)ix0 * ax;
            const float m01 = c0 + (float)iz0 * az + (float)ix1 * ax;
            const float m11 = c0 + (float)iz1 * az + (float)ix1 * ax;
            at = (int)floorf(fminf(fminf(m00, m10), fminf(m01, m11))) - 1;
            ff base = ff_make(tc.v0.x, tc.v0.y);
            base = ff_add(base, ff_mul_f(ff_make(tc.v0.z, tc.v0.w), (float)iz0));
            base = ff_add(base, ff_mul_f(ff_make(tc.v1.x, tc.v1.y), (float)ix0));
            base = ff_add_f(base, -(float)at);
            const float bh = rintf(base.hi * kHiQuant) * (1.0f / kHiQuant);
            const float bl = (base.hi - bh) + base.lo;
            p_tab[t] = make_float2(bh * kQScale, bl * kQScale);
        } else {
            at = (int)floorf(rect_min_dist(tc.v0.z, xlo, xhi, zlo, zhi) + a.O.x) - 1;
        }
        a_tab[t] = at;
    }
    // zero pad behind every window (never overwritten by staging)
    {
        const int pad = slot - a.nst;
        for (int i = tid; i < kChunk * pad; i += kThreads) {
            const int j = i / pad;
            win[j * slot + a.nst + (i - j * pad)] = make_float2(0.0f, 0.0f);
        }
    }

    // ---- this lane's pixels ------------------------------------------------
    float qz[PX], qx[PX], acc[PX];
    ff zp[PX], z2[PX], ixdx[PX];
    bool valid[PX];
    int pix_iz[PX], pix_ix[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int q = k * kThreads + tid;
        const int qzi = q & (TZ - 1);
        const int qxi = q >> a.tz_log2;
        const int iz = iz0 + qzi, ix = ix0 + qxi;
        pix_iz[k] = iz;
        pix_ix[k] = ix;
        valid[k] = (iz < a.nz) && (ix < a.nx);
        qz[k] = (float)qzi;
        qx[k] = (float)qxi;
        zp[k] = ff_add(ff_make(a.Z0.x, a.Z0.y), ff_mul_f(ff_make(a.dZ.x, a.dZ.y), (float)iz));
        z2[k] = ff_sqr(zp[k]);
        ixdx[k] = ff_mul_f(ff_make(a.dX.x, a.dX.y), (float)ix);
        acc[k] = 0.0f;
    }
    const uint32_t masked = (uint32_t)a.nst << kQBits;
    const RT* rf_frame = reinterpret_cast<const RT*>(a.rf) + (size_t)frame * a.T * a.C * a.S;

    for (int c0 = 0; c0 < a.C; c0 += kChunk) {
        __syncthreads();  // previous chunk's readers of b_tab / windows are done
        if (tid < kChunk) {
            const int c = c0 + tid;
            int b = 0;
            if (c < a.C) b = (int)floorf(rect_min_dist(a.ch_tab[c].z, xlo, xhi, zlo, zhi)) - 1;
            b_tab[tid] = b;
        }
        __syncthreads();
        int bj[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) bj[j] = __builtin_amdgcn_readfirstlane(b_tab[j]);

        // receive delays of this chunk, window-local Q9.23
        uint32_t rq[PX][kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            const int c = c0 + j;
            if (c < a.C) {
                const ChConst cc = a.ch_tab[c];
#pragma unroll
                for (int k = 0; k < PX; ++k) {
                    const ff d = ff_add(ff_make(cc.x, cc.y), ixdx[k]);
                    const bool on =
                        valid[k] && !(a.fnum2 > 0.0f && a.fnum2 * fabsf(d.hi) > zp[k].hi);
                    const uint32_t q = min(to_q(dist_ff(d, z2[k]), bj[j]), a.rxspan_q);
                    rq[k][j] = on ? q : masked;
                }
            } else {
#pragma unroll
                for (int k = 0; k < PX; ++k) rq[k][j] = masked;
            }
        }

        for (int t = 0; t < a.T; ++t) {
            const int at = __builtin_amdgcn_readfirstlane(a_tab[t]);
            uint32_t tq[PX];
            if (MODE == 1) {
                const float2 pb = p_tab[t];
                const TxConst tc = a.tx_tab[t];
                const float azh = tc.v0.z * kQScale, azl = tc.v0.w * kQScale;
                const float axh = tc.v1.x * kQScale, axl = tc.v1.y * kQScale;
#pragma unroll
                for (int k = 0; k < PX; ++k) {
                    // exact: every term is a multiple of 2^8 below 2^32
                    const float s = fmaf(qz[k], azh, fmaf(qx[k], axh, pb.x));
                    const float l = fmaf(qz[k], azl, fmaf(qx[k], axl, pb.y));
                    const uint32_t q = (uint32_t)fmaxf(s, 0.0f) + (uint32_t)(int)rintf(l);
                    tq[k] = min(q, a.txspan_q);
                }
            } else {
                const TxConst tc = a.tx_tab[t];
#pragma unroll
                for (int k = 0; k < PX; ++k) {
                    const ff d = ff_add(ff_make(tc.v0.x, tc.v0.y), ixdx[k]);
                    const ff v = ff_add(dist_ff(d, z2[k]), ff_make(a.O.x, a.O.y));
                    tq[k] = min(to_q(v, at), a.txspan_q);
                }
            }

            __syncthreads();  // everyone is done reading the previous windows
            // ---- stage windows (t, c0 .. c0+15) into LDS ------------------
            {
                const RT* rf_t = rf_frame + (size_t)t * a.C * a.S;
                for (int w = tid; w < kChunk * a.ng; w += kThreads) {
                    const int j = (w * a.ng_inv) >> 20;
                    const int g = w - j * a.ng;
                    const int c = c0 + j;
                    const int n0 = at + b_tab[j];
                    const int s0 = (n0 & ~7) + 8 * g;
                    float v[8];
                    float nxt = 0.0f;
                    const bool inr = (c < a.C) && (s0 >= 0) && (s0 + 8 <= a.S);
                    if (inr) {
                        const RT* row = rf_t + (size_t)c * a.S;
                        RfLoad<RT>::load8(row + s0, v);
                        if (s0 + 8 <= a.S - 1) nxt = RfLoad<RT>::load1(row + s0 + 8);
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) v[i] = 0.0f;
                    }
                    float4* dst = reinterpret_cast<float4*>(win + j * slot + 8 * g);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float e[2], d[2];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int m = 2 * i + h;
                            const float r0 = v[m];
                            const float r1 = (m < 7) ? v[m + 1] : nxt;
                            const bool ok = inr && (s0 + m <= a.S - 2);
                            e[h] = ok ? fmaf(2.0f, r0, -r1) : 0.0f;
                            d[h] = ok ? (r1 - r0) : 0.0f;
                        }
                        dst[i] = make_float4(e[0], d[0], e[1], d[1]);
                    }
                }
            }
            __syncthreads();

            // ---- gather / interpolate / accumulate -------------------------
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                const uint32_t off = (uint32_t)(j * slot + ((at + bj[j]) & 7)) * 8u;
#pragma unroll
                for (int k = 0; k < PX; ++k) {
                    const uint32_t u = tq[k] + rq[k][j];
                    const uint32_t idx = u >> kQBits;
                    const float f1 = __uint_as_float((u & 0x7FFFFFu) | 0x3F800000u);
                    const float2 ed = *reinterpret_cast<const float2*>(smem + off + idx * 8u);
                    acc[k] += fmaf(f1, ed.y, ed.x);
                }
            }
        }
    }

#pragma unroll
    for (int k = 0; k < PX; ++k)
        if (valid[k]) a.out[((size_t)frame * a.nz + pix_iz[k]) * a.nx + pix_ix[k]] = acc[k];
}

// ---------------------------------------------------------------------------
// K1: one-way delays of every pixel, float-float (for verification)
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(256) delays_kernel(const DelayArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int npix = a.nz * a.nx;
    if (p >= npix) return;
    const int iz = p / a.nx, ix = p - (p / a.nx) * a.nx;
    const ff zp = ff_add(ff_make(a.Z0.x, a.Z0.y), ff_mul_f(ff_make(a.dZ.x, a.dZ.y), (float)iz));
    const ff z2 = ff_sqr(zp);
    const ff ixdx = ff_mul_f(ff_make(a.dX.x, a.dX.y), (float)ix);
    for (int t = 0; t < a.T; ++t) {
        const TxConst tc = a.tx_tab[t];
        ff v;
        if (MODE == 1) {
            v = ff_make(tc.v0.x, tc.v0.y);
            v = ff_add(v, ff_mul_f(ff_make(tc.v0.z, tc.v0.w), (float)iz));
            v = ff_add(v, ff_mul_f(ff_make(tc.v1.x, tc.v1.y), (float)ix));
        } else {
            const ff d = ff_add(ff_make(tc.v0.x, tc.v0.y), ixdx);
            v = ff_add(dist_ff(d, z2), ff_make(a.O.x, a.O.y));
        }
        a.tx_hi[(size_t)t * npix + p] = v.hi;
        a.tx_lo[(size_t)t * npix + p] = v.lo;
    }
    for (int c = 0; c < a.C; ++c) {
        const ChConst cc = a.ch_tab[c];
        const ff v = dist_ff(ff_add(ff_make(cc.x, cc.y), ixdx), z2);
        a.rx_hi[(size_t)c * npix + p] = v.hi;
        a.rx_lo[(size_t)c * npix + p] = v.lo;
    }
}

template <int MODE, typename RT>
hipError_t launch_px(int px, const DasArgs& a, size_t lds, hipStream_t s) {
    dim3 grid((unsigned)(a.ntz * a.ntx), (unsigned)a.F);
    dim3 block(kThreads);
    if (px == 4) {
        hipLaunchKernelGGL((das_kernel<MODE, RT, 4>), grid, block, lds, s, a);
    } else {
        hipLaunchKernelGGL((das_kernel<MODE, RT, 1>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(int dtype, int px, const DasArgs& a, size_t lds, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_px<MODE, int16_t>(px, a, lds, s);
        case 1: return launch_px<MODE, __half>(px, a, lds, s);
        default: return launch_px<MODE, float>(px, a, lds, s);
    }
}

}  // namespace

hipError_t launch_das(int mode, int dtype, int px, const DasArgs& a, size_t lds_bytes,
                      hipStream_t s) {
    return mode == 1 ? launch_mode<1>(dtype, px, a, lds_bytes, s)
                     : launch_mode<0>(dtype, px, a, lds_bytes, s);
}

hipError_t launch_delays(int mode, const DelayArgs& a, hipStream_t s) {
    const int npix = a.nz * a.nx;
    dim3 grid((unsigned)((npix + 255) / 256));
    if (mode == 1) {
        hipLaunchKernelGGL((delays_kernel<1>), grid, dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((delays_kernel<0>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace wf
