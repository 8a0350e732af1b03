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
constexpr int kJB = 2;                 // channels per batch of LDS reads

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

typedef float v2f __attribute__((ext_vector_type(2)));

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

// ---------------------------------------------------------------------------
// K2: gather / interpolate / accumulate
// ---------------------------------------------------------------------------

// Raw RF of one staged group (8 samples + the next one), held in registers
// between the global load and the LDS commit so that the load latency hides
// behind the previous transmit's arithmetic.
template <typename RT>
struct RawGroup;

template <>
struct RawGroup<int16_t> {
    int4 q;
    int nx;
    __device__ __forceinline__ void load(const int16_t* p, bool next) {
        q = *reinterpret_cast<const int4*>(p);
        nx = next ? (int)p[8] : 0;
    }
    __device__ __forceinline__ void zero() { q = make_int4(0, 0, 0, 0); nx = 0; }
    __device__ __forceinline__ void get(float v[9]) const {
        const int w[4] = {q.x, q.y, q.z, q.w};
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
    int4 q;
    float nx;
    __device__ __forceinline__ void load(const __half* p, bool next) {
        q = *reinterpret_cast<const int4*>(p);
        nx = next ? __half2float(p[8]) : 0.0f;
    }
    __device__ __forceinline__ void zero() { q = make_int4(0, 0, 0, 0); nx = 0.0f; }
    __device__ __forceinline__ void get(float v[9]) const {
        const int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            __half_raw lo, hi;
            lo.x = (unsigned short)(w[i] & 0xFFFF);
            hi.x = (unsigned short)((unsigned)w[i] >> 16);
            v[2 * i] = __half2float(__half(lo));
            v[2 * i + 1] = __half2float(__half(hi));
        }
        v[8] = nx;
    }
};

template <>
struct RawGroup<float> {
    float4 a, b;
    float nx;
    __device__ __forceinline__ void load(const float* p, bool next) {
        a = *reinterpret_cast<const float4*>(p);
        b = *reinterpret_cast<const float4*>(p + 4);
        nx = next ? p[8] : 0.0f;
    }
    __device__ __forceinline__ void zero() {
        a = make_float4(0, 0, 0, 0);
        b = a;
        nx = 0.0f;
    }
    __device__ __forceinline__ void get(float v[9]) const {
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        v[8] = nx;
    }
};

template <int MODE, typename RT, int PX, int NG>
__global__ void __launch_bounds__(kThreads) das_kernel(const DasArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int slot = a.slot;
    const uint32_t buf_bytes = (uint32_t)kChunk * slot * sizeof(float2);
    float2* win = reinterpret_cast<float2*>(smem);  // two buffers of kChunk windows
    // per transmit: (window base a_t, PWI column step, PWI tile base hi, lo)
    int4* m_tab = reinterpret_cast<int4*>(smem + 2 * buf_bytes);
    // per transmit: PWI (Az.hi, Az.lo, Ax.hi, Ax.lo) * 2^23; STAI (DX.hi, DX.lo, xe, 0)
    float4* q_tab = reinterpret_cast<float4*>(m_tab + a.T);
    int* b_tab = reinterpret_cast<int*>(q_tab + a.T);
    // LDS byte offset of the window buffers (folded into scalar offsets)
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)smem;

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

    // ---- per-transmit window bases and constants for this tile -------------
    const float kstep = (float)(kThreads >> a.tz_log2);  // columns between a lane's pixels
    for (int t = tid; t < a.T; t += kThreads) {
        const TxConst tc = a.tx_tab[t];
        int at, dq = 0;
        float2 pb = make_float2(0.0f, 0.0f);
        float4 q;
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
            pb = make_float2(bh * kQScale, bl * kQScale);
            q = make_float4(tc.v0.z * kQScale, tc.v0.w * kQScale, tc.v1.x * kQScale,
                            tc.v1.y * kQScale);
            // a lane's pixels are kstep columns apart: the delay grows by the
            // same Q9.23 step (rounded once; <= 1.5 units of error)
            dq = (int)rintf(fmaf(kstep, q.z, kstep * q.w));
        } else {
            at = (int)floorf(rect_min_dist(tc.v0.z, xlo, xhi, zlo, zhi) + a.O.x) - 1;
            q = tc.v0;
        }
        m_tab[t] = make_int4(at, dq, __float_as_int(pb.x), __float_as_int(pb.y));
        q_tab[t] = q;
    }
    // zero pad behind every window of both buffers (never overwritten)
    {
        const int pad = slot - a.nst;
        for (int i = tid; i < 2 * kChunk * pad; i += kThreads) {
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
    const int ngroups = kChunk * a.ng;  // staged 8-sample groups per pass (<= NG * 256)

    for (int c0 = 0; c0 < a.C; c0 += kChunk) {
        __syncthreads();  // previous chunk's readers of b_tab / windows are done
        if (tid < kChunk) {
            const int c = c0 + tid;
            int b = 0, act = 0;
            if (c < a.C) {
                const float xe = a.ch_tab[c].z;
                b = (int)floorf(rect_min_dist(xe, xlo, xhi, zlo, zhi)) - 1;
                // does the receive aperture of this channel reach any pixel
                // of the tile?  (one sample of margin)
                const float dxm = fmaxf(0.0f, fmaxf(xlo - xe, xe - xhi));
                act = !(a.fnum2 > 0.0f) || (a.fnum2 * dxm <= zhi + 1.0f);
            }
            b_tab[tid] = b;
            b_tab[kChunk + tid] = act;
        }
        __syncthreads();
        int bj[kChunk];
        int any_act = 0, bmin = 0x7fffffff, bmax = -0x7fffffff;
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            bj[j] = __builtin_amdgcn_readfirstlane(b_tab[j]);
            any_act |= __builtin_amdgcn_readfirstlane(b_tab[kChunk + j]);
            bmin = min(bmin, bj[j]);
            bmax = max(bmax, bj[j]);
        }
        if (!any_act) continue;  // the whole chunk is outside the tile's aperture

        // a transmit pass whose windows all lie outside the record adds nothing
        auto next_active = [&](int t) {
            for (; t < a.T; ++t) {
                const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
                if (!(at + bmin > a.S - 2 || at + bmax + a.nst < 0)) break;
            }
            return t;
        };

        // global -> registers for pass t (nothing written yet)
        RawGroup<RT> raw[NG];
        auto issue = [&](int t) {
            const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
            const RT* rf_t = rf_frame + (size_t)t * a.C * a.S;
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                const int w = tid + gi * kThreads;
                if (w < ngroups) {
                    const int j = (w * a.ng_inv) >> 20;
                    const int g = w - j * a.ng;
                    const int c = c0 + j;
                    const int s0 = ((at + b_tab[j]) & ~7) + 8 * g;
                    if (c < a.C && s0 >= 0 && s0 + 8 <= a.S)
                        raw[gi].load(rf_t + (size_t)c * a.S + s0, s0 + 8 <= a.S - 1);
                    else
                        raw[gi].zero();
                }
            }
        };
        // registers -> interpolation pairs in LDS buffer `buf`
        auto commit = [&](int t, int buf) {
            const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                const int w = tid + gi * kThreads;
                if (w < ngroups) {
                    const int j = (w * a.ng_inv) >> 20;
                    const int g = w - j * a.ng;
                    const int c = c0 + j;
                    const int s0 = ((at + b_tab[j]) & ~7) + 8 * g;
                    float v[9];
                    raw[gi].get(v);
                    float4* dst =
                        reinterpret_cast<float4*>(win + (buf * kChunk + j) * slot + 8 * g);
                    if (c < a.C && s0 >= 0 && s0 + 8 <= a.S - 1) {
                        // whole group inside the record: every pair is valid
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            dst[i] = make_float4(fmaf(2.0f, v[2 * i], -v[2 * i + 1]),
                                                 v[2 * i + 1] - v[2 * i],
                                                 fmaf(2.0f, v[2 * i + 1], -v[2 * i + 2]),
                                                 v[2 * i + 2] - v[2 * i + 1]);
                    } else {
                        // record edge or outside: pairs with n < 0 or n > S-2 are 0
                        const bool inr = (c < a.C) && (s0 >= 0) && (s0 + 8 <= a.S);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float e[2], d[2];
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int m = 2 * i + h;
                                const bool ok = inr && (s0 + m <= a.S - 2);
                                e[h] = ok ? fmaf(2.0f, v[m], -v[m + 1]) : 0.0f;
                                d[h] = ok ? (v[m + 1] - v[m]) : 0.0f;
                            }
                            dst[i] = make_float4(e[0], d[0], e[1], d[1]);
                        }
                    }
                }
            }
        };

        int t = next_active(0);
        if (t >= a.T) continue;  // no transmit reaches this tile through this chunk

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
                    const uint32_t q = min(dist_q(d, z2[k], bj[j]), a.rxspan_q);
                    rq[k][j] = on ? q : masked;
                }
            } else {
#pragma unroll
                for (int k = 0; k < PX; ++k) rq[k][j] = masked;
            }
        }

        // software pipeline over transmit passes, two LDS buffers: commit
        // pass t into buffer `cur` (last read two passes ago, before the
        // barrier of the previous iteration), barrier, then issue the loads
        // of the next pass so that they fly while pass t is accumulated
        issue(t);
        int cur = 0;
        while (t < a.T) {
            const int tn = next_active(t + 1);
            commit(t, cur);
            __syncthreads();
            if (tn < a.T) issue(tn);
            const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);

            uint32_t tq[PX];
            if (MODE == 1) {
                const int4 m = m_tab[t];
                const float4 q = q_tab[t];
                // exact: every term is a multiple of 2^8 below 2^32
                const float s = fmaf(qz[0], q.x, fmaf(qx[0], q.z, __int_as_float(m.z)));
                const float l = fmaf(qz[0], q.y, fmaf(qx[0], q.w, __int_as_float(m.w)));
                const uint32_t q0 = (uint32_t)fmaxf(s, 0.0f) + (uint32_t)(int)rintf(l);
                const int dq = __builtin_amdgcn_readfirstlane(m.y);
#pragma unroll
                for (int k = 0; k < PX; ++k) tq[k] = min(q0 + (uint32_t)(k * dq), a.txspan_q);
            } else {
                const float4 q = q_tab[t];
#pragma unroll
                for (int k = 0; k < PX; ++k) {
                    const ff d = ff_add(ff_make(q.x, q.y), ixdx[k]);
                    const ff v = ff_add(dist_ff(d, z2[k]), ff_make(a.O.x, a.O.y));
                    tq[k] = min(to_q(v, at), a.txspan_q);
                }
            }

            // ---- gather / interpolate / accumulate -------------------------
            // batches of LDS reads are issued before their FMAs so that
            // several reads are in flight per wave
            const uint32_t base = lds0 + (uint32_t)cur * buf_bytes;
#pragma unroll
            for (int j0 = 0; j0 < kChunk; j0 += kJB) {
                float2 ed[kJB][PX];
                float f1[kJB][PX];
#pragma unroll
                for (int jj = 0; jj < kJB; ++jj) {
                    const int j = j0 + jj;
                    const uint32_t off =
                        base + (uint32_t)(j * slot + ((at + bj[j]) & 7)) * 8u;
#pragma unroll
                    for (int k = 0; k < PX; ++k) {
                        const uint32_t u = tq[k] + rq[k][j];
                        f1[jj][k] = __uint_as_float((u & 0x7FFFFFu) | 0x3F800000u);
                        const v2f e2 = *reinterpret_cast<const __attribute__((address_space(3))) v2f*>(
                            (uintptr_t)entry_addr(u, off));
                        ed[jj][k] = make_float2(e2.x, e2.y);
                    }
                }
#pragma unroll
                for (int jj = 0; jj < kJB; ++jj)
#pragma unroll
                    for (int k = 0; k < PX; ++k)
                        acc[k] += fmaf(f1[jj][k], ed[jj][k].y, ed[jj][k].x);
            }

            cur ^= 1;
            t = tn;
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

template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int MODE, typename RT, int PX, int NG>
hipError_t launch_one(const DasArgs& a, size_t lds, hipStream_t s) {
    hipError_t e = allow_lds(das_kernel<MODE, RT, PX, NG>, lds);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)(a.ntz * a.ntx), (unsigned)a.F);
    hipLaunchKernelGGL((das_kernel<MODE, RT, PX, NG>), grid, dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

template <int MODE, typename RT>
hipError_t launch_px(int px, int groups, const DasArgs& a, size_t lds, hipStream_t s) {
    if (px == 4)
        return groups <= 2 ? launch_one<MODE, RT, 4, 2>(a, lds, s)
                           : launch_one<MODE, RT, 4, 4>(a, lds, s);
    return groups <= 2 ? launch_one<MODE, RT, 1, 2>(a, lds, s)
                       : launch_one<MODE, RT, 1, 4>(a, lds, s);
}

template <int MODE>
hipError_t launch_mode(int dtype, int px, int groups, const DasArgs& a, size_t lds,
                       hipStream_t s) {
    switch (dtype) {
        case 0: return launch_px<MODE, int16_t>(px, groups, a, lds, s);
        case 1: return launch_px<MODE, __half>(px, groups, a, lds, s);
        default: return launch_px<MODE, float>(px, groups, a, lds, s);
    }
}

}  // namespace

hipError_t launch_das(int mode, int dtype, int px, int groups, const DasArgs& a,
                      size_t lds_bytes, hipStream_t s) {
    if (groups > kMaxGroups) return hipErrorInvalidValue;
    return mode == 1 ? launch_mode<1>(dtype, px, groups, a, lds_bytes, s)
                     : launch_mode<0>(dtype, px, groups, a, lds_bytes, s);
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
