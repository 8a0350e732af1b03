// Envelope (K3) and log compression / clip (K4) for gfx950 (WaveFlow,
// Fig. 2: Analytic Signal -> Absolute Value -> Dynamic Adjustment; Hilbert
// transform by FFT, Sec. II-B; dB clip, Sec. III).
//
// K3: one workgroup per group of 1, 2 or 4 adjacent image columns.  Each
// column is an nz-point complex
// FFT in LDS: a decimation-in-frequency forward pass (natural order in,
// bit-reversed out), the one-sided multiplier applied at bit-reversed
// positions, and a decimation-in-time inverse pass (bit-reversed in,
// natural out), so no permutation pass is needed; radix-2 stages run two at
// a time (4 points per lane in registers between barriers).  Twiddles come from the
// device library's sincospi, once per workgroup.  The kernel writes the
// envelope and the maximum of each column; the frame maximum is reduced
// from the column maxima by K4, so no atomics and no memset are needed and
// the result is deterministic.
//
// K4: elementwise 20 log10(env / m_f) clipped to [-DR, 0], with m_f reduced
// from the column maxima of frame f by every workgroup.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "wf_internal.h"

namespace wf {
namespace {

constexpr int kEnvThreads = 256;
#ifndef WF_ENV_GROUPS4
#define WF_ENV_GROUPS4 512  // workgroups needed before 4-column groups are used
#endif

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(fmaf(a.x, w.x, -a.y * w.y), fmaf(a.x, w.y, a.y * w.x));
}
__device__ __forceinline__ float2 cmul_conj(float2 a, float2 w) {  // a * conj(w)
    return make_float2(fmaf(a.x, w.x, a.y * w.y), fmaf(a.y, w.x, -a.x * w.y));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// LDS index of column element i: one pad slot after every 16 elements (128
// bytes), so the power-of-two strides of the butterflies (32 bytes and up
// between lanes) spread over the banks instead of stacking 16 lanes on one.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// CPW adjacent columns (and one frame) per workgroup of 256 CPW threads;
// log_n = log2(nz).
// A row's CPW values are contiguous in memory, so a wave's load or store
// covers 64 / CPW rows with CPW-wide runs instead of 64 single words on 64
// cache lines.  Radix-2 stages are fused in pairs (two spans per pass
// through LDS, 4 points per lane in registers), halving the barriers; an odd
// stage count leaves one single stage (the first forward one, the last
// inverse one).  Column c of the workgroup lives at col[c n .. c n + n).
template <int CPW>
__global__ void __launch_bounds__(kEnvThreads * CPW)
    envelope_kernel(const float* bf, float* env, float* __restrict__ col_max, int nz, int nx,
                    int log_n) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kCpwLog2 = CPW == 4 ? 2 : (CPW == 2 ? 1 : 0);
    const int n = nz;
    const int half = n >> 1;
    float2* tw = reinterpret_cast<float2*>(smem);                 // [n/2]
    float2* col = tw + (half > 0 ? half : 1);                     // [CPW][n], padded
    constexpr int kThreads = kEnvThreads * CPW;  // 256 threads a column
    __shared__ float red[kThreads / 64][CPW];

    const int tid = threadIdx.x;
    // each XCD takes a contiguous block of column groups, so the columns of
    // a cache line meet in one L2 (dealt in order, each of the 8 L2s would
    // fetch and write back every line: 8x the traffic)
    const int x0 = xcd_contiguous((int)blockIdx.x, (int)gridDim.x) * CPW;
    const int f = blockIdx.y;
    const float* src = bf + (size_t)f * nz * nx + x0;
    float* dst = env + (size_t)f * nz * nx + x0;

    // W^k = exp(-2 pi i k / n)
    for (int k = tid; k < half; k += kThreads) {
        float sn, cs;
        sincospif(-2.0f * (float)k / (float)n, &sn, &cs);
        tw[k] = make_float2(cs, sn);
    }
    // element i: row i / CPW, column i % CPW (columns fastest: contiguous)
    for (int i = tid; i < (n << kCpwLog2); i += kThreads) {
        const int z = i >> kCpwLog2, c = i & (CPW - 1);
        col[pad((c << log_n) + z)] =
            make_float2(x0 + c < nx ? src[(size_t)z * nx + c] : 0.0f, 0.0f);
    }
    __syncthreads();

    // ---- forward DIF, spans n/2 .. 1 ------------------------------------
    int h = half;
    if (log_n & 1) {  // single stage of span n/2
        for (int g = tid; g < (half << kCpwLog2); g += kThreads) {
            const int b = g & (half - 1);
            const int cb = (g >> (log_n - 1)) << log_n;
            const float2 x0v = col[pad(cb + b)], x1v = col[pad(cb + b + h)];
            col[pad(cb + b)] = cadd(x0v, x1v);
            col[pad(cb + b + h)] = cmul(csub(x0v, x1v), tw[b]);
        }
        __syncthreads();
        h >>= 1;
    }
    for (; h >= 2; h >>= 2) {  // spans h and h/2 in one pass
        const int q = h >> 1, ts = half / h;
        for (int gg = tid; gg < (n >> 2 << kCpwLog2); gg += kThreads) {
            const int g = gg & ((n >> 2) - 1);
            const int cb = (gg >> (log_n - 2)) << log_n;
            const int pos = g & (q - 1);
            const int i0 = cb + ((g - pos) << 2) + pos;  // block of 2h
            const int j0 = pad(i0), j1 = pad(i0 + q), j2 = pad(i0 + h), j3 = pad(i0 + h + q);
            float2 a0 = col[j0], a1 = col[j1], a2 = col[j2], a3 = col[j3];
            const float2 b0 = cadd(a0, a2), b2 = cmul(csub(a0, a2), tw[pos * ts]);
            const float2 b1 = cadd(a1, a3), b3 = cmul(csub(a1, a3), tw[(pos + q) * ts]);
            const float2 w2 = tw[pos * 2 * ts];
            col[j0] = cadd(b0, b1);
            col[j1] = cmul(csub(b0, b1), w2);
            col[j2] = cadd(b2, b3);
            col[j3] = cmul(csub(b2, b3), w2);
        }
        __syncthreads();
    }
    // one-sided spectrum: position p holds bin k = bitrev(p)
    for (int i = tid; i < (n << kCpwLog2); i += kThreads) {
        const int p = i & (n - 1);
        const int k = log_n > 0 ? (int)(__brev((unsigned)p) >> (32 - log_n)) : 0;
        const float gk = (k == 0 || k == half) ? 1.0f : (k < half ? 2.0f : 0.0f);
        const float2 v = col[pad(i)];
        col[pad(i)] = make_float2(v.x * gk, v.y * gk);
    }
    __syncthreads();
    // ---- inverse DIT with conjugate twiddles, spans 1 .. n/2 -------------
    h = 1;
    const int pairs = log_n >> 1;
    for (int st = 0; st < pairs; ++st, h <<= 2) {  // spans h and 2h in one pass
        const int ts = half / h, ts2 = ts >> 1;
        for (int gg = tid; gg < (n >> 2 << kCpwLog2); gg += kThreads) {
            const int g = gg & ((n >> 2) - 1);
            const int cb = (gg >> (log_n - 2)) << log_n;
            const int pos = g & (h - 1);
            const int i0 = cb + ((g - pos) << 2) + pos;  // block of 4h
            const int j0 = pad(i0), j1 = pad(i0 + h), j2 = pad(i0 + 2 * h), j3 = pad(i0 + 3 * h);
            const float2 a0 = col[j0], a1 = col[j1], a2 = col[j2], a3 = col[j3];
            const float2 w1 = tw[pos * ts];
            const float2 t1 = cmul_conj(a1, w1), t3 = cmul_conj(a3, w1);
            const float2 b0 = cadd(a0, t1), b1 = csub(a0, t1);
            const float2 b2 = cadd(a2, t3), b3 = csub(a2, t3);
            const float2 u2 = cmul_conj(b2, tw[pos * ts2]);
            const float2 u3 = cmul_conj(b3, tw[(pos + h) * ts2]);
            col[j0] = cadd(b0, u2);
            col[j2] = csub(b0, u2);
            col[j1] = cadd(b1, u3);
            col[j3] = csub(b1, u3);
        }
        __syncthreads();
    }
    if (log_n & 1) {  // last single stage, span n/2
        for (int g = tid; g < (half << kCpwLog2); g += kThreads) {
            const int b = g & (half - 1);
            const int cb = (g >> (log_n - 1)) << log_n;
            const float2 t = cmul_conj(col[pad(cb + b + half)], tw[b]);
            const float2 x0v = col[pad(cb + b)];
            col[pad(cb + b)] = cadd(x0v, t);
            col[pad(cb + b + half)] = csub(x0v, t);
        }
        __syncthreads();
    }
    // modulus, store (same contiguous order as the load), column maxima: a
    // lane's elements all belong to column tid % CPW
    const float inv_n = 1.0f / (float)n;
    const int cl = tid & (CPW - 1);
    float m = 0.0f;
    for (int i = tid; i < (n << kCpwLog2); i += kThreads) {
        const int z = i >> kCpwLog2;
        const float2 v = col[pad((cl << log_n) + z)];
        const float e = sqrtf(fmaf(v.x, v.x, v.y * v.y)) * inv_n;
        if (x0 + cl < nx) dst[(size_t)z * nx + cl] = e;
        m = fmaxf(m, e);
    }
#pragma unroll
    for (int off = 32; off >= CPW; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((tid & 63) < CPW) red[tid >> 6][tid & 63] = m;
    __syncthreads();
    if (tid < CPW && x0 + tid < nx) {
        float r = red[0][tid];
        for (int w = 1; w < kThreads / 64; ++w) r = fmaxf(r, red[w][tid]);
        col_max[(size_t)f * nx + x0 + tid] = r;
    }
}

constexpr int kLogThreads = 256;
constexpr int kLogPerBlock = 1024;

__global__ void __launch_bounds__(kLogThreads)
    log_compress_kernel(const float* env, const float* __restrict__ col_max,
                        float* out, int npix, int nx, float dr_db, float shift) {
    __shared__ float red[kLogThreads / 64];
    const int tid = threadIdx.x;
    const int f = blockIdx.y;
    float m = 0.0f;
    for (int x = tid; x < nx; x += kLogThreads) m = fmaxf(m, col_max[(size_t)f * nx + x]);
    m = wave_max(m);
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    m = red[0];
    for (int q = 1; q < kLogThreads / 64; ++q) m = fmaxf(m, red[q]);

    const float* src = env + (size_t)f * npix;
    float* dst = out + (size_t)f * npix;
    const int p0 = blockIdx.x * kLogPerBlock;
    const int p1 = min(p0 + kLogPerBlock, npix);
    // 20 log10(e / m) = 20 log10(2) (log2 e - log2 m), log2 by the hardware
    // instruction (about 1 ulp, far inside the dB tolerance)
    constexpr float kDbPerOctave = 6.020599913279624f;
    const float lm = (m > 0.0f) ? __builtin_amdgcn_logf(m) : 0.0f;
    for (int p = p0 + tid; p < p1; p += kLogThreads) {
        const float e = src[p];
        float b = -dr_db;
        if (e > 0.0f && m > 0.0f)
            b = fminf(fmaxf(kDbPerOctave * (__builtin_amdgcn_logf(e) - lm), -dr_db), 0.0f);
        dst[p] = b + shift;
    }
}

}  // namespace

hipError_t launch_envelope(const float* bf, int F, int nz, int nx, float* env, float* col_max,
                           hipStream_t s) {
    int log_n = 0;
    while ((1 << log_n) < nz) ++log_n;
    // the widest column group whose LDS stays within 64 KB and that still
    // gives about a workgroup per CU (or more, for batches)
    auto lds_of = [&](int cpw) {
        const size_t cols = (size_t)cpw * nz;
        return (size_t)((nz / 2 > 0 ? nz / 2 : 1) + cols + (cols >> 4) + 1) * sizeof(float2);
    };
    auto groups = [&](int cpw) { return (long long)((nx + cpw - 1) / cpw) * F; };
    int cpw = 1;
    if (nz >= 4 && lds_of(4) <= 65536 && groups(4) >= WF_ENV_GROUPS4) cpw = 4;
    else if (nz >= 4 && lds_of(2) <= 65536 && groups(2) >= 256) cpw = 2;
    const dim3 grid((unsigned)((nx + cpw - 1) / cpw), (unsigned)F);
    if (cpw == 4)
        hipLaunchKernelGGL(envelope_kernel<4>, grid, dim3(kEnvThreads * 4), lds_of(4), s, bf, env,
                           col_max, nz, nx, log_n);
    else if (cpw == 2)
        hipLaunchKernelGGL(envelope_kernel<2>, grid, dim3(kEnvThreads * 2), lds_of(2), s, bf, env,
                           col_max, nz, nx, log_n);
    else
        hipLaunchKernelGGL(envelope_kernel<1>, grid, dim3(kEnvThreads * 1), lds_of(1), s, bf, env,
                           col_max, nz, nx, log_n);
    return hipGetLastError();
}

hipError_t launch_log_compress(const float* env, const float* col_max, int F, int nz, int nx,
                               float dr_db, int offset, float* out, hipStream_t s) {
    const int npix = nz * nx;
    dim3 grid((unsigned)((npix + kLogPerBlock - 1) / kLogPerBlock), (unsigned)F);
    hipLaunchKernelGGL(log_compress_kernel, grid, dim3(kLogThreads), 0, s, env, col_max, out, npix,
                       nx, dr_db, offset ? dr_db : 0.0f);
    return hipGetLastError();
}

}  // namespace wf
