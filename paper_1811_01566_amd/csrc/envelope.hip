// Envelope (K3) and log compression / clip (K4) for gfx950 (WaveFlow,
// Fig. 2: Analytic Signal -> Absolute Value -> Dynamic Adjustment; Hilbert
// transform by FFT, Sec. II-B; dB clip, Sec. III).
//
// K3: one workgroup per image column.  The column is an nz-point complex
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

// One workgroup per column (and frame); log_n = log2(nz).  Radix-2
// stages are fused in pairs (two spans per pass through LDS, 4 points per
// lane in registers), halving the barriers; an odd stage count leaves one
// single stage (the first forward one, the last inverse one).
__global__ void __launch_bounds__(kEnvThreads)
    envelope_kernel(const float* bf, float* env, float* __restrict__ col_max, int nz, int nx,
                    int log_n) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = nz;
    const int half = n >> 1;
    float2* tw = reinterpret_cast<float2*>(smem);                 // [n/2]
    float2* col = tw + (half > 0 ? half : 1);                     // [n]
    __shared__ float red[kEnvThreads / 64];

    const int tid = threadIdx.x;
    const int x = blockIdx.x;
    const int f = blockIdx.y;
    const float* src = bf + (size_t)f * nz * nx + x;
    float* dst = env + (size_t)f * nz * nx + x;

    // W^k = exp(-2 pi i k / n)
    for (int k = tid; k < half; k += kEnvThreads) {
        float sn, cs;
        sincospif(-2.0f * (float)k / (float)n, &sn, &cs);
        tw[k] = make_float2(cs, sn);
    }
    for (int z = tid; z < n; z += kEnvThreads) col[z] = make_float2(src[(size_t)z * nx], 0.0f);
    __syncthreads();

    // ---- forward DIF, spans n/2 .. 1 ------------------------------------
    int h = half;
    if (log_n & 1) {  // single stage of span n/2
        for (int b = tid; b < half; b += kEnvThreads) {
            const float2 x0 = col[b], x1 = col[b + h];
            col[b] = cadd(x0, x1);
            col[b + h] = cmul(csub(x0, x1), tw[b]);
        }
        __syncthreads();
        h >>= 1;
    }
    for (; h >= 2; h >>= 2) {  // spans h and h/2 in one pass
        const int q = h >> 1, ts = half / h;
        for (int g = tid; g < (n >> 2); g += kEnvThreads) {
            const int pos = g & (q - 1);
            const int i0 = ((g - pos) << 2) + pos;  // block of 2h
            float2 a0 = col[i0], a1 = col[i0 + q], a2 = col[i0 + h], a3 = col[i0 + h + q];
            const float2 b0 = cadd(a0, a2), b2 = cmul(csub(a0, a2), tw[pos * ts]);
            const float2 b1 = cadd(a1, a3), b3 = cmul(csub(a1, a3), tw[(pos + q) * ts]);
            const float2 w2 = tw[pos * 2 * ts];
            col[i0] = cadd(b0, b1);
            col[i0 + q] = cmul(csub(b0, b1), w2);
            col[i0 + h] = cadd(b2, b3);
            col[i0 + h + q] = cmul(csub(b2, b3), w2);
        }
        __syncthreads();
    }
    // one-sided spectrum: position p holds bin k = bitrev(p)
    for (int p = tid; p < n; p += kEnvThreads) {
        const int k = log_n > 0 ? (int)(__brev((unsigned)p) >> (32 - log_n)) : 0;
        const float gk = (k == 0 || k == half) ? 1.0f : (k < half ? 2.0f : 0.0f);
        const float2 v = col[p];
        col[p] = make_float2(v.x * gk, v.y * gk);
    }
    __syncthreads();
    // ---- inverse DIT with conjugate twiddles, spans 1 .. n/2 -------------
    h = 1;
    const int pairs = log_n >> 1;
    for (int st = 0; st < pairs; ++st, h <<= 2) {  // spans h and 2h in one pass
        const int ts = half / h, ts2 = ts >> 1;
        for (int g = tid; g < (n >> 2); g += kEnvThreads) {
            const int pos = g & (h - 1);
            const int i0 = ((g - pos) << 2) + pos;  // block of 4h
            const float2 a0 = col[i0], a1 = col[i0 + h], a2 = col[i0 + 2 * h],
                         a3 = col[i0 + 3 * h];
            const float2 w1 = tw[pos * ts];
            const float2 t1 = cmul_conj(a1, w1), t3 = cmul_conj(a3, w1);
            const float2 b0 = cadd(a0, t1), b1 = csub(a0, t1);
            const float2 b2 = cadd(a2, t3), b3 = csub(a2, t3);
            const float2 u2 = cmul_conj(b2, tw[pos * ts2]);
            const float2 u3 = cmul_conj(b3, tw[(pos + h) * ts2]);
            col[i0] = cadd(b0, u2);
            col[i0 + 2 * h] = csub(b0, u2);
            col[i0 + h] = cadd(b1, u3);
            col[i0 + 3 * h] = csub(b1, u3);
        }
        __syncthreads();
    }
    if (log_n & 1) {  // last single stage, span n/2
        for (int b = tid; b < half; b += kEnvThreads) {
            const float2 t = cmul_conj(col[b + half], tw[b]);
            const float2 x0 = col[b];
            col[b] = cadd(x0, t);
            col[b + half] = csub(x0, t);
        }
        __syncthreads();
    }
    // modulus, store, column maximum
    const float inv_n = 1.0f / (float)n;
    float m = 0.0f;
    for (int z = tid; z < n; z += kEnvThreads) {
        const float2 v = col[z];
        const float e = sqrtf(fmaf(v.x, v.x, v.y * v.y)) * inv_n;
        dst[(size_t)z * nx] = e;
        m = fmaxf(m, e);
    }
    m = wave_max(m);
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        float r = red[0];
        for (int w = 1; w < kEnvThreads / 64; ++w) r = fmaxf(r, red[w]);
        col_max[(size_t)f * nx + x] = r;
    }
}

constexpr int kLogThreads = 256;
constexpr int kLogPerBlock = 4096;

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
    const float lm = (m > 0.0f) ? log10f(m) : 0.0f;
    for (int p = p0 + tid; p < p1; p += kLogThreads) {
        const float e = src[p];
        float b = -dr_db;
        if (e > 0.0f && m > 0.0f) b = fminf(fmaxf(20.0f * (log10f(e) - lm), -dr_db), 0.0f);
        dst[p] = b + shift;
    }
}

}  // namespace

hipError_t launch_envelope(const float* bf, int F, int nz, int nx, float* env, float* col_max,
                           hipStream_t s) {
    int log_n = 0;
    while ((1 << log_n) < nz) ++log_n;
    const size_t lds = (size_t)((nz / 2 > 0 ? nz / 2 : 1) + nz) * sizeof(float2);
    dim3 grid((unsigned)nx, (unsigned)F);
    hipLaunchKernelGGL(envelope_kernel, grid, dim3(kEnvThreads), lds, s, bf, env, col_max, nz, nx,
                       log_n);
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
