// Envelope (K3) and log compression / clip (K4) for gfx950 (WaveFlow,
// Fig. 2: Analytic Signal -> Absolute Value -> Dynamic Adjustment; Hilbert
// transform by FFT, Sec. II-B; dB clip, Sec. III).
//
// K3: one workgroup per pair of image columns.  Each column is an nz-point
// complex FFT in LDS: a decimation-in-frequency forward pass (natural order
// in, bit-reversed out), the one-sided multiplier applied at bit-reversed
// positions, and a decimation-in-time inverse pass (bit-reversed in,
// natural out), so no permutation pass is needed.  Twiddles come from the
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

// cols: columns per workgroup (1 or 2); log_n: log2(nz)
__global__ void __launch_bounds__(kEnvThreads)
    envelope_kernel(const float* bf, float* env,
                    float* __restrict__ col_max, int nz, int nx, int log_n, int cols) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = nz;
    const int half = n >> 1;
    float2* tw = reinterpret_cast<float2*>(smem);              // [n/2]
    float2* buf = reinterpret_cast<float2*>(smem) + (half > 0 ? half : 1);  // [cols][n]
    __shared__ float red[kEnvThreads / 64][2];

    const int tid = threadIdx.x;
    const int f = blockIdx.y;
    const int xb = blockIdx.x * cols;
    const float* src = bf + (size_t)f * nz * nx;
    float* dst = env + (size_t)f * nz * nx;

    // W^k = exp(-2 pi i k / n)
    for (int k = tid; k < half; k += kEnvThreads) {
        float s, c;
        sincospif(-2.0f * (float)k / (float)n, &s, &c);
        tw[k] = make_float2(c, s);
    }
    for (int i = tid; i < cols * n; i += kEnvThreads) {
        const int c = i % cols;
        const int z = i / cols;
        const int x = xb + c;
        const float v = (x < nx) ? src[(size_t)z * nx + x] : 0.0f;
        buf[c * n + z] = make_float2(v, 0.0f);
    }
    __syncthreads();

    const int nbf = cols * half;  // butterflies per stage
    // forward DIF: span h = n/2 .. 1
    for (int h = half; h >= 1; h >>= 1) {
        const int tstride = half / h;
        for (int b = tid; b < nbf; b += kEnvThreads) {
            const int c = b / half;
            const int bb = b - c * half;
            const int pos = bb & (h - 1);
            const int i = ((bb - pos) << 1) + pos;
            float2* col = buf + c * n;
            const float2 x0 = col[i], x1 = col[i + h];
            const float2 w = tw[pos * tstride];
            const float dr = x0.x - x1.x, di = x0.y - x1.y;
            col[i] = make_float2(x0.x + x1.x, x0.y + x1.y);
            col[i + h] = make_float2(fmaf(dr, w.x, -di * w.y), fmaf(dr, w.y, di * w.x));
        }
        __syncthreads();
    }
    // one-sided spectrum: position p holds bin k = bitrev(p)
    for (int i = tid; i < cols * n; i += kEnvThreads) {
        const int c = i / n;
        const int p = i - c * n;
        const int k = (int)(__brev((unsigned)p) >> (32 - log_n));
        const float g = (k == 0 || k == half) ? 1.0f : (k < half ? 2.0f : 0.0f);
        float2 v = buf[c * n + p];
        buf[c * n + p] = make_float2(v.x * g, v.y * g);
    }
    __syncthreads();
    // inverse DIT with conjugate twiddles: span h = 1 .. n/2
    for (int h = 1; h <= half; h <<= 1) {
        const int tstride = half / h;
        for (int b = tid; b < nbf; b += kEnvThreads) {
            const int c = b / half;
            const int bb = b - c * half;
            const int pos = bb & (h - 1);
            const int i = ((bb - pos) << 1) + pos;
            float2* col = buf + c * n;
            const float2 w = tw[pos * tstride];
            const float2 x1 = col[i + h];
            // t = conj(w) * x1
            const float tr = fmaf(x1.x, w.x, x1.y * w.y);
            const float ti = fmaf(x1.y, w.x, -x1.x * w.y);
            const float2 x0 = col[i];
            col[i] = make_float2(x0.x + tr, x0.y + ti);
            col[i + h] = make_float2(x0.x - tr, x0.y - ti);
        }
        __syncthreads();
    }
    // modulus, store, column maxima
    const float inv_n = 1.0f / (float)n;
    float m0 = 0.0f, m1 = 0.0f;
    for (int i = tid; i < cols * n; i += kEnvThreads) {
        const int c = i % cols;
        const int z = i / cols;
        const int x = xb + c;
        const float2 v = buf[c * n + z];
        const float e = sqrtf(fmaf(v.x, v.x, v.y * v.y)) * inv_n;
        if (x < nx) dst[(size_t)z * nx + x] = e;
        if (c == 0) m0 = fmaxf(m0, e); else m1 = fmaxf(m1, e);
    }
    const int lane = tid & 63, wv = tid >> 6;
    m0 = wave_max(m0);
    m1 = wave_max(m1);
    if (lane == 0) {
        red[wv][0] = m0;
        red[wv][1] = m1;
    }
    __syncthreads();
    if (tid < cols && xb + tid < nx) {
        float r = red[0][tid];
        for (int q = 1; q < kEnvThreads / 64; ++q) r = fmaxf(r, red[q][tid]);
        col_max[(size_t)f * nx + xb + tid] = r;
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
    const int cols = (nz <= 2048) ? 2 : 1;
    const size_t lds = (size_t)((nz / 2 > 0 ? nz / 2 : 1) + cols * nz) * sizeof(float2);
    dim3 grid((unsigned)((nx + cols - 1) / cols), (unsigned)F);
    hipLaunchKernelGGL(envelope_kernel, grid, dim3(kEnvThreads), lds, s, bf, env, col_max, nz,
                       nx, log_n, cols);
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
