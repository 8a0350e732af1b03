// FIR pre-filter along samples (K0) and windowed envelope moments (K7) for
// gfx950.
//
// K0 (pre-processing FIR, Sec. II-B list of ops).  Every record of S samples
// (one channel of one transmit of one frame) is filtered on its own:
//   y[s] = sum_k h[k] r[s + D - k],  D = (K - 1) / 2,  r = 0 outside [0, S),
// so an odd-length linear-phase filter adds no delay.  A workgroup filters
// one segment of up to 2048 outputs of one record, staging the segment plus
// a 32-sample halo on each side in LDS as FP32 (int16 and FP16 convert
// exactly), with zeros wherever the halo leaves the record - so no lane ever
// tests a record edge.  A lane owns 8 consecutive outputs (S % 8 == 0),
// reads its K + 7 inputs from LDS into registers and runs 8 K FMAs with the
// taps in scalar registers; lanes past the record's end exit (whole waves
// when S < 2048).  A resident grid walks the segments and loads the next
// segment into registers while filtering the current one.  The staged
// samples are stored with one pad word after
// every 8, so lane i's window starts at word 9 i: 9 is odd, so neighbouring
// lanes hit different LDS banks (a stride of 8 words would put every 4th
// lane on the same bank).  The tap count is padded to KP in {15, 31, 63} with zeros
// placed symmetrically, which adds exact zeros to the sums.  Per output: K
// FMAs, 2-4 bytes read and 4 written; at K = 31 the vector-FMA and HBM
// times are about equal.
//
// K7 (qUS moment maps, Fig. 3: slice -> E[X], E[X^2], E[X^3]).  Window
// wz x wx at origins (i sz, j sx), whole windows only.  One workgroup per
// (window row i, frame, block of 64 window columns): the lanes first sum
// env, env^2, env^3 down the wz rows of every input column the block uses
// (reads coalesced along x, 8 rows in flight), keep the column sums in LDS,
// then each lane adds wx column sums for its window and divides by wz wx.
// Fixed summation order: deterministic.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "wf_internal.h"

namespace wf {
namespace {

constexpr int kFirThreads = 256;
constexpr int kFirPerLane = 8;
constexpr int kFirBlock = kFirThreads * kFirPerLane;  // outputs per workgroup
constexpr int kFirHalo = 32;                           // >= D for KP <= 63

template <typename RT>
__device__ __forceinline__ void load8(const RT* p, float (&v)[8]);

template <>
__device__ __forceinline__ void load8<int16_t>(const int16_t* p, float (&v)[8]) {
    const int4 q = *reinterpret_cast<const int4*>(p);
    const int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[2 * i] = (float)(int16_t)(w[i] & 0xFFFF);
        v[2 * i + 1] = (float)(w[i] >> 16);
    }
}

template <>
__device__ __forceinline__ void load8<__half>(const __half* p, float (&v)[8]) {
    const int4 q = *reinterpret_cast<const int4*>(p);
    const int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[2 * i] = __half2float(__ushort_as_half((unsigned short)(w[i] & 0xFFFF)));
        v[2 * i + 1] = __half2float(__ushort_as_half((unsigned short)((unsigned)w[i] >> 16)));
    }
}

template <>
__device__ __forceinline__ void load8<float>(const float* p, float (&v)[8]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float4 b = *reinterpret_cast<const float4*>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Raw staging words of one lane: chunks c = lane and lane + 256 of the
// 264 chunks of 8 samples (only lanes < 8 have a second chunk).
template <typename RT>
struct FirRaw {
    float v[2][8];
};

template <typename RT, int KP>
__global__ void __launch_bounds__(kFirThreads)
    fir_kernel(const RT* __restrict__ rf, float* __restrict__ out, int S, int nseg,
               long long nblocks, const FirTaps taps) {
    constexpr int D = (KP - 1) / 2;
    constexpr int kStage = kFirBlock + 2 * kFirHalo;       // staged samples
    constexpr int kChunks = kStage / 8;                    // 264
    constexpr int kFirst = kFirHalo - D;                   // lane's first sample - 8 lane
    constexpr int kWin = KP + kFirPerLane - 1;             // inputs a lane needs
    // sample e of the staged range lives at word e + e / 8
    __shared__ float xs[kStage + kStage / 8];
    const int tid = threadIdx.x;

    // global -> registers for segment b: [sb - halo, sb + block + halo) of the
    // record, zeros outside it
    auto fetch = [&](long long b, FirRaw<RT>& raw) {
        const long long rec = b / nseg;
        const int sb = (int)(b - rec * nseg) * kFirBlock;
        const RT* row = rf + rec * S;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = tid + h * kFirThreads;
            const int q = sb - kFirHalo + 8 * c;  // multiple of 8, as is S
            if (c < kChunks && q >= 0 && q < S) {
                load8<RT>(row + q, raw.v[h]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) raw.v[h][i] = 0.0f;
            }
        }
    };

    FirRaw<RT> raw;
    long long b = blockIdx.x;
    if (b < nblocks) fetch(b, raw);
    for (; b < nblocks; b += gridDim.x) {
        __syncthreads();  // the previous segment's readers are done
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = tid + h * kFirThreads;
            if (c < kChunks) {
                float* d = xs + 9 * c;
#pragma unroll
                for (int i = 0; i < 8; ++i) d[i] = raw.v[h][i];
            }
        }
        __syncthreads();
        // the next segment's loads fly while this one is filtered
        if (b + gridDim.x < nblocks) fetch(b + gridDim.x, raw);

        const long long rec = b / nseg;
        const int sb = (int)(b - rec * nseg) * kFirBlock;
        const int s0 = sb + kFirPerLane * tid;
        if (s0 >= S) continue;
        // input m (record position s0 - D + m) is staged sample e = 8 lane +
        // kFirst + m, at word e + e / 8
        float xw[kWin];
        const float* src = xs + 9 * tid;
#pragma unroll
        for (int m = 0; m < kWin; ++m) xw[m] = src[(kFirst + m) + (kFirst + m) / 8];
        float acc[kFirPerLane];
#pragma unroll
        for (int i = 0; i < kFirPerLane; ++i) acc[i] = 0.0f;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const float h = taps.h[k];
#pragma unroll
            for (int i = 0; i < kFirPerLane; ++i)
                acc[i] = fmaf(h, xw[i + KP - 1 - k], acc[i]);
        }
        float4* dst = reinterpret_cast<float4*>(out + rec * S + s0);
        dst[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        dst[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    }
}

// Workgroups of `kernel` that fit on the device at once (CUs x occupancy),
// queried once per kernel and device.
template <typename K>
long long resident_blocks(K kernel) {
    static long long cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
    if (cached[dev] == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kFirThreads, 0) !=
                hipSuccess ||
            cus <= 0 || per_cu <= 0)
            return 1024;
        cached[dev] = (long long)cus * per_cu;
    }
    return cached[dev];
}

template <typename RT, int KP>
hipError_t launch_fir_kp(const RT* rf, int S, int nseg, long long nblocks, const FirTaps& taps,
                         float* out, hipStream_t s) {
    // a resident grid walks the segments, prefetching the next one
    const long long resident = resident_blocks(fir_kernel<RT, KP>);
    const dim3 grid((unsigned)(nblocks < resident ? nblocks : resident));
    hipLaunchKernelGGL((fir_kernel<RT, KP>), grid, dim3(kFirThreads), 0, s, rf, out, S, nseg,
                       nblocks, taps);
    return hipGetLastError();
}

template <typename RT>
hipError_t launch_fir_t(const RT* rf, long long n_rec, int S, int kp, const FirTaps& taps,
                        float* out, hipStream_t s) {
    const int nseg = (S + kFirBlock - 1) / kFirBlock;
    const long long nblocks = n_rec * nseg;
    if (kp == 15) return launch_fir_kp<RT, 15>(rf, S, nseg, nblocks, taps, out, s);
    if (kp == 31) return launch_fir_kp<RT, 31>(rf, S, nseg, nblocks, taps, out, s);
    return launch_fir_kp<RT, 63>(rf, S, nseg, nblocks, taps, out, s);
}

constexpr int kMomThreads = 128;
constexpr int kMomCols = 64;  // output columns per workgroup

__global__ void __launch_bounds__(kMomThreads)
    moments_kernel(const float* __restrict__ env, float* __restrict__ out, int nz, int nx,
                   int wz, int wx, int sz, int sx, int mz, int mx) {
    extern __shared__ __align__(16) unsigned char smem[];
    // window row; each XCD takes a contiguous block of them, so the wz / sz
    // window rows reading each envelope row meet in one L2
    const int i = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int f = blockIdx.y;
    const int j0 = blockIdx.z * kMomCols;  // first output column of this workgroup
    const int jn = min(kMomCols, mx - j0);
    const int xb = j0 * sx;                 // first input column used
    const int ncol = (jn - 1) * sx + wx;    // input columns used
    float* v1 = reinterpret_cast<float*>(smem);
    float* v2 = v1 + ncol;
    float* v3 = v2 + ncol;
    const float* e = env + ((size_t)f * nz + (size_t)i * sz) * nx + xb;
    for (int x = threadIdx.x; x < ncol; x += kMomThreads) {
        float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll 8
        for (int z = 0; z < wz; ++z) {
            const float v = e[(size_t)z * nx + x];
            const float q = v * v;
            s1 += v;
            s2 += q;
            s3 += q * v;
        }
        v1[x] = s1;
        v2[x] = s2;
        v3[x] = s3;
    }
    __syncthreads();
    const float cnt = (float)wz * (float)wx;
    const size_t plane = (size_t)mz * mx;
    float* o = out + (size_t)f * 3 * plane + (size_t)i * mx + j0;
    for (int j = threadIdx.x; j < jn; j += kMomThreads) {
        float a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
        const int x0 = j * sx;
        for (int x = x0; x < x0 + wx; ++x) {
            a1 += v1[x];
            a2 += v2[x];
            a3 += v3[x];
        }
        o[j] = a1 / cnt;
        o[plane + j] = a2 / cnt;
        o[2 * plane + j] = a3 / cnt;
    }
}

}  // namespace

hipError_t launch_fir(int dtype, const void* rf, long long n_rec, int S, int kp,
                      const FirTaps& taps, float* out, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_fir_t(static_cast<const int16_t*>(rf), n_rec, S, kp, taps, out, s);
        case 1: return launch_fir_t(static_cast<const __half*>(rf), n_rec, S, kp, taps, out, s);
        default: return launch_fir_t(static_cast<const float*>(rf), n_rec, S, kp, taps, out, s);
    }
}

hipError_t launch_moments(const float* env, int F, int nz, int nx, int wz, int wx, int sz,
                          int sx, int mz, int mx, float* out, hipStream_t s) {
    const int blocks = (mx + kMomCols - 1) / kMomCols;
    const size_t lds = 3 * sizeof(float) * (size_t)(min(kMomCols, mx) - 1) * sx +
                       3 * sizeof(float) * (size_t)wx;
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(moments_kernel), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(moments_kernel, dim3((unsigned)mz, (unsigned)F, (unsigned)blocks),
                       dim3(kMomThreads), lds, s, env, out, nz, nx, wz, wx, sz, sx, mz, mx);
    return hipGetLastError();
}

}  // namespace wf
