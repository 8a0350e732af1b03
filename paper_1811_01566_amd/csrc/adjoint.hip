// Adjoint of Delay-and-Sum (K5) and small helpers (fill, dot) for gfx950.
//
// The paper's reason for putting the beamformer in a dataflow graph is to
// train networks through it (Sec. I; Sec. IV).  DAS is linear in the RF for a
// fixed geometry: y(p) = sum_{t,j} w (1 - a) r[n] + a r[n+1].  Its adjoint
// scatters a cotangent g(p) back to the samples: (1 - a) w g to r[n] and
// a w g to r[n+1], for pairs with 0 <= n <= S-2.
//
// Two stages, no global atomics:
//  0. K5m: the largest |g| of the frame (one workgroup, fixed order).
//  1. K5 reuses the forward's tiles, window bases and window-local Q9.23
//     delays (das_common.h), so a contribution lands in exactly the pair the
//     forward read.  Per transmit pass it accumulates, for every window entry
//     (= pair n), G[n] = sum w g and H[n] = sum a w g in 64-bit fixed point
//     with LDS integer atomics: g is rounded once per pixel to 24 bits of the
//     frame's largest |g| (g24), G adds g24 2^23 and H adds g24 times the
//     23-bit fraction of the delay - the very fraction the forward
//     interpolates with - as one 24 x 24-bit product.  (On gfx950 an LDS
//     float atomic costs about 40 times an LDS 64-bit integer atomic.)
//     Sample A0 + e of the window then receives (G[e] - H[e]) + H[e-1] (each
//     only for valid pairs), converted back to float.  The window of every
//     (transmit, channel, tile) goes to a workspace with its first sample A0
//     (or a no-window mark when the pass or the channel chunk reaches
//     nothing).
//  2. K5r sums, for every RF sample, the windows of all tiles that cover it,
//     in tile order: one lane per sample, with a scalar test that skips the
//     tiles whose window misses the workgroup's 256 samples.  Every sample of
//     the gradient is written exactly once.
// Integer sums do not depend on their order and stage 2 has a fixed order,
// so the gradient is bitwise reproducible.  Rounding g to 24 bits of the
// frame maximum adds at most 2^-24 max|g| per pixel.
#pragma clang fp contract(off)

#include "das_common.h"

namespace wf {
namespace {

// A 64-bit integer of magnitude below 2^53 as a float: the magnitude's
// 32-bit halves are converted (the high half exactly) and summed, so the
// result is within about one ulp; full-rate FP32 instructions only.
__device__ __forceinline__ float i64_to_float(long long v) {
    const unsigned long long m = v < 0 ? 0ull - (unsigned long long)v : (unsigned long long)v;
    const float f = fmaf((float)(unsigned)(m >> 32), 4294967296.0f, (float)(unsigned)m);
    return v < 0 ? -f : f;
}

// Window sums of the adjoint: 64-bit fixed-point G and H (scale 2^23 g24),
// in two separate arrays of 8-byte entries (all G windows, then all H
// windows).  The lanes of a wave walk down one column, hitting entries about
// 1.6 apart; with 8-byte entries one wave's atomics then span half the LDS
// rows that interleaved 16-byte (G, H) entries would, and the bank
// conflicts, which bound this kernel, fall with them.
typedef unsigned long long u64;

// NB window sets: with two, the scatter of pass t + 1 goes to the other set
// while pass t is flushed, so a pass needs one barrier instead of two.  A
// wave flushes and clears its windows of pass t before it scatters pass
// t + 1, and every wave has done that before the barrier that follows the
// scatter of t + 1, so the set of pass t is clear again when pass t + 2
// scatters into it.
template <int MODE, int NT, int PX, int NB>
__global__ void __launch_bounds__(NT) das_adjoint_kernel(const DasArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int slot = a.slot;
    const int nwin = kChunk * slot;  // entries of one array of windows
    // set b: G of window j at gw[b * 2 nwin + j * slot + e], H nwin further
    u64* gw = reinterpret_cast<u64*>(smem);
    const DasLds lay = das_lds(das_adjoint_nbuf(NB), slot, a.T);
    int4* m_tab = reinterpret_cast<int4*>(smem + lay.m_tab);
    float4* q_tab = reinterpret_cast<float4*>(smem + lay.q_tab);
    int* b_tab = reinterpret_cast<int*>(smem + lay.b_tab);
    const uint32_t lds0 =
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)smem;

    const int frame = blockIdx.y;
    // (tile, split) item: from the work list or numbered tile-major; an item
    // covers channel chunks [cb, ce) x transmits [tb, te) of its tile, and
    // its windows are its own (no partial sums)
    const int item = a.items ? a.items[blockIdx.x]
                             : (int)blockIdx.z * (int)gridDim.x + (int)blockIdx.x;
    const int tile = item / a.nsplit;
    const int split = item - tile * a.nsplit;
    const int ssc = split / a.nts;
    const int cb = ssc * a.split_chunks * kChunk;
    const int ce = min(a.C, cb + a.split_chunks * kChunk);
    const int tb = (split - ssc * a.nts) * a.split_tx;
    const int te = min(a.T, tb + a.split_tx);
    const TileGeom g = tile_geom<NT, PX>(a, tile);
    tx_tables<MODE, NT, PX>(a, g, m_tab, q_tab);
    uint4* zw = reinterpret_cast<uint4*>(smem);  // all arrays, 16 bytes a store
    for (int i = tid; i < NB * nwin; i += NT) zw[i] = make_uint4(0u, 0u, 0u, 0u);

    PixelSet<PX> p;
    pixel_set<NT, PX, false>(a, g, p);
    // g rounded to 24 bits of the frame maximum: |g24| <= 2^23 - 1
    const float gmax = a.ws_gmax[frame];
    const float to24 = gmax > 0.0f ? 8388607.0f / gmax : 0.0f;
    int g24[PX];
    unsigned long long gG[PX];  // G increment: g24 * 2^23
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const float gv = p.valid[k] ? a.g[((size_t)frame * a.nz + p.iz[k]) * a.nx + p.ix[k]] : 0.0f;
        // |value| <= 2^23 - 1 (the product is rounded down to float at
        // most to 2^23 - 1 + ulp/2 < 2^23), so the 24-bit sign extension
        // keeps it and tells the compiler it is a 24-bit operand
        g24[k] = ((int)rintf(fminf(fmaxf(gv * to24, -8388607.0f), 8388607.0f)) << 8) >> 8;
        gG[k] = (unsigned long long)((long long)g24[k] << kQBits);
    }
    // fixed point -> float: 2^-23 (fraction) * gmax / (2^23 - 1) (g24),
    // applied as an exact 2^-46 and gmax 2^23 / (2^23 - 1), so nothing
    // underflows or overflows that the gradient itself does not
    const float gscale = gmax * (8388608.0f / 8388607.0f);
    const int ne = a.nst + 1;  // samples a window can touch
    // workspace slots of (transmit t, channel c) for this tile
    auto slot_of = [&](int t, int c) { return ((size_t)t * a.C + c) * a.ntiles + tile; };
    int cur = 0;  // window set of the next scattering pass

    for (int c0 = cb; c0 < ce; c0 += kChunk) {
        __syncthreads();
        chunk_tables(a, g, c0, b_tab);
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
        if (!any_act) {  // nothing of this chunk reaches the tile
            for (int w = tid; w < (te - tb) * kChunk; w += NT) {
                const int t = tb + (w >> kChunkLog2), c = c0 + (w & (kChunk - 1));
                if (c < a.C) a.ws_a0[slot_of(t, c)] = kNoWindow;
            }
            continue;
        }

        uint32_t rq[PX][kChunk];
        rx_delays<PX>(a, p, c0, bj, rq);

        for (int t = tb; t < te; ++t) {
            const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
            if (at + bmin > a.S - 2 || at + bmax + a.nst < 0) {  // nothing lands
                if (tid < kChunk && c0 + tid < a.C) a.ws_a0[slot_of(t, c0 + tid)] = kNoWindow;
                continue;
            }
            uint32_t tq[PX];
            tx_delays<MODE, PX>(a, p, m_tab[t], q_tab[t], at, tq);

            // ---- scatter into the LDS windows (integer atomics) -------------
            const uint32_t set0 = lds0 + (uint32_t)(cur * 2 * nwin) * 8u;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                const uint32_t off = set0 + (uint32_t)(j * slot + ((at + bj[j]) & 7)) * 8u;
#pragma unroll
                for (int k = 0; k < PX; ++k) {
                    const uint32_t u = tq[k] + rq[k][j];
                    const int f23 = (int)(u & 0x7FFFFFu);
                    // g24 * f23, both 24-bit signed: one 24 x 24-bit product
                    const unsigned long long h =
                        (unsigned long long)((long long)g24[k] * (long long)f23);
                    u64* e = reinterpret_cast<u64*>(smem + (entry_addr(u, off) - lds0));
                    atomicAdd(e, gG[k]);
                    atomicAdd(e + nwin, h);
                }
            }
            __syncthreads();

            // ---- flush: sample A0 + e of every window to the workspace ------
            // (a wave per channel: window base, workspace slot and A0 are
            // wave-uniform; the lanes store consecutive workspace words).
            // The wave then clears the windows it owns: its LDS reads are
            // done in order before its stores, and no other wave touches
            // them until the barrier, so no barrier is needed in between.
            for (int j = tid >> 6; j < kChunk; j += NT >> 6) {
                const int c = c0 + j;
                u64* gj = gw + (size_t)cur * 2 * nwin + j * slot;
                u64* hj = gj + nwin;
                if (c < a.C) {
                    const int A0 = __builtin_amdgcn_readfirstlane((at + b_tab[j]) & ~7);
                    const size_t sl = slot_of(t, c);
                    float* dst = a.ws_win + sl * ne;
                    for (int e = tid & 63; e < ne; e += 64) {
                        const int s = A0 + e;
                        long long v = 0;
                        if (e < a.nst && s >= 0 && s <= a.S - 2)
                            v += (long long)gj[e] - (long long)hj[e];
                        if (e >= 1 && s - 1 >= 0 && s - 1 <= a.S - 2) v += (long long)hj[e - 1];
                        dst[e] = ldexpf(i64_to_float(v), -46) * gscale;
                    }
                    if ((tid & 63) == 0) a.ws_a0[sl] = A0;
                }
                // slot is even and j slot 8 bytes a multiple of 16: 16-byte stores
                for (int e = 2 * (tid & 63); e < slot; e += 128) {
                    *reinterpret_cast<uint4*>(gj + e) = make_uint4(0u, 0u, 0u, 0u);
                    *reinterpret_cast<uint4*>(hj + e) = make_uint4(0u, 0u, 0u, 0u);
                }
            }
            // one set: its windows must be zero before the next pass scatters
            if (NB == 1) __syncthreads();
            cur ^= NB - 1;
        }
    }
}

// Stage 0: largest |g| of the frame.  Non-negative floats order like their
// bit patterns, so workgroup maxima combine with an integer atomic max into
// a word cleared by fill_kernel (no memset: the call may be captured).
constexpr int kMaxThreads = 256;

__global__ void __launch_bounds__(kMaxThreads)
    absmax_kernel(const float* __restrict__ g, size_t n, unsigned* __restrict__ out) {
    __shared__ float red[kMaxThreads];
    float m = 0.0f;
    for (size_t i = (size_t)blockIdx.x * kMaxThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kMaxThreads)
        m = fmaxf(m, fabsf(g[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = kMaxThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

// Stage 2: lane = RF sample s of row (t, c); the sum over tiles in tile
// order of the window entries that land on s.  The tiles are taken 256 at a
// time: each lane tests one tile's window against the workgroup's 256
// samples, the overlapping tiles are compacted in tile order into an LDS
// list (wave ballots and a prefix over the 4 waves), and the list is summed
// in batches of 8 whose loads fly together.
constexpr int kRedThreads = 256;
constexpr int kRedBatch = 8;

__global__ void __launch_bounds__(kRedThreads)
    adjoint_reduce_kernel(const float* __restrict__ ws_win, const int* __restrict__ ws_a0,
                          float* __restrict__ grad, int ntiles, int ne, int S) {
    __shared__ int list_k[kRedThreads + kRedBatch];   // overlapping tiles, in order
    __shared__ int list_a0[kRedThreads + kRedBatch];  // their window starts
    __shared__ int wave_cnt[kRedThreads / 64];
    const size_t row = blockIdx.x;
    const int s_lo = blockIdx.y * kRedThreads;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int s = s_lo + tid;
    const int* a0r = ws_a0 + row * ntiles;
    const float* wr = ws_win + row * ntiles * (size_t)ne;
    float acc = 0.0f;
    for (int k0 = 0; k0 < ntiles; k0 += kRedThreads) {
        // ---- compact the tiles of [k0, k0 + 256) whose window meets the block
        const int k = k0 + tid;
        const int A0 = k < ntiles ? a0r[k] : kNoWindow;
        const bool hit = (A0 != kNoWindow) && (A0 + ne > s_lo) && (A0 < s_lo + kRedThreads);
        const unsigned long long m = __ballot(hit);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        __syncthreads();  // the previous round's list readers are done
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int base = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kRedThreads / 64; ++w) {
            base += w < wave ? wave_cnt[w] : 0;
            total += wave_cnt[w];
        }
        if (hit) {
            list_k[base + before] = k;
            list_a0[base + before] = A0;
        }
        if (tid < kRedBatch) {  // pad the last batch with entries that add 0
            list_k[total + tid] = 0;
            list_a0[total + tid] = kNoWindow;
        }
        __syncthreads();
        // ---- sum the list in order ------------------------------------
        for (int b = 0; b < total; b += kRedBatch) {
            float v[kRedBatch];
#pragma unroll
            for (int i = 0; i < kRedBatch; ++i) {
                const int a0 = list_a0[b + i];
                const int e = s - a0;
                v[i] = (a0 != kNoWindow && e >= 0 && e < ne)
                           ? wr[(size_t)list_k[b + i] * ne + e] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < kRedBatch; ++i) acc += v[i];
        }
    }
    if (s < S) grad[row * S + s] = acc;
}

__global__ void __launch_bounds__(256) fill_kernel(float* p, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One workgroup, compensated (Kahan) per-thread sums, fixed-order tree:
// deterministic.
constexpr int kDotThreads = 1024;

__global__ void __launch_bounds__(kDotThreads) dot_kernel(const float* a, const float* b,
                                                         size_t n, float* out) {
    __shared__ float red[kDotThreads];
    float s = 0.0f, comp = 0.0f;
    for (size_t i = threadIdx.x; i < n; i += kDotThreads) {
        const float y = fmaf(a[i], b[i], -comp);
        const float t = s + y;
        comp = (t - s) - y;
        s = t;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kDotThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    return allow_dynamic_lds(reinterpret_cast<const void*>(kernel), lds);
}

template <int MODE, int NT, int PX, int NB>
hipError_t launch_adj(const DasArgs& a, size_t lds, hipStream_t s) {
    if (!das_lds_fits(lds, das_adjoint_nbuf(NB), a.slot, a.T)) return hipErrorInvalidValue;
    hipError_t e = allow_lds(das_adjoint_kernel<MODE, NT, PX, NB>, lds);
    if (e != hipSuccess || a.prepare_only) return e;
    const dim3 grid = a.items ? dim3((unsigned)a.nitems, (unsigned)a.F, 1u)
                              : dim3((unsigned)(a.ntz * a.ntx), (unsigned)a.F, (unsigned)a.nsplit);
    hipLaunchKernelGGL((das_adjoint_kernel<MODE, NT, PX, NB>), grid, dim3(NT), lds, s, a);
    return hipGetLastError();
}

template <int MODE, int NB>
hipError_t launch_adj_nb(int nt, int px, const DasArgs& a, size_t lds, hipStream_t s) {
    if (nt == 1024)
        return px == 1 ? launch_adj<MODE, 1024, 1, NB>(a, lds, s)
                       : launch_adj<MODE, 1024, 2, NB>(a, lds, s);
    if (nt == 512)
        return px == 1 ? launch_adj<MODE, 512, 1, NB>(a, lds, s)
                       : launch_adj<MODE, 512, 2, NB>(a, lds, s);
    return launch_adj<MODE, 256, 1, NB>(a, lds, s);
}

template <int MODE>
hipError_t launch_adj_shape(int nt, int px, int nbuf, const DasArgs& a, size_t lds,
                            hipStream_t s) {
    return nbuf == 2 ? launch_adj_nb<MODE, 2>(nt, px, a, lds, s)
                     : launch_adj_nb<MODE, 1>(nt, px, a, lds, s);
}

}  // namespace

hipError_t launch_das_adjoint(int mode, int nt, int px, int nbuf, const DasArgs& a,
                              size_t lds_bytes, hipStream_t s) {
    // the gather's shapes (1024 x 2, 512 x 2, 512 x 1, 256 x 1) and 1024 x 1
    if (!((nt == 1024 && (px == 2 || px == 1)) || (nt == 512 && (px == 2 || px == 1)) ||
          (nt == 256 && px == 1)))
        return hipErrorInvalidValue;
    return mode == 1 ? launch_adj_shape<1>(nt, px, nbuf, a, lds_bytes, s)
                     : launch_adj_shape<0>(nt, px, nbuf, a, lds_bytes, s);
}

hipError_t launch_absmax(const float* g, size_t n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, s, out, (size_t)1, 0.0f);
    size_t blocks = (n + kMaxThreads * 8 - 1) / (kMaxThreads * 8);
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)blocks), dim3(kMaxThreads), 0, s, g, n,
                       reinterpret_cast<unsigned*>(out));
    return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const float* ws_win, const int* ws_a0, float* grad, int rows,
                                 int ntiles, int ne, int S, hipStream_t s) {
    const dim3 grid((unsigned)rows, (unsigned)((S + kRedThreads - 1) / kRedThreads));
    hipLaunchKernelGGL(adjoint_reduce_kernel, grid, dim3(kRedThreads), 0, s, ws_win, ws_a0, grad,
                       ntiles, ne, S);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, size_t n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(kDotThreads), 0, s, a, b, n, out);
    return hipGetLastError();
}

}  // namespace wf
