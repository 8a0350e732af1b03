// Delay-and-Sum kernels for gfx950: delay geometry (K1) and the LDS-staged
// gather / linear-interpolate / accumulate (K2), for synthetic transmit
// aperture (STAI) and plane-wave (PWI) imaging (WaveFlow, Sec. II-B).
//
// K2 design (one workgroup = NT = 256, 512 or 1024 lanes = one tile of NT*PX
// pixels):
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

#include <algorithm>
#include <cstring>
#include <mutex>
#include <set>
#include <utility>

#include "das_common.h"

namespace wf {
namespace {

#ifndef WF_DAS_READS
#define WF_DAS_READS 8
#endif
// LDS reads in flight per lane per batch (channels per batch = this / PX)

// What the gather accumulates per contribution.
enum : int {
    kOpValue = 0,  // the interpolated sample (DAS)
    kOpDydc = 1,   // its slope times the scaled time of flight (d y / d c)
};

// ---------------------------------------------------------------------------
// K2: gather / interpolate / accumulate
// ---------------------------------------------------------------------------
// One staged pass: every lane adds its PX pixels' contributions of the
// kChunk channels of the LDS buffer at byte address BASE (transmit base at)
// into ACC, with the delays tq, rq, the bases bj, slot and a of the
// enclosing kernel.  Batches of LDS reads are issued before their FMAs so that
// several reads are in flight per wave.  A macro rather than a function:
// passing the delay arrays to a function, even one always inlined, cost
// about 40 VGPRs.
#define WF_GATHER_PASS(ACC, BASE, at) do {                                                      \
    const uint32_t base = (BASE);                                                               \
    constexpr int kJB = (WF_DAS_READS / PX) < 1 ? 1 : (WF_DAS_READS / PX);                      \
    _Pragma("unroll")                                                                           \
    for (int j0 = 0; j0 < kChunk; j0 += kJB) {                                                  \
        float2 ed[kJB][PX];                                                                     \
        float f1[kJB][PX];                                                                      \
        float nf[kJB];                                                                          \
        _Pragma("unroll")                                                                       \
        for (int jj = 0; jj < kJB; ++jj) {                                                      \
            const int j = j0 + jj;                                                              \
            const uint32_t off =                                                                \
                base + (uint32_t)(j * slot + ((at + bj[j]) & 7)) * 8u;                          \
            if (OP == kOpDydc) nf[jj] = (float)(at + bj[j]) + a.t0fs;                           \
            _Pragma("unroll")                                                                   \
            for (int k = 0; k < PX; ++k) {                                                      \
                const uint32_t u = tq[k] + rq[k][j];                                            \
                if (OP == kOpValue)                                                             \
                    f1[jj][k] = __uint_as_float((u & 0x7FFFFFu) | 0x3F800000u);                 \
                else /* absolute fractional sample index + t0 fs */                             \
                    f1[jj][k] = fmaf((float)u, 1.0f / kQScale, nf[jj]);                         \
                const v2f e2 = *reinterpret_cast<const __attribute__((address_space(3))) v2f*>( \
                    (uintptr_t)entry_addr(u, off));                                             \
                ed[jj][k] = make_float2(e2.x, e2.y);                                            \
            }                                                                                   \
        }                                                                                       \
        _Pragma("unroll")                                                                       \
        for (int jj = 0; jj < kJB; ++jj)                                                        \
            _Pragma("unroll")                                                                   \
            for (int k = 0; k < PX; ++k) {                                                      \
                if (OP == kOpValue)                                                             \
                    ACC[k] += fmaf(f1[jj][k], ed[jj][k].y, ed[jj][k].x);                        \
                else                                                                            \
                    ACC[k] = fmaf(ed[jj][k].y, f1[jj][k], ACC[k]);                              \
            }                                                                                   \
    }                                                                                           \
} while (0)

// FG frames per workgroup: the frames of a batch share the geometry, so a
// group reuses each chunk's receive delays and each pass's transmit delays;
// every frame keeps its own accumulation order, so a batch equals its
// frames one by one bit for bit.
// PP passes per barrier (1 or 2): two passes, of two transmits (FG = 1) or
// of two frames of a transmit (FG > 1), are staged into two of four LDS
// buffers per barrier, halving the barriers where one workgroup fills a
// CU; the accumulation order is unchanged.
// TAB = true: the launch has the plan's delay tables (rx_tab, and tx_tabq
// for the shapes of das_tx_words), fixed at compile time; TAB = false
// tests for them at run time.  Only PWI on 1024 x 2 tiles takes the first
// (10 VGPRs fewer there; elsewhere the run-time form measured faster).
template <int MODE, typename RT, int NT, int PX, int NG, int OP, int FG, int PP, bool TAB = false>
__global__ void __launch_bounds__(NT) das_kernel(const DasArgs a) {
    static_assert(PP == 1 || (PP == 2 && FG % 2 == 0) || (PP == 2 && FG == 1),
                  "frame pairs need an even frame group");
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int slot = a.slot;
    const uint32_t buf_bytes = (uint32_t)kChunk * slot * sizeof(float2);
    float2* win = reinterpret_cast<float2*>(smem);  // 2 PP buffers of kChunk windows
    const DasLds lay = das_lds(das_gather_nbuf(PP), slot, a.T);
    int4* m_tab = reinterpret_cast<int4*>(smem + lay.m_tab);
    float4* q_tab = reinterpret_cast<float4*>(smem + lay.q_tab);
    int* b_tab = reinterpret_cast<int*>(smem + lay.b_tab);
    // LDS byte offset of the window buffers (folded into scalar offsets)
    const uint32_t lds0 =
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)smem;

    const int frame0 = (int)blockIdx.y * FG;
    const int fgc = min(FG, a.F - frame0);  // frames of this group
    // (tile, split) item of this workgroup: from the work list, or numbered
    // tile-major in dispatch order (x fastest, then z)
    const int item = a.items ? a.items[blockIdx.x]
                             : (int)blockIdx.z * (int)gridDim.x + (int)blockIdx.x;
    const int tile = item / a.nsplit;
    const int split = item - tile * a.nsplit;
    const TileGeom g = tile_geom<NT, PX>(a, tile);
    // split: this workgroup sums channel chunks [cb, ce) x transmits [tb, te)
    const int ssc = split / a.nts;
    const int cb = ssc * a.split_chunks * kChunk;
    const int ce = min(a.C, cb + a.split_chunks * kChunk);
    const int tb = (split - ssc * a.nts) * a.split_tx;
    const int te = min(a.T, tb + a.split_tx);
    // receive words of a chunk from the plan's delay table: 16 per pixel
    // slot, 64 bytes (the first chunk's go out before any table is built)
    uint32_t rq[PX][kChunk];
    auto load_rq = [&](int c0) {
        const uint4* src = reinterpret_cast<const uint4*>(
            a.rx_tab + (((size_t)tile * ((a.C + kChunk - 1) / kChunk) + c0 / kChunk) * (NT * PX) +
                        tid) * kChunk);
#pragma unroll
        for (int k = 0; k < PX; ++k)
#pragma unroll
            for (int q = 0; q < kChunk / 4; ++q) {
                const uint4 v = src[(size_t)k * NT * (kChunk / 4) + q];
                rq[k][4 * q] = v.x;
                rq[k][4 * q + 1] = v.y;
                rq[k][4 * q + 2] = v.z;
                rq[k][4 * q + 3] = v.w;
            }
    };
    if constexpr (TAB) {
        if (cb < ce) load_rq(cb);
    } else {
        if (a.rx_tab && cb < ce) load_rq(cb);
    }
    // per-transmit tables and the first chunk's bases (the last kChunk
    // threads), published by the first chunk's barrier
    tx_tables<MODE, NT, PX>(a, g, m_tab, q_tab);
    if (cb < ce) chunk_tables(a, g, cb, b_tab, NT - kChunk);
    // zero pad behind every window of every buffer (never overwritten)
    {
        const int pad = slot - a.nst;
        for (int i = tid; i < 2 * PP * kChunk * pad; i += NT) {
            const int j = i / pad;
            win[j * slot + a.nst + (i - j * pad)] = make_float2(0.0f, 0.0f);
        }
    }

    PixelSet<PX> p;
    pixel_set<NT, PX>(a, g, p);
    float acc[FG][PX];
#pragma unroll
    for (int g = 0; g < FG; ++g)
#pragma unroll
        for (int k = 0; k < PX; ++k) acc[g][k] = 0.0f;
    const size_t frame_elems = (size_t)a.T * a.C * a.S;
    const RT* rf_frame = reinterpret_cast<const RT*>(a.rf) + (size_t)frame0 * frame_elems;
    const int ngroups = kChunk * a.ng;  // staged 8-sample groups per pass (<= NG * NT)

    for (int c0 = cb; c0 < ce; c0 += kChunk) {
        if (c0 != cb) {
            __syncthreads();  // previous chunk's readers of b_tab / windows are done
            chunk_tables(a, g, c0, b_tab);
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
            for (; t < te; ++t) {
                const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
                if (!(at + bmin > a.S - 2 || at + bmax + a.nst < 0)) break;
            }
            return t;
        };

        // this lane's staged groups in the chunk: group w = tid + gi NT is
        // channel j = w mod 16, samples [8 gg, 8 gg + 8) of its window.  A
        // group of a channel beyond C gets a base that puts it outside every
        // record, so the unsigned range test below covers it too.
        int gb[NG];        // b_j + 8 gg: s0 = (a_t + gb) & ~7
        uint32_t roff[NG]; // element offset of the channel's record in a transmit
        uint32_t dofs[NG]; // byte offset of the group inside an LDS buffer
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            const int w = tid + gi * NT;
            const int j = w & (kChunk - 1);
            const int gg = w >> kChunkLog2;
            const int c = c0 + j;
            gb[gi] = (c < a.C) ? b_tab[j] + 8 * gg : -0x40000000;
            roff[gi] = (uint32_t)min(c, a.C - 1) * (uint32_t)a.S;
            dofs[gi] = (uint32_t)(j * slot + 8 * gg) * (uint32_t)sizeof(float2);
        }
        const uint32_t rec_bytes = (uint32_t)a.C * (uint32_t)a.S * (uint32_t)sizeof(RT);
        constexpr int kElemLog2 = sizeof(RT) == 2 ? 1 : 2;

        // global -> registers for pass t (nothing written yet); a group
        // outside the record reads zeros through the buffer range check
        RawGroup<RT> raw[PP][NG];
        // transmit delays from the plan's table: loaded with the RF of their
        // pass (txr), copied aside when it is committed (txc); the plan
        // holds them for every shape but PWI on 1024 x 2 tiles
        constexpr bool kTxTab = FG == 1 && das_tx_words(MODE, NT, PX);
        const bool tx_tab = TAB ? kTxTab : kTxTab && a.tx_tabq != nullptr;
        uint32_t txr[PP][PX], txc[PP][PX];
        auto issue = [&](int t, int g, int h) {  // pass t of frame frame0 + g into raw[h]
            const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
            if (kTxTab && tx_tab) {
                const uint32_t* src = a.tx_tabq + ((size_t)tile * a.T + t) * (NT * PX) + tid;
#pragma unroll
                for (int k = 0; k < PX; ++k) txr[h][k] = src[k * NT];
            }
            // a ragged last group repeats its last frame (results not written)
            const size_t fo = FG == 1 ? 0 : (size_t)min(g, fgc - 1) * frame_elems;
            const __amdgpu_buffer_rsrc_t rsrc =
                rf_rsrc(rf_frame + fo + (size_t)t * a.C * a.S, rec_bytes);
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                const int w = tid + gi * NT;
                if (w < ngroups) {
                    const int s0 = (at + gb[gi]) & ~7;
                    const bool ok = (uint32_t)s0 <= (uint32_t)(a.S - 8);
                    raw[h][gi].load(rsrc, ok ? (roff[gi] + (uint32_t)s0) << kElemLog2 : kOffNone);
                }
            }
        };
        // registers -> interpolation pairs in LDS buffer `buf`.  S % 8 == 0,
        // so a group lies wholly inside or outside its record; inside, only
        // the last pair of the record (n = S - 1, no successor) is dropped.
        auto commit = [&](int t, int buf, int h) {  // raw[h] holds pass t
            const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
            if (kTxTab && tx_tab) {
#pragma unroll
                for (int k = 0; k < PX; ++k) txc[h][k] = txr[h][k];
            }
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                const int w = tid + gi * NT;
                if (w < ngroups) {
                    const int s0 = (at + gb[gi]) & ~7;
                    float v[9];
                    raw[h][gi].get(v);
#pragma unroll
                    for (int m = 0; m < 9; ++m) opaque(v[m]);
                    float4 o[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        o[i] = make_float4(fmaf(2.0f, v[2 * i], -v[2 * i + 1]),
                                           v[2 * i + 1] - v[2 * i],
                                           fmaf(2.0f, v[2 * i + 1], -v[2 * i + 2]),
                                           v[2 * i + 2] - v[2 * i + 1]);
                    if (s0 == a.S - 8) {
                        o[3].z = 0.0f;
                        o[3].w = 0.0f;
                    }
                    float4* dst = reinterpret_cast<float4*>(smem + buf * buf_bytes + dofs[gi]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) dst[i] = o[i];
                }
            }
        };

        int t = next_active(tb);
        if (t >= te) continue;  // no transmit reaches this tile through this chunk

        // software pipeline over the passes, two LDS buffers: commit a pass
        // into buffer `cur` (last read two passes ago, before the barrier of
        // the previous pass), barrier, then issue the loads of the next pass
        // so that they fly while this one is accumulated.  The first pass's
        // loads fly while the receive delays are formed.
        issue(t, 0, 0);
        int t1 = PP == 2 && FG == 1 ? next_active(t + 1) : te;  // second transmit of a pair
        if (PP == 2 && FG == 1 && t1 < te) issue(t1, 0, PP - 1);
        if (PP == 2 && FG > 1) issue(t, 1, PP - 1);  // second frame of a pair
        if constexpr (TAB) {
            if (c0 != cb) load_rq(c0);
        } else {
            if (a.rx_tab) {
                if (c0 != cb) load_rq(c0);
            } else {
                rx_delays<PX>(a, p, c0, bj, rq);
            }
        }
        int cur = 0;
        // two transmits per barrier: commit (t, t1) into buffers 2 cur and
        // 2 cur + 1 (last read in the pair before the previous barrier),
        // barrier, issue the next pair, accumulate t then t1
        if constexpr (PP == 2 && FG == 1) {
            while (t < te) {
                const int t2 = t1 < te ? next_active(t1 + 1) : te;
                const int t3 = t2 < te ? next_active(t2 + 1) : te;
                commit(t, 2 * cur, 0);
                if (t1 < te) commit(t1, 2 * cur + 1, PP - 1);
                __syncthreads();
                if (t2 < te) issue(t2, 0, 0);
                if (t3 < te) issue(t3, 0, PP - 1);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int th = h == 0 ? t : t1;
                    if (th < te) {
                        const int at = __builtin_amdgcn_readfirstlane(m_tab[th].x);
                        uint32_t tq[PX];
                        if (kTxTab && tx_tab) {
#pragma unroll
                            for (int k = 0; k < PX; ++k) tq[k] = txc[h][k];
                        } else {
                            tx_delays<MODE, PX>(a, p, m_tab[th], q_tab[th], at, tq);
                        }
                        WF_GATHER_PASS(acc[0], lds0 + (uint32_t)(2 * cur + h) * buf_bytes, at);
                    }
                }
                cur ^= 1;
                t = t2;
                t1 = t3;
            }
            continue;
        }
        // With FG > 1 the passes run (transmit t, frame g) with g fastest,
        // PP of them per barrier; the frame loop stays rolled, its
        // accumulators rotating by one frame per pass, so that only the
        // transmit delays are held across frames.
        while (t < te) {
            const int tn = next_active(t + 1);
            uint32_t tq[PX];
            if (FG > 1) {
                const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
                tx_delays<MODE, PX>(a, p, m_tab[t], q_tab[t], at, tq);
            }
#pragma unroll 1
            for (int g = 0; g < FG; g += PP) {
#pragma unroll
                for (int h = 0; h < PP; ++h) commit(t, PP * cur + h, h);
                __syncthreads();
#pragma unroll
                for (int h = 0; h < PP; ++h) {
                    if (g + PP < FG) issue(t, g + PP + h, h);
                    else if (tn < te) issue(tn, h, h);
                }
                const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
                if (kTxTab && tx_tab) {
#pragma unroll
                    for (int k = 0; k < PX; ++k) tq[k] = txc[0][k];
                } else if (FG == 1) {
                    tx_delays<MODE, PX>(a, p, m_tab[t], q_tab[t], at, tq);
                }
#pragma unroll
                for (int h = 0; h < PP; ++h) {
                    // 1024-thread workgroups have no registers to keep the sums
                    // of transmit and receive delays across frames: recompute
                    if (FG > 1 && NT == 1024)
#pragma unroll
                        for (int k = 0; k < PX; ++k) opaque_u(tq[k]);

                    WF_GATHER_PASS(acc[0], lds0 + (uint32_t)(PP * cur + h) * buf_bytes, at);
                    if (FG > 1) {
#pragma unroll
                        for (int k = 0; k < PX; ++k) {
                            const float x = acc[0][k];
#pragma unroll
                            for (int f = 0; f + 1 < FG; ++f) acc[f][k] = acc[f + 1][k];
                            acc[FG - 1][k] = x;
                        }
                    }
                }
                cur ^= 1;
            }
            t = tn;
        }
    }

    const float scale = (OP == kOpValue) ? 1.0f : a.neg_inv_c;
    float* dst = a.partial ? a.partial + (size_t)split * a.F * a.nz * a.nx : a.out;
#pragma unroll
    for (int g = 0; g < FG; ++g)
        if (g < fgc)
#pragma unroll
            for (int k = 0; k < PX; ++k)
                if (p.valid[k])
                    dst[((size_t)(frame0 + g) * a.nz + p.iz[k]) * a.nx + p.ix[k]] =
                        acc[g][k] * scale;
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

// ---------------------------------------------------------------------------
// Delay tables of a plan: the words the gathers would form, written once
// ---------------------------------------------------------------------------
// Workgroup (tile, y) of NT threads, the gather's tile shape: y < chunks
// writes the receive delays of chunk y, y == chunks (tx != null) the
// transmit delays of every transmit.  The tile geometry, pixel set, window
// bases and delay functions are the gather's own, so each word equals the
// one the gather forms for the same tile, chunk, transmit and lane.
template <int MODE, int NT, int PX>
__global__ void __launch_bounds__(NT) delay_table_kernel(const DasArgs a, uint32_t* __restrict__ rx,
                                                         uint32_t* __restrict__ tx) {
    extern __shared__ __align__(16) unsigned char smem[];
    int* b_tab = reinterpret_cast<int*>(smem);                      // 2 kChunk ints
    int4* m_tab = reinterpret_cast<int4*>(smem + 2 * kChunk * 4);  // T entries
    float4* q_tab = reinterpret_cast<float4*>(smem + 2 * kChunk * 4 + (size_t)a.T * 16);
    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    const int nch = (a.C + kChunk - 1) / kChunk;
    const TileGeom g = tile_geom<NT, PX>(a, tile);
    PixelSet<PX> p;
    pixel_set<NT, PX>(a, g, p);
    if ((int)blockIdx.y < nch) {
        const int c0 = (int)blockIdx.y * kChunk;
        chunk_tables(a, g, c0, b_tab);
        __syncthreads();
        int bj[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) bj[j] = __builtin_amdgcn_readfirstlane(b_tab[j]);
        uint32_t rq[PX][kChunk];
        rx_delays<PX>(a, p, c0, bj, rq);
        uint4* dst = reinterpret_cast<uint4*>(
            rx + (((size_t)tile * nch + blockIdx.y) * (NT * PX) + tid) * kChunk);
#pragma unroll
        for (int k = 0; k < PX; ++k)
#pragma unroll
            for (int q = 0; q < kChunk / 4; ++q)
                dst[(size_t)k * NT * (kChunk / 4) + q] =
                    make_uint4(rq[k][4 * q], rq[k][4 * q + 1], rq[k][4 * q + 2], rq[k][4 * q + 3]);
    } else if (tx) {
        tx_tables<MODE, NT, PX>(a, g, m_tab, q_tab);
        __syncthreads();
        for (int t = 0; t < a.T; ++t) {
            const int at = __builtin_amdgcn_readfirstlane(m_tab[t].x);
            uint32_t tq[PX];
            tx_delays<MODE, PX>(a, p, m_tab[t], q_tab[t], at, tq);
            uint32_t* dst = tx + ((size_t)tile * a.T + t) * (NT * PX) + tid;
#pragma unroll
            for (int k = 0; k < PX; ++k) dst[k * NT] = tq[k];
        }
    }
}

template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    return allow_dynamic_lds(reinterpret_cast<const void*>(kernel), lds);
}

template <int MODE, typename RT, int NT, int PX, int NG, int OP, int FG = 1, int PP = 1>
hipError_t launch_one(const DasArgs& a, size_t lds, hipStream_t s) {
    // the kernel carves its tables behind 2 PP window buffers: a smaller
    // allocation would leave them outside the LDS it is given
    if (a.pp != PP || !das_lds_fits(lds, das_gather_nbuf(PP), a.slot, a.T))
        return hipErrorInvalidValue;
    // PWI with delay tables on 1024 x 2 tiles launches the TAB variant; a
    // prepared plan sets the LDS limit of both, so its calls, with or
    // without the tables, make no attribute call
    constexpr bool kTab = MODE == 1 && NT == 1024 && PX == 2;
    const bool tab = kTab && a.rx_tab != nullptr;
    hipError_t e = hipSuccess;
    if (kTab && (a.prepare_only || tab))
        e = allow_lds(das_kernel<MODE, RT, NT, PX, NG, OP, FG, PP, kTab>, lds);
    if (e == hipSuccess && (a.prepare_only || !tab))
        e = allow_lds(das_kernel<MODE, RT, NT, PX, NG, OP, FG, PP>, lds);
    if (e != hipSuccess || a.prepare_only) return e;
    const unsigned groups = (unsigned)((a.F + FG - 1) / FG);
    const dim3 grid = a.items ? dim3((unsigned)a.nitems, groups, 1u)
                              : dim3((unsigned)(a.ntz * a.ntx), groups, (unsigned)a.nsplit);
    if (tab)
        hipLaunchKernelGGL((das_kernel<MODE, RT, NT, PX, NG, OP, FG, PP, kTab>), grid, dim3(NT),
                           lds, s, a);
    else
        hipLaunchKernelGGL((das_kernel<MODE, RT, NT, PX, NG, OP, FG, PP>), grid, dim3(NT), lds, s,
                           a);
    return hipGetLastError();
}

// Batches of the large-tile shapes run 4 frames per workgroup (value
// gather only: d y / d c runs one frame per workgroup).  16-bit RF on
// 1024-thread tiles runs two passes per barrier (transmits of a single
// frame, frames of a batch) where the host gave the LDS for it; FP32 RF
// holds too many staging registers for two passes.
template <int MODE, typename RT, int NT, int PX, int OP>
hipError_t launch_large(const DasArgs& a, size_t lds, hipStream_t s) {
    constexpr bool kPairs = NT == 1024 && sizeof(RT) == 2;
    // staged groups per lane: a pass stages 16 x nst / 8 groups, and
    // nst + span <= 511 keeps that below 1024
    constexpr int NG = NT == 1024 ? 1 : 2;
    if constexpr (OP == kOpValue) {
        if (a.F > 1) {
            if constexpr (kPairs)
                if (a.pp == 2) return launch_one<MODE, RT, NT, PX, NG, OP, 4, 2>(a, lds, s);
            return launch_one<MODE, RT, NT, PX, NG, OP, 4>(a, lds, s);
        }
    }
    if constexpr (kPairs)
        if (a.pp == 2) return launch_one<MODE, RT, NT, PX, NG, OP, 1, 2>(a, lds, s);
    return launch_one<MODE, RT, NT, PX, NG, OP, 1>(a, lds, s);
}

// (threads, pixels per thread): 1024 x 2 (large tiles, 16 waves), 512 x 2
// (8 waves), 512 x 1 (half the tile, 8 waves) or 256 x 1 (small tiles for
// coarse grids)
template <int MODE, typename RT, int OP>
hipError_t launch_px(int nt, int px, int groups, const DasArgs& a, size_t lds, hipStream_t s) {
    if (nt == 1024) return launch_large<MODE, RT, 1024, 2, OP>(a, lds, s);
    if (nt == 512)
        return px == 1 ? launch_large<MODE, RT, 512, 1, OP>(a, lds, s)
                       : launch_large<MODE, RT, 512, 2, OP>(a, lds, s);
    return groups <= 2 ? launch_one<MODE, RT, 256, 1, 2, OP>(a, lds, s)
                       : launch_one<MODE, RT, 256, 1, 4, OP>(a, lds, s);
}

template <int MODE, int OP>
hipError_t launch_mode(int dtype, int nt, int px, int groups, const DasArgs& a, size_t lds,
                       hipStream_t s) {
    switch (dtype) {
        case 0: return launch_px<MODE, int16_t, OP>(nt, px, groups, a, lds, s);
        case 1: return launch_px<MODE, __half, OP>(nt, px, groups, a, lds, s);
        default: return launch_px<MODE, float, OP>(nt, px, groups, a, lds, s);
    }
}

// Sum of the channel-split partial frames, in split order (deterministic).
// Splits whose item did not run wrote nothing and are left out of their
// tile's sum (where every item would have added exact zeros).
__global__ void __launch_bounds__(256)
    split_reduce_kernel(const float* __restrict__ partial, int nsplit, size_t n,
                        float* __restrict__ out, const SplitMasks m) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        uint64_t ran = ~0ull;
        if (m.masks) {
            const int p = (int)(i % (size_t)m.npix);
            const int iz = p / m.nx, ix = p - (p / m.nx) * m.nx;
            ran = m.masks[(ix >> m.txw_log2) * m.ntz + (iz >> m.tz_log2)];
        }
        // eight partial frames loaded at a time, then added in split order
        // (a frame that did not run is loaded but never added)
        float v = 0.0f;
        bool first = true;
        for (int k0 = 0; k0 < nsplit; k0 += 8) {
            float x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                x[j] = k0 + j < nsplit ? partial[(size_t)(k0 + j) * n + i] : 0.0f;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (k0 + j < nsplit && ((ran >> (k0 + j)) & 1ull)) {
                    v = first ? x[j] : v + x[j];
                    first = false;
                }
        }
        out[i] = v;
    }
}

// Plan tables through kernel arguments: one word per lane.
struct StoreWords {
    uint32_t w[kStoreWords];
};

__global__ void __launch_bounds__(1024) store_kernel(uint32_t* __restrict__ dst, StoreWords src,
                                                     int n) {
    const int i = (int)threadIdx.x;
    if (i < n) dst[i] = src.w[i];
}

}  // namespace

hipError_t allow_dynamic_lds(const void* kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    if (lds > kLdsPerCu) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::set<std::pair<const void*, int>> done;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count({kernel, dev})) return hipSuccess;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsPerCu);
    if (e == hipSuccess) done.insert({kernel, dev});
    return e;
}

hipError_t launch_store(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const uint32_t* w = static_cast<const uint32_t*>(src);
    uint32_t* d = static_cast<uint32_t*>(dst);
    for (size_t done = 0, n = bytes / 4; done < n;) {
        const int k = (int)std::min<size_t>(kStoreWords, n - done);
        StoreWords sw{};
        std::memcpy(sw.w, w + done, (size_t)k * 4);
        hipLaunchKernelGGL(store_kernel, dim3(1), dim3(1024), 0, s, d + done, sw, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        done += (size_t)k;
    }
    return hipSuccess;
}

static bool shape_ok(int nt, int px, int groups) {
    if (nt == 1024) return px == 2 && groups <= 1;
    if (nt == 512) return (px == 2 || px == 1) && groups <= 2;
    return nt == 256 && px == 1 && groups <= kMaxGroups;
}

hipError_t launch_split_reduce(const float* partial, int nsplit, size_t n, float* out,
                               const SplitMasks& m, hipStream_t s) {
    if (nsplit < 1 || nsplit > 64 || (m.masks && m.npix <= 0)) return hipErrorInvalidValue;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, partial,
                       nsplit, n, out, m);
    return hipGetLastError();
}

hipError_t launch_das(int mode, int dtype, int nt, int px, int groups, const DasArgs& a,
                      size_t lds_bytes, hipStream_t s) {
    if (!shape_ok(nt, px, groups)) return hipErrorInvalidValue;
    return mode == 1 ? launch_mode<1, kOpValue>(dtype, nt, px, groups, a, lds_bytes, s)
                     : launch_mode<0, kOpValue>(dtype, nt, px, groups, a, lds_bytes, s);
}

hipError_t launch_das_dydc(int mode, int dtype, int nt, int px, int groups, const DasArgs& a,
                           size_t lds_bytes, hipStream_t s) {
    if (!shape_ok(nt, px, groups)) return hipErrorInvalidValue;
    return mode == 1 ? launch_mode<1, kOpDydc>(dtype, nt, px, groups, a, lds_bytes, s)
                     : launch_mode<0, kOpDydc>(dtype, nt, px, groups, a, lds_bytes, s);
}

template <int MODE, int NT, int PX>
hipError_t launch_tables(const DasArgs& a, uint32_t* rx, uint32_t* tx, hipStream_t s) {
    const size_t lds = 2 * kChunk * 4 + (size_t)a.T * 32;
    hipError_t e = allow_lds(delay_table_kernel<MODE, NT, PX>, lds);
    if (e != hipSuccess) return e;
    const int nch = (a.C + kChunk - 1) / kChunk;
    const dim3 grid((unsigned)(a.ntz * a.ntx), (unsigned)(nch + (tx ? 1 : 0)));
    hipLaunchKernelGGL((delay_table_kernel<MODE, NT, PX>), grid, dim3(NT), lds, s, a, rx, tx);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_tables_shape(int nt, int px, const DasArgs& a, uint32_t* rx, uint32_t* tx,
                               hipStream_t s) {
    if (nt == 1024) return launch_tables<MODE, 1024, 2>(a, rx, tx, s);
    if (nt == 512) return px == 1 ? launch_tables<MODE, 512, 1>(a, rx, tx, s)
                                  : launch_tables<MODE, 512, 2>(a, rx, tx, s);
    return launch_tables<MODE, 256, 1>(a, rx, tx, s);
}

hipError_t launch_delay_tables(int mode, int nt, int px, const DasArgs& a, uint32_t* rx,
                               uint32_t* tx, hipStream_t s) {
    if (!shape_ok(nt, px, 1) || !rx || (long long)a.ntz * a.ntx > 0x7FFFFFFF ||
        (size_t)a.T * 32 + 2 * kChunk * 4 > kLdsPerCu)
        return hipErrorInvalidValue;
    return mode == 1 ? launch_tables_shape<1>(nt, px, a, rx, tx, s)
                     : launch_tables_shape<0>(nt, px, a, rx, tx, s);
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
