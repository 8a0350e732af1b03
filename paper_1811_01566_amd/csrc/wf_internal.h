// Internal interfaces between the C entry points (api.cpp) and the kernel
// launchers (das.hip, envelope.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/wf.h"
#include "das_layout.h"

namespace wf {
// Threads per DAS workgroup (4 wave64 waves); launch plans may also use
// 512-thread workgroups with 2 pixels per thread.
constexpr int kThreads = 256;
// Staged 8-sample RF groups per lane and transmit pass: the kernel is built
// for 2 or 4 (register staging), the launch plan picks the smaller that
// covers kChunk * groups-per-window.
constexpr int kMaxGroups = 4;
// Fractional bits of the fixed-point window-local delays (Q9.23): the
// fraction lines up with the float mantissa, the integer part (< 512)
// indexes the LDS window.
constexpr int kQBits = 23;
// Adjoint workspace mark: the (transmit, channel, tile) window adds nothing.
constexpr int kNoWindow = -0x40000000;

// Workgroups are dealt to the 8 XCDs round-robin along the dispatch order.
// For block b of n along the fastest grid dimension this returns the index
// to work on such that XCD k takes the contiguous range of indices
// [k floor(n/8) + min(k, n mod 8), ...) of length floor(n/8) + (k < n mod 8):
// neighbouring indices, which read or write the same cache lines, then
// meet in one L2 instead of all eight.  A bijection on [0, n).
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
    const int k = b & 7;
    return k * (n >> 3) + (k < (n & 7) ? k : (n & 7)) + (b >> 3);
}

// Per-transmit constants of a geometry, in samples (distances scaled by
// fs / c), split into float-float pairs on the host from double.
//   PWI:  v0 = (C0.hi, C0.lo, Az.hi, Az.lo), v1 = (Ax.hi, Ax.lo, 0, 0) with
//         TX(iz, ix) = C0 + iz Az + ix Ax; Az.hi and Ax.hi are multiples of
//         2^-15 so that small integer multiples of them are exact in float.
//   STAI: v0 = (DX.hi, DX.lo, xe, 0): DX = X(column 0) - x_e, xe the element
//         position (float, for window bounds); v1 unused.
struct TxConst {
    float4 v0, v1;
};

// Per-channel constants: (DX.hi, DX.lo, xe, 0), DX = X(column 0) - x_e, with
// DX.hi on the 2^-g grid of DasArgs::dxq (so is the STAI transmit DX).
typedef float4 ChConst;

struct DasArgs {
    const void* rf;
    float* out;
    int F, T, C, S, nz, nx;
    int tz_log2;        // tile depth TZ = 1 << tz_log2
    int ntz, ntx;       // tiles along z and x
    int xcd_order;      // 1: tile order grouped per XCD (tile count % 8 == 0)
    int ng;             // 8-sample groups staged per window (nst / 8)
    int nst;            // staged entries per window
    int slot;           // LDS entries per window (staged + zero pad), = 2 mod 16
    uint32_t txspan_q;  // clamp of window-local transmit delays (Q9.23)
    uint32_t rxspan_q;  // clamp of window-local receive delays (Q9.23)
    float2 Z0, dZ;      // depth of row 0 and row step, samples (float-float)
    float2 dX;          // column step, samples (float-float)
    float2 O;           // STAI: -t0 fs added to the transmit delay
    float fnum2;        // 2 F# (0: no apodisation)
    float x0f, dxf;     // lateral grid in samples (float) for window bases
    float dxq, inv_dxq; // 2^g and 2^-g: grid of the hi parts of lateral offsets
    float t0fs;         // t0 * fs (d y / d c: time of flight = index + t0 fs)
    float neg_inv_c;    // -1 / c (d y / d c scale)
    const TxConst* tx_tab;
    const ChConst* ch_tab;
    const float* g;     // adjoint: cotangent [F][nz][nx]
    float* grad;        // adjoint: d L / d rf [F][T][C][S]
    int nsplit;         // split: workgroups per tile (1: none) = chunk splits x nts
    int split_chunks;   // channel chunks of one split
    int nts;            // transmit splits per chunk split (split s: chunks s / nts,
                        // transmits s % nts)
    int split_tx;       // transmits of one split
    int nitems;         // workgroups along x when `items` is set
    const int* items;   // work list: item codes tile * nsplit + split, one per workgroup
                        // along x (null: the grid enumerates every item)
    float* partial;     // split partial frames [nsplit][F][nz][nx] (null: write out)
    int pp;             // transmits staged per barrier (2: four LDS buffers given)
    int ntiles;         // adjoint: ntz * ntx
    float* ws_win;      // adjoint workspace: window of (t, c, tile), nst + 1 samples
    int* ws_a0;         // adjoint workspace: first sample of that window or kNoWindow
    const float* ws_gmax;  // adjoint workspace: largest |g| of each launched frame
    int prepare_only;   // 1: set the launch attributes of the kernel this call would
                        // launch (its dynamic LDS limit) and launch nothing
    // Delay tables of a plan (null: the gathers form the delays themselves;
    // both give the same words): window-local Q9.23 receive delays, masked
    // and clamped as the gather uses them, [tile][chunk][pixel slot][16],
    // and transmit delays [tile][T][pixel slot]; pixel slot = k NT +
    // thread for pixel k of a thread.
    const uint32_t* rx_tab;
    const uint32_t* tx_tabq;
};

struct DelayArgs {
    float* tx_hi;
    float* tx_lo;
    float* rx_hi;
    float* rx_lo;
    int T, C, nz, nx;
    float2 Z0, dZ, dX, O;
    const TxConst* tx_tab;
    const ChConst* ch_tab;
};

// FIR taps, zero-padded symmetrically to the kernel's tap count (15, 31, 63).
struct FirTaps {
    float h[64];
};

// LDS of one gfx950 CU, the most one workgroup may take.
constexpr size_t kLdsPerCu = 163840;

// Raises the dynamic-LDS limit of `kernel` (a __global__ function's host
// address) to kLdsPerCu on the current device when `lds` exceeds the
// default 64 KB, once per kernel and device: later launches, including
// those recorded into a graph, make no attribute call.
hipError_t allow_dynamic_lds(const void* kernel, size_t lds);

// Launchers; return the hipError_t of the launch.
hipError_t launch_das(int mode, int dtype, int nt, int px, int groups, const DasArgs& a,
                      size_t lds_bytes, hipStream_t s);
hipError_t launch_das_dydc(int mode, int dtype, int nt, int px, int groups, const DasArgs& a,
                           size_t lds_bytes, hipStream_t s);
// Which splits of a tile ran, for the split reduce: masks[txi * ntz + tzi]
// has bit k set when split k of tile (tzi, txi) wrote its partial frame
// (masks = null: every split ran).
struct SplitMasks {
    const uint64_t* masks;
    int npix, nx, ntz, tz_log2, txw_log2;
};
hipError_t launch_split_reduce(const float* partial, int nsplit, size_t n, float* out,
                               const SplitMasks& m, hipStream_t s);
// nbuf: window sets of the adjoint (1 or 2; lds_bytes must hold them)
hipError_t launch_das_adjoint(int mode, int nt, int px, int nbuf, const DasArgs& a,
                              size_t lds_bytes, hipStream_t s);
hipError_t launch_absmax(const float* g, size_t n, float* out, hipStream_t s);
hipError_t launch_adjoint_reduce(const float* ws_win, const int* ws_a0, float* grad, int rows,
                                 int ntiles, int ne, int S, hipStream_t s);
hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s);
// Copies `bytes` (a multiple of 4) of host memory to device memory `dst`
// through kernel arguments, in pieces of kStoreWords words: stream-ordered,
// capturable into a graph, and the host buffer may be freed on return.
constexpr int kStoreWords = 960;
hipError_t launch_store(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_dot(const float* a, const float* b, size_t n, float* out, hipStream_t s);
hipError_t launch_delays(int mode, const DelayArgs& a, hipStream_t s);
// Writes the delay tables of a plan (DasArgs::rx_tab / tx_tabq layout) for
// the tile shape (nt, px): rx always, tx when tx != null.
hipError_t launch_delay_tables(int mode, int nt, int px, const DasArgs& a, uint32_t* rx,
                               uint32_t* tx, hipStream_t s);
hipError_t launch_envelope(const float* bf, int F, int nz, int nx, float* env, float* col_max,
                           hipStream_t s);
hipError_t launch_log_compress(const float* env, const float* col_max, int F, int nz, int nx,
                               float dr_db, int offset, float* out, hipStream_t s);
hipError_t launch_fir(int dtype, const void* rf, long long n_rec, int S, int kp,
                      const FirTaps& taps, float* out, hipStream_t s);
// DAS into caller buffers with the geometry tables, and the split's partial
// frames where they fit, in a scratch block of scratch_bytes of device
// memory that get_scratch returns once the arguments are validated (and
// that stays valid for the call's work on `stream`); mode 0 STAI, 1 PWI.
// Allocates and frees no device memory.
wf_status das_scratch(int32_t mode, const void* rf, const wf_probe* probe, const wf_acq* acq,
                      const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                      const wf_grid* grid, float* out, wf_status (*get_scratch)(void**),
                      size_t scratch_bytes, hipStream_t stream);
// Sets the calling thread's error message for a failed HIP call.
wf_status report_hip(hipError_t e, const char* what);

hipError_t launch_moments(const float* env, int F, int nz, int nx, int wz, int wx, int sz,
                          int sx, int mz, int mx, float* out, hipStream_t s);

}  // namespace wf
