// LDS layout of the DAS workgroups (forward gather, d y / d c gather and
// adjoint scatter).  Plain constexpr arithmetic with no HIP dependency, so
// the host code that sizes a launch, the kernels that carve their dynamic
// LDS, and the CPU tests all compute the same offsets.
//
// A workgroup's dynamic LDS holds, in this order:
//   nbuf arrays of kChunk windows, `slot` entries of 8 bytes each
//     (forward and d y / d c: 2 per pass staged per barrier, as double
//      buffers; adjoint: G and H arrays per window set);
//   m_tab  int4[T]    per-transmit window base and PWI tile constants;
//   q_tab  float4[T]  per-transmit delay constants;
//   b_tab  int[2 kChunk]  channel bases and aperture flags of a chunk.
// A launch whose dynamic LDS is smaller than `total` would put the tables
// past the allocation, where reads return zero and writes are dropped.
#pragma once

#include <stddef.h>

namespace wf {

// Channels staged per pass of the DAS kernels: their one-way receive delays
// stay in registers while every transmit streams through LDS.
constexpr int kChunk = 16;
constexpr int kChunkLog2 = 4;

struct DasLds {
    size_t m_tab, q_tab, b_tab, total;  // byte offsets; total = bytes needed
};

constexpr DasLds das_lds(int nbuf, int slot, int T) {
    const size_t win = (size_t)nbuf * kChunk * (size_t)slot * 8;
    return DasLds{win, win + (size_t)T * 16, win + (size_t)T * 32,
                  win + (size_t)T * 32 + (size_t)kChunk * 2 * 4};
}

// Window arrays of a gather staging pp passes per barrier (two buffers each).
constexpr int das_gather_nbuf(int pp) { return 2 * pp; }
// Window arrays of an adjoint with nsets window sets (G and H each).
constexpr int das_adjoint_nbuf(int nsets) { return 2 * nsets; }

// Whether a plan with delay tables holds transmit words for the gathers of
// this tile shape: every shape but PWI (mode 1) on 1024 x 2 tiles.  That
// gather sits at its 128-register limit, and loading the words cost it 6 %
// where forming its (linear) transmit delays costs about 0.3 VALU per
// contribution (measured on the 1024 x 512 grid).
constexpr bool das_tx_words(int mode, int nt, int px) {
    return !(mode == 1 && nt == 1024 && px == 2);
}

// True when `lds` bytes hold the layout of nbuf arrays for this slot and T.
constexpr bool das_lds_fits(size_t lds, int nbuf, int slot, int T) {
    return lds >= das_lds(nbuf, slot, T).total;
}

}  // namespace wf
