// C entry points of libwf: argument validation, per-geometry constant
// tables, tile selection and stream-ordered kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/wf.h"
#include "wf_internal.h"

namespace {

thread_local std::string g_err;

wf_status fail(wf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

wf_status ok() {
    g_err.clear();
    return WF_OK;
}

wf_status hip_fail(hipError_t e, const char* what) {
    return fail(WF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite(double v) { return std::isfinite(v); }

float2 split(double v) {
    const float h = (float)v;
    return make_float2(h, (float)(v - (double)h));
}

constexpr int kMaxTx = 1024;
constexpr int kMaxCh = 1024;
constexpr int kMaxElem = 4096;
constexpr double kMaxAngle = 80.0 * M_PI / 180.0;

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------

wf_status check_geometry(int mode, const wf_probe* probe, const wf_acq* acq,
                         const int32_t* tx_elem, const double* angles, int32_t tref,
                         const wf_grid* grid, bool need_rf) {
    if (!probe) return fail(WF_ERR_INVALID_ARG, "probe is NULL");
    if (!acq) return fail(WF_ERR_INVALID_ARG, "acq is NULL");
    if (!grid) return fail(WF_ERR_INVALID_ARG, "grid is NULL");
    if (probe->n_elem < 1 || probe->n_elem > kMaxElem)
        return fail(WF_ERR_INVALID_ARG, "probe->n_elem=%d outside [1, %d]", probe->n_elem,
                    kMaxElem);
    if (probe->elem_x) {
        for (int e = 0; e < probe->n_elem; ++e)
            if (!finite(probe->elem_x[e]))
                return fail(WF_ERR_INVALID_ARG, "probe->elem_x[%d] is not finite", e);
    } else if (!finite(probe->pitch) || probe->pitch <= 0.0) {
        return fail(WF_ERR_INVALID_ARG, "probe->pitch must be > 0 when elem_x is NULL");
    }
    if (acq->n_tx < 1 || acq->n_tx > kMaxTx)
        return fail(WF_ERR_INVALID_ARG, "acq->n_tx=%d outside [1, %d]", acq->n_tx, kMaxTx);
    if (acq->n_ch < 1 || acq->n_ch > kMaxCh)
        return fail(WF_ERR_INVALID_ARG, "acq->n_ch=%d outside [1, %d]", acq->n_ch, kMaxCh);
    if (need_rf) {
        if (acq->n_frames < 1) return fail(WF_ERR_INVALID_ARG, "acq->n_frames must be >= 1");
        if (acq->n_frames > 65535)
            return fail(WF_ERR_INVALID_ARG, "acq->n_frames=%d above 65535", acq->n_frames);
        if (acq->n_s < 16 || acq->n_s > 32768)
            return fail(WF_ERR_INVALID_ARG, "acq->n_s=%d outside [16, 32768]", acq->n_s);
        if (acq->n_s % 8 != 0)
            return fail(WF_ERR_UNSUPPORTED, "acq->n_s=%d is not a multiple of 8", acq->n_s);
        if (acq->dtype < WF_RF_I16 || acq->dtype > WF_RF_F32)
            return fail(WF_ERR_INVALID_ARG, "acq->dtype=%d is not a wf_rf_dtype", acq->dtype);
    }
    if (!finite(acq->c) || acq->c <= 0.0) return fail(WF_ERR_INVALID_ARG, "acq->c must be > 0");
    if (!finite(acq->fs) || acq->fs <= 0.0)
        return fail(WF_ERR_INVALID_ARG, "acq->fs must be > 0");
    if (!finite(acq->t0)) return fail(WF_ERR_INVALID_ARG, "acq->t0 is not finite");
    if (!finite(acq->f_number) || acq->f_number < 0.0)
        return fail(WF_ERR_INVALID_ARG, "acq->f_number must be >= 0");
    if (acq->rx_elem)
        for (int j = 0; j < acq->n_ch; ++j)
            if (acq->rx_elem[j] < 0 || acq->rx_elem[j] >= probe->n_elem)
                return fail(WF_ERR_INVALID_ARG, "acq->rx_elem[%d]=%d outside [0, %d)", j,
                            acq->rx_elem[j], probe->n_elem);
    if (!acq->rx_elem && acq->n_ch > probe->n_elem)
        return fail(WF_ERR_INVALID_ARG, "n_ch=%d > n_elem=%d with the identity channel map",
                    acq->n_ch, probe->n_elem);
    if (grid->nz < 1 || grid->nx < 1 || grid->nz > 65536 || grid->nx > 65536)
        return fail(WF_ERR_INVALID_ARG, "grid %d x %d outside [1, 65536]^2", grid->nz, grid->nx);
    if ((long long)grid->nz * grid->nx > (1LL << 28))
        return fail(WF_ERR_INVALID_ARG, "grid has more than 2^28 pixels");
    if (!finite(grid->z0) || !finite(grid->dz) || !finite(grid->x0) || !finite(grid->dx))
        return fail(WF_ERR_INVALID_ARG, "grid origin/step not finite");
    if (mode == 0) {
        if (tx_elem)
            for (int t = 0; t < acq->n_tx; ++t)
                if (tx_elem[t] < 0 || tx_elem[t] >= probe->n_elem)
                    return fail(WF_ERR_INVALID_ARG, "tx_elem[%d]=%d outside [0, %d)", t,
                                tx_elem[t], probe->n_elem);
        if (!tx_elem && acq->n_tx > probe->n_elem)
            return fail(WF_ERR_INVALID_ARG, "n_tx=%d > n_elem=%d with tx_elem NULL", acq->n_tx,
                        probe->n_elem);
    } else {
        if (!angles) return fail(WF_ERR_INVALID_ARG, "angles_rad is NULL");
        for (int t = 0; t < acq->n_tx; ++t)
            if (!finite(angles[t]) || std::fabs(angles[t]) >= kMaxAngle)
                return fail(WF_ERR_INVALID_ARG, "angles_rad[%d]=%g outside (-80, 80) deg", t,
                            angles[t]);
        if (tref != WF_PWI_TREF_FIRST && tref != WF_PWI_TREF_CENTRE)
            return fail(WF_ERR_INVALID_ARG, "tref=%d is not a wf_pwi_tref", tref);
    }
    // delays must stay in a sane sample range for the fixed-point windows
    const double k = acq->fs / acq->c;
    const double zmax = std::max(std::fabs(grid->z0), std::fabs(grid->z0 + (grid->nz - 1) * grid->dz));
    const double xspan = std::fabs(grid->x0) + std::fabs((grid->nx - 1) * grid->dx);
    if ((zmax + xspan) * k > 1.0e6 || std::fabs(acq->t0 * acq->fs) > 1.0e6)
        return fail(WF_ERR_UNSUPPORTED, "grid or t0 reaches beyond 1e6 samples");
    return WF_OK;
}

// ---------------------------------------------------------------------------
// per-geometry constant tables (device), cached
// ---------------------------------------------------------------------------

struct Geometry {
    std::vector<wf::TxConst> tx;
    std::vector<wf::ChConst> ch;
    float2 Z0, dZ, dX, O;
    float x0f, dxf, fnum2;
    float dxq;        // 2^g: grid of the hi parts of lateral offsets (samples)
    double dzs, dxs;  // |dz|, |dx| in samples
};

void build_geometry(int mode, const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                    const double* angles, int32_t tref, const wf_grid* grid, Geometry* g) {
    const double k = acq->fs / acq->c;  // samples per metre
    std::vector<double> ex(probe->n_elem);
    for (int e = 0; e < probe->n_elem; ++e)
        ex[e] = probe->elem_x ? probe->elem_x[e]
                              : (e - (probe->n_elem - 1) / 2.0) * probe->pitch;
    g->Z0 = split(grid->z0 * k);
    g->dZ = split(grid->dz * k);
    g->dX = split(grid->dx * k);
    g->O = split(-acq->t0 * acq->fs);
    g->x0f = (float)(grid->x0 * k);
    g->dxf = (float)(grid->dx * k);
    g->fnum2 = (float)(2.0 * acq->f_number);
    g->dzs = std::fabs(grid->dz * k);
    g->dxs = std::fabs(grid->dx * k);
    // Lateral offsets x - x_e (samples) are split as hi + lo with hi on a
    // grid 2^-g so coarse that every offset of a grid column from an element
    // in use, and every column offset from column 0, stays below 2^(23 - g):
    // then channel and pixel hi parts add exactly on the device.
    double xmax = std::fabs((grid->nx - 1) * grid->dx * k);
    auto widen = [&](double xe) {
        xmax = std::max(xmax, std::fabs((grid->x0 - xe) * k));
        xmax = std::max(xmax, std::fabs((grid->x0 + (grid->nx - 1) * grid->dx - xe) * k));
    };
    for (int j = 0; j < acq->n_ch; ++j) widen(ex[acq->rx_elem ? acq->rx_elem[j] : j]);
    if (mode == 0)
        for (int t = 0; t < acq->n_tx; ++t) widen(ex[tx_elem ? tx_elem[t] : t]);
    const int gexp = std::max(0, std::min(20, 23 - (int)std::ceil(std::log2(xmax + 2.0))));
    const double gq = std::ldexp(1.0, gexp);
    g->dxq = (float)gq;
    auto split_grid = [&](double v) {
        const double h = std::nearbyint(v * gq) / gq;
        return make_float2((float)h, (float)(v - h));
    };
    g->ch.resize(acq->n_ch);
    for (int j = 0; j < acq->n_ch; ++j) {
        const double xe = ex[acq->rx_elem ? acq->rx_elem[j] : j];
        const float2 d = split_grid((grid->x0 - xe) * k);
        g->ch[j] = make_float4(d.x, d.y, (float)(xe * k), 0.0f);
    }
    g->tx.resize(acq->n_tx);
    for (int t = 0; t < acq->n_tx; ++t) {
        wf::TxConst tc{};
        if (mode == 0) {
            const double xe = ex[tx_elem ? tx_elem[t] : t];
            const float2 d = split_grid((grid->x0 - xe) * k);
            tc.v0 = make_float4(d.x, d.y, (float)(xe * k), 0.0f);
            tc.v1 = make_float4(0, 0, 0, 0);
        } else {
            const double th = angles[t];
            const double st = std::sin(th), ct = std::cos(th);
            double o = 0.0;
            if (tref == WF_PWI_TREF_FIRST) {
                double mn = ex[0] * st;
                for (double x : ex) mn = std::min(mn, x * st);
                o = -mn;
            }
            const double c0 = (grid->z0 * ct + grid->x0 * st + o) * k - acq->t0 * acq->fs;
            const double az = grid->dz * ct * k, ax = grid->dx * st * k;
            const double azh = std::nearbyint(az * 32768.0) / 32768.0;
            const double axh = std::nearbyint(ax * 32768.0) / 32768.0;
            const float2 c0s = split(c0);
            tc.v0 = make_float4(c0s.x, c0s.y, (float)azh, (float)(az - azh));
            tc.v1 = make_float4((float)axh, (float)(ax - axh), 0.0f, 0.0f);
        }
        g->tx[t] = tc;
    }
}

void key_add(std::string& k, const void* p, size_t n) { k.append((const char*)p, n); }

// ---------------------------------------------------------------------------
// DAS tile selection
// ---------------------------------------------------------------------------

struct TilePlan {
    int threads = 0, px = 0, tz_log2 = 0, span = 0, nst = 0, slot = 0;
    size_t lds = 0;
    int ntz = 0, ntx = 0;
};

// LDS of a gather workgroup staging one pass per barrier (two window
// buffers, per-transmit and chunk tables)
size_t das_lds_bytes(int slot, int T) { return wf::das_lds(wf::das_gather_nbuf(1), slot, T).total; }

// LDS of one CU on gfx950 (and the most a single workgroup may take).
constexpr size_t kLdsHard = 163840;

#ifndef WF_DAS_ALLOW_1024
#define WF_DAS_ALLOW_1024 1
#endif
#ifndef WF_DAS_XCD_ORDER
#define WF_DAS_XCD_ORDER 0
#endif
#ifndef WF_DAS_TWO_PASS
#define WF_DAS_TWO_PASS 1
#endif
#ifndef WF_ADJ_TWO_SETS
#define WF_ADJ_TWO_SETS 1
#endif

// Tile plans a geometry can run: each (threads, pixels per thread) shape
// and tile height whose window fits the gather's staging limits and whose
// LDS leaves `min_waves` resident waves per CU.  Shapes: 1024 x 2 and 512 x 2
// (two pixels a thread, 16 or 8 waves), 512 x 1 and 256 x 1 (a half and a
// quarter of the 512 x 2 tile, smaller windows).  256 x 4 and 1024 x 1
// cover the tiles of 512 x 2 with fewer waves or one pixel a thread, and
// their gathers measured slower on every geometry (the adjoint still runs
// 1024 x 1: plan_adjoint).
std::vector<TilePlan> tile_candidates(const Geometry& g, const wf_acq* acq, const wf_grid* grid,
                                      int min_waves) {
    const int shapes[4][2] = {{1024, 2}, {512, 2}, {512, 1}, {256, 1}};
    std::vector<TilePlan> out;
    for (const auto& sh : shapes) {
        const int nt = sh[0], px = sh[1];
        if (nt == 1024 && !WF_DAS_ALLOW_1024) continue;
        for (int tzl = 6; tzl >= 3; --tzl) {
            const int tz = 1 << tzl;
            const int txw = (nt * px) >> tzl;
            const int ez = std::min(tz, grid->nz), ex = std::min(txw, grid->nx);
            const double d = std::hypot((ez - 1) * g.dzs, (ex - 1) * g.dxs);
            const int span = (int)std::ceil(d) + 3;
            const int nst = ((2 * span + 8) + 7) & ~7;
            // windows of consecutive channels start 16 bytes apart
            // modulo 128 (slot = 2 mod 16), so the 8 lanes that stage the
            // same group of 8 consecutive channels store to distinct banks
            const int slot = (((nst + span + 8) - 2 + 15) & ~15) + 2;
            if (nst + span > 511) continue;
            const int max_groups = nt == 1024 ? 1 : nt == 512 ? 2 : wf::kMaxGroups;
            if (wf::kChunk * (nst / 8) > max_groups * nt) continue;
            const size_t lds = das_lds_bytes(slot, acq->n_tx);
            if (lds > kLdsHard || (int)(kLdsHard / lds) * (nt / 64) < min_waves) continue;
            TilePlan tp;
            tp.threads = nt;
            tp.px = px;
            tp.tz_log2 = tzl;
            tp.span = span;
            tp.nst = nst;
            tp.slot = slot;
            tp.lds = lds;
            tp.ntz = (grid->nz + tz - 1) / tz;
            tp.ntx = (grid->nx + txw - 1) / txw;
            out.push_back(tp);
        }
    }
    return out;
}

// LDS bytes of a gather workgroup staging pp passes per barrier.
size_t das_gather_lds(const TilePlan& tp, int T, int pp) {
    return wf::das_lds(wf::das_gather_nbuf(pp), tp.slot, T).total;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

size_t rf_bytes_of(const wf_acq* acq) {
    const size_t esz = acq->dtype == WF_RF_F32 ? 4 : 2;
    return (size_t)acq->n_frames * acq->n_tx * acq->n_ch * acq->n_s * esz;
}

wf_status check_rf(const void* rf, const wf_acq* acq) {
    if (!rf) return fail(WF_ERR_INVALID_ARG, "rf is NULL");
    if (((uintptr_t)rf & 15) != 0) return fail(WF_ERR_UNSUPPORTED, "rf is not 16-byte aligned");
    return WF_OK;
}

int groups_of(const wf::DasArgs& a, const TilePlan& tp) {
    return (wf::kChunk * a.ng + tp.threads - 1) / tp.threads;
}

// forward DAS (op 0) or forward-mode d y / d c (op 1)
// Channel split for grids with few tiles: each tile's channel chunks are
// shared by nsplit workgroups that write partial frames, summed afterwards
// in split order.  The split depends on the tile count only (not on the
// number of frames), so a batch gives the same bits as its frames one by
// one.  The target is the number of workgroups the GPU holds at once
// (256 CUs x the workgroups of this shape one CU holds).
// ---------------------------------------------------------------------------
// Work split of the gather: (tile, chunk range, transmit range) items
// ---------------------------------------------------------------------------

struct SplitPlan {
    int nsplit = 1;  // items per tile = chunk splits x nts
    int chunks = 1;  // channel chunks of one split
    int nts = 1;     // transmit splits
    int txs = 1;     // transmits of one split
    // work list: the items that run any pass (code tile * nsplit + split),
    // heaviest first; empty for grids left to the plain grid order
    std::vector<int> order;
};

// Transmit passes the gather runs for each (tile, channel chunk, transmit),
// by the kernel's own tests evaluated in float on the host: a chunk runs if
// the receive aperture of one of its channels reaches the tile, a pass if
// the transmit's windows reach into the record.  A window base may differ
// from the device's by one sample at a rounding tie; the map only steers
// the split, never what is computed.  pre[(tile * nch + chunk) * (T + 1) + t]
// counts the passes of transmits [0, t).
void pass_map(int mode, const Geometry& g, const wf_acq* acq, const wf_grid* grid,
              const TilePlan& tp, std::vector<uint16_t>* pre) {
    const int T = acq->n_tx, C = acq->n_ch, S = acq->n_s;
    const int nch = (C + wf::kChunk - 1) / wf::kChunk;
    const int tiles = tp.ntz * tp.ntx;
    const int TZ = 1 << tp.tz_log2;
    const int TXW = (tp.threads * tp.px) >> tp.tz_log2;
    pre->assign((size_t)tiles * nch * (T + 1), 0);
    std::vector<int> at(T), b(C);
    std::vector<char> act(C);
    auto rmd = [](float xe, float xlo, float xhi, float zlo, float zhi) {
        const float dx = std::max(0.0f, std::max(xlo - xe, xe - xhi));
        const float dz = std::min(std::max(0.0f, zlo), zhi);
        return std::sqrt(dx * dx + dz * dz);
    };
    for (int tile = 0; tile < tiles; ++tile) {
        const int iz0 = (tile % tp.ntz) * TZ, ix0 = (tile / tp.ntz) * TXW;
        const int iz1 = std::min(iz0 + TZ, grid->nz) - 1;
        const int ix1 = std::min(ix0 + TXW, grid->nx) - 1;
        const float za = g.Z0.x + (float)iz0 * g.dZ.x, zb = g.Z0.x + (float)iz1 * g.dZ.x;
        const float xa = g.x0f + (float)ix0 * g.dxf, xb = g.x0f + (float)ix1 * g.dxf;
        const float zlo = std::min(za, zb), zhi = std::max(za, zb);
        const float xlo = std::min(xa, xb), xhi = std::max(xa, xb);
        for (int t = 0; t < T; ++t) {
            const wf::TxConst& tc = g.tx[t];
            if (mode == 1) {
                const float c0 = tc.v0.x, az = tc.v0.z, ax = tc.v1.x;
                const float m00 = c0 + (float)iz0 * az + (float)ix0 * ax;
                const float m10 = c0 + (float)iz1 * az + (float)ix0 * ax;
                const float m01 = c0 + (float)iz0 * az + (float)ix1 * ax;
                const float m11 = c0 + (float)iz1 * az + (float)ix1 * ax;
                at[t] = (int)std::floor(std::min(std::min(m00, m10), std::min(m01, m11))) - 1;
            } else {
                at[t] = (int)std::floor(rmd(tc.v0.z, xlo, xhi, zlo, zhi) + g.O.x) - 1;
            }
        }
        for (int c = 0; c < C; ++c) {
            const float xe = g.ch[c].z;
            b[c] = (int)std::floor(rmd(xe, xlo, xhi, zlo, zhi)) - 1;
            const float dxm = std::max(0.0f, std::max(xlo - xe, xe - xhi));
            act[c] = !(g.fnum2 > 0.0f) || (g.fnum2 * dxm <= zhi + 1.0f);
        }
        for (int k = 0; k < nch; ++k) {
            int bmin = INT_MAX, bmax = INT_MIN;
            bool any = false;
            for (int j = 0; j < wf::kChunk; ++j) {
                const int c = k * wf::kChunk + j;
                const int bj = c < C ? b[c] : 0;  // the kernel's table holds 0 there
                bmin = std::min(bmin, bj);
                bmax = std::max(bmax, bj);
                any = any || (c < C && act[c]);
            }
            if (!any) continue;
            uint16_t* r = pre->data() + ((size_t)tile * nch + k) * (T + 1);
            for (int t = 0; t < T; ++t)
                r[t + 1] = (uint16_t)(r[t] + !(at[t] + bmin > S - 2 || at[t] + bmax + tp.nst < 0));
        }
    }
}

// Estimated passes of every item of a plan (an item that runs nothing: 0):
// its passes, the receive delays of each chunk it runs (about 5.5 passes)
// and a fixed ~2 us (launch, tables, pixel set, scans over transmits that
// do not reach the tile), which is many passes of a small tile.
std::vector<double> item_costs(const SplitPlan& sp, const std::vector<uint16_t>& pre, int tiles,
                               int nch, int T, double pass_s) {
    const double fixed = std::max(1.0, 2e-6 / pass_s);
    const int nsc = sp.nsplit / sp.nts;
    std::vector<double> cost((size_t)tiles * sp.nsplit, 0.0);
    for (int tile = 0; tile < tiles; ++tile)
        for (int sc = 0; sc < nsc; ++sc)
            for (int st = 0; st < sp.nts; ++st) {
                long passes = 0;
                int chunks_run = 0;
                const int k1 = std::min(nch, (sc + 1) * sp.chunks);
                const int t0 = st * sp.txs, t1 = std::min(T, t0 + sp.txs);
                for (int k = sc * sp.chunks; k < k1; ++k) {
                    const uint16_t* r = pre.data() + ((size_t)tile * nch + k) * (T + 1);
                    const int n = r[t1] - r[t0];
                    passes += n;
                    chunks_run += n > 0;
                }
                if (passes > 0)
                    cost[(size_t)tile * sp.nsplit + sc * sp.nts + st] =
                        passes + 5.5 * chunks_run + fixed;
            }
    return cost;
}

// The non-empty items, heaviest first (ties by code: deterministic).
std::vector<int> item_order(const std::vector<double>& cost) {
    std::vector<int> order;
    for (size_t i = 0; i < cost.size(); ++i)
        if (cost[i] > 0.0) order.push_back((int)i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return cost[x] > cost[y]; });
    return order;
}

// Time of a plan in passes of one workgroup.  Workgroups are handed out in
// order, round-robin over the 8 XCDs, each to a free slot of its XCD (32
// CUs x `occ` co-resident workgroups, each running at 1/occ of a CU); a
// workgroup whose XCD is full holds back the ones behind it.  Items that
// run nothing are not launched: their outputs are cleared first (one
// output-sized write per split), and a split adds the reduce kernel
// (nsplit + 1 frame-sized streams) - both at ~4 TB/s, plus launches.
double plan_time(const SplitPlan& sp, const std::vector<double>& cost,
                 const std::vector<int>& order, int occ, double pass_s, double frame_bytes) {
    using MinQ = std::priority_queue<double, std::vector<double>, std::greater<double>>;
    std::vector<MinQ> xcd(8);
    for (auto& q : xcd)
        for (int i = 0; i < 32 * occ; ++i) q.push(0.0);
    double clock = 0.0, end = 0.0;
    for (size_t i = 0; i < order.size(); ++i) {
        MinQ& q = xcd[i & 7];
        const double start = std::max(clock, q.top());
        q.pop();
        const double fin = start + cost[order[i]] * occ;
        q.push(fin);
        clock = start;
        end = std::max(end, fin);
    }
    double extra = 0.0;
    if (order.size() < cost.size()) extra += sp.nsplit * frame_bytes / 4e12 + 2e-6;
    if (sp.nsplit > 1) extra += (sp.nsplit + 1) * frame_bytes / 4e12 + 3e-6;
    return end + extra / pass_s;
}

// The split of a geometry: the candidate (chunks per split x transmit
// splits of 1, 2 or 4) with the least plan_time.  It depends on the
// geometry and the tile plan only, never on the frame count, so a batch and
// its frames one by one run the same items.  Grids with many tiles per
// slot are balanced by the dispatcher already and are not split.
SplitPlan plan_split(int mode, const Geometry& g, const wf_acq* acq, const wf_grid* grid,
                     const TilePlan& tp) {
    SplitPlan base;
    const int T = acq->n_tx;
    const int nch = (acq->n_ch + wf::kChunk - 1) / wf::kChunk;
    base.chunks = nch;
    base.txs = T;
    const long long tiles = (long long)tp.ntz * tp.ntx;
    const int by_waves = std::max(1, 16 / (tp.threads / 64));
    const int by_lds = std::max(1, (int)(kLdsHard / std::max<size_t>(tp.lds, 1)));
    const int occ = std::min(by_waves, by_lds);
    if (tiles >= 8LL * 256 * occ) return base;
    // the pass map holds tiles x chunks x (T + 1) counts: planning is skipped
    // beyond 32 M of them (64 MB), where the tiles outnumber the slots anyway
    if (tiles * nch * (T + 1LL) > (32LL << 20)) return base;

    std::vector<uint16_t> pre;
    pass_map(mode, g, acq, grid, tp, &pre);
    // one pass: NT x PX pixels x 16 channels at ~8 lane-ops each on one CU,
    // and no less than ~0.5 us (barrier and LDS round trips bound small tiles)
    const double pass_s =
        std::max(0.5e-6, (double)tp.threads * tp.px * wf::kChunk * 8.0 / 153.6e9);
    const double frame_bytes = (double)grid->nz * grid->nx * 4.0;
    auto evaluate = [&](SplitPlan& sp) {
        const std::vector<double> cost = item_costs(sp, pre, (int)tiles, nch, T, pass_s);
        sp.order = item_order(cost);
        return plan_time(sp, cost, sp.order, occ, pass_s, frame_bytes);
    };
    // candidates: no split, then chunk splits x transmit splits of 1, 2, 4
    std::vector<std::pair<SplitPlan, double>> cand;
    SplitPlan none = base;
    const double none_time = evaluate(none);
    cand.emplace_back(std::move(none), none_time);
    for (int nsc = 1; nsc <= nch; ++nsc) {
        const int cps = (nch + nsc - 1) / nsc;  // even chunk ranges
        if ((nch + cps - 1) / cps != nsc) continue;  // not reachable with even ranges
        for (int nts : {1, 2, 4}) {
            if (nts > 1 && T / nts < 8) continue;
            SplitPlan sp;
            sp.chunks = cps;
            sp.nts = nts;
            sp.txs = (T + nts - 1) / nts;
            sp.nsplit = nsc * nts;
            if (sp.nsplit == 1 || sp.nsplit > 64) continue;
            const double t = evaluate(sp);
            cand.emplace_back(std::move(sp), t);
        }
    }
    // The modelled times are coarse (pass costs vary, the dispatcher is
    // modelled only roughly): the grid stays unsplit unless running it so
    // costs 3 % more than the best candidate; otherwise, among the
    // candidates within 5 % of the best, the one with the most items, whose
    // heaviest-first list then balances best (measured: finer lists win
    // where the estimate says tie).
    double tmin = none_time;
    for (const auto& c : cand) tmin = std::min(tmin, c.second);
    SplitPlan best = cand[0].first;
    if (none_time > 1.03 * tmin) {
        size_t most = 0;
        for (const auto& c : cand)
            if (c.second <= 1.05 * tmin && c.first.order.size() > most) {
                most = c.first.order.size();
                best = c.first;
            }
    }
    return best;
}

size_t split_ws_bytes(const SplitPlan& sp, int n_frames, int nz, int nx) {
    return sp.nsplit > 1 ? (size_t)sp.nsplit * n_frames * nz * nx * 4 : 0;
}

// ---------------------------------------------------------------------------
// plans: host half (geometry, tile plan, work split) and device tables
// ---------------------------------------------------------------------------

// Everything a DAS-shaped launch needs on the host for one geometry.  Two
// calls with equal keys run the same tiles, windows, delays and items.
struct PlanCore {
    int mode = 0;
    int n_tx = 0, n_ch = 0, n_s = 0, nz = 0, nx = 0;
    Geometry g;
    TilePlan tp;
    SplitPlan sp;
    TilePlan atp;   // the adjoint's tiles (plan_adjoint)
    SplitPlan asp;  // and their split
    std::string key;
};

// The key of a geometry: the dimensions and every float the kernels or the
// planner read, including the per-transmit and per-channel tables (which
// carry the speed of sound, sampling rate, time origin, probe and grid).
std::string geometry_key(int mode, const wf_acq* acq, const wf_grid* grid, const Geometry& g) {
    std::string k;
    const int32_t dims[] = {mode, acq->n_tx, acq->n_ch, acq->n_s, grid->nz, grid->nx};
    key_add(k, dims, sizeof dims);
    const float f[] = {g.Z0.x, g.Z0.y, g.dZ.x, g.dZ.y, g.dX.x, g.dX.y, g.O.x,
                       g.O.y,  g.x0f,  g.dxf,  g.fnum2, g.dxq};
    key_add(k, f, sizeof f);
    const double d[] = {g.dzs, g.dxs};
    key_add(k, d, sizeof d);
    key_add(k, g.tx.data(), g.tx.size() * sizeof(wf::TxConst));
    key_add(k, g.ch.data(), g.ch.size() * sizeof(wf::ChConst));
    return k;
}

int das_passes_per_barrier(const TilePlan& tp, int T, int dtype);

// Relative time per contribution of a tile plan and its split, a model
// fitted to the gather's measured times on gfx950 (every shape and tile
// height of the tile candidates, on STAI and PWI geometries from 128 x 128
// to 2048 x 128 pixels and 11 to 128 transmits):
//  - each staged window sample serves `reuse` pixels; staging it costs
//    about 1.5 contributions;
//  - a CU hides latency with 32 pixels in flight per lane slot (16 waves of
//    two pixels); with fewer, the cost rises by up to 2x at none;
//  - one pixel a thread shares no per-thread work (delay words, window
//    bases) between pixels: 6 %;
//  - a workgroup that takes a CU's LDS alone exposes its start (tables,
//    first window) and end (partial-frame write) whenever others queue
//    for the CU: about half the time of a 64-pass workgroup.
// Residency counts the 16-bit RF gather (two passes per barrier on
// 1024-thread tiles) so the plan does not depend on the RF type.
// With sp null: the least cost any split can give (every resident slot
// filled, no exposed start or end).
double plan_cost(const TilePlan& tp, const SplitPlan* sp, int T) {
    const int ez = 1 << tp.tz_log2;
    const int ex = (tp.threads * tp.px) >> tp.tz_log2;
    const double reuse = (double)ez * ex / tp.nst;
    const size_t lds = das_gather_lds(tp, T, das_passes_per_barrier(tp, T, WF_RF_I16));
    const int res = std::max(1, std::min((int)(kLdsHard / lds), 2048 / tp.threads));
    const double items = !sp ? 256.0 * res
                             : !sp->order.empty() ? (double)sp->order.size()
                                                  : (double)tp.ntz * tp.ntx * sp->nsplit;
    const double resident = std::min((double)res, std::max(1.0, items / 256.0));
    const double lanes = tp.px * (tp.threads / 64) * resident;
    double cost = (1.0 + 1.5 / reuse) * (1.0 + std::max(0.0, 32.0 - lanes) / 32.0);
    if (tp.px == 1) cost *= 1.06;
    if (res == 1 && sp)
        cost *= 1.0 + 0.5 * 64.0 / ((double)sp->chunks * sp->txs) *
                          std::max(0.0, 1.0 - 256.0 / items);
    return cost;
}

// Tiles of the adjoint.  It flushes every (transmit, channel, tile) window
// to its workspace and sums them into the RF gradient, so its cost grows
// with the windows of a frame (tiles x transmits x channels x nst), and its
// LDS scatter runs best with 16 waves a workgroup.  Measured: STAI full
// 1.66 ms on 1024 x 1 threads over 64 x 16 tiles against 2.55 ms on the
// gather's 512 x 1 over 32 x 16; paper STAI 5.08 ms on 1024 x 1 against
// 5.69 ms on 512 x 2 over the same tiles.  So it keeps the gather's tiles
// when they have 1024 threads, else takes the 1024-pixel candidate of most
// reuse run by 1024 x 1 threads, else the gather's tiles; the split is
// planned for its own tiles.
void plan_adjoint(PlanCore* c, const wf_acq* acq, const wf_grid* grid) {
    c->atp = c->tp;
    c->asp = c->sp;
    if (c->tp.threads == 1024 || !WF_DAS_ALLOW_1024) return;
    const TilePlan* best = nullptr;
    double best_reuse = 0.0;
    const std::vector<TilePlan> cand = tile_candidates(c->g, acq, grid, 8);
    for (const TilePlan& tp : cand) {
        if (tp.threads * tp.px != 1024) continue;
        const int ez = std::min(1 << tp.tz_log2, grid->nz);
        const int ex = std::min(1024 >> tp.tz_log2, grid->nx);
        const double reuse = (double)ez * ex / tp.nst;
        if (reuse > best_reuse * (1.0 + 1e-9)) {
            best_reuse = reuse;
            best = &tp;
        }
    }
    if (!best) return;
    c->atp = *best;
    c->atp.threads = 1024;
    c->atp.px = 1;
    c->asp = plan_split(c->mode, c->g, acq, grid, c->atp);
}

// Tile plan and work split of a geometry whose `g` and `key` are filled:
// of the tile candidates, each with its own split, the one of least
// plan_cost (ties keep the one of lesser least cost).  Candidates must leave 8 resident
// waves per CU; ones with 4 are taken only when nothing else fits.  Each
// split comes from a dispatch simulation over the pass map: a few
// milliseconds of host time per candidate on the largest grids.
wf_status plan_core(const wf_acq* acq, const wf_grid* grid, PlanCore* c) {
    for (int min_waves : {8, 4}) {
        const std::vector<TilePlan> cand = tile_candidates(c->g, acq, grid, min_waves);
        // candidates in order of their least cost: a split is planned only
        // for those that could still win
        std::vector<std::pair<double, int>> order;
        for (size_t i = 0; i < cand.size(); ++i)
            if ((long long)cand[i].ntz * cand[i].ntx <= 0x7FFFFFFF)
                order.emplace_back(plan_cost(cand[i], nullptr, acq->n_tx), (int)i);
        std::stable_sort(order.begin(), order.end(),
                         [](const auto& x, const auto& y) { return x.first < y.first; });
        double best = 0.0;
        bool found = false;
        for (const auto& o : order) {
            if (found && o.first >= best * (1.0 - 1e-9)) break;
            const TilePlan& tp = cand[o.second];
            SplitPlan sp = plan_split(c->mode, c->g, acq, grid, tp);
            const double cost = plan_cost(tp, &sp, acq->n_tx);
            if (!found || cost < best * (1.0 - 1e-9)) {
                found = true;
                best = cost;
                c->tp = tp;
                c->sp = std::move(sp);
            }
        }
        if (found) {
            plan_adjoint(c, acq, grid);
            return WF_OK;
        }
    }
    return fail(WF_ERR_UNSUPPORTED,
                "pixel spacing (%.3g x %.3g samples) too coarse for the DAS tile window",
                c->g.dzs, c->g.dxs);
}

// Geometry and key of a validated call (cheap: O(elements + transmits +
// channels)); plan_core adds the tile plan and split.
void begin_core(int mode, const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                const double* angles, int32_t tref, const wf_grid* grid, PlanCore* c) {
    c->mode = mode;
    c->n_tx = acq->n_tx;
    c->n_ch = acq->n_ch;
    c->n_s = acq->n_s;
    c->nz = grid->nz;
    c->nx = grid->nx;
    build_geometry(mode, probe, acq, tx_elem, angles, tref, grid, &c->g);
    c->key = geometry_key(mode, acq, grid, c->g);
}

wf_status make_core(int mode, const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                    const double* angles, int32_t tref, const wf_grid* grid, PlanCore* c) {
    begin_core(mode, probe, acq, tx_elem, angles, tref, grid, c);
    return plan_core(acq, grid, c);
}

// Device tables of a plan, inside one block of device memory:
// [TxConst x T][ChConst x C][int x work-list items][int x the adjoint's
// work-list items][uint64 x tiles: the splits each tile runs, for split
// plans that leave items out] and, in plans built with delay tables,
// [receive delay words][transmit delay words]; each part 256-byte aligned.
struct DevTables {
    const wf::TxConst* tx = nullptr;
    const wf::ChConst* ch = nullptr;
    const int* items = nullptr;       // null when the plan has no work list
    const int* aitems = nullptr;      // the adjoint's (null: none)
    const uint64_t* masks = nullptr;  // splits that run, per tile (null: all)
    const uint32_t* rx_q = nullptr;   // receive delay table (null: none)
    const uint32_t* tx_q = nullptr;   // transmit delay table (null: none)
};

int log2_of(int v) {  // v a power of two
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

constexpr size_t kTableAlign = 256;
size_t align_up(size_t v) { return (v + kTableAlign - 1) & ~(kTableAlign - 1); }

struct TableLayout {
    size_t ch, items, aitems, masks, rx, tx, total;
};

// Per tile (z fastest, as the split reduce reads them) the splits whose
// item is on the work list; empty where every item runs or none is split.
std::vector<uint64_t> split_masks(const PlanCore& c) {
    const SplitPlan& sp = c.sp;
    const long long tiles = (long long)c.tp.ntz * c.tp.ntx;
    if (sp.nsplit == 1 || sp.order.empty() || (long long)sp.order.size() == tiles * sp.nsplit)
        return {};
    std::vector<uint64_t> m((size_t)tiles, 0);
    const bool xcd = WF_DAS_XCD_ORDER && tiles % 8 == 0;
    const int per = (int)(tiles >> 3);
    for (int item : sp.order) {
        int tile = item / sp.nsplit;
        const int split = item - tile * sp.nsplit;
        // the kernel's remap; the result, tzi + ntz txi, is the reduce's index
        if (xcd) tile = (tile & 7) * per + (tile >> 3);
        m[(size_t)tile] |= 1ull << split;
    }
    return m;
}

void fill_args(const PlanCore& c, const DevTables& t, const wf_acq* acq, const wf_grid* grid,
               wf::DasArgs* a, const TilePlan* tiles = nullptr);

// Words of the delay tables (DasArgs::rx_tab, tx_tabq): per tile and pixel
// slot, 16 receive words per channel chunk and one transmit word
// per transmit.
size_t rx_table_words(const PlanCore& c) {
    const size_t tiles = (size_t)c.tp.ntz * c.tp.ntx;
    const size_t nch = (size_t)(c.n_ch + wf::kChunk - 1) / wf::kChunk;
    return tiles * nch * (size_t)c.tp.threads * c.tp.px * wf::kChunk;
}
size_t tx_table_words(const PlanCore& c) {
    if (!wf::das_tx_words(c.mode, c.tp.threads, c.tp.px)) return 0;
    return (size_t)c.tp.ntz * c.tp.ntx * c.n_tx * (size_t)c.tp.threads * c.tp.px;
}

TableLayout table_layout(const PlanCore& c, bool delay_tables) {
    TableLayout L;
    L.ch = align_up(c.g.tx.size() * sizeof(wf::TxConst));
    L.items = align_up(L.ch + c.g.ch.size() * sizeof(wf::ChConst));
    L.aitems = align_up(L.items + std::max<size_t>(1, c.sp.order.size()) * sizeof(int));
    L.masks = align_up(L.aitems + std::max<size_t>(1, c.asp.order.size()) * sizeof(int));
    L.rx = align_up(L.masks + std::max<size_t>(1, split_masks(c).size()) * sizeof(uint64_t));
    L.tx = L.rx + (delay_tables ? align_up(rx_table_words(c) * 4) : 0);
    L.total = L.tx + (delay_tables ? align_up(tx_table_words(c) * 4) : 0);
    return L;
}

// Writes the tables into `mem` (at least table_layout().total bytes) with
// kernel launches on `s`: stream-ordered, and capturable.  The delay
// tables come from a kernel that forms the gathers' own words.
wf_status upload_tables(const PlanCore& c, void* mem, bool delay_tables, const wf_acq* acq,
                        const wf_grid* grid, hipStream_t s, DevTables* out) {
    const TableLayout L = table_layout(c, delay_tables);
    char* m = static_cast<char*>(mem);
    hipError_t e = wf::launch_store(m, c.g.tx.data(), c.g.tx.size() * sizeof(wf::TxConst), s);
    if (e == hipSuccess)
        e = wf::launch_store(m + L.ch, c.g.ch.data(), c.g.ch.size() * sizeof(wf::ChConst), s);
    if (e == hipSuccess && !c.sp.order.empty())
        e = wf::launch_store(m + L.items, c.sp.order.data(), c.sp.order.size() * sizeof(int), s);
    if (e == hipSuccess && !c.asp.order.empty())
        e = wf::launch_store(m + L.aitems, c.asp.order.data(), c.asp.order.size() * sizeof(int),
                             s);
    const std::vector<uint64_t> masks = split_masks(c);
    if (e == hipSuccess && !masks.empty())
        e = wf::launch_store(m + L.masks, masks.data(), masks.size() * sizeof(uint64_t), s);
    if (e != hipSuccess) return hip_fail(e, "plan table upload");
    DevTables t;
    t.tx = reinterpret_cast<const wf::TxConst*>(m);
    t.ch = reinterpret_cast<const wf::ChConst*>(m + L.ch);
    t.items = c.sp.order.empty() ? nullptr : reinterpret_cast<const int*>(m + L.items);
    t.aitems = c.asp.order.empty() ? nullptr : reinterpret_cast<const int*>(m + L.aitems);
    t.masks = masks.empty() ? nullptr : reinterpret_cast<const uint64_t*>(m + L.masks);
    if (delay_tables) {
        uint32_t* rx = reinterpret_cast<uint32_t*>(m + L.rx);
        uint32_t* tx = tx_table_words(c) ? reinterpret_cast<uint32_t*>(m + L.tx) : nullptr;
        wf::DasArgs a;
        fill_args(c, t, acq, grid, &a);
        e = wf::launch_delay_tables(c.mode, c.tp.threads, c.tp.px, a, rx, tx, s);
        if (e != hipSuccess) return hip_fail(e, "delay table kernel launch");
        t.rx_q = rx;
        t.tx_q = tx;
    }
    *out = t;
    return WF_OK;
}

// Passes the value and d y / d c gathers stage per barrier: two (four
// window buffers) for 16-bit RF on 1024-thread tiles, where one workgroup
// fills a CU and the buffers fit the LDS; FP32 staging would spill.
int das_passes_per_barrier(const TilePlan& tp, int T, int dtype) {
    return WF_DAS_TWO_PASS && tp.threads == 1024 && dtype != WF_RF_F32 &&
                   das_gather_lds(tp, T, 2) <= kLdsHard
               ? 2
               : 1;
}

// Window sets of the adjoint: two where they fit the LDS (a pass then
// needs one barrier instead of two).
int adjoint_sets(const TilePlan& tp, int T) {
    return WF_ADJ_TWO_SETS &&
                   wf::das_lds(wf::das_adjoint_nbuf(2), tp.slot, T).total <= kLdsHard
               ? 2
               : 1;
}

// Sets the dynamic-LDS limit of every kernel a plan can launch (each RF
// type, single frames and batches, value and d y / d c gathers, the
// adjoint), so calls with the plan, graph capture included, make no
// attribute call.
wf_status prepare_kernels(const PlanCore& c, const wf_acq* acq, const wf_grid* grid) {
    const TilePlan& tp = c.tp;
    const int T = acq->n_tx;
    wf::DasArgs a;
    fill_args(c, DevTables{}, acq, grid, &a);
    a.prepare_only = 1;
    const int groups = (wf::kChunk * a.ng + tp.threads - 1) / tp.threads;
    for (int dtype = WF_RF_I16; dtype <= WF_RF_F32; ++dtype)
        for (int F : {1, 2}) {
            a.F = F;
            a.pp = das_passes_per_barrier(tp, T, dtype);
            const size_t lds = das_gather_lds(tp, T, a.pp);
            hipError_t e = wf::launch_das(c.mode, dtype, tp.threads, tp.px, groups, a, lds, 0);
            if (e == hipSuccess)
                e = wf::launch_das_dydc(c.mode, dtype, tp.threads, tp.px, groups, a, lds, 0);
            if (e != hipSuccess) return hip_fail(e, "DAS kernel attributes");
        }
    const TilePlan& atp = c.atp;
    fill_args(c, DevTables{}, acq, grid, &a, &atp);
    a.prepare_only = 1;
    a.F = 1;
    const int nbuf = adjoint_sets(atp, T);
    hipError_t e = wf::launch_das_adjoint(
        c.mode, atp.threads, atp.px, nbuf, a,
        wf::das_lds(wf::das_adjoint_nbuf(nbuf), atp.slot, T).total, 0);
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel attributes");
    return WF_OK;
}

// ---------------------------------------------------------------------------
// the cache behind calls made without a plan: bounded, least recently used
// ---------------------------------------------------------------------------

#ifndef WF_GEOMETRY_CACHE_ENTRIES
#define WF_GEOMETRY_CACHE_ENTRIES 64
#endif

struct Upload {
    int device = 0;
    void* mem = nullptr;
    size_t bytes = 0;
    DevTables t;
};

struct CacheEntry {
    std::shared_ptr<const PlanCore> core;
    std::vector<Upload> uploads;  // device tables, per device that used them
};

// Entries hold host plans (for the size and plan queries) and, once a call
// ran on a device, library-owned device tables.  The mutex is held from the
// lookup through the launches of a call made without a plan, so an entry
// is never evicted between its lookup and the launches that read it;
// eviction synchronises the device before it frees the tables.
struct GeometryCache {
    std::mutex mu;
    std::list<std::pair<std::string, CacheEntry>> lru;  // most recent first
    std::unordered_map<std::string, std::list<std::pair<std::string, CacheEntry>>::iterator>
        index;
    size_t device_bytes = 0;
};

GeometryCache& cache() {
    static GeometryCache* c = new GeometryCache;  // never destroyed: no teardown order issue
    return *c;
}

hipError_t free_uploads(CacheEntry& e) {
    hipError_t first = hipSuccess;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (Upload& u : e.uploads) {
        hipError_t r = hipSetDevice(u.device);
        if (r == hipSuccess) r = hipDeviceSynchronize();  // work in flight may read it
        if (r == hipSuccess) r = hipFree(u.mem);
        if (r != hipSuccess && first == hipSuccess) first = r;
        cache().device_bytes -= u.bytes;
    }
    e.uploads.clear();
    if (have_cur) (void)hipSetDevice(cur);
    return first;
}

// Host plan of a geometry through the cache (lock held by the caller).
wf_status cached_core(int mode, const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                      const double* angles, int32_t tref, const wf_grid* grid,
                      CacheEntry** out) {
    GeometryCache& gc = cache();
    PlanCore c;
    begin_core(mode, probe, acq, tx_elem, angles, tref, grid, &c);
    auto it = gc.index.find(c.key);
    if (it != gc.index.end()) {
        gc.lru.splice(gc.lru.begin(), gc.lru, it->second);
        *out = &it->second->second;
        return WF_OK;
    }
    wf_status st = plan_core(acq, grid, &c);
    if (st != WF_OK) return st;
    while (gc.lru.size() >= WF_GEOMETRY_CACHE_ENTRIES) {
        auto& victim = gc.lru.back();
        hipError_t e = free_uploads(victim.second);
        gc.index.erase(victim.first);
        gc.lru.pop_back();
        if (e != hipSuccess) return hip_fail(e, "freeing an evicted geometry table");
    }
    std::string key = c.key;
    CacheEntry ce;
    ce.core = std::make_shared<const PlanCore>(std::move(c));
    gc.lru.emplace_front(key, std::move(ce));
    gc.index[key] = gc.lru.begin();
    *out = &gc.lru.front().second;
    return WF_OK;
}

// Delay tables in cache entries: an entry gets them when they take at most
// WF_CACHE_DELAY_TABLE_MAX bytes, and the cache evicts least recently used
// entries to keep its device memory within WF_CACHE_DEVICE_BUDGET.
#ifndef WF_CACHE_DELAY_TABLE_MAX
#define WF_CACHE_DELAY_TABLE_MAX (512ull << 20)
#endif
#ifndef WF_CACHE_DEVICE_BUDGET
#define WF_CACHE_DEVICE_BUDGET (4ull << 30)
#endif

// Device tables of a cached entry on the current device: allocated and
// uploaded on first use, then `s` is synchronised so that calls on other
// streams may read them (lock held by the caller).
wf_status cached_tables(CacheEntry& ce, const wf_acq* acq, const wf_grid* grid, hipStream_t s,
                        DevTables* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (const Upload& u : ce.uploads)
        if (u.device == dev) {
            *out = u.t;
            return WF_OK;
        }
    Upload u;
    u.device = dev;
    const PlanCore& c = *ce.core;
    const size_t plain = table_layout(c, false).total;
    const size_t full = table_layout(c, true).total;
    const bool delay_tables =
        full - plain <= WF_CACHE_DELAY_TABLE_MAX && full <= WF_CACHE_DEVICE_BUDGET;
    u.bytes = delay_tables ? full : plain;
    // room within the budget: evict other entries, least recently used first
    GeometryCache& gc = cache();
    while (gc.device_bytes + u.bytes > WF_CACHE_DEVICE_BUDGET) {
        auto victim = gc.lru.end();
        for (auto it = gc.lru.begin(); it != gc.lru.end(); ++it)
            if (&it->second != &ce && !it->second.uploads.empty()) victim = it;
        if (victim == gc.lru.end()) break;
        e = free_uploads(victim->second);
        if (e != hipSuccess) return hip_fail(e, "freeing an evicted geometry table");
    }
    e = hipMalloc(&u.mem, u.bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(geometry table)");
    wf_status st = upload_tables(c, u.mem, delay_tables, acq, grid, s, &u.t);
    if (st == WF_OK) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "geometry table upload");
    }
    if (st != WF_OK) {
        (void)hipFree(u.mem);
        return st;
    }
    cache().device_bytes += u.bytes;
    ce.uploads.push_back(u);
    *out = u.t;
    return WF_OK;
}

}  // namespace

// The caller-facing plan: a host plan and the device tables it wrote into
// caller-owned memory on one device.
struct wf_plan {
    uint64_t magic;
    std::shared_ptr<const PlanCore> core;
    int device;
    DevTables t;
};

namespace {

constexpr uint64_t kPlanMagic = 0x316e616c705f6677ULL;  // "wf_plan1"

// The plan a DAS-shaped call runs with: the caller's, checked against the
// call's geometry, or the cache's.  Without a plan `lk` takes the cache
// lock and keeps it until the caller's launches are issued.
struct Resolved {
    std::shared_ptr<const PlanCore> core;
    DevTables t;
};

wf_status resolve(int mode, const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                  const double* angles, int32_t tref, const wf_grid* grid, const wf_plan* plan,
                  hipStream_t s, std::unique_lock<std::mutex>* lk, Resolved* r) {
    if (plan) {
        if (plan->magic != kPlanMagic) return fail(WF_ERR_INVALID_ARG, "plan is not a live wf_plan");
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (dev != plan->device)
            return fail(WF_ERR_INVALID_ARG, "plan was built on device %d, the call runs on %d",
                        plan->device, dev);
        Geometry g;
        build_geometry(mode, probe, acq, tx_elem, angles, tref, grid, &g);
        if (plan->core->mode != mode || geometry_key(mode, acq, grid, g) != plan->core->key)
            return fail(WF_ERR_INVALID_ARG,
                        "plan was built for another geometry (mode, sizes, probe, transmits, "
                        "channels, speed of sound, sampling or grid differ)");
        r->core = plan->core;
        r->t = plan->t;
        return WF_OK;
    }
    *lk = std::unique_lock<std::mutex>(cache().mu);
    CacheEntry* ce = nullptr;
    wf_status st = cached_core(mode, probe, acq, tx_elem, angles, tref, grid, &ce);
    if (st != WF_OK) return st;
    if ((st = cached_tables(*ce, acq, grid, s, &r->t)) != WF_OK) return st;
    r->core = ce->core;
    return WF_OK;
}

// Host plan for the size and plan queries (through the cache; no device).
wf_status query_core(int mode, const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                     const double* angles, int32_t tref, const wf_grid* grid,
                     std::shared_ptr<const PlanCore>* out) {
    std::lock_guard<std::mutex> lk(cache().mu);
    CacheEntry* ce = nullptr;
    wf_status st = cached_core(mode, probe, acq, tx_elem, angles, tref, grid, &ce);
    if (st == WF_OK) *out = ce->core;
    return st;
}

// Kernel arguments of a plan (frames, RF, outputs and split set by callers).
// Arguments of a launch on the plan's gather tiles, or on `tiles` (the
// adjoint's), which then get no delay tables (those are the gather's).
void fill_args(const PlanCore& c, const DevTables& t, const wf_acq* acq, const wf_grid* grid,
               wf::DasArgs* a, const TilePlan* tiles) {
    const Geometry& g = c.g;
    const TilePlan& tp = tiles ? *tiles : c.tp;
    *a = wf::DasArgs{};
    a->F = acq->n_frames;
    a->T = acq->n_tx;
    a->C = acq->n_ch;
    a->S = acq->n_s;
    a->nz = grid->nz;
    a->nx = grid->nx;
    a->tz_log2 = tp.tz_log2;
    a->ntz = tp.ntz;
    a->ntx = tp.ntx;
    a->xcd_order = (WF_DAS_XCD_ORDER && (tp.ntz * tp.ntx) % 8 == 0) ? 1 : 0;
    a->nsplit = 1;  // no split unless the caller's workspace allows one
    a->split_chunks = (acq->n_ch + wf::kChunk - 1) / wf::kChunk;
    a->nts = 1;
    a->split_tx = acq->n_tx;
    a->partial = nullptr;
    a->ng = tp.nst / 8;
    a->nst = tp.nst;
    a->slot = tp.slot;
    a->txspan_q = (uint32_t)tp.span << wf::kQBits;
    a->rxspan_q = (uint32_t)tp.span << wf::kQBits;
    a->Z0 = g.Z0;
    a->dZ = g.dZ;
    a->dX = g.dX;
    a->O = g.O;
    a->fnum2 = g.fnum2;
    a->dxq = g.dxq;
    a->inv_dxq = 1.0f / g.dxq;
    a->x0f = g.x0f;
    a->dxf = g.dxf;
    a->t0fs = (float)(acq->t0 * acq->fs);
    a->neg_inv_c = (float)(-1.0 / acq->c);
    a->tx_tab = t.tx;
    a->ch_tab = t.ch;
    a->rx_tab = tiles ? nullptr : t.rx_q;
    a->tx_tabq = tiles ? nullptr : t.tx_q;
}

// Checks of the buffers of a DAS-shaped call (after check_geometry).
wf_status check_das_buffers(const void* rf, const wf_acq* acq, const wf_grid* grid,
                            const float* out) {
    wf_status st = check_rf(rf, acq);
    if (st != WF_OK) return st;
    if (!out) return fail(WF_ERR_INVALID_ARG, "out is NULL");
    if (((uintptr_t)out & 3) != 0) return fail(WF_ERR_INVALID_ARG, "out is not 4-byte aligned");
    const size_t out_bytes = (size_t)acq->n_frames * grid->nz * grid->nx * 4;
    if (overlaps(rf, rf_bytes_of(acq), out, out_bytes))
        return fail(WF_ERR_INVALID_ARG, "out overlaps rf");
    return WF_OK;
}

// The launches of a validated DAS-shaped call (op 0: value, 1: d y / d c)
// with the host plan `core` and its device tables `t`: the split runs when
// the workspace holds its partial frames.
wf_status launch_gather(int mode, int op, const void* rf, const wf_acq* acq, const wf_grid* grid,
                        const PlanCore& core, const DevTables& t, float* out, void* workspace,
                        uint64_t ws_bytes, hipStream_t stream) {
    const TilePlan& tp = core.tp;
    const SplitPlan& sp = core.sp;
    const size_t out_bytes = (size_t)acq->n_frames * grid->nz * grid->nx * 4;
    wf::DasArgs a;
    fill_args(core, t, acq, grid, &a);
    a.rf = rf;
    a.out = out;
    const size_t need = split_ws_bytes(sp, acq->n_frames, grid->nz, grid->nx);
    const bool split = need > 0 && workspace && ws_bytes >= need;
    if (split) {
        if (((uintptr_t)workspace & 3) != 0)
            return fail(WF_ERR_INVALID_ARG, "workspace is not 4-byte aligned");
        if (overlaps(workspace, need, out, out_bytes) ||
            overlaps(workspace, need, rf, rf_bytes_of(acq)))
            return fail(WF_ERR_INVALID_ARG, "workspace overlaps rf or out");
        a.partial = static_cast<float*>(workspace);
        a.nsplit = sp.nsplit;
        a.split_chunks = sp.chunks;
        a.nts = sp.nts;
        a.split_tx = sp.txs;
    }
    // work list: the plan's non-empty items, heaviest first, when the split
    // it was made for is the one that runs.  The split reduce leaves out the
    // partial frames of the items the list leaves out; unsplit, their tiles
    // of the output are cleared first (a fill kernel: the call may be
    // captured).  A grid whose every tile runs, unsplit, keeps the plain
    // tile order.
    const long long all_items = (long long)tp.ntz * tp.ntx * sp.nsplit;
    const bool listed = split ? !sp.order.empty()
                              : sp.nsplit == 1 && !sp.order.empty() &&
                                    (long long)sp.order.size() < all_items;
    wf::SplitMasks masks{};
    if (listed) {
        a.items = t.items;
        a.nitems = (int)sp.order.size();
        if ((long long)sp.order.size() < all_items) {
            if (split) {
                if (!t.masks) return fail(WF_ERR_INVALID_ARG, "plan tables lack the split masks");
                masks.masks = t.masks;
                masks.npix = grid->nz * grid->nx;
                masks.nx = grid->nx;
                masks.ntz = tp.ntz;
                masks.tz_log2 = tp.tz_log2;
                masks.txw_log2 = log2_of((tp.threads * tp.px) >> tp.tz_log2);
            } else {
                hipError_t e = wf::launch_fill(out, out_bytes / 4, 0.0f, stream);
                if (e != hipSuccess) return hip_fail(e, "fill launch");
            }
        }
    }
    // value and d y / d c gathers share the tile plan and the LDS layout;
    // the dynamic LDS is sized for the passes staged per barrier
    a.pp = das_passes_per_barrier(tp, acq->n_tx, acq->dtype);
    const size_t lds = das_gather_lds(tp, acq->n_tx, a.pp);
    hipError_t e = op == 0 ? wf::launch_das(mode, acq->dtype, tp.threads, tp.px,
                                            groups_of(a, tp), a, lds, stream)
                           : wf::launch_das_dydc(mode, acq->dtype, tp.threads, tp.px,
                                                 groups_of(a, tp), a, lds, stream);
    if (e == hipSuccess && a.partial)
        e = wf::launch_split_reduce(a.partial, a.nsplit, out_bytes / 4, out, masks, stream);
    if (e != hipSuccess) return hip_fail(e, op == 0 ? "DAS kernel launch" : "dy/dc kernel launch");
    return ok();
}

wf_status das_common(int mode, int op, const void* rf, const wf_probe* probe, const wf_acq* acq,
                     const int32_t* tx_elem, const double* angles, int32_t tref,
                     const wf_grid* grid, const wf_plan* plan, float* out, void* workspace,
                     uint64_t ws_bytes, void* stream) {
    wf_status st = check_geometry(mode, probe, acq, tx_elem, angles, tref, grid, true);
    if (st != WF_OK) return st;
    if ((st = check_das_buffers(rf, acq, grid, out)) != WF_OK) return st;
    std::unique_lock<std::mutex> lk;
    Resolved r;
    if ((st = resolve(mode, probe, acq, tx_elem, angles, tref, grid, plan, (hipStream_t)stream,
                      &lk, &r)) != WF_OK)
        return st;
    return launch_gather(mode, op, rf, acq, grid, *r.core, r.t, out, workspace, ws_bytes,
                         (hipStream_t)stream);
}

// Host plans of the static-scratch entry point: a small least-recently-used
// list in host memory only.  It holds no device tables, so dropping an entry
// frees no device memory.
struct HostPlans {
    std::mutex mu;
    std::list<std::shared_ptr<const PlanCore>> lru;  // most recent first
};

HostPlans& host_plans() {
    static HostPlans* h = new HostPlans;  // never destroyed: no teardown order issue
    return *h;
}

constexpr size_t kHostPlans = 16;

wf_status host_plan(int mode, const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                    const double* angles, int32_t tref, const wf_grid* grid,
                    std::shared_ptr<const PlanCore>* out) {
    auto c = std::make_shared<PlanCore>();
    begin_core(mode, probe, acq, tx_elem, angles, tref, grid, c.get());
    HostPlans& hp = host_plans();
    std::lock_guard<std::mutex> lk(hp.mu);
    for (auto it = hp.lru.begin(); it != hp.lru.end(); ++it)
        if ((*it)->key == c->key) {
            hp.lru.splice(hp.lru.begin(), hp.lru, it);
            *out = hp.lru.front();
            return WF_OK;
        }
    wf_status st = plan_core(acq, grid, c.get());
    if (st != WF_OK) return st;
    if (hp.lru.size() >= kHostPlans) hp.lru.pop_back();
    hp.lru.push_front(c);
    *out = c;
    return WF_OK;
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

wf_status check_image(const float* a, int F, int nz, int nx, const char* name) {
    if (!a) return fail(WF_ERR_INVALID_ARG, "%s is NULL", name);
    if (F < 1 || F > 65535) return fail(WF_ERR_INVALID_ARG, "n_frames=%d outside [1, 65535]", F);
    if (nz < 1 || nx < 1 || nx > 65536)
        return fail(WF_ERR_INVALID_ARG, "image %d x %d is empty or too wide", nz, nx);
    if ((long long)nz * nx > (1LL << 28)) return fail(WF_ERR_INVALID_ARG, "image too large");
    return WF_OK;
}

}  // namespace

namespace wf {

wf_status report_hip(hipError_t e, const char* what) { return hip_fail(e, what); }

wf_status das_scratch(int32_t mode, const void* rf, const wf_probe* probe, const wf_acq* acq,
                      const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                      const wf_grid* grid, float* out, wf_status (*get_scratch)(void**),
                      size_t scratch_bytes, hipStream_t stream) {
    if (mode != 0 && mode != 1) return fail(WF_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    const int32_t* tx = mode == 0 ? tx_elem : nullptr;
    const double* ang = mode == 1 ? angles_rad : nullptr;
    wf_status st = check_geometry(mode, probe, acq, tx, ang, tref, grid, true);
    if (st != WF_OK) return st;
    if ((st = check_das_buffers(rf, acq, grid, out)) != WF_OK) return st;
    std::shared_ptr<const PlanCore> core;
    if ((st = host_plan(mode, probe, acq, tx, ang, tref, grid, &core)) != WF_OK) return st;
    const size_t tables = table_layout(*core, false).total;
    if (tables > scratch_bytes)
        return fail(WF_ERR_UNSUPPORTED,
                    "the geometry tables take %llu bytes, more than the %llu-byte static scratch",
                    (unsigned long long)tables, (unsigned long long)scratch_bytes);
    // tables first, then the split's partial frames where they fit (the
    // call runs unsplit otherwise)
    void* scratch = nullptr;
    if ((st = get_scratch(&scratch)) != WF_OK) return st;
    DevTables t;
    if ((st = upload_tables(*core, scratch, false, acq, grid, stream, &t)) != WF_OK) return st;
    char* ws = static_cast<char*>(scratch) + tables;
    return launch_gather(mode, 0, rf, acq, grid, *core, t, out, ws, scratch_bytes - tables,
                         stream);
}

}  // namespace wf

extern "C" {

int32_t wf_abi_version(void) { return WF_ABI_VERSION; }

const char* wf_last_error(void) { return g_err.c_str(); }

wf_status wf_das_stai(const void* rf, const wf_probe* probe, const wf_acq* acq,
                      const int32_t* tx_elem, const wf_grid* grid, const wf_plan* plan,
                      float* out, void* workspace, uint64_t workspace_bytes, void* stream) {
    return das_common(0, 0, rf, probe, acq, tx_elem, nullptr, 0, grid, plan, out, workspace,
                      workspace_bytes, stream);
}

wf_status wf_das_pwi(const void* rf, const wf_probe* probe, const wf_acq* acq,
                     const double* angles_rad, int32_t tref, const wf_grid* grid,
                     const wf_plan* plan, float* out, void* workspace, uint64_t workspace_bytes,
                     void* stream) {
    return das_common(1, 0, rf, probe, acq, nullptr, angles_rad, tref, grid, plan, out,
                      workspace, workspace_bytes, stream);
}

wf_status wf_das_dydc(int32_t mode, const void* rf, const wf_probe* probe, const wf_acq* acq,
                      const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                      const wf_grid* grid, const wf_plan* plan, float* dydc, void* workspace,
                      uint64_t workspace_bytes, void* stream) {
    if (mode != 0 && mode != 1) return fail(WF_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    return das_common(mode, 1, rf, probe, acq, mode == 0 ? tx_elem : nullptr,
                      mode == 1 ? angles_rad : nullptr, tref, grid, plan, dydc, workspace,
                      workspace_bytes, stream);
}

wf_status wf_das_workspace(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                           const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                           const wf_grid* grid, uint64_t* bytes) {
    if (mode != 0 && mode != 1) return fail(WF_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    if (!bytes) return fail(WF_ERR_INVALID_ARG, "bytes is NULL");
    const int32_t* tx = mode == 0 ? tx_elem : nullptr;
    const double* ang = mode == 1 ? angles_rad : nullptr;
    wf_status st = check_geometry(mode, probe, acq, tx, ang, tref, grid, true);
    if (st != WF_OK) return st;
    std::shared_ptr<const PlanCore> c;
    if ((st = query_core(mode, probe, acq, tx, ang, tref, grid, &c)) != WF_OK) return st;
    *bytes = split_ws_bytes(c->sp, acq->n_frames, grid->nz, grid->nx);
    return ok();
}

// Workspace of the two-stage adjoint for one frame: every (transmit,
// channel, tile) window (nst + 1 floats) and its first sample (int).
size_t adjoint_ws_bytes(const PlanCore& c) {
    const TilePlan& tp = c.atp;
    const size_t slots = (size_t)c.n_tx * c.n_ch * tp.ntz * tp.ntx;
    return slots * (size_t)(tp.nst + 1) * 4 + slots * 4 + 256 + 256;  // + max |g|
}

wf_status wf_das_adjoint_workspace(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                                   const int32_t* tx_elem, const double* angles_rad,
                                   int32_t tref, const wf_grid* grid, uint64_t* bytes) {
    if (mode != 0 && mode != 1) return fail(WF_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    if (!bytes) return fail(WF_ERR_INVALID_ARG, "bytes is NULL");
    const int32_t* tx = mode == 0 ? tx_elem : nullptr;
    const double* ang = mode == 1 ? angles_rad : nullptr;
    wf_status st = check_geometry(mode, probe, acq, tx, ang, tref, grid, true);
    if (st != WF_OK) return st;
    std::shared_ptr<const PlanCore> c;
    if ((st = query_core(mode, probe, acq, tx, ang, tref, grid, &c)) != WF_OK) return st;
    *bytes = adjoint_ws_bytes(*c);
    return ok();
}

wf_status wf_das_adjoint(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                         const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                         const wf_grid* grid, const wf_plan* plan, const float* g, float* grad_rf,
                         void* workspace, uint64_t workspace_bytes, void* stream) {
    if (mode != 0 && mode != 1) return fail(WF_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    const int32_t* tx = mode == 0 ? tx_elem : nullptr;
    const double* ang = mode == 1 ? angles_rad : nullptr;
    wf_status st = check_geometry(mode, probe, acq, tx, ang, tref, grid, true);
    if (st != WF_OK) return st;
    if (acq->dtype != WF_RF_F32)
        return fail(WF_ERR_INVALID_ARG, "the RF gradient is float32 (acq->dtype=%d)", acq->dtype);
    if (!g) return fail(WF_ERR_INVALID_ARG, "g is NULL");
    if (!grad_rf) return fail(WF_ERR_INVALID_ARG, "grad_rf is NULL");
    if (!workspace) return fail(WF_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)grad_rf & 3) != 0 || ((uintptr_t)g & 3) != 0 ||
        ((uintptr_t)workspace & 255) != 0)
        return fail(WF_ERR_INVALID_ARG,
                    "g and grad_rf must be 4-byte and workspace 256-byte aligned");
    const size_t gbytes = (size_t)acq->n_frames * grid->nz * grid->nx * 4;
    if (overlaps(g, gbytes, grad_rf, rf_bytes_of(acq)))
        return fail(WF_ERR_INVALID_ARG, "grad_rf overlaps g");
    std::unique_lock<std::mutex> lk;
    Resolved r;
    if ((st = resolve(mode, probe, acq, tx, ang, tref, grid, plan, (hipStream_t)stream, &lk,
                      &r)) != WF_OK)
        return st;
    const TilePlan& tp = r.core->atp;
    const SplitPlan& sp = r.core->asp;
    const size_t need = adjoint_ws_bytes(*r.core);
    if (workspace_bytes < need)
        return fail(WF_ERR_WORKSPACE, "workspace of %llu bytes, %llu needed",
                    (unsigned long long)workspace_bytes, (unsigned long long)need);
    if (overlaps(workspace, need, grad_rf, rf_bytes_of(acq)) || overlaps(workspace, need, g, gbytes))
        return fail(WF_ERR_INVALID_ARG, "workspace overlaps g or grad_rf");
    wf::DasArgs a;
    fill_args(*r.core, r.t, acq, grid, &a, &tp);
    const size_t slots = (size_t)acq->n_tx * acq->n_ch * tp.ntz * tp.ntx;
    a.ntiles = tp.ntz * tp.ntx;
    a.ws_win = static_cast<float*>(workspace);
    a.ws_a0 = reinterpret_cast<int*>(static_cast<char*>(workspace) + slots * (tp.nst + 1) * 4);
    float* gmax = reinterpret_cast<float*>(
        (reinterpret_cast<uintptr_t>(a.ws_a0 + slots) + 255) & ~(uintptr_t)255);
    a.ws_gmax = gmax;
    a.F = 1;  // one frame per launch pair: the workspace holds one frame
    // the forward's work split: items write disjoint windows, so the split
    // needs no partial sums; windows of items left out of the work list are
    // marked empty first (a fill kernel with kNoWindow's bit pattern)
    a.nsplit = sp.nsplit;
    a.split_chunks = sp.chunks;
    a.nts = sp.nts;
    a.split_tx = sp.txs;
    const long long all_items = (long long)a.ntiles * sp.nsplit;
    const bool skipped = !sp.order.empty() && (long long)sp.order.size() < all_items;
    if (!sp.order.empty() && (sp.nsplit > 1 || skipped)) {
        a.items = r.t.aitems;
        a.nitems = (int)sp.order.size();
    }
    float no_window;
    static_assert(sizeof(no_window) == sizeof(wf::kNoWindow), "kNoWindow is 32-bit");
    std::memcpy(&no_window, &wf::kNoWindow, sizeof no_window);
    // one set of 8-byte G and H windows takes the bytes of the forward's two
    // buffers of 8-byte entries; a second set, where it fits, saves a
    // barrier per pass
    const int nbuf = adjoint_sets(tp, acq->n_tx);
    const size_t lds = wf::das_lds(wf::das_adjoint_nbuf(nbuf), tp.slot, acq->n_tx).total;
    const size_t frame_rf = (size_t)acq->n_tx * acq->n_ch * acq->n_s;
    for (int f = 0; f < acq->n_frames; ++f) {
        a.g = g + (size_t)f * grid->nz * grid->nx;
        hipError_t e = wf::launch_absmax(a.g, (size_t)grid->nz * grid->nx, gmax,
                                         (hipStream_t)stream);
        if (e == hipSuccess && a.items && skipped)
            e = wf::launch_fill(reinterpret_cast<float*>(a.ws_a0), slots, no_window,
                                (hipStream_t)stream);
        if (e == hipSuccess)
            e = wf::launch_das_adjoint(mode, tp.threads, tp.px, nbuf, a, lds,
                                       (hipStream_t)stream);
        if (e == hipSuccess)
            e = wf::launch_adjoint_reduce(a.ws_win, a.ws_a0, grad_rf + (size_t)f * frame_rf,
                                          acq->n_tx * acq->n_ch, a.ntiles, tp.nst + 1, acq->n_s,
                                          (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
    }
    return ok();
}

// ---------------------------------------------------------------------------
// plans in caller memory
// ---------------------------------------------------------------------------

static wf_status check_plan_flags(int32_t flags) {
    if (flags & ~WF_PLAN_DELAY_TABLES)
        return fail(WF_ERR_INVALID_ARG, "unknown plan flags 0x%x", (unsigned)flags);
    return WF_OK;
}

static wf_status plan_bytes_common(int mode, const wf_probe* probe, const wf_acq* acq,
                                   const int32_t* tx_elem, const double* angles, int32_t tref,
                                   const wf_grid* grid, int32_t flags, uint64_t* bytes) {
    if (!bytes) return fail(WF_ERR_INVALID_ARG, "bytes is NULL");
    wf_status st = check_plan_flags(flags);
    if (st != WF_OK) return st;
    st = check_geometry(mode, probe, acq, tx_elem, angles, tref, grid, true);
    if (st != WF_OK) return st;
    PlanCore c;
    if ((st = make_core(mode, probe, acq, tx_elem, angles, tref, grid, &c)) != WF_OK) return st;
    *bytes = table_layout(c, (flags & WF_PLAN_DELAY_TABLES) != 0).total;
    return ok();
}

static wf_status plan_build_common(int mode, const wf_probe* probe, const wf_acq* acq,
                                   const int32_t* tx_elem, const double* angles, int32_t tref,
                                   const wf_grid* grid, int32_t flags, void* dev_mem,
                                   uint64_t bytes, wf_plan** out, void* stream) {
    if (!out) return fail(WF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    wf_status st = check_plan_flags(flags);
    if (st != WF_OK) return st;
    const bool delay_tables = (flags & WF_PLAN_DELAY_TABLES) != 0;
    st = check_geometry(mode, probe, acq, tx_elem, angles, tref, grid, true);
    if (st != WF_OK) return st;
    if (!dev_mem) return fail(WF_ERR_INVALID_ARG, "dev_mem is NULL");
    if (((uintptr_t)dev_mem & (kTableAlign - 1)) != 0)
        return fail(WF_ERR_INVALID_ARG, "dev_mem is not 256-byte aligned");
    auto c = std::make_shared<PlanCore>();
    if ((st = make_core(mode, probe, acq, tx_elem, angles, tref, grid, c.get())) != WF_OK)
        return st;
    const size_t need = table_layout(*c, delay_tables).total;
    if (bytes < need)
        return fail(WF_ERR_WORKSPACE, "plan memory of %llu bytes, %llu needed",
                    (unsigned long long)bytes, (unsigned long long)need);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((st = prepare_kernels(*c, acq, grid)) != WF_OK) return st;
    DevTables t;
    if ((st = upload_tables(*c, dev_mem, delay_tables, acq, grid, (hipStream_t)stream, &t)) !=
        WF_OK)
        return st;
    wf_plan* p = new (std::nothrow) wf_plan;
    if (!p) return fail(WF_ERR_DEVICE, "out of host memory for the plan handle");
    p->magic = kPlanMagic;
    p->core = std::move(c);
    p->device = dev;
    p->t = t;
    *out = p;
    return ok();
}

wf_status wf_plan_bytes_stai(const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                             const wf_grid* grid, int32_t flags, uint64_t* bytes) {
    return plan_bytes_common(0, probe, acq, tx_elem, nullptr, 0, grid, flags, bytes);
}

wf_status wf_plan_bytes_pwi(const wf_probe* probe, const wf_acq* acq, const double* angles_rad,
                            int32_t tref, const wf_grid* grid, int32_t flags, uint64_t* bytes) {
    return plan_bytes_common(1, probe, acq, nullptr, angles_rad, tref, grid, flags, bytes);
}

wf_status wf_plan_build_stai(const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                             const wf_grid* grid, int32_t flags, void* dev_mem, uint64_t bytes,
                             wf_plan** out, void* stream) {
    return plan_build_common(0, probe, acq, tx_elem, nullptr, 0, grid, flags, dev_mem, bytes,
                             out, stream);
}

wf_status wf_plan_build_pwi(const wf_probe* probe, const wf_acq* acq, const double* angles_rad,
                            int32_t tref, const wf_grid* grid, int32_t flags, void* dev_mem,
                            uint64_t bytes, wf_plan** out, void* stream) {
    return plan_build_common(1, probe, acq, nullptr, angles_rad, tref, grid, flags, dev_mem,
                             bytes, out, stream);
}

void wf_plan_destroy(wf_plan* plan) {
    if (!plan || plan->magic != kPlanMagic) return;
    plan->magic = 0;
    delete plan;
}

wf_status wf_plan_workspace(const wf_plan* plan, int32_t n_frames, uint64_t* das_bytes,
                            uint64_t* adjoint_bytes) {
    if (!plan || plan->magic != kPlanMagic)
        return fail(WF_ERR_INVALID_ARG, "plan is not a live wf_plan");
    if (n_frames < 1 || n_frames > 65535)
        return fail(WF_ERR_INVALID_ARG, "n_frames=%d outside [1, 65535]", n_frames);
    if (!das_bytes || !adjoint_bytes)
        return fail(WF_ERR_INVALID_ARG, "das_bytes and adjoint_bytes must not be NULL");
    const PlanCore& c = *plan->core;
    *das_bytes = split_ws_bytes(c.sp, n_frames, c.nz, c.nx);
    *adjoint_bytes = adjoint_ws_bytes(c);
    return ok();
}

wf_status wf_geometry_cache_info(uint64_t* entries, uint64_t* device_bytes) {
    if (!entries || !device_bytes)
        return fail(WF_ERR_INVALID_ARG, "entries and device_bytes must not be NULL");
    std::lock_guard<std::mutex> lk(cache().mu);
    *entries = cache().lru.size();
    *device_bytes = cache().device_bytes;
    return ok();
}

wf_status wf_dot(const float* a, const float* b, int64_t n, float* out, void* stream) {
    if (!a || !b || !out) return fail(WF_ERR_INVALID_ARG, "a, b and out must not be NULL");
    if (n < 0) return fail(WF_ERR_INVALID_ARG, "n=%lld is negative", (long long)n);
    hipError_t e = wf::launch_dot(a, b, (size_t)n, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dot kernel launch");
    return ok();
}

wf_status wf_das_tile_info(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                           const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                           const wf_grid* grid, int32_t* info) {
    if (mode != 0 && mode != 1) return fail(WF_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    wf_status st = check_geometry(mode, probe, acq, tx_elem, angles_rad, tref, grid, true);
    if (st != WF_OK) return st;
    if (!info) return fail(WF_ERR_INVALID_ARG, "info is NULL");
    std::shared_ptr<const PlanCore> c;
    if ((st = query_core(mode, probe, acq, mode == 0 ? tx_elem : nullptr,
                         mode == 1 ? angles_rad : nullptr, tref, grid, &c)) != WF_OK)
        return st;
    const TilePlan& tp = c->tp;
    info[0] = tp.px;
    info[1] = 1 << tp.tz_log2;
    info[2] = (tp.threads * tp.px) >> tp.tz_log2;
    info[3] = tp.span;
    info[4] = tp.nst;
    info[5] = tp.slot;
    info[6] = (int32_t)das_gather_lds(tp, acq->n_tx,
                                      das_passes_per_barrier(tp, acq->n_tx, acq->dtype));
    info[7] = tp.ntz;
    info[8] = tp.ntx;
    info[9] = wf::kChunk;
    info[10] = tp.threads;
    const SplitPlan& sp = c->sp;
    const long long all_items = (long long)tp.ntz * tp.ntx * sp.nsplit;
    const bool listed = sp.nsplit > 1 ? !sp.order.empty()
                                      : !sp.order.empty() && (long long)sp.order.size() < all_items;
    info[11] = sp.nsplit;
    info[12] = sp.chunks;
    info[13] = sp.nts;
    info[14] = sp.txs;
    info[15] = (int32_t)(listed ? (long long)sp.order.size() : all_items);
    info[16] = c->atp.threads;
    info[17] = c->atp.px;
    info[18] = 1 << c->atp.tz_log2;
    info[19] = c->asp.nsplit;
    return ok();
}

wf_status wf_delays(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                    const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                    const wf_grid* grid, float* tx_hi, float* tx_lo, float* rx_hi,
                    float* rx_lo, void* stream) {
    if (mode != 0 && mode != 1) return fail(WF_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    wf_status st = check_geometry(mode, probe, acq, tx_elem, angles_rad, tref, grid, false);
    if (st != WF_OK) return st;
    if (!tx_hi || !tx_lo || !rx_hi || !rx_lo)
        return fail(WF_ERR_INVALID_ARG, "an output pointer is NULL");
    // a verification call: the tables go to a temporary device buffer that
    // is freed once the stream has run the kernel
    PlanCore c;
    build_geometry(mode, probe, acq, tx_elem, angles_rad, tref, grid, &c.g);
    const TableLayout L = table_layout(c, false);
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, L.total);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(delay tables)");
    DevTables t;
    st = upload_tables(c, mem, false, acq, grid, (hipStream_t)stream, &t);
    if (st != WF_OK) {
        (void)hipFree(mem);
        return st;
    }
    const Geometry& g = c.g;
    wf::DelayArgs a{};
    a.tx_hi = tx_hi;
    a.tx_lo = tx_lo;
    a.rx_hi = rx_hi;
    a.rx_lo = rx_lo;
    a.T = acq->n_tx;
    a.C = acq->n_ch;
    a.nz = grid->nz;
    a.nx = grid->nx;
    a.Z0 = g.Z0;
    a.dZ = g.dZ;
    a.dX = g.dX;
    a.O = g.O;
    a.tx_tab = t.tx;
    a.ch_tab = t.ch;
    e = wf::launch_delays(mode, a, (hipStream_t)stream);
    hipError_t e2 = hipStreamSynchronize((hipStream_t)stream);
    hipError_t e3 = hipFree(mem);
    if (e != hipSuccess) return hip_fail(e, "delay kernel launch");
    if (e2 != hipSuccess) return hip_fail(e2, "delay kernel");
    if (e3 != hipSuccess) return hip_fail(e3, "hipFree(delay tables)");
    return ok();
}

wf_status wf_envelope(const float* bf, int32_t n_frames, int32_t nz, int32_t nx, float* env,
                      float* col_max, void* stream) {
    wf_status st = check_image(bf, n_frames, nz, nx, "bf");
    if (st != WF_OK) return st;
    if (!env) return fail(WF_ERR_INVALID_ARG, "env is NULL");
    if (!col_max) return fail(WF_ERR_INVALID_ARG, "col_max is NULL");
    if (!is_pow2(nz) || nz < 2 || nz > 4096)
        return fail(WF_ERR_UNSUPPORTED, "nz=%d is not a power of two in [2, 4096]", nz);
    const size_t img = (size_t)n_frames * nz * nx * 4;
    if (overlaps(col_max, (size_t)n_frames * nx * 4, bf, img) ||
        overlaps(col_max, (size_t)n_frames * nx * 4, env, img))
        return fail(WF_ERR_INVALID_ARG, "col_max overlaps an image");
    if (env != bf && overlaps(env, img, bf, img))
        return fail(WF_ERR_INVALID_ARG, "env partially overlaps bf");
    hipError_t e = wf::launch_envelope(bf, n_frames, nz, nx, env, col_max, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "envelope kernel launch");
    return ok();
}

wf_status wf_log_compress(const float* env, const float* col_max, int32_t n_frames, int32_t nz,
                          int32_t nx, float dr_db, int32_t flags, float* out_db, void* stream) {
    wf_status st = check_image(env, n_frames, nz, nx, "env");
    if (st != WF_OK) return st;
    if (!col_max) return fail(WF_ERR_INVALID_ARG, "col_max is NULL");
    if (!out_db) return fail(WF_ERR_INVALID_ARG, "out_db is NULL");
    if (!std::isfinite(dr_db) || dr_db <= 0.0f)
        return fail(WF_ERR_INVALID_ARG, "dr_db must be > 0");
    if (flags & ~WF_BMODE_OFFSET) return fail(WF_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const size_t img = (size_t)n_frames * nz * nx * 4;
    if (out_db != env && overlaps(out_db, img, env, img))
        return fail(WF_ERR_INVALID_ARG, "out_db partially overlaps env");
    if (overlaps(col_max, (size_t)n_frames * nx * 4, out_db, img))
        return fail(WF_ERR_INVALID_ARG, "col_max overlaps out_db");
    hipError_t e = wf::launch_log_compress(env, col_max, n_frames, nz, nx, dr_db,
                                           flags & WF_BMODE_OFFSET, out_db, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "log-compression kernel launch");
    return ok();
}

wf_status wf_bmode(const float* bf, int32_t n_frames, int32_t nz, int32_t nx, float dr_db,
                   int32_t flags, float* out_db, float* col_max, void* stream) {
    wf_status st = check_image(bf, n_frames, nz, nx, "bf");
    if (st != WF_OK) return st;
    if (!out_db) return fail(WF_ERR_INVALID_ARG, "out_db is NULL");
    const size_t img = (size_t)n_frames * nz * nx * 4;
    if (overlaps(out_db, img, bf, img)) return fail(WF_ERR_INVALID_ARG, "out_db overlaps bf");
    if (!std::isfinite(dr_db) || dr_db <= 0.0f)
        return fail(WF_ERR_INVALID_ARG, "dr_db must be > 0");
    if (flags & ~WF_BMODE_OFFSET) return fail(WF_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    st = wf_envelope(bf, n_frames, nz, nx, out_db, col_max, stream);
    if (st != WF_OK) return st;
    return wf_log_compress(out_db, col_max, n_frames, nz, nx, dr_db, flags, out_db, stream);
}

wf_status wf_fir(const void* rf, int32_t dtype, int64_t n_rec, int32_t n_s, const float* taps,
                 int32_t n_taps, float* out, void* stream) {
    if (!taps) return fail(WF_ERR_INVALID_ARG, "taps is NULL");
    if (dtype < WF_RF_I16 || dtype > WF_RF_F32)
        return fail(WF_ERR_INVALID_ARG, "dtype=%d is not a wf_rf_dtype", dtype);
    if (n_rec < 0) return fail(WF_ERR_INVALID_ARG, "n_rec=%lld is negative", (long long)n_rec);
    if (n_s <= 0 || n_s % 8 != 0)
        return fail(WF_ERR_UNSUPPORTED, "n_s=%d must be a positive multiple of 8", n_s);
    if (n_taps < 1 || n_taps > 63 || n_taps % 2 != 1)
        return fail(WF_ERR_UNSUPPORTED, "n_taps=%d must be odd, 1..63", n_taps);
    for (int k = 0; k < n_taps; ++k)
        if (!std::isfinite(taps[k])) return fail(WF_ERR_INVALID_ARG, "taps[%d] is not finite", k);
    if (n_rec == 0) return ok();  // nothing to filter; rf and out may be NULL
    if (!rf || !out) return fail(WF_ERR_INVALID_ARG, "rf and out must not be NULL");
    if (((uintptr_t)rf & 15) || ((uintptr_t)out & 15))
        return fail(WF_ERR_UNSUPPORTED, "rf and out must be 16-byte aligned");
    const size_t esz = dtype == WF_RF_F32 ? 4 : 2;
    if (n_rec > (1LL << 36) / n_s || n_rec * ((n_s + 2047) / 2048) > 0x7FFFFFFFLL)
        return fail(WF_ERR_INVALID_ARG, "RF too large");
    const long long total = (long long)n_rec * n_s;
    if (overlaps(rf, (size_t)total * esz, out, (size_t)total * 4))
        return fail(WF_ERR_INVALID_ARG, "out overlaps rf");
    wf::FirTaps h{};
    const int kp = n_taps <= 15 ? 15 : (n_taps <= 31 ? 31 : 63);
    const int pad = (kp - n_taps) / 2;
    for (int k = 0; k < n_taps; ++k) h.h[pad + k] = taps[k];
    hipError_t e = wf::launch_fir(dtype, rf, (long long)n_rec, n_s, kp, h, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "FIR kernel launch");
    return ok();
}

wf_status wf_moments(const float* env, int32_t n_frames, int32_t nz, int32_t nx, int32_t wz,
                     int32_t wx, int32_t sz, int32_t sx, float* out, void* stream) {
    wf_status st = check_image(env, n_frames, nz, nx, "env");
    if (st != WF_OK) return st;
    if (!out) return fail(WF_ERR_INVALID_ARG, "out is NULL");
    if (wz < 1 || wz > nz || wx < 1 || wx > nx)
        return fail(WF_ERR_INVALID_ARG, "window %dx%d does not fit the %dx%d frame", wz, wx, nz,
                    nx);
    if (sz < 1 || sx < 1) return fail(WF_ERR_INVALID_ARG, "strides must be >= 1");
    const int mz = (nz - wz) / sz + 1, mx = (nx - wx) / sx + 1;
    // column sums of one workgroup (64 window columns) live in LDS
    if (12.0 * ((double)(std::min(64, mx) - 1) * sx + wx) > 163840.0)
        return fail(WF_ERR_UNSUPPORTED, "63 x sx + wx = %lld columns exceed the LDS of a workgroup",
                    (long long)(std::min(64, mx) - 1) * sx + wx);
    if (overlaps(env, (size_t)n_frames * nz * nx * 4, out, (size_t)n_frames * 3 * mz * mx * 4))
        return fail(WF_ERR_INVALID_ARG, "out overlaps env");
    hipError_t e = wf::launch_moments(env, n_frames, nz, nx, wz, wx, sz, sx, mz, mx, out,
                                      (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "moments kernel launch");
    return ok();
}

wf_status wf_geometry_cache_clear(void) {
    GeometryCache& gc = cache();
    std::lock_guard<std::mutex> lk(gc.mu);
    hipError_t first = hipSuccess;
    for (auto& kv : gc.lru) {
        hipError_t e = free_uploads(kv.second);
        if (e != hipSuccess && first == hipSuccess) first = e;
    }
    gc.lru.clear();
    gc.index.clear();
    if (first != hipSuccess) return hip_fail(first, "hipFree(geometry table)");
    return ok();
}

}  // extern "C"
