/*
 * wf.h - C ABI of libwf: Delay-and-Sum beamforming (STAI and PWI), analytic-
 * signal envelope, and log compression with dynamic-range clipping into a
 * B-mode frame, on one AMD Instinct MI355X (gfx950).
 *
 * The pipeline is the B-mode reconstruction of the WaveFlow paper (arXiv
 * 1811.01566): Beamforming -> Analytic Signal -> Absolute Value -> Dynamic
 * Adjustment (Fig. 2), with DAS for synthetic transmit aperture (STAI) and
 * plane-wave (PWI) imaging as the mid-processing op (Sec. II-B), the
 * analytic signal formed with the FFT-based Hilbert transform (Sec. II-B),
 * and the frame clipped to a dB range (Sec. III).  The inputs follow the
 * paper's Ultrasound Environment (Sec. II-A): an RF tensor (acquisitions,
 * channels, samples) plus metadata - speed of sound, aperture, sampling
 * frequency.
 *
 * Conventions shared by every call (the paper gives no equations; these are
 * the readings the library implements):
 *  - Linear array on z = 0; element e at x_e = (e - (N-1)/2) * pitch unless
 *    an explicit host array of positions is given.  z is depth (> 0 into
 *    the medium).  Pixel (iz, ix) is at (x0 + ix*dx, z0 + iz*dz), metres.
 *  - Times of flight: receive |p - e_j| / c; STAI transmit t (one element
 *    e_t fires) |p - e_t| / c; PWI transmit k (angle theta_k, > 0 steers
 *    towards +x) (z cos theta_k + x sin theta_k + o_k) / c, with
 *    o_k = -min_e(x_e sin theta_k) (time zero when the first element fires)
 *    or o_k = 0 (time zero when the wavefront crosses x = 0).
 *  - Sample s of the record is taken at t0 + s/fs.  u = (tau_tx + tau_rx -
 *    t0) * fs; n = floor(u); the contribution is the linear interpolation
 *    (1-a) r[n] + a r[n+1], a = u - n, and 0 unless 0 <= n <= S-2.
 *  - Receive apodisation (f_number > 0): channel j counts for pixel p iff
 *    2 * f_number * |x - x_j| <= z.  No transmit apodisation, no
 *    normalisation; PWI compounding is the plain sum over angles.
 *  - Every array is dense, row-major, last index fastest.
 *
 * Memory and streams.  Pointers documented as DEVICE are HIP device
 * pointers on the current device; HOST pointers are read during the call
 * only.  Every compute call is asynchronous on `stream` (a hipStream_t
 * passed as void*, NULL = the null stream).  The caller owns every buffer:
 * RF, outputs, workspaces and the device memory of plans.
 *
 * Plans.  The DAS-shaped calls (wf_das_stai, wf_das_pwi, wf_das_dydc,
 * wf_das_adjoint) need a few KB of per-geometry device tables: the
 * per-transmit and per-channel delay constants and the work lists of the
 * launches (the adjoint may run its own tiles and work list).  With a plan (wf_plan_build_*) they live in caller-owned device
 * memory and the call neither allocates nor synchronises: it only launches
 * kernels on `stream`, so it may be captured into a HIP graph even for a
 * geometry never run before.  With plan = NULL the library keeps the tables
 * in a cache of its own: the first call of a geometry on a device
 * allocates them (hipMalloc), writes them on `stream` and synchronises
 * `stream`; the cache holds at most 64 geometries and at most 4 GiB of
 * device memory, gives an entry the delay tables of WF_PLAN_DELAY_TABLES
 * when they take at most 512 MiB, and evicting the least recently used
 * entry synchronises its device before freeing it.  Such calls
 * must not be captured into graphs (a graph would keep pointers the cache
 * may free); calls without a plan are serialised by a library lock from
 * the table lookup to their last launch.
 *
 * Errors.  Every call validates all arguments before touching the device
 * and returns a negative wf_status with a message from wf_last_error() on
 * failure; nothing is launched then.  Faults inside kernels surface at the
 * caller's next synchronisation.  Calls are re-entrant; the error string is
 * per thread.
 */
#ifndef WF_H
#define WF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WF_ABI_VERSION 8

typedef enum {
    WF_OK = 0,
    WF_ERR_INVALID_ARG = -1, /* a null pointer, a size or value out of range */
    WF_ERR_UNSUPPORTED = -2, /* valid, but outside what the kernels handle  */
    WF_ERR_DEVICE = -3,      /* a HIP runtime call failed                   */
    WF_ERR_WORKSPACE = -4    /* the caller's workspace is too small          */
} wf_status;

typedef enum {
    WF_RF_I16 = 0, /* int16 ADC counts                                    */
    WF_RF_F16 = 1, /* IEEE half                                           */
    WF_RF_F32 = 2  /* float                                               */
} wf_rf_dtype;

/* Opaque host handle of a plan: the launch plan of one geometry (tile
 * shape, work split) and the location of its device tables in caller
 * memory.  Created by wf_plan_build_*, freed by wf_plan_destroy. */
typedef struct wf_plan wf_plan;

typedef enum {
    WF_PWI_TREF_FIRST = 0, /* time zero: the first element fires          */
    WF_PWI_TREF_CENTRE = 1 /* time zero: the wavefront crosses x = 0      */
} wf_pwi_tref;

#define WF_BMODE_OFFSET 1 /* add dr_db so the output spans [0, dr_db] */

typedef struct {
    int32_t n_elem;       /* number of array elements, 1..4096              */
    double pitch;         /* element spacing (m), used when elem_x is NULL  */
    const double* elem_x; /* HOST [n_elem] lateral positions (m), or NULL   */
} wf_probe;

typedef struct {
    int32_t nz, nx;       /* pixels along depth and laterally              */
    double z0, dz;        /* depth of row 0 and row step (m)               */
    double x0, dx;        /* lateral position of column 0 and step (m)     */
} wf_grid;

typedef struct {
    int32_t n_frames;     /* F >= 1 frames sharing the geometry            */
    int32_t n_tx;         /* T, 1..1024 transmits per frame                */
    int32_t n_ch;         /* C, 1..1024 receive channels                   */
    int32_t n_s;          /* S, 16..32768 samples per record, S % 8 == 0   */
    int32_t dtype;        /* wf_rf_dtype of the RF samples                 */
    double c;             /* speed of sound (m/s), > 0                     */
    double fs;            /* sampling frequency (Hz), > 0                  */
    double t0;            /* time of sample 0 (s)                          */
    double f_number;      /* receive f-number; 0 disables apodisation      */
    const int32_t* rx_elem; /* HOST [n_ch] element of each channel, NULL = j */
} wf_acq;

/*
 * DAS for synthetic transmit aperture imaging (Sec. II-B; evaluation shape
 * (acquisitions, channels, samples), Sec. III).  Transmit t fires the single
 * element tx_elem[t] (HOST [n_tx], NULL = t); the sum runs over transmits
 * and receive channels.
 *   rf         DEVICE [F][T][C][S] of acq->dtype, 16-byte aligned.
 *   out        DEVICE float [F][nz][nx] beamformed RF (real, not IQ); must
 *              not overlap rf.
 *   workspace  optional DEVICE scratch, caller-owned, 4-byte aligned, not
 *              overlapping rf or out.  When it holds at least the bytes
 *              wf_das_workspace reports (> 0 for grids with too few tiles
 *              or too uneven work per tile to balance the GPU), each tile
 *              is split into items (channel chunks x transmit ranges) run
 *              by separate workgroups, whose partial frames are then summed
 *              in a fixed order; otherwise (NULL, or fewer bytes) the call
 *              runs unsplit.  Both are deterministic; they differ only in
 *              the order of the FP32 sums.  The split depends on the
 *              geometry only, never on n_frames.
 *   plan       NULL, or a plan built for exactly this geometry (every
 *              field of probe, acq and grid except n_frames and dtype, and
 *              tx_elem) on the current device; a plan built for another
 *              geometry gives WF_ERR_INVALID_ARG.
 * Returns WF_ERR_UNSUPPORTED when the pixel spacing is so coarse that no
 * tile shape keeps a tile's delay spread inside the kernel's window.
 */
wf_status wf_das_stai(const void* rf, const wf_probe* probe, const wf_acq* acq,
                      const int32_t* tx_elem, const wf_grid* grid, const wf_plan* plan,
                      float* out, void* workspace, uint64_t workspace_bytes, void* stream);

/*
 * DAS for plane-wave imaging with coherent compounding over angles
 * (Sec. II-B).  angles_rad: HOST [n_tx] steering angles, |theta| < 80 deg.
 * tref: wf_pwi_tref.  rf, out, workspace and plan as for wf_das_stai (the
 * plan built for these angles and tref).
 */
wf_status wf_das_pwi(const void* rf, const wf_probe* probe, const wf_acq* acq,
                     const double* angles_rad, int32_t tref, const wf_grid* grid,
                     const wf_plan* plan, float* out, void* workspace,
                     uint64_t workspace_bytes, void* stream);

/*
 * DAS (mode 0 = STAI with tx_elem, 1 = PWI with angles_rad and tref) that
 * allocates nothing: for callers that cannot call hipMalloc or have the
 * library do so - code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  rf, out and the geometry arguments are
 * those of wf_das_stai / wf_das_pwi; the result equals theirs to FP32
 * rounding (the same kernels; a grid that splits its tiles sums partial
 * frames in the same order when they fit, see below).
 *   Scratch: the geometry tables and the split's partial frames live in one
 *   static device array of WF_NOALLOC_SCRATCH_BYTES on each GPU the library
 *   runs on, held until the process ends.  Each call writes the tables on
 *   `stream` before its DAS launch (kernel stores, no memset); partial
 *   frames that do not fit beside them make the call run unsplit.
 *   Geometries whose tables exceed the array give WF_ERR_UNSUPPORTED.
 *   Every call on a GPU shares that GPU's array and leaves its contents for
 *   the next: calls that overlap on one GPU (different streams, or threads
 *   without ordering) race and must be serialised by the caller.
 *   Host: the launch plan comes from a small host-memory cache (16
 *   geometries); the call allocates no device memory, frees none and never
 *   synchronises.
 */
#define WF_NOALLOC_SCRATCH_BYTES (16u << 20)
wf_status wf_das_noalloc(int32_t mode, const void* rf, const wf_probe* probe,
                         const wf_acq* acq, const int32_t* tx_elem, const double* angles_rad,
                         int32_t tref, const wf_grid* grid, float* out, void* stream);

/*
 * Bytes of the optional workspace of wf_das_stai / wf_das_pwi / wf_das_dydc
 * for this geometry and acq->n_frames (0: the calls never split).  Host
 * only.  mode 0 = STAI (tx_elem), 1 = PWI (angles_rad, tref).
 */
wf_status wf_das_workspace(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                           const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                           const wf_grid* grid, uint64_t* bytes);

/*
 * One-way times of flight in samples as computed on the device (float-float
 * FP32 arithmetic), for testing the delay geometry of the DAS calls.
 *   tx_hi, tx_lo  DEVICE float [T][nz][nx]: (tau_tx - t0) * fs = hi + lo
 *   rx_hi, rx_lo  DEVICE float [C][nz][nx]: tau_rx * fs = hi + lo
 * For PWI pass angles_rad/tref, for STAI tx_elem; mode 0 = STAI, 1 = PWI.
 * acq->n_frames, n_s and dtype are ignored.  A verification call: it
 * allocates a temporary table, writes it on `stream`, and synchronises
 * `stream` before freeing it.
 */
wf_status wf_delays(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                    const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                    const wf_grid* grid, float* tx_hi, float* tx_lo, float* rx_hi,
                    float* rx_lo, void* stream);

/*
 * Envelope = |analytic signal| along depth of every column (Fig. 2:
 * Analytic Signal -> Absolute Value; Hilbert transform by FFT, Sec. II-B):
 * an nz-point FFT, the one-sided multiplier (1, 2, ..., 2, 1, 0, ..., 0),
 * an inverse FFT, the modulus.  nz must be a power of two, 2..4096.
 *   bf       DEVICE float [F][nz][nx] beamformed RF.
 *   env      DEVICE float [F][nz][nx]; may be the same buffer as bf.
 *   col_max  DEVICE float [F][nx]: the maximum envelope of each column.
 */
wf_status wf_envelope(const float* bf, int32_t n_frames, int32_t nz, int32_t nx,
                      float* env, float* col_max, void* stream);

/*
 * Log compression and clip (Fig. 2 "Dynamic Adjustment"; [0, DR] dB range,
 * Sec. III): B = 20 log10(env / m_f) clipped to [-dr_db, 0], m_f the frame
 * maximum (the maximum of col_max[f][:]); env = 0 or m_f = 0 gives -dr_db;
 * flags & WF_BMODE_OFFSET adds dr_db.
 *   env      DEVICE float [F][nz][nx] (>= 0).
 *   col_max  DEVICE float [F][nx] as written by wf_envelope.
 *   out_db   DEVICE float [F][nz][nx]; may be the same buffer as env.
 */
wf_status wf_log_compress(const float* env, const float* col_max, int32_t n_frames,
                          int32_t nz, int32_t nx, float dr_db, int32_t flags,
                          float* out_db, void* stream);

/*
 * Beamformed RF -> B-mode frame: wf_envelope into out_db, then
 * wf_log_compress in place.  col_max: DEVICE float [F][nx] scratch.
 * out_db must not overlap bf.
 */
wf_status wf_bmode(const float* bf, int32_t n_frames, int32_t nz, int32_t nx,
                   float dr_db, int32_t flags, float* out_db, float* col_max,
                   void* stream);

/*
 * Forward-mode derivative of DAS w.r.t. the speed of sound c, per pixel.
 * Every time of flight is a path length over c, so du/dc = -(u + t0 fs) / c
 * for the fractional sample index u, and (almost everywhere: away from the
 * integer crossings of u, where the linear interpolant has a kink)
 *   dy(p)/dc = sum_{t,j} w_j(p) (r[n+1] - r[n]) du/dc.
 * The beamformer sits in a trainable graph in the paper (Sec. I; Sec. IV);
 * this is the derivative that lets c be learned.
 *   rf    DEVICE [F][T][C][S] as for the DAS calls.
 *   dydc  DEVICE float [F][nz][nx].
 *   plan, workspace, workspace_bytes  as for wf_das_stai.
 * mode 0 = STAI (tx_elem), 1 = PWI (angles_rad, tref).
 */
wf_status wf_das_dydc(int32_t mode, const void* rf, const wf_probe* probe, const wf_acq* acq,
                      const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                      const wf_grid* grid, const wf_plan* plan, float* dydc, void* workspace,
                      uint64_t workspace_bytes, void* stream);

/*
 * Adjoint of DAS w.r.t. the RF (the transpose of the interpolating gather):
 * for a cotangent g, grad_rf[t][j][m] = sum_p w_j(p) g(p) ((1-a)[m = n] +
 * a [m = n+1]) over pairs with 0 <= n <= S-2.  The beamformer sits in a
 * trainable graph in the paper (Sec. I; Sec. IV); this is the gradient that
 * flows back to the RF.  grad_rf is overwritten (every sample written once).
 *   g          DEVICE float [F][nz][nx].
 *   grad_rf    DEVICE float [F][T][C][S]; acq->dtype must be WF_RF_F32.
 *   workspace  DEVICE, 256-byte aligned, >= the bytes wf_das_adjoint_workspace
 *              reports (it holds one frame's per-tile windows; frames run one
 *              after another on `stream`); caller-owned, contents ignored.
 *   plan       as for wf_das_stai.
 * Per-tile windows are accumulated in LDS as 64-bit fixed point (the
 * cotangent rounded once per pixel to 24 bits of its frame's largest |g|)
 * and then summed in a fixed tile order without global atomics: the
 * result is bitwise reproducible.  Returns WF_ERR_WORKSPACE if the
 * workspace is too small.  mode 0 = STAI (tx_elem), 1 = PWI (angles_rad,
 * tref).
 */
wf_status wf_das_adjoint(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                         const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                         const wf_grid* grid, const wf_plan* plan, const float* g,
                         float* grad_rf, void* workspace, uint64_t workspace_bytes,
                         void* stream);

/*
 * Device bytes of the workspace wf_das_adjoint needs for this geometry (one
 * frame; acq->n_frames is ignored).  Host only.
 */
wf_status wf_das_adjoint_workspace(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                                   const int32_t* tx_elem, const double* angles_rad,
                                   int32_t tref, const wf_grid* grid, uint64_t* bytes);

/*
 * out[0] = sum_i a[i] b[i] (DEVICE pointers, n elements; compensated sums in
 * a fixed order: deterministic).  With a = dL/dy and b = dy/dc it gives
 * dL/dc.
 */
wf_status wf_dot(const float* a, const float* b, int64_t n, float* out, void* stream);

/*
 * Launch plan the DAS calls would use for this geometry (host only; touches
 * no device).  info (HOST int32[20]) receives: pixels per lane, tile depth,
 * tile width, window-local delay clamp (samples), staged window entries,
 * LDS entries per window, LDS bytes per workgroup of wf_das (twice the
 * window buffers where it stages two passes per barrier), tiles along z, tiles
 * along x, channels per pass, threads per workgroup, then the work split
 * used when the caller passes wf_das_workspace's bytes: items per tile,
 * channel chunks per item, transmit splits, transmits per item, and the
 * workgroups launched per frame (items that run no pass are left out);
 * then the adjoint's launch (wf_das_adjoint runs its own tiles where the
 * gather's are smaller than 1024 threads): threads per workgroup, pixels
 * per lane, tile depth, items per tile.
 * mode 0 = STAI, 1 = PWI.  Returns WF_ERR_UNSUPPORTED when no tile shape
 * fits (as the DAS calls would).
 */
wf_status wf_das_tile_info(int32_t mode, const wf_probe* probe, const wf_acq* acq,
                           const int32_t* tx_elem, const double* angles_rad, int32_t tref,
                           const wf_grid* grid, int32_t* info);

/*
 * FIR pre-filter along samples (the pre-processing op of Sec. II-B): every
 * record of n_s samples is filtered on its own,
 *   out[s] = sum_k taps[k] in[s + D - k],  D = (n_taps - 1) / 2,
 * with in = 0 outside the record, so an odd-length linear-phase filter adds
 * no delay and the DAS time origin is unchanged.
 *   rf      DEVICE [n_rec][n_s] of dtype (wf_rf_dtype; int16 and FP16
 *           convert exactly), 16-byte aligned, n_s % 8 == 0; finite values.
 *   taps    HOST float [n_taps], n_taps odd, 1..63; read during the call.
 *   out     DEVICE float [n_rec][n_s], 16-byte aligned, must not overlap rf.
 * n_rec = 0 does nothing (rf and out may then be NULL).
 * FP32 fused multiply-adds in tap order.  With rf = RF [F][T][C][S] and
 * n_rec = F T C the output is RF for the DAS calls with dtype WF_RF_F32.
 */
wf_status wf_fir(const void* rf, int32_t dtype, int64_t n_rec, int32_t n_s, const float* taps,
                 int32_t n_taps, float* out, void* stream);

/*
 * Windowed moments of the envelope (the qUS estimator's inputs, Fig. 3:
 * slice -> E[X], E[X^2], E[X^3]): windows of wz x wx samples at origins
 * (i sz, j sx), whole windows only, mz = (nz - wz) / sz + 1 and
 * mx = (nx - wx) / sx + 1; E[X^p] is the mean of env^p over the window.
 *   env  DEVICE float [F][nz][nx] (the linear envelope, e.g. wf_envelope's).
 *   out  DEVICE float [F][3][mz][mx] (p = 1, 2, 3); must not overlap env.
 * 1 <= wz <= nz, 1 <= wx <= nx, sz, sx >= 1; WF_ERR_UNSUPPORTED when
 * 12 ((min(64, mx) - 1) sx + wx) exceeds 160 KB (the column sums of 64
 * windows are kept in LDS).  Deterministic.
 */
wf_status wf_moments(const float* env, int32_t n_frames, int32_t nz, int32_t nx, int32_t wz,
                     int32_t wx, int32_t sz, int32_t sx, float* out, void* stream);

/*
 * Plans (the acquisition metadata of Sec. II-A - speed of sound, aperture,
 * sampling frequency - with the transmit sequence and the pixel grid fix
 * every delay table and the launch plan of the DAS calls).
 *
 * wf_plan_bytes_stai / wf_plan_bytes_pwi: device bytes of the plan of this
 * geometry built with `flags` (host only, touches no device).
 * acq->n_frames and acq->dtype must be valid but do not enter the plan.
 *
 * flags: 0 or WF_PLAN_DELAY_TABLES.  With it the plan also holds the
 * window-local fixed-point delays the gathers use (Sec. II-B: the time of
 * flight of every pixel to every receive element and of every transmit,
 * from its element (STAI) or its plane wave (PWI)), formed once on the
 * device at build time: 4 bytes per (pixel slot, channel) and per (pixel
 * slot, transmit); the transmit words are left out for PWI on the 1024-
 * thread, 2-pixel tiles, whose gather forms them faster - 256 MiB for 128
 * channels on a 1024 x 512 PWI grid.  The DAS and d y / d c gathers then
 * read those words instead of forming them, with bitwise the same results.
 * Other flag bits are refused (WF_ERR_INVALID_ARG).
 *
 * wf_plan_build_stai / wf_plan_build_pwi: computes the launch plan on the
 * host and writes the device tables into dev_mem (DEVICE, caller-owned,
 * 256-byte aligned, >= the bytes wf_plan_bytes_* reports) with kernel
 * launches on `stream`; returns the host handle in *out.  It sets the
 * dynamic-LDS limit of the kernels the plan can launch on the current
 * device (once per process) and allocates only the host handle.  The plan
 * is valid on the current device for calls ordered after the build on
 * `stream` (another stream must wait for it, e.g. through an event).
 * dev_mem must stay allocated and unmodified while calls using the plan
 * may run, graph replays included.  WF_ERR_WORKSPACE when bytes is too
 * small; nothing is written then.
 *
 * wf_plan_destroy frees the host handle only (NULL is ignored); the device
 * memory stays the caller's.  Work already enqueued with the plan keeps
 * reading dev_mem, not the handle.
 */
#define WF_PLAN_DELAY_TABLES 1
wf_status wf_plan_bytes_stai(const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                             const wf_grid* grid, int32_t flags, uint64_t* bytes);
wf_status wf_plan_bytes_pwi(const wf_probe* probe, const wf_acq* acq, const double* angles_rad,
                            int32_t tref, const wf_grid* grid, int32_t flags, uint64_t* bytes);
wf_status wf_plan_build_stai(const wf_probe* probe, const wf_acq* acq, const int32_t* tx_elem,
                             const wf_grid* grid, int32_t flags, void* dev_mem, uint64_t bytes,
                             wf_plan** out, void* stream);
wf_status wf_plan_build_pwi(const wf_probe* probe, const wf_acq* acq, const double* angles_rad,
                            int32_t tref, const wf_grid* grid, int32_t flags, void* dev_mem,
                            uint64_t bytes, wf_plan** out, void* stream);
void wf_plan_destroy(wf_plan* plan);

/* Workspace bytes of calls made with `plan` (host only): the DAS / d y / d c
 * split workspace for n_frames frames (0: the plan never splits; see
 * wf_das_stai) and the adjoint workspace (one frame; see wf_das_adjoint). */
wf_status wf_plan_workspace(const wf_plan* plan, int32_t n_frames, uint64_t* das_bytes,
                            uint64_t* adjoint_bytes);

/* Message of the last failed call on this thread ("" after success). */
const char* wf_last_error(void);

/* WF_ABI_VERSION of the loaded library. */
int32_t wf_abi_version(void);

/* Free the library's cache of the calls made without a plan: host plans
 * and device tables on every device (each device is synchronised first).
 * Plans are not affected. */
wf_status wf_geometry_cache_clear(void);

/* Geometries held by that cache and the device bytes of their tables. */
wf_status wf_geometry_cache_info(uint64_t* entries, uint64_t* device_bytes);

#ifdef __cplusplus
}
#endif

#endif /* WF_H */
