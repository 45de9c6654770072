/*
 * simradar.h - C ABI of the MI355X fast-mode radar simulator.
 *
 * Implements the fast simulation mode of Monnier, Camus and Hellouvry,
 * "High Performance Simulation of Spaceborne Radar for Remote-Sensing
 * Oceanography" (arXiv 2408.11472), Sec. III:
 *
 *   for every update j (one every n_fast pulses) the sea surface is
 *   regenerated at the two pulses of a pair, every illuminated facet becomes
 *   a complex scatterer whose pulse-pair phase step gives its Doppler, and
 *   the scatterers are summed per (range gate, Doppler bin) into the Doppler
 *   spectrum tensor T_fast (Algorithm 1); post-processing inverse-FFTs every
 *   gate spectrum, weights the long-time signals with eq. (1) and sums them
 *   into the range-azimuth IQ matrix Y (Sec. III.B, steps 1-4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All data pointers are DEVICE pointers owned by the caller.  The library
 *    allocates no device memory: its twiddle tables are static arrays of the
 *    code object (one copy per device), filled by the first sim_create on
 *    each device.  Scratch memory (surface transform planes, per-band partial
 *    spectra) is caller-provided through sim_set_workspace.  No compute call
 *    creates HIP objects (the profiling events are made by
 *    sim_profile_enable).
 *  - Every compute call is asynchronous on the HIP stream passed as `stream`
 *    (NULL = the default stream).  Argument and shape checks are synchronous
 *    and return a status; nothing is launched when a check fails.  A launch
 *    failure returns SIM_ERR_DEVICE.  No C++ exception crosses the ABI.
 *  - Precision is fixed per context.  SIM_PREC_FP64: every real is double,
 *    every complex is two doubles (re, im).  SIM_PREC_FP32_PHASE64: facet
 *    fields are float, complex arrays are two floats; the satellite-facet
 *    range, gate, Doppler bin and carrier phase are nevertheless computed in
 *    double on the GPU (4 pi R / lambda at ~815 km in Ku band has no phase
 *    left in float).
 *  - Grid sides are powers of two: 16 <= nx <= 8192, 16 <= ny <= 16384
 *    (ny <= 8192 in FP64).
 *    Doppler bins n_doppler: power of two, 2 <= n_doppler <= 2048.
 *  - Calls that run concurrently on one context race on its workspace.
 */
#ifndef SIMRADAR_H
#define SIMRADAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_ABI_VERSION 3

typedef enum sim_status {
  SIM_OK = 0,
  SIM_ERR_ARG = 1,          /* null pointer, non-finite or out-of-range scalar */
  SIM_ERR_SHAPE = 2,        /* inconsistent sizes or index out of range        */
  SIM_ERR_UNSUPPORTED = 3,  /* size outside the supported set                  */
  SIM_ERR_WORKSPACE = 4,    /* no workspace attached, or too small             */
  SIM_ERR_DEVICE = 5        /* HIP runtime or launch failure                   */
} sim_status;

typedef enum sim_precision {
  SIM_PREC_FP64 = 0,
  SIM_PREC_FP32_PHASE64 = 1
} sim_precision;

/* Cross-fade of the long-time signals (Sec. III.A).  SQRT_TRIANGLE is
 * eq. (1), W(d) = sqrt(1 - |d|/n_fast); SQRT_RAISED_COSINE is
 * W(d) = cos(pi d / (2 n_fast)).  Both keep sum_j W^2 = 1 at every pulse. */
typedef enum sim_window {
  SIM_WIN_SQRT_TRIANGLE = 0,
  SIM_WIN_SQRT_RAISED_COSINE = 1
} sim_window;

/* Facet grid (Sec. II.B: the scene is a set of facets).  Facet (ix, iy) has
 * Lagrangian position (x_origin + ix dx, y_origin + iy dy); spectral phases
 * are referenced to facet (0, 0).  cwm != 0 switches on the Choppy Wave Model
 * horizontal displacement (Sec. II.A). */
typedef struct sim_grid {
  int32_t nx, ny;
  int32_t cwm;
  int32_t reserved;
  double dx, dy;              /* facet spacing [m], > 0            */
  double x_origin, y_origin;  /* position of facet (0, 0) [m]      */
  double gravity;             /* deep-water dispersion w^2 = g |k| */
} sim_grid;

/* Nadir radar on a straight track along +y at constant altitude; the
 * platform is at (sat_x, sat_y0 + velocity t, altitude) at time t.
 * The range window starts at window_start and has n_gates gates of
 * gate_spacing.  beamwidth_3db, fresnel_sq (|Gamma(0)|^2) and mss (slope
 * variance of the unresolved scales) set the closed-form beam and the
 * geometric-optics NRCS that stand in for the paper's look-up tables
 * (Sec. II.A). */
typedef struct sim_radar {
  double altitude;
  double velocity;
  double sat_x, sat_y0;
  double carrier_hz;
  double prf_hz;
  double gate_spacing;
  double window_start;
  double beamwidth_3db;       /* [rad] */
  double fresnel_sq;
  double mss;
  int32_t n_gates;            /* G >= 1                            */
  int32_t n_doppler;          /* N, power of two                   */
  int32_t n_fast;             /* pulses between surface updates >= 1 */
  int32_t window;             /* sim_window                        */
} sim_radar;

/* Facet set, structure of arrays, each [ny][nx] row-major, float or double
 * by context precision:
 *   disp_x, disp_y, h       position of the facet relative to its grid point
 *   sx, sy                  slopes -n_x/n_z, -n_y/n_z of the facet normal n
 *   jac                     n_z (the Lagrangian Jacobian; <= 0: folded facet)
 *   ddisp_x, ddisp_y, dh    displacement of the facet over the pulse pair   */
typedef struct sim_facets {
  void *disp_x, *disp_y, *h, *sx, *sy, *jac, *ddisp_x, *ddisp_y, *dh;
} sim_facets;

/* Facet counters (device memory, accumulated with +=).  Every facet lands
 * in exactly one of the first five; window_overflow counts partial-spectrum
 * flushes that exceeded the per-band slots and were merged with atomics. */
typedef struct sim_counters {
  uint64_t illuminated;
  uint64_t out_of_window;
  uint64_t folded;
  uint64_t backfacing;
  uint64_t nonfinite;
  uint64_t window_overflow;
} sim_counters;

/* Per-facet code written by the accumulate calls when facet_code != NULL:
 * g * n_doppler + bin for an illuminated facet, else one of these. */
#define SIM_CODE_NONFINITE (-1)
#define SIM_CODE_FOLDED (-2)
#define SIM_CODE_OUT_OF_WINDOW (-3)
#define SIM_CODE_BACKFACING (-4)

typedef struct sim_ctx sim_ctx;

/* ABI version of the loaded library (SIM_ABI_VERSION). */
int sim_abi_version(void);

/* Static text of a status code. */
const char *sim_status_string(sim_status status);

/* Create a context on HIP device `device` (made current) with the given
 * precision.  The first call on a device resolves the device addresses of
 * the library's static tables and fills the twiddles (a synchronous copy).
 * *ctx is NULL on failure. */
sim_status sim_create(sim_ctx **ctx, int device, sim_precision precision);

/* Release the context (and its profiling events).  NULL is accepted. */
sim_status sim_destroy(sim_ctx *ctx);

/* Precision of a context. */
sim_status sim_get_precision(const sim_ctx *ctx, sim_precision *precision);

/* Bytes of workspace needed by every call below for this grid and radar. */
sim_status sim_workspace_size(const sim_ctx *ctx, const sim_grid *grid,
                              const sim_radar *radar, size_t *bytes);

/* Attach caller-owned device memory as workspace (256-byte aligned).
 * The context keeps the pointer until the next call; bytes = 0 detaches. */
sim_status sim_set_workspace(sim_ctx *ctx, void *device_ptr, size_t bytes);

/* update_simulation(t) of Algorithm 1 for a pulse pair: synthesise the CWM
 * surface at time t from the initial spectral coefficients and write the
 * facet set, including its displacement between t and t + dt_pair (the
 * second pulse of the pair, dt_pair = 1/PRF).
 *   spec0  [ny][nx] complex, FFT order (index ix is wavenumber
 *          kx = 2 pi n / (nx dx) with n = ix for ix < nx/2, ix - nx otherwise;
 *          same in y).  The surface is h = Re sum c(k) exp(i(k.x - w t)),
 *          w = sqrt(g |k|); the zero mode and the Nyquist row and column are
 *          ignored.  Read only.
 *   out    facet SoA, written. */
sim_status sim_surface_update(sim_ctx *ctx, const sim_grid *grid,
                              const void *spec0, double t, double dt_pair,
                              const sim_facets *out, void *stream);

/* scatterers_complex_amplitudes(), scatterers_range(), the pulse-pair
 * Doppler and rasterize() of Algorithm 1 for spectrum j: every facet of
 * `facets` (state at pulse time t; second pulse at t + 1/PRF) is turned
 * into C = a exp(-i 4 pi R / lambda), its gate floor((R - window_start) /
 * gate_spacing) and Doppler bin floor(N u + 1/2) mod N with u the
 * pulse-pair phase step in cycles wrapped to [-1/2, 1/2), and
 * t_fast[j][g][bin] += C.
 *   t_fast      [n_spec][n_gates][n_doppler] complex, accumulated (never
 *               cleared); Doppler bin 0 is zero Doppler (FFT order).
 *   counters    device sim_counters, accumulated; may be NULL.
 *   facet_code  [ny][nx] int32, written; may be NULL. */
sim_status sim_range_doppler_accumulate(sim_ctx *ctx, const sim_grid *grid,
                                        const sim_facets *facets,
                                        const sim_radar *radar, double t,
                                        int32_t j, void *t_fast, int32_t n_spec,
                                        sim_counters *counters,
                                        int32_t *facet_code, void *stream);

/* sim_range_doppler_accumulate for callers that cannot allocate device memory
 * or attach a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, same results up to the
 * summation order of the partial spectra; no workspace is needed, and the
 * call allocates nothing: the band windows, their headers and the band
 * counters live in a static device array of the library (32 MiB + 24 KiB per
 * device, held until the process ends), which bounds the facet accumulate to
 * 256 bands of 4 windows of at most 32 KiB.  Every supported size fits;
 * anything beyond that bound returns SIM_ERR_WORKSPACE before launching.
 * All calls of this entry point on one device share that array, so calls
 * that overlap on one GPU (concurrent streams, several contexts or threads)
 * race and must be serialised by the caller. */
sim_status sim_range_doppler_accumulate_noalloc(sim_ctx *ctx, const sim_grid *grid,
                                                const sim_facets *facets,
                                                const sim_radar *radar, double t,
                                                int32_t j, void *t_fast, int32_t n_spec,
                                                sim_counters *counters,
                                                int32_t *facet_code, void *stream);

/* sim_surface_update followed by sim_range_doppler_accumulate for the pulse
 * pair (t, t + 1/PRF).  On the fused row path (SIM_TUNE_ROW_PATH) the facet
 * set is never written to memory; on the split path it goes through the
 * workspace.  Either way the result is that of the two calls (up to the
 * summation order of the partial spectra). */
sim_status sim_update_and_accumulate(sim_ctx *ctx, const sim_grid *grid,
                                     const void *spec0, const sim_radar *radar,
                                     double t, int32_t j, void *t_fast,
                                     int32_t n_spec, sim_counters *counters,
                                     int32_t *facet_code, void *stream);

/* The spectrum in the layout the surface transform's first (column) pass
 * reads: the pass works on the columns kx >= 0 only (the surface fields are
 * real), and for each strip of adjacent columns it works on, rows in order,
 * the buffer holds the pair (c(k), c(-k)) of every column of the strip, so
 * that each update reads it contiguously.  Same content as the FFT-order
 * spectrum (Sec. II.A: the surface is synthesised from it at every update);
 * made once per run.
 *   spec0     [ny][nx] complex, FFT order, read only.
 *   prepared  caller-owned device buffer of sim_prepared_spectrum_size bytes,
 *             16-byte aligned, written; its layout depends on grid and
 *             precision only. */
sim_status sim_prepared_spectrum_size(const sim_ctx *ctx, const sim_grid *grid,
                                      size_t *bytes);
sim_status sim_prepare_spectrum(sim_ctx *ctx, const sim_grid *grid, const void *spec0,
                                void *prepared, void *stream);

/* sim_update_and_accumulate from a prepared spectrum (identical results). */
sim_status sim_update_and_accumulate_prepared(sim_ctx *ctx, const sim_grid *grid,
                                              const void *prepared, const sim_radar *radar,
                                              double t, int32_t j, void *t_fast,
                                              int32_t n_spec, sim_counters *counters,
                                              int32_t *facet_code, void *stream);

/* Post-processing of Sec. III.B: s_j[g][m] = sum_k T[j][g][k]
 * exp(+2 pi i k m / N) (unnormalised), then for every pulse x in
 * [0, (n_spec - 1) n_fast):
 *   y[x][g] = sum over j in {floor(x/n_fast), floor(x/n_fast) + 1} of
 *             W(x - j n_fast) s_j[g][(x - j n_fast) mod N].
 *   t_fast  [n_spec][n_gates][n_doppler] complex, read only, n_spec >= 2.
 *   y       [(n_spec - 1) n_fast][n_gates] complex, written. */
sim_status sim_segments_to_iq(sim_ctx *ctx, const sim_radar *radar,
                              const void *t_fast, int32_t n_spec, void *y,
                              void *stream);

/* ---- differentiable chain ------------------------------------------------
 * Gradients of a multi-look waveform loss (the echoes are multi-looked before
 * retracking in Sec. IV.B; the inversion of sea-state parameters motivates
 * the gradient, Sec. V) with respect to the facet heights and slopes of every
 * update.  Gate and bin indices are piecewise constant and get no gradient;
 * the other facet fields are held fixed.  Complex gradients follow the
 * convention dL/dRe + i dL/dIm.  Reals are float or double by context. */

/* p[g] = (1/n_pulses) sum_x |y[x][g]|^2 (written); when loss != NULL also
 * loss[0] = sum_g (p[g] - target[g])^2 (target [n_gates], read only).
 *   y  [n_pulses][n_gates] complex. */
sim_status sim_waveform_loss(sim_ctx *ctx, const sim_radar *radar, const void *y,
                             int32_t n_pulses, const void *target, void *p, void *loss,
                             void *stream);

/* y_bar[x][g] = s * 2 (p[g] - target[g]) * 2 y[x][g] / n_pulses, the gradient
 * of the loss above times s = scale[0] (a device scalar; NULL means 1). */
sim_status sim_waveform_loss_adjoint(sim_ctx *ctx, const sim_radar *radar, const void *y,
                                     int32_t n_pulses, const void *p, const void *target,
                                     const void *scale, void *y_bar, void *stream);

/* Adjoint of sim_segments_to_iq:
 * t_fast_bar[j][g][k] = sum_x W(x - j n_fast) y_bar[x][g]
 *                       exp(-2 pi i k ((x - j n_fast) mod N) / N)
 * over the pulses x in [0, (n_spec - 1) n_fast) with |x - j n_fast| < n_fast.
 * Written, [n_spec][n_gates][n_doppler] complex. */
sim_status sim_segments_to_iq_adjoint(sim_ctx *ctx, const sim_radar *radar, const void *y_bar,
                                      int32_t n_spec, void *t_fast_bar, void *stream);

/* Adjoint of sim_range_doppler_accumulate for update j: every illuminated
 * facet's scatterer is recomputed from `facets` (nothing was stored) and
 *   grad_theta = Re(conj(t_fast_bar[j][g][bin]) dC/dtheta), theta = h, sx, sy;
 * dropped facets get 0.  grad_h, grad_sx, grad_sy: [ny][nx] real, written. */
sim_status sim_range_doppler_accumulate_adjoint(sim_ctx *ctx, const sim_grid *grid,
                                                const sim_facets *facets,
                                                const sim_radar *radar, double t, int32_t j,
                                                const void *t_fast_bar, int32_t n_spec,
                                                void *grad_h, void *grad_sx, void *grad_sy,
                                                void *stream);

/* ---- batches of independent realisations --------------------------------
 * The paper averages spectra over ~100 realisations of the acquisition
 * (Sec. I, Sec. IV.D).  A batch holds R realisations with their own grid
 * (sides may differ), radar and update count; running it performs Algorithm 1
 * and the post-processing for every realisation, update-major
 * (update j of every realisation, then j + 1), on one stream.  The work can be
 * captured once into a HIP graph and replayed with a single launch per run.
 * The context's workspace must cover the largest realisation
 * (sim_batch_workspace_size).  Per-realisation buffers are given as arrays of
 * device pointers (host arrays of R entries):
 *   spec0[r]   [ny_r][nx_r] complex spectrum
 *   t_fast[r]  [n_updates_r + 1][G_r][N_r] complex, cleared by the run
 *   y[r]       [n_updates_r n_fast_r][G_r] complex, written (NULL: skip IQ) */
typedef struct sim_batch sim_batch;

sim_status sim_batch_create(sim_ctx *ctx, int32_t n_real, const sim_grid *grids,
                            const sim_radar *radars, const int32_t *n_updates,
                            sim_batch **batch);
sim_status sim_batch_destroy(sim_batch *batch);
sim_status sim_batch_workspace_size(const sim_batch *batch, size_t *bytes);

/* Enqueue the whole batch on `stream`.  use_graph != 0: the first call with a
 * given set of pointers captures the launches into a graph on `stream`
 * (which must not be the NULL stream), later calls with the same pointers
 * replay it; a call with other pointers captures again. */
sim_status sim_batch_run(sim_batch *batch, void *const *spec0, void *const *t_fast,
                         void *const *y, int use_graph, void *stream);

/* ---- tuning ---------------------------------------------------------------
 * Launch parameters that do not change results beyond summation order;
 * bench/autotune code sets them per context. */
#define SIM_TUNE_ROW_BANDS 0      /* blocks of the fused row pass (bands of rows), 0 = default */
#define SIM_TUNE_ROW_PATH 1       /* row path of sim_update_and_accumulate, one of:             */
#define SIM_ROW_PATH_AUTO 0       /*   the faster on MI355X: currently the split path        */
#define SIM_ROW_PATH_FUSED 1      /*   fused row pass: facets stay on chip                    */
#define SIM_ROW_PATH_SPLIT 2      /*   facet row pass into the workspace, then facet accumulate */
sim_status sim_set_tuning(sim_ctx *ctx, int key, int value);

/* ---- per-kernel timing (profiling aid) ----------------------------------
 * While enabled, every kernel the library launches is bracketed by two HIP
 * events recorded on the stream it is launched on; sim_profile_read waits
 * for the last event and returns, per kernel kind, the summed duration and
 * the launch count since the profile was (re)enabled.  The events come from
 * a pool of 8192 pairs that the first sim_profile_enable creates; launches
 * beyond it are not timed and are counted in `dropped`. */
#define SIM_KERNEL_SURFACE_COLPASS 0      /* spectrum -> 8 half planes, FFT in y */
#define SIM_KERNEL_SURFACE_ROWPASS 1      /* FFT along x -> facet SoA            */
#define SIM_KERNEL_FUSED_ROWPASS 2        /* FFT along x + scatterers + windows  */
#define SIM_KERNEL_ACCUMULATE_FACETS 3    /* facet SoA -> scatterers + windows   */
#define SIM_KERNEL_REDUCE_PARTIALS 4      /* windows -> T_fast[j]                */
#define SIM_KERNEL_SEGMENTS_TO_IQ 5       /* T_fast -> Y                         */
#define SIM_KERNEL_ADJOINT 6              /* waveform loss and adjoint kernels   */
#define SIM_KERNEL_PREPARE 7              /* spectrum preparation, batch clears  */
#define SIM_KERNEL_KINDS 8

typedef struct sim_kernel_times {
  double ms[SIM_KERNEL_KINDS];
  uint64_t launches[SIM_KERNEL_KINDS];
  uint64_t dropped;           /* launches not timed: the event pool was full */
} sim_kernel_times;

/* enable != 0 starts (and clears) the record, creating the event pool on
 * the first call; 0 stops recording. */
sim_status sim_profile_enable(sim_ctx *ctx, int enable);

/* Synchronise on the recorded events and sum them into *out. */
sim_status sim_profile_read(sim_ctx *ctx, sim_kernel_times *out);

#ifdef __cplusplus
}
#endif

#endif /* SIMRADAR_H */
