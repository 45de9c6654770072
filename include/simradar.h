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
 *    Range gates: 1 <= n_gates <= 65536; the calls that scatter facets into
 *    spectra keep one Doppler bin of all gates in a 32 KiB LDS window, so
 *    for them (and for sim_workspace_size) n_gates <= 4096 (FP32 + FP64
 *    phase) or 2048 (FP64), else SIM_ERR_UNSUPPORTED before any launch.
 *  - A context serves one host thread at a time: calls that run concurrently
 *    on one context race on its workspace, and a run call (sim_run_updates
 *    and the accumulate run calls) also uses the context's lane streams and
 *    events.  Work queued on different streams of one context by successive
 *    calls must not overlap either (one workspace).
 */
#ifndef SIMRADAR_H
#define SIMRADAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_ABI_VERSION 6

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

/* The updates of Algorithm 1's loop over spectra (the spectra are
 * independent given the initial spectrum) in one call: for i in [0, count),
 * sim_update_and_accumulate_prepared of spectrum j0 + i at time times[i]
 * (same launches; same results up to the summation order of the window
 * atomics).  With SIM_TUNE_UPDATE_LANES = L > 1 update j0 + i runs on lane
 * i mod L with that lane's workspace slice; the lanes are forked from
 * `stream` and joined back to it, so the call stays ordered on `stream`
 * (and can be captured).  On small grids an update is a chain of short
 * dependent launches that leaves much of the GPU idle; lanes overlap them.
 *   times     host array of count pulse times [s], read during the call.
 *   t_fast    [n_spec][n_gates][n_doppler] complex, accumulated; needs
 *             0 <= j0 and j0 + count <= n_spec.
 *   counters  device sim_counters, accumulated over the updates; may be NULL.
 * Arguments are checked before anything is launched (every time must be
 * finite; with L lanes the workspace must hold L one-lane workspaces, else
 * SIM_ERR_WORKSPACE); a launch error stops the loop and is returned. */
sim_status sim_run_updates(sim_ctx *ctx, const sim_grid *grid, const void *prepared,
                           const sim_radar *radar, int32_t j0, int32_t count,
                           const double *times, void *t_fast, int32_t n_spec,
                           sim_counters *counters, void *stream);

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

/* sim_range_doppler_accumulate and its adjoint for the updates j0 .. j0 +
 * count - 1 of a run in one call, on stacked facet sets: field f of update
 * j0 + i is at facets->f + i ny nx elements (each field a [count][ny][nx]
 * array), update j0 + i at time times[i] (host array of count times, read
 * during the call); grad_h, grad_sx, grad_sy likewise [count][ny][nx].  The
 * updates are dealt to the update lanes as in sim_run_updates (the forward
 * one needs a workspace slice per lane, the adjoint none); results are those
 * of the per-update calls (the adjoint's bit for bit: a per-facet gather).
 * Arguments are checked before anything is launched. */
sim_status sim_range_doppler_accumulate_run(sim_ctx *ctx, const sim_grid *grid,
                                            const sim_facets *facets, const sim_radar *radar,
                                            int32_t j0, int32_t count, const double *times,
                                            void *t_fast, int32_t n_spec,
                                            sim_counters *counters, void *stream);
sim_status sim_range_doppler_accumulate_adjoint_run(sim_ctx *ctx, const sim_grid *grid,
                                                    const sim_facets *facets,
                                                    const sim_radar *radar, int32_t j0,
                                                    int32_t count, const double *times,
                                                    const void *t_fast_bar, int32_t n_spec,
                                                    void *grad_h, void *grad_sx, void *grad_sy,
                                                    void *stream);

/* ---- look-up tables of the facet amplitude ---------------------------------
 * Sec. II.A: the antenna patterns of a simulation are recorded on a u-v grid
 * and interpolated at each facet, and the NRCS comes from look-up tables over
 * the local scattering geometry.  With tables set, the accumulate calls of
 * the context use
 *   a = sqrt(sigma0(theta_l) A) ant(u, v) (H / R)^2       (complex)
 * where (u, v) = ((P_x - S_x) / R, (P_y - S_y) / R) are the direction
 * cosines of the line of sight, ant is interpolated bilinearly on the grid
 * u = u0 + iu du, v = v0 + iv dv of the [nv][nu] complex table (the last node
 * belonging to the cell before it, zero outside the grid), theta_l is the
 * local incidence (tan^2 theta_l = |d x m|^2 / (d . m)^2 of the closed form)
 * and sigma0 is interpolated linearly in the [n_theta] real table over
 * theta_l = i dtheta (zero beyond).  A NULL table keeps its closed form
 * (Gaussian two-way beam, geometric-optics NRCS).  The arrays are caller-owned
 * device memory in the context precision and must stay valid while the
 * context uses them.  The adjoint call rejects a context with tables
 * (SIM_ERR_UNSUPPORTED). */
typedef struct sim_tables {
  const void *antenna;      /* [nv][nu] complex, or NULL                 */
  int32_t nu, nv;           /* >= 2 each                                 */
  double u0, du, v0, dv;    /* grid origin and spacing (du, dv > 0)      */
  const void *nrcs;         /* [n_theta] real, or NULL                   */
  int32_t n_theta;          /* >= 2                                      */
  int32_t reserved;
  double dtheta;            /* [rad] > 0                                 */
} sim_tables;

/* Set (or, with NULL or two NULL tables, clear) the context's tables.  The
 * call waits for the device to be idle, then writes the table parameters to
 * a per-context block of the library's static device memory (256 contexts
 * with tables per device; SIM_ERR_UNSUPPORTED beyond). */
sim_status sim_set_tables(sim_ctx *ctx, const sim_tables *tables);

/* ---- Delay-Doppler processing --------------------------------------------
 * Focusing of the simulated IQ as in Sec. IV.C: the pulses are cut into
 * bursts of M, and for each burst b
 *   1. the Doppler centroid u_c (cycles per pulse) is removed:
 *      y'[x][g] = y[b M + x][g] exp(-2 pi i u_c x); u_c is given, or
 *      estimated per burst as arg(sum_{x,g} y[x+1][g] conj y[x][g]) / (2 pi);
 *   2. an along-track DFT forms M Doppler beams:
 *      Z[b][f][g] = sum_x y'[x][g] exp(-2 pi i f x / M) (beam f at f_s / M
 *      cycles per pulse, f_s = f or f - M);
 *   3. with migration != 0, the range migration of each beam is undone:
 *      Z[b][f][.] <- IDFT(DFT(Z[b][f][.]) exp(+2 pi i q delta_f / G)) / G over
 *      the gates (q in FFT order), delta_f = dy^2 / (2 H dr) gates for the
 *      along-track offset dy = (f_s / M) PRF lambda H / (2 v) of the beam;
 * then the beam powers are multi-looked: beam_power[f][g] = mean_b
 * |Z[b][f][g]|^2 and waveform[g] = mean_f beam_power[f][g].  Trailing pulses
 * that do not fill a burst are ignored.  The IQ convention is that of
 * sim_segments_to_iq (a scatterer of Doppler u has y[x] ~ exp(+2 pi i u x)).
 * Sizes: M a power of two in [2, 256]; n_gates a power of two in [2, 2048];
 * at least one burst.  Reals and complexes follow the context precision. */
#define SIM_DD_CENTROID_GIVEN 0
#define SIM_DD_CENTROID_ESTIMATE 1
typedef struct sim_dd_params {
  int32_t burst;            /* M, pulses per burst                        */
  int32_t centroid_mode;    /* SIM_DD_CENTROID_*                          */
  double centroid;          /* u_c [cycles per pulse] when given          */
  int32_t migration;        /* != 0: step 3                               */
  int32_t reserved;
} sim_dd_params;

/*   y           [n_pulses][n_gates] complex, read only.
 *   beams       [n_pulses / M][M][n_gates] complex, written (focused beams).
 *   centroid    [n_pulses / M] real, written (the centroid used per burst).
 *   beam_power  [M][n_gates] real, written.
 *   waveform    [n_gates] real, written.
 * radar->velocity must be nonzero when migration != 0. */
sim_status sim_delay_doppler(sim_ctx *ctx, const sim_radar *radar, const void *y,
                             int32_t n_pulses, const sim_dd_params *params, void *beams,
                             void *centroid, void *beam_power, void *waveform, void *stream);

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

/* How a batch runs its updates:
 *   SIM_BATCH_LANES       every member on its own, members dealt over four
 *                         streams that overlap the launches of small grids;
 *   SIM_BATCH_PERSISTENT  per update and per shape (members with the same
 *                         grid sides, gates and bins), each phase of the
 *                         update (column pass, facet row pass, facet
 *                         accumulate, ordered reduce) is one persistent
 *                         launch over all members of the shape: a grid of as
 *                         many blocks as the GPU holds takes (member, block)
 *                         work items from a device counter until none is left.
 * Both give the results of the single-member calls (up to summation order).
 * The default is SIM_BATCH_PERSISTENT; the batch workspace covers both. */
#define SIM_BATCH_LANES 1
#define SIM_BATCH_PERSISTENT 2
sim_status sim_batch_set_mode(sim_batch *batch, int mode);

/* Per-member tuning of the lanes mode (SIM_TUNE_ROW_PATH, SIM_TUNE_ROW_BANDS
 * or SIM_TUNE_ACC_BANDS, as sim_set_tuning): an autotuner sets each member the
 * values it found for that member's shape.  Members without their own value
 * use the context's.  The persistent mode always runs the split row path.
 * A graph captured by the batch is dropped (the next graph run captures
 * again with the new values). */
sim_status sim_batch_set_tuning(sim_batch *batch, int32_t member, int key, int value);

/* ---- out-of-core runs -------------------------------------------------------
 * Sec. III.B keeps the main tensors in host memory and only caches on the
 * GPU.  A streamer runs Algorithm 1 and the post-processing for a whole run
 * with T_fast and Y in host memory: the device holds two cache buffers of
 * K + 1 spectra and K n_fast pulses (K = chunk_updates); chunk after chunk,
 * the spectra of K update intervals are computed into one buffer (the first
 * spectrum of a chunk is the last of the previous one, copied on the device),
 * the chunk's IQ is formed from them on the device, and a copy stream of the
 * streamer moves the IQ (and the spectra) to host memory while the next chunk
 * is computed into the other buffer.  Results equal sim_update_and_accumulate
 * over every spectrum followed by sim_segments_to_iq (up to the summation
 * order of the partial spectra).  The host buffers should be pinned
 * (hipHostMalloc) for the copies to overlap the computation. */
typedef struct sim_streamer sim_streamer;

/* Streamer for runs of `radar` on the context's device (makes its copy
 * stream and events). */
sim_status sim_streamer_create(sim_ctx *ctx, const sim_radar *radar, int32_t chunk_updates,
                               sim_streamer **streamer);
sim_status sim_streamer_destroy(sim_streamer *streamer);

/* Device cache bytes sim_streamer_run needs (two buffers). */
sim_status sim_streamer_cache_size(const sim_streamer *streamer, size_t *bytes);

/* One run of n_updates update intervals on `stream`:
 *   prepared     the spectrum in the column-pass layout (sim_prepare_spectrum).
 *   t_fast_host  [n_updates + 1][G][N] complex host memory, written; may be NULL.
 *   y_host       [n_updates n_fast][G] complex host memory, written.
 *   cache        device memory of >= sim_streamer_cache_size bytes, 256-byte
 *                aligned.
 * The context's workspace serves the surface transform as in
 * sim_update_and_accumulate.  When `stream` completes, the host buffers hold
 * the results. */
sim_status sim_streamer_run(sim_streamer *streamer, const sim_grid *grid, const void *prepared,
                            int32_t n_updates, void *t_fast_host, void *y_host, void *cache,
                            size_t cache_bytes, void *stream);

/* ---- tuning ---------------------------------------------------------------
 * Launch parameters that do not change results beyond summation order;
 * bench/autotune code sets them per context. */
#define SIM_TUNE_ROW_BANDS 0      /* blocks of the fused row pass (bands of rows), 0 = default */
#define SIM_TUNE_ROW_PATH 1       /* row path of sim_update_and_accumulate, one of:             */
#define SIM_ROW_PATH_AUTO 0       /*   the faster on MI355X: currently the split path        */
#define SIM_ROW_PATH_FUSED 1      /*   fused row pass: facets stay on chip                    */
#define SIM_ROW_PATH_SPLIT 2      /*   facet row pass into the workspace, then facet accumulate */
#define SIM_TUNE_UPDATE_LANES 2   /* streams sim_run_updates deals the updates to, 1 .. 4:      */
                                  /*   lane 0 is the caller's stream, the others the context's */
                                  /*   own (made here, default priority); each lane needs a    */
                                  /*   workspace of its own, so sim_workspace_size returns     */
                                  /*   lanes x the one-lane size: set the lanes first, then    */
                                  /*   size and set the workspace.  Short updates (small grids) */
                                  /*   then overlap; per-kernel times (sim_profile_*) of       */
                                  /*   overlapping launches include each other's share.        */
#define SIM_TUNE_ACC_BANDS 3      /* most bands (blocks) of the facet accumulate: 0 = default   */
                                  /*   (512), else a power of two from 64 to 512; fewer bands  */
                                  /*   leave room on the CUs for other update lanes' kernels   */
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
#define SIM_KERNEL_DELAY_DOPPLER 8        /* Delay-Doppler processing of the IQ  */
#define SIM_KERNEL_BATCHED_UPDATE 9       /* persistent batched update (4 launches) */
#define SIM_KERNEL_KINDS 10

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
