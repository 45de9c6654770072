// Host-visible launch plans and launch wrappers of the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_common.hpp"

namespace simk {

template <typename Real>
struct FacetPtrs {
  Real* p[9];   // disp_x, disp_y, h, sx, sy, jac, ddisp_x, ddisp_y, dh
};

// Launch geometry shared by the host plans and the kernels (compile time).
constexpr size_t kLdsBudget = 159 * 1024;   // usable LDS per block
constexpr int kMinLog2 = 4;                 // grid sides 16 ..
constexpr int kMaxLog2Col = 14;             // .. 16384 along y (8192 in double)
constexpr int kMaxLog2Row = 13;             // .. 8192 along x

__host__ __device__ constexpr size_t lpad_c(size_t i) { return i + (i >> 4); }

// Column pass: CPB adjacent columns per block, ny/E threads per column, as
// many columns as fit kColLds of LDS (one column at least).  E values per
// thread: 16, or 8 in double on columns of 4096 and more (measured on the
// 4096^2 track: 29.5 -> 26.7 ms of column pass per step; half the registers
// per thread, so a CU holds twice the waves).  At those sizes the LDS alone
// sets CPB, so the plane tiles are the same for 8 and 16 values, and the
// persistent batched column pass keeps 16 (kColBatchE: its 1024-thread
// blocks of 8 values would spill).
constexpr size_t kColLds = kLdsBudget;
#ifndef SIMK_COL_E64
#define SIMK_COL_E64 8
#endif
constexpr int kColBatchE = 16;
__host__ __device__ constexpr int col_e(int log2ny, int cs) {
  return (cs == 16 && log2ny >= 12) ? SIMK_COL_E64 : 16;
}
// Short columns (ny <= kColSmallNy) get blocks of at most kColSmallThreads
// threads, so that grids of 1024^2 and 2048^2 still launch hundreds of blocks
// (measured: the 1024^2 regular-mode run 532 -> 461 ms, the 2048^2 gradient
// step 3.13 -> 3.02 ms; 256 threads was slower on 2048^2).
#ifndef SIMK_COL_SMALL_THREADS
#define SIMK_COL_SMALL_THREADS 512
#endif
constexpr int kColSmallThreads = SIMK_COL_SMALL_THREADS;
constexpr int kColSmallNy = 2048;
__host__ __device__ constexpr int col_cpb(int log2ny, int cs) {
  const int cap = (1 << log2ny) <= kColSmallNy ? kColSmallThreads : 1024;
  int cpb = 16;
  while (cpb > 1 && ((long)cpb * ((1 << log2ny) / col_e(log2ny, cs)) > cap ||
                     (size_t)cpb * lpad_c((size_t)1 << log2ny) * cs > kColLds))
    cpb >>= 1;
  return cpb;
}
__host__ __device__ constexpr int col_threads_e(int log2ny, int cs, int e) {
  return col_cpb(log2ny, cs) * ((1 << log2ny) / e);
}
__host__ __device__ constexpr int col_threads(int log2ny, int cs) {
  return col_threads_e(log2ny, cs, col_e(log2ny, cs));
}
__host__ __device__ constexpr size_t col_lds(int log2ny, int cs) {
  return (size_t)col_cpb(log2ny, cs) * lpad_c((size_t)1 << log2ny) * cs;
}

// Layout of the intermediate planes written by the column pass and read by
// the row passes: tiles of TW = CPB columns by TH rows holding kTileElems
// elements (64 bytes in float, 128 in double), tiles in row-major order.  A
// column block then stores whole 64-byte segments instead of CPB-element
// pieces of rows, and a row reads TW contiguous elements per tile; the TH
// rows of a tile row are walked together by bands on one XCD.
constexpr int kTileElems = 8;
__host__ __device__ constexpr int ilog2_c(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
__host__ __device__ constexpr int tile_lw(int log2ny, int cs) {
  return ilog2_c(col_cpb(log2ny, cs));
}
__host__ __device__ constexpr int tile_lh(int log2ny, int cs) {
  return kTileElems / col_cpb(log2ny, cs) > 1 ? ilog2_c(kTileElems / col_cpb(log2ny, cs)) : 0;
}

// The column pass transforms the columns kx >= 0 only (the fields are real,
// so a column kx < 0 is the conjugate of column -kx) and writes eight
// half-width planes, one per y-dependence of the fields.  Their width is
// nx/2, widened to one tile where nx/2 is narrower (columns past nx/2 are
// written as zeros and never read).
constexpr int kHalfPlanes = 8;
__host__ __device__ constexpr int half_lw(int log2nx, int log2ny, int cs) {
  return log2nx - 1 > tile_lw(log2ny, cs) ? log2nx - 1 : tile_lw(log2ny, cs);
}
__host__ __device__ constexpr size_t half_plane_elems(int log2nx, int log2ny, int cs) {
  return (size_t)1 << (half_lw(log2nx, log2ny, cs) + log2ny);
}

// Row passes: ER values per thread, RPB rows per block.
constexpr int kRowE = 8;
__host__ __device__ constexpr int row_tpr(int log2nx) { return (1 << log2nx) / kRowE; }
__host__ __device__ constexpr int row_rpb(int log2nx) {
  return row_tpr(log2nx) >= 256 ? 1 : 256 / row_tpr(log2nx);
}
__host__ __device__ constexpr int row_threads(int log2nx) {
  return row_rpb(log2nx) * row_tpr(log2nx);
}
__host__ __device__ constexpr size_t row_fft_lds(int log2nx, int cs) {
  return (size_t)row_rpb(log2nx) * lpad_c((size_t)1 << log2nx) * cs;
}

// Values per thread of the facet row pass (split row path): 8, or
// SIMK_ROW_E64 in double.  4 gives 1024-thread blocks of radix-4 stages with
// half the registers per thread, so a CU holds twice the waves; measured on
// the 4096^2 track it was slower (56.2 against 51.5 ms of row pass per FP64
// step: the two extra LDS exchanges per transform cost more), so 8 stays.
#ifndef SIMK_ROW_E64
#define SIMK_ROW_E64 8
#endif
__host__ __device__ constexpr int row_facets_er(int log2nx, int cs) {
  return (cs == 16 && (1 << log2nx) / SIMK_ROW_E64 <= 1024) ? SIMK_ROW_E64 : kRowE;
}
__host__ __device__ constexpr int row_facets_tpr(int log2nx, int cs) {
  return (1 << log2nx) / row_facets_er(log2nx, cs);
}
__host__ __device__ constexpr int row_facets_rpb(int log2nx, int cs) {
  return row_facets_tpr(log2nx, cs) >= 256 ? 1 : 256 / row_facets_tpr(log2nx, cs);
}
__host__ __device__ constexpr int row_facets_threads(int log2nx, int cs) {
  return row_facets_rpb(log2nx, cs) * row_facets_tpr(log2nx, cs);
}
__host__ __device__ constexpr size_t row_facets_fft_lds(int log2nx, int cs) {
  return (size_t)row_facets_rpb(log2nx, cs) * lpad_c((size_t)1 << log2nx) * cs;
}

// Staging of the next transform's input in LDS for the fused row pass
// (direct global -> LDS loads of the two half-plane rows it is built from
// while the current row transform runs), for single-row blocks whose LDS
// allows it: after the transform row, nx elements (two half rows), the
// first nx/2 twiddles e^{2 pi i k / nx} (the row transform's
// twiddles are read from LDS, so that no global load of the transform has
// to wait behind the staged row) and a second transform row (the exchanges
// alternate between the two, one barrier each).  The fused kernel keeps room
// for a full window of partial spectra.
constexpr size_t kFusedFrontMax = 120 * 1024;
// The facet row pass alternates its exchanges between two transform rows
// where both fit the LDS budget.
__host__ __device__ constexpr bool row_facets_pp(int log2nx, int cs) {
  return 2 * row_facets_fft_lds(log2nx, cs) <= kLdsBudget;
}
__host__ __device__ constexpr size_t row_facets_lds(int log2nx, int cs) {
  return (row_facets_pp(log2nx, cs) ? 2 : 1) * row_facets_fft_lds(log2nx, cs);
}
__host__ __device__ constexpr size_t row_stage_bytes(bool stage, int log2nx, int cs) {
  return stage ? ((size_t)cs << log2nx) + ((size_t)cs << (log2nx - 1)) +
                     lpad_c((size_t)1 << log2nx) * cs
               : 0;
}
__host__ __device__ constexpr bool row_stage_fused(int log2nx, int cs) {
  return row_rpb(log2nx) == 1 &&
         row_fft_lds(log2nx, cs) + row_stage_bytes(true, log2nx, cs) <= kFusedFrontMax;
}

// Threads per block of the facet accumulate (one band window per block):
// 512 in float, 256 in double (measured on 4096^2: 287 vs 340 us in float,
// 388 vs 466 us in double).
#ifndef SIMK_ACC_THREADS32
#define SIMK_ACC_THREADS32 512
#endif
__host__ __device__ constexpr int acc_threads(int cs) { return cs == 8 ? SIMK_ACC_THREADS32 : 256; }

// LDS of a window context after the partial spectra: 8 state ints, then the
// reduction scratch (6 counters x 16 waves for the band counts; the min/max
// reductions use 4 x 16).
constexpr int kWinStateInts = 8;
constexpr int kWinRedInts = 6 * 16;
constexpr size_t kWinCtxBytes = (kWinStateInts + kWinRedInts) * sizeof(int);

struct ColPlan {
  int cpb;
  int threads;
  size_t lds_bytes;
};

struct RowPlan {
  int rpb;
  int threads;
  size_t fft_bytes;   // LDS of the row transforms
  size_t front_bytes; // fft_bytes + staging row (fused kernel)
  size_t acc_bytes;   // front_bytes + window + state (fused kernel)
};

// One member of a persistent batched launch at one update: its grid (with
// the plane tiles set, grid_with_tiles), platform, windows and buffers.
struct BatchMember {
  GridP gp;
  RadarP rp;
  WinP wp;
  const void* spec;   // prepared spectrum
  void* planes;       // half planes (workspace)
  void* fac[9];       // facet SoA (workspace)
  void* Tj;           // T_fast[j] of the member
  double t, dt;       // first pulse of the pair, pair interval
};

template <typename Real>
GridP grid_with_tiles(const GridP& gp);

// The four per-update phases of the split row path for n_mem members of one
// grid shape (mem: device array), each one persistent launch taking work
// items from its counter (queues[0..3], zero before the launch).
template <typename Real>
hipError_t launch_update_batched(const BatchMember* mem, int n_mem, const GridP& gp,
                                 const RadarP& rp, const WinP& wp, size_t acc_lds, int* queues,
                                 const void* tw, hipStream_t st);

hipError_t init_kernel_attributes(int lds_bytes);
hipError_t launch_clear(void* p, size_t bytes, hipStream_t st);

template <typename Real>
hipError_t launch_colpass(const void* spec, void* planes, const GridP& gp, double t, double dt,
                          const void* tw, bool prepared, hipStream_t st);
template <typename Real>
hipError_t launch_prepare_spectrum(const void* spec, void* out, const GridP& gp, hipStream_t st);
template <typename Real>
hipError_t launch_rowpass_facets(const void* planes, const GridP& gp, void* const* out,
                                 const void* tw, hipStream_t st);
template <typename Real>
hipError_t launch_rowpass_accumulate(const void* planes, const GridP& gp, const RadarP& rp,
                                     const WinP& wp, void* Tj, int32_t* code, size_t lds,
                                     const void* tw, hipStream_t st);
template <typename Real>
hipError_t launch_accumulate_facets(void* const* fac, const GridP& gp, const RadarP& rp,
                                    const WinP& wp, void* Tj, int32_t* code, size_t lds_bytes,
                                    hipStream_t st);
template <typename Real>
hipError_t launch_reduce(const RadarP& rp, const WinP& wp, void* Tj, unsigned long long* counters,
                         hipStream_t st);
template <typename Real>
hipError_t launch_segments_to_iq(const void* T, void* Y, int G, int N, int log2N, int n_fast,
                                 int window, int n_seg, int GB, const void* tw, hipStream_t st);

template <typename Real>
hipError_t launch_waveform_loss(const void* Y, int n_pulses, int G, const void* target, void* P,
                                void* loss, hipStream_t st);
template <typename Real>
hipError_t launch_waveform_loss_adjoint(const void* Y, const void* P, const void* target,
                                        const void* scale, int n_pulses, int G, void* Ybar,
                                        hipStream_t st);
template <typename Real>
hipError_t launch_segments_to_iq_adjoint(const void* Ybar, void* Tbar, int G, int N, int n_fast,
                                         int n_pulses, int window, int n_spec, int GB,
                                         const void* tw, hipStream_t st);
template <typename Real>
hipError_t launch_accumulate_adjoint(void* const* fac, const GridP& gp, const RadarP& rp,
                                     const void* Tbar_j, void* gh, void* gsx, void* gsy,
                                     hipStream_t st);

// Delay-Doppler processing (dd.hip).
template <typename Real>
hipError_t launch_delay_doppler(const void* y, int G, int M, int n_bursts, int centroid_mode,
                                double centroid_given, double mig, int migration, void* beams,
                                void* centroid, void* beam_power, void* waveform,
                                const void* tw, hipStream_t st);

}  // namespace simk
