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

// Column pass: CPB columns per block, ny/16 threads per column.
struct ColPlan {
  int cpb;
  int threads;
  size_t lds_bytes;
};

// Row pass: RPB rows per block, nx/8 threads per row.
struct RowPlan {
  int rpb;
  int threads;
  size_t fft_bytes;   // LDS of the row transforms
  size_t acc_bytes;   // fft_bytes + window + state (fused kernel)
};

hipError_t init_kernel_attributes(int lds_bytes);

template <typename Real>
hipError_t launch_colpass(const void* spec, void* planes, const GridP& gp, double t, double dt,
                          const ColPlan& pl, const void* tw, hipStream_t st);
template <typename Real>
hipError_t launch_rowpass_facets(const void* planes, const GridP& gp, void* const* out,
                                 const RowPlan& pl, const void* tw, hipStream_t st);
template <typename Real>
hipError_t launch_rowpass_accumulate(const void* planes, const GridP& gp, const RadarP& rp,
                                     const WinP& wp, void* Tj, int32_t* code,
                                     const RowPlan& pl, const void* tw, hipStream_t st);
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

}  // namespace simk
