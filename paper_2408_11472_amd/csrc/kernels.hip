// HIP kernels of the fast-mode hot path for gfx950, with their host launch
// wrappers (called by the C ABI in api.cpp).
//
//   colpass              spectrum evolution of the half spectrum kx >= 0,
//                        one spectrum per y-dependence of the 11 real surface
//                        fields, inverse FFT along y (Sec. II.A surface
//                        synthesis, first half)
//   rowpass_facets       inverse FFT along x, facet geometry, facet SoA out
//   rowpass_accumulate   inverse FFT along x, facet geometry, scatterers and
//                        rasterisation into LDS windows (Algorithm 1), fused
//   accumulate_facets    scatterers and rasterisation from a facet SoA
//   reduce_partials      ordered sum of the band windows into T_fast[j]
//   segments_to_iq       per-gate inverse FFT, eq. (1) weights, overlap-add
#include "device_common.hpp"
#include "scatter.hpp"
#include "launch.hpp"

namespace simk {

// ---------------------------------------------------------------------------
// Column pass.  Block = CPB adjacent columns x TPS threads per column; each
// thread holds E spectral samples of its column at rows s + m * TPS.
//
// With zeta(k, t) = 1/2 [c(k) e^{-i w t} + conj(c(-k)) e^{+i w t}] (Hermitian
// in k) and its increment dzeta over dt, every real field F with multiplier
// M_F has spectrum M_F zeta.  Along a column kx is fixed, so fields whose
// multipliers differ by a factor of kx alone share one column transform
// (h and h_x = i kx h, ...), and the factor is applied by the row pass.
// Every field is real, so its column transform at -kx is the conjugate of
// the one at kx: only the columns kx >= 0 are transformed.  Half planes
// (multiplier of the column transform; fields the row pass takes from it):
//   0: 1            h, h_x          4: -ky^2/|k|      Dy_y
//   1: 1/|k|        Dx, Dx_x        5: 1 (of dzeta)   dh
//   2: i ky/|k|     Dy, Dx_y        6: 1/|k| (dzeta)  dDx
//   3: i ky         h_y             7: i ky/|k| (dz.) dDy
// (the CWM planes 1, 2, 4, 6, 7 are zero without the CWM).  Each column
// strip is handled by two blocks: group 0 makes planes 0-4 from zeta, group
// 1 planes 5-7 from dzeta, so a thread keeps one spectral state.
// PREP: spec is the prepared spectrum (prepare_spectrum_kernel): per column
// strip, rows in order, the pair (c(k), c(-k)) of each column of the strip,
// so the loads of a wave are one contiguous run instead of CPB-element
// pieces of rows and their mirrors.
// Body of one column block: blk of nblk blocks (blockIdx.x and gridDim.x for
// a plain launch, the work item and item count of a member in a batched one).
// OPAQUE_TID (the batched kernel): the thread index is made opaque per call,
// so that nothing derived from it is hoisted out of the item loop and kept
// live across it (which made that kernel spill).
template <typename Real, int LOG2NY, bool PREP, int E, bool OPAQUE_TID>
__device__ __forceinline__ void colpass_body(const cplx<Real>* __restrict__ spec,
                                             cplx<Real>* __restrict__ planes, const GridP& gp,
                                             double t, double dt,
                                             const cplx<Real>* __restrict__ tw, int blk,
                                             int nblk) {
  constexpr int ny = 1 << LOG2NY;
  constexpr int TPS = ny / E;
  constexpr int CPB = col_cpb(LOG2NY, sizeof(cplx<Real>));
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<Real>* lds = reinterpret_cast<cplx<Real>*>(smem_raw);
  const int nx = gp.nx;
  unsigned tid = threadIdx.x;
  if constexpr (OPAQUE_TID) asm volatile("" : "+v"(tid));
  const int c = tid % CPB;
  const int s = tid / CPB;
  // Workgroups are dealt to the 8 XCDs round robin; give each XCD a
  // contiguous run of (strip, group) items so that the two groups of a strip
  // and neighbouring strips, which share cache lines, meet in the same L2.
  const int item = (nblk % 8 == 0) ? (blk & 7) * (nblk >> 3) + (blk >> 3) : blk;
  const int strip = item >> 1, group = item & 1;
  const int ix = strip * CPB + c;          // kx index, 0 <= ix < half width
  const bool live = ix < nx / 2;           // the Nyquist column carries no wave
  const int mx = (nx - ix) & (nx - 1);
  const double twopi = 6.283185307179586476925;
  const double dkx = twopi / ((double)nx * gp.dx);
  const double dky = twopi / ((double)ny * gp.dy);
  const double kx = dkx * (double)ix;
  const Real dcw = gp.cwm ? (Real)1 : (Real)0;

  cplx<Real> st[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int iy = s + m * TPS;
    const int my = (ny - iy) & (ny - 1);
    const int nys = iy < ny / 2 ? iy : iy - ny;
    const bool skip = !live || (iy == ny / 2) || (ix == 0 && iy == 0);
    cplx<Real> z = mk<Real>(0, 0);
    if (!skip) {
      cplx<Real> h0, hm;
      if constexpr (PREP) {
        const cplx<Real>* pp = spec + 2 * (((size_t)strip * ny + iy) * CPB + c);
        h0 = pp[0];
        hm = pp[1];
      } else {
        h0 = spec[(size_t)iy * nx + ix];
        hm = spec[(size_t)my * nx + mx];
      }
      const double ky = dky * (double)nys;
      // w = sqrt(g) (kx^2 + ky^2)^(1/4): two reciprocal square roots refined
      // by Newton steps in double from the float estimate
      const double q2 = kx * kx + ky * ky;
      const double r1 = rsqrt_refined(q2);
      const double w = gp.sqrt_g * rsqrt_refined(r1);
      double rev = w * t * (1.0 / twopi);
      rev -= __builtin_rint(rev);
      Real sn, cs;
      sincos_pi((Real)(2.0 * rev), &sn, &cs);
      // p = 1/2 c(k) e^{-iwt}, q = 1/2 conj(c(-k)) e^{+iwt}
      const cplx<Real> p = mk<Real>((Real)0.5 * (h0.x * cs + h0.y * sn),
                                    (Real)0.5 * (h0.y * cs - h0.x * sn));
      const cplx<Real> q = mk<Real>((Real)0.5 * (hm.x * cs + hm.y * sn),
                                    (Real)0.5 * (hm.x * sn - hm.y * cs));
      if (group == 0) {
        z = cadd(p, q);
      } else {
        // e^{-i w dt} - 1 = -2 sin^2(w dt / 2) - i sin(w dt).  Over one pulse
        // interval w dt stays far below 0.01 rad and the sines are taken
        // from their Taylor series (to the a^7 term, below float and double
        // rounding there); larger steps use sin(w dt) = 2 sin(w dt / 2)
        // cos(w dt / 2) with one sincospi of the half angle, reduced in
        // double by whole turns of 2 (w dt / 4 pi).
        const Real a = (Real)(w * dt);
        Real sh, sf;
        if (a < (Real)0.01) {
          const Real a2 = a * a;
          sh = (Real)0.5 * a *
               ((Real)1 - a2 * (Real)(1.0 / 24) *
                              ((Real)1 - a2 * (Real)(1.0 / 80) * ((Real)1 - a2 * (Real)(1.0 / 168))));
          sf = a * ((Real)1 - a2 * (Real)(1.0 / 6) *
                                  ((Real)1 - a2 * (Real)(1.0 / 20) * ((Real)1 - a2 * (Real)(1.0 / 42))));
        } else {
          double qrev = w * dt * (0.5 / twopi);
          qrev -= __builtin_rint(qrev);
          Real ch;
          sincos_pi((Real)(2.0 * qrev), &sh, &ch);
          sf = (Real)2 * sh * ch;
        }
        const cplx<Real> al = mk<Real>((Real)-2 * sh * sh, -sf);
        z = cadd(cmul(p, al), cmul(q, cconj(al)));
      }
    }
    st[m] = z;
    __builtin_amdgcn_sched_barrier(0);
  }

  const int f0 = group == 0 ? 0 : 5;
  const int f1 = group == 0 ? 5 : 8;
  const int lhw = gp.lhw;
  const size_t psz = (size_t)ny << lhw;
#pragma unroll 1
  for (int f = f0; f < f1; ++f) {
    // Opaque copies of the thread coordinates: everything derived from them
    // (store addresses, wavenumbers, LDS offsets) is recomputed per plane
    // instead of being hoisted out of the loop and kept in registers.
    int sv = s, ixv = ix;
    asm volatile("" : "+v"(sv), "+v"(ixv));
    const Real kxv = (Real)dkx * (Real)ixv;
    // multiplier r (real planes) or i r (imaginary planes)
    const bool imag = f == 2 || f == 3 || f == 7;
    cplx<Real> v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int iy = sv + m * TPS;
      const int nys = iy < ny / 2 ? iy : iy - ny;
      const Real ky = (Real)dky * (Real)nys;
      // 1/|k|; the offset changes no k2 > 0 (k2 >= dk^2) and keeps the zero
      // mode (whose value is zero) finite
      const Real k2 = kxv * kxv + ky * ky;
      const Real ik = approx_rsqrt(k2 + (Real)1e-30);
      Real r;
      switch (f) {
        case 0:
        case 5: r = (Real)1; break;
        case 1:
        case 6: r = dcw * ik; break;
        case 3: r = ky; break;
        case 4: r = -dcw * ky * ky * ik; break;
        default: r = dcw * ky * ik; break;   // 2, 7
      }
      const cplx<Real> z = st[m];
      v[m] = mk<Real>(r * z.x, r * z.y);
    }
    if (imag) {   // (uniform) i r z
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = mk<Real>(-v[m].y, v[m].x);
    }
    fft_seq<Real, LOG2NY, E, CPB, +1>(v, lds + (ixv - strip * CPB), sv, tw);
    // tiled plane layout (TW = CPB columns by TH rows per tile)
    constexpr int LW = tile_lw(LOG2NY, sizeof(cplx<Real>));
    constexpr int LH = tile_lh(LOG2NY, sizeof(cplx<Real>));
    cplx<Real>* out = planes + (size_t)f * psz;
    const int cw = ixv & ((1 << LW) - 1), tx = ixv >> LW;
    if constexpr (TPS % (1 << LH) == 0) {
      // rows s + m TPS: the tile row advances by TPS / TH per slot
      out += ((((size_t)(sv >> LH) << (lhw - LW)) + tx) << (LW + LH)) +
             ((sv & ((1 << LH) - 1)) << LW) + cw;
#pragma unroll
      for (int m = 0; m < E; ++m) out[(size_t)m * TPS << lhw] = v[m];
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int iy = sv + m * TPS;
        out[((((size_t)(iy >> LH) << (lhw - LW)) + tx) << (LW + LH)) +
            ((iy & ((1 << LH) - 1)) << LW) + cw] = v[m];
      }
    }
  }
}

template <typename Real, int LOG2NY, bool PREP>
__global__ void __launch_bounds__(col_threads(LOG2NY, sizeof(cplx<Real>)))
colpass_kernel(const cplx<Real>* __restrict__ spec, cplx<Real>* __restrict__ planes, GridP gp,
               double t, double dt, const cplx<Real>* __restrict__ tw) {
  constexpr int E = col_e(LOG2NY, sizeof(cplx<Real>));
  colpass_body<Real, LOG2NY, PREP, E, false>(spec, planes, gp, t, dt, tw, blockIdx.x, gridDim.x);
}

// The prepared spectrum of the column pass: for each column ix of the half
// width (kx >= 0) and row iy, the FFT-order spectrum's element (iy, ix) and
// its mirror (-iy, -ix) side by side, at position (strip ny + iy) CPB + c
// for ix = strip CPB + c; zeros for the columns from nx/2 on.  One thread per
// element, rows read in order.
template <typename Real>
__global__ void __launch_bounds__(256)
prepare_spectrum_kernel(const cplx<Real>* __restrict__ spec, cplx<Real>* __restrict__ out, int nx,
                        int ny, int lhw, int cpb) {
  const size_t n = (size_t)ny << lhw;
  const int hw = 1 << lhw;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int iy = (int)(i >> lhw), ix = (int)(i & (size_t)(hw - 1));
    const int my = (ny - iy) & (ny - 1), mx = (nx - ix) & (nx - 1);
    const int strip = ix / cpb, c = ix % cpb;
    cplx<Real>* o = out + 2 * (((size_t)strip * ny + iy) * cpb + c);
    const bool live = ix < nx / 2;
    o[0] = live ? spec[(size_t)iy * nx + ix] : mk<Real>(0, 0);
    o[1] = live ? spec[(size_t)my * nx + mx] : mk<Real>(0, 0);
  }
}

// ---------------------------------------------------------------------------
// Row pass helpers.  Block = RPB rows x TPR threads per row; each thread holds
// ER samples of its row at columns tr + m * TPR (ER = 8, or 4 in the facet row
// pass in double; a template parameter of every helper).

// The six row transforms.  Transform q inverts A + i B along x (two real
// fields in one complex transform), A and B taken from half planes a and b
// times a factor of kx: 1, i kx or (i kx)^2 = -kx^2.  Transform 5 carries
// one field (b < 0).
constexpr int kFac1 = 0, kFacIKx = 1, kFacKx2 = 2;
struct PairSrc {
  int a, fa, b, fb;
};
__host__ __device__ constexpr PairSrc pair_src(int q) {
  return q == 0   ? PairSrc{0, kFac1, 1, kFacIKx}     // h + i Dx
         : q == 1 ? PairSrc{2, kFac1, 0, kFacIKx}     // Dy + i h_x
         : q == 2 ? PairSrc{3, kFac1, 1, kFacKx2}     // h_y + i Dx_x
         : q == 3 ? PairSrc{2, kFacIKx, 4, kFac1}     // Dx_y + i Dy_y
         : q == 4 ? PairSrc{5, kFac1, 6, kFacIKx}     // dh + i dDx
                  : PairSrc{7, kFac1, -1, kFac1};     // dDy
}

template <typename Real>
__device__ __forceinline__ cplx<Real> kx_factor(cplx<Real> z, int fac, Real kx) {
  if (fac == kFacIKx) return mk<Real>(-kx * z.y, kx * z.x);
  if (fac == kFacKx2) {
    const Real f = -kx * kx;
    return mk<Real>(f * z.x, f * z.y);
  }
  return z;
}

// Input of transform q at column i from the half-plane values a, b of
// column idx: idx = i for i < nx/2, where the fields are fa a and fb b;
// idx = nx - i above, where a real field's column is the conjugate of its
// column at -kx.  Column 0 of a real field is real (its imaginary part is
// rounding only and is dropped); column nx/2 is zero (not built here).
template <typename Real>
__device__ __forceinline__ cplx<Real> pair_value(cplx<Real> a, cplx<Real> b, const PairSrc& ps,
                                                 Real kx, bool mirror, bool col0) {
  if (col0) {
    a.y = 0;
    b.y = 0;
  }
  cplx<Real> A = kx_factor(a, ps.fa, kx);
  cplx<Real> B = ps.b >= 0 ? kx_factor(b, ps.fb, kx) : mk<Real>(0, 0);
  if (mirror) {
    A.y = -A.y;
    B.y = -B.y;
  }
  return mk<Real>(A.x - B.y, A.y + B.x);
}

// Half-plane column of slot m of thread tr (columns tr + m TPR of the row):
// slots m < ER/2 hold columns below nx/2, the others mirror columns.
template <int LOG2NX, int ER>
__device__ __forceinline__ int half_col(int tr, int m) {
  constexpr int TPR = (1 << LOG2NX) / ER;
  return m < ER / 2 ? tr + m * TPR : (TPR - tr) + (ER - 1 - m) * TPR;
}

// Input of transform q for row iy, read from the half planes in the tiled
// layout (tiles of 2^lw columns by 2^lh rows, rows 2^lhw wide).
template <typename Real, int LOG2NX, int ER>
__device__ __forceinline__ void load_pair_row(const cplx<Real>* __restrict__ planes, size_t psz,
                                              int q, int iy, bool valid, int tr, const GridP& gp,
                                              cplx<Real>* v) {
  constexpr int nx = 1 << LOG2NX, TPR = nx / ER;
  const PairSrc ps = pair_src(q);
  const int lw = gp.tlw, lh = gp.tlh;
  const size_t rb =
      ((size_t)(iy >> lh) << (gp.lhw + lh)) + ((size_t)(iy & ((1 << lh) - 1)) << lw);
  const cplx<Real>* pa = planes + (size_t)ps.a * psz + rb;
  const cplx<Real>* pb = planes + (size_t)(ps.b >= 0 ? ps.b : 0) * psz + rb;
  const Real dkx = (Real)(6.283185307179586476925 / ((double)nx * gp.dx));
  auto off = [&](int col) {
    return ((size_t)(col >> lw) << (lw + lh)) + (col & ((1 << lw) - 1));
  };
  cplx<Real> a[ER], b[ER];
  if ((TPR & ((1 << lw) - 1)) == 0) {
    // columns tr + m TPR and their mirrors: TPR / TW tiles apart per slot
    const size_t ed = off(tr), em = off(TPR - tr), step = (size_t)TPR << lh;
#pragma unroll
    for (int m = 0; m < ER; ++m) {
      const bool ok = valid && (m != ER / 2 || tr != 0);
      const size_t e = m < ER / 2 ? ed + (size_t)m * step : em + (size_t)(ER - 1 - m) * step;
      a[m] = ok ? pa[e] : mk<Real>(0, 0);
      b[m] = (ok && ps.b >= 0) ? pb[e] : mk<Real>(0, 0);
    }
  } else {
#pragma unroll
    for (int m = 0; m < ER; ++m) {
      const int col = half_col<LOG2NX, ER>(tr, m);
      const bool ok = valid && col < nx / 2;
      a[m] = ok ? pa[off(col)] : mk<Real>(0, 0);
      b[m] = (ok && ps.b >= 0) ? pb[off(col)] : mk<Real>(0, 0);
    }
  }
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    const int col = half_col<LOG2NX, ER>(tr, m);
    v[m] = pair_value(a[m], b[m], ps, dkx * (Real)col, m >= ER / 2, m == 0 && tr == 0);
  }
}

// A thread's own columns tr + m TPR (m < ER/2) of the two half planes of a
// transform, loaded ahead of use.
template <typename Real, int ER>
struct PairRegs {
  cplx<Real> a[ER / 2], b[ER / 2];
};

// Loads the own columns of transform q for row iy (zeros outside the grid)
// into r, which holds those of transform q_cur of the same row: a half plane
// the two share is kept instead of read again (the row order of the
// transforms, 3 1 0 2 4 5, puts the two users of half planes 2, 0 and 1
// next to each other).
template <typename Real, int LOG2NX, int ER>
__device__ __forceinline__ void load_pair_direct(const cplx<Real>* __restrict__ planes,
                                                 size_t psz, int q, int iy, int tr,
                                                 const GridP& gp, PairRegs<Real, ER>& r,
                                                 int q_cur = -1) {
  constexpr int nx = 1 << LOG2NX, TPR = nx / ER, H = ER / 2;
  const PairSrc ps = pair_src(q);
  // which of a, b is already in r (after moving it into place)
  bool have_a = false, have_b = false;
  if (q_cur == 3 && q == 1) {
    have_a = true;                       // half plane 2
  } else if (q_cur == 1 && q == 0) {
#pragma unroll
    for (int m = 0; m < H; ++m) r.a[m] = r.b[m];   // half plane 0
    have_a = true;
  } else if (q_cur == 0 && q == 2) {
    have_b = true;                       // half plane 1
  }
  const bool valid = iy >= 0 && iy < gp.ny;
  const int lw = gp.tlw, lh = gp.tlh;
  const size_t rb =
      ((size_t)(iy >> lh) << (gp.lhw + lh)) + ((size_t)(iy & ((1 << lh) - 1)) << lw);
  const cplx<Real>* pa = planes + (size_t)ps.a * psz + rb;
  const cplx<Real>* pb = planes + (size_t)(ps.b >= 0 ? ps.b : 0) * psz + rb;
  const size_t ed = ((size_t)(tr >> lw) << (lw + lh)) + (tr & ((1 << lw) - 1));
#pragma unroll
  for (int m = 0; m < H; ++m) {
    size_t e;
    if ((TPR & ((1 << lw) - 1)) == 0) {
      e = ed + (size_t)m * ((size_t)TPR << lh);
    } else {
      const int col = tr + m * TPR;
      e = ((size_t)(col >> lw) << (lw + lh)) + (col & ((1 << lw) - 1));
    }
    if (!have_a) r.a[m] = valid ? pa[e] : mk<Real>(0, 0);
    if (!have_b) r.b[m] = (valid && ps.b >= 0) ? pb[e] : mk<Real>(0, 0);
  }
}

// Input of transform q from the own columns in r: they are put in X (half
// plane a at [0, nx/2), b at [nx/2, nx)) and, after a barrier, the mirror
// columns are read from there, so that every half-plane element is read
// from memory once.  The barrier before the writes separates this
// transform from the previous one's LDS use.
template <typename Real, int LOG2NX, int ER>
__device__ __forceinline__ void build_pair_x(const PairRegs<Real, ER>& r, int q, int tr,
                                             const GridP& gp, cplx<Real>* v, cplx<Real>* X) {
  constexpr int nx = 1 << LOG2NX, TPR = nx / ER, H = ER / 2;
  const PairSrc ps = pair_src(q);
  const Real dkx = (Real)(6.283185307179586476925 / ((double)nx * gp.dx));
  __syncthreads();
#pragma unroll
  for (int m = 0; m < H; ++m) {
    X[tr + m * TPR] = r.a[m];
    if (ps.b >= 0) X[nx / 2 + tr + m * TPR] = r.b[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    const int col = half_col<LOG2NX, ER>(tr, m);
    cplx<Real> a, b;
    if (m < H) {
      a = r.a[m];
      b = r.b[m];
    } else {
      const bool ok = m != H || tr != 0;
      a = ok ? X[col] : mk<Real>(0, 0);
      b = (ok && ps.b >= 0) ? X[nx / 2 + col] : mk<Real>(0, 0);
    }
    v[m] = pair_value(a, b, ps, dkx * (Real)col, m >= H, m == 0 && tr == 0);
  }
}

// Direct global -> LDS loads of the first nx/2 columns of row iy of a half
// plane into S (column order), issued by the TPR threads of a single-row
// block: 16 bytes per lane (two float or one double element, adjacent within
// a tile), or 4 bytes per lane for float planes in one-column tiles.
// Completion is awaited with the vector-memory counter and a barrier before
// S is read.
template <typename Real, int LOG2NX, int ER>
__device__ __forceinline__ void stage_half_row(const cplx<Real>* __restrict__ plane, int iy,
                                               const GridP& gp, cplx<Real>* S, int tr) {
  constexpr int nx = 1 << LOG2NX, TPR = nx / ER, W = TPR / 64, NH = nx / 2;
  constexpr int cs = sizeof(cplx<Real>);
  const int lane = tr & 63, w = tr >> 6;
  const int lw = gp.tlw, lh = gp.tlh;
  const size_t rb =
      ((size_t)(iy >> lh) << (gp.lhw + lh)) + ((size_t)(iy & ((1 << lh) - 1)) << lw);
  typedef __attribute__((address_space(3))) void* lds_ptr;
  if (cs == 16 || lw >= 1) {
    constexpr int EPL = 16 / cs;       // elements per lane
    constexpr int PER = 64 * EPL;      // elements per wave instruction
#pragma unroll
    for (int c = w; c < NH / PER; c += W) {
      const int ix = c * PER + lane * EPL;
      const cplx<Real>* src =
          plane + rb + ((size_t)(ix >> lw) << (lw + lh)) + (ix & ((1 << lw) - 1));
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_ptr)(S + c * PER), 16, 0, 0);
    }
  } else {
    const Real* f = reinterpret_cast<const Real*>(plane);
#pragma unroll
    for (int c = w; c < 2 * NH / 64; c += W) {
      const int qf = c * 64 + lane;    // scalar index within the half row
      const int ix = qf >> 1;
      const size_t e = rb + ((size_t)(ix >> lw) << (lw + lh)) + (ix & ((1 << lw) - 1));
      __builtin_amdgcn_global_load_lds((const void*)(f + 2 * e + (qf & 1)),
                                       (lds_ptr)(reinterpret_cast<Real*>(S) + c * 64), 4, 0, 0);
    }
  }
}

// Stages the inputs of transform q for row iy: half plane a into S[0, nx/2),
// half plane b into S[nx/2, nx).
template <typename Real, int LOG2NX, int ER>
__device__ __forceinline__ void stage_pair(const cplx<Real>* __restrict__ planes, size_t psz,
                                           int q, int iy, const GridP& gp, cplx<Real>* S,
                                           int tr) {
  const PairSrc ps = pair_src(q);
  stage_half_row<Real, LOG2NX, ER>(planes + (size_t)ps.a * psz, iy, gp, S, tr);
  if (ps.b >= 0)
    stage_half_row<Real, LOG2NX, ER>(planes + (size_t)ps.b * psz, iy, gp, S + (1 << LOG2NX) / 2,
                                     tr);
}

// Input of transform q from its staged half rows.
template <typename Real, int LOG2NX, int ER>
__device__ __forceinline__ void read_pair_lds(const cplx<Real>* S, int q, int tr, const GridP& gp,
                                              cplx<Real>* v) {
  constexpr int nx = 1 << LOG2NX;
  const PairSrc ps = pair_src(q);
  const Real dkx = (Real)(6.283185307179586476925 / ((double)nx * gp.dx));
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    const int col = half_col<LOG2NX, ER>(tr, m);
    const bool ok = m != ER / 2 || tr != 0;
    const cplx<Real> a = ok ? S[col] : mk<Real>(0, 0);
    const cplx<Real> b = (ok && ps.b >= 0) ? S[nx / 2 + col] : mk<Real>(0, 0);
    v[m] = pair_value(a, b, ps, dkx * (Real)col, m >= ER / 2, m == 0 && tr == 0);
  }
}

// Where the next transform's input comes from (staged mode): transform
// index and row, or no next transform (q < 0).
struct NextRow {
  int q, iy;
};

// Inverse transform along x of transform q for one row.  The thread
// coordinate is made opaque per call, so that addresses and LDS offsets are
// recomputed per transform instead of being kept live across all six.
// Staged mode: the input rows were loaded into S ahead of time; once every
// thread has its values, the next transform's rows are put in flight into S.
// Unstaged mode with PP (lrow2 and pre set): the exchanges alternate between lrow and
// lrow2 (one barrier each), the mirror columns of the input go through lrow2
// before the first exchange writes lrow (build_pair_x), and the own columns
// of the next transform are loaded into pre while this one runs.
template <typename Real, int LOG2NX, int ER, bool STAGE, bool PP>
__device__ __forceinline__ void row_transform(const cplx<Real>* __restrict__ planes, size_t psz,
                                              int q, int iy, bool valid, int tr,
                                              const GridP& gp, cplx<Real>* lrow, cplx<Real>* S,
                                              NextRow nxt, const cplx<Real>* __restrict__ tw,
                                              cplx<Real>* v, cplx<Real>* lrow2 = nullptr,
                                              PairRegs<Real, ER>* pre = nullptr) {
  int trv = tr;
  asm volatile("" : "+v"(trv));
  if constexpr (STAGE) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    read_pair_lds<Real, LOG2NX, ER>(S, q, trv, gp, v);
    __syncthreads();
    if (nxt.q >= 0) stage_pair<Real, LOG2NX, ER>(planes, psz, nxt.q, nxt.iy, gp, S, trv);
    // after S: the LDS twiddles (nx/2) and the second exchange row; the two
    // barriers above separate this transform from the previous one
    constexpr int nx = 1 << LOG2NX;
    fft_seq<Real, LOG2NX, ER, 1, +1, true, true>(v, lrow, trv, S + nx, S + nx + nx / 2);
  } else {
    if constexpr (PP) {
      build_pair_x<Real, LOG2NX, ER>(*pre, q, trv, gp, v, lrow2);
      if (nxt.q >= 0)
        load_pair_direct<Real, LOG2NX, ER>(planes, psz, nxt.q, nxt.iy, trv, gp, *pre,
                                           nxt.iy == iy ? q : -1);
      fft_seq<Real, LOG2NX, ER, 1, +1, false, true>(v, lrow, trv, tw, lrow2);
    } else {
      load_pair_row<Real, LOG2NX, ER>(planes, psz, q, iy, valid, trv, gp, v);
      fft_seq<Real, LOG2NX, ER, 1, +1>(v, lrow, trv, tw);
    }
  }
}

// LDS copy of the twiddles e^{2 pi i k / nx}, k < nx/2 (from slice nx of the
// table): the radix-8 stages of an nx-point transform read no higher index.
template <typename Real, int LOG2NX>
__device__ __forceinline__ void load_row_twiddles(cplx<Real>* dst,
                                                  const cplx<Real>* __restrict__ tw) {
  constexpr int nx = 1 << LOG2NX;
  for (int i = threadIdx.x; i < nx / 2; i += blockDim.x) dst[i] = tw[nx + i];
}

// The nine facet quantities of one row.  The transforms run in the order
// 3 1 0 2 (geometry: the normal needs 3, 1 and 2; 0 gives the position), then
// 4 5 (displacement over the pulse pair); each quantity is handed to emit(i,
// values) as soon as it is formed, i its index in the facet SoA.
template <typename Real, int ER>
struct RowFacets {
  Real Dx[ER], Dy[ER], h[ER], sx[ER], sy[ER], jac[ER], dDx[ER], dDy[ER], dh[ER];
};

struct NoEmit {
  template <typename T>
  __device__ void operator()(int, const T*) const {}
};

template <typename Real, int LOG2NX, int ER, bool STAGE, bool PP, typename Emit>
__device__ __forceinline__ void row_geometry(const cplx<Real>* __restrict__ planes, size_t psz,
                                             int iy, bool valid, int tr, const GridP& gp,
                                             cplx<Real>* lrow, cplx<Real>* S, int iy_stage,
                                             const cplx<Real>* __restrict__ tw,
                                             RowFacets<Real, ER>& F, Emit emit,
                                             cplx<Real>* lrow2 = nullptr,
                                             PairRegs<Real, ER>* pre = nullptr) {
  cplx<Real> v[ER];
  Real dxy[ER], dyy[ER], hx[ER];
  row_transform<Real, LOG2NX, ER, STAGE, PP>(planes, psz, 3, iy, valid, tr, gp, lrow, S,
                                     NextRow{1, iy_stage}, tw, v, lrow2, pre);  // Dx_y + i Dy_y
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    dxy[m] = v[m].x;
    dyy[m] = v[m].y;
  }
  row_transform<Real, LOG2NX, ER, STAGE, PP>(planes, psz, 1, iy, valid, tr, gp, lrow, S,
                                     NextRow{0, iy_stage}, tw, v, lrow2, pre);  // Dy + i h_x
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    F.Dy[m] = v[m].x;
    hx[m] = v[m].y;
  }
  emit(1, F.Dy);
  row_transform<Real, LOG2NX, ER, STAGE, PP>(planes, psz, 0, iy, valid, tr, gp, lrow, S,
                                     NextRow{2, iy_stage}, tw, v, lrow2, pre);  // h + i Dx
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    F.h[m] = v[m].x;
    F.Dx[m] = v[m].y;
  }
  emit(0, F.Dx);
  emit(2, F.h);
  row_transform<Real, LOG2NX, ER, STAGE, PP>(planes, psz, 2, iy, valid, tr, gp, lrow, S,
                                     NextRow{4, iy_stage}, tw, v, lrow2, pre);  // h_y + i Dx_x
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    const Real hy = v[m].x, dxx = v[m].y;
    // n = r_x x r_y with r_x = (1 + Dx_x, Dx_y, h_x), r_y = (Dx_y, 1 + Dy_y, h_y)
    const Real nxn = dxy[m] * hy - hx[m] * ((Real)1 + dyy[m]);
    const Real nyn = hx[m] * dxy[m] - ((Real)1 + dxx) * hy;
    const Real nzn = ((Real)1 + dxx) * ((Real)1 + dyy[m]) - dxy[m] * dxy[m];
    const Real inz = approx_rcp(nzn);
    F.jac[m] = nzn;
    F.sx[m] = -nxn * inz;
    F.sy[m] = -nyn * inz;
  }
  emit(3, F.sx);
  emit(4, F.sy);
  emit(5, F.jac);
}

template <typename Real, int LOG2NX, int ER, bool STAGE, bool PP, typename Emit>
__device__ __forceinline__ void row_motion(const cplx<Real>* __restrict__ planes, size_t psz,
                                           int iy, bool valid, int tr, const GridP& gp,
                                           cplx<Real>* lrow, cplx<Real>* S, int iy_stage,
                                           int iy_next, const cplx<Real>* __restrict__ tw,
                                           RowFacets<Real, ER>& F, Emit emit,
                                           cplx<Real>* lrow2 = nullptr,
                                           PairRegs<Real, ER>* pre = nullptr) {
  cplx<Real> v[ER];
  row_transform<Real, LOG2NX, ER, STAGE, PP>(planes, psz, 4, iy, valid, tr, gp, lrow, S,
                                     NextRow{5, iy_stage}, tw, v, lrow2, pre);  // dh + i dDx
#pragma unroll
  for (int m = 0; m < ER; ++m) {
    F.dh[m] = v[m].x;
    F.dDx[m] = v[m].y;
  }
  emit(6, F.dDx);
  emit(8, F.dh);
  // the row after this one starts with transform 3 (iy_next < 0: none)
  row_transform<Real, LOG2NX, ER, STAGE, PP>(planes, psz, 5, iy, valid, tr, gp, lrow, S,
                                     NextRow{iy_next >= 0 ? 3 : -1, iy_next}, tw, v, lrow2,
                                     pre);  // dDy
#pragma unroll
  for (int m = 0; m < ER; ++m) F.dDy[m] = v[m].x;
  emit(7, F.dDy);
}

template <typename Real, int LOG2NX>
__device__ __forceinline__ void rowpass_facets_body(const cplx<Real>* __restrict__ planes,
                                                    const GridP& gp, const FacetPtrs<Real>& out,
                                                    const cplx<Real>* __restrict__ tw, int blk,
                                                    int nblk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int nx = 1 << LOG2NX;
  constexpr int cs = sizeof(cplx<Real>);
  constexpr int ER = row_facets_er(LOG2NX, cs);
  constexpr int TPR = row_facets_tpr(LOG2NX, cs);
  constexpr int RPB = row_facets_rpb(LOG2NX, cs);
  constexpr bool PP = row_facets_pp(LOG2NX, cs);
  const int ny = gp.ny;
  // No staging here: the wait for a staged row (vector-memory counter) would
  // also wait for this kernel's facet stores, which costs more than the load
  // latency it hides.
  constexpr bool STAGE = false;
  const int rl = threadIdx.x / TPR, tr = threadIdx.x % TPR;
  cplx<Real>* lrow = reinterpret_cast<cplx<Real>*>(smem_raw) + (size_t)rl * lpad(nx);
  cplx<Real>* S = nullptr;   // (no staging row)
  // second exchange buffer of this row (ping-pong exchanges), where it fits
  cplx<Real>* lrow2 =
      PP ? reinterpret_cast<cplx<Real>*>(smem_raw) + (size_t)(RPB + rl) * lpad(nx) : nullptr;
  const size_t psz = (size_t)ny << gp.lhw;
  // Workgroups are dealt to the 8 XCDs round robin: give each XCD a
  // contiguous run of row chunks, so that the chunks sharing a plane tile
  // (and its cache lines) are read through the same L2 at about the same time.
  const int q = (nblk % 8 == 0) ? (blk & 7) * (nblk >> 3) + (blk >> 3) : blk;

  // with two exchange rows, the own columns of each transform's input are
  // loaded one transform ahead (first: transform 3 of the first row)
  PairRegs<Real, ER> pre;
  if (PP) load_pair_direct<Real, LOG2NX, ER>(planes, psz, 3, q * RPB + rl, tr, gp, pre);
  for (int iy0 = q * RPB; iy0 < ny; iy0 += nblk * RPB) {
    const int iy = iy0 + rl;
    const bool valid = iy < ny;
    const int iy_next = iy0 + nblk * RPB < ny ? iy0 + nblk * RPB + rl : -1;
    // each facet quantity is stored as soon as it is formed
    auto emit = [&](int field, const Real* val) {
      if (valid) {
#pragma unroll
        for (int m = 0; m < ER; ++m) out.p[field][(size_t)iy * nx + tr + m * TPR] = val[m];
      }
    };
    RowFacets<Real, ER> F;
    row_geometry<Real, LOG2NX, ER, STAGE, PP>(planes, psz, iy, valid, tr, gp, lrow, S, iy, tw,
                                              F, emit, lrow2, &pre);
    row_motion<Real, LOG2NX, ER, STAGE, PP>(planes, psz, iy, valid, tr, gp, lrow, S, iy, iy_next,
                                            tw, F, emit, lrow2, &pre);
  }
}

template <typename Real, int LOG2NX>
__global__ void __launch_bounds__(row_facets_threads(LOG2NX, sizeof(cplx<Real>)))
rowpass_facets_kernel(const cplx<Real>* __restrict__ planes, GridP gp, FacetPtrs<Real> out,
                      const cplx<Real>* __restrict__ tw) {
  rowpass_facets_body<Real, LOG2NX>(planes, gp, out, tw, blockIdx.x, gridDim.x);
}

// Shared LDS carve-up for the accumulating kernels: [fft rows][window][state]
template <typename Real>
__device__ __forceinline__ WinCtx<Real> win_ctx(unsigned char* smem, size_t fft_bytes,
                                                const RadarP& rp, const WinP& wp,
                                                cplx<Real>* Tj, int band) {
  WinCtx<Real> w;
  w.win = reinterpret_cast<cplx<Real>*>(smem + fft_bytes);
  int* ints = reinterpret_cast<int*>(smem + fft_bytes + (size_t)rp.G * wp.WK * sizeof(cplx<Real>));
  w.st = ints;
  w.red = ints + kWinStateInts;
  w.Tj = Tj;
  w.band = band;
  return w;
}

template <typename Real, int LOG2NX>
__global__ void __launch_bounds__(row_threads(LOG2NX))
rowpass_accumulate_kernel(const cplx<Real>* __restrict__ planes, GridP gp, RadarP rp, WinP wp,
                          cplx<Real>* __restrict__ Tj, int32_t* __restrict__ code_out,
                          const cplx<Real>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int nx = 1 << LOG2NX;
  constexpr int ER = kRowE;
  constexpr int TPR = row_tpr(LOG2NX);
  constexpr int RPB = row_rpb(LOG2NX);
  const int ny = gp.ny;
  constexpr bool STAGE = row_stage_fused(LOG2NX, sizeof(cplx<Real>));
  const int rl = threadIdx.x / TPR, tr = threadIdx.x % TPR;
  const size_t fft_bytes = (size_t)RPB * lpad(nx) * sizeof(cplx<Real>);
  cplx<Real>* lrow = reinterpret_cast<cplx<Real>*>(smem_raw) + (size_t)rl * lpad(nx);
  cplx<Real>* S = reinterpret_cast<cplx<Real>*>(smem_raw + fft_bytes);
  const int band = blockIdx.x;
  WinCtx<Real> w = win_ctx<Real>(
      smem_raw, fft_bytes + row_stage_bytes(STAGE, LOG2NX, sizeof(cplx<Real>)), rp, wp, Tj, band);
  win_init(w, rp, wp);
  uint32_t cnt[5] = {0, 0, 0, 0, 0};
  uint32_t overflow = 0;
  const size_t psz = (size_t)ny << gp.lhw;
  // Row walk of this band.  The rows of one plane tile (TH rows) are split
  // over M = TH / RPB bands that run on the same XCD (workgroups are dealt
  // to the XCDs round robin) and walk the same tile rows together, so each
  // cache line fetched for a tile is read by all of them through one L2.
  // Group g of M bands takes tile rows [g band_rows, (g + 1) band_rows);
  // member r takes rows r RPB .. r RPB + RPB - 1 of each.  Without enough
  // bands for that, a band takes band_rows consecutive rows.
  const int TH = 1 << gp.tlh;
  const int M = TH > RPB ? TH / RPB : 1;
  const int nb = wp.n_bands;
  int first_tile_row = 0, member = 0, step_rows = RPB;
  const bool grouped =
      M > 1 && nb % (8 * M) == 0 && wp.band_rows % RPB == 0 && wp.band_rows * nb == ny;
  const int n_steps = grouped ? wp.band_rows / RPB : (wp.band_rows + RPB - 1) / RPB;
  if (grouped) {
    const int l = band >> 3, per_xcd = nb >> 3;
    const int group = (band & 7) * (per_xcd / M) + l / M;
    member = l % M;
    first_tile_row = group * n_steps;
    step_rows = TH;
  }
  const int row_begin = grouped ? first_tile_row * TH + member * RPB : band * wp.band_rows;
  const int row_end = grouped ? ny : min(ny, row_begin + wp.band_rows);
  // staged rows are clamped into the grid (a row past the band end is
  // transformed but not scattered)
  if (STAGE) load_row_twiddles<Real, LOG2NX>(S + nx, tw);   // ordered by the first barrier
  if (STAGE && n_steps > 0)
    stage_pair<Real, LOG2NX, ER>(planes, psz, 3, min(row_begin, ny - 1), gp, S, tr);
  for (int k = 0; k < n_steps; ++k) {
    const int iy0 = row_begin + k * step_rows;
    const int iy = iy0 + rl;
    const bool valid = iy < row_end;
    const int iy_stage = min(iy, ny - 1);
    const int iy_next = k + 1 < n_steps ? min(iy0 + step_rows + rl, ny - 1) : -1;
    RowFacets<Real, ER> F;
    row_geometry<Real, LOG2NX, ER, STAGE, false>(planes, psz, iy, valid, tr, gp, lrow, S,
                                                 iy_stage, tw, F, NoEmit());
    row_motion<Real, LOG2NX, ER, STAGE, false>(planes, psz, iy, valid, tr, gp, lrow, S, iy_stage,
                                               iy_next, tw, F, NoEmit());
    int key[ER];
    cplx<Real> cv[ER];
    // opaque row coordinates: the grid positions of the facets are
    // recomputed per row rather than kept live across the row loop
    int trv = tr, iyv = iy;
    asm volatile("" : "+v"(trv), "+v"(iyv));
#pragma unroll
    for (int m = 0; m < ER; ++m) {
      const int ix = trv + m * TPR;
      key[m] = -100;
      cv[m] = mk<Real>(0, 0);
      if (valid) {
        key[m] = scatterer<Real>(rp, gp, ix, iyv, F.Dx[m], F.Dy[m], F.h[m], F.sx[m], F.sy[m],
                                 F.jac[m], F.dDx[m], F.dDy[m], F.dh[m], cv[m]);
        count_code(key[m], cnt);
        if (code_out) code_out[(size_t)iyv * nx + ix] = key[m];
      }
      // one facet at a time: keeps the double temporaries of a single
      // scatterer live instead of eight
      __builtin_amdgcn_sched_barrier(0);
    }
    win_add<Real, ER>(w, rp, wp, key, cv, overflow);
  }
  win_finish(w, rp, wp, overflow);
  store_band_counts(wp, band, cnt, overflow, w.red);
}

// ---------------------------------------------------------------------------
// Scatterers from a facet SoA: band = contiguous facet range, chunks of
// EA * blockDim facets.
#ifndef SIMK_EA
#define SIMK_EA 8
#endif
constexpr int EA = SIMK_EA;

template <typename Real>
__device__ __forceinline__ void accumulate_facets_body(const FacetPtrs<Real>& fac,
                                                       const GridP& gp, const RadarP& rp,
                                                       const WinP& wp,
                                                       cplx<Real>* __restrict__ Tj,
                                                       int32_t* __restrict__ code_out,
                                                       int band) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  WinCtx<Real> w = win_ctx<Real>(smem_raw, 0, rp, wp, Tj, band);
  win_init(w, rp, wp);
  uint32_t cnt[5] = {0, 0, 0, 0, 0};
  uint32_t overflow = 0;
  const size_t nfac = (size_t)gp.nx * gp.ny;
  const size_t f_begin = (size_t)band * wp.band_rows;
  const size_t f_end = min(nfac, f_begin + (size_t)wp.band_rows);
  for (size_t c0 = f_begin; c0 < f_begin + (size_t)wp.band_rows; c0 += (size_t)EA * blockDim.x) {
    int key[EA];
    cplx<Real> cv[EA];
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const size_t f = c0 + threadIdx.x + (size_t)e * blockDim.x;
      key[e] = -100;
      cv[e] = mk<Real>(0, 0);
      if (f < f_end) {
        const int iy = (int)(f >> gp.log2nx);
        const int ix = (int)(f & (size_t)(gp.nx - 1));
        key[e] = scatterer<Real>(rp, gp, ix, iy, fac.p[0][f], fac.p[1][f], fac.p[2][f],
                                 fac.p[3][f], fac.p[4][f], fac.p[5][f], fac.p[6][f],
                                 fac.p[7][f], fac.p[8][f], cv[e]);
        count_code(key[e], cnt);
        if (code_out) code_out[f] = key[e];
      }
    }
    win_add<Real, EA>(w, rp, wp, key, cv, overflow);
  }
  win_finish(w, rp, wp, overflow);
  store_band_counts(wp, band, cnt, overflow, w.red);
}

// The double constants of the scatterer's range and index arithmetic, held
// in vector registers (one copy per lane) instead of scalar ones: the facet
// loop is short of scalar registers, and a spilled scalar costs a vector
// instruction (readlane) at every use (measured: ~2% of the kernel's time).
// The empty asm only moves the value; the arithmetic is unchanged.
__device__ __forceinline__ void to_vgpr(double& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin_scatter_constants(GridP& g, RadarP& r) {
  to_vgpr(g.x_origin);
  to_vgpr(g.dx);
  to_vgpr(g.y_origin);
  to_vgpr(g.dy);
  to_vgpr(r.sat_x);
  to_vgpr(r.sat_y1);
  to_vgpr(r.sat_y2);
  to_vgpr(r.altitude);
  to_vgpr(r.window_start);
  to_vgpr(r.gate_spacing);
  to_vgpr(r.k2);
}

template <typename Real>
__global__ void __launch_bounds__(acc_threads(sizeof(cplx<Real>)))
accumulate_facets_kernel(FacetPtrs<Real> fac, GridP gp, RadarP rp, WinP wp,
                         cplx<Real>* __restrict__ Tj, int32_t* __restrict__ code_out) {
  pin_scatter_constants(gp, rp);
  accumulate_facets_body<Real>(fac, gp, rp, wp, Tj, code_out, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Ordered reduction of the band windows into T_fast[j]: one block per gate.
// The slots covering the gate are compacted in slot order and cut into
// contiguous chunks, one per wave.  Each wave adds its chunk, slot after
// slot, into its own double accumulator in LDS (lanes = bins of the window,
// a batch of loads in flight); the wave accumulators are then added in wave
// order.  The association of the sum is fixed, so the result does not
// depend on scheduling.  Block 0 also adds the band counters.
constexpr int kReduceThreads = 1024;
constexpr int kReduceBatch = 8;

template <typename Real>
__device__ __forceinline__ void reduce_partials_body(const RadarP& rp, const WinP& wp,
                                                     cplx<Real>* __restrict__ Tj,
                                                     unsigned long long* __restrict__ counters,
                                                     int n_acc, int g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nslots = wp.n_bands * wp.S;
  const int N = rp.N, WK = wp.WK;
  cplx<double>* acc = reinterpret_cast<cplx<double>*>(smem_raw);          // [n_acc][N]
  int* list = reinterpret_cast<int*>(acc + (size_t)n_acc * N);             // [nslots]
  int* lk0 = list + nslots;                                                // [nslots]
  __shared__ int wcount[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = threadIdx.x; i < n_acc * N; i += blockDim.x) acc[i] = mk<double>(0.0, 0.0);
  int base = 0;
  for (int s0 = 0; s0 < nslots; s0 += blockDim.x) {
    const int s = s0 + threadIdx.x;
    bool take = false;
    int k0 = 0;
    if (s < nslots) {
      const int4 h = wp.hdr[s];
      take = h.x != 0 && g >= h.z && g <= h.w;
      k0 = h.y;
    }
    const unsigned long long bal = __ballot(take);
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wv] = __popcll(bal);
    __syncthreads();
    int off = base, tot = 0;
    for (int w2 = 0; w2 < nw; ++w2) {
      if (w2 < wv) off += wcount[w2];
      tot += wcount[w2];
    }
    if (take) {
      list[off + rank] = s;
      lk0[off + rank] = k0;
    }
    __syncthreads();
    base += tot;
  }
  // wave wv < n_acc takes entries [lo, hi) in order
  const cplx<Real>* part = (const cplx<Real>*)wp.part;
  if (wv < n_acc) {
    const int per = (base + n_acc - 1) / n_acc;
    const int lo = min(base, wv * per), hi = min(base, lo + per);
    cplx<double>* a = acc + (size_t)wv * N;
    for (int d0 = 0; d0 < WK; d0 += 64) {
      const int d = d0 + lane;
      for (int i0 = lo; i0 < hi; i0 += kReduceBatch) {
        cplx<Real> v[kReduceBatch];
#pragma unroll
        for (int b = 0; b < kReduceBatch; ++b) {
          v[b] = mk<Real>(0, 0);
          if (i0 + b < hi && d < WK)
            v[b] = part[((size_t)list[i0 + b] * rp.G + g) * WK + d];
        }
#pragma unroll
        for (int b = 0; b < kReduceBatch; ++b) {
          if (i0 + b < hi && d < WK) {
            cplx<double>& c = a[(lk0[i0 + b] + d) & (N - 1)];
            c.x += (double)v[b].x;
            c.y += (double)v[b].y;
          }
        }
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    double ax = 0.0, ay = 0.0;
    for (int w2 = 0; w2 < n_acc; ++w2) {
      ax += acc[(size_t)w2 * N + k].x;
      ay += acc[(size_t)w2 * N + k].y;
    }
    cplx<Real> t = Tj[(size_t)g * N + k];
    t.x = (Real)((double)t.x + ax);
    t.y = (Real)((double)t.y + ay);
    Tj[(size_t)g * N + k] = t;
  }
  if (g == 0 && counters != nullptr) {
    unsigned long long v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < wp.n_bands; b += blockDim.x)
      for (int i = 0; i < 6; ++i) v[i] += wp.bandcnt[(size_t)b * 8 + i];
    __shared__ unsigned long long red[6][16];
    for (int i = 0; i < 6; ++i) {
      unsigned long long x = v[i];
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) red[i][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      unsigned long long sum = 0;
      for (int w2 = 0; w2 < nw; ++w2) sum += red[threadIdx.x][w2];
      // atomic: updates of one run may overlap on several streams
      atomicAdd(&counters[threadIdx.x], sum);
    }
  }
}

template <typename Real>
__global__ void __launch_bounds__(kReduceThreads)
reduce_partials_kernel(RadarP rp, WinP wp, cplx<Real>* __restrict__ Tj,
                       unsigned long long* __restrict__ counters, int n_acc) {
  reduce_partials_body<Real>(rp, wp, Tj, counters, n_acc, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Persistent batched launches.  The members of a batch that share a grid
// shape run each phase of an update (column pass, facet row pass, facet
// accumulate, ordered reduce) in one launch of a grid sized to what the GPU
// holds at once.  Work items are (member, block of that member), numbered
// member-major; blocks take them from a device counter (one counter per
// launch, cleared with the batch) and run them until the counter passes the
// item count, which every block reaches.  The per-member parameters of the
// update are read from a descriptor array in device memory.

// Next work item of the block (uniform over the block): thread 0 takes it
// from the counter, the block reads it after a barrier; the second barrier
// keeps it until every thread has it (and orders the previous item's LDS
// use before the next item's).
__device__ __forceinline__ int next_item(int* queue, int* s_item) {
  if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
  __syncthreads();
  const int item = __builtin_amdgcn_readfirstlane(*s_item);
  __syncthreads();
  return item;
}

template <typename Real, int LOG2NY>
__global__ void __launch_bounds__(col_threads_e(LOG2NY, sizeof(cplx<Real>), kColBatchE))
colpass_batched_kernel(const BatchMember* __restrict__ mem, int per, int n_items,
                       int* __restrict__ queue, const cplx<Real>* __restrict__ tw) {
  __shared__ int s_item;
  for (;;) {
    const int item = next_item(queue, &s_item);
    if (item >= n_items) break;
    const int m = item / per, blk = item - m * per;
    const BatchMember& b = mem[m];
    colpass_body<Real, LOG2NY, true, kColBatchE, true>((const cplx<Real>*)b.spec,
                                                       (cplx<Real>*)b.planes, b.gp, b.t, b.dt,
                                                       tw, blk, per);
  }
}

template <typename Real, int LOG2NX>
__global__ void __launch_bounds__(row_facets_threads(LOG2NX, sizeof(cplx<Real>)))
rowpass_facets_batched_kernel(const BatchMember* __restrict__ mem, int per, int n_items,
                              int* __restrict__ queue, const cplx<Real>* __restrict__ tw) {
  __shared__ int s_item;
  for (;;) {
    const int item = next_item(queue, &s_item);
    if (item >= n_items) break;
    const int m = item / per, blk = item - m * per;
    const BatchMember& b = mem[m];
    FacetPtrs<Real> fp;
#pragma unroll
    for (int i = 0; i < 9; ++i) fp.p[i] = (Real*)b.fac[i];
    rowpass_facets_body<Real, LOG2NX>((const cplx<Real>*)b.planes, b.gp, fp, tw, blk, per);
  }
}

template <typename Real>
__global__ void __launch_bounds__(acc_threads(sizeof(cplx<Real>)))
accumulate_facets_batched_kernel(const BatchMember* __restrict__ mem, int per, int n_items,
                                 int* __restrict__ queue) {
  __shared__ int s_item;
  for (;;) {
    const int item = next_item(queue, &s_item);
    if (item >= n_items) break;
    const int m = item / per, blk = item - m * per;
    const BatchMember& b = mem[m];
    FacetPtrs<Real> fp;
#pragma unroll
    for (int i = 0; i < 9; ++i) fp.p[i] = (Real*)b.fac[i];
    // (the constants stay scalar here: in vector registers they take this
    // kernel past 128 VGPRs and halve the blocks a CU holds)
    accumulate_facets_body<Real>(fp, b.gp, b.rp, b.wp, (cplx<Real>*)b.Tj, nullptr, blk);
  }
}

template <typename Real>
__global__ void __launch_bounds__(kReduceThreads)
reduce_partials_batched_kernel(const BatchMember* __restrict__ mem, int per, int n_items,
                               int* __restrict__ queue, int n_acc) {
  __shared__ int s_item;
  for (;;) {
    const int item = next_item(queue, &s_item);
    if (item >= n_items) break;
    const int m = item / per, blk = item - m * per;
    const BatchMember& b = mem[m];
    reduce_partials_body<Real>(b.rp, b.wp, (cplx<Real>*)b.Tj, nullptr, n_acc, blk);
  }
}

// ---------------------------------------------------------------------------
// Post-processing: block = (gate group, segment j).  The spectra j and j + 1
// of GB gates are inverse transformed in LDS (radix-2 Stockham, ping-pong)
// and the pulses [j n_fast, (j + 1) n_fast) of those gates are formed.
template <typename Real>
__global__ void __launch_bounds__(256)
segments_to_iq_kernel(const cplx<Real>* __restrict__ T, cplx<Real>* __restrict__ Y, int G, int N,
                      int log2N, int n_fast, int window, int GB,
                      const cplx<Real>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nseq = 2 * GB;
  cplx<Real>* bufA = reinterpret_cast<cplx<Real>*>(smem_raw);
  cplx<Real>* bufB = bufA + (size_t)nseq * N;
  const int g0 = blockIdx.x * GB;
  const int j = blockIdx.y;
  for (int i = threadIdx.x; i < nseq * N; i += blockDim.x) {
    const int sq = i / N, k = i - sq * N;
    const int g = g0 + (sq % GB), jj = j + sq / GB;
    bufA[i] = (g < G) ? T[((size_t)jj * G + g) * N + k] : mk<Real>(0, 0);
  }
  __syncthreads();
  cplx<Real>* src = bufA;
  cplx<Real>* dst = bufB;
  const int half = N / 2;
  for (int Ns = 1; Ns < N; Ns <<= 1) {
    for (int i = threadIdx.x; i < nseq * half; i += blockDim.x) {
      const int sq = i / half, b = i - sq * half;
      const int jb = b & (Ns - 1);
      const cplx<Real>* in = src + (size_t)sq * N;
      cplx<Real>* out = dst + (size_t)sq * N;
      const cplx<Real> a = in[b];
      const cplx<Real> w = tw[2 * Ns + jb];
      const cplx<Real> c = cmul(in[b + half], w);
      const int o = (b - jb) * 2 + jb;
      out[o] = cadd(a, c);
      out[o + Ns] = csub(a, c);
    }
    __syncthreads();
    cplx<Real>* tmp = src;
    src = dst;
    dst = tmp;
  }
  for (int i = threadIdx.x; i < n_fast * GB; i += blockDim.x) {
    const int xl = i / GB, gl = i - xl * GB;
    const int g = g0 + gl;
    if (g >= G) continue;
    const int d0 = xl, d1 = xl - n_fast;
    // eq. (1) with |d| <= n_fast; the numerators are exact integers
    double w0, w1;
    if (window == 0) {
      w0 = __builtin_sqrt((double)(n_fast - d0) / (double)n_fast);
      w1 = __builtin_sqrt((double)(n_fast + d1) / (double)n_fast);
    } else {
      w0 = cos(1.5707963267948966192 * ((double)d0 / (double)n_fast));
      w1 = cos(1.5707963267948966192 * ((double)d1 / (double)n_fast));
    }
    const cplx<Real> s0 = src[(size_t)gl * N + (d0 & (N - 1))];
    const cplx<Real> s1 = src[(size_t)(GB + gl) * N + (d1 & (N - 1))];
    cplx<Real> y = cadd(cscale(s0, (Real)w0), cscale(s1, (Real)w1));
    Y[((size_t)j * n_fast + xl) * G + g] = y;
  }
}

// ---------------------------------------------------------------------------
// Differentiable chain (adjoint of rasterisation and post-processing).

// P[g] = mean_x |Y[x][g]|^2 over the run.  Block = 64 gates x 4 pulse lanes;
// each lane sums its pulses in order (double), lanes are added in order.
template <typename Real>
__global__ void __launch_bounds__(256)
waveform_kernel(const cplx<Real>* __restrict__ Y, int n_pulses, int G, Real* __restrict__ P) {
  __shared__ double part[4][64];
  const int gl = threadIdx.x & 63, xl = threadIdx.x >> 6;
  const int g = blockIdx.x * 64 + gl;
  double acc = 0.0;
  if (g < G) {
    for (int x = xl; x < n_pulses; x += 4) {
      const cplx<Real> y = Y[(size_t)x * G + g];
      acc += (double)y.x * (double)y.x + (double)y.y * (double)y.y;
    }
  }
  part[xl][gl] = acc;
  __syncthreads();
  if (xl == 0 && g < G)
    P[g] = (Real)((((part[0][gl] + part[1][gl]) + part[2][gl]) + part[3][gl]) / (double)n_pulses);
}

// loss = sum_g (P[g] - target[g])^2, one block, fixed summation order.
template <typename Real>
__global__ void __launch_bounds__(256)
waveform_loss_kernel(const Real* __restrict__ P, const Real* __restrict__ target, int G,
                     Real* __restrict__ loss) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    const double d = (double)P[g] - (double)target[g];
    acc += d * d;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (Real)part[0];
}

// Y_bar[x][g] = s * 2 (P[g] - target[g]) * 2 Y[x][g] / n_pulses, s = *scale (or 1).
template <typename Real>
__global__ void __launch_bounds__(256)
waveform_loss_adjoint_kernel(const cplx<Real>* __restrict__ Y, const Real* __restrict__ P,
                             const Real* __restrict__ target, const Real* __restrict__ scale,
                             int n_pulses, int G, cplx<Real>* __restrict__ Ybar) {
  const size_t n = (size_t)n_pulses * G;
  const Real s = scale ? scale[0] : (Real)1;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int g = (int)(i % G);
    const Real f = s * (Real)4 * (P[g] - target[g]) / (Real)n_pulses;
    Ybar[i] = cscale(Y[i], f);
  }
}

// T_bar[j][g][k] = sum_x W(x - c_j) Y_bar[x][g] e^{-2 pi i k ((x - c_j) mod N) / N}:
// the windowed pulses of segment j are folded modulo N (in increasing x per
// bin) and forward transformed in LDS (radix-2 Stockham, ping-pong).
template <typename Real>
__global__ void __launch_bounds__(256)
segments_to_iq_adjoint_kernel(const cplx<Real>* __restrict__ Ybar, cplx<Real>* __restrict__ Tbar,
                              int G, int N, int n_fast, int n_pulses, int window, int GB,
                              const cplx<Real>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<Real>* bufA = reinterpret_cast<cplx<Real>*>(smem_raw);
  cplx<Real>* bufB = bufA + (size_t)GB * N;
  const int g0 = blockIdx.x * GB;
  const int j = blockIdx.y;
  const int c = j * n_fast;
  for (int i = threadIdx.x; i < GB * N; i += blockDim.x) {
    const int gl = i % GB, m = i / GB;
    const int g = g0 + gl;
    double ax = 0.0, ay = 0.0;
    if (g < G) {
      // smallest d > -n_fast with d = m (mod N), then every N up to n_fast - 1
      int d = m - N * ((m + n_fast - 1) / N);
      for (; d < n_fast; d += N) {
        const int x = c + d;
        if (x < 0 || x >= n_pulses) continue;
        const int ad = d < 0 ? -d : d;
        const double w = window == 0 ? __builtin_sqrt((double)(n_fast - ad) / (double)n_fast)
                                     : cos(1.5707963267948966192 * ((double)d / (double)n_fast));
        const cplx<Real> y = Ybar[(size_t)x * G + g];
        ax += w * (double)y.x;
        ay += w * (double)y.y;
      }
    }
    bufA[(size_t)gl * N + m] = mk<Real>((Real)ax, (Real)ay);
  }
  __syncthreads();
  cplx<Real>* src = bufA;
  cplx<Real>* dst = bufB;
  const int half = N / 2;
  for (int Ns = 1; Ns < N; Ns <<= 1) {
    for (int i = threadIdx.x; i < GB * half; i += blockDim.x) {
      const int sq = i / half, b = i - sq * half;
      const int jb = b & (Ns - 1);
      const cplx<Real>* in = src + (size_t)sq * N;
      cplx<Real>* out = dst + (size_t)sq * N;
      const cplx<Real> a = in[b];
      const cplx<Real> w = cconj(tw[2 * Ns + jb]);
      const cplx<Real> cc = cmul(in[b + half], w);
      const int o = (b - jb) * 2 + jb;
      out[o] = cadd(a, cc);
      out[o + Ns] = csub(a, cc);
    }
    __syncthreads();
    cplx<Real>* tmp = src;
    src = dst;
    dst = tmp;
  }
  for (int i = threadIdx.x; i < GB * N; i += blockDim.x) {
    const int gl = i / N, k = i - gl * N;
    const int g = g0 + gl;
    if (g < G) Tbar[((size_t)j * G + g) * N + k] = src[i];
  }
}

// Per-facet gradients of one update: the scatterer and its indices are
// recomputed, C_bar = T_bar[j][g][bin] is gathered and
// dL/dtheta = Re(conj(C_bar) C (d ln a/dtheta + i d phi/dtheta)).
template <typename Real>
__global__ void __launch_bounds__(256)
accumulate_adjoint_kernel(FacetPtrs<Real> fac, GridP gp, RadarP rp,
                          const cplx<Real>* __restrict__ Tbar_j, Real* __restrict__ gh,
                          Real* __restrict__ gsx, Real* __restrict__ gsy) {
  const size_t nfac = (size_t)gp.nx * gp.ny;
  for (size_t f = blockIdx.x * (size_t)blockDim.x + threadIdx.x; f < nfac;
       f += (size_t)gridDim.x * blockDim.x) {
    const int iy = (int)(f >> gp.log2nx);
    const int ix = (int)(f & (size_t)(gp.nx - 1));
    const Real Dx = fac.p[0][f], Dy = fac.p[1][f], h = fac.p[2][f], sx = fac.p[3][f],
               sy = fac.p[4][f];
    cplx<Real> C;
    const int key = scatterer<Real>(rp, gp, ix, iy, Dx, Dy, h, sx, sy, fac.p[5][f], fac.p[6][f],
                                    fac.p[7][f], fac.p[8][f], C);
    Real a = 0, b = 0, cgrad = 0;
    if (key >= 0) {
      const cplx<Real> Cb = Tbar_j[key];   // key = g N + bin indexes [G][N]
      const FacetDeriv D = facet_derivatives<Real>(rp, gp, ix, iy, Dx, Dy, h, sx, sy);
      // Re(conj(Cb) C (l + i p)) = Re(conj(Cb) C) l - Im(conj(Cb) C) p
      const double re = (double)Cb.x * (double)C.x + (double)Cb.y * (double)C.y;
      const double im = (double)Cb.x * (double)C.y - (double)Cb.y * (double)C.x;
      a = (Real)(re * D.lnh - im * D.phih);
      b = (Real)(re * D.lnsx);
      cgrad = (Real)(re * D.lnsy);
    }
    gh[f] = a;
    gsx[f] = b;
    gsy[f] = cgrad;
  }
}

// ---------------------------------------------------------------------------
// Host launch wrappers.  The FFT kernels are instantiated for every
// supported power-of-two side and selected here by log2 of the side.

#define SIMK_COL_SIZES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#define SIMK_ROW_SIZES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13)

// The grid parameters with the plane tile geometry of this precision.
template <typename Real>
static GridP with_tiles(const GridP& gp) {
  return grid_with_tiles<Real>(gp);
}

template <typename Real>
GridP grid_with_tiles(const GridP& gp) {
  GridP g = gp;
  g.tlw = tile_lw(gp.log2ny, sizeof(cplx<Real>));
  g.tlh = tile_lh(gp.log2ny, sizeof(cplx<Real>));
  g.lhw = half_lw(gp.log2nx, gp.log2ny, sizeof(cplx<Real>));
  return g;
}

template <typename Real, int L>
static hipError_t colpass_t(const void* spec, void* planes, const GridP& gp, double t, double dt,
                            const void* tw, bool prepared, hipStream_t st) {
  constexpr int cs = sizeof(cplx<Real>);
  if constexpr (col_lds(L, cs) > kLdsBudget) {
    return hipErrorInvalidValue;
  } else {
    const int strips = (1 << half_lw(gp.log2nx, L, cs)) / col_cpb(L, cs);
    const int blocks = 2 * strips;
    if (prepared)
      hipLaunchKernelGGL((colpass_kernel<Real, L, true>), dim3(blocks),
                         dim3(col_threads(L, cs)), col_lds(L, cs), st, (const cplx<Real>*)spec,
                         (cplx<Real>*)planes, with_tiles<Real>(gp), t, dt, (const cplx<Real>*)tw);
    else
      hipLaunchKernelGGL((colpass_kernel<Real, L, false>), dim3(blocks),
                         dim3(col_threads(L, cs)), col_lds(L, cs), st, (const cplx<Real>*)spec,
                         (cplx<Real>*)planes, with_tiles<Real>(gp), t, dt, (const cplx<Real>*)tw);
    return hipGetLastError();
  }
}

template <typename Real>
hipError_t launch_colpass(const void* spec, void* planes, const GridP& gp, double t, double dt,
                          const void* tw, bool prepared, hipStream_t st) {
  switch (gp.log2ny) {
#define SIMK_CASE(L) \
  case L: return colpass_t<Real, L>(spec, planes, gp, t, dt, tw, prepared, st);
    SIMK_COL_SIZES(SIMK_CASE)
#undef SIMK_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t launch_prepare_spectrum(const void* spec, void* out, const GridP& gp, hipStream_t st) {
  constexpr int cs = sizeof(cplx<Real>);
  const int cpb = col_cpb(gp.log2ny, cs);
  const int lhw = half_lw(gp.log2nx, gp.log2ny, cs);
  const size_t n = (size_t)gp.ny << lhw;
  const size_t want = (n + 255) / 256;
  const int blocks = (int)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(prepare_spectrum_kernel<Real>, dim3(blocks), dim3(256), 0, st,
                     (const cplx<Real>*)spec, (cplx<Real>*)out, gp.nx, gp.ny, lhw, cpb);
  return hipGetLastError();
}

template <typename Real, int L>
static hipError_t rowpass_facets_t(const void* planes, const GridP& gp, const FacetPtrs<Real>& fp,
                                   const void* tw, hipStream_t st) {
  constexpr int cs = sizeof(cplx<Real>);
  const int blocks = (gp.ny + row_facets_rpb(L, cs) - 1) / row_facets_rpb(L, cs);
  hipLaunchKernelGGL((rowpass_facets_kernel<Real, L>), dim3(blocks),
                     dim3(row_facets_threads(L, cs)),
                     row_facets_lds(L, cs), st,
                     (const cplx<Real>*)planes,
                     with_tiles<Real>(gp), fp, (const cplx<Real>*)tw);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_rowpass_facets(const void* planes, const GridP& gp, void* const* out,
                                 const void* tw, hipStream_t st) {
  FacetPtrs<Real> fp;
  for (int i = 0; i < 9; ++i) fp.p[i] = (Real*)out[i];
  switch (gp.log2nx) {
#define SIMK_CASE(L) \
  case L: return rowpass_facets_t<Real, L>(planes, gp, fp, tw, st);
    SIMK_ROW_SIZES(SIMK_CASE)
#undef SIMK_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename Real, int L>
static hipError_t rowpass_accumulate_t(const void* planes, const GridP& gp, const RadarP& rp,
                                       const WinP& wp, void* Tj, int32_t* code, size_t lds,
                                       const void* tw, hipStream_t st) {
  hipLaunchKernelGGL((rowpass_accumulate_kernel<Real, L>), dim3(wp.n_bands), dim3(row_threads(L)),
                     lds, st, (const cplx<Real>*)planes, with_tiles<Real>(gp), rp, wp,
                     (cplx<Real>*)Tj, code, (const cplx<Real>*)tw);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_rowpass_accumulate(const void* planes, const GridP& gp, const RadarP& rp,
                                     const WinP& wp, void* Tj, int32_t* code, size_t lds,
                                     const void* tw, hipStream_t st) {
  switch (gp.log2nx) {
#define SIMK_CASE(L) \
  case L: return rowpass_accumulate_t<Real, L>(planes, gp, rp, wp, Tj, code, lds, tw, st);
    SIMK_ROW_SIZES(SIMK_CASE)
#undef SIMK_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t launch_accumulate_facets(void* const* fac, const GridP& gp, const RadarP& rp,
                                    const WinP& wp, void* Tj, int32_t* code, size_t lds_bytes,
                                    hipStream_t st) {
  FacetPtrs<Real> fp;
  for (int i = 0; i < 9; ++i) fp.p[i] = (Real*)fac[i];
  hipLaunchKernelGGL(accumulate_facets_kernel<Real>, dim3(wp.n_bands),
                     dim3(acc_threads(sizeof(cplx<Real>))), lds_bytes, st,
                     fp, gp, rp, wp, (cplx<Real>*)Tj, code);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_reduce(const RadarP& rp, const WinP& wp, void* Tj, unsigned long long* counters,
                         hipStream_t st) {
  // one double accumulator of N bins per wave, as many waves as 64 KiB allow
  int n_acc = (int)(65536 / ((size_t)rp.N * sizeof(cplx<double>)));
  if (n_acc > kReduceThreads / 64) n_acc = kReduceThreads / 64;
  if (n_acc < 1) n_acc = 1;
  const size_t lds = (size_t)n_acc * rp.N * sizeof(cplx<double>) +
                     (size_t)2 * wp.n_bands * wp.S * sizeof(int);
  hipLaunchKernelGGL(reduce_partials_kernel<Real>, dim3(rp.G), dim3(kReduceThreads), lds, st, rp,
                     wp, (cplx<Real>*)Tj, counters, n_acc);
  return hipGetLastError();
}

// Grid of a persistent launch: the blocks the device holds at once (at the
// kernel's occupancy), at most one per item.
static int persistent_grid(const void* kernel, int threads, size_t lds, int n_items) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess) {
    (void)hipGetLastError();
    cus = 256;
    per_cu = 1;
  }
  if (per_cu < 1) per_cu = 1;
  const long cap = (long)cus * per_cu;
  return (int)(n_items < cap ? n_items : cap);
}

template <typename Real, int L>
static hipError_t colpass_batched_t(const BatchMember* mem, int n_mem, const GridP& gp,
                                    int* queue, const void* tw, hipStream_t st) {
  constexpr int cs = sizeof(cplx<Real>);
  if constexpr (col_lds(L, cs) > kLdsBudget) {
    return hipErrorInvalidValue;
  } else {
    const int strips = (1 << half_lw(gp.log2nx, L, cs)) / col_cpb(L, cs);
    const int per = 2 * strips;
    const int n = n_mem * per;
    const void* k = (const void*)colpass_batched_kernel<Real, L>;
    const int grid = persistent_grid(k, col_threads_e(L, cs, kColBatchE), col_lds(L, cs), n);
    hipLaunchKernelGGL((colpass_batched_kernel<Real, L>), dim3(grid),
                       dim3(col_threads_e(L, cs, kColBatchE)),
                       col_lds(L, cs), st, mem, per, n, queue, (const cplx<Real>*)tw);
    return hipGetLastError();
  }
}

template <typename Real, int L>
static hipError_t rowpass_batched_t(const BatchMember* mem, int n_mem, const GridP& gp,
                                    int* queue, const void* tw, hipStream_t st) {
  constexpr int cs = sizeof(cplx<Real>);
  const int per = (gp.ny + row_facets_rpb(L, cs) - 1) / row_facets_rpb(L, cs);
  const int n = n_mem * per;
  const void* k = (const void*)rowpass_facets_batched_kernel<Real, L>;
  const int grid = persistent_grid(k, row_facets_threads(L, cs), row_facets_lds(L, cs), n);
  hipLaunchKernelGGL((rowpass_facets_batched_kernel<Real, L>), dim3(grid),
                     dim3(row_facets_threads(L, cs)),
                     row_facets_lds(L, cs), st, mem, per, n, queue, (const cplx<Real>*)tw);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_update_batched(const BatchMember* mem, int n_mem, const GridP& gp,
                                 const RadarP& rp, const WinP& wp, size_t acc_lds, int* queues,
                                 const void* tw, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  switch (gp.log2ny) {
#define SIMK_CASE(L) \
  case L: e = colpass_batched_t<Real, L>(mem, n_mem, gp, queues + 0, tw, st); break;
    SIMK_COL_SIZES(SIMK_CASE)
#undef SIMK_CASE
    default: break;
  }
  if (e != hipSuccess) return e;
  e = hipErrorInvalidValue;
  switch (gp.log2nx) {
#define SIMK_CASE(L) \
  case L: e = rowpass_batched_t<Real, L>(mem, n_mem, gp, queues + 1, tw, st); break;
    SIMK_ROW_SIZES(SIMK_CASE)
#undef SIMK_CASE
    default: break;
  }
  if (e != hipSuccess) return e;
  {
    const int per = wp.n_bands, n = n_mem * per;
    const int threads = acc_threads(sizeof(cplx<Real>));
    const void* k = (const void*)accumulate_facets_batched_kernel<Real>;
    const int grid = persistent_grid(k, threads, acc_lds, n);
    hipLaunchKernelGGL(accumulate_facets_batched_kernel<Real>, dim3(grid), dim3(threads),
                       acc_lds, st, mem, per, n, queues + 2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int n_acc = (int)(65536 / ((size_t)rp.N * sizeof(cplx<double>)));
  if (n_acc > kReduceThreads / 64) n_acc = kReduceThreads / 64;
  if (n_acc < 1) n_acc = 1;
  const size_t lds = (size_t)n_acc * rp.N * sizeof(cplx<double>) +
                     (size_t)2 * wp.n_bands * wp.S * sizeof(int);
  const int per = rp.G, n = n_mem * per;
  const void* k = (const void*)reduce_partials_batched_kernel<Real>;
  const int grid = persistent_grid(k, kReduceThreads, lds, n);
  hipLaunchKernelGGL(reduce_partials_batched_kernel<Real>, dim3(grid), dim3(kReduceThreads), lds,
                     st, mem, per, n, queues + 3, n_acc);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_segments_to_iq(const void* T, void* Y, int G, int N, int log2N, int n_fast,
                                 int window, int n_seg, int GB, const void* tw, hipStream_t st) {
  const size_t lds = (size_t)2 * 2 * GB * N * sizeof(cplx<Real>);
  hipLaunchKernelGGL(segments_to_iq_kernel<Real>, dim3((G + GB - 1) / GB, n_seg), dim3(256), lds,
                     st, (const cplx<Real>*)T, (cplx<Real>*)Y, G, N, log2N, n_fast, window, GB,
                     (const cplx<Real>*)tw);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_waveform_loss(const void* Y, int n_pulses, int G, const void* target, void* P,
                                void* loss, hipStream_t st) {
  hipLaunchKernelGGL(waveform_kernel<Real>, dim3((G + 63) / 64), dim3(256), 0, st,
                     (const cplx<Real>*)Y, n_pulses, G, (Real*)P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !loss) return e;
  hipLaunchKernelGGL(waveform_loss_kernel<Real>, dim3(1), dim3(256), 0, st, (const Real*)P,
                     (const Real*)target, G, (Real*)loss);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_waveform_loss_adjoint(const void* Y, const void* P, const void* target,
                                        const void* scale, int n_pulses, int G, void* Ybar,
                                        hipStream_t st) {
  const size_t n = (size_t)n_pulses * G;
  const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL(waveform_loss_adjoint_kernel<Real>, dim3(blocks), dim3(256), 0, st,
                     (const cplx<Real>*)Y, (const Real*)P, (const Real*)target,
                     (const Real*)scale, n_pulses, G, (cplx<Real>*)Ybar);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_segments_to_iq_adjoint(const void* Ybar, void* Tbar, int G, int N, int n_fast,
                                         int n_pulses, int window, int n_spec, int GB,
                                         const void* tw, hipStream_t st) {
  const size_t lds = (size_t)2 * GB * N * sizeof(cplx<Real>);
  hipLaunchKernelGGL(segments_to_iq_adjoint_kernel<Real>, dim3((G + GB - 1) / GB, n_spec),
                     dim3(256), lds, st, (const cplx<Real>*)Ybar, (cplx<Real>*)Tbar, G, N, n_fast,
                     n_pulses, window, GB, (const cplx<Real>*)tw);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_accumulate_adjoint(void* const* fac, const GridP& gp, const RadarP& rp,
                                     const void* Tbar_j, void* gh, void* gsx, void* gsy,
                                     hipStream_t st) {
  FacetPtrs<Real> fp;
  for (int i = 0; i < 9; ++i) fp.p[i] = (Real*)fac[i];
  const size_t n = (size_t)gp.nx * gp.ny;
  const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL(accumulate_adjoint_kernel<Real>, dim3(blocks), dim3(256), 0, st, fp, gp, rp,
                     (const cplx<Real>*)Tbar_j, (Real*)gh, (Real*)gsx, (Real*)gsy);
  return hipGetLastError();
}

// Zero a buffer with a kernel (no memset node when captured into a graph).
__global__ void __launch_bounds__(256) clear_kernel(uint4* __restrict__ p, size_t n16,
                                                    unsigned char* __restrict__ tail, int ntail) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_clear(void* p, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16;
  const int ntail = (int)(bytes - n16 * 16);
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(clear_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint4*)p, n16,
                     (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError();
}

// Allow every kernel `lds` bytes of dynamic LDS (the device limit per block).
template <typename Real>
static hipError_t set_attributes(int lds) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  };
#define SIMK_CASE(L)                                                                           \
  if constexpr (col_lds(L, sizeof(cplx<Real>)) <= kLdsBudget) {                                \
    set((const void*)colpass_kernel<Real, L, false>);                                          \
    set((const void*)colpass_kernel<Real, L, true>);                                           \
  }
  SIMK_COL_SIZES(SIMK_CASE)
#undef SIMK_CASE
#define SIMK_CASE(L)                                   \
  set((const void*)rowpass_facets_kernel<Real, L>);    \
  set((const void*)rowpass_accumulate_kernel<Real, L>);
  SIMK_ROW_SIZES(SIMK_CASE)
#undef SIMK_CASE
  set((const void*)accumulate_facets_kernel<Real>);
  set((const void*)reduce_partials_kernel<Real>);
#define SIMK_CASE(L)                                                      \
  if constexpr (col_lds(L, sizeof(cplx<Real>)) <= kLdsBudget) {           \
    set((const void*)colpass_batched_kernel<Real, L>);                    \
  }
  SIMK_COL_SIZES(SIMK_CASE)
#undef SIMK_CASE
#define SIMK_CASE(L) set((const void*)rowpass_facets_batched_kernel<Real, L>);
  SIMK_ROW_SIZES(SIMK_CASE)
#undef SIMK_CASE
  set((const void*)accumulate_facets_batched_kernel<Real>);
  set((const void*)reduce_partials_batched_kernel<Real>);
  set((const void*)segments_to_iq_kernel<Real>);
  set((const void*)segments_to_iq_adjoint_kernel<Real>);
  return e;
}

hipError_t init_kernel_attributes(int lds) {
  hipError_t e = set_attributes<float>(lds);
  if (e != hipSuccess) return e;
  return set_attributes<double>(lds);
}

#define SIMK_INSTANTIATE(R)                                                                      \
  template hipError_t launch_colpass<R>(const void*, void*, const GridP&, double, double,       \
                                        const void*, bool, hipStream_t);                        \
  template hipError_t launch_prepare_spectrum<R>(const void*, void*, const GridP&, hipStream_t); \
  template hipError_t launch_rowpass_facets<R>(const void*, const GridP&, void* const*,         \
                                               const void*, hipStream_t);                       \
  template hipError_t launch_rowpass_accumulate<R>(const void*, const GridP&, const RadarP&,     \
                                                   const WinP&, void*, int32_t*, size_t,        \
                                                   const void*, hipStream_t);                   \
  template hipError_t launch_accumulate_facets<R>(void* const*, const GridP&, const RadarP&,    \
                                                  const WinP&, void*, int32_t*, size_t,         \
                                                  hipStream_t);                                 \
  template hipError_t launch_reduce<R>(const RadarP&, const WinP&, void*, unsigned long long*,  \
                                       hipStream_t);                                            \
  template hipError_t launch_segments_to_iq<R>(const void*, void*, int, int, int, int, int, int, \
                                               int, const void*, hipStream_t);                  \
  template hipError_t launch_waveform_loss<R>(const void*, int, int, const void*, void*, void*, \
                                              hipStream_t);                                     \
  template hipError_t launch_waveform_loss_adjoint<R>(const void*, const void*, const void*,    \
                                                      const void*, int, int, void*, hipStream_t); \
  template hipError_t launch_segments_to_iq_adjoint<R>(const void*, void*, int, int, int, int,  \
                                                       int, int, int, const void*, hipStream_t); \
  template hipError_t launch_accumulate_adjoint<R>(void* const*, const GridP&, const RadarP&,   \
                                                   const void*, void*, void*, void*, hipStream_t); \
  template hipError_t launch_update_batched<R>(const BatchMember*, int, const GridP&,           \
                                               const RadarP&, const WinP&, size_t, int*,        \
                                               const void*, hipStream_t);                       \
  template GridP grid_with_tiles<R>(const GridP&);

SIMK_INSTANTIATE(float)
SIMK_INSTANTIATE(double)

}  // namespace simk
