// Facet -> scatterer (Algorithm 1: scatterers_complex_amplitudes,
// scatterers_range and the pulse-pair Doppler) and the LDS-private window of
// partial Doppler spectra that implements rasterize() without global atomics.
#pragma once

#include "device_common.hpp"

namespace simk {

// Bilinear interpolation of the antenna table at (u, v) and linear
// interpolation of the NRCS table at theta_l = atan(sqrt(tan^2)) (cell index
// from the fractional grid coordinate, the last node belonging to the cell
// before it, zero outside the table); a missing table uses its closed form.
// Returns sqrt(sigma0 A) G.
template <typename Real>
__device__ __forceinline__ cplx<Real> tabulated_amplitude(const TabP& T, const RadarP& rp,
                                                          Real tan2, Real sec2, Real sin2, Real u,
                                                          Real v, Real area) {
  Real sigma0;
  if (T.nrcs) {
    const Real* s = (const Real*)T.nrcs;
    const Real f = atan(approx_sqrt(tan2)) * (Real)T.inv_dtheta;
    const int n = T.n_theta;
    sigma0 = (Real)0;
    if (f >= (Real)0 && f <= (Real)(n - 1)) {
      const int i = min((int)f, n - 2);
      const Real w = f - (Real)i;
      sigma0 = ((Real)1 - w) * s[i] + w * s[i + 1];
    }
  } else {
    sigma0 = (Real)rp.fresnel_over_mss * sec2 * sec2 * exp(-(Real)rp.inv_mss * tan2);
  }
  const Real amp = approx_sqrt(sigma0 * area);
  if (!T.ant) {
    const Real ga = exp(-(Real)rp.two_over_gamma * sin2);
    return mk<Real>(amp * ga, (Real)0);
  }
  const cplx<Real>* a = (const cplx<Real>*)T.ant;
  const Real fu = (u - (Real)T.u0) * (Real)T.inv_du;
  const Real fv = (v - (Real)T.v0) * (Real)T.inv_dv;
  if (!(fu >= (Real)0 && fu <= (Real)(T.nu - 1) && fv >= (Real)0 && fv <= (Real)(T.nv - 1)))
    return mk<Real>((Real)0, (Real)0);
  const int iu = min((int)fu, T.nu - 2), iv = min((int)fv, T.nv - 2);
  const Real wu = fu - (Real)iu, wv = fv - (Real)iv;
  const cplx<Real>* r0 = a + (size_t)iv * T.nu + iu;
  const cplx<Real>* r1 = r0 + T.nu;
  const Real w00 = ((Real)1 - wv) * ((Real)1 - wu), w01 = ((Real)1 - wv) * wu;
  const Real w10 = wv * ((Real)1 - wu), w11 = wv * wu;
  const Real gx = w00 * r0[0].x + w01 * r0[1].x + w10 * r1[0].x + w11 * r1[1].x;
  const Real gy = w00 * r0[0].y + w01 * r0[1].y + w10 * r1[0].y + w11 * r1[1].y;
  return mk<Real>(amp * gx, amp * gy);
}

// Scatterer of one facet.  Returns g * N + bin for an illuminated facet, or
// a negative drop code (tested in the order nonfinite, folded, out of
// window, backfacing).  The range, gate, Doppler bin and carrier phase are
// evaluated in double with the operation order fixed below and no fused
// multiply-add, so that the integer decisions are reproducible bit for bit
// by any IEEE double implementation of the same expressions.  The amplitude
// (geometric-optics NRCS, Gaussian two-way beam, (H/R)^2, facet area) is
// evaluated in Real.
template <typename Real>
__device__ __forceinline__ int scatterer(const RadarP& rp, const GridP& gp, int ix, int iy,
                                         Real Dx, Real Dy, Real h, Real sx, Real sy, Real jac,
                                         Real dDx, Real dDy, Real dh, cplx<Real>& C) {
  C = mk<Real>((Real)0, (Real)0);
  if (!(__builtin_isfinite(Dx) && __builtin_isfinite(Dy) && __builtin_isfinite(h) &&
        __builtin_isfinite(sx) && __builtin_isfinite(sy) && __builtin_isfinite(jac) &&
        __builtin_isfinite(dDx) && __builtin_isfinite(dDy) && __builtin_isfinite(dh)))
    return kCodeNonfinite;
  if (!(jac > (Real)0)) return kCodeFolded;

  double ddx, ddy, ddz, r, xi, q, frac;
  int g, kbin;
  {
#pragma clang fp contract(off)
    const double x0 = gp.x_origin + (double)ix * gp.dx;
    const double y0 = gp.y_origin + (double)iy * gp.dy;
    const double px = x0 + (double)Dx;
    const double py = y0 + (double)Dy;
    const double pz = (double)h;
    ddx = rp.sat_x - px;
    ddy = rp.sat_y1 - py;
    ddz = rp.altitude - pz;
    r = __builtin_sqrt((ddx * ddx + ddy * ddy) + ddz * ddz);
    xi = (r - rp.window_start) / rp.gate_spacing;
    if (!(xi >= 0.0 && xi < (double)rp.G)) return kCodeOutOfWindow;
    q = ((-(double)sx) * ddx - (double)sy * ddy) + ddz;
    if (!(q > 0.0)) return kCodeBackfacing;
    const double px2 = px + (double)dDx;
    const double py2 = py + (double)dDy;
    const double pz2 = pz + (double)dh;
    const double ex = rp.sat_x - px2;
    const double ey = rp.sat_y2 - py2;
    const double ez = rp.altitude - pz2;
    const double r2 = __builtin_sqrt((ex * ex + ey * ey) + ez * ez);
    const double u_raw = -(r2 - r) * rp.k2;
    const double u = u_raw - __builtin_floor(u_raw + 0.5);
    kbin = (int)__builtin_floor((double)rp.N * u + 0.5) & (rp.N - 1);
    g = (int)__builtin_floor(xi);
    const double cyc = r * rp.k2;
    frac = cyc - __builtin_floor(cyc);
  }
  // local incidence: tan^2 = |d x m|^2 / (d . m)^2 with m = (-sx, -sy, 1);
  // the cross product is formed in double (it differences ~1e5 m terms),
  // the rest in Real
  const double msx = -(double)sx, msy = -(double)sy;
  const Real cx = (Real)(ddy - ddz * msy);
  const Real cy = (Real)(ddz * msx - ddx);
  const Real cz = (Real)(ddx * msy - ddy * msx);
  const Real qr = (Real)q;
  const Real iq = approx_rcp(qr);
  const Real tan2 = (cx * cx + cy * cy + cz * cz) * (iq * iq);
  const Real sec2 = (Real)1 + tan2;
  const Real ir = approx_rcp((Real)r);
  const Real fx = (Real)ddx, fy = (Real)ddy;
  const Real sin2 = (fx * fx + fy * fy) * (ir * ir);
  const Real hr = (Real)rp.altitude * ir;
  if (rp.tab) {
    // tabulated NRCS and/or antenna pattern (complex amplitude)
    const Real area = jac * approx_sqrt((Real)1 + sx * sx + sy * sy) * (Real)rp.cell_area;
    const cplx<Real> a = tabulated_amplitude<Real>(*rp.tab, rp, tan2, sec2, sin2,
                                                   (Real)(-ddx / r), (Real)(-ddy / r), area);
    Real sn, cs;
    sincos_pi((Real)2 * (Real)frac, &sn, &cs);
    const Real h2 = hr * hr;
    C = cmul(mk<Real>(a.x * h2, a.y * h2), mk<Real>(cs, -sn));
    return g * rp.N + kbin;
  }
  // a = sqrt(sigma0 A) Ga (H/R)^2 with sigma0 = (|G0|^2/mss) sec^4 exp(-tan^2/mss)
  // and Ga = exp(-(2/gamma) sin^2): one exponential for both
  const Real area = jac * approx_sqrt((Real)1 + sx * sx + sy * sy) * (Real)rp.cell_area;
  const Real ex = -(Real)0.5 * (Real)rp.inv_mss * tan2 - (Real)rp.two_over_gamma * sin2;
  const Real a = approx_sqrt((Real)rp.fresnel_over_mss * area) * sec2 * exp(ex) * hr * hr;
  Real sn, cs;
  sincos_pi((Real)2 * (Real)frac, &sn, &cs);
  C = mk<Real>(a * cs, -a * sn);
  return g * rp.N + kbin;
}

// ---------------------------------------------------------------------------
// Window of partial spectra private to one workgroup (a "band" of facets).
//
// The window holds all G gates and WK consecutive Doppler bins starting at
// bin k0 (cyclically).  Facets are added with LDS atomics.  When a chunk of
// facets does not fit the current bins, the window is flushed to the next of
// the band's S partial slots in the workspace and re-centred on the chunk;
// a chunk wider than WK bins is processed in several windows.  Slots are
// later summed per gate, in slot order, by the reduce kernel (a fixed
// association over the bands; within a window cell the atomics add in
// scheduling order).  A band that runs out of slots merges the extra windows
// into T with atomics and counts them (window_overflow).
//
// LDS state (ints): 0 active, 1 k0, 2 g_lo, 3 g_hi, 4 next slot, 5 dirty.

template <typename Real>
struct WinCtx {
  cplx<Real>* win;   // LDS [G][WK]
  int* st;           // LDS state[8]
  int* red;          // LDS scratch[kWinRedInts]
  cplx<Real>* Tj;    // T_fast[j] (overflow path only)
  int band;
};

template <typename Real>
__device__ __forceinline__ void lds_add(cplx<Real>* p, cplx<Real> v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}

// Value of lane l xor 1 (CTRL 0xB1) or l xor 2 (CTRL 0x4E) within a quad.
template <int CTRL>
__device__ __forceinline__ int quad_swap(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float quad_swap(float x) {
  return __builtin_bit_cast(float, quad_swap<CTRL>(__builtin_bit_cast(int, x)));
}
template <int CTRL>
__device__ __forceinline__ double quad_swap(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)quad_swap<CTRL>((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)quad_swap<CTRL>((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

// Adds v to win[idx] for every lane with idx >= 0; every lane of the wave
// must call it.  LDS atomics cost per adding lane, and neighbouring facets
// (neighbouring lanes) mostly fall into the same gate and Doppler bin: lanes
// l and l xor 1, then l and l xor 2, with the same index are merged into the
// lower one first.
template <typename Real>
__device__ __forceinline__ void quad_lds_add(cplx<Real>* win, int idx, cplx<Real> v) {
  const int lane = threadIdx.x & 63;
  {
    const int pi = quad_swap<0xB1>(idx);
    const Real px = quad_swap<0xB1>(v.x), py = quad_swap<0xB1>(v.y);
    if (idx >= 0 && pi == idx) {
      if (lane & 1) {
        idx = -1;
      } else {
        v.x += px;
        v.y += py;
      }
    }
  }
  {
    const int pi = quad_swap<0x4E>(idx);
    const Real px = quad_swap<0x4E>(v.x), py = quad_swap<0x4E>(v.y);
    if (idx >= 0 && pi == idx) {
      if (lane & 2) {
        idx = -1;
      } else {
        v.x += px;
        v.y += py;
      }
    }
  }
  if (idx >= 0) lds_add(&win[idx], v);
}

template <typename Real>
__device__ void win_init(const WinCtx<Real>& w, const RadarP& rp, const WinP& wp) {
  const int n = rp.G * wp.WK;
  for (int i = threadIdx.x; i < n; i += blockDim.x) w.win[i] = mk<Real>((Real)0, (Real)0);
  if (threadIdx.x == 0) {
    w.st[0] = (wp.WK >= rp.N) ? 1 : 0;
    w.st[1] = 0;
    w.st[2] = 0x7fffffff;
    w.st[3] = -1;
    w.st[4] = 0;
    w.st[5] = 0;
  }
  __syncthreads();
}

template <typename Real>
__device__ void win_flush(const WinCtx<Real>& w, const RadarP& rp, const WinP& wp,
                          uint32_t& overflow) {
  const int k0 = w.st[1], glo = w.st[2], ghi = w.st[3], slot = w.st[4];
  const int WK = wp.WK;
  if (ghi >= glo) {
    const int n = (ghi - glo + 1) * WK;
    cplx<Real>* src = w.win + glo * WK;
    if (slot < wp.S) {
      const size_t s = (size_t)w.band * wp.S + slot;
      cplx<Real>* dst = (cplx<Real>*)wp.part + s * (size_t)rp.G * WK + (size_t)glo * WK;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        dst[i] = src[i];
        src[i] = mk<Real>((Real)0, (Real)0);
      }
      if (threadIdx.x == 0) wp.hdr[s] = make_int4(1, k0, glo, ghi);
    } else {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const cplx<Real> v = src[i];
        if (v.x != (Real)0 || v.y != (Real)0) {
          const int g = glo + (i >> wp.log2WK);
          const int k = (k0 + (i & (WK - 1))) & (rp.N - 1);
          atomicAdd(&w.Tj[(size_t)g * rp.N + k].x, v.x);
          atomicAdd(&w.Tj[(size_t)g * rp.N + k].y, v.y);
        }
        src[i] = mk<Real>((Real)0, (Real)0);
      }
      if (threadIdx.x == 0) overflow++;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    w.st[4] = (ghi >= glo) ? slot + 1 : slot;
    w.st[5] = 0;
    w.st[2] = 0x7fffffff;
    w.st[3] = -1;
  }
  __syncthreads();
}

// Add one chunk of facets (E per thread, key < 0 for dropped facets).
template <typename Real, int E>
__device__ void win_add(const WinCtx<Real>& w, const RadarP& rp, const WinP& wp,
                        const int* key, const cplx<Real>* cv, uint32_t& overflow) {
  const int N = rp.N, WK = wp.WK, lgN = rp.log2N;
  if (WK >= N) {
    int gmin = 0x7fffffff, gmax = -1, d0 = 0, d1 = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int g = key[e] >> lgN;
      quad_lds_add(w.win, key[e] >= 0 ? g * WK + (key[e] & (N - 1)) : -1, cv[e]);
      if (key[e] >= 0) {
        gmin = min(gmin, g);
        gmax = max(gmax, g);
      }
    }
    block_minmax2(gmin, gmax, d0, d1, w.red);
    if (threadIdx.x == 0 && gmax >= 0) {
      w.st[2] = min(w.st[2], gmin);
      w.st[3] = max(w.st[3], gmax);
      w.st[5] = 1;
    }
    __syncthreads();
    return;
  }
  int A;
  if (w.st[0]) {
    A = (w.st[1] + WK / 2) & (N - 1);
  } else {
    int kmax = -1;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (key[e] >= 0) kmax = max(kmax, key[e] & (N - 1));
    A = block_max(kmax, w.red);
    if (A < 0) return;
  }
  int rel[E];
  int rmin = 0x7fffffff, rmax = -0x7fffffff, gmin = 0x7fffffff, gmax = -1;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    rel[e] = 0;
    if (key[e] >= 0) {
      rel[e] = (((key[e] & (N - 1)) - A + N / 2) & (N - 1)) - N / 2;
      rmin = min(rmin, rel[e]);
      rmax = max(rmax, rel[e]);
      const int g = key[e] >> lgN;
      gmin = min(gmin, g);
      gmax = max(gmax, g);
    }
  }
  // (rmin, rmax) as a min/max pair; (gmin, gmax) as the second pair
  block_minmax2(rmin, rmax, gmin, gmax, w.red);
  if (gmax < 0) return;
  const int active = w.st[0];
  if (active && rmin >= -WK / 2 && rmax < WK / 2) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      quad_lds_add(w.win, key[e] >= 0 ? (key[e] >> lgN) * WK + rel[e] + WK / 2 : -1, cv[e]);
    __syncthreads();
    if (threadIdx.x == 0) {
      w.st[2] = min(w.st[2], gmin);
      w.st[3] = max(w.st[3], gmax);
      w.st[5] = 1;
    }
    __syncthreads();
    return;
  }
  if (active && w.st[5]) win_flush(w, rp, wp, overflow);
  if (rmax - rmin + 1 <= WK) {
    const int c0 = ((rmin + rmax + 1) >> 1) - WK / 2;
#pragma unroll
    for (int e = 0; e < E; ++e)
      quad_lds_add(w.win, key[e] >= 0 ? (key[e] >> lgN) * WK + rel[e] - c0 : -1, cv[e]);
    __syncthreads();
    if (threadIdx.x == 0) {
      w.st[0] = 1;
      w.st[1] = (A + c0) & (N - 1);
      w.st[2] = gmin;
      w.st[3] = gmax;
      w.st[5] = 1;
    }
    __syncthreads();
    return;
  }
  for (int c0 = rmin; c0 <= rmax; c0 += WK) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      quad_lds_add(w.win,
                   key[e] >= 0 && rel[e] >= c0 && rel[e] < c0 + WK
                       ? (key[e] >> lgN) * WK + rel[e] - c0
                       : -1,
                   cv[e]);
    __syncthreads();
    if (threadIdx.x == 0) {
      w.st[0] = 1;
      w.st[1] = (A + c0) & (N - 1);
      w.st[2] = gmin;
      w.st[3] = gmax;
      w.st[5] = 1;
    }
    __syncthreads();
    if (c0 + WK <= rmax) win_flush(w, rp, wp, overflow);
  }
}

// Flush what is left and invalidate the band's unused slots.
template <typename Real>
__device__ void win_finish(const WinCtx<Real>& w, const RadarP& rp, const WinP& wp,
                           uint32_t& overflow) {
  if (w.st[5]) win_flush(w, rp, wp, overflow);
  const int used = w.st[4];
  for (int s = used + (int)threadIdx.x; s < wp.S; s += blockDim.x)
    wp.hdr[(size_t)w.band * wp.S + s] = make_int4(0, 0, 0, -1);
}

// Per-thread facet counters -> band totals in the workspace.
__device__ __forceinline__ void store_band_counts(const WinP& wp, int band, const uint32_t* c,
                                                  uint32_t overflow, int* red) {
  // overflow is nonzero on thread 0 only, so its block sum is the count
  uint32_t v[6] = {c[0], c[1], c[2], c[3], c[4], overflow};
  const int wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    v[i] = wave_sum(v[i]);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int i = 0; i < 6; ++i) red[i * 16 + wv] = (int)v[i];
  __syncthreads();
  if (threadIdx.x < 6) {
    uint32_t s = 0;
    for (int w = 0; w < nw; ++w) s += (uint32_t)red[threadIdx.x * 16 + w];
    wp.bandcnt[(size_t)band * 8 + threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void count_code(int code, uint32_t* c) {
  // c: illuminated, out_of_window, folded, backfacing, nonfinite
  if (code >= 0) c[0]++;
  else if (code == kCodeOutOfWindow) c[1]++;
  else if (code == kCodeFolded) c[2]++;
  else if (code == kCodeBackfacing) c[3]++;
  else c[4]++;
}

}  // namespace simk

namespace simk {

// Derivatives of the scatterer of one illuminated facet with respect to its
// height and slopes, for the adjoint: with C = a exp(i phi),
// dC/dtheta = C (d ln a / dtheta + i d phi / dtheta).  The geometry is
// recomputed from the facet fields exactly as the forward does.  Terms:
//   ln a = 1/2 ln(|G0|^2 A / mss) + ln(1 + tan^2) - tan^2/(2 mss)
//          - (2/gamma) sin^2 + 2 ln H - 2 ln R,   phi = -2 pi R k2 (mod 2 pi)
//   tan^2 = |c|^2/q^2, c = d x m, q = d . m, m = (-sx, -sy, 1), d = S - P,
//   dd/dh = (0, 0, -1), dm/dsx = (-1, 0, 0), dm/dsy = (0, -1, 0),
//   ln A = ln jac + 1/2 ln(1 + sx^2 + sy^2), dR/dh = -d_z / R.
struct FacetDeriv {
  double lnh, phih;   // d ln a / dh, d phi / dh
  double lnsx, lnsy;  // d ln a / dsx, d ln a / dsy (phi does not depend on slopes)
};

template <typename Real>
__device__ __forceinline__ FacetDeriv facet_derivatives(const RadarP& rp, const GridP& gp, int ix,
                                                        int iy, Real Dx, Real Dy, Real h, Real sx,
                                                        Real sy) {
  const double x0 = gp.x_origin + (double)ix * gp.dx;
  const double y0 = gp.y_origin + (double)iy * gp.dy;
  const double dx = rp.sat_x - (x0 + (double)Dx);
  const double dy = rp.sat_y1 - (y0 + (double)Dy);
  const double dz = rp.altitude - (double)h;
  const double r = sqrt((dx * dx + dy * dy) + dz * dz);
  const double sxd = (double)sx, syd = (double)sy;
  const double mx = -sxd, my = -syd;
  const double cx = dy - dz * my, cy = dz * mx - dx, cz = dx * my - dy * mx;
  const double q = dx * mx + dy * my + dz;
  const double c2 = cx * cx + cy * cy + cz * cz;
  const double q2 = q * q;
  const double tan2 = c2 / q2;
  const double sin2 = (dx * dx + dy * dy) / (r * r);
  const double s2 = 1.0 + sxd * sxd + syd * syd;
  const double k_tan = 1.0 / (1.0 + tan2) - 0.5 * rp.inv_mss;   // d ln a / d tan^2
  auto dtan = [&](double dcx, double dcy, double dcz, double dq) {
    return 2.0 * (cx * dcx + cy * dcy + cz * dcz) / q2 - 2.0 * c2 * dq / (q2 * q);
  };
  FacetDeriv D;
  const double dR = -dz / r;
  D.lnh = k_tan * dtan(-syd, sxd, 0.0, -1.0) - rp.two_over_gamma * (-2.0 * sin2 * dR / r) -
          2.0 * dR / r;
  D.phih = -6.283185307179586476925 * rp.k2 * dR;
  D.lnsx = 0.5 * sxd / s2 + k_tan * dtan(0.0, -dz, dy, -dx);
  D.lnsy = 0.5 * syd / s2 + k_tan * dtan(dz, 0.0, -dx, -dy);
  return D;
}

}  // namespace simk
