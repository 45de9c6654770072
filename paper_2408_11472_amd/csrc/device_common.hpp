// Device-side building blocks shared by the kernels: complex arithmetic,
// register-resident small DFTs, a Stockham FFT over LDS for one sequence,
// block reductions and the kernel parameter blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace simk {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T x, T y) {
  cplx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return mk(a.x, -a.y); }

// Reciprocal, square root and reciprocal square root for amplitude-type
// quantities and spectral multipliers: the hardware approximations (within
// about 1 ulp) in float, the library's double routines in double.
__device__ __forceinline__ float approx_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double approx_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float approx_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double approx_sqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float approx_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double approx_rsqrt(double x) { return rsqrt(x); }

// sin(pi x), cos(pi x) in the precision of the argument.
__device__ __forceinline__ void sincos_pi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincos_pi(double x, double* s, double* c) { sincospi(x, s, c); }

// 1/sqrt(x) in double from the float estimate and two Newton steps
// (relative error ~1e-16 for x in the float range).
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = (double)__builtin_amdgcn_rsqf((float)x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Twiddle table: for every power of two M <= kTwMax the M roots
// e^{+2 pi i m / M}, m < M, stored contiguously at offset M (entries
// [M, 2M)), so each transform size reads a compact slice.
constexpr int kTwLog2 = 15;
constexpr int kTwMax = 1 << kTwLog2;
constexpr int kTwEntries = 2 * kTwMax;

// v * e^{DIR 2 pi i k16 / 16} for a compile-time k16 (after unrolling).
template <typename T, int DIR>
__device__ __forceinline__ cplx<T> rot16(cplx<T> v, int k16) {
  // cos and sin of 2 pi k / 16 for k = 0..4
  constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
  constexpr double R2 = 0.70710678118654752440;  // cos(pi/4)
  k16 &= 15;
  const T s = (T)DIR;
  switch (k16) {
    case 0: return v;
    case 4: return mk<T>(-s * v.y, s * v.x);                       // * (+-i)
    case 8: return mk<T>(-v.x, -v.y);
    case 12: return mk<T>(s * v.y, -s * v.x);                      // * (-+i)
    case 2: return mk<T>((T)R2 * (v.x - s * v.y), (T)R2 * (v.y + s * v.x));
    case 6: return mk<T>((T)R2 * (-v.x - s * v.y), (T)R2 * (-v.y + s * v.x));
    case 10: return mk<T>((T)R2 * (-v.x + s * v.y), (T)R2 * (-v.y - s * v.x));
    case 14: return mk<T>((T)R2 * (v.x + s * v.y), (T)R2 * (v.y - s * v.x));
    default: break;
  }
  // general odd k: cos/sin from the octant table
  T c, sn;
  switch (k16) {
    case 1: c = (T)C1; sn = (T)S1; break;
    case 3: c = (T)S1; sn = (T)C1; break;
    case 5: c = -(T)S1; sn = (T)C1; break;
    case 7: c = -(T)C1; sn = (T)S1; break;
    case 9: c = -(T)C1; sn = -(T)S1; break;
    case 11: c = -(T)S1; sn = -(T)C1; break;
    case 13: c = (T)S1; sn = -(T)C1; break;
    default: c = (T)C1; sn = -(T)S1; break;  // 15
  }
  sn *= s;
  return mk<T>(v.x * c - v.y * sn, v.x * sn + v.y * c);
}

__host__ __device__ constexpr int bitrev_c(int i, int n) {
  int r = 0;
  for (int b = 1; b < n; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register DFT of size R (2, 4, 8, 16), natural order in and out:
// X[k] = sum_n x[n] e^{DIR 2 pi i n k / R}.  Iterative radix-2 DIT.
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft(cplx<T>* v) {
  cplx<T> w[R];
#pragma unroll
  for (int i = 0; i < R; ++i) w[i] = v[bitrev_c(i, R)];
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        cplx<T> a = w[i + k];
        cplx<T> b = rot16<T, DIR>(w[i + k + len / 2], k * (16 / len));
        w[i + k] = cadd(a, b);
        w[i + k + len / 2] = csub(a, b);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = w[i];
}

// LDS index with one padding element every 16 (breaks the stride-16
// bank pattern of the first Stockham stage).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// Compile-time plan of an N = 2^LOG2N point transform held as E values per
// thread (E in {4, 8, 16}): an optional first stage of radix
// 2^(LOG2N mod log2 E), then radix-E stages.
template <int LOG2N, int E>
struct FftPlan {
  static_assert(E == 4 || E == 8 || E == 16, "4, 8 or 16 values per thread");
  static constexpr int LE = (E == 16) ? 4 : (E == 8) ? 3 : 2;
  static constexpr int REM = LOG2N % LE;
  static constexpr int NSTAGES = LOG2N / LE + (REM ? 1 : 0);
  static constexpr int radix(int s) { return (s == 0 && REM) ? (1 << REM) : E; }
  static constexpr int ns(int s) {
    int n = 1;
    for (int i = 0; i < s; ++i) n *= radix(i);
    return n;
  }
};

// One Stockham radix-R stage on a sequence of N points held as E values per
// thread by T = N/E threads: register slot m holds position tid + m*T.
// Butterfly q (q < E/R) of this thread is b = tid + q*T with inputs at
// slots q + r*(E/R); its outputs go to the self-sorting positions
// (b - j) * R + j + r * Ns, j = b mod Ns.  On the last stage those positions
// coincide with the register slots, so the data stays in registers.  LDS
// element i of the sequence lives at lds[lpad(i) * LS].
// Twiddles: with FULL == false, tw is the global table of slices (entry
// M + m = e^{2 pi i m / M}); with FULL == true, tw holds the N entries
// e^{2 pi i k / N} of this transform size (an LDS copy), and the size-M
// slice is read with stride N / M.
// PP (ping-pong): exchanges alternate between lds and lds2 (stage parity
// SI), so a stage's reads need no closing barrier: the next stage writes the
// other buffer, and the one after that is behind the next stage's barrier.
// The caller separates consecutive transforms by a barrier.
template <typename T, int N, int E, int R, int Ns, bool LAST, int LS, int DIR, bool FULL,
          bool PP, int SI>
__device__ __forceinline__ void stockham_stage(cplx<T>* v, cplx<T>* lds0, cplx<T>* lds2, int tid,
                                               const cplx<T>* __restrict__ tw) {
  cplx<T>* lds = (PP && (SI & 1)) ? lds2 : lds0;
  constexpr int Tn = N / E;
  constexpr int TS = FULL ? N / (Ns * R) : 1;     // stride of the slice in the table
#pragma unroll
  for (int q = 0; q < E / R; ++q) {
    cplx<T> u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[q + r * (E / R)];
    const int b = tid + q * Tn;
    const int j = b & (Ns - 1);
    if (Ns > 1) {
      // u[r] *= w^r with w = e^{DIR 2 pi i j / (Ns R)}: w and w^4 are read
      // from the size-(Ns R) slice of the table, the other powers are formed
      // with at most three products and applied at once, so no power is
      // kept live beyond its use.
      const cplx<T>* twm = FULL ? tw : tw + Ns * R;
      cplx<T> w1 = twm[(unsigned)(j * TS)];
      if (DIR < 0) w1.y = -w1.y;
      const cplx<T> w2 = cmul(w1, w1);
      const cplx<T> w3 = cmul(w2, w1);
      u[1] = cmul(u[1], w1);
      if (R > 2) u[2] = cmul(u[2], w2);
      if (R > 3) u[3] = cmul(u[3], w3);
      if (R > 4) {
        cplx<T> w4 = twm[(unsigned)(4 * j * TS)];
        if (DIR < 0) w4.y = -w4.y;
        u[4] = cmul(u[4], w4);
        u[5] = cmul(u[5], cmul(w4, w1));
        u[6] = cmul(u[6], cmul(w4, w2));
        u[7] = cmul(u[7], cmul(w4, w3));
        if (R > 8) {
          const cplx<T> w8 = cmul(w4, w4);
          u[8] = cmul(u[8], w8);
          u[9] = cmul(u[9], cmul(w8, w1));
          u[10] = cmul(u[10], cmul(w8, w2));
          u[11] = cmul(u[11], cmul(w8, w3));
          const cplx<T> w12 = cmul(w8, w4);
          u[12] = cmul(u[12], w12);
          u[13] = cmul(u[13], cmul(w12, w1));
          u[14] = cmul(u[14], cmul(w12, w2));
          u[15] = cmul(u[15], cmul(w12, w3));
        }
      }
    }
    dft<T, R, DIR>(u);
    if (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * (E / R)] = u[r];
    } else {
      const int base = (b - j) * R + j;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lpad(base + r * Ns) * LS] = u[r];
    }
  }
  if (!LAST) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[lpad(tid + m * Tn) * LS];
    if (!PP) __syncthreads();
  }
}

template <typename T, int LOG2N, int E, int LS, int DIR, bool FULL, bool PP, int S>
__device__ __forceinline__ void fft_stages(cplx<T>* v, cplx<T>* lds, cplx<T>* lds2, int tid,
                                           const cplx<T>* __restrict__ tw) {
  using P = FftPlan<LOG2N, E>;
  if constexpr (S < P::NSTAGES) {
    stockham_stage<T, (1 << LOG2N), E, P::radix(S), P::ns(S), S == P::NSTAGES - 1, LS, DIR,
                   FULL, PP, S>(v, lds, lds2, tid, tw);
    fft_stages<T, LOG2N, E, LS, DIR, FULL, PP, S + 1>(v, lds, lds2, tid, tw);
  }
}

// Unnormalised DFT of one sequence of N = 2^LOG2N points (N >= E),
// X[k] = sum_n x[n] e^{DIR 2 pi i n k / N}, held in registers as E values
// per thread in slot order (slot m = position tid + m*N/E) on entry and on
// exit.  lds points at this sequence's LDS region (lpad(N) elements, element
// stride LS).  Every thread of the block must call it (barriers).
template <typename T, int LOG2N, int E, int LS, int DIR, bool FULL = false, bool PP = false>
__device__ __forceinline__ void fft_seq(cplx<T>* v, cplx<T>* lds, int tid,
                                        const cplx<T>* __restrict__ tw,
                                        cplx<T>* lds2 = nullptr) {
  static_assert((1 << LOG2N) >= E, "transform shorter than the values per thread");
  fft_stages<T, LOG2N, E, LS, DIR, FULL, PP, 0>(v, lds, lds2, tid, tw);
}

// ---------------------------------------------------------------------------
// Block reductions (blockDim.x a multiple of 64, at most 1024 threads).
// Within a wave the lanes are combined with DPP moves (quad swaps, half-row
// and row mirrors: each row of 16 lanes then holds its reduction) and the
// four rows are read with readlane, so no LDS instruction is issued.
template <typename T, typename Op>
__device__ __forceinline__ T row16_reduce(T v, Op op) {
  v = op(v, (T)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = op(v, (T)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = op(v, (T)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = op(v, (T)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  return v;
}
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
  v = row16_reduce(v, op);
  const T a = (T)__builtin_amdgcn_readlane((int)v, 0), b = (T)__builtin_amdgcn_readlane((int)v, 16);
  const T c = (T)__builtin_amdgcn_readlane((int)v, 32), d = (T)__builtin_amdgcn_readlane((int)v, 48);
  return op(op(a, b), op(c, d));
}
struct OpMin { __device__ int operator()(int a, int b) const { return min(a, b); } };
struct OpMax { __device__ int operator()(int a, int b) const { return max(a, b); } };
struct OpAdd { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; } };

__device__ __forceinline__ int wave_min(int v) { return wave_reduce(v, OpMin()); }
__device__ __forceinline__ int wave_max(int v) { return wave_reduce(v, OpMax()); }
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return wave_reduce(v, OpAdd()); }

// Reduce four ints (two mins, two maxes) over the block; scratch holds
// 4 * 16 ints.  Result broadcast to every thread: lane l of each wave reads
// wave l's partials and the first 16 lanes are reduced with DPP.
__device__ __forceinline__ void block_minmax2(int& amin, int& amax, int& bmin, int& bmax,
                                              int* scratch) {
  amin = wave_min(amin);
  amax = wave_max(amax);
  bmin = wave_min(bmin);
  bmax = wave_max(bmax);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    scratch[wv] = amin;
    scratch[16 + wv] = amax;
    scratch[32 + wv] = bmin;
    scratch[48 + wv] = bmax;
  }
  __syncthreads();
  const bool in = lane < nw;
  int p0 = in ? scratch[lane] : 0x7fffffff;
  int p1 = in ? scratch[16 + lane] : -0x7fffffff - 1;
  int p2 = in ? scratch[32 + lane] : 0x7fffffff;
  int p3 = in ? scratch[48 + lane] : -0x7fffffff - 1;
  p0 = row16_reduce(p0, OpMin());
  p1 = row16_reduce(p1, OpMax());
  p2 = row16_reduce(p2, OpMin());
  p3 = row16_reduce(p3, OpMax());
  amin = __builtin_amdgcn_readlane(p0, 0);
  amax = __builtin_amdgcn_readlane(p1, 0);
  bmin = __builtin_amdgcn_readlane(p2, 0);
  bmax = __builtin_amdgcn_readlane(p3, 0);
  __syncthreads();
}

__device__ __forceinline__ int block_max(int a, int* scratch) {
  a = wave_max(a);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) scratch[wv] = a;
  __syncthreads();
  int p = lane < nw ? scratch[lane] : -0x7fffffff - 1;
  p = row16_reduce(p, OpMax());
  a = __builtin_amdgcn_readlane(p, 0);
  __syncthreads();
  return a;
}

// ---------------------------------------------------------------------------
// Parameter blocks (plain values, passed by value to kernels).

struct GridP {
  int nx, ny, log2nx, log2ny;
  int cwm;
  int tlw, tlh;   // log2 of the plane tile width and height (set at launch)
  int lhw;        // log2 of the half-plane width (set at launch)
  double dx, dy, x_origin, y_origin, gravity, sqrt_g;
};

// Look-up tables of the facet amplitude (device memory, one block per
// context): a two-way complex antenna pattern on a u-v grid and the NRCS over
// the local incidence angle; a null table means the closed form.
struct TabP {
  const void* ant;    // [nv][nu] complex (context precision) or null
  const void* nrcs;   // [n_theta] real or null
  int nu, nv, n_theta, pad;
  double u0, inv_du, v0, inv_dv, inv_dtheta;
};

struct RadarP {
  double altitude, sat_x;
  double sat_y1, sat_y2;   // platform y at the two pulses of the pair
  double k2;               // 2 f_c / c
  double gate_spacing, window_start;
  double fresnel_over_mss, inv_mss, two_over_gamma, cell_area;
  const TabP* tab;         // look-up tables, or null for the closed forms
  int G, N, log2N;
};

// Per-band partial spectra ("window") bookkeeping.
struct WinP {
  int WK, log2WK;   // bins per window (power of two, <= N)
  int S;            // slots per band
  int n_bands;
  int band_rows;    // rows per band (fused) or facets per band (standalone)
  void* part;       // [n_bands * S][G][WK] complex
  int4* hdr;        // [n_bands * S] {valid, k0, g_lo, g_hi}
  uint32_t* bandcnt;  // [n_bands][8]
};

constexpr int kCodeNonfinite = -1;
constexpr int kCodeFolded = -2;
constexpr int kCodeOutOfWindow = -3;
constexpr int kCodeBackfacing = -4;

}  // namespace simk
