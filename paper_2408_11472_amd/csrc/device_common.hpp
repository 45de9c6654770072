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

// Size of the master twiddle table e^{+2 pi i m / kTwSize}.
constexpr int kTwLog2 = 16;
constexpr int kTwSize = 1 << kTwLog2;

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

// Twiddle w^r of a butterfly from the exact table powers w, w^2, w^4, w^8
// (at most three products, compile-time r after unrolling).
template <typename T>
__device__ __forceinline__ cplx<T> twiddle_pow(const cplx<T>* base, int r) {
  cplx<T> acc = mk<T>((T)1, (T)0);
  bool first = true;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (r & (1 << b)) {
      acc = first ? base[b] : cmul(acc, base[b]);
      first = false;
    }
  }
  return acc;
}

// One Stockham radix-R stage on a sequence of length N held as E values per
// thread by T = N/E threads: register slot m holds position tid + m*T.
// Butterfly q (q < E/R) of this thread is b = tid + q*T with inputs at
// slots q + r*(E/R).  The outputs go to LDS at the self-sorting positions
// ((b - j) * R + j + r * Ns, j = b mod Ns), except on the last stage, whose
// output positions coincide with the register slots.
template <typename T, int E, int R, int DIR>
__device__ __forceinline__ void stockham_stage(cplx<T>* v, cplx<T>* lds, int ls, int N,
                                               int tid, int Ns, bool last,
                                               const cplx<T>* __restrict__ tw) {
  const int Tn = N / E;
#pragma unroll
  for (int q = 0; q < E / R; ++q) {
    cplx<T> u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[q + r * (E / R)];
    const int b = tid + q * Tn;
    const int j = b & (Ns - 1);
    if (Ns > 1) {
      // w = e^{DIR 2 pi i j / (Ns R)}: table entries j s, 2 j s, 4 j s, 8 j s
      const int step = j * (kTwSize / (Ns * R));
      cplx<T> base[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        if ((1 << bb) < R) {
          base[bb] = tw[(step << bb) & (kTwSize - 1)];
          if (DIR < 0) base[bb].y = -base[bb].y;
        } else {
          base[bb] = mk<T>((T)1, (T)0);
        }
      }
#pragma unroll
      for (int r = 1; r < R; ++r) u[r] = cmul(u[r], twiddle_pow(base, r));
    }
    dft<T, R, DIR>(u);
    if (last) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * (E / R)] = u[r];
    } else {
      const int base = (b - j) * R + j;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lpad(base + r * Ns) * ls] = u[r];
    }
  }
  if (!last) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[lpad(tid + m * Tn) * ls];
    __syncthreads();
  }
}

// Unnormalised DFT of one sequence of length N (power of two, N >= E),
// X[k] = sum_n x[n] e^{DIR 2 pi i n k / N}, held in registers as E values
// per thread in slot order (slot m = position tid + m*N/E) on entry and on
// exit.  lds points at this sequence's LDS region (lpad(N) elements with
// element stride ls).  Every thread of the block must call it (barriers).
template <typename T, int E, int DIR>
__device__ __forceinline__ void fft_seq(cplx<T>* v, cplx<T>* lds, int ls, int N, int log2N,
                                        int tid, const cplx<T>* __restrict__ tw) {
  constexpr int LE = (E == 16) ? 4 : (E == 8) ? 3 : (E == 4) ? 2 : 1;
  const int full = log2N / LE;
  const int rem = log2N - full * LE;
  int Ns = 1;
  if (rem == 1) {
    stockham_stage<T, E, 2, DIR>(v, lds, ls, N, tid, Ns, false, tw);
    Ns *= 2;
  } else if (rem == 2) {
    stockham_stage<T, E, (E >= 4 ? 4 : 2), DIR>(v, lds, ls, N, tid, Ns, false, tw);
    Ns *= 4;
  } else if (rem == 3) {
    stockham_stage<T, E, (E >= 8 ? 8 : 2), DIR>(v, lds, ls, N, tid, Ns, false, tw);
    Ns *= 8;
  }
  for (int s = 0; s < full; ++s) {
    stockham_stage<T, E, E, DIR>(v, lds, ls, N, tid, Ns, s == full - 1, tw);
    Ns *= E;
  }
}

// ---------------------------------------------------------------------------
// Block reductions (blockDim.x a multiple of 64, at most 1024 threads).
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduce four ints (two mins, two maxes) over the block; scratch holds
// 4 * 16 ints.  Result broadcast to every thread.
__device__ __forceinline__ void block_minmax2(int& amin, int& amax, int& bmin, int& bmax,
                                              int* scratch) {
  amin = wave_min(amin);
  amax = wave_max(amax);
  bmin = wave_min(bmin);
  bmax = wave_max(bmax);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    scratch[wv] = amin;
    scratch[16 + wv] = amax;
    scratch[32 + wv] = bmin;
    scratch[48 + wv] = bmax;
  }
  __syncthreads();
  amin = scratch[0];
  amax = scratch[16];
  bmin = scratch[32];
  bmax = scratch[48];
  for (int w = 1; w < nw; ++w) {
    amin = min(amin, scratch[w]);
    amax = max(amax, scratch[16 + w]);
    bmin = min(bmin, scratch[32 + w]);
    bmax = max(bmax, scratch[48 + w]);
  }
  __syncthreads();
}

__device__ __forceinline__ int block_max(int a, int* scratch) {
  a = wave_max(a);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) scratch[wv] = a;
  __syncthreads();
  a = scratch[0];
  for (int w = 1; w < nw; ++w) a = max(a, scratch[w]);
  __syncthreads();
  return a;
}

// ---------------------------------------------------------------------------
// Parameter blocks (plain values, passed by value to kernels).

struct GridP {
  int nx, ny, log2nx, log2ny;
  int cwm;
  double dx, dy, x_origin, y_origin, gravity, sqrt_g;
};

struct RadarP {
  double altitude, sat_x;
  double sat_y1, sat_y2;   // platform y at the two pulses of the pair
  double k2;               // 2 f_c / c
  double gate_spacing, window_start;
  double fresnel_over_mss, inv_mss, two_over_gamma, cell_area;
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
