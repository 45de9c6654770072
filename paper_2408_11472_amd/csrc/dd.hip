// Delay-Doppler processing of the range-azimuth IQ (Sec. IV.C): bursts of M
// pulses, Doppler-centroid removal, along-track FFT into M Doppler beams,
// range-migration correction with delay phase coefficients, multi-look.
//
//   dd_centroid          pulse-pair centroid of every burst (or the given one)
//   dd_azimuth           centroid ramp and M-point forward DFT along the
//                        pulses, per (burst, gate group)
//   dd_range             per (burst, beam group): forward DFT over the gates,
//                        exp(+2 pi i q delta_f / G), inverse DFT / G
//   dd_multilook         mean over the bursts of |beam|^2 per (beam, gate),
//                        then over the beams per gate
#include "device_common.hpp"
#include "launch.hpp"

namespace simk {

namespace {

constexpr int kDDThreads = 256;

// Radix-2 Stockham transforms of nseq sequences of n = 2^log2n points held
// contiguously in LDS (sequence s at src + s * n), ping-pong between src and
// dst; X[k] = sum_j x[j] e^{DIR 2 pi i j k / n}.  Returns the buffer holding
// the result.  Twiddles from the global table (entries [M, 2M) hold
// e^{+2 pi i m / M}).  Every thread of the block calls it.
template <typename Real, int DIR>
__device__ cplx<Real>* lds_fft_r2(cplx<Real>* src, cplx<Real>* dst, int n, int nseq,
                                  const cplx<Real>* __restrict__ tw) {
  const int half = n >> 1;
  for (int ns = 1; ns < n; ns <<= 1) {
    for (int i = threadIdx.x; i < nseq * half; i += blockDim.x) {
      const int s = i / half, b = i - s * half;
      const int jb = b & (ns - 1);
      const cplx<Real>* in = src + (size_t)s * n;
      cplx<Real>* out = dst + (size_t)s * n;
      cplx<Real> w = tw[2 * ns + jb];
      if (DIR < 0) w.y = -w.y;
      const cplx<Real> a = in[b];
      const cplx<Real> c = cmul(in[b + half], w);
      const int o = (b - jb) * 2 + jb;
      out[o] = cadd(a, c);
      out[o + ns] = csub(a, c);
    }
    __syncthreads();
    cplx<Real>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

}  // namespace

// Pulse-pair centroid of burst b: u_c = arg(sum_{x < M-1, g} Y[x+1][g]
// conj Y[x][g]) / (2 pi), the sum in double with a fixed association (each
// thread its own strided terms in order, then the block partials in thread
// order).  mode 0: the given centroid is written instead.
template <typename Real>
__global__ void __launch_bounds__(kDDThreads)
dd_centroid_kernel(const cplx<Real>* __restrict__ Y, int G, int M, int mode, double given,
                   Real* __restrict__ centroid) {
  __shared__ double part[2][kDDThreads];
  const int b = blockIdx.x;
  double sx = 0.0, sy = 0.0;
  if (mode != 0) {
    const cplx<Real>* y = Y + (size_t)b * M * G;
    const int n = (M - 1) * G;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const cplx<Real> a = y[i + G], c = y[i];
      // a conj(c)
      sx += (double)a.x * (double)c.x + (double)a.y * (double)c.y;
      sy += (double)a.y * (double)c.x - (double)a.x * (double)c.y;
    }
  }
  part[0][threadIdx.x] = sx;
  part[1][threadIdx.x] = sy;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ax = 0.0, ay = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      ax += part[0][t];
      ay += part[1][t];
    }
    double u = given;
    if (mode != 0) u = (ax != 0.0 || ay != 0.0) ? atan2(ay, ax) / 6.283185307179586476925 : 0.0;
    centroid[b] = (Real)u;
  }
}

// Burst b, gates [g0, g0 + GB): Y'[x][g] = Y[b M + x][g] e^{-2 pi i u_c x},
// Z[b][f][g] = sum_x Y'[x][g] e^{-2 pi i f x / M}.  The ramp's phase u_c x is
// reduced in double to a fraction of a turn before the sine and cosine.
template <typename Real>
__global__ void __launch_bounds__(kDDThreads)
dd_azimuth_kernel(const cplx<Real>* __restrict__ Y, int G, int M, int GB,
                  const Real* __restrict__ centroid, cplx<Real>* __restrict__ Z,
                  const cplx<Real>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<Real>* A = reinterpret_cast<cplx<Real>*>(smem_raw);
  cplx<Real>* B = A + (size_t)GB * M;
  const int b = blockIdx.x, g0 = blockIdx.y * GB;
  const double uc = (double)centroid[b];
  for (int i = threadIdx.x; i < GB * M; i += blockDim.x) {
    const int x = i / GB, gl = i - x * GB;   // pulse-major reads, gate fastest
    const int g = g0 + gl;
    cplx<Real> v = mk<Real>(0, 0);
    if (g < G) {
      v = Y[((size_t)b * M + x) * G + g];
      double rev = uc * (double)x;
      rev -= __builtin_rint(rev);
      Real s, c;
      sincos_pi((Real)(2.0 * rev), &s, &c);
      v = cmul(v, mk<Real>(c, -s));
    }
    A[(size_t)gl * M + x] = v;
  }
  __syncthreads();
  const cplx<Real>* R = lds_fft_r2<Real, -1>(A, B, M, GB, tw);
  for (int i = threadIdx.x; i < GB * M; i += blockDim.x) {
    const int f = i / GB, gl = i - f * GB;
    const int g = g0 + gl;
    if (g < G) Z[((size_t)b * M + f) * G + g] = R[(size_t)gl * M + f];
  }
}

// Burst b, beams [f0, f0 + FB): in place, Z[b][f][.] <- IDFT_G(DFT_G(Z[b][f][.])
// e^{+2 pi i q delta_f / G}) / G with q in FFT order and delta_f the range
// migration of beam f in gates, mig * (f_s / M)^2, f_s = f or f - M (mig =
// (PRF lambda H / (2 v))^2 / (2 H dr), formed on the host in double).
template <typename Real>
__global__ void __launch_bounds__(kDDThreads)
dd_range_kernel(cplx<Real>* __restrict__ Z, int G, int M, int FB, double mig,
                const cplx<Real>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<Real>* A = reinterpret_cast<cplx<Real>*>(smem_raw);
  cplx<Real>* B = A + (size_t)FB * G;
  const int b = blockIdx.x, f0 = blockIdx.y * FB;
  const int nf = min(FB, M - f0);
  cplx<Real>* zb = Z + ((size_t)b * M + f0) * G;
  for (int i = threadIdx.x; i < nf * G; i += blockDim.x) A[i] = zb[i];
  __syncthreads();
  cplx<Real>* R = lds_fft_r2<Real, -1>(A, B, G, nf, tw);
  cplx<Real>* O = R == A ? B : A;
  for (int i = threadIdx.x; i < nf * G; i += blockDim.x) {
    const int fl = i / G, q = i - fl * G;
    const int f = f0 + fl;
    const double fs = (double)(f < M / 2 ? f : f - M) / (double)M;
    const double delta = mig * fs * fs;
    const int qs = q < G / 2 ? q : q - G;
    double rev = (double)qs * delta / (double)G;
    rev -= __builtin_rint(rev);
    Real s, c;
    sincos_pi((Real)(2.0 * rev), &s, &c);
    R[i] = cmul(R[i], mk<Real>(c, s));
  }
  __syncthreads();
  cplx<Real>* R2 = lds_fft_r2<Real, +1>(R, O, G, nf, tw);
  const Real inv = (Real)1 / (Real)G;
  for (int i = threadIdx.x; i < nf * G; i += blockDim.x) zb[i] = cscale(R2[i], inv);
}

// beam_power[f][g] = mean over bursts of |Z[b][f][g]|^2 (double).  A block
// takes 64 cells (f, g); wave w of its four adds the bursts b = w mod 4 in
// order, and the four partial sums are added in wave order, so the
// association is fixed.
template <typename Real>
__global__ void __launch_bounds__(kDDThreads)
dd_multilook_beams_kernel(const cplx<Real>* __restrict__ Z, int G, int M, int nb,
                          Real* __restrict__ beam_power) {
  __shared__ double part[kDDThreads / 64][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (i < M * G) {
    for (int b = w; b < nb; b += nw) {
      const cplx<Real> z = Z[(size_t)b * M * G + i];
      acc += (double)z.x * (double)z.x + (double)z.y * (double)z.y;
    }
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && i < M * G) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += part[k][lane];
    beam_power[i] = (Real)(s / (double)nb);
  }
}

// waveform[g] = mean over beams of beam_power[f][g] (double, beams in order).
template <typename Real>
__global__ void __launch_bounds__(kDDThreads)
dd_multilook_gates_kernel(const Real* __restrict__ beam_power, int G, int M,
                          Real* __restrict__ waveform) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  double acc = 0.0;
  for (int f = 0; f < M; ++f) acc += (double)beam_power[(size_t)f * G + g];
  waveform[g] = (Real)(acc / (double)M);
}

template <typename Real>
hipError_t launch_delay_doppler(const void* y, int G, int M, int n_bursts, int centroid_mode,
                                double centroid_given, double mig, int migration, void* beams,
                                void* centroid, void* beam_power, void* waveform,
                                const void* tw, hipStream_t st) {
  const size_t cs = sizeof(cplx<Real>);
  const size_t lds_budget = 64 * 1024;
  int GB = (int)(lds_budget / (2 * (size_t)M * cs));
  if (GB > G) GB = G;
  int FB = (int)(lds_budget / (2 * (size_t)G * cs));
  if (FB > M) FB = M;
  if (GB < 1 || FB < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dd_centroid_kernel<Real>, dim3(n_bursts), dim3(kDDThreads), 0, st,
                     (const cplx<Real>*)y, G, M, centroid_mode, centroid_given, (Real*)centroid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dd_azimuth_kernel<Real>, dim3(n_bursts, (G + GB - 1) / GB),
                     dim3(kDDThreads), 2 * (size_t)GB * M * cs, st, (const cplx<Real>*)y, G, M,
                     GB, (const Real*)centroid, (cplx<Real>*)beams, (const cplx<Real>*)tw);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (migration) {
    hipLaunchKernelGGL(dd_range_kernel<Real>, dim3(n_bursts, (M + FB - 1) / FB),
                       dim3(kDDThreads), 2 * (size_t)FB * G * cs, st, (cplx<Real>*)beams, G, M,
                       FB, mig, (const cplx<Real>*)tw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(dd_multilook_beams_kernel<Real>, dim3((M * G + 63) / 64),
                     dim3(kDDThreads), 0, st, (const cplx<Real>*)beams, G, M, n_bursts,
                     (Real*)beam_power);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dd_multilook_gates_kernel<Real>, dim3((G + kDDThreads - 1) / kDDThreads),
                     dim3(kDDThreads), 0, st, (const Real*)beam_power, G, M, (Real*)waveform);
  return hipGetLastError();
}

template hipError_t launch_delay_doppler<float>(const void*, int, int, int, int, double, double,
                                                int, void*, void*, void*, void*, const void*,
                                                hipStream_t);
template hipError_t launch_delay_doppler<double>(const void*, int, int, int, int, double, double,
                                                 int, void*, void*, void*, void*, const void*,
                                                 hipStream_t);

}  // namespace simk
