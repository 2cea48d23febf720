// Frequency response of probe waveforms (Sec. V: resonant frequencies of the
// cavities, Sec. V-A; transmission and reflection coefficients of the guide
// and the microstrip, Sec. V-B and V-D, are read from spectra of time-domain
// probe records).  A discrete-time Fourier transform at arbitrary
// frequencies, sample n taken at time t0 + n dt:
//   Y_p(f) = dt * sum_n w_n y_p^n exp(-j 2 pi f (t0 + n dt)),
// with an optional Hann taper w_n = sin^2(pi (n + 1/2) / N) (w_n = 1 off).
// One workgroup per frequency: its threads stride the samples, each keeping
// one complex FP64 sum per probe, then an LDS tree adds the threads' sums.
// The phase is formed from the exact product f * t in FP64 and sincospi.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace yr {

constexpr int kDftThreads = 256;
constexpr int kDftProbes = 16;  // probes per launch (one complex sum each per thread)

template <typename T>
__global__ void __launch_bounds__(kDftThreads)
    k_probe_dft(const T* __restrict__ y, int64_t nsteps, int nprb, int p0, int np,
                double dt, double t0, const double* __restrict__ freqs, int hann,
                double* __restrict__ out) {
  __shared__ double red[2][kDftProbes][kDftThreads / 64];
  const double f = freqs[blockIdx.x];
  double re[kDftProbes], im[kDftProbes];
#pragma unroll
  for (int p = 0; p < kDftProbes; ++p) re[p] = im[p] = 0.0;
  const double inv_n = nsteps > 0 ? 1.0 / (double)nsteps : 0.0;
  for (int64_t n = threadIdx.x; n < nsteps; n += kDftThreads) {
    // exp(-j 2 pi f t) with f t formed in FP64; sincospi keeps the reduction
    // of the argument exact for |2 f t| up to 2^52
    double s, c;
    sincospi(2.0 * f * (t0 + (double)n * dt), &s, &c);
    double w = dt;
    if (hann) {
      const double sw = sinpi(((double)n + 0.5) * inv_n);
      w *= sw * sw;
    }
    const T* yn = y + n * nprb + p0;
#pragma unroll
    for (int p = 0; p < kDftProbes; ++p) {
      if (p < np) {
        const double v = w * (double)yn[p];
        re[p] += v * c;
        im[p] -= v * s;
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < kDftProbes; ++p) {
    double a = re[p], b = im[p];
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, 64);
      b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) {
      red[0][p][wid] = a;
      red[1][p][wid] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < np) {
    const int p = threadIdx.x;
    double a = 0, b = 0;
    for (int w = 0; w < kDftThreads / 64; ++w) {
      a += red[0][p][w];
      b += red[1][p][w];
    }
    double* o = out + 2 * ((int64_t)blockIdx.x * nprb + p0 + p);
    o[0] = a;
    o[1] = b;
  }
}

}  // namespace yr

using namespace yr;

extern "C" int probe_dft(yr_dtype dtype, const void* y, int64_t nsteps, int32_t nprb, double dt,
                         double t0, int32_t nf, const double* freqs, int32_t hann, void* out,
                         void* stream_) {
  YR_REQUIRE(dtype == YR_F32 || dtype == YR_F64, YR_EINVAL, "dtype must be YR_F32 or YR_F64");
  YR_REQUIRE(nsteps >= 0 && nprb >= 0 && nf >= 0, YR_EINVAL, "negative size");
  YR_REQUIRE(dt > 0 && std::isfinite(dt) && std::isfinite(t0), YR_EINVAL,
             "dt must be positive and t0 finite");
  if (nf == 0 || nprb == 0) return YR_OK;
  YR_REQUIRE(freqs && out, YR_EINVAL, "null frequency list or output");
  YR_REQUIRE(y || nsteps == 0, YR_EINVAL, "null waveform");
  for (int32_t i = 0; i < nf; ++i)
    YR_REQUIRE(std::isfinite(freqs[i]), YR_EINVAL, "frequencies must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream_);
  double* df = nullptr;
  YR_TRY_HIP(hipMallocAsync(&df, (size_t)nf * sizeof(double), s));
  YR_TRY_HIP(hipMemcpyAsync(df, freqs, (size_t)nf * sizeof(double), hipMemcpyHostToDevice, s));
  YR_TRY_HIP(hipStreamSynchronize(s));  // pageable source
  double* o = static_cast<double*>(out);
  for (int p0 = 0; p0 < nprb; p0 += kDftProbes) {
    const int np = nprb - p0 < kDftProbes ? nprb - p0 : kDftProbes;
    if (dtype == YR_F64)
      k_probe_dft<double><<<nf, kDftThreads, 0, s>>>(static_cast<const double*>(y), nsteps, nprb,
                                                     p0, np, dt, t0, df, hann ? 1 : 0, o);
    else
      k_probe_dft<float><<<nf, kDftThreads, 0, s>>>(static_cast<const float*>(y), nsteps, nprb,
                                                    p0, np, dt, t0, df, hann ? 1 : 0, o);
  }
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipFreeAsync(df, s));
  return YR_OK;
}
