// Total-error estimate of the feedback interpolant (Sec. 4.3): at sample
// states, the interpolant is compared with BVP solutions that are more
// accurate than those at the grid nodes.  The reference at a sample is the
// Richardson extrapolation of two solutions of a formula of order p, on N
// and 2N intervals: (2^p f_2N - f_N) / (2^p - 1) cancels the h^p term of the
// error (p = 2 for the trapezoid, p = 6 for the four-point Lobatto IIIA
// formula), and |f_2N - ref| estimates the error of the finer solution.
//
// One workgroup of 1024 threads (16 wavefronts) does the whole estimate: the
// sample sets are small (the paper uses 1280 states) and the statistics need
// one reduction, so a single launch with no scratch memory is enough.  The
// samples are read once, coalesced (thread t takes rows t, t + 1024, ...).
#include <hip/hip_runtime.h>

#include <cmath>

#include "sgcm_internal.h"
#include "trace.h"

namespace sgcm {
namespace {

constexpr int kThreads = 1024;

// max that keeps a NaN once it has appeared (fmax would drop it), so that a
// failed solve or a non-finite interpolant value shows in the statistics
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double wave_reduce_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = nan_max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_reduce_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kThreads) void k_total_error(int64_t n, int m, double scale,
                                                          const double* __restrict__ interp,
                                                          const double* __restrict__ coarse,
                                                          const double* __restrict__ fine, double* __restrict__ ref,
                                                          double* __restrict__ err, double* __restrict__ stats) {
  __shared__ double part[5][kThreads / 64];
  double emax = 0.0, esq = 0.0, cmax = 0.0, esum = 0.0, rsum = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    double e = 0.0, c = 0.0, rm = 0.0;
    for (int j = 0; j < m; ++j) {
      const int64_t k = i * m + j;
      const double f = fine[k];
      const double r = (scale * f - coarse[k]) / (scale - 1.0);
      ref[k] = r;
      e = nan_max(e, fabs(interp[k] - r));
      c = nan_max(c, fabs(f - r));
      rm = nan_max(rm, fabs(r));
    }
    err[i] = e;
    emax = nan_max(emax, e);
    esq = fma(e, e, esq);
    cmax = nan_max(cmax, c);
    esum += e;
    rsum += e / fmax(rm, 1e-8);
  }
  emax = wave_reduce_max(emax);
  esq = wave_reduce_sum(esq);
  cmax = wave_reduce_max(cmax);
  esum = wave_reduce_sum(esum);
  rsum = wave_reduce_sum(rsum);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    part[0][w] = emax;
    part[1][w] = esq;
    part[2][w] = cmax;
    part[3][w] = esum;
    part[4][w] = rsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = part[0][0], s = part[1][0], c = part[2][0], es = part[3][0], rs = part[4][0];
    for (int q = 1; q < kThreads / 64; ++q) {
      a = nan_max(a, part[0][q]);
      s += part[1][q];
      c = nan_max(c, part[2][q]);
      es += part[3][q];
      rs += part[4][q];
    }
    stats[0] = a;
    stats[1] = n > 0 ? sqrt(s / (double)n) : 0.0;
    stats[2] = c;
    stats[3] = n > 0 ? es / (double)n : 0.0;
    stats[4] = n > 0 ? rs / (double)n : 0.0;
  }
}

}  // namespace
}  // namespace sgcm

extern "C" int sgcm_total_error(int64_t n, int32_t m, int32_t order, const double* interp, const double* coarse,
                                const double* fine, double* ref, double* err, double* stats, void* stream) {
  sgcm::CallRange range("sgcm_total_error");
  if (n < 0 || m < 1 || m > 64 || !stats) return SGCM_EINVAL;
  if (order < 1 || order > 16) return SGCM_EINVAL;
  if (n > 0 && (!interp || !coarse || !fine || !ref || !err)) return SGCM_EINVAL;
  if (n > INT64_MAX / 64) return SGCM_EINVAL;
  const double scale = std::ldexp(1.0, order);  // 2^p
  hipLaunchKernelGGL(sgcm::k_total_error, dim3(1), dim3(sgcm::kThreads), 0, (hipStream_t)stream, n, (int)m, scale,
                     interp, coarse, fine, ref, err, stats);
  return hipGetLastError() == hipSuccess ? SGCM_OK : SGCM_EDEVICE;
}
