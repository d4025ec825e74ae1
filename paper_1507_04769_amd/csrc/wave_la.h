// Wavefront-level dense linear algebra on small matrices, for the kernels
// whose 6 x 6 algebra runs in one wavefront with one matrix column per lane:
// the elimination broadcasts the pivot column from its lane (readlane), and a
// product is a matrix-vector product per lane with the other matrix in LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace sgcm {

// x of lane `from` (a wavefront constant).
__device__ __forceinline__ double bcast(double x, int from) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, from);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), from);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Gauss-Jordan elimination with partial pivoting of an n-row augmented matrix
// whose column l is v in lane l (lanes 0..n-1: the square part): afterwards
// the lanes of the other columns hold the solution's columns.  A zero pivot
// leaves non-finite values.  Every lane of the wavefront takes part.  With
// W < 64 every group of W consecutive lanes eliminates a matrix of its own
// (column l in the group's lane l; the pivot column is then read with a lane
// permute instead of readlane).  Returns false when a pivot was exactly zero
// (the values are then not finite), and with FINITE also when a pivot was not
// finite.
template <int n, int W = 64, bool FINITE = false>
__device__ __forceinline__ bool gauss_jordan(double (&v)[n]) {
  bool regular = true;
#pragma unroll
  for (int c = 0; c < n; ++c) {
    double col[n];
#pragma unroll
    for (int i = 0; i < n; ++i) col[i] = W == 64 ? bcast(v[i], c) : __shfl(v[i], c, W);
    int p = c;
    double best = fabs(col[c]);
#pragma unroll
    for (int i = c + 1; i < n; ++i) {
      const double a = fabs(col[i]);
      if (a > best) {
        best = a;
        p = i;
      }
    }
    // rows c and p trade places
    const double cc = col[c], vc = v[c];
    double cp = cc, vp = vc;
#pragma unroll
    for (int i = c + 1; i < n; ++i)
      if (p == i) {
        cp = col[i];
        vp = v[i];
        col[i] = cc;
        v[i] = vc;
      }
    regular = regular && cp != 0.0 && (!FINITE || isfinite(cp));
    const double nv = vp * (1.0 / cp);
#pragma unroll
    for (int i = 0; i < n; ++i)
      if (i != c) v[i] = fma(-col[i], nv, v[i]);
    v[c] = nv;
  }
  return regular;
}

// y = M x for a 6 x 6 row-major M in LDS.
__device__ __forceinline__ void matvec(const double* M, const double (&x)[6], double (&y)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = M[i * 6] * x[0];
#pragma unroll
    for (int l = 1; l < 6; ++l) s = fma(M[i * 6 + l], x[l], s);
    y[i] = s;
  }
}

__device__ __forceinline__ void load_col(const double* M, int j, double (&x)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) x[i] = M[i * 6 + j];
}

__device__ __forceinline__ void store_col(double* M, int j, const double (&x)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) M[i * 6 + j] = x[i];
}

}  // namespace sgcm
