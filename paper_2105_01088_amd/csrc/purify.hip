// First-order step and return to a pure state (App. A).
//
// Eq. (RKstep): X = Gamma + ds dGamma (skew).  Eq. (CM-normal-form) with every
// lambda_j rescaled to unit modulus is the orthogonal polar factor of X; it is
// reached by Newton-Schulz iterations X <- X (3 - X^T X) / 2 = X (3 + X^2) / 2
// (X skew), two grouped GEMMs each, converging quadratically because X is
// within O(ds^2) of orthogonal.  k_ns_resid measures max |X^2 + 1| of the last
// iterate's square; the final error is about 1.5 times its square.
#include "sgs_internal.h"

namespace sgs {

__global__ void k_euler(const double* __restrict__ gam, const double* __restrict__ dG, double dtau,
                        long long total, double* __restrict__ X) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    X[e] = gam[e] + dtau * dG[e];
}

// max over all states of |Q + 1| (Q = X X), as an ordered bit pattern
__global__ void k_ns_resid(const double* __restrict__ Q, int n, long long total,
                           unsigned long long* __restrict__ out) {
  __shared__ double red[256];
  double mx = 0.0;
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % nn;
    const int i = (int)(r / n), j = (int)(r - (long long)i * n);
    const double v = Q[e] + (i == j ? 1.0 : 0.0);
    mx = fmax(mx, fabs(v));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

// Gamma <- (X - X^T) / 2 (exactly skew); also checks the residual bound.
__global__ void k_finalize(const double* __restrict__ X, int n, int R, double* __restrict__ gam,
                           const unsigned long long* __restrict__ resid, double tol,
                           int* __restrict__ status) {
  const long long nn = (long long)n * n;
  const long long total = nn * R;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long mu = e / nn, r = e - mu * nn;
    const int i = (int)(r / n), j = (int)(r - (long long)i * n);
    gam[e] = 0.5 * (X[e] - X[mu * nn + (long long)j * n + i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double d = __longlong_as_double((long long)resid[0]);
    if (!(1.5 * d * d <= tol)) atomicCAS(status, ST_OK, ST_NOCONV);
  }
}

__global__ void k_zero_u64(unsigned long long* p) { p[0] = 0ull; }

static int grid_for(long long total) {
  long long b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_euler(const double* gam, const double* dG, double dtau, long long total, double* X,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_euler, dim3(grid_for(total)), dim3(256), 0, s, gam, dG, dtau, total, X);
  return hipGetLastError();
}

hipError_t launch_ns_resid(const double* Q, int n, long long total, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, out);
  hipLaunchKernelGGL(k_ns_resid, dim3(grid_for(total)), dim3(256), 0, s, Q, n, total, out);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* X, int n, int R, double* gam, const unsigned long long* resid,
                           double tol, int* status, hipStream_t s) {
  long long total = (long long)n * n * R;
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(total)), dim3(256), 0, s, X, n, R, gam, resid, tol, status);
  return hipGetLastError();
}

}  // namespace sgs

namespace sgs {

// max |G + G^T| over a stack of matrices (input validation)
__global__ void k_skew_resid(const double* __restrict__ G, int n, long long total,
                             unsigned long long* __restrict__ out) {
  __shared__ double red[256];
  double mx = 0.0;
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long mu = e / nn, r = e - mu * nn;
    const int i = (int)(r / n), j = (int)(r - (long long)i * n);
    mx = fmax(mx, fabs(G[e] + G[mu * nn + (long long)j * n + i]));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

hipError_t launch_skew_resid(const double* G, int n, long long total, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, out);
  long long b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_skew_resid, dim3((int)b), dim3(256), 0, s, G, n, total, out);
  return hipGetLastError();
}

}  // namespace sgs
