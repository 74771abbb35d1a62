// First-order step and return to a pure state (App. A).
//
// Eq. (RKstep): X = Gamma + ds dGamma (skew).  Eq. (CM-normal-form) with every
// lambda_j rescaled to unit modulus is the orthogonal polar factor of X.
// Because dGamma anticommutes with Gamma (purity is preserved to first
// order, Sec. III.B), X^T X = 1 + ds^2 dGamma^T dGamma: every singular value of
// X lies in [1, sqrt(1 + ds^2 |dGamma|_2^2)].  The Newton-Schulz iteration
// X <- X (3 - X^T X) / 2 = X (3 + X^2) / 2 (two grouped GEMMs) converges for
// singular values in (0, sqrt 3) and fastest near 1; the polar factor is
// unchanged by a positive scaling.  k_euler scales each state by
// min(1, 1.6 / sqrt(1 + ds^2 |dGamma|_1^2)) (|.|_1 >= |.|_2 for a skew
// matrix): the spectrum stays below 1.6 < sqrt 3, and the smallest singular
// values (exactly 1) are not pushed down unless the bound forces it.  (The
// plain 1 / sqrt(1 + ds^2 |dGamma|_1^2) put them at ~0.6 for the usual step
// sizes: 6 iterations where this takes 4.)  Each state converges
// on its own: the square's epilogue records max |X_mu^2 + 1| per state, and
// the next product marks the first iteration below the detection threshold
// as that state's last (ctl[2 + mu]); later GEMM jobs of the state exit at
// once, and once every state is marked whole launches do (ctl[0], ctl[1]).
#include "sgs_internal.h"
#include "wave_ops.h"

namespace sgs {

static int grid_for(long long total) {
  long long b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

// X = alpha_mu (Gamma + ds dGamma), alpha_mu = min(1, 1.6 / sqrt(1 + (ds |dGamma_mu|_1)^2));
// also resets the polar iteration's control words (one per state) and
// residual slots.
__global__ __launch_bounds__(256) void k_euler(const double* __restrict__ gam, const double* __restrict__ dG,
                                               double dtau, int n, int R, double* __restrict__ X,
                                               const unsigned long long* __restrict__ nrm,
                                               int* __restrict__ ctl, unsigned long long* __restrict__ resid,
                                               int nresid) {
  const long long nn = (long long)n * n, total = nn * R;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int mu = (int)(e / nn);
    const double t = dtau * __longlong_as_double((long long)nrm[mu]);
    const double alpha = fmin(1.0, 1.6 / sqrt(1.0 + t * t));
    X[e] = alpha * (gam[e] + dtau * dG[e]);
  }
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < R + 2; t += blockDim.x) ctl[t] = t == 1 ? R : 0x7fffffff;
    for (int t = threadIdx.x; t < nresid; t += blockDim.x) resid[t] = 0ull;
  }
}

__global__ void k_zero_u64(unsigned long long* p) { p[0] = 0ull; }

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
    mx = nan_max(mx, fabs(v));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = nan_max(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

// Gamma_mu <- (X - X^T) / 2 from the buffer holding state mu's last iterate
__global__ void k_finalize(const double* __restrict__ X0, const double* __restrict__ X1, int n, int R,
                           double* __restrict__ gam, const int* __restrict__ ctl, int maxit,
                           int* __restrict__ status) {
  const long long nn = (long long)n * n;
  const long long total = nn * R;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long mu = e / nn, r = e - mu * nn;
    const int c = ctl[2 + mu];
    const int last = (c == 0x7fffffff) ? maxit : c + 1;
    const double* X = (last & 1) ? X1 : X0;
    const int i = (int)(r / n), j = (int)(r - (long long)i * n);
    gam[e] = 0.5 * (X[e] - X[mu * nn + (long long)j * n + i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bool conv = true;
    for (int mu = 0; mu < R; ++mu) conv = conv && ctl[2 + mu] != 0x7fffffff;
    if (!conv) atomicCAS(status, ST_OK, ST_NOCONV);
  }
}

hipError_t launch_euler(const double* gam, const double* dG, double dtau, int n, int R, double* X, int* ctl,
                        unsigned long long* resid, int nresid, unsigned long long* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_euler, dim3(grid_for((long long)n * n * R)), dim3(256), 0, s, gam, dG, dtau, n, R, X,
                     (const unsigned long long*)nrm, ctl, resid, nresid);
  return hipGetLastError();
}

hipError_t launch_ns_resid(const double* Q, int n, long long total, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, out);
  hipLaunchKernelGGL(k_ns_resid, dim3(grid_for(total)), dim3(256), 0, s, Q, n, total, out);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* X0, const double* X1, int n, int R, double* gam, const int* ctl,
                           int maxit, int* status, hipStream_t s) {
  long long total = (long long)n * n * R;
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(total)), dim3(256), 0, s, X0, X1, n, R, gam, ctl, maxit, status);
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
    mx = nan_max(mx, fabs(G[e] + G[mu * nn + (long long)j * n + i]));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = nan_max(red[threadIdx.x], red[threadIdx.x + off]);
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

namespace sgs {

// Sign of Pf(Gamma) of each covariance matrix (the parity of the Gaussian
// state, +1 even), for the check of sgs_init.  One workgroup per matrix works
// on a copy in S by 2 x 2 pivot elimination: with the largest entry of the
// current first column moved to position 1 by a symmetric swap (a sign flip),
// [[0, a, b0], [-a, 0, b1], [-b0^T, -b1^T, D]] has Pfaffian
// a Pf(D + (b1 b0^T - b0 b1^T) / a).  Only the signs of the pivots and the
// flips are kept.  out[mu] = +1 or -1, or 0 for a singular or non-finite
// matrix.  Run once per context, so the plain (unblocked) form: each step
// reads and writes the trailing matrix.
// dynamic LDS: 2 n doubles (rows 0 and 1 of the current step)
__global__ __launch_bounds__(1024) void k_pf_sign(const double* __restrict__ G, double* __restrict__ S, int n,
                                                  double* __restrict__ out) {
  extern __shared__ double brow[];  // b0 then b1
  __shared__ unsigned long long wkey[16];
  __shared__ int spiv;
  const int mu = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const long long nn = (long long)n * n;
  const double* __restrict__ g = G + mu * nn;
  double* __restrict__ M = S + mu * nn;
  for (long long e = tid; e < nn; e += nt) M[e] = g[e];
  __syncthreads();
  double sgn = 1.0;
  bool bad = false;
  for (int k = 0; k + 1 < n; k += 2) {
    // pivot: largest |M[i][k]|, i > k
    unsigned long long key = 0;
    for (int i = k + 1 + tid; i < n; i += nt) key = umax64(key, pivot_key(M[(long long)i * n + k], i));
    key = wave_max_u64(key);
    if (lane == 0) wkey[w] = key;
    __syncthreads();
    if (tid == 0) {
      unsigned long long best = 0;
      for (int x = 0; x < nw; ++x) best = umax64(best, wkey[x]);
      spiv = best == 0ull ? -1 : 0xffff - (int)(best & 0xffffull);
    }
    __syncthreads();
    const int q = spiv;
    if (q < 0 || q <= k || q >= n) { bad = true; break; }
    if (q != k + 1) {
      // symmetric swap of rows and columns k + 1 and q
      for (int j = tid; j < n; j += nt) {
        const double t = M[(long long)(k + 1) * n + j];
        M[(long long)(k + 1) * n + j] = M[(long long)q * n + j];
        M[(long long)q * n + j] = t;
      }
      __syncthreads();
      for (int j = tid; j < n; j += nt) {
        const double t = M[(long long)j * n + k + 1];
        M[(long long)j * n + k + 1] = M[(long long)j * n + q];
        M[(long long)j * n + q] = t;
      }
      sgn = -sgn;
      __syncthreads();
    }
    const double a = M[(long long)k * n + k + 1];
    if (!(fabs(a) > 0.0) || !isfinite(a)) { bad = true; break; }
    if (a < 0.0) sgn = -sgn;
    const int m = n - k - 2;
    for (int j = tid; j < m; j += nt) {
      brow[j] = M[(long long)k * n + k + 2 + j];
      brow[n + j] = M[(long long)(k + 1) * n + k + 2 + j];
    }
    __syncthreads();
    const double ra = 1.0 / a;
    for (long long e = tid; e < (long long)m * m; e += nt) {
      const int i = (int)(e / m), j = (int)(e - (long long)i * m);
      M[(long long)(k + 2 + i) * n + k + 2 + j] += (brow[n + i] * brow[j] - brow[i] * brow[n + j]) * ra;
    }
    __syncthreads();
  }
  if (tid == 0) out[mu] = bad ? 0.0 : sgn;
}

hipError_t launch_pf_sign(const double* G, double* S, int n, int R, double* out, hipStream_t s) {
  if (n < 2 || (n & 1) || n > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pf_sign, dim3(R), dim3(1024), 2 * (size_t)n * sizeof(double), s, G, S, n, out);
  return hipGetLastError();
}

hipError_t set_pf_sign_lds_limit(int n) {
  return hipFuncSetAttribute((const void*)k_pf_sign, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(2 * (size_t)n * sizeof(double)));
}

}  // namespace sgs
