// Exponential-map update (App. A, Eq. ExpStep): Gamma' = R Gamma R^T with
// R = exp(K), K = c ds [Gamma, dGamma].
//
// [Gamma, dGamma] = P - P^T with P = Gamma dGamma (skew, so R is orthogonal
// and Gamma' stays pure without a purification).  For a tangent dGamma,
// [[Gamma, dGamma], Gamma] = 4 dGamma, so c = 1/4 makes the first-order term
// the Euler step of Eq. (RKstep); c is an option (the printed value is 1/2).
//
// exp(K) by scaling and squaring: s = max(0, ceil(log2 |K|_1)) (one s for all
// states of a problem), K_s = K / 2^s, then the Taylor polynomial of degree 17
// split into even and odd parts in Y = K_s^2 (symmetric, like every
// polynomial in Y, so those products run as mirrored GEMMs):
//   exp(K_s) = C(Y) + K_s S(Y),  C = sum_j Y^j / (2j)!,  S = sum_j Y^j / (2j+1)!,
// j = 0..8, each evaluated by Paterson-Stockmeyer in Z = Y^2 (three products
// per polynomial, both polynomials in one grouped launch).  The truncation
// error is below |K_s|^18 / 18! <= 1.6e-16.  Then s squarings, gated on the
// device by the control word (launches past s exit at once).
//
// This file holds the elementwise pieces; the products are grouped GEMMs.
#include "sgs_internal.h"

namespace sgs {

static int egrid(long long total) {
  long long b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

constexpr int EXP_STRIP = 32;  // rows of K per workgroup of k_exp_gen

// K = c ds (P - P^T) for one 32-row strip of one state, and the row sums of
// |K| of that strip (the 1-norm of a skew matrix is its largest row sum).
// grid: (ceil(n / 32), R), 256 threads.  P^T comes in through LDS so that
// both reads and the write are row-contiguous.
__global__ __launch_bounds__(256) void k_exp_gen(const double* __restrict__ P, int n, double cds,
                                                 double* __restrict__ K, double* __restrict__ rowsum) {
  __shared__ double Pa[EXP_STRIP][64 + 1];
  __shared__ double Pb[64][EXP_STRIP + 1];
  const int mu = blockIdx.y;
  const long long nn = (long long)n * n;
  const double* Pm = P + mu * nn;
  double* Km = K + mu * nn;
  const int i0 = blockIdx.x * EXP_STRIP;
  const int t = threadIdx.x;
  double acc = 0.0;  // row sum of row i0 + (t >> 3), partial over this lane's columns
  for (int j0 = 0; j0 < n; j0 += 64) {
    // Pa[r][c] = P[i0 + r][j0 + c]
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = (t >> 6) + 4 * k, c = t & 63;
      const int i = i0 + r, j = j0 + c;
      Pa[r][c] = (i < n && j < n) ? Pm[(long long)i * n + j] : 0.0;
    }
    // Pb[c][r] = P[j0 + c][i0 + r]
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = t & 31, c = (t >> 5) + 8 * k;
      const int i = i0 + r, j = j0 + c;
      Pb[c][r] = (i < n && j < n) ? Pm[(long long)j * n + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = (t >> 6) + 4 * k, c = t & 63;
      const int i = i0 + r, j = j0 + c;
      const double v = cds * (Pa[r][c] - Pb[c][r]);
      if (i < n && j < n) Km[(long long)i * n + j] = v;
      Pa[r][c] = fabs(v);  // zero outside the matrix
    }
    __syncthreads();
    {
      const int r = t >> 3, c0 = (t & 7) * 8;
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += Pa[r][c0 + u];
    }
    __syncthreads();
  }
  // reduce the 8 partial sums of each row (lanes 8r .. 8r + 7 of a wave)
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 4);
  const int i = i0 + (t >> 3);
  if ((t & 7) == 0 && i < n) rowsum[(long long)mu * n + i] = acc;
}

// s from max |K|_1 over the states; ctl[0] = s - 1 (squaring launch `it`
// runs while it <= ctl[0]); par[0] = 2^-s, par[1] = |K|_1.  A norm beyond
// 2^smax flags ST_RANGE.  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_exp_norm(const double* __restrict__ rowsum, int total, int smax,
                                                  int* __restrict__ ctl, double* __restrict__ par,
                                                  int* __restrict__ status) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int e = threadIdx.x; e < total; e += 256) mx = nan_max(mx, rowsum[e]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = nan_max(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nrm = red[0];
    int s = 0;
    if (nrm > 1.0) {
      int e = 0;
      (void)frexp(nrm, &e);  // nrm < 2^e
      s = e;
    }
    if (!(nrm == nrm) || s > smax) {  // NaN or too large a step
      atomicCAS(status, ST_OK, ST_RANGE);
      s = smax;
    }
    ctl[0] = s - 1;
    par[0] = ldexp(1.0, -s);
    par[1] = nrm;
  }
}

// K *= 2^-s over the R states
__global__ __launch_bounds__(256) void k_exp_scale(double* __restrict__ K, long long total,
                                                   const double* __restrict__ par) {
  const double f = par[0];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    K[e] *= f;
}

// Innermost Paterson-Stockmeyer terms of both polynomials:
//   E0 = c6 + c7 Y + c8 Z,  E1 = s6 + s7 Y + s8 Z
__global__ __launch_bounds__(256) void k_exp_b3(const double* __restrict__ Y, const double* __restrict__ Z, int n,
                                                long long total, ExpCoef cf, double* __restrict__ E0,
                                                double* __restrict__ E1) {
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % nn;
    const double d = (r / n == r % n) ? 1.0 : 0.0;
    const double y = Y[e], z = Z[e];
    E0[e] = cf.c[6] * d + cf.c[7] * y + cf.c[8] * z;
    E1[e] = cf.s[6] * d + cf.s[7] * y + cf.s[8] * z;
  }
}

// After the squarings R sits in X0 when s is even, in X1 when s is odd:
// bring it to X0.
__global__ __launch_bounds__(256) void k_exp_pick(double* __restrict__ X0, const double* __restrict__ X1,
                                                  long long total, const int* __restrict__ ctl) {
  const int s = ctl[0] + 1;
  if ((s & 1) == 0) return;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    X0[e] = X1[e];
}

// The mirrored product writes each off-diagonal 64 x 64 block of Gamma' and
// its negated transpose; the diagonal blocks are computed whole and are skew
// only to rounding.  Make them exactly skew: D <- (D - D^T) / 2 there.
// grid: (ceil(n / 64), R), 256 threads.
__global__ __launch_bounds__(256) void k_exp_skew_diag(double* __restrict__ D, int n) {
  __shared__ double T[64][64 + 1];
  const int mu = blockIdx.y;
  double* Dm = D + (long long)mu * n * n;
  const int b0 = blockIdx.x * 64;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = (t >> 6) + 4 * k, c = t & 63;
    T[r][c] = (b0 + r < n && b0 + c < n) ? Dm[(long long)(b0 + r) * n + b0 + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = (t >> 6) + 4 * k, c = t & 63;
    if (b0 + r < n && b0 + c < n) Dm[(long long)(b0 + r) * n + b0 + c] = 0.5 * (T[r][c] - T[c][r]);
  }
}

hipError_t launch_exp_skew_diag(double* D, int n, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_exp_skew_diag, dim3((n + 63) / 64, R), dim3(256), 0, s, D, n);
  return hipGetLastError();
}

hipError_t launch_exp_gen(const double* P, int n, int R, double cds, double* K, double* rowsum, int smax,
                          int* ctl, double* par, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_exp_gen, dim3((n + EXP_STRIP - 1) / EXP_STRIP, R), dim3(256), 0, s, P, n, cds, K, rowsum);
  hipLaunchKernelGGL(k_exp_norm, dim3(1), dim3(256), 0, s, (const double*)rowsum, R * n, smax, ctl, par, status);
  const long long total = (long long)n * n * R;
  hipLaunchKernelGGL(k_exp_scale, dim3(egrid(total)), dim3(256), 0, s, K, total, (const double*)par);
  return hipGetLastError();
}

hipError_t launch_exp_b3(const double* Y, const double* Z, int n, int R, const ExpCoef& cf, double* E0, double* E1,
                         hipStream_t s) {
  const long long total = (long long)n * n * R;
  hipLaunchKernelGGL(k_exp_b3, dim3(egrid(total)), dim3(256), 0, s, Y, Z, n, total, cf, E0, E1);
  return hipGetLastError();
}

hipError_t launch_exp_pick(double* X0, const double* X1, int n, int R, const int* ctl, hipStream_t s) {
  const long long total = (long long)n * n * R;
  hipLaunchKernelGGL(k_exp_pick, dim3(egrid(total)), dim3(256), 0, s, X0, X1, total, ctl);
  return hipGetLastError();
}

}  // namespace sgs
