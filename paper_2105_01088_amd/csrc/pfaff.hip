// Batched Pfaffian of complex skew-symmetric matrices (planar storage).
//
// Used for the overlap phase: the triple product <0|a><a|b><b|0> (Bravyi &
// Gosset, cited in Sec. II.B) reduces by Schur complements to
// 4^{-N} i^N Pf(i G_0) Pf(i (G_a + G_0)) Pf(C_ab); only arg Pf(C_ab) is not
// known in closed form.
//
// Elimination with 2 x 2 pivot blocks: for [[P, B], [-B^T, D]] with
// P = [[0, a], [-a, 0]], Pf = a Pf(D + (b1 b0^T - b0 b1^T) / a), b0 / b1 the
// first two rows of B.  Before each step the largest entry of the current
// first column is moved to position 1 by a symmetric swap (sign flip).
// Blocked with delayed updates: inside a panel of nbh steps the current
// trailing matrix is A + U V^T - V U^T (U = b1, V = b0 / a per step); only the
// two columns a step needs are formed, and after the panel the whole trailing
// matrix takes A += [U V] [V -U]^T as one complex GEMM.
#include "sgs_internal.h"

namespace sgs {

struct CArg {
  double v;
  int i;
};

__device__ __forceinline__ CArg cbetter(CArg a, CArg b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

__device__ CArg cblock_argmax(CArg x, CArg* red) {
  for (int off = 32; off > 0; off >>= 1) {
    CArg o;
    o.v = __shfl_xor(x.v, off);
    o.i = __shfl_xor(x.i, off);
    x = cbetter(x, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  CArg r = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = cbetter(r, red[k]);
  __syncthreads();
  return r;
}

// One panel of nbh elimination steps starting at pivot position p0, for every
// matrix of the batch (one workgroup each).
//   A   : matrices, planar (re plane, then im plane at +n*n), stride astride
//   UV  : per matrix n x (2 nbh) planar (im plane at +uv_im): [U | V]
//   RM  : per matrix n x (2 nbh) planar: [V | -U] (GEMM operand)
//   acc : per matrix {ln|Pf|, cos arg, sin arg}
// dynamic LDS: 2 n + 8 nbh doubles
__global__ __launch_bounds__(256) void k_pf_panel(double* __restrict__ Aall, long long astride,
                                                  int n, int p0, int nbh,
                                                  double* __restrict__ UVall, double* __restrict__ RMall,
                                                  long long uvstride, long long uv_im,
                                                  double* __restrict__ acc,
                                                  int* __restrict__ status) {
  extern __shared__ double smem[];
  __shared__ CArg red[8];
  const int mat = blockIdx.x;
  const long long nn = (long long)n * n;
  double* __restrict__ Ar = Aall + (long long)mat * astride;
  double* __restrict__ Ai = Ar + nn;
  double* __restrict__ Ur = UVall + (long long)mat * uvstride;  // U: cols [0, nbh), V: [nbh, 2nbh)
  double* __restrict__ Ui = Ur + uv_im;
  double* __restrict__ Rr = RMall + (long long)mat * uvstride;
  double* __restrict__ Ri = Rr + uv_im;
  const int ldu = 2 * nbh;
  double* c0r = smem;
  double* c0i = c0r + n;
  double* rowr = c0i + n;   // 4 nbh: U_p re, U_p im, V_p re, V_p im
  double* rowi = rowr + 4 * nbh;
  const int tid = threadIdx.x, nt = blockDim.x;

  double la = 0.0, pr = 1.0, pim = 0.0;
  if (tid == 0 && p0 > 0) { la = acc[mat * 3]; pr = acc[mat * 3 + 1]; pim = acc[mat * 3 + 2]; }
  bool sing = false;

  const int nsteps = min(nbh, (n - p0) / 2);
  for (int s = 0; s < nsteps; ++s) {
    const int p = p0 + 2 * s;
    // row p of U and V
    for (int t = tid; t < s; t += nt) {
      rowr[t] = Ur[(long long)p * ldu + t];
      rowr[nbh + t] = Ui[(long long)p * ldu + t];
      rowr[2 * nbh + t] = Ur[(long long)p * ldu + nbh + t];
      rowr[3 * nbh + t] = Ui[(long long)p * ldu + nbh + t];
    }
    __syncthreads();
    // current column p: c0[i] = B[i][p] = -A[p][i] + sum_t (U_i V_p - V_i U_p)
    CArg best{-1.0, 0x7fffffff};
    for (int i = p + 1 + tid; i < n; i += nt) {
      double xr = -Ar[(long long)p * n + i], xi = -Ai[(long long)p * n + i];
      const double* ur = Ur + (long long)i * ldu;
      const double* ui = Ui + (long long)i * ldu;
      for (int t = 0; t < s; ++t) {
        double uir = ur[t], uii = ui[t], vir = ur[nbh + t], vii = ui[nbh + t];
        double upr = rowr[t], upi = rowr[nbh + t], vpr = rowr[2 * nbh + t], vpi = rowr[3 * nbh + t];
        xr += uir * vpr - uii * vpi - (vir * upr - vii * upi);
        xi += uir * vpi + uii * vpr - (vir * upi + vii * upr);
      }
      c0r[i] = xr;
      c0i[i] = xi;
      best = cbetter(best, CArg{xr * xr + xi * xi, i});
    }
    best = cblock_argmax(best, red);
    // a NaN column leaves the sentinel index: no swap (status set below)
    const int q = (best.i > p && best.i < n) ? best.i : p + 1;
    if (q != p + 1) {
      // symmetric swap of index p+1 and q in the trailing matrix (rows, then columns)
      for (int j = p + tid; j < n; j += nt) {
        long long a1 = (long long)(p + 1) * n + j, a2 = (long long)q * n + j;
        double tr = Ar[a1], ti = Ai[a1];
        Ar[a1] = Ar[a2]; Ai[a1] = Ai[a2];
        Ar[a2] = tr; Ai[a2] = ti;
      }
      __syncthreads();
      for (int i = p + tid; i < n; i += nt) {
        long long a1 = (long long)i * n + p + 1, a2 = (long long)i * n + q;
        double tr = Ar[a1], ti = Ai[a1];
        Ar[a1] = Ar[a2]; Ai[a1] = Ai[a2];
        Ar[a2] = tr; Ai[a2] = ti;
      }
      for (int t = tid; t < s; t += nt) {
        for (int h = 0; h < 2; ++h) {
          long long a1 = (long long)(p + 1) * ldu + h * nbh + t, a2 = (long long)q * ldu + h * nbh + t;
          double tr = Ur[a1], ti = Ui[a1];
          Ur[a1] = Ur[a2]; Ui[a1] = Ui[a2];
          Ur[a2] = tr; Ui[a2] = ti;
        }
      }
      if (tid == 0) {
        double tr = c0r[p + 1], ti = c0i[p + 1];
        c0r[p + 1] = c0r[q]; c0i[p + 1] = c0i[q];
        c0r[q] = tr; c0i[q] = ti;
      }
      __syncthreads();
    }
    // pivot a = B[p][p+1] = -c0[p+1]
    const double ar = -c0r[p + 1], ai = -c0i[p + 1];
    const double a2 = ar * ar + ai * ai;
    if (tid == 0) {
      if (!(a2 > 0.0) || !isfinite(a2)) sing = true;
      const double mag = sqrt(a2);
      la += log(mag);
      double nr = pr * ar - pim * ai, ni = pr * ai + pim * ar;
      if (q != p + 1) { nr = -nr; ni = -ni; }
      const double nm = 1.0 / sqrt(nr * nr + ni * ni);
      pr = nr * nm;
      pim = ni * nm;
    }
    // row p+1 of U and V (after the swap)
    for (int t = tid; t < s; t += nt) {
      rowr[t] = Ur[(long long)(p + 1) * ldu + t];
      rowr[nbh + t] = Ui[(long long)(p + 1) * ldu + t];
      rowr[2 * nbh + t] = Ur[(long long)(p + 1) * ldu + nbh + t];
      rowr[3 * nbh + t] = Ui[(long long)(p + 1) * ldu + nbh + t];
    }
    __syncthreads();
    const double inr = ar / a2, ini = -ai / a2;  // 1 / a
    for (int i = p + 2 + tid; i < n; i += nt) {
      double xr = -Ar[(long long)(p + 1) * n + i], xi = -Ai[(long long)(p + 1) * n + i];
      const double* ur = Ur + (long long)i * ldu;
      const double* ui = Ui + (long long)i * ldu;
      for (int t = 0; t < s; ++t) {
        double uir = ur[t], uii = ui[t], vir = ur[nbh + t], vii = ui[nbh + t];
        double upr = rowr[t], upi = rowr[nbh + t], vpr = rowr[2 * nbh + t], vpi = rowr[3 * nbh + t];
        xr += uir * vpr - uii * vpi - (vir * upr - vii * upi);
        xi += uir * vpi + uii * vpr - (vir * upi + vii * upr);
      }
      // U[i][s] = b1_i = B[p+1][i] = -c1_i ; V[i][s] = b0_i / a = -c0_i / a
      Ur[(long long)i * ldu + s] = -xr;
      Ui[(long long)i * ldu + s] = -xi;
      const double br = -c0r[i], bi = -c0i[i];
      Ur[(long long)i * ldu + nbh + s] = br * inr - bi * ini;
      Ui[(long long)i * ldu + nbh + s] = br * ini + bi * inr;
    }
    __syncthreads();
  }
  // GEMM operand [V | -U] for the trailing rows
  const int pe = p0 + 2 * nsteps;
  for (long long e = (long long)pe * ldu + tid; e < (long long)n * ldu; e += nt) {
    const int t = (int)(e % ldu);
    const long long i = e / ldu;
    if (t < nbh) {
      const bool ok = t < nsteps;
      Rr[i * ldu + t] = ok ? Ur[i * ldu + nbh + t] : 0.0;
      Ri[i * ldu + t] = ok ? Ui[i * ldu + nbh + t] : 0.0;
    } else {
      const bool ok = (t - nbh) < nsteps;
      Rr[i * ldu + t] = ok ? -Ur[i * ldu + (t - nbh)] : 0.0;
      Ri[i * ldu + t] = ok ? -Ui[i * ldu + (t - nbh)] : 0.0;
    }
  }
  if (tid == 0) {
    acc[mat * 3] = la;
    acc[mat * 3 + 1] = pr;
    acc[mat * 3 + 2] = pim;
    if (sing) atomicCAS(status, ST_OK, ST_SINGULAR);
  }
}

// Zero the unused U/V columns so the trailing GEMM (K = 2 nbh) may read them.
__global__ void k_pf_zero(double* __restrict__ UVall, long long total) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    UVall[e] = 0.0;
}

size_t pf_panel_lds_bytes(int n, int nbh) { return sizeof(double) * (2 * (size_t)n + 8 * (size_t)nbh); }

hipError_t launch_pf_panel(double* A, long long astride, int nmat, int n, int p0, int nbh,
                           double* UV, double* RM, long long uvstride, long long uv_im,
                           double* acc, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_pf_panel, dim3(nmat), dim3(256), pf_panel_lds_bytes(n, nbh), s, A, astride, n,
                     p0, nbh, UV, RM, uvstride, uv_im, acc, status);
  return hipGetLastError();
}

hipError_t launch_pf_zero(double* UV, long long total, hipStream_t s) {
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_pf_zero, dim3(blocks), dim3(256), 0, s, UV, total);
  return hipGetLastError();
}

}  // namespace sgs
