// Batched in-place Gauss-Jordan inversion with partial (row) pivoting, for the
// pair matrices S_ab = Gamma_a + Gamma_b.  W_ab = S_ab^{-1} enters the
// transition matrix of Eq. (def-delta-matrix), and
// ln|det S_ab| = sum ln|pivot| gives the overlap magnitude
// |<a|b>|^2 = 2^{-N} |det S_ab|^{1/2} (Sec. II.B).
//
// Blocked form.  For each column panel J = [k, k+b):
//   1. k_gj_panel (one workgroup per matrix): LU with partial pivoting of the
//      (n-k) x b panel held in LDS; the row swaps are applied to the other
//      columns; with D = (pivot block)^{-1} it writes the multipliers
//      E (n x b: rows above k: M[i,J] D; pivot rows: 1 - D; rows below:
//      L21 L11^{-1}), the pivot rows Brow (b x n, zero on J) and the final
//      panel columns (-E, and D on the pivot rows).
//   2. grouped GEMM: M <- M - E Brow  (every row, every column outside J).
// After the last panel, k_gj_unscramble undoes the row pivoting by permuting
// columns (the swaps taken in reverse order).
#include "sgs_internal.h"

namespace sgs {

struct ArgMax {
  double v;  // |value|
  int i;
};

__device__ __forceinline__ ArgMax better(ArgMax a, ArgMax b) {
  // larger value wins; ties go to the smaller index (deterministic)
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

// block-wide argmax (up to 16 waves); red: LDS scratch of 16 entries
__device__ ArgMax block_argmax(ArgMax x, ArgMax* red) {
  for (int off = 32; off > 0; off >>= 1) {
    ArgMax o;
    o.v = __shfl_xor(x.v, off);
    o.i = __shfl_xor(x.i, off);
    x = better(x, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  ArgMax r = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = better(r, red[k]);
  __syncthreads();
  return r;
}

// grid: one workgroup per matrix (up to 1024 threads); dynamic LDS:
// (n-k)*(b+1) + (n-k) + 3*b*b doubles
__global__ __launch_bounds__(1024) void k_gj_panel(double* __restrict__ Mall, long long mstride,
                                                   int n, int k, int b,
                                                   double* __restrict__ Eall, long long estride,
                                                   double* __restrict__ Ball, long long bstride,
                                                   int* __restrict__ pivall,
                                                   double* __restrict__ logdet,
                                                   int* __restrict__ status) {
  extern __shared__ double smem[];
  __shared__ ArgMax red[16];
  __shared__ int lpiv[64];
  const int mat = blockIdx.x;
  double* __restrict__ M = Mall + (long long)mat * mstride;
  double* __restrict__ E = Eall + (long long)mat * estride;
  double* __restrict__ Br = Ball + (long long)mat * bstride;
  int* __restrict__ piv = pivall + (long long)mat * n;
  const int m = n - k;
  const int pitch = b + 1;
  double* P = smem;                        // m x pitch
  double* lcol = P + (long long)m * pitch; // m: multipliers of the current column
  double* Linv = lcol + m;                 // b x b
  double* Uinv = Linv + b * b;             // b x b
  double* Dinv = Uinv + b * b;             // b x b
  const int tid = threadIdx.x, nt = blockDim.x;

  for (int e = tid; e < m * b; e += nt) {
    int r = e / b, c = e - r * b;
    P[r * pitch + c] = M[(long long)(k + r) * n + k + c];
  }
  __syncthreads();

  double ld = 0.0;
  bool sing = false;
  for (int j = 0; j < b; ++j) {
    ArgMax best{-1.0, 0x7fffffff};
    for (int r = j + tid; r < m; r += nt) best = better(best, ArgMax{fabs(P[r * pitch + j]), r});
    best = block_argmax(best, red);
    // a NaN column leaves the sentinel index: keep the diagonal (status set below)
    const int pr = (best.i >= j && best.i < m) ? best.i : j;
    const double pv = P[pr * pitch + j];
    if (tid == 0) lpiv[j] = pr;
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) sing = true;
    ld += log(fabs(pv));
    const double inv = 1.0 / pv;
    // multipliers of the rows below the pivot (reading the pre-swap rows) ...
    for (int r = j + 1 + tid; r < m; r += nt) lcol[r] = (r == pr ? P[j * pitch + j] : P[r * pitch + j]) * inv;
    __syncthreads();
    // ... then the row swap (no thread reads column j of rows j / pr any more)
    if (pr != j)
      for (int c = tid; c < b; c += nt) {
        const double t0 = P[j * pitch + c];
        P[j * pitch + c] = P[pr * pitch + c];
        P[pr * pitch + c] = t0;
      }
    __syncthreads();
    // rank-1 update of the panel, one thread per element (r > j, c >= j)
    const int w = b - j;
    const int tot = (m - j - 1) * w;
    for (int e = tid; e < tot; e += nt) {
      const int r = j + 1 + e / w, c = j + e % w;
      const double l = lcol[r];
      if (c == j) P[r * pitch + j] = l;
      else P[r * pitch + c] -= l * P[j * pitch + c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    logdet[mat] += ld;
    if (sing) atomicCAS(status, ST_OK, ST_SINGULAR);
  }

  // row swaps on the columns outside the panel; pivot rows into Brow
  for (int c = tid; c < n; c += nt) {
    const bool inJ = (c >= k && c < k + b);
    if (!inJ) {
      for (int j = 0; j < b; ++j) {
        int r1 = k + j, r2 = k + lpiv[j];
        if (r1 != r2) {
          double t0 = M[(long long)r1 * n + c];
          M[(long long)r1 * n + c] = M[(long long)r2 * n + c];
          M[(long long)r2 * n + c] = t0;
        }
      }
    }
    for (int j = 0; j < b; ++j) Br[(long long)j * n + c] = inJ ? 0.0 : M[(long long)(k + j) * n + c];
  }
  if (tid < b) piv[k + tid] = k + lpiv[tid];

  // inverses of the unit-lower L11 and upper U11 (one column per thread)
  if (tid < b) {
    const int c = tid;
    for (int r = 0; r < b; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int q = c; q < r; ++q) s -= P[r * pitch + q] * Linv[q * b + c];
      Linv[r * b + c] = (r < c) ? 0.0 : s;
    }
    for (int r = b - 1; r >= 0; --r) {
      if (r > c) { Uinv[r * b + c] = 0.0; continue; }
      double s = (r == c) ? 1.0 : 0.0;
      for (int q = r + 1; q <= c; ++q) s -= P[r * pitch + q] * Uinv[q * b + c];
      Uinv[r * b + c] = s / P[r * pitch + r];
    }
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += nt) {
    int r = e / b, c = e - r * b;
    double s = 0.0;
    for (int q = r; q < b; ++q) s += Uinv[r * b + q] * Linv[q * b + c];
    Dinv[e] = s;
  }
  __syncthreads();

  // multipliers E (one thread per (row, column); reads of a row's panel
  // entries finish before the barrier, the panel columns are written after it)
  const int rows_per = nt / b;
  const int cc = tid % b, rs = tid / b;
  if (rs < rows_per) {
    for (int i = rs; i < n; i += rows_per) {
      double sv;
      if (i < k) {
        sv = 0.0;
        const double* mi = M + (long long)i * n + k;
        for (int q = 0; q < b; ++q) sv += mi[q] * Dinv[q * b + cc];
      } else if (i < k + b) {
        const int r = i - k;
        sv = (r == cc ? 1.0 : 0.0) - Dinv[r * b + cc];
      } else {
        const int r = i - k;
        sv = 0.0;
        for (int q = cc; q < b; ++q) sv += P[r * pitch + q] * Linv[q * b + cc];
      }
      E[(long long)i * b + cc] = sv;
    }
  }
  __syncthreads();
  if (rs < rows_per) {
    for (int i = rs; i < n; i += rows_per) {
      const bool piv_row = (i >= k && i < k + b);
      M[(long long)i * n + k + cc] = piv_row ? Dinv[(i - k) * b + cc] : -E[(long long)i * b + cc];
    }
  }
}

// grid (matrices, row chunks of 16); out[i][c] = M[i][src[c]] in place
__global__ __launch_bounds__(256) void k_gj_unscramble(double* __restrict__ Mall, long long mstride,
                                                       int n, const int* __restrict__ pivall) {
  extern __shared__ double smem[];
  double* rowbuf = smem;              // n doubles
  int* src = (int*)(smem + n);        // n ints
  const int mat = blockIdx.x;
  double* M = Mall + (long long)mat * mstride;
  const int* piv = pivall + (long long)mat * n;
  for (int c = threadIdx.x; c < n; c += blockDim.x) src[c] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = n - 1; t >= 0; --t) {
      int p = piv[t];
      if (p != t) { int x = src[t]; src[t] = src[p]; src[p] = x; }
    }
  }
  __syncthreads();
  const int r0 = blockIdx.y * 16;
  for (int r = r0; r < min(n, r0 + 16); ++r) {
    double* row = M + (long long)r * n;
    for (int c = threadIdx.x; c < n; c += blockDim.x) rowbuf[c] = row[c];
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) row[c] = rowbuf[src[c]];
    __syncthreads();
  }
}

size_t gj_panel_lds_bytes(int n, int k, int b) {
  return sizeof(double) * ((size_t)(n - k) * (b + 2) + 3 * (size_t)b * b);
}

hipError_t launch_gj_panel(double* M, long long mstride, int nmat, int n, int k, int b,
                           double* E, long long estride, double* Br, long long bstride,
                           int* piv, double* logdet, int* status, hipStream_t s) {
  size_t lds = gj_panel_lds_bytes(n, k, b);
  int nt = ((n - k) * b / 4 + 63) / 64 * 64;  // about 4 update elements per thread
  if (nt > 1024) nt = 1024;
  if (nt < 256) nt = 256;
  hipLaunchKernelGGL(k_gj_panel, dim3(nmat), dim3(nt), lds, s, M, mstride, n, k, b, E, estride,
                     Br, bstride, piv, logdet, status);
  return hipGetLastError();
}

hipError_t launch_gj_unscramble(double* M, long long mstride, int nmat, int n, const int* piv,
                                hipStream_t s) {
  size_t lds = sizeof(int) * n + sizeof(double) * n;
  hipLaunchKernelGGL(k_gj_unscramble, dim3(nmat, (n + 15) / 16), dim3(256), lds, s, M, mstride, n,
                     piv);
  return hipGetLastError();
}

hipError_t set_gj_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_gj_panel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace sgs
