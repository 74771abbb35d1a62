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

constexpr int GJ_STAGE_DOUBLES = 6144;  // 48 KB of LDS for the row gather

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

// Row-owning panel kernel.  Thread t owns the rows i = t + r nt (r < RPT) of
// the whole matrix and keeps their b panel entries M[i, J] in registers
// (J = [k, k + b), b <= B).  For the rows i >= k (logical rows l = i - k of
// the panel) it runs LU with partial pivoting column by column: argmax over
// the owned entries, the pivot row and the displaced row exchange registers
// through LDS, and every row below updates itself from the broadcast pivot
// row (three barriers per column).  Then, with L11 / U11 in LDS, every row
// solves for its multipliers in registers:
//   rows above the panel:  E_i = M[i, J] U^-1 L^-1       (M[i, J] <- -E_i)
//   pivot rows (l < b):    D_l = e_l U^-1 L^-1, E_i = e_l - D_l (M[i, J] <- D_l)
//   rows below:            E_i = L21_l L^-1              (M[i, J] <- -E_i)
// The row swaps reach the other columns as one gather of the moved rows, the
// pivot rows go to Brow (zero on J), and the composed row permutation
// pi (new row r = old row pi[r]) is kept per matrix; after the last panel
// src = pi^-1 drives the column unscramble.
// dynamic LDS: see gj_panel_lds_bytes
template <int B, int RPT>
__global__ __launch_bounds__(512) void k_gj_panel(double* __restrict__ Mall, long long mstride,
                                                  int n, int k, int b,
                                                  double* __restrict__ Eall, long long estride,
                                                  double* __restrict__ Ball, long long bstride,
                                                  int* __restrict__ pivall,
                                                  double* __restrict__ logdet,
                                                  int* __restrict__ status) {
  extern __shared__ double smem[];
  __shared__ ArgMax red[16];
  __shared__ double pivrow[B], swrow[B];
  __shared__ int cnt;
  const int mat = blockIdx.x;
  double* __restrict__ M = Mall + (long long)mat * mstride;
  double* __restrict__ E = Eall + (long long)mat * estride;
  double* __restrict__ Br = Ball + (long long)mat * bstride;
  int* __restrict__ pi = pivall + (long long)mat * n;
  int* __restrict__ src = pivall + (long long)gridDim.x * n + (long long)mat * n;
  const int m = n - k;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* LU = smem;                    // B x (B + 1)
  int* permr = (int*)(LU + B * (B + 1)); // m: logical row l now holds old logical row permr[l]
  int* trow = permr + m;                 // moved logical rows (<= 2B)
  int* pis = trow + 2 * B;               // m: staging of pi
  double* stage = (double*)(pis + ((m + 1) & ~1));  // gather staging
  const int stage_cap = GJ_STAGE_DOUBLES;

  double x[RPT][B];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * nt;
#pragma unroll
    for (int c = 0; c < B; ++c) x[r][c] = (i < n && c < b) ? M[(long long)i * n + k + c] : 0.0;
  }
  for (int l = tid; l < m; l += nt) permr[l] = l;
  double ld = 0.0;
  bool sing = false;
  __syncthreads();

#pragma unroll
  for (int j = 0; j < B; ++j) {
    if (j < b) {  // uniform
      ArgMax best{-1.0, 0x7fffffff};
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int l = tid + r * nt - k;
        if (l >= j && l < m) best = better(best, ArgMax{fabs(x[r][j]), l});
      }
      best = block_argmax(best, red);
      const int pr = (best.i >= j && best.i < m) ? best.i : j;  // NaN column: keep the diagonal
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int l = tid + r * nt - k;
        if (l == pr) {
#pragma unroll
          for (int c = 0; c < B; ++c) pivrow[c] = x[r][c];
        }
        if (l == j && pr != j) {
#pragma unroll
          for (int c = 0; c < B; ++c) swrow[c] = x[r][c];
        }
      }
      if (tid == 0 && pr != j) { const int t0 = permr[j]; permr[j] = permr[pr]; permr[pr] = t0; }
      __syncthreads();
      const double pv = pivrow[j];
      if (tid == 0) {
        if (!(fabs(pv) > 0.0) || !isfinite(pv)) sing = true;
        ld += log(fabs(pv));
      }
      const double inv = 1.0 / pv;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int l = tid + r * nt - k;
        if (l == j) {
#pragma unroll
          for (int c = 0; c < B; ++c) x[r][c] = pivrow[c];
        } else if (l == pr) {
#pragma unroll
          for (int c = 0; c < B; ++c) x[r][c] = swrow[c];
        }
        if (l > j && l < m) {
          const double f = x[r][j] * inv;
          x[r][j] = f;
#pragma unroll
          for (int c = j + 1; c < B; ++c) x[r][c] -= f * pivrow[c];
        }
      }
    }
  }
  if (tid == 0) {
    logdet[mat] += ld;
    if (sing) atomicCAS(status, ST_OK, ST_SINGULAR);
  }
  // L11 / U11 of the pivot block
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int l = tid + r * nt - k;
    if (l >= 0 && l < b) {
#pragma unroll
      for (int c = 0; c < B; ++c) LU[l * (B + 1) + c] = x[r][c];
    }
  }
  __syncthreads();
  // multipliers, by triangular solves in registers (in place on the row)
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * nt;
    const int l = i - k;
    if (i < n) {
      if (l >= 0 && l < b) {
#pragma unroll
        for (int c = 0; c < B; ++c) x[r][c] = (c == l) ? 1.0 : 0.0;  // pivot row: e_l
      }
      if (l < b) {
        // x <- x U^-1 (rows above the panel and pivot rows)
#pragma unroll
        for (int c = 0; c < B; ++c) {
          double s = x[r][c];
#pragma unroll
          for (int q = 0; q < c; ++q) s -= x[r][q] * LU[q * (B + 1) + c];
          x[r][c] = (c < b) ? s / LU[c * (B + 1) + c] : 0.0;
        }
      }
      // x <- x L^-1 (L unit lower); below the panel x already holds L21
#pragma unroll
      for (int c = B - 1; c >= 0; --c) {
        double s = x[r][c];
#pragma unroll
        for (int q = c + 1; q < B; ++q) s -= x[r][q] * LU[q * (B + 1) + c];
        x[r][c] = (c < b) ? s : 0.0;
      }
      double* ei = E + (long long)i * b;
      double* mi = M + (long long)i * n + k;
      if (l >= 0 && l < b) {
#pragma unroll
        for (int c = 0; c < B; ++c)
          if (c < b) { ei[c] = (c == l ? 1.0 : 0.0) - x[r][c]; mi[c] = x[r][c]; }
      } else {
#pragma unroll
        for (int c = 0; c < B; ++c)
          if (c < b) { ei[c] = x[r][c]; mi[c] = -x[r][c]; }
      }
    }
  }
  // rows that moved (and the pivot rows, for Brow); composed permutation
  if (tid == 0) cnt = 0;
  if (k == 0)
    for (int l = tid; l < m; l += nt) pis[l] = permr[l];
  else
    for (int l = tid; l < m; l += nt) pis[l] = pi[k + permr[l]];
  __syncthreads();
  for (int l = tid; l < m; l += nt) {
    pi[k + l] = pis[l];
    if (l < b || permr[l] != l) trow[atomicAdd(&cnt, 1)] = l;
  }
  __syncthreads();
  const int nto = cnt;
  const int chunk = max(1, min(n, stage_cap / max(1, nto)));
  for (int c0 = 0; c0 < n; c0 += chunk) {
    const int cw = min(chunk, n - c0);
    for (int e = tid; e < nto * cw; e += nt) {
      const int t = e / cw, c = c0 + e % cw;
      stage[e] = (c >= k && c < k + b) ? 0.0 : M[(long long)(k + permr[trow[t]]) * n + c];
    }
    __syncthreads();
    for (int e = tid; e < nto * cw; e += nt) {
      const int t = e / cw, c = c0 + e % cw;
      const int l = trow[t];
      if (c < k || c >= k + b) M[(long long)(k + l) * n + c] = stage[e];
      if (l < b) Br[(long long)l * n + c] = stage[e];
    }
    __syncthreads();
  }
  // after the last panel: src = pi^-1 for the column unscramble
  if (k + b == n) {
    __syncthreads();
    for (int c = tid; c < n; c += nt) src[pi[c]] = c;
  }
}

// grid (matrices, row chunks of 16); out[i][c] = M[i][src[c]] in place
__global__ __launch_bounds__(256) void k_gj_unscramble(double* __restrict__ Mall, long long mstride,
                                                       int n, const int* __restrict__ pivall, int rpb) {
  extern __shared__ double smem[];
  double* rowbuf = smem;  // rpb rows
  const int mat = blockIdx.x;
  double* M = Mall + (long long)mat * mstride;
  const int* src = pivall + (long long)gridDim.x * n + (long long)mat * n;
  const int r0 = blockIdx.y * rpb, r1 = min(n, r0 + rpb);
  for (long long e = threadIdx.x; e < (long long)(r1 - r0) * n; e += blockDim.x)
    rowbuf[e] = M[(long long)r0 * n + e];
  __syncthreads();
  for (long long e = threadIdx.x; e < (long long)(r1 - r0) * n; e += blockDim.x) {
    const long long r = e / n, c = e - r * n;
    M[(long long)(r0 + r) * n + c] = rowbuf[r * n + src[c]];
  }
}

GjPanelShape gj_panel_shape(int n) {
  GjPanelShape sh;
  if (n <= 512) { sh.B = 32; sh.rpt = 1; }
  else if (n <= 1024) { sh.B = 16; sh.rpt = 2; }
  else if (n <= 2048) { sh.B = 8; sh.rpt = 4; }
  else if (n <= 4096) { sh.B = 4; sh.rpt = 8; }
  else { sh.B = 2; sh.rpt = 16; }
  const int rows = (n + sh.rpt - 1) / sh.rpt;
  sh.nt = ((rows + 63) / 64) * 64;
  if (sh.nt > 512) sh.nt = 512;
  if (sh.nt < 64) sh.nt = 64;
  return sh;
}

size_t gj_panel_lds_bytes(int n, int k, int b) {
  (void)k;
  const int m = n;  // largest panel
  return sizeof(double) * ((size_t)b * (b + 1) + GJ_STAGE_DOUBLES) + sizeof(int) * (2 * (size_t)m + 2 * b + 2) + 64;
}

hipError_t launch_gj_panel(double* M, long long mstride, int nmat, int n, int k, int b,
                           double* E, long long estride, double* Br, long long bstride,
                           int* piv, double* logdet, int* status, hipStream_t s) {
  const GjPanelShape sh = gj_panel_shape(n);
  const size_t lds = gj_panel_lds_bytes(n, k, sh.B);
#define GJ_LAUNCH(BB, RP)                                                                                    \
  hipLaunchKernelGGL((k_gj_panel<BB, RP>), dim3(nmat), dim3(sh.nt), lds, s, M, mstride, n, k, b, E, estride, \
                     Br, bstride, piv, logdet, status)
  if (sh.B == 32) GJ_LAUNCH(32, 1);
  else if (sh.B == 16) GJ_LAUNCH(16, 2);
  else if (sh.B == 8) GJ_LAUNCH(8, 4);
  else if (sh.B == 4) GJ_LAUNCH(4, 8);
  else GJ_LAUNCH(2, 16);
#undef GJ_LAUNCH
  return hipGetLastError();
}

hipError_t launch_gj_unscramble(double* M, long long mstride, int nmat, int n, const int* piv,
                                hipStream_t s) {
  int rpb = (int)(((size_t)48 * 1024 / sizeof(double)) / (size_t)n);  // rows per block, <= 48 KB of LDS
  if (rpb > 16) rpb = 16;
  if (rpb < 1) rpb = 1;
  size_t lds = sizeof(double) * (size_t)rpb * n;
  hipLaunchKernelGGL(k_gj_unscramble, dim3(nmat, (n + rpb - 1) / rpb), dim3(256), lds, s, M, mstride, n,
                     piv, rpb);
  return hipGetLastError();
}

hipError_t set_gj_lds_limit(size_t bytes) {
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<32, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<16, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<8, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<4, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_gj_panel<2, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace sgs
