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
// Blocked with delayed updates: inside a panel of NBH steps the current
// trailing matrix is A + U V^T - V U^T (U = b1, V = b0 / a per step); only the
// two columns a step needs are formed, and after the panel the trailing
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

// block-wide argmax (up to 16 waves); red: LDS scratch of 16 entries
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

// One panel of NBH elimination steps on the compact m x m trailing matrix A
// (planar, leading dimension ld, imaginary plane at +plane), for every
// matrix of the batch (one workgroup each).  Logical row l of the panel is
// owned by thread l % nt (slot l / nt < RPT) and keeps its U and V entries in
// registers.  Pivoting swaps two entries of a permutation in LDS (logical ->
// stored index) and exchanges the two rows' registers; the stored matrix is
// never written during the panel.  At the end the panel writes, for the
// trailing logical rows l >= 2 NBH, the GEMM operands L = [U | V] and
// Rm = [V | -U] (row l - 2 NBH, leading dimension 2 NBH) and perm[l]; the
// trailing GEMM reads the old matrix through that permutation and writes the
// next, compact trailing matrix into the other buffer.
//   acc : per matrix {ln|Pf|, cos arg, sin arg}; first: start from Pf = 1
// dynamic LDS: m ints + 3 (4 NBH + 2) doubles
template <int NBH, int RPT>
__global__ __launch_bounds__(512) void k_pf_panel(const double* __restrict__ Aall, long long astride,
                                                   long long plane, int ld, int m,
                                                   double* __restrict__ Lall, double* __restrict__ RMall,
                                                   long long lstride, long long l_im,
                                                   int* __restrict__ permall, int pstride,
                                                   double* __restrict__ acc, int first,
                                                   int* __restrict__ status) {
  extern __shared__ double smem[];
  __shared__ CArg red[16];
  constexpr int BW = 4 * NBH + 2;  // record: U re, U im, V re, V im, c0 re, c0 im
  int* perm = (int*)smem;
  double* bc = smem + ((m + 1) / 2);
  double* sw = bc + BW;  // two records
  const int mat = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const double* __restrict__ Ar = Aall + (long long)mat * astride;
  const double* __restrict__ Ai = Ar + plane;

  double ur[RPT][NBH], ui[RPT][NBH], vr[RPT][NBH], vi[RPT][NBH], c0r[RPT], c0i[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    c0r[r] = 0.0;
    c0i[r] = 0.0;
#pragma unroll
    for (int t = 0; t < NBH; ++t) { ur[r][t] = 0.0; ui[r][t] = 0.0; vr[r][t] = 0.0; vi[r][t] = 0.0; }
  }
  for (int l = tid; l < m; l += nt) perm[l] = l;
  double la = 0.0, phr = 1.0, phi = 0.0;
  if (tid == 0 && !first) { la = acc[mat * 3]; phr = acc[mat * 3 + 1]; phi = acc[mat * 3 + 2]; }
  bool sing = false;
  const int ns = min(NBH, m / 2);
  __syncthreads();

#pragma unroll
  for (int s = 0; s < NBH; ++s) {
    if (s < ns) {  // uniform: every thread takes the same branch
    const int p = 2 * s;
    // broadcast U, V of logical row p
    if (tid == p % nt) {
      const int rs = p / nt;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r == rs) {
#pragma unroll
          for (int t = 0; t < s; ++t) {
            bc[t] = ur[r][t]; bc[NBH + t] = ui[r][t]; bc[2 * NBH + t] = vr[r][t]; bc[3 * NBH + t] = vi[r][t];
          }
        }
    }
    __syncthreads();
    // current column p: c0[l] = -A[p][l] + sum_t (U_l V_p - V_l U_p), l > p
    const long long prow = (long long)perm[p] * ld;
    CArg best{-1.0, 0x7fffffff};
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = tid + r * nt;
      if (l > p && l < m) {
        const long long o = prow + perm[l];
        double xr = -Ar[o], xi = -Ai[o];
#pragma unroll
        for (int t = 0; t < s; ++t) {
          const double upr = bc[t], upi = bc[NBH + t], vpr = bc[2 * NBH + t], vpi = bc[3 * NBH + t];
          xr += ur[r][t] * vpr - ui[r][t] * vpi - (vr[r][t] * upr - vi[r][t] * upi);
          xi += ur[r][t] * vpi + ui[r][t] * vpr - (vr[r][t] * upi + vi[r][t] * upr);
        }
        c0r[r] = xr;
        c0i[r] = xi;
        best = cbetter(best, CArg{xr * xr + xi * xi, l});
      }
    }
    best = cblock_argmax(best, red);
    const int q = (best.i > p && best.i < m) ? best.i : p + 1;  // NaN column: no swap
    const bool flip = q != p + 1;
    if (flip) {
      // exchange the records of logical rows p+1 and q
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int l = tid + r * nt;
        if (l == p + 1 || l == q) {
          double* rec = sw + (l == q ? BW : 0);
#pragma unroll
          for (int t = 0; t < s; ++t) {
            rec[t] = ur[r][t]; rec[NBH + t] = ui[r][t]; rec[2 * NBH + t] = vr[r][t]; rec[3 * NBH + t] = vi[r][t];
          }
          rec[4 * NBH] = c0r[r];
          rec[4 * NBH + 1] = c0i[r];
        }
      }
      if (tid == 0) {
        const int x = perm[p + 1];
        perm[p + 1] = perm[q];
        perm[q] = x;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int l = tid + r * nt;
        if (l == p + 1 || l == q) {
          const double* rec = sw + (l == q ? 0 : BW);
#pragma unroll
          for (int t = 0; t < s; ++t) {
            ur[r][t] = rec[t]; ui[r][t] = rec[NBH + t]; vr[r][t] = rec[2 * NBH + t]; vi[r][t] = rec[3 * NBH + t];
          }
          c0r[r] = rec[4 * NBH];
          c0i[r] = rec[4 * NBH + 1];
        }
      }
    }
    // broadcast row p+1 (after the swap) and its c0
    if (tid == (p + 1) % nt) {
      const int rs = (p + 1) / nt;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r == rs) {
#pragma unroll
          for (int t = 0; t < s; ++t) {
            bc[t] = ur[r][t]; bc[NBH + t] = ui[r][t]; bc[2 * NBH + t] = vr[r][t]; bc[3 * NBH + t] = vi[r][t];
          }
          bc[4 * NBH] = c0r[r];
          bc[4 * NBH + 1] = c0i[r];
        }
    }
    __syncthreads();
    // pivot a = B[p][p+1] = -c0[p+1]
    const double ar = -bc[4 * NBH], ai = -bc[4 * NBH + 1];
    const double a2 = ar * ar + ai * ai;
    if (tid == 0) {
      if (!(a2 > 0.0) || !isfinite(a2)) sing = true;
      la += 0.5 * log(a2);
      double nr = phr * ar - phi * ai, ni = phr * ai + phi * ar;
      if (flip) { nr = -nr; ni = -ni; }
      const double nm = 1.0 / sqrt(nr * nr + ni * ni);
      phr = nr * nm;
      phi = ni * nm;
    }
    const double inr = ar / a2, ini = -ai / a2;  // 1 / a
    const long long prow1 = (long long)perm[p + 1] * ld;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = tid + r * nt;
      if (l > p + 1 && l < m) {
        const long long o = prow1 + perm[l];
        double xr = -Ar[o], xi = -Ai[o];
#pragma unroll
        for (int t = 0; t < s; ++t) {
          const double upr = bc[t], upi = bc[NBH + t], vpr = bc[2 * NBH + t], vpi = bc[3 * NBH + t];
          xr += ur[r][t] * vpr - ui[r][t] * vpi - (vr[r][t] * upr - vi[r][t] * upi);
          xi += ur[r][t] * vpi + ui[r][t] * vpr - (vr[r][t] * upi + vi[r][t] * upr);
        }
        // U[l][s] = b1_l = -c1_l ; V[l][s] = b0_l / a = -c0_l / a
        ur[r][s] = -xr;
        ui[r][s] = -xi;
        const double br = -c0r[r], bi = -c0i[r];
        vr[r][s] = br * inr - bi * ini;
        vi[r][s] = br * ini + bi * inr;
      }
    }
    __syncthreads();
    }
  }
  // GEMM operands for the trailing rows, and the permutation
  const int pe = 2 * ns;
  double* Lr = Lall + (long long)mat * lstride;
  double* Li = Lr + l_im;
  double* Rr = RMall + (long long)mat * lstride;
  double* Ri = Rr + l_im;
  int* gperm = permall + (long long)mat * pstride;
  constexpr int K = 2 * NBH;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int l = tid + r * nt;
    if (l >= pe && l < m) {
      const long long o = (long long)(l - pe) * K;
#pragma unroll
      for (int t = 0; t < NBH; ++t) {
        Lr[o + t] = ur[r][t]; Li[o + t] = ui[r][t];
        Lr[o + NBH + t] = vr[r][t]; Li[o + NBH + t] = vi[r][t];
        Rr[o + t] = vr[r][t]; Ri[o + t] = vi[r][t];
        Rr[o + NBH + t] = -ur[r][t]; Ri[o + NBH + t] = -ui[r][t];
      }
    }
  }
  for (int l = pe + tid; l < m; l += nt) gperm[l - pe] = perm[l];
  if (tid == 0) {
    acc[mat * 3] = la;
    acc[mat * 3 + 1] = phr;
    acc[mat * 3 + 2] = phi;
    if (sing) atomicCAS(status, ST_OK, ST_SINGULAR);
  }
}

size_t pf_panel_lds_bytes(int m, int nbh) {
  return sizeof(double) * ((size_t)(m + 1) / 2 + 3 * (size_t)(4 * nbh + 2)) + 64;
}

PfPanelShape pf_panel_shape(int m) {
  PfPanelShape sh;
  // at most 512 threads (256 VGPRs each): register rows x panel depth fixed
  if (m <= 512) { sh.nbh = 16; sh.rpt = 1; }
  else if (m <= 1024) { sh.nbh = 8; sh.rpt = 2; }
  else if (m <= 2048) { sh.nbh = 4; sh.rpt = 4; }
  else if (m <= 4096) { sh.nbh = 2; sh.rpt = 8; }
  else { sh.nbh = 1; sh.rpt = 16; }
  const int rows = (m + sh.rpt - 1) / sh.rpt;
  sh.nt = ((rows + 63) / 64) * 64;
  if (sh.nt > 512) sh.nt = 512;
  if (sh.nt < 64) sh.nt = 64;
  sh.ns = sh.nbh < m / 2 ? sh.nbh : m / 2;
  return sh;
}

hipError_t launch_pf_panel(const double* A, long long astride, long long plane, int ld, int m, int nmat,
                           double* L, double* RM, long long lstride, long long l_im, int* perm, int pstride,
                           double* acc, int first, int* status, hipStream_t s) {
  const PfPanelShape sh = pf_panel_shape(m);
  const size_t lds = pf_panel_lds_bytes(m, sh.nbh);
#define PF_LAUNCH(NB, RP)                                                                               \
  hipLaunchKernelGGL((k_pf_panel<NB, RP>), dim3(nmat), dim3(sh.nt), lds, s, A, astride, plane, ld, m, L, \
                     RM, lstride, l_im, perm, pstride, acc, first, status)
  if (sh.nbh == 16) PF_LAUNCH(16, 1);
  else if (sh.nbh == 8) PF_LAUNCH(8, 2);
  else if (sh.nbh == 4) PF_LAUNCH(4, 4);
  else if (sh.nbh == 2) PF_LAUNCH(2, 8);
  else PF_LAUNCH(1, 16);
#undef PF_LAUNCH
  return hipGetLastError();
}

}  // namespace sgs
