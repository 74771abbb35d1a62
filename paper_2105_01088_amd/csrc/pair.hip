// Per-pair kernels that are not dense contractions (HBM- or latency-bound).
//
// Notation: for the unordered pair p = (a < b) the library keeps
//   W   = (Gamma_a + Gamma_b)^{-1}                     (gj.hip)
//   Di  = Im Delta^{ba} = 2 Gamma_b W - 1               (one GEMM)
// so that Delta^{ba} = -2 W + i Di (Eq. def-delta-matrix with a, b swapped)
// and Delta^{ab} = conj(Delta^{ba}) (A and u are real).
//
//   <phi_a| c_k c_l |phi_b> = i G_ab Delta^{ba}_kl      (Sec. III.B)
//   eps_ab = h_ab / G_ab = e0 + Tr(A Delta^{ba}) - sum_q u_q Pf4(Delta^{ba}[q])
//   F^{ba} = A + 6 U Delta^{ba}: differs from A on the impurity block only;
//            a quartic word (q0<q1<q2<q3) with coefficient u adds
//            F_{q0q1} += u/2 D_{q2q3}, F_{q0q2} -= u/2 D_{q1q3}, F_{q0q3} += u/2 D_{q1q2},
//            F_{q1q2} += u/2 D_{q0q3}, F_{q1q3} -= u/2 D_{q0q2}, F_{q2q3} += u/2 D_{q0q1}
//            (and the skew partners).
//   Words of m = 6 or 8 Majoranas (term v i^((m/2) mod 2) c_w, v real): the
//   transition value is i^(m/2) Pf(Delta[w]), so eps gains v Pf(Delta[w]);
//   F, minus half the derivative of <H>_t in the entries Delta_kl (k < l),
//   which is A + 6 U Delta for quartic words, gains for positions a < b
//            F_{w_a w_b} += -(v / 2) (-1)^(a+b+1) Pf(Delta[w without a, b])
//   (the Pfaffian cofactor of entry (a, b)) and the skew partner.
#include "sgs_internal.h"

namespace sgs {

// S_p = Gamma_a + Gamma_b for every pair; also clears ln|det| accumulators.
__global__ void k_pair_sum(const double* __restrict__ gam, int n, const int* __restrict__ pa,
                           const int* __restrict__ pb, double* __restrict__ S,
                           double* __restrict__ logdet) {
  const int p = blockIdx.y;
  const long long nn = (long long)n * n;
  const double* ga = gam + pa[p] * nn;
  const double* gb = gam + pb[p] * nn;
  double* sp = S + p * nn;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x)
    sp[e] = ga[e] + gb[e];
  if (blockIdx.x == 0 && threadIdx.x == 0) logdet[p] = 0.0;
}

// Complex helpers.
struct cplx {
  double r, i;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.r - b.r, a.i - b.i}; }


// Delta element reader: pair (-2W + i Di) or diagonal (Gamma, real)
__device__ __forceinline__ cplx dget(const double* W, const double* Di, const double* G, int n, int k, int l) {
  if (G) return {G[(long long)k * n + l], 0.0};
  return {-2.0 * W[(long long)k * n + l], Di[(long long)k * n + l]};
}

// Pfaffian of Delta[x, x] for K = 0, 2, 4, 6 or 8 increasing indices x, by
// expansion along the first row (no pivots, no division)
template <int K>
__device__ cplx pf_idx(const double* W, const double* Di, const double* G, int n, const int* x) {
  if constexpr (K == 0) {
    return {1.0, 0.0};
  } else if constexpr (K == 2) {
    return dget(W, Di, G, n, x[0], x[1]);
  } else {
    cplx r{0.0, 0.0};
#pragma unroll 1
    for (int j = 1; j < K; ++j) {
      int rest[K - 2];
#pragma unroll
      for (int i = 1; i < K - 1; ++i) rest[i - 1] = x[i < j ? i : i + 1];
      const cplx v = cmul(dget(W, Di, G, n, x[0], x[j]), pf_idx<K - 2>(W, Di, G, n, rest));
      r = (j & 1) ? cadd(r, v) : csub(r, v);  // sign (-1)^(j+1)
    }
    return r;
  }
}

// grid: P + R blocks (pairs first, then the diagonal states), 256 threads.
//   eps_out[blk] = eps (complex); Fc_out[blk] = 6 U Delta on the impurity block
//   (M x M, planar: re plane then im plane).
__global__ __launch_bounds__(256) void k_eps_fock(HamDev h, int P, const double* __restrict__ W,
                                                  const double* __restrict__ Di,
                                                  const double* __restrict__ gam,
                                                  const int* __restrict__ pa, const int* __restrict__ pb,
                                                  double* __restrict__ eps_out, double* __restrict__ Fc_out) {
  __shared__ double redr[256], redi[256];
  const int blk = blockIdx.x;
  const int n = h.n;
  const long long nn = (long long)n * n;
  const double *w = nullptr, *di = nullptr, *g = nullptr;
  if (blk < P) { w = W + blk * nn; di = Di + blk * nn; }
  else g = gam + (long long)(blk - P) * nn;

  // Tr(A Delta) = -2 sum_{k<l} A_kl Delta_kl
  double sr = 0.0, si = 0.0;
  for (int e = threadIdx.x; e < h.nnz_up; e += blockDim.x) {
    cplx d = dget(w, di, g, n, h.up_k[e], h.up_l[e]);
    sr += -2.0 * h.up_v[e] * d.r;
    si += -2.0 * h.up_v[e] * d.i;
  }
  // quartic words: <c c c c>_t = i^2 Pf4(Delta[q]) -> -u Pf4
  for (int q = threadIdx.x; q < h.nq; q += blockDim.x) {
    const int* x = h.q_idx + 4 * q;
    cplx d01 = dget(w, di, g, n, x[0], x[1]), d02 = dget(w, di, g, n, x[0], x[2]);
    cplx d03 = dget(w, di, g, n, x[0], x[3]), d12 = dget(w, di, g, n, x[1], x[2]);
    cplx d13 = dget(w, di, g, n, x[1], x[3]), d23 = dget(w, di, g, n, x[2], x[3]);
    cplx pf = cadd(csub(cmul(d01, d23), cmul(d02, d13)), cmul(d03, d12));
    sr -= h.q_val[q] * pf.r;
    si -= h.q_val[q] * pf.i;
  }
  redr[threadIdx.x] = sr;
  redi[threadIdx.x] = si;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      redr[threadIdx.x] += redr[threadIdx.x + off];
      redi[threadIdx.x] += redi[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    eps_out[2 * blk] = redr[0] + h.e0;
    eps_out[2 * blk + 1] = redi[0];
  }
  // impurity-block Fock correction (serial: a handful of words)
  const int M = h.M;
  double* fr = Fc_out + (long long)blk * 2 * M * M;
  double* fi = fr + M * M;
  for (int e = threadIdx.x; e < M * M; e += blockDim.x) { fr[e] = 0.0; fi[e] = 0.0; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < h.nq; ++q) {
      const int* x = h.q_idx + 4 * q;
      const int* y = h.q_loc + 4 * q;
      const double hu = 0.5 * h.q_val[q];
      // (row, col, partner pair, sign)
      const int rc[6][5] = {{0, 1, 2, 3, 1}, {0, 2, 1, 3, -1}, {0, 3, 1, 2, 1},
                            {1, 2, 0, 3, 1}, {1, 3, 0, 2, -1}, {2, 3, 0, 1, 1}};
      for (int t = 0; t < 6; ++t) {
        cplx d = dget(w, di, g, n, x[rc[t][2]], x[rc[t][3]]);
        const double s = hu * rc[t][4];
        const int r = y[rc[t][0]], c = y[rc[t][1]];
        fr[r * M + c] += s * d.r;
        fi[r * M + c] += s * d.i;
        fr[c * M + r] -= s * d.r;
        fi[c * M + r] -= s * d.i;
      }
    }
  }
}

// Words of 6 or 8 Majoranas, after k_eps_fock (same grid, 64 threads):
// eps += v Pf(Delta[w]); one thread per touched impurity entry (r < c) adds
// its cofactor items, in a fixed order, to F.  Kept apart so that the
// quartic-only kernel keeps its registers.
__global__ __launch_bounds__(64) void k_eps_fock_words(HamDev h, int P, const double* __restrict__ W,
                                                       const double* __restrict__ Di,
                                                       const double* __restrict__ gam,
                                                       double* __restrict__ eps_out, double* __restrict__ Fc_out) {
  __shared__ double redr[64], redi[64];
  const int blk = blockIdx.x;
  const int n = h.n, M = h.M;
  const long long nn = (long long)n * n;
  const double *w = nullptr, *di = nullptr, *g = nullptr;
  if (blk < P) { w = W + blk * nn; di = Di + blk * nn; }
  else g = gam + (long long)(blk - P) * nn;
  double sr = 0.0, si = 0.0;
  for (int q = threadIdx.x; q < h.nw; q += blockDim.x) {
    const int* x = h.w_idx + 8 * q;
    const cplx pf = h.w_len[q] == 6 ? pf_idx<6>(w, di, g, n, x) : pf_idx<8>(w, di, g, n, x);
    sr += h.w_val[q] * pf.r;
    si += h.w_val[q] * pf.i;
  }
  redr[threadIdx.x] = sr;
  redi[threadIdx.x] = si;
  __syncthreads();
  for (int off = 32; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      redr[threadIdx.x] += redr[threadIdx.x + off];
      redi[threadIdx.x] += redi[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    eps_out[2 * blk] += redr[0];
    eps_out[2 * blk + 1] += redi[0];
  }
  double* fr = Fc_out + (long long)blk * 2 * M * M;
  double* fi = fr + M * M;
  // words of 6 or 8: one thread per impurity entry (r < c), its cofactor
  // items in a fixed order
  for (int e = threadIdx.x; e < h.nfe; e += blockDim.x) {
    double ar = 0.0, ai = 0.0;
    for (int t = h.fe_off[e]; t < h.fe_off[e + 1]; ++t) {
      const int4 it = h.fe_item[t];
      const int* x = h.w_idx + 8 * it.x;
      const int m = h.w_len[it.x];
      // the word without positions a < b
      int rest[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) rest[i] = x[i < it.y ? i : (i + 1 < it.z ? i + 1 : i + 2)];
      const cplx pf = m == 6 ? pf_idx<4>(w, di, g, n, rest) : pf_idx<6>(w, di, g, n, rest);
      const double s = -0.5 * h.w_val[it.x] * (((it.y + it.z + 1) & 1) ? -1.0 : 1.0);
      ar += s * pf.r;
      ai += s * pf.i;
    }
    const int2 rc = h.fe_ent[e];
    fr[rc.x * M + rc.y] += ar;
    fi[rc.x * M + rc.y] += ai;
    fr[rc.y * M + rc.x] -= ar;
    fi[rc.y * M + rc.x] -= ai;
  }
}

// Y = Delta F for pairs (complex, planar) and Yd = Gamma F for the diagonal.
// A in compressed-column form; F = A + Fc on the impurity block.
// grid: (ceil(n*n / 256), P + R)

__global__ __launch_bounds__(256) void k_apply_fock(SparseA sa, int n, int P, const double* __restrict__ W,
                                                    const double* __restrict__ Di,
                                                    const double* __restrict__ gam,
                                                    const double* __restrict__ Fc,
                                                    double* __restrict__ Y, double* __restrict__ Yd) {
  const int blk = blockIdx.y;
  const long long nn = (long long)n * n;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / n), j = (int)(e - (long long)i * n);
  const int M = sa.M;
  const double* fr = Fc + (long long)blk * 2 * M * M;
  const double* fi = fr + M * M;
  const int jl = sa.impos[j];
  if (blk < P) {
    const double* w = W + blk * nn + (long long)i * n;
    const double* di = Di + blk * nn + (long long)i * n;
    double yr = 0.0, yi = 0.0;
    for (int q = sa.colptr[j]; q < sa.colptr[j + 1]; ++q) {
      const int k = sa.row[q];
      const double v = sa.val[q];
      yr += -2.0 * w[k] * v;
      yi += di[k] * v;
    }
    if (jl >= 0) {
      for (int kl = 0; kl < M; ++kl) {
        const int k = sa.imp[kl];
        const double xr = -2.0 * w[k], xi = di[k];
        const double cr = fr[kl * M + jl], ci = fi[kl * M + jl];
        yr += xr * cr - xi * ci;
        yi += xr * ci + xi * cr;
      }
    }
    double* y = Y + (long long)blk * 2 * nn;
    y[e] = yr;
    y[e + nn] = yi;
  } else {
    const int mu = blk - P;
    const double* g = gam + mu * nn + (long long)i * n;
    double y = 0.0;
    for (int q = sa.colptr[j]; q < sa.colptr[j + 1]; ++q) y += g[sa.row[q]] * sa.val[q];
    if (jl >= 0)
      for (int kl = 0; kl < M; ++kl) y += g[sa.imp[kl]] * fr[kl * M + jl];
    Yd[mu * nn + e] = y;
  }
}

// Dense A: Y = Delta A and Yd = Gamma A come from grouped GEMMs; this adds
// the impurity-block Fock correction Delta[:, imp] Fc (Gamma[:, imp] Fc_r for
// the states) on the M impurity columns.  grid: (ceil(n M / 256), P + R)
__global__ __launch_bounds__(256) void k_fock_imp(SparseA sa, int n, int P, const double* __restrict__ W,
                                                  const double* __restrict__ Di,
                                                  const double* __restrict__ gam,
                                                  const double* __restrict__ Fc,
                                                  double* __restrict__ Y, double* __restrict__ Yd) {
  const int blk = blockIdx.y;
  const int M = sa.M;
  const long long nn = (long long)n * n;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)n * M) return;
  const int i = (int)(e / M), jl = (int)(e - (long long)i * M);
  const int j = sa.imp[jl];
  const double* fr = Fc + (long long)blk * 2 * M * M;
  const double* fi = fr + M * M;
  const long long o = (long long)i * n + j;
  if (blk < P) {
    const double* w = W + blk * nn + (long long)i * n;
    const double* di = Di + blk * nn + (long long)i * n;
    double yr = 0.0, yi = 0.0;
    for (int kl = 0; kl < M; ++kl) {
      const int k = sa.imp[kl];
      const double xr = -2.0 * w[k], xi = di[k];
      const double cr = fr[kl * M + jl], ci = fi[kl * M + jl];
      yr += xr * cr - xi * ci;
      yi += xr * ci + xi * cr;
    }
    double* y = Y + (long long)blk * 2 * nn;
    y[o] += yr;
    y[o + nn] += yi;
  } else {
    const int mu = blk - P;
    const double* g = gam + mu * nn + (long long)i * n;
    double y = 0.0;
    for (int kl = 0; kl < M; ++kl) y += g[sa.imp[kl]] * fr[kl * M + jl];
    Yd[mu * nn + o] += y;
  }
}

hipError_t launch_fock_imp(const SparseA& sa, int n, int P, int R, const double* W, const double* Di,
                           const double* gam, const double* Fc, double* Y, double* Yd, hipStream_t s) {
  if (sa.M <= 0) return hipSuccess;
  const long long cnt = (long long)n * sa.M;
  hipLaunchKernelGGL(k_fock_imp, dim3((unsigned)((cnt + 255) / 256), P + R), dim3(256), 0, s, sa, n, P, W, Di,
                     gam, Fc, Y, Yd);
  return hipGetLastError();
}

// C_ab = i (Gamma_b + Gamma_0) - i X_a for 1 <= a < b, planar:
//   Re C = Im X_a = T_a^T - T_a  (T_a = Gamma_0 W_0a),
//   Im C = Gamma_b + Gamma_0 - Re X_a.
// grid: (ceil(n/32), ceil(n/32), Q), block 32 x 8
__global__ __launch_bounds__(256) void k_build_c(int n, const double* __restrict__ gam,
                                                 const double* __restrict__ T, const double* __restrict__ Xr,
                                                 const int* __restrict__ qa, const int* __restrict__ qb,
                                                 double* __restrict__ Cm) {
  __shared__ double tile[32][33];
  const int q = blockIdx.z;
  const int a = qa[q], b = qb[q];
  const long long nn = (long long)n * n;
  const double* t = T + (long long)(a - 1) * nn;
  const double* xr = Xr + (long long)(a - 1) * nn;
  const double* g0 = gam;
  const double* gb = gam + (long long)b * nn;
  double* cr = Cm + (long long)q * 2 * nn;
  double* ci = cr + nn;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  // load T[by.., bx..] transposed source: tile[y][x] = T[bx + y][by + x]
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    int r = bx + yy, c = by + threadIdx.x;
    tile[yy][threadIdx.x] = (r < n && c < n) ? t[(long long)r * n + c] : 0.0;
  }
  __syncthreads();
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    int r = by + yy, c = bx + threadIdx.x;
    if (r < n && c < n) {
      long long o = (long long)r * n + c;
      cr[o] = tile[threadIdx.x][yy] - t[o];
      ci[o] = gb[o] + g0[o] - xr[o];
    }
  }
}

hipError_t launch_pair_sum(const double* gam, int n, const int* pa, const int* pb, int P, double* S,
                           double* logdet, hipStream_t s) {
  long long nn = (long long)n * n;
  int bx = (int)((nn + 1023) / 1024);
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_pair_sum, dim3(bx, P), dim3(256), 0, s, gam, n, pa, pb, S, logdet);
  return hipGetLastError();
}

hipError_t launch_eps_fock(const HamDev& h, int P, int R, const double* W, const double* Di,
                           const double* gam, const int* pa, const int* pb, double* eps,
                           double* Fc, hipStream_t s) {
  hipLaunchKernelGGL(k_eps_fock, dim3(P + R), dim3(256), 0, s, h, P, W, Di, gam, pa, pb, eps, Fc);
  if (h.nw > 0) hipLaunchKernelGGL(k_eps_fock_words, dim3(P + R), dim3(64), 0, s, h, P, W, Di, gam, eps, Fc);
  return hipGetLastError();
}

hipError_t launch_apply_fock(const SparseA& sa, int n, int P, int R, const double* W, const double* Di,
                             const double* gam, const double* Fc, double* Y, double* Yd, hipStream_t s) {
  long long nn = (long long)n * n;
  hipLaunchKernelGGL(k_apply_fock, dim3((unsigned)((nn + 255) / 256), P + R), dim3(256), 0, s, sa, n, P,
                     W, Di, gam, Fc, Y, Yd);
  return hipGetLastError();
}

hipError_t launch_build_c(int n, const double* gam, const double* T, const double* Xr, const int* qa,
                          const int* qb, int Q, double* Cm, hipStream_t s) {
  if (Q <= 0) return hipSuccess;
  dim3 g((n + 31) / 32, (n + 31) / 32, Q);
  hipLaunchKernelGGL(k_build_c, g, dim3(32, 8), 0, s, n, gam, T, Xr, qa, qb, Cm);
  return hipGetLastError();
}

// Transition matrices for the caller (Eq. def-delta-matrix):
// Delta^{ba} = -2 W + i Im Delta^{ba}, complex interleaved, for the pairs
// (a < b) in order.
__global__ __launch_bounds__(256) void k_delta_out(const double* __restrict__ W, const double* __restrict__ Di,
                                                   long long total, double* __restrict__ out) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    out[2 * e] = -2.0 * W[e];
    out[2 * e + 1] = Di[e];
  }
}

hipError_t launch_delta_out(const double* W, const double* Di, long long total, double* out, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  long long b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(k_delta_out, dim3((int)b), dim3(256), 0, s, W, Di, total, out);
  return hipGetLastError();
}

}  // namespace sgs
