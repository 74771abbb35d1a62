// Observables of an SGS state |psi> = sum_mu lambda_mu |phi_mu> (Sec. IV).
//
// Expectation of a Majorana polynomial O (Sec. IV.B, Eq. Cr):
//   <psi|O|psi> = sum_{mu,b} lambda_mu^* lambda_b G_{mu b} <O>_t(Delta^{b mu}),
// with the transition value of a sorted distinct word c_k1 .. c_km given by
// Wick's theorem (Sec. III.B): i^{m/2} Pf(Delta[w, w]) (1 for m = 0).
//
// Renyi-2 entropy of the subsystem A = Majoranas 0 .. nA-1 (Eq. S2_SGS,
// App. B): Tr rho_A^2 = sum_{a,b,g,d} lambda_a lambda_b^* lambda_g lambda_d^*
// G_ba G_dg Tr_A(rho^{ab}_A rho^{gd}_A), where rho^{ab} = |a><b| / <b|a> is a
// Gaussian operator whose two-point matrix on A is Delta^{ab}_A
// (Delta^{aa} = Gamma_a), and the trace of a product of two such operators on
// N_A = nA / 2 modes is 2^{-N_A} Pf([[D_1, i 1], [-i 1, D_2]]).
//
// Variance of the Hamiltonian, Eq. (residual): delta_H^2 = <H^2> - <H>^2.
// On the transition operator of a pair Wick's theorem holds for any product
// with the two-point matrix K = 1 + i Delta (K_kl = <c_k c_l>_t, K_kk = 1).
// With H = e0 + H2 + H4, H2 = sum_{k<l} alpha_kl c_k c_l (alpha = 2 i A) and
// H4 = sum_q u_q c_q0 c_q1 c_q2 c_q3 (Sec. II.A):
//   <H2>_t = -2 sum_{k<l} A_kl Delta_kl,
//   <H2 H2>_t = <H2>_t^2 + (1/2) Tr(alpha K alpha K^T)
//             = <H2>_t^2 + 2 |A|_F^2 - 2 Tr(U U),  U = A Delta
// (K^T = 2 - K; with A and Delta skew the terms linear in U cancel and
// U_ji = (Delta A)_ij, so Tr(U U) = sum_ij (A Delta)_ij (Delta A)_ij: both
// factors combine rows of Delta), and every product with a quartic word is
// the Pfaffian of the contraction matrix of its 6 or 8 Majoranas
// (M_ab = K_{i_a i_b}, a < b).
//
// Storage: the pair p = (a < b) keeps W = (Gamma_a + Gamma_b)^{-1} and
// Im Delta^{ba}; Delta^{ba} = -2 W + i Im, Delta^{ab} = its conjugate.
#include "obs_common.h"

namespace sgs {

// block-wide complex sum in a fixed order (deterministic); red holds blockDim.x
// entries, blockDim.x a power of two
__device__ cd block_sum(cd v, cd* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) { red[t].r += red[t + h].r; red[t].i += red[t + h].i; }
    __syncthreads();
  }
  cd r = red[0];
  __syncthreads();
  return r;
}

// grid: npoly blocks of 256 threads.  rows: 6 ints per term (poly, m, k0..k3),
// sorted by polynomial with offsets off[npoly + 1]; coef: complex per term.
__global__ __launch_bounds__(256) void k_obs_poly(ObsState s, const int* __restrict__ rows,
                                                  const double* __restrict__ coef, const int* __restrict__ off,
                                                  double* __restrict__ out) {
  __shared__ cd red[256];
  const int t = blockIdx.x;
  const int t0 = off[t], nterm = off[t + 1] - t0;
  const int R = s.R;
  cd acc{0.0, 0.0};
  for (long long e = threadIdx.x; e < (long long)R * R * nterm; e += blockDim.x) {
    const int term = t0 + (int)(e % nterm);
    const int mb = (int)(e / nterm);
    const int mu = mb / R, b = mb % R;
    const int* w = rows + 6 * term;
    const int m = w[1];
    cd v{1.0, 0.0};
    if (m == 2) {
      const cd d = delta_at(s, b, mu, w[2], w[3]);
      v = {-d.i, d.r};  // i d
    } else if (m == 4) {
      const cd d01 = delta_at(s, b, mu, w[2], w[3]), d23 = delta_at(s, b, mu, w[4], w[5]);
      const cd d02 = delta_at(s, b, mu, w[2], w[4]), d13 = delta_at(s, b, mu, w[3], w[5]);
      const cd d03 = delta_at(s, b, mu, w[2], w[5]), d12 = delta_at(s, b, mu, w[3], w[4]);
      const cd x = cmul(d01, d23), y = cmul(d02, d13), z = cmul(d03, d12);
      v = {-(x.r - y.r + z.r), -(x.i - y.i + z.i)};  // i^2 Pf4
    }
    const cd c{coef[2 * term], coef[2 * term + 1]};
    const cd wgt = cmul(cmul(cconj(lam_at(s, mu)), lam_at(s, b)), g_at(s, mu, b));
    const cd r = cmul(cmul(wgt, c), v);
    acc.r += r.r;
    acc.i += r.i;
  }
  const cd tot = block_sum(acc, red);
  if (threadIdx.x == 0) { out[2 * t] = tot.r; out[2 * t + 1] = tot.i; }
}

// ---- variance of H ----

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.r - b.r, a.i - b.i}; }

// K_ij = <c_i c_j>_t of the transition matrix Delta^{xy}
__device__ __forceinline__ cd kval(const ObsState& s, int x, int y, int i, int j) {
  if (i == j) return {1.0, 0.0};
  const cd d = delta_at(s, x, y, i, j);
  return {-d.i, d.r};
}

// Pfaffians of the contraction matrix M (upper entries M[a][b], a < b) of an
// ordered product, by expansion along the first index
__device__ cd pf4p(const cd (&M)[8][8], int a, int b, int c, int d) {
  return cadd(csub(cmul(M[a][b], M[c][d]), cmul(M[a][c], M[b][d])), cmul(M[a][d], M[b][c]));
}
__device__ cd pf6p(const cd (&M)[8][8], const int* p) {
  cd r{0.0, 0.0};
#pragma unroll
  for (int j = 1; j < 6; ++j) {
    int q[4], t = 0;
#pragma unroll
    for (int x = 1; x < 6; ++x)
      if (x != j) q[t++] = p[x];
    const cd v = cmul(M[p[0]][p[j]], pf4p(M, q[0], q[1], q[2], q[3]));
    r = (j & 1) ? cadd(r, v) : csub(r, v);
  }
  return r;
}
__device__ cd pf8p(const cd (&M)[8][8]) {
  cd r{0.0, 0.0};
  for (int j = 1; j < 8; ++j) {
    int q[6], t = 0;
    for (int x = 1; x < 8; ++x)
      if (x != j) q[t++] = x;
    const cd v = cmul(M[0][j], pf6p(M, q));
    r = (j & 1) ? cadd(r, v) : csub(r, v);
  }
  return r;
}
// <c_i0 ... c_i(m-1)>_t, m = 4, 6, 8
__device__ cd wick_product(const ObsState& s, int x, int y, const int* idx, int m) {
  cd M[8][8];
  for (int a = 0; a < m; ++a)
    for (int b = a + 1; b < m; ++b) M[a][b] = kval(s, x, y, idx[a], idx[b]);
  if (m == 4) return pf4p(M, 0, 1, 2, 3);
  if (m == 6) {
    const int p[6] = {0, 1, 2, 3, 4, 5};
    return pf6p(M, p);
  }
  return pf8p(M);
}

// Blocks (mu, b) with b <= mu, m = mu (mu + 1) / 2 + b: block (mu, b) works on
// Delta^{b mu}; the block (b, mu) is its complex conjugate (H and H^2 are
// Hermitian) and is not computed.  Chunk `chunk` of block m writes five
// complex partial sums to part[(m VAR_CHUNKS + chunk) 10 ..]: Tr(U U) (by
// k_var_uu), <H2>_t, <H4>_t, <H2 H4 + H4 H2>_t, <H4 H4>_t (by k_var_part).
__device__ __forceinline__ int tri_row(int m) {
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= m) ++r;
  return r;
}

// grid: (R (R + 1) / 2, VAR_CHUNKS), 512 threads.  Tr(U U) = sum_ij U_ij U_ji
// by 64 x 64 tiles: for tiles I >= J the block stores U[I, J] in LDS, then
// forms U[J, I] and multiplies entrywise with the transposed tile
// (off-diagonal tile pairs count twice).  Row i of U is
// -sum_{k in column i} A_ki Delta_k,: (A skew), so a wave walks one column of
// A for all 64 lanes and reads 64 consecutive entries of a row of Delta.
constexpr int VAR_T = 64;
constexpr int VAR_NW = 8;                // waves per block
constexpr int VAR_RPW = VAR_T / VAR_NW;  // tile rows per wave

// U_{r_k, c} = -sum_{q in column r_k} A_{row q, r_k} Delta_{row q, c} for the
// rows r_k = r0 + VAR_NW k of one wave (zero for r_k >= n or c >= n).  The
// rows advance together, one nonzero each per step, with clamped indices and
// zero weights past a column's end, so each step has VAR_RPW independent loads.
__device__ __forceinline__ void u_rows(const ObsState& s, const VarHam& h, int x, int y, int r0, int c,
                                       double (&er)[VAR_RPW], double (&ei)[VAR_RPW]) {
  const int n = s.n;
  int beg[VAR_RPW], len[VAR_RPW], mx = 0;
#pragma unroll
  for (int k = 0; k < VAR_RPW; ++k) {
    const int i = r0 + VAR_NW * k;
    beg[k] = i < n ? h.colptr[i] : 0;
    len[k] = i < n ? h.colptr[i + 1] - beg[k] : 0;
    mx = max(mx, len[k]);
    er[k] = 0.0;
    ei[k] = 0.0;
  }
  const bool cin = c < n;
  const int cc = cin ? c : n - 1;
  for (int t = 0; t < mx; ++t) {  // mx > 0 only if A has nonzeros
#pragma unroll
    for (int k = 0; k < VAR_RPW; ++k) {
      const bool v = t < len[k];
      const int q = v ? beg[k] + t : 0;
      const double a = v && cin ? h.colval[q] : 0.0;
      const cd d = delta_at(s, x, y, h.rowidx[q], cc);
      er[k] -= a * d.r;
      ei[k] -= a * d.i;
    }
  }
}

__global__ __launch_bounds__(VAR_NW * 64) void k_var_uu(ObsState s, VarHam h, double* __restrict__ part) {
  __shared__ double ur[VAR_T][VAR_T + 1], ui[VAR_T][VAR_T + 1];
  __shared__ cd red[VAR_NW * 64];
  const int n = s.n;
  const int m = blockIdx.x, ch = blockIdx.y;
  const int mu = tri_row(m), b = m - mu * (mu + 1) / 2;
  const int x = b, y = mu;  // Delta^{b mu}
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cd tuu{0.0, 0.0};
  const int nt = (n + VAR_T - 1) / VAR_T;
  for (int tp = ch; tp < nt * (nt + 1) / 2; tp += VAR_CHUNKS) {
    const int I = tri_row(tp);
    const int J = tp - I * (I + 1) / 2;  // J <= I
    const int i0 = I * VAR_T, j0 = J * VAR_T;
    double er[VAR_RPW], ei[VAR_RPW];
    u_rows(s, h, x, y, i0 + wv, j0 + lane, er, ei);  // U[i0 + r, j0 + lane]
#pragma unroll
    for (int k = 0; k < VAR_RPW; ++k) {
      ur[wv + VAR_NW * k][lane] = er[k];
      ui[wv + VAR_NW * k][lane] = ei[k];
    }
    __syncthreads();
    u_rows(s, h, x, y, j0 + wv, i0 + lane, er, ei);  // U[j0 + r, i0 + lane]
    cd acc{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < VAR_RPW; ++k) {
      const int r = wv + VAR_NW * k;
      acc = cadd(acc, cmul(cd{er[k], ei[k]}, cd{ur[lane][r], ui[lane][r]}));
    }
    __syncthreads();
    const double f = I == J ? 1.0 : 2.0;
    tuu.r += f * acc.r;
    tuu.i += f * acc.i;
  }
  const cd sum = block_sum(tuu, red);
  if (threadIdx.x == 0) {
    double* o = part + ((long long)m * VAR_CHUNKS + ch) * 10;
    o[0] = sum.r;
    o[1] = sum.i;
  }
}

// grid: (R (R + 1) / 2, VAR_CHUNKS), 256 threads: the sums over the sparse
// quadratic part and the quartic words
__global__ __launch_bounds__(256) void k_var_part(ObsState s, VarHam h, double* __restrict__ part) {
  __shared__ cd red[256];
  const int m = blockIdx.x, ch = blockIdx.y;
  const int mu = tri_row(m), b = m - mu * (mu + 1) / 2;
  const int x = b, y = mu;  // Delta^{b mu}
  const int stride = VAR_CHUNKS * blockDim.x;
  const int t0 = ch * blockDim.x + threadIdx.x;
  cd h2{0.0, 0.0}, h4{0.0, 0.0}, hx{0.0, 0.0}, h44{0.0, 0.0};
  // <H2>_t = sum_{k<l} alpha_kl K_kl = -2 sum_{k<l} A_kl Delta_kl
  for (int u = t0; u < h.nnz_up; u += stride) {
    const cd d = delta_at(s, x, y, h.up_k[u], h.up_l[u]);
    h2.r -= 2.0 * h.up_v[u] * d.r;
    h2.i -= 2.0 * h.up_v[u] * d.i;
  }
  for (int q = t0; q < h.nq; q += stride) {
    const cd v = wick_product(s, x, y, h.q_idx + 4 * q, 4);
    h4.r += h.q_val[q] * v.r;
    h4.i += h.q_val[q] * v.i;
  }
  // quadratic x quartic, both orders: alpha_kl u_q (<c_k c_l w_q> + <w_q c_k c_l>)
  for (long long e = t0; e < (long long)h.nnz_up * h.nq; e += stride) {
    const int u = (int)(e / h.nq), q = (int)(e - (long long)u * h.nq);
    const int* w = h.q_idx + 4 * q;
    const int k = h.up_k[u], l = h.up_l[u];
    const int i1[6] = {k, l, w[0], w[1], w[2], w[3]};
    const int i2[6] = {w[0], w[1], w[2], w[3], k, l};
    const cd v = cadd(wick_product(s, x, y, i1, 6), wick_product(s, x, y, i2, 6));
    const cd c = cmul(cd{0.0, 2.0 * h.up_v[u]}, cd{h.q_val[q], 0.0});
    hx = cadd(hx, cmul(c, v));
  }
  for (int e = t0; e < h.nq * h.nq; e += stride) {
    const int q1 = e / h.nq, q2 = e - q1 * h.nq;
    int i8[8];
    for (int a = 0; a < 4; ++a) { i8[a] = h.q_idx[4 * q1 + a]; i8[4 + a] = h.q_idx[4 * q2 + a]; }
    const cd v = wick_product(s, x, y, i8, 8);
    const double c = h.q_val[q1] * h.q_val[q2];
    h44.r += c * v.r;
    h44.i += c * v.i;
  }
  const cd sums[4] = {block_sum(h2, red), block_sum(h4, red), block_sum(hx, red), block_sum(h44, red)};
  if (threadIdx.x == 0) {
    double* o = part + ((long long)m * VAR_CHUNKS + ch) * 10;
    for (int k = 0; k < 4; ++k) { o[2 + 2 * k] = sums[k].r; o[3 + 2 * k] = sums[k].i; }
  }
}

// one workgroup: per block (mu, b) <H'>_t = <H2>_t + <H4>_t and
// <H'^2>_t = <H2>_t^2 + 2 |A|_F^2 - 2 Tr(U U) + <H2 H4 + H4 H2>_t + <H4 H4>_t
// (H' = H - e0), weighted by lambda_mu^* lambda_b G_{mu b}, the block (b, mu)
// taking the conjugate values; out = {<H>, <H^2>, delta_H^2}, normalized by
// sum lambda_mu^* lambda_b G_{mu b}
__global__ __launch_bounds__(256) void k_var_final(ObsState s, const double* __restrict__ part, double e0,
                                                   double a2, double* __restrict__ out) {
  __shared__ cd red[256];
  const int R = s.R;
  cd s1{0.0, 0.0}, s2{0.0, 0.0}, nr{0.0, 0.0};
  for (int m = threadIdx.x; m < R * (R + 1) / 2; m += blockDim.x) {
    cd v[5];
    for (int k = 0; k < 5; ++k) v[k] = {0.0, 0.0};
    for (int ch = 0; ch < VAR_CHUNKS; ++ch) {
      const double* o = part + ((long long)m * VAR_CHUNKS + ch) * 10;
      for (int k = 0; k < 5; ++k) { v[k].r += o[2 * k]; v[k].i += o[2 * k + 1]; }
    }
    const cd X = cadd(v[1], v[2]);
    cd Y = cmul(v[1], v[1]);
    Y.r += 2.0 * a2 - 2.0 * v[0].r;
    Y.i -= 2.0 * v[0].i;
    Y = cadd(cadd(Y, v[3]), v[4]);
    const int mu = tri_row(m), b = m - mu * (mu + 1) / 2;
    const cd c = cmul(cmul(cconj(lam_at(s, mu)), lam_at(s, b)), g_at(s, mu, b));
    s1 = cadd(s1, cmul(c, X));
    s2 = cadd(s2, cmul(c, Y));
    nr = cadd(nr, c);
    if (b != mu) {
      const cd ct = cmul(cmul(cconj(lam_at(s, b)), lam_at(s, mu)), g_at(s, b, mu));
      s1 = cadd(s1, cmul(ct, cconj(X)));
      s2 = cadd(s2, cmul(ct, cconj(Y)));
      nr = cadd(nr, ct);
    }
  }
  const cd S1 = block_sum(s1, red), S2 = block_sum(s2, red), N = block_sum(nr, red);
  if (threadIdx.x == 0) {
    const double d = N.r * N.r + N.i * N.i;
    const cd inv{N.r / d, -N.i / d};
    const cd x = cmul(S1, inv), yv = cmul(S2, inv);
    const cd xx = cmul(x, x);
    out[0] = e0 + x.r;
    out[1] = e0 * e0 + 2.0 * e0 * x.r + yv.r;
    out[2] = yv.r - xx.r;
  }
}

hipError_t launch_variance(const ObsState& s, const VarHam& h, double e0, double a2, double* part, double* out,
                           hipStream_t st) {
  if (s.R < 1 || s.R > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_var_uu, dim3(s.R * (s.R + 1) / 2, VAR_CHUNKS), dim3(VAR_NW * 64), 0, st, s, h, part);
  hipLaunchKernelGGL(k_var_part, dim3(s.R * (s.R + 1) / 2, VAR_CHUNKS), dim3(256), 0, st, s, h, part);
  hipLaunchKernelGGL(k_var_final, dim3(1), dim3(256), 0, st, s, (const double*)part, e0, a2, out);
  return hipGetLastError();
}

hipError_t launch_obs_poly(const ObsState& s, const int* rows, const double* coef, const int* off, int npoly,
                           double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_obs_poly, dim3(npoly), dim3(256), 0, st, s, rows, coef, off, out);
  return hipGetLastError();
}

}  // namespace sgs
