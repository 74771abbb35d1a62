// Renyi-2 entropy of the subsystem A = Majoranas 0 .. nA-1 of an SGS state
// (App. B, Eqs. S2_SGS, TrArho2_final, pfMA):
//   Tr rho_A^2 = sum over ordered pairs of states p = (a, b), q = (g, d) of
//   T(p, q) = lambda_a lambda_b^* lambda_g lambda_d^* G_ba G_dg 2^{-N_A} Pf(Z_pq),
//   Z_pq = [[K_p, i 1], [-i 1, K_q]],   K_ab = Delta^{ab} on A, K_aa = Gamma_a on A,
// N_A = nA / 2 modes.  The rank-4 tensor T has two symmetries: the exchange
// of the two blocks, T(p, q) = T(q, p), and conjugation, T(p*, q*) = T(p, q)^*
// with (a, b)* = (b, a), because K_ba = K_ab^* and G_ab = G_ba^*.  The sum is
// real, so one representative of each orbit contributes w Re T with w its
// orbit size (about R^4 / 4 Pfaffians instead of R^4); the host lists the
// representatives.
//
// Pf(Z_pq) is taken in one of two forms:
//  * block form: the Pfaffian of order 2 nA, no assumption on the blocks;
//  * split form: Pf(Z_pq) = Pf(K_q) Pf(K_p - K_q^{-1}), of order nA, which
//    needs the inverse of one block.  Which block is inverted is free (the
//    exchange symmetry); the host inverts the one with the smaller condition
//    number and keeps the block form for terms where neither block is well
//    conditioned (an impurity state with a mode half in A has a singular
//    Gamma_a on A).
// Small subsystems (2 nA <= 64) take the block form in LDS, one wave per
// term.  Larger ones build batches of matrices for the batched blocked
// Pfaffian of the overlap phase (pfaff.hip): the blocks K_u (u = (x <= y))
// once, with their inverses and condition numbers, then the split or block
// matrices of every term.
#include "obs_common.h"

namespace sgs {

// ---- small subsystems: block form in LDS, one wave per term ----

// Pfaffian of the m x m complex skew matrix in LDS (planes Zr / Zi, leading
// dimension ld, m <= 64) by elimination with 2 x 2 pivots and symmetric
// row / column exchanges (each a sign flip); lane j updates column j.
// Returns false for a vanishing pivot column (Pf = 0).
__device__ bool lds_pfaffian(double* Zr, double* Zi, int m, int ld, double& la, double& pr, double& pi) {
  const int lane = threadIdx.x;
  la = 0.0; pr = 1.0; pi = 0.0;
  for (int k = 0; k < m; k += 2) {
    // pivot: largest |Z[i][k]|, i > k (lane i)
    double best = -1.0;
    int bi = k + 1;
    if (lane > k && lane < m) {
      const double xr = Zr[lane * ld + k], xi = Zi[lane * ld + k];
      best = xr * xr + xi * xi;
      bi = lane;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const int q = bi;
    if (q != k + 1) {
      if (lane < m) {
        double t = Zr[q * ld + lane]; Zr[q * ld + lane] = Zr[(k + 1) * ld + lane]; Zr[(k + 1) * ld + lane] = t;
        t = Zi[q * ld + lane]; Zi[q * ld + lane] = Zi[(k + 1) * ld + lane]; Zi[(k + 1) * ld + lane] = t;
      }
      __syncthreads();
      if (lane < m) {
        double t = Zr[lane * ld + q]; Zr[lane * ld + q] = Zr[lane * ld + k + 1]; Zr[lane * ld + k + 1] = t;
        t = Zi[lane * ld + q]; Zi[lane * ld + q] = Zi[lane * ld + k + 1]; Zi[lane * ld + k + 1] = t;
      }
      __syncthreads();
      pr = -pr;
      pi = -pi;
    }
    const double ar = Zr[k * ld + k + 1], ai = Zi[k * ld + k + 1];
    const double a2 = ar * ar + ai * ai;
    if (!(a2 > 0.0)) return false;
    la += 0.5 * log(a2);
    {
      const double nr = pr * ar - pi * ai, ni = pr * ai + pi * ar;
      const double nm = 1.0 / sqrt(nr * nr + ni * ni);
      pr = nr * nm;
      pi = ni * nm;
    }
    // Z[i][j] += (Z[k+1][i] Z[k][j] - Z[k][i] Z[k+1][j]) / a for i, j >= k + 2
    const double ir = ar / a2, ii = -ai / a2;
    if (lane >= k + 2 && lane < m) {
      const int j = lane;
      const cd b0j{Zr[k * ld + j], Zi[k * ld + j]}, b1j{Zr[(k + 1) * ld + j], Zi[(k + 1) * ld + j]};
      for (int i = k + 2; i < m; ++i) {
        const cd b0i{Zr[k * ld + i], Zi[k * ld + i]}, b1i{Zr[(k + 1) * ld + i], Zi[(k + 1) * ld + i]};
        const cd x = cmul(b1i, b0j), y = cmul(b0i, b1j);
        const cd u = cmul(cd{x.r - y.r, x.i - y.i}, cd{ir, ii});
        Zr[i * ld + j] += u.r;
        Zi[i * ld + j] += u.i;
      }
    }
    __syncthreads();
  }
  return true;
}

// w Re T(p, q) from ln|Pf|, the unit phase of the Pfaffian(s) and the
// coefficient lambda_a lambda_b^* lambda_g lambda_d^* G_ba G_dg (log form)
__device__ double term_value(const ObsState& s, int nA, RenTerm t, double la, cd ph) {
  const int R = s.R;
  const int a = t.p / R, b = t.p % R, g = t.q / R, d = t.q % R;
  const cd c = cmul(cmul(cmul(lam_at(s, a), cconj(lam_at(s, b))), cmul(lam_at(s, g), cconj(lam_at(s, d)))),
                    cmul(g_at(s, b, a), g_at(s, d, g)));
  const double cm = sqrt(c.r * c.r + c.i * c.i);
  if (!(cm > 0.0) || !isfinite(la)) return 0.0;
  const double ln2 = 0.69314718055994530942;
  const double mag = exp(log(cm) + la - 0.5 * nA * ln2);  // 2^{-N_A}
  const cd v = cmul(cd{c.r / cm, c.i / cm}, ph);
  return t.w * mag * v.r;
}

// grid: nterm blocks of one wave; dynamic LDS: two m x (m + 1) planes, m = 2 nA <= 64
__global__ __launch_bounds__(64) void k_ren_lds(ObsState s, int nA, const RenTerm* __restrict__ terms,
                                                double* __restrict__ tval) {
  extern __shared__ double zs[];
  const int m = 2 * nA, ld = m + 1;
  double* Zr = zs;
  double* Zi = zs + m * ld;
  const RenTerm t = terms[blockIdx.x];
  const int R = s.R;
  const int a = t.p / R, b = t.p % R, g = t.q / R, d = t.q % R;
  for (int e = threadIdx.x; e < m * m; e += 64) {
    const int i = e / m, j = e % m;
    cd v{0.0, 0.0};
    if (i < nA && j < nA) v = delta_at(s, a, b, i, j);
    else if (i >= nA && j >= nA) v = delta_at(s, g, d, i - nA, j - nA);
    else if (i < nA && j == i + nA) v = {0.0, 1.0};
    else if (i >= nA && i == j + nA) v = {0.0, -1.0};
    Zr[i * ld + j] = v.r;
    Zi[i * ld + j] = v.i;
  }
  __syncthreads();
  double la, pr, pi;
  const bool nz = lds_pfaffian(Zr, Zi, m, ld, la, pr, pi);
  if (threadIdx.x == 0) tval[blockIdx.x] = nz ? term_value(s, nA, t, la, cd{pr, pi}) : 0.0;
}

// ---- batched path ----

// class index of the unordered pair x <= y (row-major over x)
__device__ __forceinline__ int uidx(int x, int y, int R) { return x * (2 * R - x + 1) / 2 + (y - x); }

// K^{-1}_{q, ij} for the ordered pair q = (g, d) from the stored inverses of
// the classes (K_dg = K_gd^*)
__device__ __forceinline__ cd kinv_at(const double* __restrict__ inv, long long mm, int R, int g, int d, int i,
                                      int j, int nA) {
  const bool cj = g > d;
  const int u = cj ? uidx(d, g, R) : uidx(g, d, R);
  const double* base = inv + (long long)u * 2 * mm;
  const long long o = (long long)i * nA + j;
  const double re = base[o], im = base[mm + o];
  return cj ? cd{re, -im} : cd{re, im};
}

// slot of a batch past the last matrix: J = diag([[0, 1], [-1, 0]]), Pf = 1
__device__ __forceinline__ cd pad_entry(int i, int j) {
  if ((i & 1) == 0 && j == i + 1) return {1.0, 0.0};
  if ((i & 1) == 1 && j == i - 1) return {-1.0, 0.0};
  return {0.0, 0.0};
}

// grid (nb, ceil(nA^2 / 256)): K_u for the classes u0 .. u0 + nb - 1 into
// batch slot b (planar, order nA) and, when inv is set, into the class's
// inverse buffer (inverted in place afterwards)
__global__ __launch_bounds__(256) void k_ren_blocks(ObsState s, int nA, const int2* __restrict__ uxy, int u0,
                                                    int nu, double* __restrict__ dst, double* __restrict__ inv) {
  const long long mm = (long long)nA * nA;
  const int b = blockIdx.x, u = u0 + b;
  const long long e = (long long)blockIdx.y * 256 + threadIdx.x;
  if (e >= mm) return;
  const int i = (int)(e / nA), j = (int)(e % nA);
  cd v;
  if (u < nu) {
    const int2 xy = uxy[u];
    v = delta_at(s, xy.x, xy.y, i, j);
    if (inv) {
      inv[(long long)u * 2 * mm + e] = v.r;
      inv[(long long)u * 2 * mm + mm + e] = v.i;
    }
  } else {
    v = pad_entry(i, j);
  }
  dst[(long long)b * 2 * mm + e] = v.r;
  dst[(long long)b * 2 * mm + mm + e] = v.i;
}

// block-wide argmax of v (ties: the smaller index); red_v / red_i hold 256
__device__ void block_argmax(double& v, int& idx, double* red_v, int* red_i) {
  const int t = threadIdx.x;
  red_v[t] = v;
  red_i[t] = idx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      const double ov = red_v[t + h];
      const int oi = red_i[t + h];
      if (ov > red_v[t] || (ov == red_v[t] && oi < red_i[t])) { red_v[t] = ov; red_i[t] = oi; }
    }
    __syncthreads();
  }
  v = red_v[0];
  idx = red_i[0];
  __syncthreads();
}

// 1-norm (largest column sum of moduli) of the planar m x m matrix
__device__ double norm1(const double* Ar, const double* Ai, int m, double* red_v, int* red_i) {
  double mx = 0.0;
  for (int j = threadIdx.x; j < m; j += 256) {
    double sum = 0.0;
    for (int i = 0; i < m; ++i) sum += hypot(Ar[(long long)i * m + j], Ai[(long long)i * m + j]);
    mx = nan_max(mx, sum);
  }
  int dummy = 0;
  block_argmax(mx, dummy, red_v, red_i);
  return mx;
}

// grid: nu workgroups of 256 threads.  In-place Gauss-Jordan inverse with
// partial (row) pivoting of every class block K_u (planar, order m): for the
// pivot p = A_kk after the exchange of rows k and r_k,
//   A_kk = 1/p,  A_kj = A_kj / p,  A_ik = -A_ik / p,  A_ij -= A_ik A_kj / p,
// then the columns are exchanged back in reverse order.  kappa[u] = the
// 1-norm condition number, +inf for a vanishing pivot column.
// dynamic LDS: 4 m doubles (scaled row k, column k) + m ints
__global__ __launch_bounds__(256) void k_ren_inverse(double* __restrict__ Kall, int m,
                                                     double* __restrict__ kappa) {
  extern __shared__ double sh[];
  double* rr = sh;
  double* ri = sh + m;
  double* cr = sh + 2 * m;
  double* ci = sh + 3 * m;
  int* rk = (int*)(sh + 4 * m);
  __shared__ double red_v[256];
  __shared__ int red_i[256];
  const long long mm = (long long)m * m;
  double* Ar = Kall + (long long)blockIdx.x * 2 * mm;
  double* Ai = Ar + mm;
  const int tid = threadIdx.x;
  const double nK = norm1(Ar, Ai, m, red_v, red_i);
  bool sing = false;
  for (int k = 0; k < m; ++k) {
    double v = -1.0;
    int r = k;
    for (int i = k + tid; i < m; i += 256) {
      const double x = Ar[(long long)i * m + k], y = Ai[(long long)i * m + k];
      const double a = x * x + y * y;
      if (a > v) { v = a; r = i; }
    }
    block_argmax(v, r, red_v, red_i);
    if (!(v > 0.0) || !isfinite(v)) { sing = true; break; }
    if (tid == 0) rk[k] = r;
    if (r != k)
      for (int j = tid; j < m; j += 256) {
        const long long o1 = (long long)k * m + j, o2 = (long long)r * m + j;
        double t = Ar[o1]; Ar[o1] = Ar[o2]; Ar[o2] = t;
        t = Ai[o1]; Ai[o1] = Ai[o2]; Ai[o2] = t;
      }
    __syncthreads();
    const double pr = Ar[(long long)k * m + k], pim = Ai[(long long)k * m + k];
    const double p2 = pr * pr + pim * pim;
    const double ir = pr / p2, ii = -pim / p2;  // 1 / p
    for (int j = tid; j < m; j += 256) {
      cd row;
      if (j == k) row = {ir, ii};
      else row = cmul(cd{Ar[(long long)k * m + j], Ai[(long long)k * m + j]}, cd{ir, ii});
      rr[j] = row.r;
      ri[j] = row.i;
      cr[j] = j == k ? 0.0 : Ar[(long long)j * m + k];
      ci[j] = j == k ? 0.0 : Ai[(long long)j * m + k];
    }
    __syncthreads();
    for (int e = tid; e < (int)mm; e += 256) {
      const int i = e / m, j = e - i * m;
      if (i == k) {
        Ar[e] = rr[j];
        Ai[e] = ri[j];
      } else if (j == k) {
        const cd t = cmul(cd{cr[i], ci[i]}, cd{ir, ii});
        Ar[e] = -t.r;
        Ai[e] = -t.i;
      } else {
        const cd t = cmul(cd{cr[i], ci[i]}, cd{rr[j], ri[j]});
        Ar[e] -= t.r;
        Ai[e] -= t.i;
      }
    }
    __syncthreads();
  }
  if (sing) {
    if (tid == 0) kappa[blockIdx.x] = __builtin_huge_val();
    return;
  }
  for (int k = m - 1; k >= 0; --k) {
    const int r = rk[k];
    if (r != k)
      for (int i = tid; i < m; i += 256) {
        const long long o1 = (long long)i * m + k, o2 = (long long)i * m + r;
        double t = Ar[o1]; Ar[o1] = Ar[o2]; Ar[o2] = t;
        t = Ai[o1]; Ai[o1] = Ai[o2]; Ai[o2] = t;
      }
    __syncthreads();
  }
  const double nI = norm1(Ar, Ai, m, red_v, red_i);
  if (tid == 0) {
    const double kp = nK * nI;
    kappa[blockIdx.x] = isfinite(kp) ? kp : __builtin_huge_val();
  }
}

// grid (nb, ceil(ord^2 / 256)): the matrices of the terms t0 .. t0 + count - 1
// into batch slots 0 .. nb - 1 (slots past count get J).  split: ord = nA,
// Y = K_p - (K_q^{-1} - K_q^{-T}) / 2 (the inverse made exactly skew);
// block: ord = 2 nA, Z = [[K_p, i 1], [-i 1, K_q]].
__global__ __launch_bounds__(256) void k_ren_terms(ObsState s, int nA, int split, const RenTerm* __restrict__ terms,
                                                   int t0, int count, const double* __restrict__ inv,
                                                   double* __restrict__ dst) {
  const int ord = split ? nA : 2 * nA;
  const long long oo = (long long)ord * ord;
  const int b = blockIdx.x;
  const long long e = (long long)blockIdx.y * 256 + threadIdx.x;
  if (e >= oo) return;
  const int i = (int)(e / ord), j = (int)(e % ord);
  cd v;
  if (b < count) {
    const RenTerm t = terms[t0 + b];
    const int R = s.R;
    const int a = t.p / R, bb = t.p % R, g = t.q / R, d = t.q % R;
    if (split) {
      const long long mm = (long long)nA * nA;
      const cd k = delta_at(s, a, bb, i, j);
      const cd x = kinv_at(inv, mm, R, g, d, i, j, nA), y = kinv_at(inv, mm, R, g, d, j, i, nA);
      v = {k.r - 0.5 * (x.r - y.r), k.i - 0.5 * (x.i - y.i)};
    } else {
      v = {0.0, 0.0};
      if (i < nA && j < nA) v = delta_at(s, a, bb, i, j);
      else if (i >= nA && j >= nA) v = delta_at(s, g, d, i - nA, j - nA);
      else if (i < nA && j == i + nA) v = {0.0, 1.0};
      else if (i >= nA && i == j + nA) v = {0.0, -1.0};
    }
  } else {
    v = pad_entry(i, j);
  }
  dst[(long long)b * 2 * oo + e] = v.r;
  dst[(long long)b * 2 * oo + oo + e] = v.i;
}

// one thread per term of the batch: w Re T from the batch's Pfaffians (acc:
// {ln|Pf|, cos, sin} per slot) and, for the split form, Pf(K_q) from the
// classes' Pfaffians uacc (conjugated for g > d)
__global__ void k_ren_combine(ObsState s, int nA, int split, const RenTerm* __restrict__ terms, int t0, int count,
                              const double* __restrict__ acc, const double* __restrict__ uacc,
                              double* __restrict__ tval) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  const RenTerm t = terms[t0 + b];
  double la = acc[3 * b];
  cd ph{acc[3 * b + 1], acc[3 * b + 2]};
  if (split) {
    const int R = s.R, g = t.q / R, d = t.q % R;
    const int u = g > d ? uidx(d, g, R) : uidx(g, d, R);
    la += uacc[3 * u];
    const cd pk{uacc[3 * u + 1], g > d ? -uacc[3 * u + 2] : uacc[3 * u + 2]};
    ph = cmul(ph, pk);
  }
  tval[t0 + b] = term_value(s, nA, t, la, ph);
}

// one workgroup of 256: S_2 = -ln(sum of the term values), in a fixed order
__global__ __launch_bounds__(256) void k_ren_sum(const double* __restrict__ tval, int nterm,
                                                 double* __restrict__ out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int t = threadIdx.x; t < nterm; t += 256) v += tval[t];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = -log(red[0]);
}

size_t ren_lds_bytes(int nA) {
  const size_t m = 2 * (size_t)nA;
  return 2 * m * (m + 1) * sizeof(double);
}

hipError_t set_ren_lds_limit() {
  return hipFuncSetAttribute((const void*)k_ren_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ren_lds_bytes(REN_LDS_MAX_NA));
}

hipError_t launch_ren_lds(const ObsState& s, int nA, const RenTerm* terms, int nterm, double* tval, hipStream_t st) {
  if (nA < 2 || nA > REN_LDS_MAX_NA || (nA & 1) || nterm < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ren_lds, dim3(nterm), dim3(64), ren_lds_bytes(nA), st, s, nA, terms, tval);
  return hipGetLastError();
}

hipError_t launch_ren_blocks(const ObsState& s, int nA, const int2* uxy, int u0, int nb, int nu, double* dst,
                             double* inv, hipStream_t st) {
  const long long mm = (long long)nA * nA;
  hipLaunchKernelGGL(k_ren_blocks, dim3(nb, (unsigned)((mm + 255) / 256)), dim3(256), 0, st, s, nA, uxy, u0, nu,
                     dst, inv);
  return hipGetLastError();
}

hipError_t launch_ren_inverse(double* K, int nu, int m, double* kappa, hipStream_t st) {
  if (m < 2 || m > REN_MAX_NA) return hipErrorInvalidValue;
  const size_t lds = 4 * (size_t)m * sizeof(double) + (size_t)m * sizeof(int);
  hipLaunchKernelGGL(k_ren_inverse, dim3(nu), dim3(256), lds, st, K, m, kappa);
  return hipGetLastError();
}

hipError_t launch_ren_terms(const ObsState& s, int nA, int split, const RenTerm* terms, int t0, int count, int nb,
                            const double* inv, double* dst, hipStream_t st) {
  const int ord = split ? nA : 2 * nA;
  const long long oo = (long long)ord * ord;
  hipLaunchKernelGGL(k_ren_terms, dim3(nb, (unsigned)((oo + 255) / 256)), dim3(256), 0, st, s, nA, split, terms,
                     t0, count, inv, dst);
  return hipGetLastError();
}

hipError_t launch_ren_combine(const ObsState& s, int nA, int split, const RenTerm* terms, int t0, int count,
                              const double* acc, const double* uacc, double* tval, hipStream_t st) {
  hipLaunchKernelGGL(k_ren_combine, dim3((count + 63) / 64), dim3(64), 0, st, s, nA, split, terms, t0, count, acc,
                     uacc, tval);
  return hipGetLastError();
}

hipError_t launch_ren_sum(const double* tval, int nterm, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_ren_sum, dim3(1), dim3(256), 0, st, tval, nterm, out);
  return hipGetLastError();
}

}  // namespace sgs
