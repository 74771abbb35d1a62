// The R x R problem of Sec. II.C and the per-state weights of Sec. III.A,
// on one workgroup (a single wave) per problem, in float64.
//
//  1. Tables: G_ab = exp(ln|G_ab|) e^{i arg G_ab} with
//       ln|G_ab| = -(N/2) ln 2 + (1/4) ln|det(Gamma_a + Gamma_b)|   (|<a|b>|^2 = 2^{-N} |Pf|)
//       arg G_0a = 0 (reference gauge), arg G_ab = arg(i^{3N} Pf(C_ab)) for a, b >= 1
//       (the Schur-reduced triple product; Pf(i Gamma_0) = i^N and
//        Pf(Gamma_a + Gamma_0) > 0 for states of equal parity), h_ab = G_ab eps_ab.
//  2. h lambda = E G lambda (Eq. eigLambda): canonical orthogonalization
//     (eigenvectors of G below g_rel_threshold * max dropped) and the lowest
//     root of the projected h, both by cyclic Jacobi on the real 2R x 2R
//     embedding [[Re, -Im], [Im, Re]] of the Hermitian matrices.
//  3. lambda~ = G lambda; w_mu lambda_b for the chosen c_mu (Eq. Bmu);
//     force coefficients c1 = 4 w_mu lambda_b G_mb, c2 = -2 w_mu lambda_b (h_mb - E G_mb).
#include "sgs_internal.h"

namespace sgs {


// Cyclic Jacobi (round-robin ordering) on the symmetric m x m matrix A
// (pitch ld) in LDS; V receives the eigenvectors (columns).  64 threads.
__device__ void jacobi(double* A, double* V, int m, int ld, double* rc, double* rs, int* rp,
                       int* rq, int* flag) {
  const int tid = threadIdx.x;
  for (int e = tid; e < m * m; e += blockDim.x) V[(e / m) * ld + e % m] = (e / m == e % m) ? 1.0 : 0.0;
  __syncthreads();
  if (m < 2) return;
  const int mm = m + (m & 1);  // round-robin needs an even count: pad with a dummy index
  const int half = mm / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < mm - 1; ++round) {
      for (int t = tid; t < half; t += blockDim.x) {
        int x, y;
        if (t == 0) { x = mm - 1; y = round; }
        else { x = (round + t) % (mm - 1); y = (round - t + (mm - 1)) % (mm - 1); }
        const int p = x < y ? x : y, q = x < y ? y : x;
        double c = 1.0, s = 0.0;
        const bool real_pair = q < m;
        const double app = real_pair ? A[p * ld + p] : 0.0, aqq = real_pair ? A[q * ld + q] : 0.0;
        const double apq = real_pair ? A[p * ld + q] : 0.0;
        if (real_pair && apq != 0.0 && fabs(apq) > 1e-18 * (fabs(app) + fabs(aqq))) {
          const double th = (aqq - app) / (2.0 * apq);
          const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(tt * tt + 1.0);
          s = tt * c;
          *flag = 1;
        }
        rc[t] = c; rs[t] = s; rp[t] = p; rq[t] = q;
      }
      __syncthreads();
      // rows: A <- P^T A
      for (int e = tid; e < half * m; e += blockDim.x) {
        const int t = e / m, j = e % m;
        const double c = rc[t], s = rs[t];
        if (s == 0.0) continue;
        const int p = rp[t], q = rq[t];
        const double ap = A[p * ld + j], aq = A[q * ld + j];
        A[p * ld + j] = c * ap - s * aq;
        A[q * ld + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A P, V <- V P
      for (int e = tid; e < half * m; e += blockDim.x) {
        const int t = e / m, i = e % m;
        const double c = rc[t], s = rs[t];
        if (s == 0.0) continue;
        const int p = rp[t], q = rq[t];
        const double ap = A[i * ld + p], aq = A[i * ld + q];
        A[i * ld + p] = c * ap - s * aq;
        A[i * ld + q] = s * ap + c * aq;
        const double vp = V[i * ld + p], vq = V[i * ld + q];
        V[i * ld + p] = c * vp - s * vq;
        V[i * ld + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (!f) break;
  }
}

// dynamic LDS: 3 m*m + 12 R + 4 m doubles-ish (see solve_lds_bytes)
__global__ __launch_bounds__(64) void k_solve(SolveArgs a) {
  extern __shared__ double smem[];
  const int R = a.R, m = 2 * R, ld = m;
  double* A = smem;
  double* V = A + m * m;
  double* C = V + m * m;
  double* Gr = C + m * m;      // R*R
  double* Gi = Gr + R * R;
  double* Hr = Gi + R * R;
  double* Hi = Hr + R * R;
  double* sv = Hi + R * R;     // m eigenvalues of G
  double* lr = sv + m;         // R
  double* li = lr + R;
  double* ltr = li + R;
  double* lti = ltr + R;
  double* rc = lti + R;        // m/2 + 1 rotation slots
  double* rs = rc + R + 1;
  int* rp = (int*)(rs + R + 1);
  int* rq = rp + R + 1;
  int* keep = rq + R + 1;      // m
  __shared__ int flag, K;
  __shared__ double Es;
  const int tid = threadIdx.x;
  const double PI = 3.14159265358979323846;

  // 1. tables
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e / R, j = e % R;
    double la = 0.0, ar = 0.0, er, ei;
    if (i == j) {
      er = a.eps[2 * (a.P + i)];
      ei = 0.0;
    } else {
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      const int p = a.pidx[lo * R + hi];
      la = -0.5 * a.N * log(2.0) + 0.25 * a.logdet[p];
      double th = 0.0;
      if (lo > 0) {
        const int q = a.qidx[lo * R + hi];
        th = fmod(1.5 * PI * (double)(a.N % 4) + atan2(a.pfacc[3 * q + 2], a.pfacc[3 * q + 1]), 2.0 * PI);
        if (th > PI) th -= 2.0 * PI;
        if (th <= -PI) th += 2.0 * PI;
      }
      ar = (i < j) ? th : -th;
      er = a.eps[2 * p];
      ei = (i < j) ? a.eps[2 * p + 1] : -a.eps[2 * p + 1];
    }
    const double mag = exp(la);
    const double gr = (i == j) ? 1.0 : mag * cos(ar), gi = (i == j) ? 0.0 : mag * sin(ar);
    Gr[e] = gr; Gi[e] = gi;
    Hr[e] = gr * er - gi * ei;
    Hi[e] = gr * ei + gi * er;
    if (a.tab_la) a.tab_la[e] = la;
    if (a.tab_arg) a.tab_arg[e] = ar;
    if (a.tab_eps) { a.tab_eps[2 * e] = er; a.tab_eps[2 * e + 1] = ei; }
    a.Gt[2 * e] = gr; a.Gt[2 * e + 1] = gi;
    a.ht[2 * e] = Hr[e]; a.ht[2 * e + 1] = Hi[e];
  }
  __syncthreads();

  // 2a. Jacobi on the embedding of G (Hermitian parts)
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e / m, j = e % m;
    const int ii = i % R, jj = j % R;
    const double re = 0.5 * (Gr[ii * R + jj] + Gr[jj * R + ii]);
    const double im = 0.5 * (Gi[ii * R + jj] - Gi[jj * R + ii]);
    double v;
    if ((i < R) == (j < R)) v = re;
    else if (i < R) v = -im;   // top-right block: -Im
    else v = im;               // bottom-left: +Im
    A[i * ld + j] = v;
  }
  __syncthreads();
  jacobi(A, V, m, ld, rc, rs, rp, rq, &flag);
  for (int k = tid; k < m; k += blockDim.x) sv[k] = A[k * ld + k];
  __syncthreads();
  if (tid == 0) {
    double smax = 0.0;
    for (int k = 0; k < m; ++k) smax = fmax(smax, sv[k]);
    int cnt = 0;
    if (!(smax > 0.0) || !isfinite(smax)) atomicCAS(a.status, ST_OK, ST_SINGULAR);
    for (int k = 0; k < m; ++k)
      if (sv[k] > a.g_thr * smax) keep[cnt++] = k;
    K = cnt;
  }
  __syncthreads();
  const int Kk = K;
  // X = V[:, keep] diag(s^{-1/2}), compacted in place (row by row)
  for (int i = tid; i < m; i += blockDim.x)
    for (int c = 0; c < Kk; ++c) V[i * ld + c] = V[i * ld + keep[c]] / sqrt(sv[keep[c]]);
  __syncthreads();
  // 2b. h' = X^T He X
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e / m, j = e % m;
    const int ii = i % R, jj = j % R;
    const double re = 0.5 * (Hr[ii * R + jj] + Hr[jj * R + ii]);
    const double im = 0.5 * (Hi[ii * R + jj] - Hi[jj * R + ii]);
    double v;
    if ((i < R) == (j < R)) v = re;
    else if (i < R) v = -im;
    else v = im;
    A[i * ld + j] = v;
  }
  __syncthreads();
  for (int e = tid; e < m * Kk; e += blockDim.x) {  // C = He X  (m x K)
    const int i = e / Kk, c = e % Kk;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += A[i * ld + k] * V[k * ld + c];
    C[i * ld + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < Kk * Kk; e += blockDim.x) {  // A = X^T C (K x K)
    const int r = e / Kk, c = e % Kk;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += V[k * ld + r] * C[k * ld + c];
    A[r * ld + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < Kk * Kk; e += blockDim.x) {  // exact symmetry
    const int r = e / Kk, c = e % Kk;
    if (r < c) {
      const double s = 0.5 * (A[r * ld + c] + A[c * ld + r]);
      A[r * ld + c] = s;
      A[c * ld + r] = s;
    }
  }
  __syncthreads();
  jacobi(A, C, Kk, ld, rc, rs, rp, rq, &flag);
  if (tid == 0) {
    int k0 = 0;
    for (int k = 1; k < Kk; ++k)
      if (A[k * ld + k] < A[k0 * ld + k0]) k0 = k;
    Es = A[k0 * ld + k0];
    flag = k0;
  }
  __syncthreads();
  const int k0 = flag;
  const double E = Es;
  // lambda_e = X z
  for (int i = tid; i < m; i += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < Kk; ++c) s += V[i * ld + c] * C[c * ld + k0];
    if (i < R) lr[i] = s; else li[i - R] = s;
  }
  __syncthreads();
  // 3. lambda~ = G lambda, weights, coefficients
  for (int i = tid; i < R; i += blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < R; ++j) {
      sr += Gr[i * R + j] * lr[j] - Gi[i * R + j] * li[j];
      si += Gr[i * R + j] * li[j] + Gi[i * R + j] * lr[j];
    }
    ltr[i] = sr; lti[i] = si;
    a.lam[2 * i] = lr[i]; a.lam[2 * i + 1] = li[i];
    a.lamt[2 * i] = sr; a.lamt[2 * i + 1] = si;
  }
  __syncthreads();
  double lmax = 0.0;
  for (int j = 0; j < R; ++j) lmax = fmax(lmax, sqrt(lr[j] * lr[j] + li[j] * li[j]));
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int mu = e / R, b = e % R;
    double rr, ri;  // w_mu lambda_b
    const double lm2 = lr[mu] * lr[mu] + li[mu] * li[mu];
    if (a.weight == 0) {
      // c_mu = 1 / (lambda_mu lambda~_mu^*):  w_mu lambda_b = lambda_b / lambda_mu
      if (b == mu) { rr = 1.0; ri = 0.0; }
      else if (sqrt(lm2) > 1e-13 * lmax) {
        rr = (lr[b] * lr[mu] + li[b] * li[mu]) / lm2;
        ri = (li[b] * lr[mu] - lr[b] * li[mu]) / lm2;
      } else { rr = 0.0; ri = 0.0; }
    } else {
      // c_mu = lambda~_mu lambda_mu^* / |lambda~_mu lambda_mu|:
      // w_mu lambda_b = |lambda~_mu| (lambda_mu^* / |lambda_mu|) lambda_b
      const double lt = sqrt(ltr[mu] * ltr[mu] + lti[mu] * lti[mu]);
      double pr = 1.0, pi = 0.0;
      if (lm2 > 0.0) { const double l = sqrt(lm2); pr = lr[mu] / l; pi = -li[mu] / l; }
      rr = lt * (pr * lr[b] - pi * li[b]);
      ri = lt * (pr * li[b] + pi * lr[b]);
    }
    const double gr = Gr[mu * R + b], gi = Gi[mu * R + b];
    const double hr = Hr[mu * R + b] - E * gr, hi = Hi[mu * R + b] - E * gi;
    a.coef[2 * e] = 4.0 * (rr * gr - ri * gi);
    a.coef[2 * e + 1] = 4.0 * (rr * gi + ri * gr);
    a.coef[2 * R * R + 2 * e] = -2.0 * (rr * hr - ri * hi);
    a.coef[2 * R * R + 2 * e + 1] = -2.0 * (rr * hi + ri * hr);
  }
  if (tid == 0) {
    a.E[0] = E;
    if (a.energy_slot) a.energy_slot[0] = E;
  }
}

size_t solve_lds_bytes(int R) {
  const int m = 2 * R;
  return sizeof(double) * (3 * (size_t)m * m + 4 * (size_t)R * R + m + 4 * R + 2 * (R + 1)) +
         sizeof(int) * (2 * (R + 1) + m) + 64;
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_solve, dim3(1), dim3(64), solve_lds_bytes(a.R), s, a);
  return hipGetLastError();
}

hipError_t set_solve_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_solve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace sgs
