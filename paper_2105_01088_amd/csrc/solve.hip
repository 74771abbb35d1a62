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
//     root of the projected h, both by cyclic complex Jacobi on the
//     Hermitian parts of G and h.
//  3. lambda~ = G lambda; w_mu lambda_b for the chosen c_mu (Eq. Bmu);
//     force coefficients c1 = 4 w_mu lambda_b G_mb, c2 = -2 w_mu lambda_b (h_mb - E G_mb).
#include "sgs_internal.h"

namespace sgs {

struct JacobiSlots {
  double *c, *s, *er, *ei;  // rotation and phase of each pair of a round
  int *p, *q;
};

// Cyclic Jacobi (round-robin ordering) on the Hermitian m x m matrix
// A = Ar + i Ai (pitch ld) in LDS; V = Vr + i Vi receives the eigenvectors
// (columns), the diagonal of Ar the eigenvalues.  The rotation of a pair
// (p, q) with a_pq = r e^{i phi} is U = D G: D = diag(1, e^{-i phi}) makes the
// pivot real, G = [[c, s], [-s, c]] is the real symmetric rotation that
// zeroes it; A <- U^H A U, V <- V U.  Sweeps end when a whole sweep finds
// every |a_pq| <= 1e-18 (|a_pp| + |a_qq|).  64 threads.
__device__ void jacobi_herm(double* Ar, double* Ai, double* Vr, double* Vi, int m, int ld, const JacobiSlots& r,
                            int* flag) {
  const int tid = threadIdx.x;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e / m, j = e % m;
    Vr[i * ld + j] = (i == j) ? 1.0 : 0.0;
    Vi[i * ld + j] = 0.0;
  }
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
        double c = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
        if (q < m) {
          const double app = Ar[p * ld + p], aqq = Ar[q * ld + q];
          const double xr = Ar[p * ld + q], xi = Ai[p * ld + q];
          const double rr = hypot(xr, xi);
          if (rr != 0.0 && rr > 1e-18 * (fabs(app) + fabs(aqq))) {
            er = xr / rr;
            ei = xi / rr;
            const double th = (aqq - app) / (2.0 * rr);
            const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            sn = tt * c;
            *flag = 1;
          }
        }
        r.c[t] = c; r.s[t] = sn; r.er[t] = er; r.ei[t] = ei; r.p[t] = p; r.q[t] = q;
      }
      __syncthreads();
      // rows: a_p <- c a_p - s e^{i phi} a_q,  a_q <- s a_p + c e^{i phi} a_q
      for (int e = tid; e < half * m; e += blockDim.x) {
        const int t = e / m, j = e % m;
        const double sn = r.s[t];
        if (sn == 0.0) continue;
        const double c = r.c[t], er = r.er[t], ei = r.ei[t];
        const int p = r.p[t], q = r.q[t];
        const double apr = Ar[p * ld + j], api = Ai[p * ld + j];
        const double aqr = Ar[q * ld + j], aqi = Ai[q * ld + j];
        const double br = er * aqr - ei * aqi, bi = er * aqi + ei * aqr;
        Ar[p * ld + j] = c * apr - sn * br;
        Ai[p * ld + j] = c * api - sn * bi;
        Ar[q * ld + j] = sn * apr + c * br;
        Ai[q * ld + j] = sn * api + c * bi;
      }
      __syncthreads();
      // columns of A and V: x_p <- c x_p - s e^{-i phi} x_q,  x_q <- s x_p + c e^{-i phi} x_q
      for (int e = tid; e < half * m; e += blockDim.x) {
        const int t = e / m, i = e % m;
        const double sn = r.s[t];
        if (sn == 0.0) continue;
        const double c = r.c[t], er = r.er[t], ei = r.ei[t];
        const int p = r.p[t], q = r.q[t];
        {
          const double apr = Ar[i * ld + p], api = Ai[i * ld + p];
          const double aqr = Ar[i * ld + q], aqi = Ai[i * ld + q];
          const double br = er * aqr + ei * aqi, bi = er * aqi - ei * aqr;
          Ar[i * ld + p] = c * apr - sn * br;
          Ai[i * ld + p] = c * api - sn * bi;
          Ar[i * ld + q] = sn * apr + c * br;
          Ai[i * ld + q] = sn * api + c * bi;
        }
        {
          const double vpr = Vr[i * ld + p], vpi = Vi[i * ld + p];
          const double vqr = Vr[i * ld + q], vqi = Vi[i * ld + q];
          const double br = er * vqr + ei * vqi, bi = er * vqi - ei * vqr;
          Vr[i * ld + p] = c * vpr - sn * br;
          Vi[i * ld + p] = c * vpi - sn * bi;
          Vr[i * ld + q] = sn * vpr + c * br;
          Vi[i * ld + q] = sn * vpi + c * bi;
        }
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (!f) break;
  }
}

// dynamic LDS: see solve_lds_bytes
__global__ __launch_bounds__(64) void k_solve(SolveArgs a) {
  extern __shared__ double smem[];
  const int R = a.R, ld = R + 1;  // odd pitch: column walks spread over the banks
  const int RL = R * ld;
  double* Ar = smem;           // working Hermitian matrix
  double* Ai = Ar + RL;
  double* Vr = Ai + RL;        // eigenvectors of G, then X
  double* Vi = Vr + RL;
  double* Cr = Vi + RL;        // He X, then the eigenvectors of h'
  double* Ci = Cr + RL;
  double* Gr = Ci + RL;        // R*R (pitch R)
  double* Gi = Gr + R * R;
  double* Hr = Gi + R * R;
  double* Hi = Hr + R * R;
  double* sv = Hi + R * R;     // R eigenvalues of G
  double* lr = sv + R;         // R
  double* li = lr + R;
  double* ltr = li + R;
  double* lti = ltr + R;
  JacobiSlots js;
  js.c = lti + R;              // R/2 + 1 rotation slots each
  js.s = js.c + R + 1;
  js.er = js.s + R + 1;
  js.ei = js.er + R + 1;
  js.p = (int*)(js.ei + R + 1);
  js.q = js.p + R + 1;
  int* keep = js.q + R + 1;    // R
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

  // 2a. Jacobi on the Hermitian part of G
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e / R, j = e % R;
    Ar[i * ld + j] = 0.5 * (Gr[i * R + j] + Gr[j * R + i]);
    Ai[i * ld + j] = 0.5 * (Gi[i * R + j] - Gi[j * R + i]);
  }
  __syncthreads();
  jacobi_herm(Ar, Ai, Vr, Vi, R, ld, js, &flag);
  for (int k = tid; k < R; k += blockDim.x) sv[k] = Ar[k * ld + k];
  __syncthreads();
  if (tid == 0) {
    double smax = 0.0;
    for (int k = 0; k < R; ++k) smax = nan_max(smax, sv[k]);
    int cnt = 0;
    if (!(smax > 0.0) || !isfinite(smax)) atomicCAS(a.status, ST_OK, ST_SINGULAR);
    for (int k = 0; k < R; ++k)
      if (sv[k] > a.g_thr * smax) keep[cnt++] = k;
    K = cnt;
  }
  __syncthreads();
  const int Kk = K;
  // X = V[:, keep] diag(s^{-1/2}), compacted in place (row by row)
  for (int i = tid; i < R; i += blockDim.x)
    for (int c = 0; c < Kk; ++c) {
      const double f = 1.0 / sqrt(sv[keep[c]]);
      Vr[i * ld + c] = Vr[i * ld + keep[c]] * f;
      Vi[i * ld + c] = Vi[i * ld + keep[c]] * f;
    }
  __syncthreads();
  // 2b. h' = X^H He X with He the Hermitian part of h
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e / R, j = e % R;
    Ar[i * ld + j] = 0.5 * (Hr[i * R + j] + Hr[j * R + i]);
    Ai[i * ld + j] = 0.5 * (Hi[i * R + j] - Hi[j * R + i]);
  }
  __syncthreads();
  for (int e = tid; e < R * Kk; e += blockDim.x) {  // C = He X  (R x K)
    const int i = e / Kk, c = e % Kk;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < R; ++k) {
      const double ar = Ar[i * ld + k], ai = Ai[i * ld + k], xr = Vr[k * ld + c], xi = Vi[k * ld + c];
      sr += ar * xr - ai * xi;
      si += ar * xi + ai * xr;
    }
    Cr[i * ld + c] = sr;
    Ci[i * ld + c] = si;
  }
  __syncthreads();
  for (int e = tid; e < Kk * Kk; e += blockDim.x) {  // A = X^H C (K x K)
    const int rr = e / Kk, c = e % Kk;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < R; ++k) {
      const double xr = Vr[k * ld + rr], xi = -Vi[k * ld + rr], yr = Cr[k * ld + c], yi = Ci[k * ld + c];
      sr += xr * yr - xi * yi;
      si += xr * yi + xi * yr;
    }
    Ar[rr * ld + c] = sr;
    Ai[rr * ld + c] = si;
  }
  __syncthreads();
  for (int e = tid; e < Kk * Kk; e += blockDim.x) {  // exactly Hermitian
    const int rr = e / Kk, c = e % Kk;
    if (rr < c) {
      const double sr = 0.5 * (Ar[rr * ld + c] + Ar[c * ld + rr]);
      const double si = 0.5 * (Ai[rr * ld + c] - Ai[c * ld + rr]);
      Ar[rr * ld + c] = sr; Ai[rr * ld + c] = si;
      Ar[c * ld + rr] = sr; Ai[c * ld + rr] = -si;
    } else if (rr == c) {
      Ai[rr * ld + c] = 0.0;
    }
  }
  __syncthreads();
  jacobi_herm(Ar, Ai, Cr, Ci, Kk, ld, js, &flag);
  if (tid == 0) {
    int k0 = 0;
    for (int k = 1; k < Kk; ++k)
      if (Ar[k * ld + k] < Ar[k0 * ld + k0]) k0 = k;
    Es = Ar[k0 * ld + k0];
    flag = k0;
  }
  __syncthreads();
  const int k0 = flag;
  const double E = Es;
  // lambda = X z
  for (int i = tid; i < R; i += blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < Kk; ++c) {
      const double xr = Vr[i * ld + c], xi = Vi[i * ld + c], zr = Cr[c * ld + k0], zi = Ci[c * ld + k0];
      sr += xr * zr - xi * zi;
      si += xr * zi + xi * zr;
    }
    lr[i] = sr;
    li[i] = si;
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
  for (int j = 0; j < R; ++j) lmax = nan_max(lmax, sqrt(lr[j] * lr[j] + li[j] * li[j]));
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int mu = e / R, b = e % R;
    double rr, ri;  // w_mu lambda_b
    const double lm2 = lr[mu] * lr[mu] + li[mu] * li[mu];
    if (a.weight == 0) {
      // c_mu = 1 / (lambda_mu lambda~_mu^*):  w_mu lambda_b = lambda_b / lambda_mu
      // (exactly 1 for b = mu).  The printed weight diverges as lambda_mu -> 0
      // (Sec. III.A); a state at the float64 floor (|lambda_mu| <= 1e-13
      // max|lambda|, where the ratio carries no information) is left unchanged.
      if (!(sqrt(lm2) > 1e-13 * lmax)) { rr = 0.0; ri = 0.0; }
      else if (b == mu) { rr = 1.0; ri = 0.0; }
      else {
        rr = (lr[b] * lr[mu] + li[b] * li[mu]) / lm2;
        ri = (li[b] * lr[mu] - lr[b] * li[mu]) / lm2;
      }
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
    if (a.energy_slot) a.energy_slot[a.slot_ctr ? (long long)*a.slot_ctr * a.slot_stride : 0] = E;
  }
}

size_t solve_lds_bytes(int R) {
  const size_t RL = (size_t)R * (R + 1);
  return sizeof(double) * (6 * RL + 4 * (size_t)R * R + 5 * (size_t)R + 4 * (size_t)(R + 1)) +
         sizeof(int) * (2 * (size_t)(R + 1) + R) + 64;
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_solve, dim3(1), dim3(64), solve_lds_bytes(a.R), s, a);
  return hipGetLastError();
}

__global__ void k_set_counter(int* ctr, int v) { *ctr = v; }
__global__ void k_bump_counter(int* ctr) { *ctr += 1; }

hipError_t launch_set_counter(int* ctr, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, s, ctr, v);
  return hipGetLastError();
}

hipError_t launch_bump_counter(int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_bump_counter, dim3(1), dim3(1), 0, s, ctr);
  return hipGetLastError();
}

hipError_t set_solve_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_solve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace sgs
