// Device accessors of the tables of one problem, shared by the observable
// kernels: complex helpers, Delta^{xy} entries from the pair storage, the
// amplitudes and the overlaps.
#pragma once
#include "sgs_internal.h"

namespace sgs {

struct cd {
  double r, i;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.r, -a.i}; }

// Delta^{xy}_{kl} of problem tables (x, y states; x == y gives Gamma_x).
// The pair p = (a < b) keeps W = (Gamma_a + Gamma_b)^{-1} and Im Delta^{ba};
// Delta^{ba} = -2 W + i Im, Delta^{ab} = its conjugate.
__device__ __forceinline__ cd delta_at(const ObsState& s, int x, int y, int k, int l) {
  const long long nn = (long long)s.n * s.n;
  const long long o = (long long)k * s.n + l;
  if (x == y) return {s.gam[(long long)x * nn + o], 0.0};
  const int p = s.pidx[x * s.R + y];
  const double re = -2.0 * s.W[(long long)p * nn + o];
  const double im = s.Di[(long long)p * nn + o];
  return x > y ? cd{re, im} : cd{re, -im};
}

__device__ __forceinline__ cd lam_at(const ObsState& s, int i) { return {s.lam[2 * i], s.lam[2 * i + 1]}; }
__device__ __forceinline__ cd g_at(const ObsState& s, int i, int j) {
  return {s.Gt[2 * (i * s.R + j)], s.Gt[2 * (i * s.R + j) + 1]};
}

}  // namespace sgs
