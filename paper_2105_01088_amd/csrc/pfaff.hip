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
// Blocked with delayed updates, on two levels: inside a super-panel of up to
// 32 steps the current trailing matrix is A + U V^T - V U^T (U = b1, V = b0 / a
// per step); only the two columns a step needs are formed, each as a gathered
// row of A plus the sum over the earlier steps.  Panels of up to NBH steps
// keep their own U, V in registers and take the super-panel's earlier steps
// from a small global buffer; after the super-panel the trailing matrix takes
// A += [U V] [V -U]^T as one complex GEMM of depth up to 64 (the matrix is read
// and written once per super-panel instead of once per register panel).
#include "sgs_internal.h"
#include "wave_ops.h"

namespace sgs {

constexpr int PF_MAX_WAVES = 8;

// Deferred columns of one super-panel: for every earlier step t < kd of the
// super-panel, U_t and V_t of every stored row, kept twice per matrix:
//  * row-major, entry [(row * PF_DEFER + t) * 4 + {U re, U im, V re, V im}]:
//    a gathered row's entries are contiguous (uniform loads);
//  * step-major (after 4 m0 PF_DEFER doubles), complex U_t[row] at pair
//    t m0 + row and V_t[row] at pair (PF_DEFER + t) m0 + row: the lanes' own
//    rows at one step are consecutive, so a load instruction reads one
//    contiguous segment instead of a cache line per lane.
// The current matrix of the super-panel is
//   B[i][j] = A[i][j] + sum_t (U_t[i] V_t[j] - V_t[i] U_t[j])
// over those steps and the panel's own (held in registers); a gather of row g
// at the lanes' rows adds sum_{t < kd} (U_t[l] V_t[g] - V_t[l] U_t[g]).
constexpr int PF_DEFER = 32;   // deferred steps per super-panel, at most
typedef double dpair __attribute__((ext_vector_type(2)));

// One panel of at most NBH elimination steps of a super-panel, for every
// matrix of the batch (one workgroup each).  A is the stored (compact)
// m0 x m0 matrix the super-panel started from (planar, leading dimension ld,
// imaginary plane at +plane); the panel takes the steps at logical positions
// p0, p0 + 2, ..., p0 + 2 (ns - 1).  Logical row l >= p0 is owned by thread
// (l - p0) % nt (slot (l - p0) / nt < RPT), which keeps in registers its U
// and V entries of this panel, its current column value c0 and its stored
// index pl (logical row l is stored row perm[l]; the stored matrix is never
// written during a super-panel).  Step s (p = p0 + 2 s):
//   c0_l = B[l][p]                                         (l > p)
// the pivot row q maximizes |c0_q| (wave maxima of a packed key, posted per
// wave with the candidate's record: U, V, c0, pl); after one barrier every
// thread takes the best post.  Rows p+1 and q exchange (a sign flip of the
// Pfaffian): the owner of row q takes the record that row p+1 posted; row
// p+1 is eliminated and needs no registers.  With a = -c0_q:
//   c1_l = B[l][q],  U_l[s] = -c1_l,  V_l[s] = -c0_l / a          (l > p + 1)
// The gather of row pl_q for c1 and the gather of the next step's pivot row
// are issued together (with their deferred sums), and the owner of row p + 2
// posts its U and V for the next step before the second barrier: two barriers
// and one global latency per step.
// At the end the panel appends its steps to the deferred columns and saves
// perm; the super-panel's last panel instead writes, for the trailing logical
// rows l >= pe = p0 + 2 ns, the GEMM operands L = [U | V] and Rm = [V | -U]
// of all kall steps of the super-panel, stored transposed (2 kall x mp, mp =
// m0 - pe, row l - pe in column l - pe), and perm[l] = pl_l; the trailing
// GEMM reads the old matrix through perm + pe and writes the next, compact
// trailing matrix into the other buffer.
//   acc : per matrix {ln|Pf|, cos arg, sin arg}; first_acc: start from Pf = 1
//   first: the super-panel's first panel (perm starts as the identity)
// dynamic LDS: m0 ints
template <int NBH, int RPT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_pf_panel(const double* __restrict__ Aall, long long astride, long long plane, int ld, int m0, int p0,
                int ns, int kd, int kall, int first, int last, const double* __restrict__ Dall,
                double* __restrict__ Dwall, long long dstride, double* __restrict__ Lall,
                double* __restrict__ RMall, long long lstride, long long l_im, int* __restrict__ permall,
                int pstride, double* __restrict__ acc, int first_acc, int* __restrict__ status) {
  constexpr int RB = 4 * NBH + 4;  // record: U re, U im, V re, V im (NBH each), c0 re, c0 im, pl (+ pad)
  __shared__ __attribute__((aligned(16))) double slot[2][PF_MAX_WAVES][RB];
  __shared__ unsigned long long skey[2][PF_MAX_WAVES];
  __shared__ __attribute__((aligned(16))) double p1rec[2][RB];
  __shared__ __attribute__((aligned(16))) double bc[4 * NBH];  // U re, U im, V re, V im of row p
  extern __shared__ int perm[];   // logical -> stored index (entries >= p0)
  const int mat = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const int m = m0;
  const double* __restrict__ Ar = Aall + (long long)mat * astride;
  const double* __restrict__ Ai = Ar + plane;
  int* __restrict__ gperm = permall + (long long)mat * pstride;
  // deferred columns: read through Db (entries t < kd), written through Dw
  // (entries kd .. kd + ns - 1 of the trailing rows) at the end
  const dpair* __restrict__ Db = (const dpair*)(Dall + (long long)mat * dstride);
  dpair* __restrict__ Dw = (dpair*)(Dwall + (long long)mat * dstride);
  constexpr int RS = 2 * PF_DEFER;  // row stride in pairs
  const long long tm = 2LL * m0 * PF_DEFER;  // the step-major copy, in pairs
  const dpair* __restrict__ Tu = Db + tm;
  const dpair* __restrict__ Tv = Tu + (long long)PF_DEFER * m0;
  dpair* __restrict__ Twu = Dw + tm;
  dpair* __restrict__ Twv = Twu + (long long)PF_DEFER * m0;

  for (int l = p0 + tid; l < m; l += nt) perm[l] = first ? l : gperm[l];
  for (int e = tid; e < 4 * NBH; e += nt) bc[e] = 0.0;  // row p0's U, V before the first step
  __syncthreads();

  double ur[RPT][NBH], ui[RPT][NBH], vr[RPT][NBH], vi[RPT][NBH];
  double c0r[RPT], c0i[RPT], prr[RPT], pri[RPT];
  int pl[RPT];
  // sum over the deferred steps of (U_t[l] V_t[g] - V_t[l] U_t[g]) for the
  // lanes' rows l against rows g1 and g2 (complex, accumulated into d*).
  // The rows g are uniform: their entries come through the scalar cache.
  auto deferred = [&](int g1, int g2, double (&d1r)[RPT], double (&d1i)[RPT], double (&d2r)[RPT],
                      double (&d2i)[RPT]) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) { d1r[r] = 0.0; d1i[r] = 0.0; d2r[r] = 0.0; d2i[r] = 0.0; }
    const dpair* __restrict__ B1 = Db + (long long)__builtin_amdgcn_readfirstlane(g1) * RS;
    const dpair* __restrict__ B2 = Db + (long long)__builtin_amdgcn_readfirstlane(g2) * RS;
#pragma unroll 4
    for (int t = 0; t < kd; ++t) {
      const dpair u1 = B1[2 * t], v1 = B1[2 * t + 1];
      const dpair u2 = B2[2 * t], v2 = B2[2 * t + 1];
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const long long o = (long long)t * m0 + pl[r];
        const dpair ou = Tu[o], ov = Tv[o];
        d1r[r] = fma(ou.x, v1.x, d1r[r]); d1r[r] = fma(-ou.y, v1.y, d1r[r]);
        d1r[r] = fma(-ov.x, u1.x, d1r[r]); d1r[r] = fma(ov.y, u1.y, d1r[r]);
        d1i[r] = fma(ou.x, v1.y, d1i[r]); d1i[r] = fma(ou.y, v1.x, d1i[r]);
        d1i[r] = fma(-ov.x, u1.y, d1i[r]); d1i[r] = fma(-ov.y, u1.x, d1i[r]);
        d2r[r] = fma(ou.x, v2.x, d2r[r]); d2r[r] = fma(-ou.y, v2.y, d2r[r]);
        d2r[r] = fma(-ov.x, u2.x, d2r[r]); d2r[r] = fma(ov.y, u2.y, d2r[r]);
        d2i[r] = fma(ou.x, v2.y, d2i[r]); d2i[r] = fma(ou.y, v2.x, d2i[r]);
        d2i[r] = fma(-ov.x, u2.y, d2i[r]); d2i[r] = fma(-ov.y, u2.x, d2i[r]);
      }
    }
  };
  {
    const int g0 = perm[p0];  // the first pivot row
    double d1r[RPT], d1i[RPT], d2r[RPT], d2i[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = p0 + tid + r * nt;
      pl[r] = l < m ? perm[l] : 0;  // a valid row index for every slot
    }
    deferred(g0, g0, d1r, d1i, d2r, d2i);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = p0 + tid + r * nt;
      c0r[r] = 0.0;
      c0i[r] = 0.0;
#pragma unroll
      for (int t = 0; t < NBH; ++t) { ur[r][t] = 0.0; ui[r][t] = 0.0; vr[r][t] = 0.0; vi[r][t] = 0.0; }
      const bool act = l > p0 && l < m;
      const long long o = (long long)g0 * ld + pl[r];
      prr[r] = act ? -Ar[o] + d1r[r] : 0.0;
      pri[r] = act ? -Ai[o] + d1i[r] : 0.0;
    }
  }
  double la = 0.0, phr = 1.0, phi = 0.0;  // uniform
  if (!first_acc) { la = acc[mat * 3]; phr = acc[mat * 3 + 1]; phi = acc[mat * 3 + 2]; }
  bool sing = false;

  // The step loop stays rolled (unrolled it is tens of KB of code fetched once
  // per panel: instruction-cache bound).  U and V entries are kept by age:
  // after s steps entries 0 .. s-1 sit at positions NBH-s .. NBH-1 and the
  // positions before them are zero, so every sum runs over all NBH positions
  // with constant register indices; each step shifts them left by one and
  // appends the new entry.  Posted records carry the same layout.
#pragma unroll 1
  for (int s = 0; s < ns; ++s) {
    const int p = p0 + 2 * s, par = s & 1;
    // current column p and the pivot search keys
    unsigned long long mine[RPT];
    unsigned long long key = 0;
    // row p's U, V are read by every lane from the same LDS addresses
    // (broadcast reads; the VALU only multiplies)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = p0 + tid + r * nt;
      const bool act = l > p && l < m;
      double xr = prr[r], xi = pri[r], yr = 0.0, yi = 0.0;
#pragma unroll
      for (int t = 0; t < NBH; ++t) {
        const double upr = bc[t], upi = bc[NBH + t];
        const double vpr = bc[2 * NBH + t], vpi = bc[3 * NBH + t];
        // (U_l V_p - V_l U_p)_t, four fused multiply-adds per component;
        // even and odd t in separate accumulators (two dependency chains)
        double& sr = (t & 1) ? yr : xr;
        double& si = (t & 1) ? yi : xi;
        sr = fma(ur[r][t], vpr, sr);
        sr = fma(-ui[r][t], vpi, sr);
        sr = fma(-vr[r][t], upr, sr);
        sr = fma(vi[r][t], upi, sr);
        si = fma(ur[r][t], vpi, si);
        si = fma(ui[r][t], vpr, si);
        si = fma(-vr[r][t], upi, si);
        si = fma(-vi[r][t], upr, si);
      }
      xr += yr;
      xi += yi;
      c0r[r] = act ? xr : c0r[r];
      c0i[r] = act ? xi : c0i[r];
      mine[r] = act ? pivot_key(xr * xr + xi * xi, l) : 0ull;
      key = umax64(key, mine[r]);
    }
    const int pp1 = perm[p + 1];
    const int pp2 = (p + 2 < m) ? perm[p + 2] : 0;
    key = wave_max_u64(key);
    if (lane == 0) skey[par][w] = key;
    // post the wave's candidate record, and row p + 1's record (for the exchange)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
      for (int k2 = 0; k2 < 2; ++k2) {
        const bool post = k2 == 0 ? (key != 0ull && mine[r] == key) : (p0 + tid + r * nt == p + 1);
        if (post) {
          double* rec = k2 == 0 ? slot[par][w] : p1rec[par];
#pragma unroll
          for (int t = 0; t < NBH; ++t) {
            rec[t] = ur[r][t]; rec[NBH + t] = ui[r][t]; rec[2 * NBH + t] = vr[r][t]; rec[3 * NBH + t] = vi[r][t];
          }
          rec[4 * NBH] = c0r[r];
          rec[4 * NBH + 1] = c0i[r];
          rec[4 * NBH + 2] = (double)pl[r];
        }
      }
    }
    __syncthreads();
    // best post: pivot row q
    unsigned long long kq[PF_MAX_WAVES];
#pragma unroll
    for (int x = 0; x < PF_MAX_WAVES; ++x) kq[x] = x < nw ? skey[par][x] : 0ull;
    unsigned long long best = kq[0];
    int ww = 0;
#pragma unroll
    for (int x = 1; x < PF_MAX_WAVES; ++x)
      if (kq[x] > best) { best = kq[x]; ww = x; }
    int q = 0xffff - (int)(best & 0xffffull);
    const bool bad = best == 0ull || q <= p || q >= m;
    if (bad) q = p + 1;  // no usable pivot (flagged below): keep the order
    const double* __restrict__ rq = bad ? p1rec[par] : slot[par][ww];
    const bool flip = q != p + 1;
    const double ar = -rq[4 * NBH], ai = -rq[4 * NBH + 1];  // a = B[p][p+1] = -c0 of the new row p + 1
    const int plq = min(max((int)rq[4 * NBH + 2], 0), m - 1);
    const double a2 = ar * ar + ai * ai;
    if (bad || !(a2 > 0.0) || !isfinite(a2)) sing = true;
    la += 0.5 * log(a2);
    {
      double nr = phr * ar - phi * ai, ni = phr * ai + phi * ar;
      if (flip) { nr = -nr; ni = -ni; }
      const double nm = 1.0 / sqrt(nr * nr + ni * ni);
      phr = nr * nm;
      phi = ni * nm;
    }
    const double inr = ar / a2, ini = -ai / a2;  // 1 / a
    if (tid == 0 && flip) { perm[p + 1] = plq; perm[q] = pp1; }
    // the row that moves to position q takes the record of the old row p + 1
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (flip && p0 + tid + r * nt == q) {
#pragma unroll
        for (int t = 0; t < NBH; ++t) {
          ur[r][t] = p1rec[par][t]; ui[r][t] = p1rec[par][NBH + t];
          vr[r][t] = p1rec[par][2 * NBH + t]; vi[r][t] = p1rec[par][3 * NBH + t];
        }
        c0r[r] = p1rec[par][4 * NBH];
        c0i[r] = p1rec[par][4 * NBH + 1];
        pl[r] = pp1;
      }
    }
    // gathers: row pl_q now (c1) and the next step's pivot row, each with its
    // deferred sum
    const int p2 = (q == p + 2) ? pp1 : pp2;
    const bool more = s + 1 < ns;
    double d1r[RPT], d1i[RPT], d2r[RPT], d2i[RPT];
    deferred(plq, p2, d1r, d1i, d2r, d2i);
    // row q's U, V: broadcast reads from its LDS record
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = p0 + tid + r * nt;
      const bool act = l > p + 1 && l < m;
      const long long o1 = (long long)plq * ld + pl[r];
      const long long o2 = (long long)p2 * ld + pl[r];
      const double g1r = act ? Ar[o1] : 0.0, g1i = act ? Ai[o1] : 0.0;
      const bool nxt = more && l > p + 2 && l < m;
      const double g2r = nxt ? Ar[o2] : 0.0, g2i = nxt ? Ai[o2] : 0.0;
      double xr = -g1r + d1r[r], xi = -g1i + d1i[r], yr = 0.0, yi = 0.0;
#pragma unroll
      for (int t = 0; t < NBH; ++t) {
        const double upr = rq[t], upi = rq[NBH + t];
        const double vpr = rq[2 * NBH + t], vpi = rq[3 * NBH + t];
        // (U_l V_p - V_l U_p)_t, four fused multiply-adds per component;
        // even and odd t in separate accumulators (two dependency chains)
        double& sr = (t & 1) ? yr : xr;
        double& si = (t & 1) ? yi : xi;
        sr = fma(ur[r][t], vpr, sr);
        sr = fma(-ui[r][t], vpi, sr);
        sr = fma(-vr[r][t], upr, sr);
        sr = fma(vi[r][t], upi, sr);
        si = fma(ur[r][t], vpi, si);
        si = fma(ui[r][t], vpr, si);
        si = fma(-vr[r][t], upi, si);
        si = fma(-vi[r][t], upr, si);
      }
      xr += yr;
      xi += yi;
      // U[l][s] = b1_l = -c1_l ; V[l][s] = b0_l / a = -c0_l / a, appended after a shift
      const double br = -c0r[r], bi = -c0i[r];
#pragma unroll
      for (int t = 0; t + 1 < NBH; ++t) {
        ur[r][t] = ur[r][t + 1]; ui[r][t] = ui[r][t + 1];
        vr[r][t] = vr[r][t + 1]; vi[r][t] = vi[r][t + 1];
      }
      ur[r][NBH - 1] = act ? -xr : 0.0;
      ui[r][NBH - 1] = act ? -xi : 0.0;
      vr[r][NBH - 1] = act ? br * inr - bi * ini : 0.0;
      vi[r][NBH - 1] = act ? br * ini + bi * inr : 0.0;
      prr[r] = nxt ? -g2r + d2r[r] : 0.0;
      pri[r] = nxt ? -g2i + d2i[r] : 0.0;
    }
    // the next step's pivot row posts its U and V
    if (more) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        if (p0 + tid + r * nt == p + 2) {
#pragma unroll
          for (int t = 0; t < NBH; ++t) {
            bc[t] = ur[r][t]; bc[NBH + t] = ui[r][t]; bc[2 * NBH + t] = vr[r][t]; bc[3 * NBH + t] = vi[r][t];
          }
        }
      }
    }
    __syncthreads();
  }
  // entries 0 .. ns-1 to positions 0 .. ns-1
#pragma unroll 1
  for (int s = ns; s < NBH; ++s) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
      for (int t = 0; t + 1 < NBH; ++t) {
        ur[r][t] = ur[r][t + 1]; ui[r][t] = ui[r][t + 1];
        vr[r][t] = vr[r][t + 1]; vi[r][t] = vi[r][t + 1];
      }
      ur[r][NBH - 1] = 0.0; ui[r][NBH - 1] = 0.0; vr[r][NBH - 1] = 0.0; vi[r][NBH - 1] = 0.0;
    }
  }
  const int pe = p0 + 2 * ns;
  if (!last) {
    // append this panel's steps to the deferred columns (trailing rows only:
    // eliminated rows are never gathered again) and keep the permutation
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = p0 + tid + r * nt;
      if (l >= pe && l < m) {
        dpair* __restrict__ own = Dw + (long long)pl[r] * RS;
#pragma unroll
        for (int t = 0; t < NBH; ++t) {
          if (t < ns) {
            const dpair u = dpair{ur[r][t], ui[r][t]}, v = dpair{vr[r][t], vi[r][t]};
            own[2 * (kd + t)] = u;
            own[2 * (kd + t) + 1] = v;
            Twu[(long long)(kd + t) * m0 + pl[r]] = u;
            Twv[(long long)(kd + t) * m0 + pl[r]] = v;
          }
        }
        gperm[l] = pl[r];
      }
    }
  } else {
    // GEMM operands for the trailing rows, stored transposed (K x mp, leading
    // dimension mp = m - pe) so that consecutive lanes write consecutive
    // addresses: Lt = [U | V]^T, Rt = [V | -U]^T over all kall steps (the
    // deferred ones first); and the permutation
    const int mp = m - pe;
    double* Lr = Lall + (long long)mat * lstride;
    double* Li = Lr + l_im;
    double* Rr = RMall + (long long)mat * lstride;
    double* Ri = Rr + l_im;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = p0 + tid + r * nt;
      if (l >= pe && l < m) {
        const int i = l - pe;
        for (int t = 0; t < kd; ++t) {
          const long long o = (long long)t * m0 + pl[r];
          const dpair xu = Tu[o], xv = Tv[o];
          const long long ou = (long long)t * mp + i, ov = (long long)(kall + t) * mp + i;
          Lr[ou] = xu.x; Li[ou] = xu.y;
          Lr[ov] = xv.x; Li[ov] = xv.y;
          Rr[ou] = xv.x; Ri[ou] = xv.y;
          Rr[ov] = -xu.x; Ri[ov] = -xu.y;
        }
#pragma unroll
        for (int t = 0; t < NBH; ++t) {
          if (t < ns) {
            const long long ou = (long long)(kd + t) * mp + i, ov = (long long)(kall + kd + t) * mp + i;
            Lr[ou] = ur[r][t]; Li[ou] = ui[r][t];
            Lr[ov] = vr[r][t]; Li[ov] = vi[r][t];
            Rr[ou] = vr[r][t]; Ri[ou] = vi[r][t];
            Rr[ov] = -ur[r][t]; Ri[ov] = -ui[r][t];
          }
        }
        gperm[l] = pl[r];
      }
    }
  }
  if (tid == 0) {
    acc[mat * 3] = la;
    acc[mat * 3 + 1] = phr;
    acc[mat * 3 + 2] = phi;
    if (sing) atomicCAS(status, ST_OK, ST_SINGULAR);
  }
}

size_t pf_panel_lds_bytes(int m, int nbh) {
  (void)nbh;
  return sizeof(int) * (size_t)m + 64;
}

PfPanelShape pf_panel_shape(int m) {
  PfPanelShape sh;
  // at most 512 threads (256 VGPRs each): register rows x panel depth fixed.
  // Every shape up to m = 2048 compiles without spilling (with the deferred
  // sums 7 x 2 spilled 2 VGPRs, 4 x 4 112); above that the 1 x 8 one spills
  // (correct, slower).  The rank of the trailing updates is set by the
  // super-panel, not by these depths.
  if (m <= 512) { sh.nbh = 16; sh.rpt = 1; }
  else if (m <= 1024) { sh.nbh = 6; sh.rpt = 2; }
  else if (m <= 1536) { sh.nbh = 4; sh.rpt = 3; }
  else if (m <= 2048) { sh.nbh = 2; sh.rpt = 4; }
  else { sh.nbh = 1; sh.rpt = 8; }
  const int rows = (m + sh.rpt - 1) / sh.rpt;
  sh.nt = ((rows + 63) / 64) * 64;
  if (sh.nt > 512) sh.nt = 512;
  if (sh.nt < 64) sh.nt = 64;
  sh.ns = sh.nbh < m / 2 ? sh.nbh : m / 2;
  return sh;
}

hipError_t launch_pf_panel(const double* A, long long astride, long long plane, int ld, int m0, int p0, int ns,
                           int kd, int kall, int first, int last, int nmat, double* D, long long dstride, double* L,
                           double* RM, long long lstride, long long l_im, int* perm, int pstride, double* acc,
                           int first_acc, int* status, hipStream_t s) {
  const PfPanelShape sh = pf_panel_shape(m0 - p0);
  if (p0 < 0 || (p0 & 1) || ns < 1 || ns > sh.nbh || p0 + 2 * ns > m0 || kd < 0 || kd + ns > kall ||
      kall > PF_DEFER || (last && kd + ns != kall) || (long long)sh.nt * sh.rpt < m0 - p0 || m0 > 0xffff ||
      (long long)m0 * 8 * PF_DEFER > dstride)
    return hipErrorInvalidValue;
  const size_t lds = pf_panel_lds_bytes(m0, sh.nbh);
#define PF_LAUNCH(NB, RP)                                                                                        \
  hipLaunchKernelGGL((k_pf_panel<NB, RP>), dim3(nmat), dim3(sh.nt), lds, s, A, astride, plane, ld, m0, p0, ns, kd, \
                     kall, first, last, (const double*)D, D, dstride, L, RM, lstride, l_im, perm, pstride, acc,  \
                     first_acc, status)
  if (sh.nbh == 16) PF_LAUNCH(16, 1);
  else if (sh.nbh == 6) PF_LAUNCH(6, 2);
  else if (sh.nbh == 4) PF_LAUNCH(4, 3);
  else if (sh.nbh == 2) PF_LAUNCH(2, 4);
  else PF_LAUNCH(1, 8);
#undef PF_LAUNCH
  return hipGetLastError();
}

}  // namespace sgs
