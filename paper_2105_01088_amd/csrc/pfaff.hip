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
#include "wave_ops.h"

namespace sgs {

constexpr int PF_MAX_WAVES = 8;

// One panel of NBH elimination steps on the compact m x m trailing matrix A
// (planar, leading dimension ld, imaginary plane at +plane), for every
// matrix of the batch (one workgroup each).  Logical row l of the panel is
// owned by thread l % nt (slot l / nt < RPT), which keeps in registers its U
// and V entries, its current column value c0 and its stored index pl (row l
// of the panel is stored row pl of A; the stored matrix is never written
// during the panel).  Step s (p = 2 s):
//   c0_l = -A[pl_p][pl_l] + sum_t (U_l V_p - V_l U_p)_t      (l > p)
// the pivot row q maximizes |c0_q| (wave maxima of a packed key, posted per
// wave with the candidate's record: U, V, c0, pl); after one barrier every
// thread takes the best post.  Rows p+1 and q exchange (a sign flip of the
// Pfaffian): the owner of row q takes the record that row p+1 posted; row
// p+1 is eliminated and needs no registers.  With a = -c0_q:
//   c1_l = -A[pl_q][pl_l] + sum_t (U_l V_q - V_l U_q)_t,
//   U_l[s] = -c1_l,  V_l[s] = -c0_l / a                         (l > p + 1)
// The gather of row pl_q for c1 and the gather of the next step's pivot row
// are issued together, and the owner of row p + 2 posts its U and V for the
// next step before the second barrier: two barriers and one global latency
// per step.  At the end the panel writes, for the trailing logical rows
// l >= 2 ns, the GEMM operands L = [U | V] and Rm = [V | -U] transposed
// (2 NBH x mp, row l - 2 ns in column l - 2 ns) and perm[l] = pl_l; the
// trailing GEMM reads the old matrix through that permutation and writes the
// next, compact trailing matrix into the other buffer.
//   acc : per matrix {ln|Pf|, cos arg, sin arg}; first: start from Pf = 1
// dynamic LDS: m ints
template <int NBH, int RPT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_pf_panel(const double* __restrict__ Aall, long long astride, long long plane, int ld, int m,
                double* __restrict__ Lall, double* __restrict__ RMall, long long lstride, long long l_im,
                int* __restrict__ permall, int pstride, double* __restrict__ acc, int first,
                int* __restrict__ status) {
  constexpr int RB = 4 * NBH + 4;  // record: U re, U im, V re, V im (NBH each), c0 re, c0 im, pl (+ pad)
  __shared__ __attribute__((aligned(16))) double slot[2][PF_MAX_WAVES][RB];
  __shared__ unsigned long long skey[2][PF_MAX_WAVES];
  __shared__ __attribute__((aligned(16))) double p1rec[2][RB];
  __shared__ __attribute__((aligned(16))) double bc[4 * NBH];  // U re, U im, V re, V im of row p
  extern __shared__ int perm[];   // logical -> stored index, for the pivot rows of later steps
  const int mat = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const double* __restrict__ Ar = Aall + (long long)mat * astride;
  const double* __restrict__ Ai = Ar + plane;

  double ur[RPT][NBH], ui[RPT][NBH], vr[RPT][NBH], vi[RPT][NBH];
  double c0r[RPT], c0i[RPT], prr[RPT], pri[RPT];
  int pl[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int l = tid + r * nt;
    c0r[r] = 0.0;
    c0i[r] = 0.0;
    pl[r] = l;
#pragma unroll
    for (int t = 0; t < NBH; ++t) { ur[r][t] = 0.0; ui[r][t] = 0.0; vr[r][t] = 0.0; vi[r][t] = 0.0; }
    // the first pivot row is stored row 0
    prr[r] = (l > 0 && l < m) ? -Ar[l] : 0.0;
    pri[r] = (l > 0 && l < m) ? -Ai[l] : 0.0;
  }
  for (int l = tid; l < m; l += nt) perm[l] = l;
  for (int e = tid; e < 4 * NBH; e += nt) bc[e] = 0.0;  // row p's U, V before the first step
  double la = 0.0, phr = 1.0, phi = 0.0;  // uniform
  if (!first) { la = acc[mat * 3]; phr = acc[mat * 3 + 1]; phi = acc[mat * 3 + 2]; }
  bool sing = false;
  const int ns = min(NBH, m / 2);
  __syncthreads();

  // The step loop stays rolled (unrolled it is tens of KB of code fetched once
  // per panel: instruction-cache bound).  U and V entries are kept by age:
  // after s steps entries 0 .. s-1 sit at positions NBH-s .. NBH-1 and the
  // positions before them are zero, so every sum runs over all NBH positions
  // with constant register indices; each step shifts them left by one and
  // appends the new entry.  Posted records carry the same layout.
#pragma unroll 1
  for (int s = 0; s < ns; ++s) {
    const int p = 2 * s, par = s & 1;
    // current column p and the pivot search keys
    unsigned long long mine[RPT];
    unsigned long long key = 0;
    // row p's U, V are read by every lane from the same LDS addresses
    // (broadcast reads; the VALU only multiplies)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = tid + r * nt;
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
        const bool post = k2 == 0 ? (key != 0ull && mine[r] == key) : (tid + r * nt == p + 1);
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
    const int plq = (int)rq[4 * NBH + 2];
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
      if (flip && tid + r * nt == q) {
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
    // gathers: row pl_q now (c1) and the next step's pivot row
    const int p2 = (q == p + 2) ? pp1 : pp2;
    const bool more = s + 1 < ns;
    // row q's U, V: broadcast reads from its LDS record
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int l = tid + r * nt;
      const bool act = l > p + 1 && l < m;
      const long long o1 = (long long)plq * ld + pl[r];
      const long long o2 = (long long)p2 * ld + pl[r];
      const double g1r = act ? Ar[o1] : 0.0, g1i = act ? Ai[o1] : 0.0;
      const bool nxt = more && l > p + 2 && l < m;
      const double g2r = nxt ? Ar[o2] : 0.0, g2i = nxt ? Ai[o2] : 0.0;
      double xr = -g1r, xi = -g1i, yr = 0.0, yi = 0.0;
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
      prr[r] = -g2r;
      pri[r] = -g2i;
    }
    // the next step's pivot row posts its U and V
    if (more) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        if (tid + r * nt == p + 2) {
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
  // GEMM operands for the trailing rows, stored transposed (K x mp, leading
  // dimension mp = m - 2 ns) so that consecutive lanes write consecutive
  // addresses: Lt = [U | V]^T, Rt = [V | -U]^T; and the permutation
  const int pe = 2 * ns, mp = m - pe;
  double* Lr = Lall + (long long)mat * lstride;
  double* Li = Lr + l_im;
  double* Rr = RMall + (long long)mat * lstride;
  double* Ri = Rr + l_im;
  int* gperm = permall + (long long)mat * pstride;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int l = tid + r * nt;
    if (l >= pe && l < m) {
      const int i = l - pe;
#pragma unroll
      for (int t = 0; t < NBH; ++t) {
        const long long ou = (long long)t * mp + i, ov = (long long)(NBH + t) * mp + i;
        Lr[ou] = ur[r][t]; Li[ou] = ui[r][t];
        Lr[ov] = vr[r][t]; Li[ov] = vi[r][t];
        Rr[ou] = vr[r][t]; Ri[ou] = vi[r][t];
        Rr[ov] = -ur[r][t]; Ri[ov] = -ui[r][t];
      }
      gperm[i] = pl[r];
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
  // at most 512 threads (256 VGPRs each): register rows x panel depth fixed;
  // the shapes up to m = 1536 compile without spilling (8 x 2 and 4 x 4
  // spill 18 and 58 VGPRs: 4 x 4 took ~100 us per step at m = 1204)
  if (m <= 512) { sh.nbh = 16; sh.rpt = 1; }
  else if (m <= 1024) { sh.nbh = 7; sh.rpt = 2; }
  else if (m <= 1536) { sh.nbh = 4; sh.rpt = 3; }
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
  else if (sh.nbh == 7) PF_LAUNCH(7, 2);
  else if (sh.nbh == 4 && sh.rpt == 3) PF_LAUNCH(4, 3);
  else if (sh.nbh == 4) PF_LAUNCH(4, 4);
  else if (sh.nbh == 2) PF_LAUNCH(2, 8);
  else PF_LAUNCH(1, 16);
#undef PF_LAUNCH
  return hipGetLastError();
}

}  // namespace sgs
