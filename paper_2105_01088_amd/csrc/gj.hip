// Batched Gauss-Jordan inversion with partial pivoting, for the pair
// matrices S_ab = Gamma_a + Gamma_b.  W_ab = S_ab^{-1} enters the transition
// matrix of Eq. (def-delta-matrix), and ln|det S_ab| = sum ln|pivot| gives the
// overlap magnitude |<a|b>|^2 = 2^{-N} |det S_ab|^{1/2} (Sec. II.B).
//
// Pivoting is virtual: rows never move.  Logical row r of the elimination is
// physical row piv[r], the row chosen as pivot for column r.  Two levels of
// column panels: super-panels Js = [k0, k0+S) of up to 256 columns, each
// swept by panels J_t = [k, k+b) of up to 32 (position kl = k - k0 = t nbp
// inside the super-panel).  Panel t's exchange updates the whole block,
// B <- B - E_t Brow_t, with E_t = B[:, J_t] D (D = (pivot block)^-1; e_l - D_l
// on the pivot row of position l) and Brow_t = the pivot rows on Js (zero on
// J_t).  These updates are deferred: the stored block only changes in the
// columns of the panels swept so far (each holding its panel's output), and
// E_t, Brow_t are kept for the super-panel (E_all n x S, Brow_all S x S):
//   1. grouped GEMM (t > 0): M[:, J_t] -= E_all[:, 0:kl] Brow_all[0:kl, J_t],
//      the earlier panels' updates of this panel's columns only;
//   2. k_gj_panel (one workgroup per matrix) sweeps the n x b panel with
//      partial pivoting over the free rows and writes the final panel
//      columns (-E_i; D_l on the pivot rows), E_t into E_all and Brow_t into
//      Brow_all: its pivot rows as stored plus their deferred sums (columns
//      of later panels take every earlier panel's update, columns of an
//      earlier panel v those of the panels after v);
//   3. after the last panel, grouped GEMM: for every panel v but the last,
//      M[:, J_v] -= E_all[:, J_>v] Brow_all[J_>v, J_v] (the later panels'
//      updates of its output).
// The block is then read and written about twice per super-panel instead of
// once per panel.  Without deferral (a small batch, where the extra launch
// before every panel costs more than it saves) step 1 is absent, the panel
// takes its pivot rows as stored, and after it
//   M[:, Js] -= E_t Brow_t   (every column of the super-panel)
// replaces step 3.  After the super-panel it holds the exchange of the whole
// block (exchanges of column blocks compose): with P the pivot rows of Js,
// M[P, Js] = (M_old[P, Js])^-1 and M[i, Js] = -M_old[i, Js] M_old[P, Js]^-1
// elsewhere, and the rest of the matrix takes one rank-nb update:
//   3. k_gj_gather copies Brow = M[P, :] (zero on Js) and clears M[P, :]
//      outside Js;
//   4. grouped GEMM: M[:, c] <- M[:, c] + M[:, Js] Brow[:, c] for c outside Js
//      (on the cleared pivot rows this leaves M[P, Js] Brow, elsewhere the
//      exchange update), one read and write of the matrix per super-panel
//      instead of one per panel.
// Afterwards M[piv[r]][c] = W[r][pi(c)] with pi = piv, and k_gj_unscramble
// writes W[r][c] = M[piv[r]][piv^-1[c]] into a separate buffer.
#include "sgs_internal.h"
#include "wave_ops.h"

namespace sgs {

constexpr int GJ_MAX_WAVES = 8;

// Columns per LDS staging pass of a panel of width B: a divisor of B, at most
// 16 (a wave's 64 x (CB + 1) tile, 8.7 KB at CB = 16).
__host__ __device__ constexpr int gj_stage_cols(int B) {
  return B <= 16 ? B : B % 16 == 0 ? 16 : B % 12 == 0 ? 12 : B % 8 == 0 ? 8 : 1;
}

// Panel kernel.  Thread t owns the physical rows i = t + r nt (r < RPT) and
// keeps their b panel entries in registers.  The panel is swept column by
// column with the exchange (Gauss-Jordan pivot) operation: for the pivot row
// p of column j (pivot a = x[p][j]) every other row takes f = x[i][j] / a,
// x[i][c] -= f x[p][c] (c != j), x[i][j] = f, and the pivot row becomes
// x[p][c] = -x[p][c] / a, x[p][j] = 1 / a.  After the b columns the pivot row
// of position l holds row l of D = (pivot block)^-1 and every other row holds
// E_i = M[i, J] D, so the panel's outputs are read off the registers.
//
// Pivot search, column j: every free row (no pivot yet) offers a key, a wave
// maximum picks each wave's candidate, whose lane posts the key and its row
// to LDS; after the one barrier of the column every thread takes the best of
// the waves' posts.  Posts alternate between two LDS slots.  The next
// column's key is formed as soon as that column is updated, so its wave
// maximum overlaps the rest of the row update.  The column loop is rolled,
// with the row registers rotated one column per step.
// The panel moves between HBM and registers through a per-wave LDS tile, so
// that global loads and stores are row segments rather than one row per lane.
template <int B, int RPT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gj_panel(double* __restrict__ Mall, long long mstride,
                                                  int n, int k, int b,
                                                  double* __restrict__ Eall, long long estride, int eld,
                                                  double* __restrict__ Ball, long long bstride, int brld,
                                                  int bc0, int bc1, int nbp, int defer,
                                                  int* __restrict__ pivall, int* __restrict__ srcall,
                                                  double* __restrict__ logdet,
                                                  int* __restrict__ status) {
  constexpr int CB = gj_stage_cols(B);  // columns per LDS staging pass
  static_assert(B % CB == 0, "staging passes must tile the panel");
  // dynamic LDS: tag (n ints: 1 if the row is a pivot of an earlier panel),
  // then per wave a 64 x (CB + 1) staging tile, then per wave 64 ints
  extern __shared__ int tag[];
  __shared__ unsigned long long skey[2][GJ_MAX_WAVES];
  __shared__ __attribute__((aligned(16))) double srow[2][GJ_MAX_WAVES][B];
  __shared__ int pivl[B];
  const int mat = blockIdx.x;
  double* __restrict__ M = Mall + (long long)mat * mstride;
  double* __restrict__ E = Eall + (long long)mat * estride;
  double* __restrict__ Br = Ball + (long long)mat * bstride;
  int* __restrict__ piv = pivall + (long long)mat * n;
  int* __restrict__ src = srcall + (long long)mat * n;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const int kl = k - bc0;  // the panel's position in the super-panel

  for (int i = tid; i < n; i += nt) tag[i] = 0;
  // the panel into registers, through the wave's LDS tile: element e of a
  // 64 x CB chunk (row e / CB, column e % CB) goes to lane e % 64 of pass
  // e / 64, so a load instruction reads whole row segments; then every lane
  // takes its row
  double* __restrict__ stg = (double*)(tag + ((n + 3) & ~3)) + w * 64 * (CB + 1);
  int* __restrict__ spos = (int*)((double*)(tag + ((n + 3) & ~3)) + nw * 64 * (CB + 1)) + w * 64;
  double x[RPT][B];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int rbase = r * nt + w * 64;
#pragma unroll
    for (int h = 0; h < B / CB; ++h) {
#pragma unroll
      for (int s = 0; s < CB; ++s) {
        const int e = s * 64 + lane, rr = e / CB, cc = e % CB;
        const int i = rbase + rr, c = h * CB + cc;
        stg[rr * (CB + 1) + cc] = (i < n && c < b) ? M[(long long)i * n + k + c] : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) x[r][h * CB + cc] = stg[lane * (CB + 1) + cc];
      __builtin_amdgcn_wave_barrier();
      // (no global load of a later pass is hoisted above this one: their
      // registers would be live at once)
      __asm__ volatile("" ::: "memory");
    }
  }
  __syncthreads();
  for (int l = tid; l < k; l += nt) tag[piv[l]] = 1;
  __syncthreads();
  bool act[RPT];  // free: not a pivot row yet
  int pos[RPT];   // panel position of a pivot row of this panel, else -1
  unsigned long long mine[RPT];
  unsigned long long key = 0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * nt;
    act[r] = i < n && tag[i] == 0;
    pos[r] = -1;
    mine[r] = act[r] ? pivot_key(x[r][0], i) : 0ull;
    key = umax64(key, mine[r]);
  }
  key = wave_max_u64(key);
  // running |product of pivots| = pm 2^pe; singularity flag (all uniform)
  double pm = 1.0;
  int pe = 0;
  bool sing = false;

  // The column loop stays rolled over groups of U columns (its unrolled form
  // is tens of KB of code, fetched once per panel: instruction-cache bound).
  // Inside a group the current column is x[r][u]; after the group the
  // registers rotate by U columns, so the next group starts at x[r][0].
  // Posted rows carry the same rotation.
  constexpr int U = B < 4 ? B : 4;
#pragma unroll 1
  for (int j0 = 0; j0 < b; j0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u;
      if (j < b) {
        const int par = j & 1;
        if (lane == 0) skey[par][w] = key;
        int sel = -1;  // which owned row posts (selected by value, not by address)
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if (key != 0ull && mine[r] == key) sel = r;
        if (sel >= 0) {
#pragma unroll
          for (int c = 0; c < B; ++c) {
            double v = x[0][c];
#pragma unroll
            for (int r = 1; r < RPT; ++r) v = (sel == r) ? x[r][c] : v;
            srow[par][w][c] = v;
          }
        }
        __syncthreads();
        // best of the waves' posts: lane q < nw holds wave q's key
        const unsigned long long best = max8_u64(lane < nw ? skey[par][lane] : 0ull);
        int p = 0xffff - (int)(best & 0xffffull);
        const bool bad = best == 0ull || p >= n;
        if (bad) p = 0;  // cannot happen for b <= n - k; keeps every index in range
        const int ww = (p % nt) >> 6;  // the wave holding row p posted it
        // the pivot row, read by every lane from the same LDS address
        // (broadcast); ps is 16-byte aligned, so these are 128-bit reads
        const double* __restrict__ ps = srow[par][ww];
        double prow[B];
#pragma unroll
        for (int c = 0; c < B; ++c) prow[c] = ps[c];
        const double a = bad ? 0.0 : prow[u];
        if (bad || !(fabs(a) > 0.0) || !isfinite(a)) sing = true;
        {
          int e;
          pm *= frexp(fabs(a), &e);
          pe += e;
        }
        // 1 / a: hardware reciprocal and two Newton steps
        double ra = __builtin_amdgcn_rcp(a);
        ra = fma(ra, fma(-a, ra, 1.0), ra);
        ra = fma(ra, fma(-a, ra, 1.0), ra);
        if (tid == 0) pivl[j] = p;
        // the pivot row takes f = 0 in the common update and is then
        // rewritten in place from its own registers
        double f[RPT];
        bool isp[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          isp[r] = tid + r * nt == p;
          f[r] = isp[r] ? 0.0 : x[r][u] * ra;
          if (isp[r]) {
            act[r] = false;
            pos[r] = j;
          }
        }
        const int un = (u + 1) % B;  // the next column
        {
          const double p1 = prow[un];
#pragma unroll
          for (int r = 0; r < RPT; ++r) x[r][un] -= f[r] * p1;
        }
        if (j + 1 < b) {
          key = 0;
#pragma unroll
          for (int r = 0; r < RPT; ++r) {
            mine[r] = act[r] ? pivot_key(x[r][un], tid + r * nt) : 0ull;
            key = umax64(key, mine[r]);
          }
          key = wave_max_u64(key);
        }
#pragma unroll
        for (int c = 0; c < B; ++c) {
          if (c != u && c != un) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) x[r][c] -= f[r] * prow[c];
          }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) x[r][u] = f[r];
        // the pivot row's rewrite, behind a branch that is uniform per wave
        // (only the wave holding row p takes it)
        if (ww == w) {
#pragma unroll
          for (int r = 0; r < RPT; ++r) {
            if (isp[r]) {
#pragma unroll
              for (int c = 0; c < B; ++c)
                if (c != u) x[r][c] = -x[r][c] * ra;
              x[r][u] = ra;
            }
          }
        }
      }
    }
    // rotate by U: column j0 + U becomes x[r][0]
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      double t[U];
#pragma unroll
      for (int c = 0; c < U; ++c) t[c] = x[r][c];
#pragma unroll
      for (int c = 0; c + U < B; ++c) x[r][c] = x[r][c + U];
#pragma unroll
      for (int c = 0; c < U; ++c) x[r][B - U + c] = t[c];
    }
  }
  // after the groups column c sits at (c - U ceil(b / U)) mod B: rotate the
  // rest of the way to a multiple of B (U ceil(b / U) exceeds B when B is
  // not a multiple of U, as for B = 6)
  const int rot = (U * ((b + U - 1) / U)) % B;
#pragma unroll 1
  for (int j = rot == 0 ? B : rot; j < B; ++j) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const double t0 = x[r][0];
#pragma unroll
      for (int c = 0; c + 1 < B; ++c) x[r][c] = x[r][c + 1];
      x[r][B - 1] = t0;
    }
  }
  if (tid == 0) {
    logdet[mat] += log(pm) + (double)pe * 0.69314718055994530942;
    if (sing) atomicCAS(status, ST_OK, ST_SINGULAR);
  }
  __syncthreads();  // pivl complete
  // panel outputs (pivot rows M[i, J] = D_l, E_i = e_l - D_l; others
  // M[i, J] = -E_i), through the wave's LDS tile as row segments (the map of
  // the loads).  The lane index is passed through an empty asm statement so
  // that the addresses are formed here, not kept live across the column loop
  // from the loads (a register budget that otherwise spills).
  {
    int ln = lane;
    __asm__ volatile("" : "+v"(ln));
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int rbase = r * nt + w * 64;
      spos[ln] = pos[r];
#pragma unroll
      for (int h = 0; h < B / CB; ++h) {
#pragma unroll
        for (int cc = 0; cc < CB; ++cc) stg[ln * (CB + 1) + cc] = x[r][h * CB + cc];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s = 0; s < CB; ++s) {
          const int e = s * 64 + ln, rr = e / CB, cc = e % CB;
          const int i = rbase + rr, c = h * CB + cc;
          if (i < n && c < b) {
            const double v = stg[rr * (CB + 1) + cc];
            const int l = spos[rr];
            M[(long long)i * n + k + c] = l >= 0 ? v : -v;
            E[(long long)i * eld + kl + c] = l >= 0 ? (c == l ? 1.0 : 0.0) - v : v;
          }
        }
        __builtin_amdgcn_wave_barrier();
        __asm__ volatile("" ::: "memory");
      }
    }
  }
  // Brow_t: the pivot rows on the super-panel's columns (row kl + l of
  // Brow_all, leading dimension brld), zero on J_t, with the deferred sums of
  // the earlier panels: a column of a later panel takes every earlier
  // panel's update, a column of an earlier panel v those of panels v+1 ..
  // t-1.  The pivot rows' E entries of the earlier panels go to LDS first
  // (read as broadcasts); every thread then takes (row, column) items, a
  // wave covering consecutive columns of one row.
  // (after the per-wave row positions of every wave)
  double* __restrict__ es = (double*)((int*)((double*)(tag + ((n + 3) & ~3)) + nw * 64 * (CB + 1)) + nw * 64);
  const int kd = defer ? kl : 0;  // earlier panels whose updates are deferred
  for (int e = tid; e < b * kd; e += nt) {
    const int l = e / kd, j = e - l * kd;
    es[e] = E[(long long)pivl[l] * eld + j];
  }
  __syncthreads();
  // (BU items per thread and pass, their loads issued together: one
  // dependent load after another cost more than the rest of the panel)
  const int sw = bc1 - bc0, tot = b * sw;
  constexpr int BU = 8;
  for (int e0 = tid; e0 < tot; e0 += BU * nt) {
    double v[BU];
#pragma unroll
    for (int u = 0; u < BU; ++u) {
      const int e = e0 + u * nt;
      v[u] = 0.0;
      if (e < tot) {
        const int l = e / sw, lc = e - l * sw, c = bc0 + lc;
        if (c < k || c >= k + b) v[u] = M[(long long)pivl[l] * n + c];
      }
    }
#pragma unroll
    for (int u = 0; u < BU; ++u) {
      const int e = e0 + u * nt;
      if (e < tot) {
        const int l = e / sw, lc = e - l * sw, c = bc0 + lc;
        double y = v[u];
        if (c < k || c >= k + b) {
          const int js = c < k ? (lc / nbp + 1) * nbp : 0;
          const double* __restrict__ el = es + l * kd;
          for (int j = js; j < kd; ++j) y = fma(-el[j], Br[(long long)j * brld + lc], y);
        }
        Br[(long long)(kl + l) * brld + lc] = y;
      }
    }
  }
  if (tid < b) piv[k + tid] = pivl[tid];
  // after the last panel: src = piv^-1 for the unscramble
  if (k + b == n) {
    for (int c = tid; c < n; c += nt) src[c < k ? piv[c] : pivl[c - k]] = c;
  }
}

// Super-panel [k0, k0 + nb) done: Br[l][c] = M[piv[k0 + l]][c] (zero for c in
// the super-panel), then M[piv[k0 + l]][c] = 0 outside it.  grid (matrices,
// chunks); each element is read and cleared by the same thread.
__global__ __launch_bounds__(256) void k_gj_gather(double* __restrict__ Mall, long long mstride, int n, int k0,
                                                   int nb, const int* __restrict__ pivall, double* __restrict__ Ball,
                                                   long long bstride) {
  const int mat = blockIdx.x;
  double* __restrict__ M = Mall + (long long)mat * mstride;
  double* __restrict__ Br = Ball + (long long)mat * bstride;
  const int* __restrict__ piv = pivall + (long long)mat * n + k0;
  const long long total = (long long)nb * n;
  for (long long e = (long long)blockIdx.y * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.y * blockDim.x) {
    const int l = (int)(e / n), c = (int)(e - (long long)l * n);
    const bool ins = c >= k0 && c < k0 + nb;
    // (pivot index clamped: a singular matrix, flagged in the status word,
    // may leave the pivot list short of a permutation)
    const long long o = (long long)min(max(piv[l], 0), n - 1) * n + c;
    const double v = ins ? 0.0 : M[o];
    Br[e] = v;
    if (!ins) M[o] = 0.0;
  }
}

// grid (matrices, row chunks of rpb): W[r][c] = M[piv[r]][src[c]]
__global__ __launch_bounds__(256) void k_gj_unscramble(const double* __restrict__ Mall, double* __restrict__ Wall,
                                                       long long mstride, int n, const int* __restrict__ pivall,
                                                       const int* __restrict__ srcall, int rpb) {
  extern __shared__ double rowbuf[];  // rpb rows
  const int mat = blockIdx.x;
  const double* M = Mall + (long long)mat * mstride;
  double* W = Wall + (long long)mat * mstride;
  const int* piv = pivall + (long long)mat * n;
  const int* src = srcall + (long long)mat * n;
  const int r0 = blockIdx.y * rpb, nr = min(rpb, n - r0);
  // (indices clamped: a singular matrix, flagged in the status word, may leave
  // the pivot list short of a permutation)
  for (int r = 0; r < nr; ++r) {
    const double* mrow = M + (long long)min(max(piv[r0 + r], 0), n - 1) * n;
    for (int c = threadIdx.x; c < n; c += blockDim.x) rowbuf[r * n + c] = mrow[c];
  }
  __syncthreads();
  for (int r = 0; r < nr; ++r)
    for (int c = threadIdx.x; c < n; c += blockDim.x)
      W[(long long)(r0 + r) * n + c] = rowbuf[r * n + min(max(src[c], 0), n - 1)];
}

// Register budget: the panel (n x B doubles) lives in the registers of one
// workgroup of at most 512 threads, RPT x B doubles per thread (n <= 4096).
// Every shape compiles without spilling (32 x 3 spilled 377 VGPRs and took
// ~1 ms per panel at n = 1204; 8 x 8 spilled 21).
GjPanelShape gj_panel_shape(int n) {
  GjPanelShape sh;
  if (n <= 512) { sh.B = 32; sh.rpt = 1; }
  else if (n <= 1024) { sh.B = 32; sh.rpt = 2; }
  else if (n <= 1536) { sh.B = 24; sh.rpt = 3; }
  else if (n <= 2048) { sh.B = 16; sh.rpt = 4; }
  else { sh.B = 6; sh.rpt = 8; }
  const int rows = (n + sh.rpt - 1) / sh.rpt;
  sh.nt = ((rows + 63) / 64) * 64;
  if (sh.nt > 512) sh.nt = 512;
  if (sh.nt < 64) sh.nt = 64;
  return sh;
}

// tag, the per-wave staging tiles and row positions, then the b x kl pivot
// rows' E entries (kl = the panel's position in its super-panel)
size_t gj_panel_lds_bytes(int n, int kl, int b) {
  const GjPanelShape sh = gj_panel_shape(n);
  const int cb = gj_stage_cols(sh.B);
  const size_t nw = (size_t)sh.nt / 64;
  return sizeof(int) * (size_t)((n + 3) & ~3) + nw * 64 * (cb + 1) * sizeof(double) + nw * 64 * sizeof(int) +
         (size_t)b * kl * sizeof(double) + 64;
}

hipError_t launch_gj_panel(double* M, long long mstride, int nmat, int n, int k, int b,
                           double* E, long long estride, int eld, double* Br, long long bstride, int brld,
                           int bc0, int bc1, int nbp, int defer, int* piv, int* src, double* logdet,
                           int* status, hipStream_t s) {
  const GjPanelShape sh = gj_panel_shape(n);
  if (b < 1 || b > sh.B || k < 0 || k + b > n || (long long)sh.nt * sh.rpt < n) return hipErrorInvalidValue;
  if (bc0 < 0 || bc1 > n || bc0 > k || bc1 < k + b || nbp < b || (k - bc0) % nbp != 0 || eld < bc1 - bc0 ||
      brld < bc1 - bc0 || (long long)n * eld > estride || (long long)(bc1 - bc0) * brld > bstride)
    return hipErrorInvalidValue;
  const size_t lds = gj_panel_lds_bytes(n, defer ? k - bc0 : 0, b);
#define GJ_LAUNCH(BB, RP)                                                                                    \
  hipLaunchKernelGGL((k_gj_panel<BB, RP>), dim3(nmat), dim3(sh.nt), lds, s, M, mstride, n, k, b, E, estride, \
                     eld, Br, bstride, brld, bc0, bc1, nbp, defer, piv, src, logdet, status)
  if (sh.rpt == 1) GJ_LAUNCH(32, 1);
  else if (sh.rpt == 2) GJ_LAUNCH(32, 2);
  else if (sh.rpt == 3) GJ_LAUNCH(24, 3);
  else if (sh.rpt == 4) GJ_LAUNCH(16, 4);
  else GJ_LAUNCH(6, 8);
#undef GJ_LAUNCH
  return hipGetLastError();
}

hipError_t launch_gj_gather(double* M, long long mstride, int nmat, int n, int k0, int nb, const int* piv,
                            double* Br, long long bstride, hipStream_t s) {
  if (nb < 1 || k0 < 0 || k0 + nb > n || (long long)nb * n > bstride) return hipErrorInvalidValue;
  int chunks = (int)(((long long)nb * n + 255) / 256);
  if (chunks > 32) chunks = 32;
  hipLaunchKernelGGL(k_gj_gather, dim3(nmat, chunks), dim3(256), 0, s, M, mstride, n, k0, nb, piv, Br, bstride);
  return hipGetLastError();
}

hipError_t launch_gj_unscramble(const double* M, double* W, long long mstride, int nmat, int n, const int* piv,
                                const int* src, hipStream_t s) {
  // rows per block, <= 16 KB of LDS: a memory-bound copy wants many
  // workgroups per CU (48 KB blocks ran at 2.6 TB/s, 16 KB ones at 4.7 at
  // n = 1204)
  int rpb = (int)(((size_t)16 * 1024 / sizeof(double)) / (size_t)n);
  if (rpb > 16) rpb = 16;
  if (rpb < 1) rpb = 1;
  size_t lds = sizeof(double) * (size_t)rpb * n;
  hipLaunchKernelGGL(k_gj_unscramble, dim3(nmat, (n + rpb - 1) / rpb), dim3(256), lds, s, M, W, mstride, n,
                     piv, src, rpb);
  return hipGetLastError();
}

hipError_t set_gj_lds_limit(size_t bytes) {
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<32, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<32, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<24, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_gj_panel<16, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_gj_panel<6, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace sgs
