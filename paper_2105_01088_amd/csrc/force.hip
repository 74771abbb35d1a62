// Covariance-matrix force, Eq. (EOM-Gamma3) in the compact form that holds
// when lambda solves Eq. (eigLambda):
//   dGamma_mu = 2 Re{ w_mu sum_b lambda_b [ 2 G_mb K F K^T - (h_mb - E G_mb) D ] }
//   K F K^T   = F + i (Y - Y^T) + Y D,   D = Delta^{b mu}, F = F^{b mu}, Y = D F,
// with w_mu = lambda~_mu^* c_mu (c_mu of Eq. Bmu).  With c1 = 4 w_mu lambda_b G_mb
// and c2 = -2 w_mu lambda_b (h_mb - E G_mb) (tables from the amplitude solve):
//   dGamma_mu = sum_b Re{c1 (F + i (Y - Y^T) + Y D) + c2 D}.
// The dense part Re(c1 Y D) = Y_r Re(c1 D) - Y_i Im(c1 D) is one real GEMM of
// depth 2n per term; in k_force the workgroup for an output tile streams
// every term b through the matrix cores, forming the B operand Re(c1 D) /
// -Im(c1 D) on the fly from W (D_r = -2 W) and D_i, and writes the tile and
// its skew mirror (the force is skew: only tiles I <= J run).  In float64
// the B operand is c1 (D + i 1) (a 1 on the diagonal while staging), so
// the product also carries Re(c1 i Y).  The remaining terms,
// Re{c1 (F - i Y^T) + c2 D} (float32 products: also Re(c1 i Y), kept in
// float64), are elementwise and memory-bound: k_force_elem sums them into a
// second buffer on another stream while the matrix cores run (few
// registers, many waves to hide the loads), and k_force_join adds the two
// and takes the 1-norm the Euler step needs.  Each part is skew-completed
// (strict upper triangle of tiles mirrored, diagonal tiles antisymmetrized).
// That is exact for their sum, the skew force, when both parts use the same
// tiles, or when each part is skew by itself: Re(c1 Y D) = Re(c1 D F D) is,
// Re(c1 i Y) is not.  So only the 64 x 64 products, tiled like k_force_elem,
// carry Re(c1 i Y); with 128 x 128 or 80 x 80 product tiles k_force_elem
// adds it (direct_y), in float64.
// The pair (a < b) stores Delta^{ba}; the term for mu = b uses its complex
// conjugate (sgn = -1 on every imaginary part).
//
// Precision: TT = double runs the product on the FP64 matrix cores.  TT =
// float (the FP32 path) rounds both operands to float when they are staged
// and accumulates in float on the FP32 matrix cores (about 1e-7 relative);
// every other term is added in float64.
#include "sgs_internal.h"

#include <type_traits>

namespace sgs {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dvec4 mfma_t(double a, double b, dvec4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fvec4 mfma_t(float a, float b, fvec4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// accumulator register r of lane l holds row acc_row(l, r), column l % 16
// (f64: 4 r + l / 16; f32: 4 (l / 16) + r; both measured on gfx950)
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return 4 * r + (lane >> 4); }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef dvec4 type; };
template <> struct Vec4<float> { typedef fvec4 type; };

constexpr int FTK = 16;
constexpr int FLP = 64 + 1;

constexpr size_t force_lds_bytes(size_t elem) {
  return (2 * 2 * FTK * FLP * elem) > (64 * FLP * sizeof(double)) ? (2 * 2 * FTK * FLP * elem)
                                                                  : (64 * FLP * sizeof(double));
}

// grid: 8 * ceil(R / 8) * ntri blocks of 256 threads.  Blocks are dispatched
// round-robin over the 8 XCDs; block b serves state mu = b % 8 + 8 s on XCD
// b % 8, so all tiles of a state share that XCD's L2 (every tile of state mu
// streams the same Y and Delta panels).  terms: R*R descriptors (mu-major);
// coef: c1 then c2 tables, complex interleaved, R*R each.
template <typename TT, bool IY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_force(int n, int R, int T, int nsplit, const ForceTerm* __restrict__ terms,
                                               const double* __restrict__ coef,
                                               double* __restrict__ dG, double* __restrict__ dP,
                                               unsigned long long* __restrict__ nrm) {
  typedef typename Vec4<TT>::type V4;
  // K-loop staging As[re/im], Bs[re/im] and the epilogue's transposed block
  // (Tt, float64) share LDS
  __shared__ __attribute__((aligned(16))) char lds_raw[force_lds_bytes(sizeof(TT))];
  typedef TT Slab[FTK][FLP];
  Slab* As = (Slab*)lds_raw;      // As[part]
  Slab* Bs = (Slab*)lds_raw + 2;  // Bs[part]
  double (*Tt)[FLP] = (double (*)[FLP])lds_raw;  // 64 x FLP

  const int ntri = T * (T + 1) / 2;
  const int xcd = blockIdx.x & 7, loc2 = blockIdx.x >> 3;
  // each tile's terms are split over nsplit workgroups (the same XCD);
  // split h sums terms [h R / S, (h + 1) R / S) into dG (h = 0) or slice
  // h - 1 of dP
  const int split = loc2 % nsplit, loc = loc2 / nsplit;
  const int mu = xcd + 8 * (loc / ntri);
  if (mu >= R) return;
  const int b_lo = split * R / nsplit, b_hi = (split + 1) * R / nsplit;
  // upper-triangular tile index -> (I, J), I <= J
  if (loc % ntri == 0 && split == 0 && threadIdx.x == 0) nrm[mu] = 0ull;  // k_force_join accumulates it
  int tri = loc % ntri, I = 0;
  while (tri >= T - I) { tri -= T - I; ++I; }
  const int J = I + tri;
  const int row0 = I * 64, col0 = J * 64;
  const long long nn = (long long)n * n;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

  const double* c1t = coef;
  const double* c2t = coef + 2 * R * R;

  // A slab: rows row0..+63, k kc..kc+15  (thread: row tid>>2, 4 consecutive k)
  const int a_i = tid >> 2, a_k = (tid & 3) * 4;
  // B slab: k kc..kc+15, cols col0..+63 (thread: column tid & 63, k rows
  // 4 (tid >> 6) + r: every wave reads and writes 64 consecutive columns, so
  // the loads are row segments and the LDS stores hit distinct banks)
  const int b_k = (tid >> 6) * 4, b_j = tid & 63;

  // One loop for every term (one set of accumulator registers): `im` (the
  // term has imaginary planes) is uniform, so its branches are scalar.
  for (int b = b_lo; b < b_hi; ++b) {
    const ForceTerm tm = terms[mu * R + b];
    const double x1 = c1t[2 * tm.coef], y1 = c1t[2 * tm.coef + 1];
    const bool im = tm.Yi != nullptr;
    const double sg = tm.sgn, ds = tm.dr_scale;
    const SGS_GLOBAL double* __restrict__ Yr = as_global(tm.Yr);
    const SGS_GLOBAL double* __restrict__ Yi = as_global(im ? tm.Yi : tm.Yr);
    const SGS_GLOBAL double* __restrict__ Dr = as_global(tm.Dr);
    const SGS_GLOBAL double* __restrict__ Di = as_global(im ? tm.Di : tm.Dr);
    // raw prefetch registers: the B operand Re(c1 D) / -Im(c1 D) is formed
    // when the slab is written to LDS, so the loads of the next slab stay in
    // flight across the current slab's matrix-core work (a term without
    // imaginary planes reads its real ones twice and ignores the copy)
    double ra[2][4], rd[2][4];
    auto load = [&](int kc) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = row0 + a_i, gk = kc + a_k + r;
        const bool ok = gi < n && gk < n;
        const long long o = (long long)gi * n + gk;
        ra[0][r] = ok ? Yr[o] : 0.0;
        ra[1][r] = ok ? Yi[o] : 0.0;
        const int gk2 = kc + b_k + r, gj = col0 + b_j;
        const bool okb = gk2 < n && gj < n;
        const long long ob = (long long)gk2 * n + gj;
        rd[0][r] = okb ? Dr[ob] : 0.0;
        rd[1][r] = okb ? Di[ob] : 0.0;
      }
    };
    const double sgi = im ? sg : 0.0;  // zero imaginary parts for a real term
    load(0);
    for (int kc = 0; kc < n; kc += FTK) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // IY: B = c1 (D + i 1), so the product also carries Re(c1 i Y)
        const double dr = ds * rd[0][r],
                     di = sgi * rd[1][r] + (IY && kc + b_k + r == col0 + b_j && col0 + b_j < n ? 1.0 : 0.0);
        // A: Y_r, sg Y_i; B: Re(c1 D), -Im(c1 D)
        As[0][a_k + r][a_i] = (TT)ra[0][r];
        As[1][a_k + r][a_i] = (TT)(sgi * ra[1][r]);
        Bs[0][b_k + r][b_j] = (TT)(x1 * dr - y1 * di);
        Bs[1][b_k + r][b_j] = (TT)(-(x1 * di + y1 * dr));
      }
      __syncthreads();
      if (kc + FTK < n) load(kc + FTK);
      // operand fragments of k-step kk + 1 are read from LDS while the
      // matrix cores work on k-step kk
      TT ah[2][2][2], bh[2][2][2];  // [buffer][re/im][q]
      auto frag = [&](int kk, int buf) {
        const int kr = kk * 4 + (lane >> 4);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            ah[buf][u][q] = As[u][kr][wm * 32 + q * 16 + (lane & 15)];
            bh[buf][u][q] = Bs[u][kr][wn * 32 + q * 16 + (lane & 15)];
          }
      };
      frag(0, 0);
#pragma unroll
      for (int kk = 0; kk < FTK / 4; ++kk) {
        const int cur = kk & 1;
        if (kk + 1 < FTK / 4) frag(kk + 1, cur ^ 1);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma_t(ah[cur][0][bi], bh[cur][0][bj], acc[bi][bj]);
        if (im) {
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma_t(ah[cur][1][bi], bh[cur][1][bj], acc[bi][bj]);
        }
      }
    }
  }

  // ---- total, skew write-out ----
  __syncthreads();
  double* out = (split == 0 ? dG : dP + (long long)(split - 1) * R * nn) + (long long)mu * nn;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = wm * 32 + bi * 16 + acc_row<TT>(lane, r);
        const int lj = wn * 32 + bj * 16 + (lane & 15);
        const int gi = row0 + li, gj = col0 + lj;
        double v = 0.0;
        if (gi < n && gj < n) v = (double)acc[bi][bj][r];
        if (I == J) Tt[li][lj] = v;
        else if (gi < n && gj < n) {
          out[(long long)gi * n + gj] = v;
          out[(long long)gj * n + gi] = -v;
        }
      }
  if (I == J) {
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
      const int li = e >> 6, lj = e & 63;
      const int gi = row0 + li, gj = col0 + lj;
      if (gi < n && gj < n) out[(long long)gi * n + gj] = 0.5 * (Tt[li][lj] - Tt[lj][li]);
    }
  }
}

// The FP32 products with 80 x 80 output tiles, for n where they waste less
// padding than 64 x 64 ones (n = 400 and 800 are multiples of 80: 15 and 55
// upper tiles per state instead of 28 and 91 of 64, 16% and 6% fewer
// matrix-core operations).  Five waves per workgroup, each owning a 16-row
// strip of the tile (1 x 5 MFMA blocks): a wave reads its own A rows and
// every B column from LDS.  Grid, XCD mapping, term split and write-out as
// in k_force.  (At n = 400, R = 16: 0.72 ms instead of 0.96.  The float64
// instance needs 190 VGPRs, one workgroup per CU, or stalls on LDS when held
// to three waves per SIMD: 2.06 ms instead of 1.15, so float64 keeps the
// 64 x 64 kernel.)
constexpr int FS_T = 80;             // tile edge
constexpr int FS_W = FS_T / 16;      // waves per workgroup
constexpr int FS_LP = FS_T + 1;      // LDS pitch
constexpr int FS_THREADS = 64 * FS_W;

template <typename TT>
__global__ __launch_bounds__(FS_THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_force_strip(int n, int R, int T, int nsplit, const ForceTerm* __restrict__ terms,
                                                          const double* __restrict__ coef,
                                                          double* __restrict__ dG, double* __restrict__ dP,
                                                          unsigned long long* __restrict__ nrm) {
  typedef typename Vec4<TT>::type V4;
  constexpr size_t stage_bytes = 2 * 2 * FTK * FS_LP * sizeof(TT);
  constexpr size_t tt_bytes = FS_T * FS_LP * sizeof(double);
  __shared__ __attribute__((aligned(16))) char lds_raw[stage_bytes > tt_bytes ? stage_bytes : tt_bytes];
  typedef TT Slab[FTK][FS_LP];
  Slab* As = (Slab*)lds_raw;      // As[part]
  Slab* Bs = (Slab*)lds_raw + 2;  // Bs[part]
  double (*Tt)[FS_LP] = (double (*)[FS_LP])lds_raw;

  const int ntri = T * (T + 1) / 2;
  const int xcd = blockIdx.x & 7, loc2 = blockIdx.x >> 3;
  const int split = loc2 % nsplit, loc = loc2 / nsplit;
  const int mu = xcd + 8 * (loc / ntri);
  if (mu >= R) return;
  const int b_lo = split * R / nsplit, b_hi = (split + 1) * R / nsplit;
  if (loc % ntri == 0 && split == 0 && threadIdx.x == 0) nrm[mu] = 0ull;  // k_force_join accumulates it
  int tri = loc % ntri, I = 0;
  while (tri >= T - I) { tri -= T - I; ++I; }
  const int J = I + tri;
  const int row0 = I * FS_T, col0 = J * FS_T;
  const long long nn = (long long)n * n;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  V4 acc[FS_W];
#pragma unroll
  for (int j = 0; j < FS_W; ++j) acc[j] = V4{0, 0, 0, 0};

  const double* c1t = coef;
  // A slab: rows row0 .. +79, k kc .. kc+15 (thread: row tid >> 2, 4 consecutive k)
  const int a_i = tid >> 2, a_k = (tid & 3) * 4;
  // B slab: k kc .. kc+15, columns col0 .. +79 (thread: column tid % 80, 4 rows)
  const int b_k = (tid / FS_T) * 4, b_j = tid % FS_T;

  auto run_term = [&](const ForceTerm& tm, double x1, double y1, auto im_tag) {
    constexpr bool IM = decltype(im_tag)::value;
    const double sg = tm.sgn, ds = tm.dr_scale;
    const SGS_GLOBAL double* __restrict__ Yr = as_global(tm.Yr);
    const SGS_GLOBAL double* __restrict__ Yi = as_global(IM ? tm.Yi : tm.Yr);
    const SGS_GLOBAL double* __restrict__ Dr = as_global(tm.Dr);
    const SGS_GLOBAL double* __restrict__ Di = as_global(IM ? tm.Di : tm.Dr);
    double ra[2][4], rd[2][4];
    auto load = [&](int kc) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = row0 + a_i, gk = kc + a_k + r;
        const bool ok = gi < n && gk < n;
        const long long o = (long long)gi * n + gk;
        ra[0][r] = ok ? Yr[o] : 0.0;
        ra[1][r] = (IM && ok) ? Yi[o] : 0.0;
        const int gk2 = kc + b_k + r, gj = col0 + b_j;
        const bool okb = gk2 < n && gj < n;
        const long long ob = (long long)gk2 * n + gj;
        rd[0][r] = okb ? Dr[ob] : 0.0;
        rd[1][r] = (IM && okb) ? Di[ob] : 0.0;
      }
    };
    load(0);
    for (int kc = 0; kc < n; kc += FTK) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double dr = ds * rd[0][r], di = sg * rd[1][r];
        As[0][a_k + r][a_i] = (TT)ra[0][r];
        Bs[0][b_k + r][b_j] = (TT)(x1 * dr - y1 * di);
        if (IM) {
          As[1][a_k + r][a_i] = (TT)(sg * ra[1][r]);
          Bs[1][b_k + r][b_j] = (TT)(-(x1 * di + y1 * dr));
        }
      }
      __syncthreads();
      if (kc + FTK < n) load(kc + FTK);
#pragma unroll
      for (int kk = 0; kk < FTK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (!IM && u) continue;
          const TT ah = As[u][kr][w * 16 + (lane & 15)];
          TT bh[FS_W];
#pragma unroll
          for (int bj = 0; bj < FS_W; ++bj) bh[bj] = Bs[u][kr][bj * 16 + (lane & 15)];
#pragma unroll
          for (int bj = 0; bj < FS_W; ++bj) acc[bj] = mfma_t(ah, bh[bj], acc[bj]);
        }
      }
    }
  };
  for (int b = b_lo; b < b_hi; ++b) {
    const ForceTerm tm = terms[mu * R + b];
    const double x1 = c1t[2 * tm.coef], y1 = c1t[2 * tm.coef + 1];
    if (tm.Yi != nullptr) run_term(tm, x1, y1, std::true_type{});
    else run_term(tm, x1, y1, std::false_type{});
  }

  // ---- total, skew write-out ----
  __syncthreads();
  double* out = (split == 0 ? dG : dP + (long long)(split - 1) * R * nn) + (long long)mu * nn;
#pragma unroll
  for (int bj = 0; bj < FS_W; ++bj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int li = w * 16 + acc_row<TT>(lane, r);
      const int lj = bj * 16 + (lane & 15);
      const int gi = row0 + li, gj = col0 + lj;
      double v = 0.0;
      if (gi < n && gj < n) v = (double)acc[bj][r];
      if (I == J) Tt[li][lj] = v;
      else if (gi < n && gj < n) {
        out[(long long)gi * n + gj] = v;
        out[(long long)gj * n + gi] = -v;
      }
    }
  if (I == J) {
    __syncthreads();
    for (int e = tid; e < FS_T * FS_T; e += FS_THREADS) {
      const int li = e / FS_T, lj = e % FS_T;
      const int gi = row0 + li, gj = col0 + lj;
      if (gi < n && gj < n) out[(long long)gi * n + gj] = 0.5 * (Tt[li][lj] - Tt[lj][li]);
    }
  }
}

// Elementwise terms of state mu, tile (I, J), I <= J:
//   sum_b Re{c1 (F + i (Y - Y^T)) + c2 D}
// written out: (y1 Yr + x1 sg Yi)(j, i) - y1 Yr(i, j) - x1 sg Yi(i, j)
// + x2 ds Dr(i, j) - y2 sg Di(i, j), plus x1 F_r - y1 sg F_i on the impurity
// block, plus (sum_b x1) A (F = A + the impurity correction).
// grid: (ntri, R), 512 threads; thread: column tid & 63, rows tid >> 6 + 8 k.
// The (j, i) terms are read row-contiguous from block (J, I) and summed over
// b in registers at the thread's own (J, I) positions; one transpose through
// LDS at the end puts them at (i, j), so the term loop has no barrier.
__global__ __launch_bounds__(512) void k_force_elem(int n, int R, int T, const ForceTerm* __restrict__ terms,
                                                    const double* __restrict__ coef,
                                                    const double* __restrict__ Adense,
                                                    const int* __restrict__ impos, int M, int direct_y,
                                                    double* __restrict__ dE) {
  __shared__ double Tt[64][64 + 1];
  const int mu = blockIdx.y;
  int tri = blockIdx.x, I = 0;
  while (tri >= T - I) { tri -= T - I; ++I; }
  const int J = I + tri;
  const int row0 = I * 64, col0 = J * 64;
  const long long nn = (long long)n * n;
  const int tid = threadIdx.x, lj = tid & 63, lr = tid >> 6;
  const int gj = col0 + lj;   // direct element (row0 + li, gj)
  const int gc = row0 + lj;   // transposed element (col0 + li, gc)
  const double* c1t = coef;
  const double* c2t = coef + 2 * R * R;
  double lin[8], tsum[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) { lin[k] = 0.0; tsum[k] = 0.0; }
  double sx1 = 0.0;
  for (int b = 0; b < R; ++b) {
    const ForceTerm tm = terms[mu * R + b];
    const double x1 = c1t[2 * tm.coef], y1 = c1t[2 * tm.coef + 1];
    const double x2 = c2t[2 * tm.coef], y2 = c2t[2 * tm.coef + 1];
    const bool has_im = tm.Yi != nullptr;
    const double im = has_im ? 1.0 : 0.0;  // terms without imaginary planes read Yr / Dr in their place
    const double sg = tm.sgn, ds = tm.dr_scale;
    const SGS_GLOBAL double* __restrict__ Yr = as_global(tm.Yr);
    const SGS_GLOBAL double* __restrict__ Yi = as_global(has_im ? tm.Yi : tm.Yr);
    const SGS_GLOBAL double* __restrict__ Dr = as_global(tm.Dr);
    const SGS_GLOBAL double* __restrict__ Di = as_global(has_im ? tm.Di : tm.Dr);
    sx1 += x1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int li = lr + 8 * k;
      // (y1 Yr + x1 sg Yi) at (col0 + li, row0 + lj): the (j, i) term of
      // output element (row0 + lj, col0 + li)
      const int gr = col0 + li;
      const bool okt = gr < n && gc < n;
      const long long ot = okt ? (long long)gr * n + gc : 0;
      tsum[k] += okt ? y1 * Yr[ot] + im * x1 * sg * Yi[ot] : 0.0;
      const int gi = row0 + li;
      const bool ok = gi < n && gj < n;
      const long long o = ok ? (long long)gi * n + gj : 0;
      double v = x2 * ds * Dr[o] - im * y2 * sg * Di[o];
      if (direct_y) v += -y1 * Yr[o] - im * x1 * sg * Yi[o];
      if (M > 0 && ok) {
        const int pi = impos[gi], pj = impos[gj];
        if (pi >= 0 && pj >= 0) {
          v += x1 * as_global(tm.Fcr)[pi * M + pj];
          if (tm.Fci) v -= y1 * sg * as_global(tm.Fci)[pi * M + pj];
        }
      }
      if (ok) lin[k] += v;
    }
  }
  // Tt[lj][li] = tsum: the (j, i) sums of output element (row0 + lj, col0 + li)
#pragma unroll
  for (int k = 0; k < 8; ++k) Tt[lj][lr + 8 * k] = tsum[k];
  __syncthreads();
  double* out = dE + (long long)mu * nn;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int li = lr + 8 * k, gi = row0 + li;
    v[k] = (gi < n && gj < n) ? lin[k] + Tt[li][lj] + sx1 * Adense[(long long)gi * n + gj] : 0.0;
  }
  if (I == J) {
    // the diagonal tile antisymmetrized through LDS
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) Tt[lr + 8 * k][lj] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int li = lr + 8 * k, gi = row0 + li;
      if (gi < n && gj < n) out[(long long)gi * n + gj] = 0.5 * (Tt[li][lj] - Tt[lj][li]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int li = lr + 8 * k, gi = row0 + li;
      if (gi < n && gj < n) {
        out[(long long)gi * n + gj] = v[k];
        out[(long long)gj * n + gi] = -v[k];
      }
    }
  }
}

// dG <- dG + (the partial products in dP) + dE (the elementwise terms), and
// the largest row sum of |dG_mu| (= 1-norm: skew) into
// nrm[mu] as an ordered bit pattern (k_force cleared it).  grid:
// (ceil(n / 16), R); one wave per row.
__global__ __launch_bounds__(256) void k_force_join(double* __restrict__ dG, const double* __restrict__ dP,
                                                    const double* __restrict__ dE, int n, int R, int nsplit,
                                                    unsigned long long* __restrict__ nrm) {
  __shared__ double red[4];
  const int mu = blockIdx.y;
  const long long nn = (long long)n * n;
  double* d = dG + mu * nn;
  const double* de = dE + mu * nn;
  const double* dp = dP + mu * nn;
  const long long pstride = (long long)R * nn;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double mx = 0.0;
  for (int i = blockIdx.x * 16 + wv; i < min(n, (int)blockIdx.x * 16 + 16); i += 4) {
    double s = 0.0;
    for (int j = lane; j < n; j += 64) {
      const long long o = (long long)i * n + j;
      double v = d[o] + de[o];
      for (int h = 0; h + 1 < nsplit; ++h) v += dp[h * pstride + o];
      d[o] = v;
      s += fabs(v);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    mx = nan_max(mx, s);
  }
  if (lane == 0) red[wv] = mx;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(nrm + mu, (unsigned long long)__double_as_longlong(nan_max(nan_max(red[0], red[1]), nan_max(red[2], red[3]))));
}

// The dense products with 128 x 128 output tiles, for large n: eight waves,
// each holding a 32 x 64 block of the tile in 2 x 4 MFMA accumulators, so a
// workgroup stages twice the operand bytes of a 64 x 64 tile per slab for four
// times the matrix-core work (16 instead of 8 flops per staged byte).  The K
// slabs (16 deep) are double-buffered in LDS: the raw loads of slab k + 1 are
// in flight while slab k is multiplied, then written (with the B operand
// formed, as in k_force) into the other buffer, one barrier per slab.  One
// workgroup per CU (the buffers take 132 KB of LDS in float64), two waves per
// SIMD.  (Four waves of 64 x 64, one per SIMD, left the LDS-to-MFMA latency
// exposed: 49 instead of 26 ms at n = 800, R = 32.)  Grid, XCD mapping,
// term split and skew write-out as in k_force; diagonal tiles are made
// exactly skew through LDS.
constexpr int FB_T = 128;            // tile edge
// LDS layout of the slabs: element (k, i) at row k, column i ^ swz(k), rows
// LP elements apart.  A-operand stores put 4 slab rows 4 apart in one pass
// (4 columns each for float64, 8 for float32); reads put one row (float64)
// or two consecutive rows (float32) in a pass.
//  * float64, 16 lanes a pass: a pitch of 1 mod 4 puts the store rows on
//    disjoint banks (132 made every A store a 4-way conflict);
//  * float32, 32 lanes a pass: no pitch serves both patterns, so the column
//    is swizzled by the row: bit 4 by its parity (two consecutive rows on
//    disjoint halves) and bits 3-4 by row / 4 (the 4 store rows on distinct
//    groups of 8).
template <typename TT> struct FbLds;
template <> struct FbLds<double> {
  static constexpr int LP = FB_T + 1;
  static __device__ __forceinline__ int swz(int) { return 0; }
};
template <> struct FbLds<float> {
  static constexpr int LP = FB_T;
  static __device__ __forceinline__ int swz(int k) { return ((k & 1) << 4) ^ (((k >> 2) & 3) << 3); }
};

template <typename TT>
constexpr size_t force_big_lds_bytes() {
  return (2 * 2 * 2 * FTK * FbLds<TT>::LP * sizeof(TT)) > (FB_T * (FB_T + 1) * sizeof(double))
             ? (2 * 2 * 2 * FTK * FbLds<TT>::LP * sizeof(TT))
             : (FB_T * (FB_T + 1) * sizeof(double));
}

// (no Re(c1 i Y) fold: its tiles are not those of k_force_elem)
template <typename TT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_force_big(
    int n, int R, int T, int nsplit, const ForceTerm* __restrict__ terms, const double* __restrict__ coef,
    double* __restrict__ dG, double* __restrict__ dP, unsigned long long* __restrict__ nrm) {
  typedef typename Vec4<TT>::type V4;
  extern __shared__ __attribute__((aligned(16))) char lds_big[];
  typedef TT Slab[FTK][FbLds<TT>::LP];
  Slab* As = (Slab*)lds_big;      // As[buf * 2 + part]
  Slab* Bs = (Slab*)lds_big + 4;  // Bs[buf * 2 + part]
  double (*Tt)[FB_T + 1] = (double (*)[FB_T + 1])lds_big;

  const int ntri = T * (T + 1) / 2;
  const int xcd = blockIdx.x & 7, loc2 = blockIdx.x >> 3;
  const int split = loc2 % nsplit, loc = loc2 / nsplit;
  const int mu = xcd + 8 * (loc / ntri);
  if (mu >= R) return;
  const int b_lo = split * R / nsplit, b_hi = (split + 1) * R / nsplit;
  if (loc % ntri == 0 && split == 0 && threadIdx.x == 0) nrm[mu] = 0ull;  // k_force_join accumulates it
  int tri = loc % ntri, I = 0;
  while (tri >= T - I) { tri -= T - I; ++I; }
  const int J = I + tri;
  const int row0 = I * FB_T, col0 = J * FB_T;
  const long long nn = (long long)n * n;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;  // rows wm * 32 .. +31, columns wn * 64 .. +63
  V4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = V4{0, 0, 0, 0};

  const double* c1t = coef;
  // A slab: rows row0 .. +127, k kc .. kc+15 (thread: row tid >> 2, 4
  // consecutive k); B slab: k kc .. kc+15, columns col0 .. +127 (thread:
  // column tid & 127, k rows 4 (tid >> 7) + r)
  const int a_i = tid >> 2, a_k = (tid & 3) * 4;
  const int b_k = (tid >> 7) * 4, b_j = tid & 127;

  for (int b = b_lo; b < b_hi; ++b) {
    const ForceTerm tm = terms[mu * R + b];
    const double x1 = c1t[2 * tm.coef], y1 = c1t[2 * tm.coef + 1];
    const bool im = tm.Yi != nullptr;
    const double sg = tm.sgn, ds = tm.dr_scale;
    const double sgi = im ? sg : 0.0;  // zero imaginary parts for a real term
    const SGS_GLOBAL double* __restrict__ Yr = as_global(tm.Yr);
    const SGS_GLOBAL double* __restrict__ Yi = as_global(im ? tm.Yi : tm.Yr);
    const SGS_GLOBAL double* __restrict__ Dr = as_global(tm.Dr);
    const SGS_GLOBAL double* __restrict__ Di = as_global(im ? tm.Di : tm.Dr);
    double ra[2][4], rd[2][4];
    auto load = [&](int kc) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = row0 + a_i, gk = kc + a_k + r;
        const bool ok = gi < n && gk < n;
        const long long o = ok ? (long long)gi * n + gk : 0;
        ra[0][r] = ok ? Yr[o] : 0.0;
        ra[1][r] = ok ? Yi[o] : 0.0;
        const int gk2 = kc + b_k + r, gj = col0 + b_j;
        const bool okb = gk2 < n && gj < n;
        const long long ob = okb ? (long long)gk2 * n + gj : 0;
        rd[0][r] = okb ? Dr[ob] : 0.0;
        rd[1][r] = okb ? Di[ob] : 0.0;
      }
    };
    auto store = [&](int kc, int buf) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double dr = ds * rd[0][r], di = sgi * rd[1][r];
        const int ai = a_i ^ FbLds<TT>::swz(a_k + r), bj = b_j ^ FbLds<TT>::swz(b_k + r);
        As[2 * buf][a_k + r][ai] = (TT)ra[0][r];
        As[2 * buf + 1][a_k + r][ai] = (TT)(sgi * ra[1][r]);
        Bs[2 * buf][b_k + r][bj] = (TT)(x1 * dr - y1 * di);
        Bs[2 * buf + 1][b_k + r][bj] = (TT)(-(x1 * di + y1 * dr));
      }
    };
    // the slab loop, compiled once for complex and once for real terms (no
    // branch between the matrix instructions); the operand fragments of
    // k-step kk + 1 are read from LDS while the matrix cores work on kk
    auto slabs = [&](auto im_tag) {
      constexpr bool IM = decltype(im_tag)::value;
      constexpr int NU = IM ? 2 : 1;
      __syncthreads();  // the previous term's last slab has been read
      load(0);
      store(0, 0);
      __syncthreads();
      int buf = 0;
      for (int kc = 0; kc < n; kc += FTK) {
        const bool more = kc + FTK < n;
        if (more) load(kc + FTK);
        TT ah[2][2][2], bh[2][2][4];  // [fragment buffer][re / im][q]
        auto frag = [&](int kk, int fb) {
          const int kr = kk * 4 + (lane >> 4);
#pragma unroll
          for (int u = 0; u < NU; ++u) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
              ah[fb][u][q] = As[2 * buf + u][kr][(wm * 32 + q * 16 + (lane & 15)) ^ FbLds<TT>::swz(kr)];
#pragma unroll
            for (int q = 0; q < 4; ++q)
              bh[fb][u][q] = Bs[2 * buf + u][kr][(wn * 64 + q * 16 + (lane & 15)) ^ FbLds<TT>::swz(kr)];
          }
        };
        frag(0, 0);
#pragma unroll
        for (int kk = 0; kk < FTK / 4; ++kk) {
          const int cur = kk & 1;
          if (kk + 1 < FTK / 4) frag(kk + 1, cur ^ 1);
#pragma unroll
          for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
              for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma_t(ah[cur][u][bi], bh[cur][u][bj], acc[bi][bj]);
        }
        if (more) store(kc + FTK, buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
    };
    if (im) slabs(std::true_type{});
    else slabs(std::false_type{});
  }

  // ---- total, skew write-out ----
  __syncthreads();
  double* out = (split == 0 ? dG : dP + (long long)(split - 1) * R * nn) + (long long)mu * nn;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = wm * 32 + bi * 16 + acc_row<TT>(lane, r);
        const int lj = wn * 64 + bj * 16 + (lane & 15);
        const int gi = row0 + li, gj = col0 + lj;
        double v = 0.0;
        if (gi < n && gj < n) v = (double)acc[bi][bj][r];
        if (I == J) Tt[li][lj] = v;
        else if (gi < n && gj < n) {
          out[(long long)gi * n + gj] = v;
          out[(long long)gj * n + gi] = -v;
        }
      }
  if (I == J) {
    __syncthreads();
    for (int e = tid; e < FB_T * FB_T; e += 512) {
      const int li = e / FB_T, lj = e % FB_T;
      const int gi = row0 + li, gj = col0 + lj;
      if (gi < n && gj < n) out[(long long)gi * n + gj] = 0.5 * (Tt[li][lj] - Tt[lj][li]);
    }
  }
}

hipError_t set_force_lds_limit() {
  hipError_t e = hipFuncSetAttribute((const void*)k_force_big<double>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)force_big_lds_bytes<double>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_force_big<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)force_big_lds_bytes<float>());
}

// upper-triangle tiles of edge e that cover n, times the tile area
static long long force_area(int n, int e) {
  const long long t = (n + e - 1) / e;
  return t * (t + 1) / 2 * e * e;
}

// Built-in tile edge: 128 x 128 where measured faster (float64 at n = 1204:
// 64.7 instead of 69.2 ms; at n = 800 the 64 x 64 tiles win, 25.7 against
// 35.6 ms; float32 from n = 600: 68 -> ~50 ms at n = 1204)
int force_tile_default(int n, int mode) { return n >= (mode == FORCE_FP32 ? 600 : 1000) ? 128 : 64; }

hipError_t launch_force(int n, int R, const ForceTerm* terms, const double* coef, double* dG, double* dP,
                        unsigned long long* nrm, int mode, int nsplit, int tile, hipStream_t s) {
  const bool big = tile == 128;
  if (nsplit < 1 || nsplit > FORCE_SPLIT_MAX || nsplit > R) return hipErrorInvalidValue;
  const int per_xcd = (R + 7) / 8;
  if (mode == FORCE_FP32 && !big && force_area(n, FS_T) < force_area(n, 64)) {
    const int T = (n + FS_T - 1) / FS_T;
    const dim3 grid(8 * per_xcd * (T * (T + 1) / 2) * nsplit), block(FS_THREADS);
    hipLaunchKernelGGL((k_force_strip<float>), grid, block, 0, s, n, R, T, nsplit, terms, coef, dG, dP, nrm);
    return hipGetLastError();
  }
  if (big) {
    const int T = (n + FB_T - 1) / FB_T;
    const dim3 grid(8 * per_xcd * (T * (T + 1) / 2) * nsplit), block(512);
    if (mode == FORCE_FP64)
      hipLaunchKernelGGL((k_force_big<double>), grid, block, force_big_lds_bytes<double>(), s, n, R, T, nsplit,
                         terms, coef, dG, dP, nrm);
    else
      hipLaunchKernelGGL((k_force_big<float>), grid, block, force_big_lds_bytes<float>(), s, n, R, T, nsplit,
                         terms, coef, dG, dP, nrm);
    return hipGetLastError();
  }
  const int T = (n + 63) / 64;
  const int ntri = T * (T + 1) / 2;
  const dim3 grid(8 * per_xcd * ntri * nsplit), block(256);
  if (mode == FORCE_FP64)
    hipLaunchKernelGGL((k_force<double, true>), grid, block, 0, s, n, R, T, nsplit, terms, coef, dG, dP, nrm);
  else
    hipLaunchKernelGGL((k_force<float, false>), grid, block, 0, s, n, R, T, nsplit, terms, coef, dG, dP, nrm);
  return hipGetLastError();
}

hipError_t launch_force_elem(int n, int R, const ForceTerm* terms, const double* coef, const double* A,
                             const int* impos, int M, int direct_y, double* dE, hipStream_t s) {
  const int T = (n + 63) / 64;
  hipLaunchKernelGGL(k_force_elem, dim3(T * (T + 1) / 2, R), dim3(512), 0, s, n, R, T, terms, coef, A, impos, M,
                     direct_y, dE);
  return hipGetLastError();
}

hipError_t launch_force_join(double* dG, const double* dP, const double* dE, int n, int R, int nsplit,
                             unsigned long long* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_force_join, dim3((n + 15) / 16, R), dim3(256), 0, s, dG, dP, dE, n, R, nsplit, nrm);
  return hipGetLastError();
}

}  // namespace sgs
