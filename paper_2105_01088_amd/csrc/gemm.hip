// Grouped GEMM on the CDNA4 matrix cores.
//
// One launch runs a whole table of independent jobs of arbitrary (M, N, K).
// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8), each with its own L2; the host assigns every job to one XCD, so all
// tiles of a job share the panels of A and B in that XCD's L2.  Workgroup b
// searches the jobs of XCD b % 8 for local tile b / 8.  Each workgroup computes
// a 64 x 64 output tile with 4 waves of 32 x 32 (2 x 2 MFMA blocks of
// 16 x 16); K advances in slabs of 16 staged through LDS, with the next slab
// prefetched into registers while the current one is multiplied.
//
// MFMA operand layout (v_mfma_{f64,f32}_16x16x4): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator register r of lane l
// holds C[row][l % 16] with row = 4 r + l / 16 for the f64 instruction and
// row = 4 (l / 16) + r for the f32 one (AccRow below; both measured on gfx950).
#include "sgs_internal.h"

namespace sgs {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dvec4 mfma(double a, double b, dvec4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fvec4 mfma(float a, float b, fvec4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct AccRow;
template <> struct AccRow<double> {
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct AccRow<float> {
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T> struct VecOf;
template <> struct VecOf<double> { typedef dvec4 type; };
template <> struct VecOf<float> { typedef fvec4 type; };

template <typename Job>
__device__ __forceinline__ int find_job(const Job* __restrict__ jobs, int lo, int hi, int tile) {
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int TK = 16;
constexpr int LDP = 64 + 1;  // LDS row pitch (elements), padded

// Iterative callers (the polar iteration) pass control words ctl, one per
// gate (a job's `gate` field, its state): the workgroups of a job of
// iteration `it` exit at once when ctl[gate] < it.  rchk (optional) holds the
// residuals measured on this iteration's inputs: if rchk[gate] is below thr,
// this iteration is the job's last one (ctl[gate] = it).  rmax (optional)
// receives max |D + 1| over each job's outputs (D square) in rmax[gate], as
// an ordered bit pattern.  ctl[0] is the last iteration of every job (the
// whole launch exits at once past it, before reading its job) and ctl[1]
// counts the gates not yet marked: the workgroup that marks the last one sets
// ctl[0].  Gates of marked jobs start at 2.
template <typename T, typename Job, bool CPLX, bool LATE_C = CPLX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm(const Job* __restrict__ jobs, XcdMap xm,
                                              int* __restrict__ ctl, int it,
                                              const unsigned long long* __restrict__ rchk, double thr,
                                              unsigned long long* __restrict__ rmax) {
  typedef typename VecOf<T>::type V4;
  constexpr int NP = CPLX ? 2 : 1;
  __shared__ T smem_ab[2 * NP * TK * LDP];  // As, Bs; reused by the mirrored write
  T(*As)[TK][LDP] = (T(*)[TK][LDP])smem_ab;
  T(*Bs)[TK][LDP] = (T(*)[TK][LDP])(smem_ab + NP * TK * LDP);

  if (ctl != nullptr && ctl[0] < it) return;
  const int x = blockIdx.x & 7;
  const int tile = blockIdx.x >> 3;
  if (xm.off[x] >= xm.off[x + 1]) return;
  // one load instead of a chain of dependent ones: for the short-K updates
  // the prologue's latency is a large part of the kernel
  const int jid = xm.map ? xm.map[blockIdx.x] : find_job(jobs, xm.off[x], xm.off[x + 1] - 1, tile);
  if (jid < 0) return;
  const Job J = jobs[jid];  // by value: the fields live in scalar registers
  if (ctl != nullptr) {
    const int g = J.gate;
    if (ctl[g] < it) return;
    if (rchk != nullptr && threadIdx.x == 0 && __longlong_as_double((long long)rchk[g]) < thr) {
      // exactly one workgroup of the job sees the old value above it
      if (atomicMin(ctl + g, it) > it && atomicSub(ctl + 1, 1) == 1) ctl[0] = it;
    }
  }
  const int mirror = J.mirror;
  const int ntile_job = mirror ? J.tiles_n * (J.tiles_n + 1) / 2 : J.tiles_n * ((J.M + 63) / 64);
  if (tile - J.tile_begin >= ntile_job) return;
  const SGS_GLOBAL T* __restrict__ A = as_global(J.A);
  const SGS_GLOBAL T* __restrict__ B = as_global(J.B);
  const int M = J.M, N = J.N, K = J.K;
  const int lda = J.lda, ldb = J.ldb;
  const int ta = J.ta, tb = J.tb;
  const long long aim = J.a_im, bim = J.b_im;
  const int t = tile - J.tile_begin;
  int ti, tj;
  if (mirror) {  // upper-triangular tile index -> (ti, tj), ti <= tj
    int tri = t;
    ti = 0;
    while (tri >= J.tiles_n - ti) { tri -= J.tiles_n - ti; ++ti; }
    tj = ti + tri;
  } else {
    ti = t / J.tiles_n;
    tj = t % J.tiles_n;
  }
  const int row0 = ti * 64;
  const int col0 = tj * 64;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;

  // C values of this lane's outputs.  For long K they are loaded before the
  // K loop: their latency hides behind it, and no load of C can wait on a
  // store of D (they may alias: in-place updates pass C == D).  Short-K
  // tables (the complex Pfaffian updates, the Gauss-Jordan updates) load them
  // after it, still before any store (every lane reads only the elements it
  // writes): the registers they would hold across the loop cost a wave per
  // SIMD.
  const T beta = J.beta;
  const SGS_GLOBAL T* __restrict__ C = as_global(J.C);
  const int ldc = J.ldc;
  const SGS_GLOBAL int* __restrict__ cperm = as_global(J.cperm);
  const long long cim = J.c_im;
  T cval[NP][2][2][4];
  if constexpr (!LATE_C) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm * 32 + bi * 16 + AccRow<T>::row(lane, r);
        const int col = col0 + wn * 32 + bj * 16 + (lane & 15);
        const bool ok = beta != T(0) && row < M && col < N;
        const long long co = !ok ? 0 : (cperm ? (long long)cperm[row] * ldc + cperm[col] : (long long)row * ldc + col);
#pragma unroll
        for (int p = 0; p < NP; ++p) cval[p][bi][bj][r] = ok ? C[co + p * cim] : T(0);
      }
  }

  V4 acc[NP][2][2];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[p][i][j] = V4{0, 0, 0, 0};

  T ra[NP][4], rb[NP][4];

  // index pattern of this thread's 4 A and 4 B elements inside a slab: a
  // thread holds one row (A) or column (B) of the tile at 4 consecutive k.
  // Row-major operands put 4 threads on one row (A: 128-byte row segments);
  // the others put a wave on 64 consecutive rows / columns of one k, so the
  // loads are row segments and the LDS stores below hit distinct banks.
  const int a_i = ta ? (tid & 63) : (tid >> 2);
  const int a_k = ta ? (tid >> 6) * 4 : (tid & 3) * 4;
  const int b_k = tb ? (tid & 3) * 4 : (tid >> 6) * 4;
  const int b_j = tb ? (tid >> 2) : (tid & 63);

  auto load = [&](int kc) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = row0 + a_i, gk = kc + a_k + r;
      const bool ok = gi < M && gk < K;
      const long long off = ta ? (long long)gk * lda + gi : (long long)gi * lda + gk;
#pragma unroll
      for (int p = 0; p < NP; ++p) ra[p][r] = ok ? A[off + p * aim] : T(0);
      const int gj = col0 + b_j, gk2 = kc + b_k + r;
      const bool okb = gj < N && gk2 < K;
      const long long offb = tb ? (long long)gj * ldb + gk2 : (long long)gk2 * ldb + gj;
#pragma unroll
      for (int p = 0; p < NP; ++p) rb[p][r] = okb ? B[offb + p * bim] : T(0);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        As[p][a_k + r][a_i] = ra[p][r];
        Bs[p][b_k + r][b_j] = rb[p][r];
      }
    }
  };

  load(0);
  for (int kc = 0; kc < K; kc += TK) {
    __syncthreads();
    store();
    __syncthreads();
    if (kc + TK < K) load(kc + TK);
#pragma unroll
    for (int kk = 0; kk < TK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      T a[NP][2], b[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          a[p][q] = As[p][kr][wm * 32 + q * 16 + (lane & 15)];
          b[p][q] = Bs[p][kr][wn * 32 + q * 16 + (lane & 15)];
        }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          if (CPLX) {
            acc[0][bi][bj] = mfma(a[0][bi], b[0][bj], acc[0][bi][bj]);
            acc[0][bi][bj] = mfma(-a[NP - 1][bi], b[NP - 1][bj], acc[0][bi][bj]);
            acc[NP - 1][bi][bj] = mfma(a[0][bi], b[NP - 1][bj], acc[NP - 1][bi][bj]);
            acc[NP - 1][bi][bj] = mfma(a[NP - 1][bi], b[0][bj], acc[NP - 1][bi][bj]);
          } else {
            acc[0][bi][bj] = mfma(a[0][bi], b[0][bj], acc[0][bi][bj]);
          }
        }
    }
  }

  if constexpr (LATE_C) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm * 32 + bi * 16 + AccRow<T>::row(lane, r);
        const int col = col0 + wn * 32 + bj * 16 + (lane & 15);
        const bool ok = beta != T(0) && row < M && col < N;
        const long long co = !ok ? 0 : (cperm ? (long long)cperm[row] * ldc + cperm[col] : (long long)row * ldc + col);
#pragma unroll
        for (int p = 0; p < NP; ++p) cval[p][bi][bj][r] = ok ? C[co + p * cim] : T(0);
      }
  }
  const T alpha = J.alpha, diag = J.diag;
  SGS_GLOBAL T* D = as_global(J.D);
  const int ldd = J.ldd;
  const long long dim = J.d_im;
  double rm = 0.0;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = row0 + wm * 32 + bi * 16 + AccRow<T>::row(lane, r);
        int col = col0 + wn * 32 + bj * 16 + (lane & 15);
        if (row < M && col < N) {
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            T v = alpha * acc[p][bi][bj][r] + beta * cval[p][bi][bj][r];
            if (p == 0 && row == col) v += diag;
            D[(long long)row * ldd + col + p * dim] = v;
            if (rmax != nullptr) rm = nan_max(rm, fabs((double)v + (row == col ? 1.0 : 0.0)));
          }
        }
      }
  if (mirror && ti != tj) {
    // mirrored block D[col][row] = mirror * D[row][col], transposed through
    // LDS in two halves of 32 output rows (32 x LDP fits in As + Bs)
    T(*Tt)[LDP] = (T(*)[LDP])smem_ab;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        __syncthreads();
        if (wn == h) {
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int li = wm * 32 + bi * 16 + AccRow<T>::row(lane, r);
                const int lj = bj * 16 + (lane & 15);  // within the half
                const int row = row0 + li, col = col0 + h * 32 + lj;
                T v = T(0);
                if (row < M && col < N) v = alpha * acc[p][bi][bj][r] + beta * cval[p][bi][bj][r];
                Tt[lj][li] = v;
              }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 64; e += 256) {
          const int r = e >> 6, c = e & 63;  // D row col0 + 32 h + r, column row0 + c
          const int row = col0 + h * 32 + r, col = row0 + c;
          if (row < N && col < M) D[(long long)row * ldd + col + p * dim] = T(mirror) * Tt[r][c];
        }
      }
  }
  if (rmax != nullptr) {
    __shared__ double red[256];
    red[threadIdx.x] = rm;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] = nan_max(red[threadIdx.x], red[threadIdx.x + off]);
      __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(rmax + J.gate, (unsigned long long)__double_as_longlong(red[0]));
  }
}

hipError_t launch_gemm(const GemmJob* jobs, const XcdMap& xm, bool cplx, hipStream_t s, int* ctl, int it,
                       const unsigned long long* rchk, double thr, unsigned long long* rmax) {
  if (xm.max_tiles <= 0) return hipSuccess;
  const dim3 grid(8 * xm.max_tiles);
  if (cplx)
    hipLaunchKernelGGL((k_gemm<double, GemmJob, true>), grid, dim3(256), 0, s, jobs, xm, ctl, it, rchk, thr, rmax);
  else
    hipLaunchKernelGGL((k_gemm<double, GemmJob, false>), grid, dim3(256), 0, s, jobs, xm, ctl, it, rchk, thr, rmax);
  return hipGetLastError();
}

hipError_t launch_gemm_late_c(const GemmJob* jobs, const XcdMap& xm, hipStream_t s) {
  if (xm.max_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm<double, GemmJob, false, true>), dim3(8 * xm.max_tiles), dim3(256), 0, s, jobs, xm,
                     (int*)nullptr, 0, (const unsigned long long*)nullptr, 0.0, (unsigned long long*)nullptr);
  return hipGetLastError();
}

hipError_t launch_gemm_f32(const GemmJobF* jobs, const XcdMap& xm, hipStream_t s) {
  if (xm.max_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm<float, GemmJobF, false>), dim3(8 * xm.max_tiles), dim3(256), 0, s, jobs, xm,
                     (int*)nullptr, 0, (const unsigned long long*)nullptr, 0.0, (unsigned long long*)nullptr);
  return hipGetLastError();
}

}  // namespace sgs
