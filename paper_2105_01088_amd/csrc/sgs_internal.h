// Internal declarations shared by the HIP kernels and the host driver of the
// SGS library.  Not part of the public ABI (include/sgs.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgs {

// ---------------------------------------------------------------------------
// Grouped GEMM: D = alpha * op(A) op(B) + beta * C (+ diag on the diagonal)
// for a table of independent jobs of any size, one launch for all of them.
// op(A) is M x K: ta = 0 reads A[i*lda + k], ta = 1 reads A[k*lda + i].
// op(B) is K x N: tb = 0 reads B[k*ldb + j], tb = 1 reads B[j*ldb + k].
// Complex jobs are planar: the imaginary plane of X sits at X + x_im.
// ---------------------------------------------------------------------------
struct GemmJob {
  const double* A;
  const double* B;
  const double* C;  // may be null when beta == 0
  double* D;
  long long a_im, b_im, c_im, d_im;  // complex: offsets of imaginary planes
  int M, N, K;
  int lda, ldb, ldc, ldd;
  int ta, tb;
  double alpha, beta, diag;
  int tiles_n;     // ceil(N / 64)
  int tile_begin;  // first global tile index of this job
  const int* cperm;  // optional: C element (i, j) read at (cperm[i], cperm[j])
  int mirror;        // 0, or +1 / -1: D (square) is symmetric / skew; only
                     // tiles I <= J run and write the mirrored block too
  int gate;          // iterative callers: index of this job's control word
                     // and residual slots (the job's state)
};

// float32 twin used by the precision path (same layout, float operands).
struct GemmJobF {
  const float* A;
  const float* B;
  const float* C;
  float* D;
  long long a_im, b_im, c_im, d_im;
  int M, N, K;
  int lda, ldb, ldc, ldd;
  int ta, tb;
  float alpha, beta, diag;
  int tiles_n;
  int tile_begin;
  const int* cperm;
  int mirror;
  int gate;
};

constexpr int GEMM_TILE = 64;

// Pointers read from device-side tables are generic (flat) to the compiler;
// flat loads also count against the LDS wait counter, which serializes them
// with the LDS traffic of a K loop.  Kernels cast such pointers to the global
// address space.
#define SGS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const SGS_GLOBAL T* as_global(const T* p) {
  return (const SGS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ SGS_GLOBAL T* as_global(T* p) {
  return (SGS_GLOBAL T*)p;
}

// Maximum that keeps NaN (fmax drops it): a residual or norm over data with a
// NaN must not look small.  With values >= 0 or NaN (a positive quiet NaN)
// the unsigned order of the bit patterns agrees, so atomicMax on them keeps
// NaN as well.
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || b != b) ? __builtin_nan("") : (a > b ? a : b);
}

// Jobs of XCD x occupy table entries [off[x], off[x+1]); their tile_begin
// counts tiles within that XCD; max_tiles = largest per-XCD tile count.
// map (optional, device): the job of every workgroup b (tile b / 8 of XCD
// b % 8), -1 for none; without it the job is found by binary search.
struct XcdMap {
  int off[9];
  int max_tiles;
  const int* map;
};

// Launch helpers (gemm.hip).  jobs: device table ordered by XCD.
hipError_t launch_gemm(const GemmJob* jobs, const XcdMap& xm, bool cplx,
                       hipStream_t s, int* ctl = nullptr, int it = 0,
                       const unsigned long long* rchk = nullptr, double thr = 0.0,
                       unsigned long long* rmax = nullptr);
// real jobs with short K (C loaded after the K loop; may be in place)
hipError_t launch_gemm_late_c(const GemmJob* jobs, const XcdMap& xm, hipStream_t s);
hipError_t launch_gemm_f32(const GemmJobF* jobs, const XcdMap& xm, hipStream_t s);

// ---------------------------------------------------------------------------
// Status word (device int): first failure wins.
// ---------------------------------------------------------------------------
enum : int { ST_OK = 0, ST_SINGULAR = -5, ST_NOCONV = -6, ST_RANGE = -10 };

// ---------------------------------------------------------------------------
// Force accumulation: one output state mu, R descriptors (one per beta).
// ---------------------------------------------------------------------------
struct ForceTerm {
  const double* Dr;   // real part source: W (scaled by dr_scale) or Gamma_mu
  const double* Di;   // imaginary part of Delta (null on the diagonal)
  const double* Yr;   // Delta F, real plane
  const double* Yi;   // Delta F, imaginary plane (null on the diagonal)
  const double* Fci;  // impurity-block Fock correction, imaginary (M*M) or null
  const double* Fcr;  // impurity-block Fock correction, real (M*M)
  double dr_scale;    // -2 (pair) or 1 (diagonal)
  double sgn;         // +1: stored orientation; -1: complex conjugate
  int coef;           // index into the (R x R) coefficient tables
  int pad;
};


// Hamiltonian tables on the device (pair.hip)
struct HamDev {
  int n, nnz_up, nq, M;
  const int* up_k;     // upper-triangle nonzeros of A: (k < l, A_kl)
  const int* up_l;
  const double* up_v;
  const int* q_idx;    // nq x 4 global Majorana indices
  const int* q_loc;    // nq x 4 positions in the impurity list
  const double* q_val;
  double e0;
  // words of 6 or 8 Majoranas: nw x 8 indices (padded), lengths, v_w; the
  // impurity entries (r < c) they touch with the ranges of their
  // (word, a, b) cofactor items
  int nw;
  const int* w_idx;
  const int* w_len;
  const double* w_val;
  int nfe;
  const int2* fe_ent;
  const int* fe_off;
  const int4* fe_item;
};

// A in compressed-column form plus the impurity index maps (pair.hip)
struct SparseA {
  const int* colptr;  // n + 1
  const int* row;
  const double* val;
  const int* imp;     // M impurity Majoranas
  const int* impos;   // n: position in imp, or -1
  int M;
};

// Arguments of the amplitude solve (solve.hip)
struct SolveArgs {
  int N, R, P;
  const int* pidx;      // R*R: pair index of (min, max), -1 on the diagonal
  const int* qidx;      // R*R: phase-matrix index for 1 <= a < b, else -1
  const double* logdet; // P
  const double* pfacc;  // Q*3: ln|Pf|, cos, sin
  const double* eps;    // (P + R) complex: pairs then diagonal
  double* tab_la;       // R*R outputs
  double* tab_arg;
  double* tab_eps;      // R*R complex
  double* Gt;           // R*R complex
  double* ht;           // R*R complex
  double* lam;          // R complex
  double* lamt;         // R complex
  double* coef;         // c1 (R*R complex) then c2 (R*R complex)
  double* E;            // 1
  double* energy_slot;  // optional: energies[k * nprob + p]
  const int* slot_ctr;  // optional: energy_slot is advanced by *slot_ctr * slot_stride
  int slot_stride;
  int* status;
  double g_thr;
  int weight;           // 0 printed, 1 unit
};

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
struct GjPanelShape {
  int B, rpt, nt;
};
GjPanelShape gj_panel_shape(int n);
size_t gj_panel_lds_bytes(int n, int kl, int b);
// Super-panel [bc0, bc1) of panels nbp wide: E_all (n x (bc1 - bc0), leading
// dimension eld) and Brow_all ((bc1 - bc0) x (bc1 - bc0), leading dimension
// brld) per matrix; the panel at k writes its columns of E_all and its rows
// of Brow_all (k - bc0 onward)
hipError_t launch_gj_panel(double* M, long long mstride, int nmat, int n, int k, int b,
                           double* E, long long estride, int eld, double* Br, long long bstride, int brld,
                           int bc0, int bc1, int nbp, int defer, int* piv, int* src, double* logdet,
                           int* status, hipStream_t s);
// super-panel [k0, k0 + nb) done: Br = its pivot rows (nb x n, zero on the
// super-panel), which are then cleared outside it
hipError_t launch_gj_gather(double* M, long long mstride, int nmat, int n, int k0, int nb, const int* piv,
                            double* Br, long long bstride, hipStream_t s);
hipError_t launch_gj_unscramble(const double* M, double* W, long long mstride, int nmat, int n, const int* piv,
                                const int* src, hipStream_t s);
hipError_t set_gj_lds_limit(size_t bytes);
struct PfPanelShape {
  int nbh, rpt, nt, ns;
};
PfPanelShape pf_panel_shape(int m);
size_t pf_panel_lds_bytes(int m, int nbh);
// one panel of ns steps at logical positions p0, p0 + 2, ... of the
// super-panel (kall <= 32 steps in all, kd before this panel) of the stored
// m0 x m0 matrix A; D: the super-panel's deferred columns (dstride >= 128 m0
// doubles per matrix, row-major [row][t][U re, U im, V re, V im]); last:
// write the trailing GEMM operands L, RM and perm (entries >= p0 + 2 ns)
hipError_t launch_pf_panel(const double* A, long long astride, long long plane, int ld, int m0, int p0, int ns,
                           int kd, int kall, int first, int last, int nmat, double* D, long long dstride, double* L,
                           double* RM, long long lstride, long long l_im, int* perm, int pstride, double* acc,
                           int first_acc, int* status, hipStream_t s);
hipError_t launch_pair_sum(const double* gam, int n, const int* pa, const int* pb, int P, double* S,
                           double* logdet, hipStream_t s);
hipError_t launch_eps_fock(const HamDev& h, int P, int R, const double* W, const double* Di,
                           const double* gam, const int* pa, const int* pb, double* eps, double* Fc,
                           hipStream_t s);
hipError_t launch_apply_fock(const SparseA& sa, int n, int P, int R, const double* W, const double* Di,
                             const double* gam, const double* Fc, double* Y, double* Yd, hipStream_t s);
// dense A: adds the impurity-block Fock correction into Y = Delta A, Yd = Gamma A
hipError_t launch_fock_imp(const SparseA& sa, int n, int P, int R, const double* W, const double* Di,
                           const double* gam, const double* Fc, double* Y, double* Yd, hipStream_t s);
// out (complex interleaved) = -2 W + i Di over total elements
hipError_t launch_delta_out(const double* W, const double* Di, long long total, double* out, hipStream_t s);
hipError_t launch_build_c(int n, const double* gam, const double* T, const double* Xr, const int* qa,
                          const int* qb, int Q, double* Cm, hipStream_t s);
size_t solve_lds_bytes(int R);
hipError_t launch_solve(const SolveArgs& a, hipStream_t s);
// *ctr = v / *ctr += 1 (one thread), for the step counter of a replayed graph
hipError_t launch_set_counter(int* ctr, int v, hipStream_t s);
hipError_t launch_bump_counter(int* ctr, hipStream_t s);
hipError_t set_solve_lds_limit(size_t bytes);
// Observables (obs.hip): the current tables of one problem.
struct ObsState {
  int n, R;
  const double* gam;  // R covariance matrices
  const double* W;    // per pair: (Gamma_a + Gamma_b)^{-1}
  const double* Di;   // per pair: Im Delta^{ba}
  const double* lam;  // R complex amplitudes
  const double* Gt;   // R x R complex overlaps
  const int* pidx;    // R x R pair index
};
// Gamma' = Q Gamma Q^T, exactly skew (rotate.hip); work: n*n doubles
hipError_t launch_rotate(const double* Q, const double* G, double* work, double* out, int n, hipStream_t s);
// the allocation-free variant's scratch (rotate.hip): n <= ROTATE_SCRATCH_N,
// address on the current device (looked up once per device)
constexpr int ROTATE_SCRATCH_N = 1536;
hipError_t rotate_scratch(double** out);

// Hamiltonian tables for the variance of H (obs.hip): dense A, its upper
// nonzeros, its compressed columns, the quartic words
struct VarHam {
  const double* Ad;
  int nnz_up;
  const int* up_k;
  const int* up_l;
  const double* up_v;
  const int* colptr;
  const int* rowidx;
  const double* colval;
  int nq;
  const int* q_idx;
  const double* q_val;
};
constexpr int VAR_CHUNKS = 16;  // workgroups per transition block
// a2 = |A|_F^2
hipError_t launch_variance(const ObsState& s, const VarHam& h, double e0, double a2, double* part, double* out,
                           hipStream_t st);
constexpr int OBS_MAX_TERMS = 16384;
constexpr int OBS_MAX_POLY = 4096;
hipError_t launch_obs_poly(const ObsState& s, const int* rows, const double* coef, const int* off, int npoly,
                           double* out, hipStream_t st);
// Renyi-2 (renyi.hip): one representative term of the rank-4 tensor, the
// ordered pairs p = a R + b, q = g R + d and the orbit size w; the split form
// inverts block q
struct RenTerm {
  int p, q, split, w;
};
constexpr int REN_LDS_MAX_NA = 32;  // block form in LDS (order 2 nA <= 64)
constexpr int REN_MAX_NA = 1024;    // batched path (block form of order <= 2048)
size_t ren_lds_bytes(int nA);
hipError_t set_ren_lds_limit();
hipError_t launch_ren_lds(const ObsState& s, int nA, const RenTerm* terms, int nterm, double* tval, hipStream_t st);
hipError_t launch_ren_blocks(const ObsState& s, int nA, const int2* uxy, int u0, int nb, int nu, double* dst,
                             double* inv, hipStream_t st);
hipError_t launch_ren_inverse(double* K, int nu, int m, double* kappa, hipStream_t st);
hipError_t launch_ren_terms(const ObsState& s, int nA, int split, const RenTerm* terms, int t0, int count, int nb,
                            const double* inv, double* dst, hipStream_t st);
hipError_t launch_ren_combine(const ObsState& s, int nA, int split, const RenTerm* terms, int t0, int count,
                              const double* acc, const double* uacc, double* tval, hipStream_t st);
hipError_t launch_ren_sum(const double* tval, int nterm, double* out, hipStream_t st);

enum : int { FORCE_FP64 = 0, FORCE_FP32 = 1 };
// k_force: the dense products, nsplit workgroups per output tile, each
// summing one range of the terms b: range 0 into dG, range h > 0 into slice
// h - 1 of dP ((FORCE_SPLIT_MAX - 1) R n^2 float64; clears nrm); k_force_elem:
// the elementwise terms into dE; k_force_join: dG += (the dP slices) + dE and
// the 1-norms.
constexpr int FORCE_SPLIT_MAX = 4;
hipError_t set_force_lds_limit();  // the 128 x 128 tile kernels' LDS (once per context)
int force_tile_default(int n, int mode);  // 64 or 128
// whether k_force_elem adds Re(c1 i Y): every product but the FP64 64 x 64
// one (whose tiles are k_force_elem's, so the fold into its B operand stays
// exact under the skew completion)
inline bool force_direct_y(int mode, int tile) { return mode != FORCE_FP64 || tile == 128; }
// tile: output tile edge, 64 or 128
hipError_t launch_force(int n, int R, const ForceTerm* terms, const double* coef, double* dG, double* dP,
                        unsigned long long* nrm, int mode, int nsplit, int tile, hipStream_t s);
// direct_y = 0: the products carry Re(c1 i Y) (FP64 64 x 64 tiles: B =
// c1 (D + i 1)) and k_force_elem leaves it out; any other product adds it
// here (force_direct_y)
hipError_t launch_force_elem(int n, int R, const ForceTerm* terms, const double* coef, const double* A,
                             const int* impos, int M, int direct_y, double* dE, hipStream_t s);
hipError_t launch_force_join(double* dG, const double* dP, const double* dE, int n, int R, int nsplit,
                             unsigned long long* nrm, hipStream_t s);
hipError_t launch_euler(const double* gam, const double* dG, double dtau, int n, int R, double* X,
                        int* ctl, unsigned long long* resid, int nresid, unsigned long long* nrm,
                        hipStream_t s);
hipError_t launch_ns_resid(const double* Q, int n, long long total, unsigned long long* out, hipStream_t s);
// Taylor coefficients of the even and odd parts of exp: c[j] = 1 / (2j)!,
// s[j] = 1 / (2j + 1)!, j = 0..8.
struct ExpCoef {
  double c[9];
  double s[9];
};
constexpr int EXP_SMAX = 12;  // squarings: |c ds [Gamma, dGamma]|_1 <= 2^12
hipError_t launch_exp_gen(const double* P, int n, int R, double cds, double* K, double* rowsum, int smax,
                          int* ctl, double* par, int* status, hipStream_t s);
hipError_t launch_exp_b3(const double* Y, const double* Z, int n, int R, const ExpCoef& cf, double* E0, double* E1,
                         hipStream_t s);
hipError_t launch_exp_skew_diag(double* D, int n, int R, hipStream_t s);
hipError_t launch_exp_pick(double* X0, const double* X1, int n, int R, const int* ctl, hipStream_t s);
hipError_t launch_finalize(const double* X0, const double* X1, int n, int R, double* gam, const int* ctl,
                           int maxit, int* status, hipStream_t s);
hipError_t launch_skew_resid(const double* G, int n, long long total, unsigned long long* out,
                             hipStream_t s);
// sign of Pf(Gamma_mu) for R matrices (out: +1, -1, or 0 if singular), working
// on copies in S (R n^2 doubles); one workgroup per matrix
hipError_t launch_pf_sign(const double* G, double* S, int n, int R, double* out, hipStream_t s);
hipError_t set_pf_sign_lds_limit(int n);

}  // namespace sgs
