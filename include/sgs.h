/*
 * sgs.h -- C ABI of the MI355X library for one imaginary-time step of the
 * superposition-of-Gaussians (SGS) variational method of Boutin & Bauer,
 * "Quantum impurity models using superpositions of fermionic Gaussian
 * states: practical methods and applications" (arXiv:2105.01088).
 *
 * The library computes, on one GPU and entirely in its own HIP kernels:
 *   - for every pair (a,b) of the R Gaussian states of the ansatz (Eq. Ansatz),
 *     the overlap G_ab = <phi_a|phi_b> as log-magnitude and phase in the
 *     reference gauge <phi_0|phi_mu> > 0 (Sec. II.B), the transition matrix
 *     Delta^{ba} (Eq. def-delta-matrix) and the Hamiltonian element
 *     h_ab = <phi_a|H|phi_b> by generalized Wick contraction (Sec. III.B);
 *   - the R x R generalized eigenproblem h lambda = E G lambda (Eq. eigLambda);
 *   - the covariance-matrix force of Eq. (EOM-Gamma3), the first-order step of
 *     Eq. (RKstep) and the return to a pure state through the canonical form of
 *     Eq. (CM-normal-form) (every lambda_j rescaled to unit modulus).
 *
 * Conventions.  n = 2N Majoranas c_0..c_{n-1}; mode j is
 * a_j = (c_{2j} + i c_{2j+1})/2.  A covariance matrix (Eq. CMdef) is a real
 * skew n x n matrix with Gamma^2 = -1, stored row-major in float64.
 * H = e0 + i sum_{k,l} A_kl c_k c_l + sum_q u_q c_{q0} c_{q1} c_{q2} c_{q3}
 * with A real skew (both index orders summed, Sec. II.A) and quartic words
 * q0 < q1 < q2 < q3 (u = 24 U_{q0 q1 q2 q3} for the antisymmetric U of Sec. II.A).
 * Complex numbers are interleaved (re, im) float64 pairs.
 *
 * Ownership.  The caller owns every buffer.  Device buffers (covariance
 * matrices, workspace, outputs) must stay valid until sgs_destroy; the context
 * keeps non-owning pointers to them.  Host arrays in sgs_problem are read
 * during sgs_init only.  The library never allocates device memory.
 *
 * Asynchrony.  Every call enqueues work on the stream given to sgs_init and
 * returns without waiting; device outputs are valid once that stream has
 * been synchronized.  Numerical failures found on the device (a singular pair
 * matrix, a non-positive Gram matrix, a purification that did not converge)
 * are recorded in a device status word that sgs_status reads.
 *
 * Errors.  Every int-returning call returns SGS_OK (0) or a negative code;
 * sgs_strerror gives a message.  Nothing aborts or throws across this ABI.
 */
#ifndef SGS_H
#define SGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGS_OK 0
#define SGS_EINVAL (-1)    /* bad argument: null pointer, size, index, option */
#define SGS_ENOTSKEW (-2)  /* an input covariance matrix is not skew-symmetric */
#define SGS_ENOTPURE (-3)  /* an input covariance matrix violates Gamma^2 = -1 */
#define SGS_EPARITY (-4)   /* an input state has odd parity (Pf Gamma != +1)  */
#define SGS_ESINGULAR (-5) /* Gamma_a + Gamma_b singular, or G not positive     */
#define SGS_ENOCONV (-6)   /* purification or eigen-solve did not converge      */
#define SGS_EHIP (-7)      /* a HIP runtime call failed                         */
#define SGS_ESTATE (-8)    /* call order: e.g. sgs_energy before any evaluation */
#define SGS_EWORKSPACE (-9)/* workspace smaller than sgs_workspace_bytes        */
#define SGS_ERANGE (-10)   /* exponential map: |c dtau [Gamma, dGamma]|_1 above */
                           /* 2^12 (or not finite) for some state             */
#define SGS_ESCRATCH (-11) /* sgs_rotate_noalloc: n above its fixed scratch    */

/* sgs_options.precision */
#define SGS_FP64 0          /* every stage in float64                          */
#define SGS_FP32_FORCE 1    /* the force's dense product (Eq. EOM-Gamma3) on   */
                            /* the float32 matrix cores (about 1e-7 relative, */
                            /* far below the O(dtau) error of the Euler step);*/
                            /* inverses, overlaps, Wick elements, eigen-solve */
                            /* stay float64, and the float64 purification     */
                            /* returns every step to the pure states.  (No    */
                            /* float32 inverse with float64 refinement: its   */
                            /* float64 residual alone costs what the float64  */
                            /* inverse does at the 2:1 float32:float64 matrix */
                            /* rate of this GPU.)                             */
/* sgs_options.weight: the scalar c_mu of Eq. (Bmu) (Sec. III.A) */
#define SGS_W_PRINTED 0     /* c_mu = 1 / (lambda_mu lambda~_mu^*)             */
#define SGS_W_UNIT 1        /* c_mu = lambda~_mu lambda_mu^* / |lambda~_mu lambda_mu| */

/* sgs_options.update: how a step moves the states (App. A) */
#define SGS_UPD_EULER 0     /* Eq. (RKstep) Gamma + dtau dGamma, then the polar */
                            /* factor (Eq. CM-normal-form with unit moduli)    */
#define SGS_UPD_EXP 1       /* Eq. (ExpStep) R Gamma R^T, R = exp(c dtau        */
                            /* [Gamma, dGamma]) with c = exp_coef: orthogonal, */
                            /* no purification; scaling and squaring with a   */
                            /* degree-17 Taylor polynomial (error < 2e-16)    */

/* sgs_observables kinds */
#define SGS_OBS_POLY 1      /* <psi| O |psi> for Majorana polynomials O        */
#define SGS_OBS_RENYI2 2    /* S_2 = -ln Tr rho_A^2, Eq. (S2_SGS)              */
#define SGS_OBS_VARIANCE 3  /* <H>, <H^2>, delta_H^2 of Eq. (residual)         */

/* Renyi-2 evaluation methods (SGS_OBS_RENYI2, optional third iarg) */
#define SGS_REN_AUTO 0   /* by subsystem size and conditioning               */
#define SGS_REN_BLOCK 1  /* block form of order 2 nA for every term          */
#define SGS_REN_SPLIT 2  /* split form wherever a block is invertible        */

typedef struct sgs_ctx sgs_ctx; /* opaque */

/* One impurity problem (Sec. II.A).  Host pointers, read by sgs_init only. */
typedef struct {
  int32_t N;             /* fermionic modes, n = 2N Majoranas, 1 <= N <= 2048  */
  int32_t R;             /* rank of the ansatz, 1 <= R <= 32                   */
  const double* A;       /* n*n row-major, real skew (checked)                 */
  int32_t nq;            /* number of quartic words, 0 <= nq <= 256            */
  const int32_t* q_idx;  /* nq*4 Majorana indices, each row strictly increasing*/
  const double* q_val;   /* nq coefficients u_q                                */
  double e0;             /* constant energy offset                             */
  /* Interaction words of m = 6 or 8 Majoranas (the weight-m terms of
   * Sec. III.C); all zero / NULL when there are none.  Word w is the
   * Hermitian term v_w i^((m/2) mod 2) c_w0 ... c_w(m-1) (i for m = 6, 1 for
   * m = 8); its transition value is i^(m/2) Pf(Delta[w]) (Sec. III.B) and it
   * adds Pfaffian cofactors of order m - 2 to the transition Fock matrix. */
  int32_t nw;            /* number of such words, 0 <= nw <= 256               */
  const int32_t* w_len;  /* nw lengths, each 6 or 8                            */
  const int32_t* w_idx;  /* sum of w_len Majorana indices, word after word,    */
                         /* each word strictly increasing                      */
  const double* w_val;   /* nw real coefficients v_w                           */
} sgs_problem;

/* One row of a tuning table (written by the project autotuner,
 * paper_2105_01088_amd/autotune.py, from measured step times): the row with
 * the smallest n_max >= n applies to a problem of n Majoranas.  A field <= 0
 * keeps the library's built-in choice for that n.  Choices change only
 * scheduling and blocking, never the arithmetic of a result beyond rounding
 * order. */
typedef struct {
  int32_t n_max;     /* largest n the row applies to                          */
  int32_t gj_super;  /* Gauss-Jordan super-panel width, a multiple of the     */
                     /* panel width, <= 256 (rank of the trailing updates)    */
  int32_t gj_first;  /* 1: the pairs (0, a), which feed the overlap phases,   */
                     /* are inverted before the other pairs start; 2: both    */
                     /* batches start together                                */
  int32_t pf_super;  /* Pfaffian: elimination steps per trailing update       */
                     /* (rank 2 pf_super), 1..32                              */
  int32_t force_split;  /* force products: workgroups per output tile, each */
                        /* summing a range of the terms, 1..4                */
  int32_t force_elem;   /* elementwise force terms: 1 beside the products on */
                        /* a second stream, 2 after them on the same stream  */
  int32_t force_tile;   /* force products: output tile edge, 64 or 128      */
  int32_t gj_defer;     /* Gauss-Jordan inner updates deferred to one update */
  /* per super-panel (each panel then first takes the earlier panels'       */
  /* updates of its own columns): 1 in neither batch of pairs, 2 in the     */
  /* pairs not involving state 0, 3 in both                                */
} sgs_tune;

typedef struct {
  int32_t precision;       /* SGS_FP64 (default) or SGS_FP32_FORCE            */
  int32_t weight;          /* SGS_W_PRINTED (default) or SGS_W_UNIT            */
  double g_rel_threshold;  /* canonical orthogonalization: eigenvectors of G   */
                           /* below this fraction of its largest eigenvalue are*/
                           /* dropped (default 1e-12)                          */
  double purify_tol;       /* purification: iterations stop once max|X^2 + 1|  */
                           /* < min(1e-8, sqrt(purify_tol)) (default 1e-12)    */
  int32_t purify_iters;    /* max Newton-Schulz polar iterations (default 24); */
                           /* not converging sets SGS_ENOCONV                  */
  int32_t streams;         /* independent problems run concurrently on up to  */
                           /* this many worker streams, each with its own     */
                           /* scratch (1..8, default 4).  A worker uses three */
                           /* HIP streams (its main stream, the phase chain,  */
                           /* the inverses of the pairs not involving state   */
                           /* 0); workers run truly concurrently only with as */
                           /* many hardware queues (HIP's GPU_MAX_HW_QUEUES,  */
                           /* default 4, set before the process starts HIP)   */
  int32_t update;          /* SGS_UPD_EULER (default) or SGS_UPD_EXP           */
  double exp_coef;         /* c of SGS_UPD_EXP, 0 < c <= 1e6 (default 1/4:    */
                           /* for a tangent dGamma [[Gamma, dGamma], Gamma] = */
                           /* 4 dGamma, so 1/4 makes the first-order term the */
                           /* Euler step; the value printed in App. A, 1/2,   */
                           /* takes a step of 2 dtau)                         */
  const sgs_tune* tune;    /* host, ntune rows sorted by n_max, read by        */
  int32_t ntune;           /* sgs_workspace_bytes / sgs_init; NULL / 0: the    */
                           /* built-in choices (default)                      */
  int32_t graph;           /* 1: sgs_step captures one step of every problem  */
                           /* into a HIP graph (again when dtau changes) and  */
                           /* launches it once per step: one launch per step  */
                           /* for the whole batch.  Results are identical.    */
                           /* The problems then share one worker stream       */
                           /* (streams is ignored); stage timing is not       */
                           /* recorded.  0 (default): kernels are enqueued    */
                           /* per step                                        */
} sgs_options;

/* Fill *opt with the defaults listed above. */
void sgs_default_options(sgs_options* opt);

/* Device workspace, in bytes, that sgs_init needs for these problems.
 * probs: nprob problems (host).  Returns SGS_OK or SGS_EINVAL. */
int sgs_workspace_bytes(const sgs_problem* probs, int32_t nprob,
                        const sgs_options* opt, size_t* bytes);

/* Create a context.
 *   probs, nprob : the problems (host, read now; 1 <= nprob <= 1024)
 *   gamma        : device float64 buffer holding, problem after problem and
 *                  state after state, the R_p covariance matrices (n_p*n_p
 *                  row-major each): sum_p R_p n_p^2 doubles.  Read by every
 *                  evaluation and overwritten in place by sgs_step.  Each
 *                  matrix must be skew (|Gamma + Gamma^T| <= 1e-12), pure
 *                  (|Gamma^2 + 1| <= 1e-10) and of even parity (Pf Gamma =
 *                  +1, as for every state generated from the vacuum by
 *                  SO(2N); the overlap phases of Sec. II.B are taken for
 *                  those), all checked here, synchronously; a NaN fails the
 *                  first check that meets it.
 *   workspace    : device buffer of at least sgs_workspace_bytes, 256-byte
 *                  aligned, owned by the caller.
 *   opt          : NULL for defaults.
 *   stream       : hipStream_t to enqueue on (NULL = the default stream).
 * On success *out holds the context.  Errors: SGS_EINVAL, SGS_ENOTSKEW,
 * SGS_ENOTPURE, SGS_EPARITY, SGS_EWORKSPACE, SGS_EHIP. */
int sgs_init(sgs_ctx** out, const sgs_problem* probs, int32_t nprob,
             double* gamma, void* workspace, size_t ws_bytes,
             const sgs_options* opt, void* stream);

/* Overlaps and Hamiltonian elements of every pair, for the current states
 * (Secs. II.B, II.C, III.B).  Device outputs, problem after problem, R_p*R_p
 * entries each, row-major in (a, b):
 *   log_abs_G[a*R+b] = ln|<phi_a|phi_b>|       (0 on the diagonal)
 *   arg_G[a*R+b]     = arg <phi_a|phi_b>       (gauge <phi_0|phi_mu> > 0)
 *   eps[2*(a*R+b)+{0,1}] = h_ab / G_ab         (complex, interleaved)
 * and, problem after problem, for its P_p = R_p (R_p - 1) / 2 pairs a < b in
 * the order (0,1), (0,2), ..., (0,R-1), (1,2), ..., the transition matrix of
 * Eq. (def-delta-matrix)
 *   delta[2*(p*n*n + k*n + l) + {0,1}] = Delta^{ba}_kl
 *          = [(i (Gamma_b - Gamma_a) - 2) (Gamma_a + Gamma_b)^{-1}]_kl
 *   (complex interleaved, n_p x n_p row-major; <phi_a| c_k c_l |phi_b> =
 *   i G_ab Delta^{ba}_kl for k != l; Delta^{ab} is its complex conjugate).
 * Any output may be NULL.  Errors: SGS_EINVAL, SGS_EHIP. */
int sgs_pair_eval(sgs_ctx* ctx, double* log_abs_G, double* arg_G, double* eps, double* delta);

/* Advance every problem by nsteps imaginary-time steps of size dtau
 * (Sec. III.C, App. A).  energies (device, may be NULL): nsteps*nprob
 * doubles, energies[k*nprob+p] = E of the states entering step k of problem p
 * (lowest root of Eq. eigLambda).  gamma is overwritten with the new states.
 * Errors: SGS_EINVAL. */
int sgs_step(sgs_ctx* ctx, double dtau, int32_t nsteps, double* energies);

/* Energy and amplitudes of the current states (Eq. eigLambda).
 *   E      : device, nprob doubles
 *   lambda : device complex (interleaved), sum_p R_p entries, or NULL;
 *            normalized lambda^dag G lambda = 1, global phase arbitrary.
 * Errors: SGS_EINVAL. */
int sgs_energy(sgs_ctx* ctx, double* E, double* lambda);

/* Observables of the current SGS state of one problem (the states in gamma
 * now; tables are re-evaluated when the states changed since the last
 * evaluation).  iargs and dargs are host arrays, read before return.
 *   SGS_OBS_POLY  : expectation values <psi|O_t|psi> of npoly Majorana
 *                   polynomials (Sec. IV.B, Eq. Cr, uses this for S(0).S(r)).
 *                   iargs = {problem, npoly, nterm, then nterm rows of
 *                   (poly_index, m, k0, k1, k2, k3)} with m in {0, 2, 4}
 *                   distinct increasing Majorana indices (unused = -1);
 *                   dargs = 2*nterm doubles, complex coefficients;
 *                   out (device) = 2*npoly doubles, complex results.
 *                   Limits: npoly <= 4096, nterm <= 16384.  Waits for the
 *                   stream before returning.
 *   SGS_OBS_RENYI2: iargs = {problem, nA} or {problem, nA, method} with nA
 *                   even, 2 <= nA <= min(n, 1024), the subsystem being
 *                   Majoranas 0..nA-1; dargs unused; out (device) =
 *                   1 double, S_2 = -ln Tr rho_A^2 (Eq. S2_SGS, App. B).
 *                   Only one term per orbit of the rank-4 tensor's two
 *                   symmetries (exchange of the pairs, complex
 *                   conjugation) is evaluated, about R^4 / 4 Pfaffians.
 *                   method: SGS_REN_AUTO (default): block form of
 *                   Eq. (pfMA), order 2 nA, in on-chip memory for
 *                   nA <= 32; above that the split form of
 *                   Eq. (TrArho2_final), Pf(K_q) Pf(K_p - K_q^{-1}) of
 *                   order nA, inverting the better-conditioned block, and
 *                   the block form for terms whose blocks both have a
 *                   1-norm condition number above 1e6.  SGS_REN_BLOCK:
 *                   block form for every term (batched).  SGS_REN_SPLIT:
 *                   split form wherever a block is invertible.
 *                   Above nA = 32 the call allocates device memory (kept
 *                   by the context, up to about 2 GiB plus
 *                   R (R + 1) nA^2 16 bytes) and waits for the stream.
 *   SGS_OBS_VARIANCE: iargs = {problem}; dargs unused; out (device) =
 *                   3 doubles {<H>, <H^2>, delta_H^2 = <H^2> - <H>^2} of the
 *                   problem's Hamiltonian (Eq. residual, Sec. IV.A), by
 *                   Wick's theorem on every transition operator: the
 *                   quadratic part in matrix form (O(n^2 nnz(A)/n) per pair
 *                   of states), products with quartic words as Pfaffians of
 *                   6 and 8 Majoranas.  R <= 32; not available for a
 *                   problem with words of more than 4 Majoranas (nw > 0).
 * Errors: SGS_EINVAL (kind, sizes, indices), SGS_EHIP. */
int sgs_observables(sgs_ctx* ctx, int32_t kind, const int32_t* iargs,
                    int32_t niargs, const double* dargs, int32_t ndargs,
                    double* out);

/* Rank growing (Sec. III.C): the state added to the ansatz is a random
 * special orthogonal transformation Q, close to the identity, of a state of
 * high amplitude.  gamma_out = Q gamma Q^T, made exactly skew.
 *   Q, gamma  : device, n x n float64, row-major (Q orthogonal, gamma a pure
 *               covariance matrix; neither is checked)
 *   work      : device, n*n float64 scratch owned by the caller
 *   gamma_out : device, n x n; must not overlap gamma or work
 *   stream    : hipStream_t the work is enqueued on (NULL: the null stream);
 *               returns without waiting.
 * Needs no context.  Errors: SGS_EINVAL (null pointer, n odd or outside
 * 2..8192), SGS_EHIP. */
int sgs_rotate(const double* Q, const double* gamma, double* work, double* gamma_out, int32_t n,
               void* stream);

/* sgs_rotate without a work buffer, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and result as sgs_rotate; the n x n intermediate
 * lives in a fixed scratch array of the library (18 MiB per device, held from
 * the first call on a device until the process ends), so n <= 1536.  No
 * allocation of any kind is made.  Every call on one device shares that
 * scratch: calls that overlap on a device (different streams, or threads
 * without ordering) race and must be serialized by the caller.
 * Errors: SGS_EINVAL (null pointer, n odd or < 2), SGS_ESCRATCH (n > 1536),
 * SGS_EHIP. */
int sgs_rotate_noalloc(const double* Q, const double* gamma, double* gamma_out, int32_t n, void* stream);

/* Wait for the context's stream and return the device status word:
 * SGS_OK, SGS_ESINGULAR, SGS_ENOCONV or SGS_ERANGE (first failure since the last call;
 * reading it clears it), or SGS_EHIP. */
int sgs_status(sgs_ctx* ctx);

/* Diagnostics: device time per stage of the step.  After sgs_set_timing(ctx, 1)
 * every later evaluation records a pair of HIP events on the context's stream
 * around each stage (no device memory is allocated; events are pooled).
 * sgs_stage_times waits for the stream, adds the elapsed times recorded since
 * the previous call into ms[s] (milliseconds) and launches[s] (number of
 * timed intervals; for SGS_STAGE_FORCE and SGS_STAGE_SOLVE one kernel
 * launch each) for s < nstage, and clears the record.  Errors: SGS_EINVAL,
 * SGS_EHIP. */
#define SGS_STAGE_INVERSE 0   /* Gamma_a + Gamma_b, blocked Gauss-Jordan        */
#define SGS_STAGE_DELTA 1     /* Im Delta^{ba} = 2 Gamma_b W - 1 (GEMM)          */
#define SGS_STAGE_WICK 2      /* eps_ab, Fock blocks, Y = Delta F               */
#define SGS_STAGE_PHASE 3     /* X_a and C_ab for the overlap phases            */
#define SGS_STAGE_PFAFFIAN 4  /* complex Pfaffians of C_ab                       */
#define SGS_STAGE_SOLVE 5     /* h lambda = E G lambda, weights, coefficients   */
#define SGS_STAGE_FORCE 6     /* Eq. (EOM-Gamma3) accumulation                   */
#define SGS_STAGE_PURIFY 7    /* Euler step and polar purification, or the      */
                              /* exponential map                                 */
#define SGS_NSTAGE 8
int sgs_set_timing(sgs_ctx* ctx, int32_t enable);
int sgs_stage_times(sgs_ctx* ctx, double* ms, int32_t* launches, int32_t nstage);

/* Release host-side state.  Device buffers stay owned by the caller. */
void sgs_destroy(sgs_ctx* ctx);

/* Static message for an error code. */
const char* sgs_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SGS_H */
