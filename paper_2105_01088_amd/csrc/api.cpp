// Host side of the C ABI declared in include/sgs.h: validation, workspace
// layout (the caller's buffer is carved up; nothing is allocated), the static
// tables every step reuses (pair lists, sparse A, GEMM job tables, force
// descriptors), and the order of the device stages of one imaginary-time step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "sgs_internal.h"
#include "../../include/sgs.h"

using namespace sgs;

namespace {

constexpr int GJ_NB_MAX = 32;   // Gauss-Jordan panel width
constexpr int GJ_SUPER_MAX = 256;  // Gauss-Jordan super-panel width (rank of the trailing updates), at most
constexpr int PF_SUPER_MAX = 32;  // Pfaffian steps per trailing update (rank 2 x this), at most

struct Arena {
  char* base;
  size_t off;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct JobTable {
  GemmJob* dev = nullptr;
  int* dmap = nullptr;  // workgroup -> job
  int map_cap = 0;
  std::vector<GemmJob> host;
  int ntiles = 0;
  bool cplx = false;
  bool late_c = false;  // real, short K: the C tile is loaded after the K loop
  XcdMap xm{};
};

// Batched Pfaffians of B complex skew matrices of order m, planar (matrix b
// at A0 + 2 m^2 b, imaginary plane at + m^2, leading dimension m).  Blocked
// on two levels (register panels inside super-panels of `super` steps, then
// one trailing complex GEMM per super-panel); the trailing matrices ping-pong
// between A0 and A1, so A0 does not survive a run.
struct PfBatch {
  int m = 0, B = 0, super = PF_SUPER_MAX;
  double *A0 = nullptr, *A1 = nullptr, *UV = nullptr, *RM = nullptr, *PD = nullptr;
  int* perm = nullptr;
  long long uvstride = 0, uv_im = 0, pdstride = 0;
  struct Panel { int sp, p0, ns, kd; };
  std::vector<int> sm, sk;   // super-panels: stored order, steps
  std::vector<Panel> pan;    // register panels of every super-panel
  std::vector<JobTable> jt;  // trailing update of each super-panel
};

struct Prob {
  int N = 0, n = 0, R = 0, P = 0, Q = 0, M = 0, nq = 0, nnz_up = 0, nnz = 0;
  int nw = 0, nfe = 0, nfi = 0;  // higher words, Fock entries they touch, (word, a, b) items
  int gj_nb = 16;
  int gj_super = 128;  // super-panel width (a multiple of gj_nb)
  bool gj_first = false;  // pairs (0, a) inverted before the others start
  // deferred Gauss-Jordan inner updates: 1 neither batch, 2 the pairs
  // (a >= 1, b), 3 both.  Measured at n = 400, 800, 1204 (ms per step):
  // 5.72 / 5.82 / 6.06, 92.7 / 93.3 / 93.7, 185.9 / 185.7 / 186.5: the
  // shorter inverse and Pfaffian chains do not shorten the step (the extra
  // launch before every panel lengthens the chain the others wait on), so
  // the built-in choice applies every panel's update at once
  int gj_defer = 1;
  int force_split = 2;    // workgroups per force output tile (term ranges; set by pick_tuning)
  int force_tile = 0;     // force output tile edge (64 or 128; 0: by size and precision)
  bool force_seq = false;  // elementwise force terms after the products, same stream
  int worker = 0;  // stream (and scratch region) this problem runs on
  bool expmap = false;  // exponential-map update instead of Euler + purification
  bool denseA = false;  // A has many nonzeros per column: Y = Delta A by GEMM
  double e0 = 0.0;
  double a2 = 0.0;  // |A|_F^2
  double* gam = nullptr;
  // dense work
  double *W, *Di, *Y, *Yd, *T1, *Xr, *gjE, *gjB, *dG, *dP, *dE, *nsX0, *nsX1, *nsQ, *Adense;
  // small
  double *pfacc, *logdet, *eps, *Fc, *coef, *Gt, *ht, *lam, *lamt, *E, *tab_la, *tab_arg, *tab_eps;
  double *up_v, *colval, *q_val;
  int *piv, *pa, *pb, *qa, *qb, *pidx, *qidx, *up_k, *up_l, *colptr, *rowidx, *imp, *impos, *q_idx, *q_loc;
  // higher words: 8 indices (padded), lengths and v per word; per touched
  // impurity entry (r < c) the range of its (word, a, b) cofactor items
  int *w_idx = nullptr, *w_len = nullptr, *fe_off = nullptr;
  int2* fe_ent = nullptr;
  int4* fe_item = nullptr;
  double* w_val = nullptr;
  unsigned long long* resid;
  unsigned long long* nsres;
  unsigned long long* dgnorm;
  int* nsctl;
  ForceTerm* terms;
  JobTable jdi, jt1, jxr, jnsq[2], jnsx[2], jval;
  JobTable jya;  // dense A: Y_r = -2 W A, Y_i = Im Delta A per pair, Yd = Gamma A per state
  // exponential map: P = Gamma dGamma, Y = K^2, Z = Y^2, the three
  // Paterson-Stockmeyer steps, R = C + K S, squarings, R Gamma, (R Gamma) R^T
  double *ex0 = nullptr, *ex1 = nullptr, *ex2 = nullptr, *ex3 = nullptr, *exrow = nullptr, *expar = nullptr;
  JobTable jexp_p, jexp_y, jexp_z, jexp_h[3], jexp_r, jexp_sq[2], jexp_q, jexp_g;
  ExpCoef excf{};
  // Gauss-Jordan: inner updates per panel and trailing updates per
  // super-panel, for the pairs (0, a) (jgj0, jgs0) and the rest (jgj1, jgs1)
  std::vector<JobTable> jgj0, jgj1, jgs0, jgs1, jgf0, jgf1;
  std::vector<int> gj_k, gj_b, gj_s, gs_k, gs_nb;
  // Pfaffians of the Q matrices C_ab (order n)
  PfBatch pf;
};

// per pair: the panel's Brow (b x super-panel) or a super-panel's pivot rows (nb x n)
// whether the batch half (0: pairs (0, a), 1: the others) defers its
// Gauss-Jordan inner updates
static bool gj_deferred(const Prob& q, int half) { return half == 0 ? q.gj_defer == 3 : q.gj_defer >= 2; }

long long gj_brow_stride(int n) { return std::max((long long)GJ_NB_MAX * GJ_SUPER_MAX, (long long)GJ_SUPER_MAX * n); }

int gemm_tiles(int M, int N, int mirror = 0) {
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  return mirror ? tn * (tn + 1) / 2 : tm * tn;
}

void add_job(JobTable& t, GemmJob j) {
  j.tiles_n = (j.N + 63) / 64;
  j.tile_begin = 0;
  t.ntiles += gemm_tiles(j.M, j.N, j.mirror);
  t.host.push_back(j);
}

// Assign every job to one XCD (largest first, to the least loaded XCD), order
// the table by XCD and number each XCD's tiles from 0.
void place_jobs(JobTable& t) {
  std::vector<int> order(t.host.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return gemm_tiles(t.host[a].M, t.host[a].N, t.host[a].mirror) > gemm_tiles(t.host[b].M, t.host[b].N, t.host[b].mirror);
  });
  std::vector<std::vector<GemmJob>> per(8);
  int load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i : order) {
    int x = 0;
    for (int y = 1; y < 8; ++y)
      if (load[y] < load[x]) x = y;
    GemmJob j = t.host[i];
    j.tile_begin = load[x];
    load[x] += gemm_tiles(j.M, j.N, j.mirror);
    per[x].push_back(j);
  }
  t.host.clear();
  t.xm.max_tiles = 0;
  for (int x = 0; x < 8; ++x) {
    t.xm.off[x] = (int)t.host.size();
    for (auto& j : per[x]) t.host.push_back(j);
    t.xm.max_tiles = std::max(t.xm.max_tiles, load[x]);
  }
  t.xm.off[8] = (int)t.host.size();
}

// workgroup -> job map of a placed table (entries 8 * tile + xcd)
std::vector<int> job_map(const JobTable& t) {
  std::vector<int> m(8 * (size_t)t.xm.max_tiles, -1);
  for (int x = 0; x < 8; ++x)
    for (int jid = t.xm.off[x]; jid < t.xm.off[x + 1]; ++jid) {
      const GemmJob& j = t.host[jid];
      const int nt = gemm_tiles(j.M, j.N, j.mirror);
      for (int u = 0; u < nt; ++u) m[8 * (size_t)(j.tile_begin + u) + x] = jid;
    }
  return m;
}

GemmJob job(const double* A, int lda, int ta, const double* B, int ldb, int tb, const double* C, int ldc,
            double* D, int ldd, int M, int N, int K, double alpha, double beta, double diag = 0.0) {
  GemmJob j;
  std::memset(&j, 0, sizeof(j));
  j.A = A; j.B = B; j.C = C; j.D = D;
  j.lda = lda; j.ldb = ldb; j.ldc = ldc; j.ldd = ldd;
  j.ta = ta; j.tb = tb;
  j.M = M; j.N = N; j.K = K;
  j.alpha = alpha; j.beta = beta; j.diag = diag;
  return j;
}

}  // namespace

constexpr int NSTAGES = 8;  // SGS_STAGE_INVERSE .. SGS_STAGE_PURIFY

struct StageTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> rec;
  hipEvent_t cur[NSTAGES] = {};
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  // stages may overlap (two streams): each stage has its own open event
  void begin(int stage, hipStream_t s) {
    if (!on) return;
    cur[stage] = get();
    if (cur[stage]) (void)hipEventRecord(cur[stage], s);
  }
  void end(int stage, hipStream_t s) {
    if (!on || !cur[stage]) return;
    hipEvent_t e = get();
    if (!e) return;
    (void)hipEventRecord(e, s);
    rec.push_back({stage, cur[stage], e});
    cur[stage] = nullptr;
  }
  ~StageTimer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// device staging of the observables (polynomial terms, partial sums)
constexpr int GRAPH_RING = 1024;  // replays between copies of the energies

struct ObsBuf {
  double* ering = nullptr;  // energies of graph replays: GRAPH_RING x nprob
  int* rows = nullptr;
  double* coef = nullptr;
  int* off = nullptr;
  double* vpart = nullptr;  // variance partial sums, R (R + 1) / 2 x VAR_CHUNKS x 5 complex
};

// One stream of independent problems.  Worker 0 runs on the context's
// stream; every worker forks its phase chain onto its own second stream.
struct Worker {
  hipStream_t s = nullptr;
  bool own_s = false;
  hipStream_t s2 = nullptr;  // phase chain
  hipStream_t s3 = nullptr;  // inverses of the pairs not involving state 0
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_done = nullptr, ev_gj = nullptr, ev_gj_done = nullptr;
  hipEvent_t ev_f = nullptr, ev_fe = nullptr;  // elementwise force terms on s2
  int owner = -1;  // problem whose scratch tables are current
};

struct sgs_ctx {
  std::vector<Prob> pr;
  hipStream_t s = nullptr;
  std::vector<Worker> wk;
  hipEvent_t ev_start = nullptr;
  sgs_options opt;
  int* status = nullptr;
  int lds_max = 65536;
  bool evaluated = false;
  StageTimer timer;
  StageTimer mute;  // never switched on
  ObsBuf obs;
  // device buffers of the Renyi-2 evaluation, grown on demand
  void* ren = nullptr;
  size_t ren_bytes = 0;
  // graph replay of one step (sgs_options.graph): the energies of successive
  // replays go to ering[ctr * nprob + p], copied out after the replays
  hipGraphExec_t gexec = nullptr;
  hipStream_t gs = nullptr;  // capture stream (the caller's may be the legacy default stream)
  double gdtau = 0.0;
  int* ectr = nullptr;
  double* ering = nullptr;
  bool capturing = false;
  ~sgs_ctx() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gs) (void)hipStreamDestroy(gs);
    for (auto& w : wk) {
      if (w.ev_fork) (void)hipEventDestroy(w.ev_fork);
      if (w.ev_join) (void)hipEventDestroy(w.ev_join);
      if (w.ev_done) (void)hipEventDestroy(w.ev_done);
      if (w.ev_gj) (void)hipEventDestroy(w.ev_gj);
      if (w.ev_gj_done) (void)hipEventDestroy(w.ev_gj_done);
      if (w.ev_f) (void)hipEventDestroy(w.ev_f);
      if (w.ev_fe) (void)hipEventDestroy(w.ev_fe);
      if (w.s2) (void)hipStreamDestroy(w.s2);
      if (w.s3) (void)hipStreamDestroy(w.s3);
      if (w.own_s && w.s) (void)hipStreamDestroy(w.s);
    }
    if (ev_start) (void)hipEventDestroy(ev_start);
    if (ren) (void)hipFree(ren);
  }
  // fork: every worker stream waits for the work enqueued so far on s
  // (workers run on streams of their own, so that the caller's stream, which
  // may be the null stream, holds only these events while they work)
  hipError_t fork() {
    hipError_t e = hipEventRecord(ev_start, s);
    for (size_t w = 0; w < wk.size() && e == hipSuccess; ++w)
      if (wk[w].s != s) e = hipStreamWaitEvent(wk[w].s, ev_start, 0);
    return e;
  }
  // join: s waits for every worker stream
  hipError_t join() {
    hipError_t e = hipSuccess;
    for (size_t w = 0; w < wk.size() && e == hipSuccess; ++w) {
      if (wk[w].s == s) continue;
      e = hipEventRecord(wk[w].ev_done, wk[w].s);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, wk[w].ev_done, 0);
    }
    return e;
  }
};

// ---------------------------------------------------------------------------
// layout
// ---------------------------------------------------------------------------
static int check_problem(const sgs_problem& p) {
  if (p.N < 1 || p.N > 2048 || p.R < 1 || p.R > 32 || !p.A || p.nq < 0 || p.nq > 256) return SGS_EINVAL;
  if (p.nq > 0 && (!p.q_idx || !p.q_val)) return SGS_EINVAL;
  if (p.nw < 0 || p.nw > 256 || (p.nw > 0 && (!p.w_len || !p.w_idx || !p.w_val))) return SGS_EINVAL;
  const int n = 2 * p.N;
  for (int q = 0; q < p.nq; ++q) {
    const int* x = p.q_idx + 4 * q;
    for (int t = 0; t < 4; ++t)
      if (x[t] < 0 || x[t] >= n || (t > 0 && x[t] <= x[t - 1])) return SGS_EINVAL;
  }
  for (int w = 0, o = 0; w < p.nw; o += p.w_len[w], ++w) {
    if (p.w_len[w] != 6 && p.w_len[w] != 8) return SGS_EINVAL;
    const int* x = p.w_idx + o;
    for (int t = 0; t < p.w_len[w]; ++t)
      if (x[t] < 0 || x[t] >= n || (t > 0 && x[t] <= x[t - 1])) return SGS_EINVAL;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j)
      if (p.A[(size_t)i * n + j] != -p.A[(size_t)j * n + i]) return SGS_EINVAL;
  return SGS_OK;
}

// sorted Majorana indices touched by the interaction words (quartic and higher)
static std::vector<int> impurity_list(const sgs_problem& p) {
  std::vector<int> v(p.q_idx, p.q_idx + 4 * p.nq);
  for (int w = 0, o = 0; w < p.nw; o += p.w_len[w], ++w) v.insert(v.end(), p.w_idx + o, p.w_idx + o + p.w_len[w]);
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

// Fock items of the higher words: for every position pair a < b of word w an
// item (w, a, b) on the impurity entry (loc w_a, loc w_b), grouped by entry
struct FockItems {
  std::vector<int2> ent;
  std::vector<int> off;
  std::vector<int4> item;
};
static FockItems fock_items(const sgs_problem& p, const std::vector<int>& impos) {
  std::map<std::pair<int, int>, std::vector<int4>> by;
  for (int w = 0, o = 0; w < p.nw; o += p.w_len[w], ++w)
    for (int a = 0; a < p.w_len[w]; ++a)
      for (int b = a + 1; b < p.w_len[w]; ++b)
        by[{impos[p.w_idx[o + a]], impos[p.w_idx[o + b]]}].push_back(make_int4(w, a, b, 0));
  FockItems f;
  f.off.push_back(0);
  for (auto& kv : by) {
    f.ent.push_back(make_int2(kv.first.first, kv.first.second));
    f.item.insert(f.item.end(), kv.second.begin(), kv.second.end());
    f.off.push_back((int)f.item.size());
  }
  return f;
}

static int nnz_count(const sgs_problem& p, int* up) {
  const int n = 2 * p.N;
  int nz = 0, u = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (p.A[(size_t)i * n + j] != 0.0) { ++nz; if (j > i) ++u; }
  *up = u;
  return nz;
}

// Buffers of a Pfaffian batch (order m, B matrices).
static void pf_carve(PfBatch& b, Arena& ar) {
  const long long mm = (long long)b.m * b.m;
  b.uvstride = 2LL * b.m * 2 * PF_SUPER_MAX;  // planar: re block then im block
  b.uv_im = (long long)b.m * 2 * PF_SUPER_MAX;
  // deferred columns, twice: [row][step][U re, U im, V re, V im], then
  // step-major (U then V planes of complex pairs [step][row])
  b.pdstride = 8LL * b.m * PF_SUPER_MAX;
  b.A0 = ar.take<double>(std::max(1LL, 2 * b.B * mm));
  b.A1 = ar.take<double>(std::max(1LL, 2 * b.B * mm));
  b.perm = ar.take<int>(std::max(1LL, (long long)b.B * b.m));
  b.UV = ar.take<double>(std::max(1LL, b.B * b.uvstride));
  b.RM = ar.take<double>(std::max(1LL, b.B * b.uvstride));
  b.PD = ar.take<double>(std::max(1LL, b.B * b.pdstride));
}

// Schedule of a Pfaffian batch: super-panels of `super` steps (fewer at the
// end), each swept by register panels sized for the rows they hold; storage
// for the job table of every super-panel's trailing update.
static void pf_schedule(PfBatch& b, Arena& ar) {
  b.sm.clear(); b.sk.clear(); b.pan.clear();
  for (int m = b.m; m > 0;) {
    const int k = std::min(b.super, m / 2);
    const int sp = (int)b.sm.size();
    b.sm.push_back(m);
    b.sk.push_back(k);
    for (int done = 0; done < k;) {
      const int p0 = 2 * done;
      const int ns = std::min(pf_panel_shape(m - p0).nbh, k - done);
      b.pan.push_back({sp, p0, ns, done});
      done += ns;
    }
    m -= 2 * k;
  }
  const int T = (b.m + 63) / 64;
  const int jobs = std::max(1, b.B);
  b.jt.assign(b.sm.size(), JobTable());
  for (auto& t : b.jt) {
    t.dev = ar.take<GemmJob>(jobs);
    t.map_cap = 8 * jobs * T * T;
    t.dmap = ar.take<int>((size_t)t.map_cap);
  }
}

// Scratch of one evaluation: per-pair and per-state dense matrices.  Problems
// that run one after another on the same worker stream share one region.
static void carve_scratch(Prob& q, Arena& ar) {
  const long long nn = (long long)q.n * q.n;
  const int R = q.R, P = q.P, Q = q.Q, n = q.n;
  q.W = ar.take<double>(std::max(1LL, P * nn));
  q.Di = ar.take<double>(std::max(1LL, P * nn));
  q.Y = ar.take<double>(std::max(1LL, 2 * P * nn));
  q.Yd = ar.take<double>(R * nn);
  q.T1 = ar.take<double>(std::max(1LL, (R - 1) * nn));
  q.Xr = ar.take<double>(std::max(1LL, (R - 1) * nn));
  pf_carve(q.pf, ar);
  q.gjE = ar.take<double>(std::max(1LL, (long long)P * n * q.gj_super));  // E_all per pair
  q.gjB = ar.take<double>(std::max(1LL, (long long)P * gj_brow_stride(n)));
  q.dG = ar.take<double>(R * nn);
  q.dP = ar.take<double>(std::max(1LL, (FORCE_SPLIT_MAX - 1) * R * nn));  // partial force products, added into dG
  q.dE = ar.take<double>(R * nn);  // elementwise force terms, added into dG
  q.nsX0 = ar.take<double>(R * nn);
  q.nsX1 = ar.take<double>(R * nn);
  q.nsQ = ar.take<double>(R * nn);
  q.piv = ar.take<int>(std::max(1LL, 2LL * P * n));  // pivots, then unscramble sources
  if (q.expmap) {
    q.ex0 = ar.take<double>(R * nn);
    q.ex1 = ar.take<double>(R * nn);
    q.ex2 = ar.take<double>(R * nn);
    q.ex3 = ar.take<double>(R * nn);
    q.exrow = ar.take<double>((long long)R * n);
    q.expar = ar.take<double>(4);
  }
}

// Per-problem state that persists between calls (tables, amplitudes, the
// Hamiltonian in device form).
static void carve(Prob& q, Arena& ar) {
  const long long nn = (long long)q.n * q.n;
  const int R = q.R, P = q.P, Q = q.Q, M = q.M, n = q.n;
  q.Adense = ar.take<double>(nn);
  q.pfacc = ar.take<double>(std::max(1, 3 * Q));
  q.logdet = ar.take<double>(std::max(1, P));
  q.eps = ar.take<double>(2 * (P + R));
  q.Fc = ar.take<double>(std::max(1, 2 * M * M * (P + R)));
  q.coef = ar.take<double>(4 * R * R);
  q.Gt = ar.take<double>(2 * R * R);
  q.ht = ar.take<double>(2 * R * R);
  q.lam = ar.take<double>(2 * R);
  q.lamt = ar.take<double>(2 * R);
  q.E = ar.take<double>(1);
  q.tab_la = ar.take<double>(R * R);
  q.tab_arg = ar.take<double>(R * R);
  q.tab_eps = ar.take<double>(2 * R * R);
  q.up_v = ar.take<double>(std::max(1, q.nnz_up));
  q.colval = ar.take<double>(std::max(1, q.nnz));
  q.q_val = ar.take<double>(std::max(1, q.nq));
  q.pa = ar.take<int>(std::max(1, P));
  q.pb = ar.take<int>(std::max(1, P));
  q.qa = ar.take<int>(std::max(1, Q));
  q.qb = ar.take<int>(std::max(1, Q));
  q.pidx = ar.take<int>(R * R);
  q.qidx = ar.take<int>(R * R);
  q.up_k = ar.take<int>(std::max(1, q.nnz_up));
  q.up_l = ar.take<int>(std::max(1, q.nnz_up));
  q.colptr = ar.take<int>(n + 1);
  q.rowidx = ar.take<int>(std::max(1, q.nnz));
  q.imp = ar.take<int>(std::max(1, M));
  q.impos = ar.take<int>(n);
  q.q_idx = ar.take<int>(std::max(1, 4 * q.nq));
  q.q_loc = ar.take<int>(std::max(1, 4 * q.nq));
  q.w_idx = ar.take<int>(std::max(1, 8 * q.nw));
  q.w_len = ar.take<int>(std::max(1, q.nw));
  q.w_val = ar.take<double>(std::max(1, q.nw));
  q.fe_ent = ar.take<int2>(std::max(1, q.nfe));
  q.fe_off = ar.take<int>(q.nfe + 1);
  q.fe_item = ar.take<int4>(std::max(1, q.nfi));
  q.resid = ar.take<unsigned long long>(8);  // [0]: input validation
  q.nsctl = ar.take<int>(R + 4);  // [0] all done, [1] count, [2 + mu] per state
  q.nsres = ar.take<unsigned long long>(64 * (size_t)(R + 2));  // [it (R + 2) + 2 + mu]: polar residuals
  q.dgnorm = ar.take<unsigned long long>(32);
  q.terms = ar.take<ForceTerm>((size_t)R * R);
}

static void carve_jobs(Prob& q, Arena& ar) {
  const int n = q.n;
  const int T = (n + 63) / 64;
  // job array plus a workgroup -> job map sized for jobs x T^2 tiles (every
  // job of a table is at most n x n)
  auto table = [&](JobTable& t, int jobs) {
    jobs = std::max(1, jobs);
    t.dev = ar.take<GemmJob>(jobs);
    t.map_cap = 8 * jobs * T * T;
    t.dmap = ar.take<int>((size_t)t.map_cap);
  };
  // panels and super-panels of the Gauss-Jordan inverse
  q.gj_k.clear(); q.gj_b.clear(); q.gj_s.clear(); q.gs_k.clear(); q.gs_nb.clear();
  for (int k0 = 0; k0 < n; k0 += q.gj_super) {
    const int nbs = std::min(q.gj_super, n - k0);
    for (int k = k0; k < k0 + nbs; k += q.gj_nb) {
      q.gj_k.push_back(k);
      q.gj_b.push_back(std::min(q.gj_nb, k0 + nbs - k));
      q.gj_s.push_back((int)q.gs_k.size());
    }
    q.gs_k.push_back(k0);
    q.gs_nb.push_back(nbs);
  }
  const int P0 = std::min(q.P, q.R - 1);
  q.jgj0.assign(q.gj_k.size(), JobTable());
  q.jgj1.assign(q.gj_k.size(), JobTable());
  q.jgs0.assign(q.gs_k.size(), JobTable());
  q.jgs1.assign(q.gs_k.size(), JobTable());
  q.jgf0.assign(q.gs_k.size(), JobTable());
  q.jgf1.assign(q.gs_k.size(), JobTable());
  for (auto& t : q.jgj0) table(t, P0);
  for (auto& t : q.jgj1) table(t, q.P - P0);
  for (auto& t : q.jgs0) table(t, 2 * P0);
  for (auto& t : q.jgs1) table(t, 2 * (q.P - P0));
  const int pps = GJ_SUPER_MAX / std::max(1, q.gj_nb);  // panels per super-panel, at most
  for (auto& t : q.jgf0) table(t, pps * P0);
  for (auto& t : q.jgf1) table(t, pps * (q.P - P0));
  pf_schedule(q.pf, ar);
  table(q.jdi, q.P);
  table(q.jya, q.denseA ? 2 * q.P + q.R : 0);
  table(q.jt1, q.R - 1);
  table(q.jxr, q.R - 1);
  for (int k = 0; k < 2; ++k) {
    table(q.jnsq[k], q.R);
    table(q.jnsx[k], q.R);
  }
  table(q.jval, q.R);
  if (q.expmap) {
    table(q.jexp_p, q.R);
    table(q.jexp_y, q.R);
    table(q.jexp_z, q.R);
    for (auto& t : q.jexp_h) table(t, 2 * q.R);
    table(q.jexp_r, q.R);
    for (auto& t : q.jexp_sq) table(t, q.R);
    table(q.jexp_q, q.R);
    table(q.jexp_g, q.R);
  }
}

static int pick_gj_nb(int n, int lds_max) {
  (void)lds_max;
  return std::min(gj_panel_shape(n).B, n);
}

static int device_lds_max() {
  int dev = 0, v = 65536;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
  return v;
}

constexpr int MAX_WORKERS = 8;  // concurrent worker streams for independent problems
constexpr int DEFAULT_WORKERS = 4;
// more nonzeros of A per column than this: Y = Delta A by grouped GEMMs
// instead of the compressed-column product
constexpr int DENSE_A_PER_COLUMN = 16;

// Pfaffian super-panels of 32 steps (rank-64 trailing updates) beat 16 and
// 24 at n = 800 and 1204 (92.5 / 95.0 / 93.3 and 190 / 200 / 193 ms per
// step); at n = 400 one register panel of 16 steps per update is best (the
// chain is bound by the panels' latency there, not by the updates)
static int pf_super_default(int m) { return m <= 512 ? 16 : PF_SUPER_MAX; }

// Built-in scheduling choices by size, then the caller's tuning row (if any).
static void pick_tuning(Prob& q, const sgs_options& o) {
  // measured at n = 400, 800, 1204, alternating the settings in one
  // session: both batches of inverses start together (with the pairs (0, a)
  // first the phase chain shares the GPU with the other inverses for its
  // whole length); Gauss-Jordan super-panels of 128 (256 ties at n = 1204,
  // 180.3 ms per step either way); force tiles of one workgroup between
  // n = 600 and 1002 (89.5 instead of 91.0 ms at n = 800), of two elsewhere
  // (5.72 instead of 5.80 ms at n = 400, 180.9 instead of 181.2 at 1204)
  q.gj_nb = pick_gj_nb(q.n, 0);
  q.gj_super = 128;
  q.pf.super = pf_super_default(q.n);
  q.force_split = q.n > 600 && q.n <= 1002 ? 1 : 2;
  q.gj_first = false;
  for (int i = 0; i < o.ntune; ++i) {
    const sgs_tune& t = o.tune[i];
    if (q.n > t.n_max) continue;
    if (t.gj_super > 0) q.gj_super = t.gj_super;
    if (t.gj_first > 0) q.gj_first = t.gj_first == 1;
    if (t.pf_super > 0) q.pf.super = t.pf_super;
    if (t.force_split > 0) q.force_split = t.force_split;
    if (t.force_elem > 0) q.force_seq = t.force_elem == 2;
    if (t.force_tile > 0) q.force_tile = t.force_tile;
    if (t.gj_defer > 0) q.gj_defer = t.gj_defer;
    break;
  }
  q.gj_super = std::max(q.gj_nb, std::min(GJ_SUPER_MAX, q.gj_super / q.gj_nb * q.gj_nb));
  q.pf.super = std::max(1, std::min(PF_SUPER_MAX, q.pf.super));
  q.force_split = std::max(1, std::min(std::min(FORCE_SPLIT_MAX, q.R), q.force_split));
}

static size_t plan(std::vector<Prob>& pr, const sgs_problem* probs, int nprob, char* base, int lds_max,
                   int max_workers, bool expmap, const sgs_options& opt, ObsBuf* ob = nullptr,
                   int* nworkers = nullptr) {
  Arena ar{base, 0};
  ar.take<int>(64);  // status word and spare (the graph's step counter)
  {
    ObsBuf o;
    o.rows = ar.take<int>(6 * (size_t)OBS_MAX_TERMS);
    o.coef = ar.take<double>(2 * (size_t)OBS_MAX_TERMS);
    o.off = ar.take<int>((size_t)OBS_MAX_POLY + 1);
    o.vpart = ar.take<double>((size_t)32 * 32 * VAR_CHUNKS * 10);
    o.ering = ar.take<double>((size_t)GRAPH_RING * nprob);
    if (ob) *ob = o;
  }
  pr.assign(nprob, Prob());
  for (int p = 0; p < nprob; ++p) {
    Prob& q = pr[p];
    const sgs_problem& sp = probs[p];
    q.N = sp.N; q.n = 2 * sp.N; q.R = sp.R;
    q.P = q.R * (q.R - 1) / 2;
    q.Q = (q.R - 1) * (q.R - 2) / 2;
    q.pf.m = q.n;
    q.pf.B = q.Q;
    q.nq = sp.nq; q.e0 = sp.e0;
    q.M = (int)impurity_list(sp).size();
    q.nw = sp.nw;
    q.nfi = 0;
    for (int w = 0; w < sp.nw; ++w) q.nfi += sp.w_len[w] * (sp.w_len[w] - 1) / 2;
    q.nfe = q.nfi;  // at most one entry per item
    q.nnz = nnz_count(sp, &q.nnz_up);
    q.denseA = q.nnz > DENSE_A_PER_COLUMN * q.n;
    (void)lds_max;
    pick_tuning(q, opt);
    q.expmap = expmap;
    carve(q, ar);
    carve_jobs(q, ar);
  }
  // workers: problems go, largest first, to the least loaded stream (work
  // ~ R^2 n^3); each stream's scratch region fits its largest problem
  const int K = std::max(1, std::min(nprob, max_workers));
  std::vector<size_t> need(nprob);
  std::vector<int> order(nprob);
  for (int p = 0; p < nprob; ++p) {
    Arena probe{nullptr, 0};
    carve_scratch(pr[p], probe);
    need[p] = probe.off;
    order[p] = p;
  }
  auto work = [&](int p) { return (double)pr[p].R * pr[p].R * pr[p].n * (double)pr[p].n * pr[p].n; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  std::vector<double> load(K, 0.0);
  std::vector<size_t> region(K, 0);
  for (int p : order) {
    int w = 0;
    for (int v = 1; v < K; ++v)
      if (load[v] < load[w]) w = v;
    pr[p].worker = w;
    load[w] += work(p);
    region[w] = std::max(region[w], need[p]);
  }
  for (int w = 0; w < K; ++w) {
    const size_t start = (ar.off + 255) & ~(size_t)255;
    for (int p = 0; p < nprob; ++p)
      if (pr[p].worker == w) {
        Arena sub{base ? base + start : nullptr, 0};
        carve_scratch(pr[p], sub);
      }
    ar.off = start + region[w];
  }
  if (nworkers) *nworkers = K;
  return ar.off + 256;
}

// ---------------------------------------------------------------------------
// static tables
// ---------------------------------------------------------------------------
#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return SGS_EHIP; \
  } while (0)

template <class T>
static hipError_t up(T* dev, const std::vector<T>& host) {
  if (host.empty()) return hipSuccess;
  return hipMemcpy(dev, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
}

static hipError_t upload_jobs(JobTable& t) {
  place_jobs(t);
  t.xm.map = nullptr;
  if (t.host.empty()) return hipSuccess;
  hipError_t e = hipMemcpy(t.dev, t.host.data(), t.host.size() * sizeof(GemmJob), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  const std::vector<int> m = job_map(t);
  if (t.dmap && (int)m.size() <= t.map_cap) {
    e = hipMemcpy(t.dmap, m.data(), m.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) t.xm.map = t.dmap;
  }
  return e;
}

// Trailing updates of a Pfaffian batch: super-panel t reads the compact
// trailing matrix from buffer t % 2 and its GEMM writes the next one, read
// through the super-panel's permutation, into the other buffer:
//   A' = A[perm, perm] + [U V] [V -U]^T   (depth 2 k)
static hipError_t pf_jobs(PfBatch& b) {
  const int n = b.m;
  const long long nn = (long long)n * n;
  for (size_t t = 0; t < b.sm.size(); ++t) {
    const int m = b.sm[t], k = b.sk[t];
    const int mp = m - 2 * k, K = 2 * k;
    JobTable& jt = b.jt[t];
    jt.host.clear(); jt.ntiles = 0; jt.cplx = true;
    double* cin = (t & 1) ? b.A1 : b.A0;
    double* cout = (t & 1) ? b.A0 : b.A1;
    if (mp > 0)
      for (int qq = 0; qq < b.B; ++qq) {
        // the last panel stores [U V] and [V -U] transposed (K x mp)
        GemmJob j = job(b.UV + qq * b.uvstride, mp, 1, b.RM + qq * b.uvstride, mp, 0, cin + qq * 2 * nn, n,
                        cout + qq * 2 * nn, n, mp, mp, K, 1.0, 1.0);
        j.a_im = b.uv_im; j.b_im = b.uv_im; j.c_im = nn; j.d_im = nn;
        j.cperm = b.perm + (long long)qq * n + 2 * k;
        j.mirror = -1;  // the trailing matrix stays skew
        add_job(jt, j);
      }
    hipError_t e = upload_jobs(jt);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Job tables of the exponential-map update (buffers: P -> nsX0, K -> nsQ,
// Y -> nsX1, Z -> dG; the even / odd polynomials ping-pong between ex0 / ex1
// and ex2 / ex3; R -> nsX0, squarings nsX0 <-> ex0; R Gamma -> nsQ).
static hipError_t build_exp_jobs(Prob& q) {
  const int n = q.n, R = q.R;
  const long long nn = (long long)n * n;
  double cf[9], sf[9];
  {
    double f = 1.0;  // k!
    for (int k = 0; k <= 17; ++k) {
      if (k > 0) f *= k;
      if (k % 2 == 0) cf[k / 2] = 1.0 / f; else sf[k / 2] = 1.0 / f;
    }
  }
  auto reset = [](JobTable& t) { t.host.clear(); t.ntiles = 0; };
  JobTable* all[] = {&q.jexp_p, &q.jexp_y, &q.jexp_z, &q.jexp_h[0], &q.jexp_h[1], &q.jexp_h[2],
                     &q.jexp_r, &q.jexp_sq[0], &q.jexp_sq[1], &q.jexp_q, &q.jexp_g};
  for (JobTable* t : all) reset(*t);
  for (int mu = 0; mu < R; ++mu) {
    const long long o = mu * nn;
    double *P = q.nsX0 + o, *K = q.nsQ + o, *Y = q.nsX1 + o, *Z = q.dG + o, *G = q.gam + o;
    add_job(q.jexp_p, job(G, n, 0, q.dG + o, n, 0, nullptr, n, P, n, n, n, n, 1.0, 0.0));
    GemmJob jy = job(K, n, 0, K, n, 0, nullptr, n, Y, n, n, n, n, 1.0, 0.0);
    jy.mirror = 1;
    add_job(q.jexp_y, jy);
    GemmJob jz = job(Y, n, 0, Y, n, 0, nullptr, n, Z, n, n, n, n, 1.0, 0.0);
    jz.mirror = 1;
    add_job(q.jexp_z, jz);
    // B_{k} = Z B_{k+1} + c_{2k+1} Y + c_{2k} I for k = 2, 1, 0 (C and S)
    double* cin[3] = {q.ex0 + o, q.ex2 + o, q.ex0 + o};
    double* cout[3] = {q.ex2 + o, q.ex0 + o, q.ex2 + o};
    double* sin_[3] = {q.ex1 + o, q.ex3 + o, q.ex1 + o};
    double* sout[3] = {q.ex3 + o, q.ex1 + o, q.ex3 + o};
    for (int h = 0; h < 3; ++h) {
      const int k = 2 - h;
      GemmJob jc = job(Z, n, 0, cin[h], n, 0, Y, n, cout[h], n, n, n, n, 1.0, cf[2 * k + 1], cf[2 * k]);
      jc.mirror = 1;
      add_job(q.jexp_h[h], jc);
      GemmJob js = job(Z, n, 0, sin_[h], n, 0, Y, n, sout[h], n, n, n, n, 1.0, sf[2 * k + 1], sf[2 * k]);
      js.mirror = 1;
      add_job(q.jexp_h[h], js);
    }
    // R = K S + C into nsX0 (P is no longer needed)
    add_job(q.jexp_r, job(K, n, 0, q.ex3 + o, n, 0, q.ex2 + o, n, q.nsX0 + o, n, n, n, n, 1.0, 1.0));
    add_job(q.jexp_sq[0], job(q.nsX0 + o, n, 0, q.nsX0 + o, n, 0, nullptr, n, q.ex0 + o, n, n, n, n, 1.0, 0.0));
    add_job(q.jexp_sq[1], job(q.ex0 + o, n, 0, q.ex0 + o, n, 0, nullptr, n, q.nsX0 + o, n, n, n, n, 1.0, 0.0));
    add_job(q.jexp_q, job(q.nsX0 + o, n, 0, G, n, 0, nullptr, n, q.nsQ + o, n, n, n, n, 1.0, 0.0));
    GemmJob jg = job(q.nsQ + o, n, 0, q.nsX0 + o, n, 1, nullptr, n, G, n, n, n, n, 1.0, 0.0);
    jg.mirror = -1;  // R Gamma R^T is skew
    add_job(q.jexp_g, jg);
  }
  for (JobTable* t : all) {
    hipError_t e = upload_jobs(*t);
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k < 9; ++k) { q.excf.c[k] = cf[k]; q.excf.s[k] = sf[k]; }
  return hipSuccess;
}

static int build_tables(Prob& q, const sgs_problem& sp) {
  const int n = q.n, R = q.R, P = q.P;
  const long long nn = (long long)n * n;
  // pair lists
  std::vector<int> pa(P), pb(P), pidx(R * R, -1), qa, qb, qidx(R * R, -1);
  int p = 0;
  for (int a = 0; a < R; ++a)
    for (int b = a + 1; b < R; ++b) {
      pa[p] = a; pb[p] = b; pidx[a * R + b] = pidx[b * R + a] = p; ++p;
    }
  for (int a = 1; a < R; ++a)
    for (int b = a + 1; b < R; ++b) {
      qidx[a * R + b] = (int)qa.size();
      qa.push_back(a); qb.push_back(b);
    }
  HIPCHK(up(q.pa, pa)); HIPCHK(up(q.pb, pb)); HIPCHK(up(q.pidx, pidx));
  HIPCHK(up(q.qa, qa)); HIPCHK(up(q.qb, qb)); HIPCHK(up(q.qidx, qidx));
  // A: dense, upper nonzeros, compressed columns
  std::vector<double> Ad(sp.A, sp.A + nn);
  HIPCHK(up(q.Adense, Ad));
  std::vector<int> uk, ul, colptr(n + 1, 0), rowidx;
  std::vector<double> uv, colval;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (Ad[(size_t)i * n + j] != 0.0) { uk.push_back(i); ul.push_back(j); uv.push_back(Ad[(size_t)i * n + j]); }
  q.a2 = 0.0;
  for (double v : uv) q.a2 += 2.0 * v * v;
  for (int j = 0; j < n; ++j) {
    colptr[j] = (int)rowidx.size();
    for (int i = 0; i < n; ++i)
      if (Ad[(size_t)i * n + j] != 0.0) { rowidx.push_back(i); colval.push_back(Ad[(size_t)i * n + j]); }
  }
  colptr[n] = (int)rowidx.size();
  HIPCHK(up(q.up_k, uk)); HIPCHK(up(q.up_l, ul)); HIPCHK(up(q.up_v, uv));
  HIPCHK(up(q.colptr, colptr)); HIPCHK(up(q.rowidx, rowidx)); HIPCHK(up(q.colval, colval));
  // impurity Majoranas
  std::vector<int> imp = impurity_list(sp);
  std::vector<int> impos(n, -1), qloc(4 * sp.nq), qidxv(sp.q_idx, sp.q_idx + 4 * sp.nq);
  for (size_t t = 0; t < imp.size(); ++t) impos[imp[t]] = (int)t;
  for (int t = 0; t < 4 * sp.nq; ++t) qloc[t] = impos[sp.q_idx[t]];
  std::vector<double> qv(sp.q_val, sp.q_val + sp.nq);
  HIPCHK(up(q.imp, imp)); HIPCHK(up(q.impos, impos)); HIPCHK(up(q.q_loc, qloc));
  HIPCHK(up(q.q_idx, qidxv)); HIPCHK(up(q.q_val, qv));
  if (sp.nw > 0) {
    std::vector<int> widx(8 * sp.nw, -1), wlen(sp.w_len, sp.w_len + sp.nw);
    for (int w = 0, o = 0; w < sp.nw; o += sp.w_len[w], ++w)
      for (int t = 0; t < sp.w_len[w]; ++t) widx[8 * w + t] = sp.w_idx[o + t];
    std::vector<double> wv(sp.w_val, sp.w_val + sp.nw);
    const FockItems f = fock_items(sp, impos);
    q.nfe = (int)f.ent.size();
    HIPCHK(up(q.w_idx, widx)); HIPCHK(up(q.w_len, wlen)); HIPCHK(up(q.w_val, wv));
    HIPCHK(up(q.fe_ent, f.ent)); HIPCHK(up(q.fe_off, f.off)); HIPCHK(up(q.fe_item, f.item));
  } else {
    q.nfe = 0;
  }

  // --- GEMM job tables ---
  // Gauss-Jordan.  Pairs are ordered (0,1) .. (0,R-1), (1,2), ...: the first
  // R - 1 feed the phases and form their own batch.  Per pair E_all (n x ES)
  // and Brow_all (ES x ES, in the Brow buffer), ES = gj_super; panel t covers
  // columns [k, k + b), kl = k - k0, of super-panel [k0, k0 + nbs).  A batch
  // with deferred inner updates runs before the panel (kl > 0)
  //   M[:, k:k+b] -= E_all[:, 0:kl] Brow_all[0:kl, kl:kl+b]
  // and after the super-panel's last panel, for every panel v = [kv, kv + bv)
  // but the last (kv local),
  //   M[:, k0+kv : k0+kv+bv] -= E_all[:, kv+bv : nbs] Brow_all[kv+bv : nbs, kv : kv+bv];
  // a batch without runs after the panel
  //   M[:, k0:k0+nbs] -= E_all[:, kl:kl+b] Brow_all[kl:kl+b, 0:nbs].
  // Trailing update of super-panel s, the columns left and right of it:
  //   M[:, c] += M[:, k0:k0+nbs] Brow[:, c]   (Brow: nbs x n)
  const long long bstr = gj_brow_stride(n);
  const int ES = q.gj_super;
  for (size_t t = 0; t < q.gj_k.size(); ++t) {
    const int b = q.gj_b[t], s = q.gj_s[t], k0 = q.gs_k[s], nbs = q.gs_nb[s], kl = q.gj_k[t] - k0;
    for (int half = 0; half < 2; ++half) {
      JobTable& jt = half == 0 ? q.jgj0[t] : q.jgj1[t];
      jt.host.clear(); jt.ntiles = 0; jt.late_c = true;
      const int p0 = half == 0 ? 0 : std::min(P, R - 1), p1 = half == 0 ? std::min(P, R - 1) : P;
      const bool defer = gj_deferred(q, half);
      for (int pp = p0; pp < p1; ++pp) {
        const double* Ea = q.gjE + (long long)pp * n * ES;
        const double* Ba = q.gjB + pp * bstr;
        if (defer && kl > 0) {
          double* Mk = q.Di + pp * nn + q.gj_k[t];
          add_job(jt, job(Ea, ES, 0, Ba + kl, ES, 0, Mk, n, Mk, n, n, b, kl, -1.0, 1.0));
        } else if (!defer && nbs > b) {  // a super-panel of one panel has nothing else to update
          double* Ms = q.Di + pp * nn + k0;
          add_job(jt, job(Ea + kl, ES, 0, Ba + (long long)kl * ES, ES, 0, Ms, n, Ms, n, n, nbs, b, -1.0, 1.0));
        }
      }
      HIPCHK(upload_jobs(jt));
    }
  }
  for (size_t s = 0; s < q.gs_k.size(); ++s) {
    const int k0 = q.gs_k[s], nbs = q.gs_nb[s];
    for (int half = 0; half < 2; ++half) {
      JobTable& jt = half == 0 ? q.jgf0[s] : q.jgf1[s];
      jt.host.clear(); jt.ntiles = 0; jt.late_c = true;
      const int p0 = half == 0 ? 0 : std::min(P, R - 1);
      const int p1 = !gj_deferred(q, half) ? p0 : (half == 0 ? std::min(P, R - 1) : P);
      for (size_t t = 0; t < q.gj_k.size(); ++t) {
        if (q.gj_s[t] != (int)s) continue;
        const int kv = q.gj_k[t] - k0, bv = q.gj_b[t];
        if (kv + bv >= nbs) continue;  // the last panel: no later panel
        for (int pp = p0; pp < p1; ++pp) {
          double* Mv = q.Di + pp * nn + k0 + kv;
          const double* Ea = q.gjE + (long long)pp * n * ES + kv + bv;
          const double* Bv = q.gjB + pp * bstr + (long long)(kv + bv) * ES + kv;
          add_job(jt, job(Ea, ES, 0, Bv, ES, 0, Mv, n, Mv, n, n, bv, nbs - kv - bv, -1.0, 1.0));
        }
      }
      HIPCHK(upload_jobs(jt));
    }
  }
  for (size_t s = 0; s < q.gs_k.size(); ++s) {
    const int k0 = q.gs_k[s], nbs = q.gs_nb[s];
    for (int half = 0; half < 2; ++half) {
      JobTable& jt = half == 0 ? q.jgs0[s] : q.jgs1[s];
      jt.host.clear(); jt.ntiles = 0; jt.late_c = true;
      const int p0 = half == 0 ? 0 : std::min(P, R - 1), p1 = half == 0 ? std::min(P, R - 1) : P;
      for (int pp = p0; pp < p1; ++pp) {
        double* M = q.Di + pp * nn;
        const double* Br = q.gjB + pp * bstr;
        if (k0 > 0) add_job(jt, job(M + k0, n, 0, Br, n, 0, M, n, M, n, n, k0, nbs, 1.0, 1.0));
        if (k0 + nbs < n)
          add_job(jt, job(M + k0, n, 0, Br + k0 + nbs, n, 0, M + k0 + nbs, n, M + k0 + nbs, n, n, n - k0 - nbs, nbs,
                          1.0, 1.0));
      }
      HIPCHK(upload_jobs(jt));
    }
  }
  // Im Delta^{ba} = 2 Gamma_b W - 1
  q.jdi.host.clear(); q.jdi.ntiles = 0;
  for (int pp = 0; pp < P; ++pp)
  {
    GemmJob j = job(q.gam + (long long)pb[pp] * nn, n, 0, q.W + pp * nn, n, 0, nullptr, n, q.Di + pp * nn, n,
                    n, n, n, 2.0, 0.0, -1.0);
    j.mirror = -1;  // Im Delta is skew
    add_job(q.jdi, j);
  }
  HIPCHK(upload_jobs(q.jdi));
  // dense A: the products with A on the matrix cores
  q.jya.host.clear(); q.jya.ntiles = 0;
  if (q.denseA) {
    for (int pp = 0; pp < P; ++pp) {
      add_job(q.jya, job(q.W + pp * nn, n, 0, q.Adense, n, 0, nullptr, n, q.Y + 2 * pp * nn, n, n, n, n, -2.0, 0.0));
      add_job(q.jya, job(q.Di + pp * nn, n, 0, q.Adense, n, 0, nullptr, n, q.Y + (2 * pp + 1) * nn, n, n, n, n,
                         1.0, 0.0));
    }
    for (int mu = 0; mu < R; ++mu)
      add_job(q.jya, job(q.gam + mu * nn, n, 0, q.Adense, n, 0, nullptr, n, q.Yd + mu * nn, n, n, n, n, 1.0, 0.0));
  }
  HIPCHK(upload_jobs(q.jya));
  // phase matrices: T_a = Gamma_0 W_0a ; Re X_a = T_a Gamma_0 + W_0a
  q.jt1.host.clear(); q.jt1.ntiles = 0; q.jxr.host.clear(); q.jxr.ntiles = 0;
  for (int a = 1; a < R; ++a) {
    const int p0a = pidx[a];
    add_job(q.jt1, job(q.gam, n, 0, q.W + p0a * nn, n, 0, nullptr, n, q.T1 + (a - 1) * nn, n, n, n, n, 1.0, 0.0));
    add_job(q.jxr, job(q.T1 + (a - 1) * nn, n, 0, q.gam, n, 0, q.W + p0a * nn, n, q.Xr + (a - 1) * nn, n, n, n, n,
                       1.0, 1.0));
  }
  HIPCHK(upload_jobs(q.jt1)); HIPCHK(upload_jobs(q.jxr));
  HIPCHK(pf_jobs(q.pf));
  // Newton-Schulz: Q = X X ; X' = 0.5 X Q + 1.5 X (ping-pong)
  for (int par = 0; par < 2; ++par) {
    double* Xin = par ? q.nsX1 : q.nsX0;
    double* Xout = par ? q.nsX0 : q.nsX1;
    q.jnsq[par].host.clear(); q.jnsq[par].ntiles = 0;
    q.jnsx[par].host.clear(); q.jnsx[par].ntiles = 0;
    for (int mu = 0; mu < R; ++mu) {
      GemmJob jq = job(Xin + mu * nn, n, 0, Xin + mu * nn, n, 0, nullptr, n, q.nsQ + mu * nn, n, n, n, n, 1.0, 0.0);
      jq.mirror = 1;  // X^2 is symmetric for skew X
      jq.gate = 2 + mu;
      add_job(q.jnsq[par], jq);
      GemmJob jx = job(Xin + mu * nn, n, 0, q.nsQ + mu * nn, n, 0, Xin + mu * nn, n, Xout + mu * nn, n, n, n, n,
                       0.5, 1.5);
      jx.mirror = -1;  // X (3 + X^2) / 2 is skew
      jx.gate = 2 + mu;
      add_job(q.jnsx[par], jx);
    }
    HIPCHK(upload_jobs(q.jnsq[par])); HIPCHK(upload_jobs(q.jnsx[par]));
  }
  // validation: Q = Gamma Gamma
  q.jval.host.clear(); q.jval.ntiles = 0;
  for (int mu = 0; mu < R; ++mu)
    add_job(q.jval, job(q.gam + mu * nn, n, 0, q.gam + mu * nn, n, 0, nullptr, n, q.nsQ + mu * nn, n, n, n, n, 1.0, 0.0));
  HIPCHK(upload_jobs(q.jval));
  if (q.expmap) HIPCHK(build_exp_jobs(q));

  // force descriptors
  std::vector<ForceTerm> terms((size_t)R * R);
  const int M = q.M;
  for (int mu = 0; mu < R; ++mu)
    for (int b = 0; b < R; ++b) {
      ForceTerm& t = terms[(size_t)mu * R + b];
      std::memset(&t, 0, sizeof(t));
      t.coef = mu * R + b;
      if (b == mu) {
        t.Dr = q.gam + mu * nn; t.Di = nullptr;
        t.Yr = q.Yd + mu * nn; t.Yi = nullptr;
        t.Fcr = q.Fc + (long long)(P + mu) * 2 * M * M; t.Fci = nullptr;
        t.dr_scale = 1.0; t.sgn = 1.0;
      } else {
        const int pp = pidx[mu * R + b];
        t.Dr = q.W + pp * nn; t.Di = q.Di + pp * nn;
        t.Yr = q.Y + pp * 2 * nn; t.Yi = q.Y + pp * 2 * nn + nn;
        t.Fcr = q.Fc + (long long)pp * 2 * M * M; t.Fci = t.Fcr + M * M;
        t.dr_scale = -2.0;
        t.sgn = (mu < b) ? 1.0 : -1.0;  // pair stores Delta^{ba} (a < b); mu = b takes its conjugate
      }
    }
  HIPCHK(up(q.terms, terms));
  return SGS_OK;
}

// ---------------------------------------------------------------------------
// stages
// ---------------------------------------------------------------------------
static hipError_t run_gemm(const JobTable& t, hipStream_t s) {
  return t.late_c ? launch_gemm_late_c(t.dev, t.xm, s) : launch_gemm(t.dev, t.xm, t.cplx, s);
}

#define HCHK(x)                               \
  do {                                        \
    hipError_t _e = (x);                      \
    if (_e != hipSuccess) return _e;          \
  } while (0)

// All B Pfaffians of a batch: {ln|Pf|, cos arg, sin arg} per matrix into acc;
// a vanishing pivot sets ST_SINGULAR in *status (ln|Pf| is then not finite).
static hipError_t pf_run(const PfBatch& b, double* acc, int* status, hipStream_t s) {
  const long long nn = (long long)b.m * b.m;
  for (size_t i = 0; i < b.pan.size(); ++i) {
    const PfBatch::Panel& pp = b.pan[i];
    const int sp = pp.sp, k = b.sk[sp];
    const bool last = pp.kd + pp.ns == k;
    const double* cin = (sp & 1) ? b.A1 : b.A0;
    HCHK(launch_pf_panel(cin, 2 * nn, nn, b.m, b.sm[sp], pp.p0, pp.ns, pp.kd, k, pp.kd == 0, last, b.B, b.PD,
                         b.pdstride, b.UV, b.RM, b.uvstride, b.uv_im, b.perm, b.m, acc, i == 0, status, s));
    if (last) HCHK(run_gemm(b.jt[sp], s));
  }
  return hipSuccess;
}

static hipError_t pair_stage(sgs_ctx* c, Prob& q, double* energy_slot, double* o_la, double* o_arg, double* o_eps) {
  Worker& wk = c->wk[q.worker];
  hipStream_t s = wk.s;
  const int n = q.n, P = q.P, R = q.R;
  const long long nn = (long long)n * n;
  // stage times are recorded for the problems of worker 0 (not while a step
  // is being captured into a graph)
  StageTimer& tm = q.worker == 0 && !c->capturing ? c->timer : c->mute;
  const int P0 = std::min(P, R - 1);  // pairs (0, a): their inverses feed the phases
  const bool fork = q.Q > 0;
  if (P > 0) {
    // overlap magnitudes and W = (Gamma_a + Gamma_b)^{-1}; the elimination
    // runs in the Di buffer (overwritten by the transition matrices next)
    tm.begin(SGS_STAGE_INVERSE, s);
    // one batch of inverses: panels, grouped updates, unscramble
    auto inverses = [&](int half, hipStream_t st) -> hipError_t {
      const int off = half == 0 ? 0 : P0, cnt = half == 0 ? P0 : P - P0;
      const long long bstr = gj_brow_stride(n);
      const int ES = q.gj_super;
      for (size_t t = 0; t < q.gj_k.size(); ++t) {
        const int s = q.gj_s[t], k0 = q.gs_k[s], nbs = q.gs_nb[s];
        const bool defer = gj_deferred(q, half);
        const JobTable& inner = half == 0 ? q.jgj0[t] : q.jgj1[t];
        if (defer) HCHK(run_gemm(inner, st));  // the earlier panels' updates of this panel's columns
        HCHK(launch_gj_panel(q.Di + off * nn, nn, cnt, n, q.gj_k[t], q.gj_b[t],
                             q.gjE + (long long)off * n * ES, (long long)n * ES, ES,
                             q.gjB + off * bstr, bstr, ES, k0, k0 + nbs, q.gj_nb, defer ? 1 : 0,
                             q.piv + (long long)off * n, q.piv + (long long)(P + off) * n, q.logdet + off,
                             c->status, st));
        if (!defer) HCHK(run_gemm(inner, st));  // this panel's update of the whole super-panel
        if (t + 1 == q.gj_k.size() || q.gj_s[t + 1] != s) {  // the super-panel's last panel
          HCHK(run_gemm(half == 0 ? q.jgf0[s] : q.jgf1[s], st));
          HCHK(launch_gj_gather(q.Di + off * nn, nn, cnt, n, k0, nbs, q.piv + (long long)off * n,
                                q.gjB + off * bstr, bstr, st));
          HCHK(run_gemm(half == 0 ? q.jgs0[s] : q.jgs1[s], st));
        }
      }
      return launch_gj_unscramble(q.Di + off * nn, q.W + off * nn, nn, cnt, n, q.piv + (long long)off * n,
                                  q.piv + (long long)(P + off) * n, st);
    };
    // the pairs (a, b), 1 <= a < b, on the third stream from the start; the
    // pairs (0, a) on the main stream, then the phase chain forks from it
    // (with gj_first the third stream starts after the pairs (0, a),
    // together with the phase chain)
    const bool rest = P - P0 > 0;
    auto rest_inverses = [&]() -> hipError_t {
      HCHK(hipEventRecord(wk.ev_gj, s));
      HCHK(hipStreamWaitEvent(wk.s3, wk.ev_gj, 0));
      HCHK(launch_pair_sum(q.gam, n, q.pa + P0, q.pb + P0, P - P0, q.Di + P0 * nn, q.logdet + P0, wk.s3));
      HCHK(inverses(1, wk.s3));
      return hipEventRecord(wk.ev_gj_done, wk.s3);
    };
    if (rest && !q.gj_first) HCHK(rest_inverses());
    if (P0 > 0) {
      HCHK(launch_pair_sum(q.gam, n, q.pa, q.pb, P0, q.Di, q.logdet, s));
      HCHK(inverses(0, s));
    }
    if (rest && q.gj_first) HCHK(rest_inverses());
    if (fork) {
      // phases on the second stream, concurrent with the other inverses
      HCHK(hipEventRecord(wk.ev_fork, s));
      HCHK(hipStreamWaitEvent(wk.s2, wk.ev_fork, 0));
      hipStream_t s2 = wk.s2;
      tm.begin(SGS_STAGE_PHASE, s2);
      HCHK(run_gemm(q.jt1, s2));
      HCHK(run_gemm(q.jxr, s2));
      HCHK(launch_build_c(n, q.gam, q.T1, q.Xr, q.qa, q.qb, q.Q, q.pf.A0, s2));
      tm.end(SGS_STAGE_PHASE, s2);
      tm.begin(SGS_STAGE_PFAFFIAN, s2);
      HCHK(pf_run(q.pf, q.pfacc, c->status, s2));
      tm.end(SGS_STAGE_PFAFFIAN, s2);
      HCHK(hipEventRecord(wk.ev_join, s2));
    }
    if (rest) HCHK(hipStreamWaitEvent(s, wk.ev_gj_done, 0));
    tm.end(SGS_STAGE_INVERSE, s);
    // transition matrices
    tm.begin(SGS_STAGE_DELTA, s);
    HCHK(run_gemm(q.jdi, s));
    tm.end(SGS_STAGE_DELTA, s);
  }
  // Hamiltonian elements, Fock corrections, Y = Delta F
  tm.begin(SGS_STAGE_WICK, s);
  HamDev h{n, q.nnz_up, q.nq, q.M, q.up_k, q.up_l, q.up_v, q.q_idx, q.q_loc, q.q_val, q.e0,
           q.nw, q.w_idx, q.w_len, q.w_val, q.nfe, q.fe_ent, q.fe_off, q.fe_item};
  HCHK(launch_eps_fock(h, P, R, q.W, q.Di, q.gam, q.pa, q.pb, q.eps, q.Fc, s));
  SparseA sa{q.colptr, q.rowidx, q.colval, q.imp, q.impos, q.M};
  if (q.denseA) {
    HCHK(run_gemm(q.jya, s));
    HCHK(launch_fock_imp(sa, n, P, R, q.W, q.Di, q.gam, q.Fc, q.Y, q.Yd, s));
  } else {
    HCHK(launch_apply_fock(sa, n, P, R, q.W, q.Di, q.gam, q.Fc, q.Y, q.Yd, s));
  }
  tm.end(SGS_STAGE_WICK, s);
  if (P > 0 && fork) HCHK(hipStreamWaitEvent(s, wk.ev_join, 0));
  SolveArgs a;
  a.N = q.N; a.R = R; a.P = P;
  a.pidx = q.pidx; a.qidx = q.qidx; a.logdet = q.logdet; a.pfacc = q.pfacc; a.eps = q.eps;
  a.tab_la = o_la ? o_la : q.tab_la;
  a.tab_arg = o_arg ? o_arg : q.tab_arg;
  a.tab_eps = o_eps ? o_eps : q.tab_eps;
  a.Gt = q.Gt; a.ht = q.ht; a.lam = q.lam; a.lamt = q.lamt; a.coef = q.coef; a.E = q.E;
  a.energy_slot = energy_slot; a.status = c->status;
  a.slot_ctr = c->capturing ? c->ectr : nullptr;
  a.slot_stride = (int)c->pr.size();
  a.g_thr = c->opt.g_rel_threshold;
  a.weight = c->opt.weight;
  tm.begin(SGS_STAGE_SOLVE, s);
  HCHK(launch_solve(a, s));
  tm.end(SGS_STAGE_SOLVE, s);
  wk.owner = (int)(&q - c->pr.data());
  return hipSuccess;
}

static hipError_t update_stage(sgs_ctx* c, Prob& q, double dtau) {
  Worker& wk = c->wk[q.worker];
  hipStream_t s = wk.s;
  const int n = q.n, R = q.R;
  const long long nn = (long long)n * n;
  StageTimer& tm = q.worker == 0 && !c->capturing ? c->timer : c->mute;
  tm.begin(SGS_STAGE_FORCE, s);
  const int fmode = c->opt.precision == SGS_FP64 ? FORCE_FP64 : FORCE_FP32;
  const int ftile = q.force_tile ? q.force_tile : force_tile_default(n, fmode);
  if (q.force_seq) {
    // the elementwise terms after the dense products, on the same stream
    HCHK(launch_force(n, R, q.terms, q.coef, q.dG, q.dP, q.dgnorm, fmode, q.force_split, ftile, s));
    HCHK(launch_force_elem(n, R, q.terms, q.coef, q.Adense, q.impos, q.M, force_direct_y(fmode, ftile), q.dE, s));
    tm.end(SGS_STAGE_FORCE, s);
  } else {
    // the elementwise terms on the second stream (idle here: the phase chain
    // joined before the solve), concurrent with the dense products
    HCHK(hipEventRecord(wk.ev_f, s));
    HCHK(hipStreamWaitEvent(wk.s2, wk.ev_f, 0));
    HCHK(launch_force_elem(n, R, q.terms, q.coef, q.Adense, q.impos, q.M, force_direct_y(fmode, ftile), q.dE,
                           wk.s2));
    HCHK(hipEventRecord(wk.ev_fe, wk.s2));
    HCHK(launch_force(n, R, q.terms, q.coef, q.dG, q.dP, q.dgnorm, fmode, q.force_split, ftile, s));
    tm.end(SGS_STAGE_FORCE, s);
    HCHK(hipStreamWaitEvent(s, wk.ev_fe, 0));
  }
  HCHK(launch_force_join(q.dG, q.dP, q.dE, n, R, q.force_split, q.dgnorm, s));
  (void)nn;
  tm.begin(SGS_STAGE_PURIFY, s);
  if (q.expmap) {
    HCHK(run_gemm(q.jexp_p, s));
    HCHK(launch_exp_gen(q.nsX0, n, R, c->opt.exp_coef * dtau, q.nsQ, q.exrow, EXP_SMAX, q.nsctl, q.expar,
                        c->status, s));
    HCHK(run_gemm(q.jexp_y, s));
    HCHK(run_gemm(q.jexp_z, s));
    HCHK(launch_exp_b3(q.nsX1, q.dG, n, R, q.excf, q.ex0, q.ex1, s));
    for (int h = 0; h < 3; ++h) HCHK(run_gemm(q.jexp_h[h], s));
    HCHK(run_gemm(q.jexp_r, s));
    for (int it = 0; it < EXP_SMAX; ++it)
      HCHK(launch_gemm(q.jexp_sq[it & 1].dev, q.jexp_sq[it & 1].xm, false, s, q.nsctl, it, nullptr, 0.0, nullptr));
    HCHK(launch_exp_pick(q.nsX0, q.ex0, n, R, q.nsctl, s));
    HCHK(run_gemm(q.jexp_q, s));
    HCHK(run_gemm(q.jexp_g, s));
    HCHK(launch_exp_skew_diag(q.gam, n, R, s));
    tm.end(SGS_STAGE_PURIFY, s);
    return hipSuccess;
  }
  const int maxit = c->opt.purify_iters;
  unsigned long long* rs = q.nsres;
  HCHK(launch_euler(q.gam, q.dG, dtau, n, R, q.nsX0, q.nsctl, rs, maxit * (R + 2), q.dgnorm, s));
  const double thr = std::min(1e-8, std::sqrt(c->opt.purify_tol));
  for (int it = 0; it < maxit; ++it) {
    const int par = it & 1;
    // Q = X X with max|Q + 1| of state mu into rs[it (R + 2) + 2 + mu] (the
    // job's gate); then X' = X (3 + Q) / 2, which marks this iteration as
    // state mu's last when that residual is below thr
    unsigned long long* ri = rs + (size_t)it * (R + 2);
    HCHK(launch_gemm(q.jnsq[par].dev, q.jnsq[par].xm, false, s, q.nsctl, it, nullptr, 0.0, ri));
    HCHK(launch_gemm(q.jnsx[par].dev, q.jnsx[par].xm, false, s, q.nsctl, it, ri, thr, nullptr));
  }
  HCHK(launch_finalize(q.nsX0, q.nsX1, n, R, q.gam, q.nsctl, c->opt.purify_iters, c->status, s));
  tm.end(SGS_STAGE_PURIFY, s);
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

void sgs_default_options(sgs_options* o) {
  if (!o) return;
  o->precision = SGS_FP64;
  o->weight = SGS_W_PRINTED;
  o->g_rel_threshold = 1e-12;
  o->purify_tol = 1e-12;
  o->purify_iters = 24;
  o->streams = DEFAULT_WORKERS;
  o->update = SGS_UPD_EULER;
  o->exp_coef = 0.25;
  o->tune = nullptr;
  o->ntune = 0;
  o->graph = 0;
}

static int check_options(const sgs_options& o) {
  if (o.precision != SGS_FP64 && o.precision != SGS_FP32_FORCE) return SGS_EINVAL;
  if (o.weight != SGS_W_PRINTED && o.weight != SGS_W_UNIT) return SGS_EINVAL;
  if (!(o.g_rel_threshold > 0.0 && o.g_rel_threshold < 1.0)) return SGS_EINVAL;
  if (!(o.purify_tol > 0.0) || o.purify_iters < 1 || o.purify_iters > 64) return SGS_EINVAL;
  if (o.streams < 1 || o.streams > MAX_WORKERS) return SGS_EINVAL;
  if (o.update != SGS_UPD_EULER && o.update != SGS_UPD_EXP) return SGS_EINVAL;
  if (!(o.exp_coef > 0.0 && o.exp_coef <= 1e6)) return SGS_EINVAL;
  if (o.ntune < 0 || o.ntune > 64 || (o.ntune > 0 && !o.tune)) return SGS_EINVAL;
  if (o.graph != 0 && o.graph != 1) return SGS_EINVAL;
  for (int i = 0; i < o.ntune; ++i) {
    const sgs_tune& t = o.tune[i];
    if (t.n_max < 2 || (i > 0 && t.n_max <= o.tune[i - 1].n_max)) return SGS_EINVAL;
    if (t.gj_super > GJ_SUPER_MAX || t.gj_first > 2 || t.pf_super > PF_SUPER_MAX ||
        t.force_split > FORCE_SPLIT_MAX || t.force_elem > 2 ||
        (t.force_tile != 0 && t.force_tile != 64 && t.force_tile != 128) || t.gj_defer > 3)
      return SGS_EINVAL;
  }
  return SGS_OK;
}

int sgs_workspace_bytes(const sgs_problem* probs, int32_t nprob, const sgs_options* opt, size_t* bytes) {
  if (!probs || nprob < 1 || nprob > 1024 || !bytes) return SGS_EINVAL;
  sgs_options o;
  sgs_default_options(&o);
  if (opt) o = *opt;
  int rc = check_options(o);
  if (rc) return rc;
  for (int p = 0; p < nprob; ++p)
    if ((rc = check_problem(probs[p]))) return rc;
  std::vector<Prob> pr;
  *bytes = plan(pr, probs, nprob, nullptr, device_lds_max(), o.graph ? 1 : o.streams, o.update == SGS_UPD_EXP, o);
  return SGS_OK;
}

int sgs_init(sgs_ctx** out, const sgs_problem* probs, int32_t nprob, double* gamma, void* workspace,
             size_t ws_bytes, const sgs_options* opt, void* stream) {
  if (!out || !probs || nprob < 1 || nprob > 1024 || !gamma || !workspace) return SGS_EINVAL;
  if (((uintptr_t)workspace) & 255) return SGS_EINVAL;
  *out = nullptr;
  sgs_options o;
  sgs_default_options(&o);
  if (opt) o = *opt;
  int rc = check_options(o);
  if (rc) return rc;
  for (int p = 0; p < nprob; ++p)
    if ((rc = check_problem(probs[p]))) return rc;
  sgs_ctx* c = new sgs_ctx();
  c->opt = o;
  c->s = (hipStream_t)stream;
  c->lds_max = device_lds_max();
  int nworkers = 1;
  // graph mode: one worker stream (the capture of several workers' fork and
  // join ended the process in sgs_step on the device tested, cause not
  // found; each problem still runs its inverses and phase chain on streams
  // of its own inside the graph)
  const size_t need = plan(c->pr, probs, nprob, (char*)workspace, c->lds_max, c->opt.graph ? 1 : c->opt.streams,
                           c->opt.update == SGS_UPD_EXP, c->opt, &c->obs, &nworkers);
  c->opt.tune = nullptr;  // read above; the caller's table need not outlive init
  c->opt.ntune = 0;
  if (ws_bytes < need) { delete c; return SGS_EWORKSPACE; }
  c->status = (int*)workspace;
  c->ectr = (int*)workspace + 16;
  c->ering = c->obs.ering;
  double* g = gamma;
  for (int p = 0; p < nprob; ++p) {
    c->pr[p].gam = g;
    g += (long long)c->pr[p].R * c->pr[p].n * c->pr[p].n;
  }
  size_t lds_gj = 0, lds_solve = 0;
  for (auto& q : c->pr) {
    lds_gj = std::max(lds_gj, gj_panel_lds_bytes(q.n, q.gj_super - q.gj_nb, q.gj_nb));
    lds_solve = std::max(lds_solve, solve_lds_bytes(q.R));
  }
  int nmax = 2;
  for (auto& q : c->pr) nmax = std::max(nmax, q.n);
  if (set_gj_lds_limit(lds_gj) != hipSuccess || set_solve_lds_limit(lds_solve) != hipSuccess ||
      set_ren_lds_limit() != hipSuccess || set_pf_sign_lds_limit(nmax) != hipSuccess ||
      set_force_lds_limit() != hipSuccess) {
    delete c;
    return SGS_EHIP;
  }
  for (int p = 0; p < nprob; ++p)
    if ((rc = build_tables(c->pr[p], probs[p]))) { delete c; return rc; }
  // worker streams (default priority, non-blocking, forked from and joined to
  // the context's stream), each with a second stream for its phase chain and
  // a third for the other pairs' inverses, and the fork / join events
  c->wk.assign(nworkers, Worker());
  if (hipEventCreateWithFlags(&c->ev_start, hipEventDisableTiming) != hipSuccess) { delete c; return SGS_EHIP; }
  for (int w = 0; w < nworkers; ++w) {
    Worker& k = c->wk[w];
    if (hipStreamCreateWithFlags(&k.s, hipStreamNonBlocking) != hipSuccess) { delete c; return SGS_EHIP; }
    k.own_s = true;
    if (hipStreamCreateWithFlags(&k.s2, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&k.s3, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&k.ev_gj, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&k.ev_gj_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&k.ev_f, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&k.ev_fe, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&k.ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&k.ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&k.ev_done, hipEventDisableTiming) != hipSuccess) { delete c; return SGS_EHIP; }
  }
  if (hipMemsetAsync(c->status, 0, sizeof(int), c->s) != hipSuccess) { delete c; return SGS_EHIP; }
  // validate the covariance matrices: skew, Gamma^2 = -1
  for (auto& q : c->pr) {
    const long long nn = (long long)q.n * q.n;
    unsigned long long hv = 0;
    if (launch_skew_resid(q.gam, q.n, q.R * nn, q.resid, c->s) != hipSuccess ||
        hipMemcpyAsync(&hv, q.resid, sizeof(hv), hipMemcpyDeviceToHost, c->s) != hipSuccess ||
        hipStreamSynchronize(c->s) != hipSuccess) { delete c; return SGS_EHIP; }
    double d;
    std::memcpy(&d, &hv, sizeof(d));
    if (!(d <= 1e-12)) { delete c; return SGS_ENOTSKEW; }
    if (run_gemm(q.jval, c->s) != hipSuccess || launch_ns_resid(q.nsQ, q.n, q.R * nn, q.resid, c->s) != hipSuccess ||
        hipMemcpyAsync(&hv, q.resid, sizeof(hv), hipMemcpyDeviceToHost, c->s) != hipSuccess ||
        hipStreamSynchronize(c->s) != hipSuccess) { delete c; return SGS_EHIP; }
    std::memcpy(&d, &hv, sizeof(d));
    if (!(d <= 1e-10)) { delete c; return SGS_ENOTPURE; }
    // parity: Pf Gamma = +1 for every state (the overlap phases of Sec. II.B
    // are taken for even states generated from the vacuum)
    double* signs = reinterpret_cast<double*>(q.nsres);
    std::vector<double> hs(q.R, 0.0);
    if (launch_pf_sign(q.gam, q.nsX0, q.n, q.R, signs, c->s) != hipSuccess ||
        hipMemcpyAsync(hs.data(), signs, q.R * sizeof(double), hipMemcpyDeviceToHost, c->s) != hipSuccess ||
        hipStreamSynchronize(c->s) != hipSuccess) { delete c; return SGS_EHIP; }
    for (double v : hs)
      if (v != 1.0) { delete c; return SGS_EPARITY; }
  }
  *out = c;
  return SGS_OK;
}

int sgs_pair_eval(sgs_ctx* c, double* log_abs_G, double* arg_G, double* eps, double* delta) {
  if (!c) return SGS_EINVAL;
  long long off = 0, doff = 0;
  if (c->fork() != hipSuccess) return SGS_EHIP;
  for (auto& q : c->pr) {
    const int RR = q.R * q.R;
    if (pair_stage(c, q, nullptr, log_abs_G ? log_abs_G + off : nullptr, arg_G ? arg_G + off : nullptr,
                   eps ? eps + 2 * off : nullptr) != hipSuccess)
      return SGS_EHIP;
    const long long tot = (long long)q.P * q.n * q.n;
    // the worker's scratch holds this problem's transition matrices until its
    // next problem: copied out on the worker's stream
    if (delta && launch_delta_out(q.W, q.Di, tot, delta + 2 * doff, c->wk[q.worker].s) != hipSuccess)
      return SGS_EHIP;
    off += RR;
    doff += tot;
  }
  if (c->join() != hipSuccess) return SGS_EHIP;
  c->evaluated = true;
  return SGS_OK;
}

// One step of every problem, enqueued (or captured) on the context's streams.
static hipError_t enqueue_step(sgs_ctx* c, double dtau, double* energies, long long k) {
  const int np = (int)c->pr.size();
  if (c->fork() != hipSuccess) return hipErrorUnknown;
  for (int p = 0; p < np; ++p) {
    Prob& q = c->pr[p];
    double* slot = c->capturing ? c->ering + p : (energies ? energies + k * np + p : nullptr);
    HCHK(pair_stage(c, q, slot, nullptr, nullptr, nullptr));
    HCHK(update_stage(c, q, dtau));
  }
  return c->join();
}

// Graph replay: one step of every problem captured once (again when dtau
// changes), then launched nsteps times; the solve writes each replay's
// energies at a device counter into the ring, which is copied out in chunks.
static int step_graph(sgs_ctx* c, double dtau, int nsteps, double* energies) {
  const int np = (int)c->pr.size();
  if (!c->gexec || c->gdtau != dtau) {
    if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    if (!c->gs && hipStreamCreateWithFlags(&c->gs, hipStreamNonBlocking) != hipSuccess) return SGS_EHIP;
    hipGraph_t g = nullptr;
    // the private stream stands in for the context's stream and worker 0's
    // while the step is captured; the graph is launched on the context's
    hipStream_t s0 = c->s, w0 = c->wk[0].s;
    c->s = c->gs;
    c->wk[0].s = c->gs;
    hipError_t e = hipStreamBeginCapture(c->gs, hipStreamCaptureModeThreadLocal);
    const bool began = e == hipSuccess;
    if (began) {
      c->capturing = true;
      e = enqueue_step(c, dtau, nullptr, 0);
      if (e == hipSuccess) e = launch_bump_counter(c->ectr, c->gs);
      c->capturing = false;
    }
    const hipError_t e2 = began ? hipStreamEndCapture(c->gs, &g) : e;
    c->s = s0;
    c->wk[0].s = w0;
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return SGS_EHIP;
    }
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { c->gexec = nullptr; return SGS_EHIP; }
    c->gdtau = dtau;
  }
  for (int k0 = 0; k0 < nsteps; k0 += GRAPH_RING) {
    const int kn = std::min(GRAPH_RING, nsteps - k0);
    if (launch_set_counter(c->ectr, 0, c->s) != hipSuccess) return SGS_EHIP;
    for (int k = 0; k < kn; ++k)
      if (hipGraphLaunch(c->gexec, c->s) != hipSuccess) return SGS_EHIP;
    if (energies && hipMemcpyAsync(energies + (long long)k0 * np, c->ering, (size_t)kn * np * sizeof(double),
                                   hipMemcpyDeviceToDevice, c->s) != hipSuccess)
      return SGS_EHIP;
  }
  return SGS_OK;
}

int sgs_step(sgs_ctx* c, double dtau, int32_t nsteps, double* energies) {
  if (!c || nsteps < 0 || !std::isfinite(dtau) || dtau <= 0.0) return SGS_EINVAL;
  const int np = (int)c->pr.size();
  if (c->opt.graph && nsteps > 0) {
    const int rc = step_graph(c, dtau, nsteps, energies);
    if (rc != SGS_OK) return rc;
    c->evaluated = false;
    for (auto& w : c->wk) w.owner = -1;
    return SGS_OK;
  }
  // independent problems run concurrently, one stream per worker
  if (c->fork() != hipSuccess) return SGS_EHIP;
  for (int k = 0; k < nsteps; ++k)
    for (int p = 0; p < np; ++p) {
      Prob& q = c->pr[p];
      if (pair_stage(c, q, energies ? energies + (long long)k * np + p : nullptr, nullptr, nullptr, nullptr) !=
          hipSuccess)
        return SGS_EHIP;
      if (update_stage(c, q, dtau) != hipSuccess) return SGS_EHIP;
    }
  if (c->join() != hipSuccess) return SGS_EHIP;
  if (nsteps > 0) {
    c->evaluated = false;
    for (auto& w : c->wk) w.owner = -1;
  }
  return SGS_OK;
}

int sgs_energy(sgs_ctx* c, double* E, double* lambda) {
  if (!c || !E) return SGS_EINVAL;
  if (!c->evaluated) {
    if (c->fork() != hipSuccess) return SGS_EHIP;
    for (auto& q : c->pr)
      if (pair_stage(c, q, nullptr, nullptr, nullptr, nullptr) != hipSuccess) return SGS_EHIP;
    if (c->join() != hipSuccess) return SGS_EHIP;
    c->evaluated = true;
  }
  long long off = 0;
  for (size_t p = 0; p < c->pr.size(); ++p) {
    Prob& q = c->pr[p];
    if (hipMemcpyAsync(E + p, q.E, sizeof(double), hipMemcpyDeviceToDevice, c->s) != hipSuccess) return SGS_EHIP;
    if (lambda && hipMemcpyAsync(lambda + 2 * off, q.lam, 2 * q.R * sizeof(double), hipMemcpyDeviceToDevice, c->s) !=
                      hipSuccess)
      return SGS_EHIP;
    off += q.R;
  }
  return SGS_OK;
}

// The scratch tables (W, Im Delta) of problem p for its current states; other
// problems of the same worker may have overwritten them since.
static hipError_t ensure_tables(sgs_ctx* c, int p) {
  Prob& q = c->pr[p];
  if (c->evaluated && c->wk[q.worker].owner == p) return hipSuccess;
  hipError_t e = c->fork();
  if (e == hipSuccess) e = pair_stage(c, q, nullptr, nullptr, nullptr, nullptr);
  if (e == hipSuccess) e = c->join();
  return e;
}

// ---------------------------------------------------------------------------
// Renyi-2 entropy (App. B)
// ---------------------------------------------------------------------------
constexpr double REN_KAPPA_MAX = 1e6;  // split form only with a block better conditioned than this
constexpr size_t REN_BATCH_BYTES = (size_t)1 << 30;  // device memory of one Pfaffian batch, about
constexpr int REN_BATCH_MAX = 512;  // matrices per batch

// bytes of a Pfaffian batch of B matrices of order m with its job tables and
// results (3 doubles per matrix)
static size_t ren_batch_bytes(int m, int B) {
  Arena probe{nullptr, 0};
  PfBatch b;
  b.m = m; b.B = B; b.super = pf_super_default(m);
  pf_carve(b, probe);
  pf_schedule(b, probe);
  probe.take<double>(3 * (size_t)B);
  return probe.off + 256;
}

static int ren_batch_size(int m, int want) {
  const size_t one = ren_batch_bytes(m, 1);
  const long long fit = (long long)(REN_BATCH_BYTES / one);
  return (int)std::max(1LL, std::min<long long>(fit, std::min(REN_BATCH_MAX, std::max(1, want))));
}

static void ren_batch_carve(PfBatch& b, int m, int B, double** acc, Arena& ar) {
  b.m = m; b.B = B; b.super = pf_super_default(m);
  pf_carve(b, ar);
  pf_schedule(b, ar);
  *acc = ar.take<double>(3 * (size_t)B);
}

// S_2 of problem q into out (device).  One representative (p, q) per orbit of
// the exchange and conjugation symmetries, p <= q over ordered pairs
// p = a R + b and orbit size w = (p == q ? 1 : 2) ((p*, q*) == (p, q) ? 1 : 2).
// Waits for the stream before returning.
static int renyi2(sgs_ctx* c, Prob& q, int nA, int method, double* out) {
  const int R = q.R, RR = R * R, nu = R * (R + 1) / 2;
  const hipStream_t st = c->s;
  ObsState s{q.n, R, q.gam, q.W, q.Di, q.lam, q.Gt, q.pidx};
  std::vector<RenTerm> reps;
  auto conj_pair = [R](int p) { return (p % R) * R + p / R; };
  for (int p = 0; p < RR; ++p)
    for (int r = p; r < RR; ++r) {
      int cp = conj_pair(p), cr = conj_pair(r);
      if (cp > cr) std::swap(cp, cr);
      if (cp < p || (cp == p && cr < r)) continue;  // (p*, r*) represents this orbit
      const int w = (p == r ? 1 : 2) * (cp == p && cr == r ? 1 : 2);
      reps.push_back({p, r, 0, w});
    }
  const int nterm = (int)reps.size();
  const bool lds = method == SGS_REN_AUTO && nA <= REN_LDS_MAX_NA;
  const bool split = !lds && method != SGS_REN_BLOCK;
  const long long mm = (long long)nA * nA;
  const int B1 = split ? ren_batch_size(nA, std::max(nu, nterm)) : 0;
  const int B2 = lds ? 0 : ren_batch_size(2 * nA, nterm);
  // device memory: status, terms, term values, classes, inverses, condition
  // numbers, the classes' Pfaffians, then the two batches
  auto layout = [&](Arena& ar, int** status, RenTerm** dterms, double** tval, int2** uxy, double** inv,
                    double** kappa, double** uacc, PfBatch* b1, double** acc1, PfBatch* b2, double** acc2) {
    *status = ar.take<int>(64);
    *dterms = ar.take<RenTerm>(nterm);
    *tval = ar.take<double>(nterm);
    *uxy = ar.take<int2>(nu);
    *inv = split ? ar.take<double>((size_t)nu * 2 * mm) : nullptr;
    *kappa = ar.take<double>(nu);
    *uacc = ar.take<double>(3 * (size_t)nu);
    if (B1) ren_batch_carve(*b1, nA, B1, acc1, ar);
    if (B2) ren_batch_carve(*b2, 2 * nA, B2, acc2, ar);
  };
  int* status; RenTerm* dterms; double *tval, *inv, *kappa, *uacc, *acc1 = nullptr, *acc2 = nullptr;
  int2* uxy;
  PfBatch b1, b2;
  {
    Arena probe{nullptr, 0};
    layout(probe, &status, &dterms, &tval, &uxy, &inv, &kappa, &uacc, &b1, &acc1, &b2, &acc2);
    const size_t need = probe.off + 256;
    // the previous call's kernels may still read the job tables
    if (hipStreamSynchronize(st) != hipSuccess) return SGS_EHIP;
    if (c->ren_bytes < need) {
      if (c->ren) (void)hipFree(c->ren);
      c->ren = nullptr;
      c->ren_bytes = 0;
      if (hipMalloc(&c->ren, need) != hipSuccess) return SGS_EHIP;
      c->ren_bytes = need;
    }
    Arena ar{(char*)c->ren, 0};
    layout(ar, &status, &dterms, &tval, &uxy, &inv, &kappa, &uacc, &b1, &acc1, &b2, &acc2);
  }
  if (lds) {
    if (hipMemcpy(dterms, reps.data(), reps.size() * sizeof(RenTerm), hipMemcpyHostToDevice) != hipSuccess ||
        launch_ren_lds(s, nA, dterms, nterm, tval, st) != hipSuccess ||
        launch_ren_sum(tval, nterm, out, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      return SGS_EHIP;
    return SGS_OK;
  }
  // classes: Pf(K_u), K_u^{-1} and its condition number
  std::vector<double> kap(nu, __builtin_huge_val());
  if (split) {
    std::vector<int2> cls;
    for (int x = 0; x < R; ++x)
      for (int y = x; y < R; ++y) cls.push_back(make_int2(x, y));
    if (hipMemcpy(uxy, cls.data(), cls.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess ||
        pf_jobs(b1) != hipSuccess)
      return SGS_EHIP;
    for (int u0 = 0; u0 < nu; u0 += B1) {
      const int nb = std::min(B1, nu - u0);
      if (launch_ren_blocks(s, nA, uxy, u0, B1, nu, b1.A0, inv, st) != hipSuccess ||
          pf_run(b1, acc1, status, st) != hipSuccess ||
          hipMemcpyAsync(uacc + 3 * (size_t)u0, acc1, 3 * (size_t)nb * sizeof(double), hipMemcpyDeviceToDevice,
                         st) != hipSuccess)
        return SGS_EHIP;
    }
    if (launch_ren_inverse(inv, nu, nA, kappa, st) != hipSuccess ||
        hipMemcpyAsync(kap.data(), kappa, nu * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SGS_EHIP;
  }
  // split terms first (block q inverted), then block-form terms
  const double kmax = method == SGS_REN_SPLIT ? __builtin_huge_val() : REN_KAPPA_MAX;
  auto cls_of = [R](int p) {
    int x = p / R, y = p % R;
    if (x > y) std::swap(x, y);
    return x * (2 * R - x + 1) / 2 + (y - x);
  };
  std::vector<RenTerm> order;
  order.reserve(nterm);
  for (RenTerm t : reps) {
    const double kp = kap[cls_of(t.p)], kq = kap[cls_of(t.q)];
    if (split && std::min(kp, kq) < kmax) {
      if (kp < kq) std::swap(t.p, t.q);  // invert the better-conditioned block
      t.split = 1;
      order.push_back(t);
    }
  }
  const int nsplit = (int)order.size();
  for (const RenTerm& t : reps) {
    const double kp = kap[cls_of(t.p)], kq = kap[cls_of(t.q)];
    if (!(split && std::min(kp, kq) < kmax)) order.push_back(t);
  }
  if (hipMemcpy(dterms, order.data(), order.size() * sizeof(RenTerm), hipMemcpyHostToDevice) != hipSuccess)
    return SGS_EHIP;
  for (int t0 = 0; t0 < nsplit; t0 += B1) {
    const int cnt = std::min(B1, nsplit - t0);
    if (launch_ren_terms(s, nA, 1, dterms, t0, cnt, B1, inv, b1.A0, st) != hipSuccess ||
        pf_run(b1, acc1, status, st) != hipSuccess ||
        launch_ren_combine(s, nA, 1, dterms, t0, cnt, acc1, uacc, tval, st) != hipSuccess)
      return SGS_EHIP;
  }
  if (nsplit < nterm) {
    if (pf_jobs(b2) != hipSuccess) return SGS_EHIP;
    for (int t0 = nsplit; t0 < nterm; t0 += B2) {
      const int cnt = std::min(B2, nterm - t0);
      if (launch_ren_terms(s, nA, 0, dterms, t0, cnt, B2, nullptr, b2.A0, st) != hipSuccess ||
          pf_run(b2, acc2, status, st) != hipSuccess ||
          launch_ren_combine(s, nA, 0, dterms, t0, cnt, acc2, uacc, tval, st) != hipSuccess)
        return SGS_EHIP;
    }
  }
  if (launch_ren_sum(tval, nterm, out, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return SGS_EHIP;
  return SGS_OK;
}

int sgs_observables(sgs_ctx* c, int32_t kind, const int32_t* iargs, int32_t niargs, const double* dargs,
                    int32_t ndargs, double* out) {
  if (!c || !iargs || niargs < 1 || !out) return SGS_EINVAL;
  const int p = iargs[0];
  if (p < 0 || p >= (int)c->pr.size()) return SGS_EINVAL;
  Prob& q = c->pr[p];
  const int n = q.n;
  if (kind == SGS_OBS_POLY) {
    if (niargs < 3) return SGS_EINVAL;
    const int npoly = iargs[1], nterm = iargs[2];
    if (npoly < 1 || npoly > OBS_MAX_POLY || nterm < 0 || nterm > OBS_MAX_TERMS) return SGS_EINVAL;
    if (niargs != 3 + 6 * nterm || ndargs != 2 * nterm || (nterm > 0 && !dargs)) return SGS_EINVAL;
    // validate and sort the terms by polynomial (counting sort, stable)
    std::vector<int> cnt(npoly + 1, 0);
    for (int t = 0; t < nterm; ++t) {
      const int* w = iargs + 3 + 6 * t;
      const int pi = w[0], m = w[1];
      if (pi < 0 || pi >= npoly || (m != 0 && m != 2 && m != 4)) return SGS_EINVAL;
      for (int u = 0; u < 4; ++u) {
        if (u < m) {
          if (w[2 + u] < 0 || w[2 + u] >= n || (u > 0 && w[2 + u] <= w[1 + u])) return SGS_EINVAL;
        } else if (w[2 + u] != -1) {
          return SGS_EINVAL;
        }
      }
      ++cnt[pi + 1];
    }
    for (int i = 0; i < npoly; ++i) cnt[i + 1] += cnt[i];
    std::vector<int> rows(6 * (size_t)std::max(1, nterm)), pos(cnt.begin(), cnt.end() - 1);
    std::vector<double> coef(2 * (size_t)std::max(1, nterm));
    for (int t = 0; t < nterm; ++t) {
      const int* w = iargs + 3 + 6 * t;
      const int d = pos[w[0]]++;
      for (int u = 0; u < 6; ++u) rows[6 * (size_t)d + u] = w[u];
      coef[2 * (size_t)d] = dargs[2 * t];
      coef[2 * (size_t)d + 1] = dargs[2 * t + 1];
    }
    if (ensure_tables(c, p) != hipSuccess) return SGS_EHIP;
    // pageable sources: the copies complete (into staging) before return
    if (hipMemcpyAsync(c->obs.rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice, c->s) != hipSuccess ||
        hipMemcpyAsync(c->obs.coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, c->s) != hipSuccess ||
        hipMemcpyAsync(c->obs.off, cnt.data(), cnt.size() * sizeof(int), hipMemcpyHostToDevice, c->s) != hipSuccess)
      return SGS_EHIP;
    ObsState s{n, q.R, q.gam, q.W, q.Di, q.lam, q.Gt, q.pidx};
    if (launch_obs_poly(s, c->obs.rows, c->obs.coef, c->obs.off, npoly, out, c->s) != hipSuccess) return SGS_EHIP;
    // the host vectors must outlive the copies
    if (hipStreamSynchronize(c->s) != hipSuccess) return SGS_EHIP;
    return SGS_OK;
  }
  if (kind == SGS_OBS_VARIANCE) {
    if (niargs != 1) return SGS_EINVAL;
    if (q.R > 32 || q.nw > 0) return SGS_EINVAL;
    if (ensure_tables(c, p) != hipSuccess) return SGS_EHIP;
    ObsState s{n, q.R, q.gam, q.W, q.Di, q.lam, q.Gt, q.pidx};
    VarHam h{q.Adense, q.nnz_up, q.up_k, q.up_l, q.up_v, q.colptr, q.rowidx, q.colval, q.nq, q.q_idx, q.q_val};
    if (launch_variance(s, h, q.e0, q.a2, c->obs.vpart, out, c->s) != hipSuccess) return SGS_EHIP;
    return SGS_OK;
  }
  if (kind == SGS_OBS_RENYI2) {
    if (niargs != 2 && niargs != 3) return SGS_EINVAL;
    const int nA = iargs[1], method = niargs == 3 ? iargs[2] : SGS_REN_AUTO;
    if (nA < 2 || nA > REN_MAX_NA || (nA & 1) || nA > n) return SGS_EINVAL;
    if (method < SGS_REN_AUTO || method > SGS_REN_SPLIT) return SGS_EINVAL;
    if (ensure_tables(c, p) != hipSuccess) return SGS_EHIP;
    return renyi2(c, q, nA, method, out);
  }
  return SGS_EINVAL;
}

int sgs_rotate(const double* Q, const double* gamma, double* work, double* gamma_out, int32_t n, void* stream) {
  if (!Q || !gamma || !work || !gamma_out || n < 2 || n > 8192 || (n & 1)) return SGS_EINVAL;
  return launch_rotate(Q, gamma, work, gamma_out, n, (hipStream_t)stream) == hipSuccess ? SGS_OK : SGS_EHIP;
}

int sgs_rotate_noalloc(const double* Q, const double* gamma, double* gamma_out, int32_t n, void* stream) {
  if (!Q || !gamma || !gamma_out || n < 2 || (n & 1)) return SGS_EINVAL;
  if (n > ROTATE_SCRATCH_N) return SGS_ESCRATCH;
  double* work = nullptr;
  if (rotate_scratch(&work) != hipSuccess) return SGS_EHIP;
  return launch_rotate(Q, gamma, work, gamma_out, n, (hipStream_t)stream) == hipSuccess ? SGS_OK : SGS_EHIP;
}

int sgs_status(sgs_ctx* c) {
  if (!c) return SGS_EINVAL;
  int st = 0;
  if (hipStreamSynchronize(c->s) != hipSuccess) return SGS_EHIP;
  if (hipMemcpy(&st, c->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SGS_EHIP;
  const int zero = 0;
  if (hipMemcpy(c->status, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return SGS_EHIP;
  return st;
}

int sgs_set_timing(sgs_ctx* c, int32_t enable) {
  if (!c) return SGS_EINVAL;
  c->timer.on = enable != 0;
  return SGS_OK;
}

int sgs_stage_times(sgs_ctx* c, double* ms, int32_t* launches, int32_t nstage) {
  if (!c || nstage < 0 || (nstage > 0 && (!ms || !launches))) return SGS_EINVAL;
  if (hipStreamSynchronize(c->s) != hipSuccess) return SGS_EHIP;
  for (int i = 0; i < nstage; ++i) { ms[i] = 0.0; launches[i] = 0; }
  for (auto& r : c->timer.rec) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return SGS_EHIP;
    if (r.stage >= 0 && r.stage < nstage) { ms[r.stage] += t; launches[r.stage] += 1; }
  }
  c->timer.rec.clear();
  c->timer.used = 0;
  return SGS_OK;
}

void sgs_destroy(sgs_ctx* c) { delete c; }

const char* sgs_strerror(int code) {
  switch (code) {
    case SGS_OK: return "ok";
    case SGS_EINVAL: return "invalid argument";
    case SGS_ENOTSKEW: return "covariance matrix is not skew-symmetric";
    case SGS_ENOTPURE: return "covariance matrix is not pure (Gamma^2 != -1)";
    case SGS_EPARITY: return "odd-parity covariance matrix";
    case SGS_ESINGULAR: return "singular pair matrix or Gram matrix";
    case SGS_ENOCONV: return "purification or eigen-solve did not converge";
    case SGS_EHIP: return "HIP runtime error";
    case SGS_ESTATE: return "call out of order";
    case SGS_EWORKSPACE: return "workspace too small";
    case SGS_ERANGE: return "exponential-map generator too large (or not finite)";
    case SGS_ESCRATCH: return "size above the allocation-free entry point's fixed scratch";
    default: return "unknown error";
  }
}

}  // extern "C"
