// C ABI entry points (include/tucker.h): argument validation, workspace
// carving and the launch sequences of each call.  Nothing here allocates,
// frees or synchronises; every launch goes to the caller's stream.
#include <math.h>
#include <string.h>

#include <mutex>

#include "tk_internal.h"

namespace tk {

Geom make_geom(const tk_problem* p) {
  Geom g;
  memset(&g, 0, sizeof(g));
  g.order = p->order;
  int64_t off = 0, qoff = 0, roff = 0, numel = 1, d = 1;
  int32_t soff = 0;
  for (int n = 0; n < p->order; ++n) {
    g.soff[n] = soff;
    soff += p->ranks[n];
    g.ranks[n] = p->ranks[n];
    g.dims[n] = p->dims[n];
    g.off[n] = off;
    g.qoff[n] = qoff;
    g.roff[n] = roff;
    off += p->dims[n];
    qoff += p->dims[n] * p->ranks[n];
    roff += static_cast<int64_t>(p->ranks[n]) * p->ranks[n];
    numel *= p->dims[n];
    d *= p->ranks[n];
  }
  int64_t stride = 1;
  for (int n = p->order - 1; n >= 0; --n) {
    g.strides[n] = stride;
    stride *= p->dims[n];
  }
  g.total_rows = off;
  g.total_q = qoff;
  g.total_rr = roff;
  g.numel = numel;
  g.d = d;
  g.sum_r = soff;
  g.last = p->order - 1;
  while (g.last > 0 && p->ranks[g.last] < 2) --g.last;
  if (p->ranks[g.last] < 2) g.last = p->order - 1;
  return g;
}

// Geometry of the augmented row tables: mode n gets R_n more rows (the ridge
// rows' whitened digits), so qoff and total_q cover I_n + R_n rows per mode.
// Only the table offsets and ranks of this geometry are used.
Geom make_geom_aug(const tk_problem* p) {
  tk_problem q = *p;
  for (int n = 0; n < p->order; ++n) q.dims[n] += p->ranks[n];
  return make_geom(&q);
}

namespace {

constexpr int64_t kMaxD = 16384;

tk_status check_shape(const tk_problem* p) {
  if (!p) return TK_E_ARG;
  if (p->order < 1 || p->order > kMaxOrder) return TK_E_SHAPE;
  int64_t numel = 1, d = 1, sum_r = 0;
  for (int n = 0; n < p->order; ++n) {
    sum_r += p->ranks[n] > 0 ? p->ranks[n] : 0;
    if (sum_r > kMaxSumR) return TK_E_SHAPE;
    if (p->dims[n] < 1 || p->dims[n] > (int64_t(1) << 31) - 1) return TK_E_SHAPE;
    if (p->ranks[n] < 1 || p->ranks[n] > kMaxRank) return TK_E_SHAPE;
    if (p->ranks[n] > p->dims[n]) return TK_E_SHAPE;
    if (numel > (int64_t(1) << 62) / p->dims[n]) return TK_E_SHAPE;
    numel *= p->dims[n];
    d *= p->ranks[n];
    if (d > kMaxD) return TK_E_SHAPE;
  }
  if (p->dtype != TK_F64 && p->dtype != TK_F32) return TK_E_DTYPE;
  if (!(p->lambda >= 0.0) || !isfinite(p->lambda)) return TK_E_ARG;
  return TK_OK;
}

tk_status check_problem(const tk_problem* p, bool need_x) {
  tk_status s = check_shape(p);
  if (s != TK_OK) return s;
  if (need_x && !p->X) return TK_E_ARG;
  for (int n = 0; n < p->order; ++n)
    if (!p->factors[n]) return TK_E_ARG;
  return TK_OK;
}

int64_t resolve_samples(const tk_sketch_opts* o, int64_t d) {
  if (o->num_samples > 0) return o->num_samples;
  if (o->augmented) return tucker_sample_count_augmented(d, o->eps, o->delta, o->d_eff_lower);
  return tucker_sample_count(d, o->eps, o->delta);
}

// c = min{1, d - d'_eff} clamped at 0: the mass of each ridge row in the
// augmented distribution (data rows normalised to total mass d).
double ridge_row_mass(int64_t d, double d_eff_lower) {
  double c = static_cast<double>(d) - d_eff_lower;
  if (!(c > 0.0)) c = 0.0;
  return c < 1.0 ? c : 1.0;
}

// Integer weight C = ceil(c 2^Q) of the ridge branch (the data branch has 2^Q).
uint64_t ridge_coin_weight(int64_t d, double d_eff_lower, int qbits) {
  return static_cast<uint64_t>(ceil(ridge_row_mass(d, d_eff_lower) * ldexp(1.0, qbits)));
}

// Q of a sampled update's integer weights (0 selects TK_Q_BITS).
int sketch_qbits(const tk_sketch_opts* o) { return o->cdf_bits ? o->cdf_bits : TK_Q_BITS; }

// ---------------------------------------------------------------- workspaces
struct LevWS {
  double* scores;
  uint64_t* cdf;
  double* L;
  double* Linv;
  double* P;
  double* Q64;
  float* Q32;
};

void carve_lev(Carver& c, const Geom& g, LevWS& w) {
  w.scores = c.take<double>(g.total_rows);
  w.cdf = c.take<uint64_t>(g.total_rows);
  w.L = c.take<double>(g.total_rr);
  w.Linv = c.take<double>(g.total_rr);
  w.P = c.take<double>(g.total_rr);
  w.Q64 = c.take<double>(g.total_q);
  w.Q32 = c.take<float>(g.total_q);
}

void carve_bound(Carver& c, const Geom& g, double*& V, double*& C, double*& lam) {
  V = c.take<double>(g.total_rr);
  C = c.take<double>(g.total_rr);
  lam = c.take<double>(static_cast<size_t>(kMaxOrder) * kMaxRank);
}

// Eigenpairs of every C_n and the ridge-score mixture tables of K.
struct RidgeWS {
  double* V;
  double* C;
  double* lamm;
  double* W;        // A(n) V_n rows at qoff
  uint64_t* tcdf;   // [d]
  uint64_t* ccdf;   // [sum I_n R_n], column c of mode n at qoff[n] + c I_n
  double* deff;
};

void carve_ridge(Carver& c, const Geom& g, RidgeWS& r) {
  carve_bound(c, g, r.V, r.C, r.lamm);
  r.W = c.take<double>(g.total_q);
  r.tcdf = c.take<uint64_t>(g.d);
  r.ccdf = c.take<uint64_t>(g.total_q);
  r.deff = c.take<double>(1);
}

void launch_ridge(const Geom& g, const tk_problem* p, RidgeWS& r, hipStream_t st,
                  int qbits = TK_Q_BITS) {
  launch_eig_modes(g, p->factors, p->dtype, r.V, r.lamm, r.W, r.C, st);
  launch_ridge_tables(g, r.lamm, r.W, p->lambda, r.tcdf, r.ccdf, r.deff, st, qbits);
}

struct SketchWS {
  LevWS lev;
  int32_t* idx;
  double* weight;
  double* weff;
  double* xw;
  void* gpart;
  double* M;
  double* Linv_diag;
  double* rhs;
  double* h;
  double* r;
  double* ytmp;
  double* delta;
  double* ph_a;
  double* ph_b;
  double* vpart;
  double* rows64;
  float* rows32;
  double* coef;
  double* ttm_scratch;
  int32_t* flags;
  int32_t* status;
  int32_t* done;
  int32_t* steps;
  double* relres;
  double* min_pivot;
  unsigned int* missing;
  double* Q64a;  // augmented whitened row tables (augmented draws only)
  RidgeWS ridge; // ridge-score mixture tables (sampling = 1 only)
  bool has_ridge;
  void* cgws;    // conjugate-gradient scratch (cg solves only)
};

// Which optional slices a sampled update (call TK_CALL_SKETCHED) or its adjoint
// (TK_CALL_ADJOINT) reads: the FP64 sample rows feed the FP64 Gram, the
// large-d vector passes and the adjoint; the mode-product scratch serves the
// multi-launch TTM chain, used for d above the one-workgroup kernels' limit
// and by the adjoint.
struct SketchNeeds {
  bool rows64;
  bool ttm;
  bool cg;        // FP64 solve by conjugate gradients (Cholesky as fallback)
  int64_t aug_q;  // entries of the augmented row tables (0: plain draws)
  bool ridge;     // ridge-score mixture tables
};

// The FP64 update solves by conjugate gradients when d is large and the
// sample count is well above d (the sketched Gram then has eigenvalues near 1).
constexpr int kCgMaxIter = 64;
bool use_cg(const Geom& g, int64_t s, const tk_sketch_opts* o, int call) {
  return call == TK_CALL_SKETCHED && o->gram_precision == TK_F64 && cg_ok(g.d) && s >= 8 * g.d;
}

// The sampled update's right side and residual check grouped like the Gram
// (FP64 grouped Gram; the adjoint keeps the per-sample passes).
bool grouped_vectors(const GramPlan& pl, int call) {
  return call == TK_CALL_SKETCHED && grouped_resid_ok(pl.grp);
}

SketchNeeds sketch_needs(const tk_problem* p, const Geom& g, int64_t s, const tk_sketch_opts* o,
                         int call, const GramPlan& pl) {
  const bool adj = call == TK_CALL_ADJOINT;
  const int32_t prec = o->gram_precision;
  const bool gv = grouped_vectors(pl, call);
  return {adj || (prec == TK_F64 && !pl.grp.on) || (!resid_small_ok(g) && !gv),
          adj || !core_chain_small_ok(g) || !refine_check_p_ok(g), use_cg(g, s, o, call),
          o->augmented ? make_geom_aug(p).total_q : 0, o->sampling == 1};
}

// Gram plan of one sketched problem: the sample-split / stream-K plan, and the
// grouped FP64 Gram over the row geometry (augmented rows when augmented).
GramPlan plan_sketch_gram(const tk_problem* p, const Geom& g, int64_t s, const tk_sketch_opts* o) {
  GramPlan pl = plan_gram(g, s, o->gram_precision, 0);
  pl.grp = plan_grouped(o->augmented ? make_geom_aug(p) : g, s, o->gram_precision);
  return pl;
}

void carve_sketch(Carver& c, const Geom& g, int64_t s, const GramPlan& pl, SketchWS& w,
                  const SketchNeeds& need, bool with_partials = true) {
  carve_lev(c, g, w.lev);
  const int64_t d = g.d;
  w.idx = c.take<int32_t>(static_cast<size_t>(g.order) * s);
  w.weight = c.take<double>(s);
  w.weff = c.take<double>(s);
  w.xw = c.take<double>(s);
  w.gpart = with_partials ? c.take<char>(gram_partial_bytes(g, pl)) : nullptr;
  w.M = c.take<double>(static_cast<size_t>(d) * d);
  const int64_t nblk = cdiv(d, kCholNb);
  w.Linv_diag = c.take<double>(kCholAuxBlocks * nblk * kCholNb * kCholNb);
  w.rhs = c.take<double>(d);
  w.h = c.take<double>(d);
  w.r = c.take<double>(d);
  w.ytmp = c.take<double>(d);
  w.delta = c.take<double>(d);
  w.ph_a = c.take<double>(d);
  w.ph_b = c.take<double>(d);
  w.vpart = c.take<double>(vec_part_doubles(g, s));
  w.rows64 = need.rows64
                 ? c.take<double>(static_cast<size_t>(row_chunks(s)) * kRowChunk * g.sum_r)
                 : nullptr;
  w.rows32 = c.take<float>(static_cast<size_t>(row_chunks(s)) * kRowChunk * g.sum_r);
  w.coef = c.take<double>(s);
  w.ttm_scratch = need.ttm ? c.take<double>(kTtmScratchDoubles) : nullptr;
  w.flags = c.take<int32_t>(chol_flag_words(d));
  w.status = c.take<int32_t>(1);
  w.done = c.take<int32_t>(1);
  w.steps = c.take<int32_t>(1);
  w.relres = c.take<double>(1);
  w.min_pivot = c.take<double>(1);
  w.missing = c.take<unsigned int>(1);
  w.Q64a = need.aug_q ? c.take<double>(need.aug_q) : nullptr;
  w.has_ridge = need.ridge;
  if (need.ridge) carve_ridge(c, g, w.ridge);
  w.cgws = need.cg ? c.take<char>(cg_bytes(d)) : nullptr;
}

// Extra workspace of the adjoint, carved after the sampled-update workspace.
struct AdjWS {
  double* g64;    // forward core (FP64)
  double* v64;    // v = M^{-1} gbar
  double* hg;     // whitened forward core
  double* hv;     // whitened v
  double* bq;     // whitened cotangent
  double* alpha;  // per sample
  double* nbeta;  // per sample, -beta
  double* abar;   // factor adjoints (FP64), at geom.qoff
};

void carve_adjoint(Carver& c, const Geom& g, int64_t s, AdjWS& a) {
  a.g64 = c.take<double>(g.d);
  a.v64 = c.take<double>(g.d);
  a.hg = c.take<double>(g.d);
  a.hv = c.take<double>(g.d);
  a.bq = c.take<double>(g.d);
  a.alpha = c.take<double>(s);
  a.nbeta = c.take<double>(s);
  a.abar = c.take<double>(g.total_q);
}

struct ExactWS {
  double* V;
  double* lam;
  double* W;
  double* C;
  double* tA;
  double* tB;
  double* scratch;
  // conjugate gradients (masked tensors)
  double* b;
  double* y;
  double* r;
  double* p;
  double* q;
  double* scal;
  int32_t* done;
};

// largest intermediate of the mode-product chain that contracts modes in
// decreasing order, skipping `skip` (or none when skip < 0)
// Order of the mode products X x_m W_m^T over every mode but `skip`: the
// longest mode first (its product shrinks X the most and reads it in long
// runs), ties taken from the last mode down.  Returns the number of modes.
int contraction_order(const Geom& g, int skip, int* seq) {
  int k = 0;
  for (int m = g.order - 1; m >= 0; --m)
    if (m != skip) seq[k++] = m;
  for (int a = 1; a < k; ++a) {  // stable insertion sort by decreasing size
    const int v = seq[a];
    int b = a;
    while (b > 0 && g.dims[seq[b - 1]] < g.dims[v]) {
      seq[b] = seq[b - 1];
      --b;
    }
    seq[b] = v;
  }
  return k;
}

int64_t chain_max(const Geom& g, int skip) {
  int64_t dims[kMaxOrder];
  for (int n = 0; n < g.order; ++n) dims[n] = g.dims[n];
  int64_t mx = 1;
  int seq[kMaxOrder];
  const int nseq = contraction_order(g, skip, seq);
  for (int k = 0; k < nseq; ++k) {
    const int m = seq[k];
    dims[m] = g.ranks[m];
    int64_t sz = 1;
    for (int n = 0; n < g.order; ++n) sz *= dims[n];
    if (sz > mx) mx = sz;
  }
  return mx;
}

// largest intermediate of G x_0 A_0 ... x_{N-2} A_{N-2} (the loss reconstruction)
int64_t up_chain_max(const Geom& g) {
  int64_t dims[kMaxOrder];
  for (int n = 0; n < g.order; ++n) dims[n] = g.ranks[n];
  int64_t mx = g.d;
  for (int m = 0; m < g.order - 1; ++m) {
    dims[m] = g.dims[m];
    int64_t sz = 1;
    for (int n = 0; n < g.order; ++n) sz *= dims[n];
    if (sz > mx) mx = sz;
  }
  return mx;
}

void carve_exact(Carver& c, const Geom& g, ExactWS& w) {
  w.V = c.take<double>(g.total_rr);
  w.lam = c.take<double>(static_cast<size_t>(kMaxOrder) * kMaxRank);
  w.W = c.take<double>(g.total_q);
  w.C = c.take<double>(g.total_rr);
  int64_t mx = chain_max(g, -1);
  // the masked path contracts the last mode first: its largest intermediate is
  // X without the last mode times R_L (the masked right side and the operator's
  // chain)
  const int64_t masked = g.numel / g.dims[g.order - 1] * g.ranks[g.order - 1];
  if (masked > mx) mx = masked;
  w.tA = c.take<double>(mx > g.d ? mx : g.d);
  w.tB = c.take<double>(mx > g.d ? mx : g.d);
  w.scratch = c.take<double>(kTtmScratchDoubles);
  w.b = c.take<double>(g.d);
  w.y = c.take<double>(g.d);
  w.r = c.take<double>(g.d);
  w.p = c.take<double>(g.d);
  w.q = c.take<double>(g.d);
  w.scal = c.take<double>(8);
  w.done = c.take<int32_t>(1);
}

constexpr int kPcgMaxIter = 64;
constexpr double kPcgTol = 1e-10;

// q = K_W^T D K_W v (rotated masked operator without the ridge term): up the
// chain of modes 0..N-2, the masked fibre products along mode N-1, back down.
void masked_apply(const Geom& g, ExactWS& w, const uint32_t* mask, const double* v, double* q,
                  const int32_t* done, hipStream_t st) {
  const int N = g.order, L = N - 1;
  int64_t dims[kMaxOrder];
  for (int n = 0; n < N; ++n) dims[n] = g.ranks[n];
  double* bufs[2] = {w.tA, w.tB};
  int which = 0;
  const double* cur = v;
  for (int m = 0; m < L; ++m) {
    launch_ttm(cur, dims, N, m, w.W + g.qoff[m], g.dims[m], false, bufs[which], w.scratch, st,
               done);
    dims[m] = g.dims[m];
    cur = bufs[which];
    which ^= 1;
  }
  int64_t P = 1;
  for (int n = 0; n < L; ++n) P *= g.dims[n];
  launch_masked_normal(cur, mask, P, g.dims[L], w.W + g.qoff[L], g.ranks[L], bufs[which], done,
                       st);
  cur = bufs[which];
  which ^= 1;
  for (int m = L - 1; m >= 0; --m) {
    launch_ttm(cur, dims, N, m, w.W + g.qoff[m], g.ranks[m], true, bufs[which], w.scratch, st,
               done);
    dims[m] = g.ranks[m];
    cur = bufs[which];
    which ^= 1;
  }
  launch_copy_f64(g.d, cur, q, st);
}

// Masked exact core: preconditioned conjugate gradients in the eigenbasis
// (tk_masked.hip).  Leaves y = ((x) V_n)^T g in w.y.
void exact_masked(const Geom& g, const tk_problem* p, ExactWS& w, int32_t* status,
                  hipStream_t st) {
  const int N = g.order, L = N - 1;
  int64_t P = 1;
  for (int n = 0; n < L; ++n) P *= g.dims[n];
  // b = K_W^T D x
  launch_masked_rhs(p->X, p->dtype, p->mask, P, g.dims[L], w.W + g.qoff[L], g.ranks[L], w.tA, st);
  int64_t dims[kMaxOrder];
  for (int n = 0; n < N; ++n) dims[n] = g.dims[n];
  dims[L] = g.ranks[L];
  double* bufs[2] = {w.tA, w.tB};
  int which = 1;
  const double* cur = w.tA;
  for (int m = L - 1; m >= 0; --m) {
    launch_ttm(cur, dims, N, m, w.W + g.qoff[m], g.ranks[m], true, bufs[which], w.scratch, st);
    dims[m] = g.ranks[m];
    cur = bufs[which];
    which ^= 1;
  }
  launch_copy_f64(g.d, cur, w.b, st);
  // start from the unmasked solution y0 = b / ((x) Lambda_n + lambda)
  launch_pcg_guess(g, w.lam, p->lambda, w.b, w.y, st);
  masked_apply(g, w, p->mask, w.y, w.q, nullptr, st);
  launch_pcg_start(g, w.lam, p->lambda, kPcgTol, w.b, w.y, w.q, w.r, w.p, w.scal, w.done, st);
  for (int k = 0; k < kPcgMaxIter; ++k) {
    masked_apply(g, w, p->mask, w.p, w.q, w.done, st);
    launch_pcg_step(g, w.lam, p->lambda, kPcgTol, w.q, w.y, w.r, w.p, w.scal, w.done, st);
  }
  launch_pcg_finish(w.done, status, st);
}

struct FactorWS {
  double* C;
  double* A64;
  double* G64;
  double* Z;
  double* Z2;
  double* rhs;
  double* KKt;
  double* tA;
  double* tB;
  double* scratch;
};

void carve_factor(Carver& c, const Geom& g, FactorWS& w, bool masked) {
  w.A64 = c.take<double>(g.total_q);
  w.G64 = c.take<double>(g.d);
  if (masked) {  // the observed-entries pass needs only its own partials
    w.scratch = c.take<double>(factor_masked_bytes(g) / sizeof(double) + 1);
    return;
  }
  w.C = c.take<double>(g.total_rr);
  w.Z = c.take<double>(g.d);
  w.Z2 = c.take<double>(g.d);
  int64_t maxI = 1;
  for (int n = 0; n < g.order; ++n) maxI = g.dims[n] > maxI ? g.dims[n] : maxI;
  w.rhs = c.take<double>(maxI * kMaxRank);
  w.KKt = c.take<double>(kMaxRank * kMaxRank);
  int64_t mx = 1;
  for (int n = 0; n < g.order; ++n) {
    const int64_t v = chain_max(g, n);
    mx = v > mx ? v : mx;
  }
  if (g.order == 1) mx = g.numel;  // no contraction: W is X itself, converted to FP64
  w.tA = c.take<double>(mx);
  w.tB = c.take<double>(mx);
  w.scratch = c.take<double>(kTtmScratchDoubles);
}

constexpr int64_t kLossParts = 1024;

struct LossWS {
  double* A64;
  double* G64;
  double* tA;
  double* tB;
  double* psq;
  double* pcnt;
  double* preg;
  double* scratch;
};

void carve_loss(Carver& c, const Geom& g, LossWS& w) {
  w.A64 = c.take<double>(g.total_q);
  w.G64 = c.take<double>(g.d);
  const int64_t mx = up_chain_max(g);
  w.tA = c.take<double>(mx);
  w.tB = c.take<double>(mx);
  w.psq = c.take<double>(kLossParts);
  w.pcnt = c.take<double>(kLossParts);
  w.preg = c.take<double>(static_cast<size_t>(kMaxOrder + 1) * 64);
  w.scratch = c.take<double>(kTtmScratchDoubles);
}

// ---------------------------------------------------------------- helpers
// T <- T x_n M_n over all modes (core-sized ping-pong).  Returns the buffer
// holding the result (a or b).
double* core_chain(const Geom& g, double* a, double* b, const double* mats, bool trans,
                   double* scratch, hipStream_t st, const int32_t* done = nullptr) {
  int64_t dims[kMaxOrder];
  for (int n = 0; n < g.order; ++n) dims[n] = g.ranks[n];
  double* cur = a;
  double* nxt = b;
  for (int n = 0; n < g.order; ++n) {
    launch_ttm(cur, dims, g.order, n, mats + g.roff[n], g.ranks[n], trans, nxt, scratch, st,
               done);
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  return cur;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

int32_t tucker_abi_version(void) { return 1; }

const char* tucker_status_string(tk_status s) {
  switch (s) {
    case TK_OK: return "ok";
    case TK_E_ARG: return "invalid argument";
    case TK_E_SHAPE: return "unsupported shape";
    case TK_E_DTYPE: return "unsupported dtype";
    case TK_E_WORKSPACE: return "workspace too small";
    case TK_E_NOT_SPD: return "matrix not positive definite";
    case TK_E_RANK_DEFICIENT: return "rank-deficient factor matrix";
    case TK_E_NO_CONVERGE: return "refinement did not converge";
    case TK_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

int64_t tucker_sample_count(int64_t d, double eps, double delta) {
  if (d < 1 || !(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0)) return 0;
  const double a = 420.0 * log(4.0 * static_cast<double>(d) / delta);
  const double b = 1.0 / (delta * eps);
  return static_cast<int64_t>(ceil(8.0 * static_cast<double>(d) * (a > b ? a : b)));
}

int64_t tucker_sample_count_augmented(int64_t d, double eps, double delta, double d_eff_lower) {
  if (d < 1 || !(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0) || !isfinite(d_eff_lower))
    return 0;
  const double c = ridge_row_mass(d, d_eff_lower);
  const double a = 420.0 * log(4.0 * static_cast<double>(d) / delta);
  const double b = 1.0 / (delta * eps);
  return static_cast<int64_t>(ceil(4.0 * static_cast<double>(d) * (1.0 + c) * (a > b ? a : b)));
}

size_t tucker_workspace_bytes(const tk_problem* p, const tk_sketch_opts* opts, int32_t call) {
  if (check_shape(p) != TK_OK) return 0;
  const Geom g = make_geom(p);
  Carver c(nullptr);
  switch (call) {
    case TK_CALL_LEVERAGE: {
      LevWS w;
      carve_lev(c, g, w);
      break;
    }
    case TK_CALL_SKETCHED: {
      if (!opts) return 0;
      const int64_t s = resolve_samples(opts, g.d);
      if (s < 1) return 0;
      const GramPlan pl = plan_sketch_gram(p, g, s, opts);
      SketchWS w;
      carve_sketch(c, g, s, pl, w, sketch_needs(p, g, s, opts, call, pl));
      break;
    }
    case TK_CALL_ADJOINT: {
      if (!opts) return 0;
      const int64_t s = resolve_samples(opts, g.d);
      if (s < 1) return 0;
      const GramPlan pl = plan_sketch_gram(p, g, s, opts);
      SketchWS w;
      carve_sketch(c, g, s, pl, w, sketch_needs(p, g, s, opts, call, pl));
      AdjWS a;
      carve_adjoint(c, g, s, a);
      break;
    }
    case TK_CALL_EXACT: {
      ExactWS w;
      carve_exact(c, g, w);
      break;
    }
    case TK_CALL_FACTOR: {
      FactorWS w;
      carve_factor(c, g, w, p->mask != nullptr);
      break;
    }
    case TK_CALL_LOSS: {
      LossWS w;
      carve_loss(c, g, w);
      break;
    }
    case TK_CALL_MASKED_BOUND: {
      double *V, *C, *lam;
      carve_bound(c, g, V, C, lam);
      break;
    }
    case TK_CALL_RIDGE_TABLES: {
      RidgeWS r;
      carve_ridge(c, g, r);
      break;
    }
    default:
      return 0;
  }
  return c.used + 256;
}

tk_status tucker_masked_sample_bound(const tk_problem* p, double eps, double delta,
                                     double d_eff_lower, double* out, void* ws, size_t ws_bytes,
                                     void* stream) {
  tk_status s = check_problem(p, false);
  if (s != TK_OK) return s;
  if (!out || !ws) return TK_E_ARG;
  if (!(p->lambda > 0.0)) return TK_E_ARG;  // Cor. B.1 needs lambda > 0
  if (!(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0) || !isfinite(d_eff_lower)) return TK_E_ARG;
  const Geom g = make_geom(p);
  if (ws_bytes < tucker_workspace_bytes(p, nullptr, TK_CALL_MASKED_BOUND)) return TK_E_WORKSPACE;
  Carver c(ws);
  double *V, *C, *lam;
  carve_bound(c, g, V, C, lam);
  const double cm = ridge_row_mass(g.d, d_eff_lower);
  const double a = 420.0 * log(4.0 * static_cast<double>(g.d) / delta);
  const double b = 1.0 / (delta * eps);
  const double k = 4.0 * static_cast<double>(g.d) * (1.0 + cm) * (a > b ? a : b);
  hipStream_t st = static_cast<hipStream_t>(stream);
  launch_eig_modes(g, p->factors, p->dtype, V, lam, nullptr, C, st);
  launch_masked_bound(g, lam, p->lambda, k, 1.0 + cm, out, st);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_ridge_tables(const tk_problem* p, uint64_t* tuple_cdf, uint64_t* col_cdf,
                              double* d_eff, void* ws, size_t ws_bytes, void* stream) {
  tk_status s = check_problem(p, false);
  if (s != TK_OK) return s;
  if (!tuple_cdf || !col_cdf || !ws) return TK_E_ARG;
  if (ws_bytes < tucker_workspace_bytes(p, nullptr, TK_CALL_RIDGE_TABLES)) return TK_E_WORKSPACE;
  const Geom g = make_geom(p);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws);
  RidgeWS r;
  carve_ridge(c, g, r);
  launch_ridge(g, p, r, st);
  TK_HIP_CHECK(hipMemcpyAsync(tuple_cdf, r.tcdf, sizeof(uint64_t) * g.d, hipMemcpyDeviceToDevice,
                              st));
  TK_HIP_CHECK(hipMemcpyAsync(col_cdf, r.ccdf, sizeof(uint64_t) * g.total_q,
                              hipMemcpyDeviceToDevice, st));
  if (d_eff)
    TK_HIP_CHECK(hipMemcpyAsync(d_eff, r.deff, sizeof(double), hipMemcpyDeviceToDevice, st));
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_sample_ridge(int32_t order, const int64_t* dims, const int32_t* ranks,
                              const uint64_t* tuple_cdf, const uint64_t* col_cdf, int64_t s,
                              uint64_t seed, uint64_t counter, uint64_t problem,
                              int32_t augmented, double d_eff_lower, int32_t* idx,
                              double* weight, void* stream) {
  if (order < 1 || order > kMaxOrder || !dims || !ranks || !tuple_cdf || !col_cdf || !idx ||
      !weight || s < 1 || (augmented != 0 && augmented != 1) || !isfinite(d_eff_lower))
    return TK_E_ARG;
  tk_problem p;
  memset(&p, 0, sizeof(p));
  p.order = order;
  int64_t d = 1;
  for (int n = 0; n < order; ++n) {
    if (dims[n] < 1 || dims[n] > (int64_t(1) << 31) - 1 - kMaxRank) return TK_E_SHAPE;
    if (ranks[n] < 1 || ranks[n] > kMaxRank || ranks[n] > dims[n]) return TK_E_SHAPE;
    p.dims[n] = dims[n];
    p.ranks[n] = ranks[n];
    d *= ranks[n];
    if (d > kMaxD) return TK_E_SHAPE;
  }
  const Geom g = make_geom(&p);
  launch_sample_ridge(g, tuple_cdf, col_cdf, s, seed, counter, problem, idx, weight,
                      static_cast<hipStream_t>(stream), augmented,
                      augmented ? ridge_coin_weight(d, d_eff_lower, TK_Q_BITS) : 0);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_leverage_scores(const tk_problem* p, double* scores, uint64_t* cdf,
                                 int32_t* dev_status, void* ws, size_t ws_bytes, void* stream) {
  tk_status s = check_problem(p, false);
  if (s != TK_OK) return s;
  if (!cdf || !dev_status || !ws) return TK_E_ARG;
  if (ws_bytes < tucker_workspace_bytes(p, nullptr, TK_CALL_LEVERAGE)) return TK_E_WORKSPACE;
  const Geom g = make_geom(p);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws);
  LevWS w;
  carve_lev(c, g, w);
  launch_fill_i32(1, 0, dev_status, st);
  launch_leverage(g, p->factors, p->dtype, scores ? scores : w.scores, cdf, w.L, w.Linv, w.P,
                  w.Q64, w.Q32, dev_status, st);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_sample(int32_t order, const int64_t* dims, const uint64_t* cdf, int64_t s,
                        uint64_t seed, uint64_t counter, uint64_t problem, int32_t* idx,
                        double* weight, void* stream) {
  if (order < 1 || order > kMaxOrder || !dims || !cdf || !idx || !weight || s < 1)
    return TK_E_ARG;
  tk_problem p;
  memset(&p, 0, sizeof(p));
  p.order = order;
  for (int n = 0; n < order; ++n) {
    if (dims[n] < 1 || dims[n] > (int64_t(1) << 31) - 1) return TK_E_SHAPE;
    p.dims[n] = dims[n];
    p.ranks[n] = 1;
  }
  const Geom g = make_geom(&p);
  launch_sample(g, cdf, s, seed, counter, problem, idx, weight, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_sample_augmented(int32_t order, const int64_t* dims, const int32_t* ranks,
                                  const uint64_t* cdf, int64_t s, uint64_t seed, uint64_t counter,
                                  uint64_t problem, double d_eff_lower, int32_t* idx,
                                  double* weight, void* stream) {
  if (order < 1 || order > kMaxOrder || !dims || !ranks || !cdf || !idx || !weight || s < 1 ||
      !isfinite(d_eff_lower))
    return TK_E_ARG;
  tk_problem p;
  memset(&p, 0, sizeof(p));
  p.order = order;
  int64_t d = 1;
  for (int n = 0; n < order; ++n) {
    if (dims[n] < 1 || dims[n] > (int64_t(1) << 31) - 1 - kMaxRank) return TK_E_SHAPE;
    if (ranks[n] < 1 || ranks[n] > kMaxRank) return TK_E_SHAPE;
    p.dims[n] = dims[n];
    p.ranks[n] = ranks[n];
    d *= ranks[n];
    if (d > kMaxD) return TK_E_SHAPE;
  }
  const Geom g = make_geom(&p);
  launch_sample(g, cdf, s, seed, counter, problem, idx, weight, static_cast<hipStream_t>(stream),
                1, ridge_coin_weight(d, d_eff_lower, TK_Q_BITS));
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

}  // extern "C"

namespace tk {
namespace {

// State shared by the sampled update and its adjoint: steps 1-6 of the
// sampled update leave the FP64 Cholesky factor of G_Q + lambda P in w.M.
struct SketchRun {
  Geom g;
  int64_t s = 0;
  GramPlan pl;
  SketchWS w;
  int32_t* status = nullptr;
  const int32_t* idx = nullptr;
  const double* weight = nullptr;
  hipStream_t st = nullptr;
  const tk_sketch_opts* o = nullptr;
  Carver carver{nullptr};
  // the FP64 sample rows are read by the FP64 Gram, the large-d vector passes
  // and the adjoint; the small-d passes read the factor tables instead
  bool want_rows64 = true;
  // Augmented draws (Alg. 1 over [K; sqrt(lambda) I]): the sample-side kernels
  // read the augmented tables in geometry ga, and the ridge enters only
  // through the sampled ridge rows, so no lambda P is added (lam_sys = 0).
  bool aug = false;
  Geom ga;
  const double* q64s = nullptr;  // whitened row tables the sample-side kernels read
  double lam_sys = 0.0;          // lambda of the assembled and refined system
  int chol_grid = 0;             // cap of the Cholesky's workgroups (0: one per CU)
  bool cg = false;               // FP64 solve by conjugate gradients, Cholesky only as fallback
  bool grp_vec = false;          // right side and residual grouped like the Gram (no sample rows)
  void stage(int k) const {
    if (o->stage_events) (void)hipEventRecord(static_cast<hipEvent_t>(o->stage_events[k]), st);
  }
};

tk_status check_sketch_args(const tk_problem* p, const tk_sketch_opts* o, int64_t& s) {
  if (o->gram_precision != TK_F64 && o->gram_precision != TK_F32 && o->gram_precision != TK_BF16)
    return TK_E_DTYPE;
  if (o->augmented != 0 && o->augmented != 1) return TK_E_ARG;
  if (o->sampling != 0 && o->sampling != 1) return TK_E_ARG;
  if (o->augmented && !isfinite(o->d_eff_lower)) return TK_E_ARG;
  if (o->augmented) {
    for (int n = 0; n < p->order; ++n)
      if (p->dims[n] > (int64_t(1) << 31) - 1 - kMaxRank) return TK_E_SHAPE;
  }
  if (o->refine_max < 0 || o->refine_max > 1000 || !(o->refine_tol >= 0.0)) return TK_E_ARG;
  if (o->cdf_bits != 0 && (o->cdf_bits < TK_Q_BITS_MIN || o->cdf_bits > TK_Q_BITS_MAX))
    return TK_E_ARG;
  const Geom g = make_geom(p);
  s = resolve_samples(o, g.d);
  if (s < 1 || s > (int64_t(1) << 31) - 1) return TK_E_ARG;
  return TK_OK;
}

// Steps 1-3: leverage scores and whitened rows, samples, gather and the
// pre-gathered sample rows.  With frozen samples (idx_in) the sampler is
// skipped.
tk_status sketch_pre(SketchRun& R, const tk_problem* p, const int32_t* idx_in,
                     const double* weight_in, int32_t* idx_out, double* weight_out) {
  const Geom& g = R.g;
  SketchWS& w = R.w;
  hipStream_t st = R.st;
  R.stage(0);
  launch_init_words(R.status, w.done, w.steps, w.relres, w.min_pivot, w.missing, st);

  // 1. factor leverage scores, whitened rows, CDF tables (Alg. 3, first step)
  const int qbits = sketch_qbits(R.o);
  launch_leverage(g, p->factors, p->dtype, w.lev.scores, w.lev.cdf, w.lev.L, w.lev.Linv, w.lev.P,
                  w.lev.Q64, w.lev.Q32, R.status, st, qbits);
  if (R.aug) launch_aug_tables(g, R.ga, w.lev.Q64, w.lev.Linv, p->lambda, w.Q64a, st);
  R.stage(1);
  // 2. samples (Alg. 3 sampler) or the frozen set
  R.idx = idx_in;
  R.weight = weight_in;
  if (!idx_in) {
    int32_t* io = idx_out ? idx_out : w.idx;
    double* wo = weight_out ? weight_out : w.weight;
    const uint64_t coin = R.aug ? ridge_coin_weight(g.d, R.o->d_eff_lower, qbits) : 0;
    if (R.o->sampling == 1) {  // the ridge-score mixture of K
      launch_ridge(g, p, w.ridge, st, qbits);
      launch_sample_ridge(g, w.ridge.tcdf, w.ridge.ccdf, R.s, R.o->seed, R.o->counter,
                          R.o->problem, io, wo, st, R.aug ? 1 : 0, coin, qbits);
    } else {
      launch_sample(g, w.lev.cdf, R.s, R.o->seed, R.o->counter, R.o->problem, io, wo, st,
                    R.aug ? 1 : 0, coin, qbits);
    }
    R.idx = io;
    R.weight = wo;
  } else if (idx_out) {
    TK_HIP_CHECK(hipMemcpyAsync(idx_out, idx_in, sizeof(int32_t) * g.order * R.s,
                                hipMemcpyDeviceToDevice, st));
    TK_HIP_CHECK(hipMemcpyAsync(weight_out, weight_in, sizeof(double) * R.s,
                                hipMemcpyDeviceToDevice, st));
  }
  R.stage(2);
  // 3. sampled entries (x_t, mask) and effective weights; sample rows
  launch_gather(g, p->X, p->dtype, p->mask, R.idx, R.weight, R.s, w.weff, w.xw, w.missing,
                R.status, st, R.aug ? 1 : 0);
  if (!R.grp_vec)  // the grouped Gram and vectors stage their own sorted rows
    launch_pregather(R.ga, R.idx, w.weff, R.s, R.q64s, R.want_rows64 ? w.rows64 : nullptr,
                     w.rows32, st);
  R.stage(3);
  return TK_OK;
}

// Steps 5-6 after the Gram is assembled: right side and FP64 Cholesky.
void sketch_factor(SketchRun& R) {
  const Geom& g = R.g;
  SketchWS& w = R.w;
  // 5. right-hand side sum_t w_t x_t q_t (FP64)
  if (R.grp_vec)
    launch_grouped_resid(R.ga, R.pl.grp, R.q64s, w.gpart, nullptr, w.rhs, R.st);
  else if (resid_small_ok(g))
    launch_resid_small(R.ga, R.idx, R.q64s, w.xw, nullptr, nullptr, R.s, w.vpart, w.rhs, nullptr,
                       R.st);
  else if (resid_big_ok(g))
    launch_resid_big(g, w.rows64, w.xw, nullptr, nullptr, R.s, w.vpart, w.rhs, nullptr, R.st);
  else
    launch_rows_t_vec(g, w.rows64, w.xw, R.s, w.vpart, w.rhs, nullptr, R.st);
  R.stage(5);
  // 6. FP64 Cholesky (with conjugate gradients: run by the solve, if needed)
  if (!R.cg)
    launch_cholesky(w.M, g.d, w.Linv_diag, w.min_pivot, R.status, w.flags, R.st, R.chol_grid);
  R.stage(6);
}

// Step 4: M = sketched Gram + lambda P (grouped FP64, or partials then assembly).
void sketch_gram(SketchRun& R) {
  SketchWS& w = R.w;
  if (R.pl.grp.on) {
    launch_grouped_gram(R.ga, R.pl.grp, R.idx, R.q64s, w.weff, w.xw, w.lev.P, R.lam_sys, w.gpart, w.M,
                        R.st);
    R.stage(4);
    return;
  }
  launch_gram(R.g, R.pl, w.rows64, w.rows32, w.weff, R.s, w.gpart, R.st);
  R.stage(4);
  launch_assemble(R.g, R.pl, w.gpart, w.lev.P, R.lam_sys, w.M, R.st);
}

// Steps 1-6 of one problem: ... the sketched Gram on MFMA (4) and its
// assembly with lambda P, then the right side and the Cholesky factor.
tk_status sketch_setup(SketchRun& R, const tk_problem* p, const int32_t* idx_in,
                       const double* weight_in, int32_t* idx_out, double* weight_out) {
  tk_status stt = sketch_pre(R, p, idx_in, weight_in, idx_out, weight_out);
  if (stt != TK_OK) return stt;
  // 4. sketched Gram on MFMA, plus lambda P
  sketch_gram(R);
  sketch_factor(R);
  return TK_OK;
}

// h = (G_Q + lambda P)^{-1} b with FP64 iterative refinement against the
// matrix-free FP64 residual
//   r = b + sum_t q_t (xw_t - weff_t q_t . h) - lambda P h
// (xw == nullptr: the xw term is absent).  The sampled update passes b = 0
// and its xw (so that r = rhs - M h); the adjoint passes its right side b
// and no xw.  `norm_ref` is the vector whose norm scales the stopping test.
void refined_solve(SketchRun& R, double lambda, const double* b, const double* xw,
                   const double* norm_ref, double* h) {
  const Geom& g = R.g;
  SketchWS& w = R.w;
  hipStream_t st = R.st;
  const bool refine = R.o->gram_precision != TK_F64;
  const int iters = refine ? R.o->refine_max : 0;
  if (resid_small_ok(g) && refine_small_ok(g)) {
    // small d: the first solve in the one-workgroup step kernel (which also
    // clears done), then the residual's partials and one fused step (sum,
    // P h, test, block solve, update) per iteration
    launch_refine_step_small(g, nullptr, 0, w.lev.P, b ? b : w.rhs, lambda, norm_ref, -1.0, w.M,
                             w.Linv_diag, h, w.done, w.steps, w.relres, 1, st, 1);
    R.stage(7);
    for (int k = 0; k <= iters; ++k) {
      const int64_t np =
          launch_resid_small_parts(R.ga, R.idx, R.q64s, xw, w.weff, h, R.s, w.vpart, w.done, st);
      launch_refine_step_small(g, w.vpart, np, w.lev.P, b, lambda, norm_ref,
                               refine ? R.o->refine_tol : -1.0, w.M, w.Linv_diag, h, w.done,
                               w.steps, w.relres, k < iters ? 1 : 0, st);
    }
    if (refine) launch_finish_refine(w.done, 1, R.status, st);
    R.stage(8);
    return;
  }
  launch_fill_i32(1, 0, w.done, st);
  if (R.cg) {
    // conjugate gradients; the factorisation and its solves run only when
    // they did not converge (they return at once on the done word otherwise)
    launch_cg(w.M, g.d, b ? b : w.rhs, h, w.cgws, w.steps, w.relres, w.min_pivot, R.status,
              kCgMaxIter, st);
    const int32_t* cdone = cg_done_word(w.cgws, g.d);
    launch_cholesky(w.M, g.d, w.Linv_diag, w.min_pivot, R.status, w.flags, st, R.chol_grid, cdone);
    launch_chol_solve(w.M, w.Linv_diag, g.d, h, w.ytmp, w.flags, cdone, R.status, st);
  } else {
    launch_copy_f64(g.d, b ? b : w.rhs, h, st);
    launch_chol_solve(w.M, w.Linv_diag, g.d, h, w.ytmp, w.flags, nullptr, R.status, st);
  }
  R.stage(7);
  for (int k = 0; k <= iters; ++k) {
    if (R.grp_vec && xw == w.xw && !refine) {  // one check of the FP64 solve
      launch_grouped_resid(R.ga, R.pl.grp, R.q64s, w.gpart, h, w.r, st);
    } else if (resid_small_ok(g)) {
      launch_resid_small(R.ga, R.idx, R.q64s, xw, w.weff, h, R.s, w.vpart, w.r, w.done, st);
    } else if (resid_big_ok(g)) {
      launch_resid_big(g, w.rows64, xw, w.weff, h, R.s, w.vpart, w.r, w.done, st);
    } else {
      launch_residual_coef(g, w.rows64, xw, w.weff, h, R.s, w.vpart, w.coef, w.done, st);
      launch_rows_t_vec(g, w.rows64, w.coef, R.s, w.vpart, w.r, w.done, st);
    }
    // the check also prepares the correction solve that follows it
    const bool prep = refine_check_p_ok(g) && k < iters;
    if (refine_check_p_ok(g)) {
      launch_refine_check_p(g, w.r, h, w.lev.P, b, lambda, norm_ref,
                            refine ? R.o->refine_tol : -1.0, w.done, w.steps, w.relres,
                            k < iters ? 1 : 0, st, prep ? w.flags : nullptr,
                            prep ? w.ytmp : nullptr);
    } else {
      launch_copy_f64(g.d, h, w.ph_a, st);
      const double* ph = core_chain(g, w.ph_a, w.ph_b, w.lev.P, false, w.ttm_scratch, st, w.done);
      launch_refine_check(g.d, w.r, ph, b, lambda, norm_ref, refine ? R.o->refine_tol : -1.0,
                          w.done, w.steps, w.relres, k < iters ? 1 : 0, st);
    }
    if (k < iters)  // h += (L L^T)^{-1} r, added as the solve publishes it
      launch_chol_solve(w.M, w.Linv_diag, g.d, w.r, w.ytmp, w.flags, w.done, R.status, st, h,
                        prep);
  }
  if (refine) launch_finish_refine(w.done, 1, R.status, st);
  R.stage(8);
}

// Validates one problem's sampled-update arguments and carves its workspace
// from `c` (the Gram partials too unless the problem is part of a batch).
tk_status sketch_carve(SketchRun& R, const tk_problem* p, const tk_sketch_opts* o,
                       int32_t* dev_status, Carver& c, void* stream, bool with_partials,
                       int call) {
  int64_t s = 0;
  tk_status stt = check_sketch_args(p, o, s);
  if (stt != TK_OK) return stt;
  R.g = make_geom(p);
  R.s = s;
  R.o = o;
  R.st = static_cast<hipStream_t>(stream);
  R.pl = plan_sketch_gram(p, R.g, s, o);
  const SketchNeeds need = sketch_needs(p, R.g, s, o, call, R.pl);
  R.grp_vec = grouped_vectors(R.pl, call);
  R.want_rows64 = need.rows64;
  R.cg = need.cg;
  carve_sketch(c, R.g, s, R.pl, R.w, need, with_partials);
  R.status = dev_status ? dev_status : R.w.status;
  R.aug = o->augmented != 0;
  R.ga = R.aug ? make_geom_aug(p) : R.g;
  R.q64s = R.aug ? R.w.Q64a : R.w.lev.Q64;
  R.lam_sys = R.aug ? 0.0 : p->lambda;
  return TK_OK;
}

tk_status sketch_begin(SketchRun& R, const tk_problem* p, const tk_sketch_opts* o,
                       int32_t* dev_status, void* ws, size_t ws_bytes, void* stream, int call) {
  if (ws_bytes < tucker_workspace_bytes(p, o, call)) {
    int64_t s = 0;
    const tk_status stt = check_sketch_args(p, o, s);
    return stt != TK_OK ? stt : TK_E_WORKSPACE;
  }
  R.carver = Carver(ws);
  return sketch_carve(R, p, o, dev_status, R.carver, stream, true, call);
}

// ---------------------------------------------------------------- batches
constexpr int kTuneCandidates = 6;
const SkConfig kTuneSet[kTuneCandidates] = {{128, 3}, {128, 2}, {256, 1},
                                             {64, 4},  {64, 5},  {64, 6}};

SkConfig batch_config(const tk_batch_config* cfg) {
  SkConfig c{128, 3};
  if (cfg && cfg->tile) c.tile = cfg->tile;
  if (cfg && cfg->wg_per_cu) c.wg_per_cu = cfg->wg_per_cu;
  return c;
}

tk_status check_batch(const tk_problem* probs, const tk_sketch_opts* opts, int32_t count) {
  if (!probs || !opts || count < 1 || count > kSkMaxBatch) return TK_E_ARG;
  const int32_t prec = opts[0].gram_precision;
  if (prec != TK_F32 && prec != TK_BF16) return TK_E_DTYPE;
  for (int k = 0; k < count; ++k) {
    const tk_status stt = check_problem(&probs[k], true);
    if (stt != TK_OK) return stt;
    if (opts[k].gram_precision != prec) return TK_E_DTYPE;
    int64_t s = 0;
    const tk_status st2 = check_sketch_args(&probs[k], &opts[k], s);
    if (st2 != TK_OK) return st2;
  }
  return TK_OK;
}

// Carves every problem's workspace (without per-problem partials) and fills
// the stream-K batch descriptor; then the shared partial slots and index.
void carve_batch(Carver& c, const tk_problem* probs, const tk_sketch_opts* opts, int32_t count,
                 const SkConfig& cfg, SketchRun* runs, int32_t* dev_status, void* stream,
                 SkBatch& b, float*& slots, int64_t*& index) {
  b.count = count;
  for (int k = 0; k < count; ++k) {
    (void)sketch_carve(runs[k], &probs[k], &opts[k], dev_status ? dev_status + k : nullptr, c,
                       stream, false, TK_CALL_SKETCHED);
    b.p[k] = sk_prob(runs[k].g, runs[k].s, runs[k].w.rows32);
  }
  sk_finalize(b, static_cast<tk_dtype>(opts[0].gram_precision), cfg);
  slots = c.take<float>(sk_slot_bytes(b) / sizeof(float));
  index = c.take<int64_t>(sk_index_bytes(b) / sizeof(int64_t));
}

// Streams the per-problem chains of a batch spread over: the caller's stream
// plus kAuxStreams of the library's own (default priority, created once per
// device, kept until the process ends).  Work joins them through events
// recorded on the caller's stream and waited for there again at the end, so
// the call stays one stream's worth of ordered work (and capturable into a
// graph).  The events are reused, so one batched call enqueues at a time per
// device.
constexpr int kAuxStreams = 3;
constexpr int kAuxMaxDevices = 64;
struct AuxPool {
  std::mutex mu;
  bool ready = false;
  hipStream_t s[kAuxStreams];
  hipEvent_t fork;
  hipEvent_t join[kAuxStreams];
};
AuxPool g_aux[kAuxMaxDevices];
std::mutex g_aux_init_mu;

// The current device's pool, created on first use; none (the chains then run
// on the caller's stream alone) if that first use is under stream capture or
// creation fails.
AuxPool* aux_pool(hipStream_t st) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kAuxMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_aux_init_mu);
  AuxPool& p = g_aux[dev];
  if (!p.ready) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return nullptr;
    if (hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
    for (int i = 0; i < kAuxStreams; ++i) {
      if (hipStreamCreateWithFlags(&p.s[i], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming) != hipSuccess)
        return nullptr;  // the objects made so far stay until the process ends
    }
    p.ready = true;
  }
  return &p;
}

// Problem k's stream, and the fork / join of the streams in use.
struct Spread {
  AuxPool* pool;
  hipStream_t st;
  int n;  // streams in use, the caller's first
  hipStream_t stream(int k) const {
    const int i = k % n;
    return i == 0 ? st : pool->s[i - 1];
  }
  bool fork() const {
    if (n <= 1) return true;
    bool ok = hipEventRecord(pool->fork, st) == hipSuccess;
    for (int i = 0; i + 1 < n; ++i) ok = ok && hipStreamWaitEvent(pool->s[i], pool->fork, 0) == hipSuccess;
    return ok;
  }
  bool join() const {
    bool ok = true;
    for (int i = 0; i + 1 < n; ++i)
      ok = ok && hipEventRecord(pool->join[i], pool->s[i]) == hipSuccess &&
           hipStreamWaitEvent(st, pool->join[i], 0) == hipSuccess;
    return ok;
  }
};

size_t batch_bytes(const tk_problem* probs, const tk_sketch_opts* opts, int32_t count,
                   const SkConfig& cfg) {
  SketchRun runs[kSkMaxBatch];
  SkBatch b;
  Carver c(nullptr);
  float* slots;
  int64_t* index;
  carve_batch(c, probs, opts, count, cfg, runs, nullptr, nullptr, b, slots, index);
  return c.used + 256;
}

}  // namespace
}  // namespace tk

extern "C" {

tk_status tucker_core_update_sketched(const tk_problem* p, const tk_sketch_opts* o,
                                      const int32_t* idx_in, const double* weight_in,
                                      int32_t* idx_out, double* weight_out, void* core_out,
                                      int32_t* dev_status, double* dev_info, void* ws,
                                      size_t ws_bytes, void* stream) {
  tk_status stt = check_problem(p, true);
  if (stt != TK_OK) return stt;
  if (!o || !core_out || !ws) return TK_E_ARG;
  if ((idx_in == nullptr) != (weight_in == nullptr)) return TK_E_ARG;
  if ((idx_out == nullptr) != (weight_out == nullptr)) return TK_E_ARG;
  SketchRun R;
  stt = sketch_begin(R, p, o, dev_status, ws, ws_bytes, stream, TK_CALL_SKETCHED);
  if (stt != TK_OK) return stt;
  stt = sketch_setup(R, p, idx_in, weight_in, idx_out, weight_out);
  if (stt != TK_OK) return stt;
  // 7. FP64 solve with refinement (low-precision Gram) or one residual check
  refined_solve(R, R.lam_sys, nullptr, R.w.xw, R.w.rhs, R.w.h);
  // 8. back from whitened coordinates: g = ((x) L_n^{-T}) h
  const Geom& g = R.g;
  SketchWS& w = R.w;
  if (core_chain_small_ok(g)) {
    launch_core_chain_small(g, w.h, w.lev.Linv, true, core_out, p->dtype, R.st);
  } else {
    launch_copy_f64(g.d, w.h, w.ph_a, R.st);
    const double* gres = core_chain(g, w.ph_a, w.ph_b, w.lev.Linv, true, w.ttm_scratch, R.st);
    launch_cast_out(g.d, gres, core_out, p->dtype, R.st);
  }
  if (dev_info) launch_info(dev_info, R.s, w.missing, w.steps, w.relres, w.min_pivot, R.st);
  R.stage(9);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_sketched_system(const tk_problem* p, const tk_sketch_opts* o,
                                 const int32_t* idx, const double* weight, double* M_out,
                                 double* b_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                                 void* stream) {
  tk_status stt = check_problem(p, true);
  if (stt != TK_OK) return stt;
  if (!o || !idx || !weight || !M_out || !b_out || !ws) return TK_E_ARG;
  SketchRun R;
  stt = sketch_begin(R, p, o, dev_status, ws, ws_bytes, stream, TK_CALL_SKETCHED);
  if (stt != TK_OK) return stt;
  stt = sketch_pre(R, p, idx, weight, nullptr, nullptr);
  if (stt != TK_OK) return stt;
  const Geom& g = R.g;
  SketchWS& w = R.w;
  sketch_gram(R);
  if (R.grp_vec)
    launch_grouped_resid(R.ga, R.pl.grp, R.q64s, w.gpart, nullptr, w.rhs, R.st);
  else if (resid_small_ok(g))
    launch_resid_small(R.ga, R.idx, R.q64s, w.xw, nullptr, nullptr, R.s, w.vpart, w.rhs, nullptr,
                       R.st);
  else if (resid_big_ok(g))
    launch_resid_big(g, w.rows64, w.xw, nullptr, nullptr, R.s, w.vpart, w.rhs, nullptr, R.st);
  else
    launch_rows_t_vec(g, w.rows64, w.xw, R.s, w.vpart, w.rhs, nullptr, R.st);
  R.stage(5);
  TK_HIP_CHECK(hipMemcpyAsync(M_out, w.M, sizeof(double) * g.d * g.d, hipMemcpyDeviceToDevice,
                              R.st));
  TK_HIP_CHECK(hipMemcpyAsync(b_out, w.rhs, sizeof(double) * g.d, hipMemcpyDeviceToDevice, R.st));
  R.stage(9);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_core_update_sketched_adjoint(const tk_problem* p, const tk_sketch_opts* o,
                                              const int32_t* idx, const double* weight,
                                              const void* core, const void* core_bar,
                                              void* const* factor_bar, void* x_bar,
                                              int32_t* dev_status, double* dev_info, void* ws,
                                              size_t ws_bytes, void* stream) {
  tk_status stt = check_problem(p, true);
  if (stt != TK_OK) return stt;
  if (!o || !idx || !weight || !core || !core_bar || !factor_bar || !ws) return TK_E_ARG;
  if (o->augmented) return TK_E_ARG;  // the adjoint is of the Gram + lambda I form
  for (int n = 0; n < p->order; ++n)
    if (!factor_bar[n]) return TK_E_ARG;
  SketchRun R;
  stt = sketch_begin(R, p, o, dev_status, ws, ws_bytes, stream, TK_CALL_ADJOINT);
  if (stt != TK_OK) return stt;
  AdjWS a;
  carve_adjoint(R.carver, R.g, R.s, a);
  stt = sketch_setup(R, p, idx, weight, nullptr, nullptr);
  if (stt != TK_OK) return stt;
  const Geom& g = R.g;
  SketchWS& w = R.w;
  hipStream_t st = R.st;
  // whitened forward core h_g = ((x) L_n^T) g, so that k_t . g = q_t . h_g
  launch_cast_in(g.d, core, p->dtype, a.g64, st);
  launch_copy_f64(g.d, a.g64, w.ph_a, st);
  launch_copy_f64(g.d, core_chain(g, w.ph_a, w.ph_b, w.lev.L, true, w.ttm_scratch, st), a.hg, st);
  // whitened cotangent b = ((x) L_n^{-1}) gbar; then (G_Q + lambda P) h_v = b
  launch_cast_in(g.d, core_bar, p->dtype, w.ph_a, st);
  launch_copy_f64(g.d, core_chain(g, w.ph_a, w.ph_b, w.lev.Linv, false, w.ttm_scratch, st), a.bq,
                  st);
  refined_solve(R, p->lambda, a.bq, nullptr, a.bq, a.hv);
  // v = ((x) L_n^{-T}) h_v = M^{-1} gbar
  launch_copy_f64(g.d, a.hv, w.ph_a, st);
  launch_copy_f64(g.d, core_chain(g, w.ph_a, w.ph_b, w.lev.Linv, true, w.ttm_scratch, st), a.v64,
                  st);
  // alpha_t = weff_t (x_t - k_t . g), -beta_t = -weff_t (k_t . v)
  launch_residual_coef(g, w.rows64, w.xw, w.weff, a.hg, R.s, w.vpart, a.alpha, nullptr, st);
  launch_residual_coef(g, w.rows64, nullptr, w.weff, a.hv, R.s, w.vpart, a.nbeta, nullptr, st);
  // factor adjoints
  launch_fill_f64(g.total_q, 0.0, a.abar, st);
  launch_adjoint_factors(g, p->factors, p->dtype, idx, R.s, a.v64, a.g64, a.alpha, a.nbeta,
                         a.abar, st);
  for (int n = 0; n < g.order; ++n)
    launch_cast_out(g.dims[n] * g.ranks[n], a.abar + g.qoff[n], factor_bar[n], p->dtype, st);
  // tensor adjoint: nonzero only at sampled observed entries
  if (x_bar) {
    launch_zero(x_bar, static_cast<size_t>(g.numel) * (p->dtype == TK_F64 ? 8 : 4), st);
    launch_adjoint_x(g, idx, R.s, a.nbeta, x_bar, p->dtype, st);
  }
  if (dev_info) launch_info(dev_info, R.s, w.missing, w.steps, w.relres, w.min_pivot, st);
  R.stage(9);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

size_t tucker_workspace_bytes_batched(const tk_problem* probs, const tk_sketch_opts* opts,
                                      int32_t count, const tk_batch_config* cfg) {
  if (check_batch(probs, opts, count) != TK_OK) return 0;
  if (cfg) {
    const SkConfig c = batch_config(cfg);
    if (!sk_config_valid(c)) return 0;
    return batch_bytes(probs, opts, count, c);
  }
  size_t mx = 0;  // enough for every configuration the tuner tries
  for (int k = 0; k < kTuneCandidates; ++k) {
    const size_t v = batch_bytes(probs, opts, count, kTuneSet[k]);
    mx = v > mx ? v : mx;
  }
  return mx;
}

tk_status tucker_core_update_sketched_batched(const tk_problem* probs, const tk_sketch_opts* opts,
                                              int32_t count, const tk_batch_config* cfg,
                                              void* const* core_out, int32_t* dev_status,
                                              double* dev_info, void* ws, size_t ws_bytes,
                                              void* stream) {
  tk_status stt = check_batch(probs, opts, count);
  if (stt != TK_OK) return stt;
  if (!core_out || !dev_status || !ws) return TK_E_ARG;
  for (int k = 0; k < count; ++k)
    if (!core_out[k]) return TK_E_ARG;
  const SkConfig conf = batch_config(cfg);
  if (!sk_config_valid(conf)) return TK_E_ARG;
  if (ws_bytes < batch_bytes(probs, opts, count, conf)) return TK_E_WORKSPACE;
  SketchRun runs[kSkMaxBatch];
  SkBatch b;
  float* slots = nullptr;
  int64_t* index = nullptr;
  Carver c(ws);
  carve_batch(c, probs, opts, count, conf, runs, dev_status, stream, b, slots, index);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // The problems' chains are independent (each has its own workspace and
  // status word; the partial slots are only read after the Gram), so they
  // run spread over several streams.
  Spread sp{aux_pool(st), st, 1};
  std::unique_lock<std::mutex> pool_lock;
  if (sp.pool) {
    pool_lock = std::unique_lock<std::mutex>(sp.pool->mu);
    sp.n = count < kAuxStreams + 1 ? count : kAuxStreams + 1;
  }
  // steps 1-3 per problem
  if (!sp.fork()) return TK_E_HIP;
  for (int k = 0; k < count; ++k) {
    runs[k].st = sp.stream(k);
    stt = sketch_pre(runs[k], &probs[k], nullptr, nullptr, nullptr, nullptr);
    if (stt != TK_OK) {
      sp.join();
      return stt;
    }
  }
  if (!sp.join()) return TK_E_HIP;
  // step 4 for the whole batch: one persistent stream-K launch
  launch_gram_sk(b, slots, index, st);
  // steps 4 (assembly) to 8 per problem
  if (!sp.fork()) return TK_E_HIP;
  for (int k = 0; k < count; ++k) {
    SketchRun& R = runs[k];
    const tk_problem* p = &probs[k];
    hipStream_t sk = sp.stream(k);
    R.st = sk;
    // concurrent Cholesky launches share the CUs (their task workers would
    // otherwise hold every CU while spinning on their chains)
    if (sp.n > 1) R.chol_grid = device_cu_count() / sp.n;
    launch_assemble_sk(b, k, R.g, slots, index, R.w.lev.P, R.lam_sys, R.w.M, sk);
    sketch_factor(R);
    refined_solve(R, R.lam_sys, nullptr, R.w.xw, R.w.rhs, R.w.h);
    if (core_chain_small_ok(R.g)) {
      launch_core_chain_small(R.g, R.w.h, R.w.lev.Linv, true, core_out[k], p->dtype, sk);
    } else {
      launch_copy_f64(R.g.d, R.w.h, R.w.ph_a, sk);
      const double* gres =
          core_chain(R.g, R.w.ph_a, R.w.ph_b, R.w.lev.Linv, true, R.w.ttm_scratch, sk);
      launch_cast_out(R.g.d, gres, core_out[k], p->dtype, sk);
    }
    if (dev_info)
      launch_info(dev_info + static_cast<int64_t>(k) * TK_INFO_LEN, R.s, R.w.missing, R.w.steps,
                  R.w.relres, R.w.min_pivot, sk);
  }
  if (!sp.join()) return TK_E_HIP;
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_tune_batched(const tk_problem* probs, const tk_sketch_opts* opts, int32_t count,
                              void* ws, size_t ws_bytes, void* stream, tk_batch_config* best,
                              double* times_ms, int32_t* n_candidates) {
  tk_status stt = check_batch(probs, opts, count);
  if (stt != TK_OK) return stt;
  if (!ws || !best) return TK_E_ARG;
  if (ws_bytes < tucker_workspace_bytes_batched(probs, opts, count, nullptr))
    return TK_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return TK_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TK_E_HIP;
  }
  double best_ms = 1e300;
  int best_k = 0;
  for (int k = 0; k < kTuneCandidates; ++k) {
    SketchRun runs[kSkMaxBatch];
    SkBatch b;
    float* slots = nullptr;
    int64_t* index = nullptr;
    Carver c(ws);
    carve_batch(c, probs, opts, count, kTuneSet[k], runs, nullptr, stream, b, slots, index);
    if (k == 0)  // the samples and rows are the same for every candidate
      for (int q = 0; q < count; ++q)
        (void)sketch_pre(runs[q], &probs[q], nullptr, nullptr, nullptr, nullptr);
    launch_gram_sk(b, slots, index, st);  // warm-up
    (void)hipEventRecord(e0, st);
    launch_gram_sk(b, slots, index, st);
    (void)hipEventRecord(e1, st);
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      stt = TK_E_HIP;
      break;
    }
    if (times_ms) times_ms[k] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best_k = k;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (stt != TK_OK) return stt;
  best->tile = kTuneSet[best_k].tile;
  best->wg_per_cu = kTuneSet[best_k].wg_per_cu;
  if (n_candidates) *n_candidates = kTuneCandidates;
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_core_update_exact(const tk_problem* p, void* core_out, int32_t* dev_status,
                                   void* ws, size_t ws_bytes, void* stream) {
  tk_status stt = check_problem(p, true);
  if (stt != TK_OK) return stt;
  if (!core_out || !dev_status || !ws) return TK_E_ARG;
  if (ws_bytes < tucker_workspace_bytes(p, nullptr, TK_CALL_EXACT)) return TK_E_WORKSPACE;
  const Geom g = make_geom(p);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws);
  ExactWS w;
  carve_exact(c, g, w);
  launch_fill_i32(1, 0, dev_status, st);
  launch_eig_modes(g, p->factors, p->dtype, w.V, w.lam, w.W, w.C, st);
  if (p->mask) {
    exact_masked(g, p, w, dev_status, st);
    const double* G = core_chain(g, w.y, w.tA, w.V, false, w.scratch, st);
    launch_cast_out(g.d, G, core_out, p->dtype, st);
    return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
  }
  // K^T vec X = X x_N W_N^T ... x_1 W_1^T (W_n = A(n) V_n), longest mode first
  int64_t dims[kMaxOrder];
  for (int n = 0; n < g.order; ++n) dims[n] = g.dims[n];
  const void* cur = p->X;
  tk_dtype cur_dt = p->dtype;
  double* bufs[2] = {w.tA, w.tB};
  int which = 0;
  int seq[kMaxOrder];
  const int nseq = contraction_order(g, -1, seq);
  for (int k = 0; k < nseq; ++k) {
    const int m = seq[k];
    double* out = bufs[which];
    launch_ttm_any(cur, cur_dt, dims, g.order, m, w.W + g.qoff[m], g.ranks[m], true, out,
                   w.scratch, st);
    dims[m] = g.ranks[m];
    cur = out;
    cur_dt = TK_F64;
    which ^= 1;
  }
  double* B = const_cast<double*>(static_cast<const double*>(cur));
  launch_kron_scale(g, w.lam, p->lambda, B, st);
  double* other = (B == w.tA) ? w.tB : w.tA;
  const double* G = core_chain(g, B, other, w.V, false, w.scratch, st);
  launch_cast_out(g.d, G, core_out, p->dtype, st);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_factor_update(const tk_problem* p, const void* core, int32_t mode,
                               void* factor_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                               void* stream) {
  tk_status stt = check_problem(p, true);
  if (stt != TK_OK) return stt;
  if (!core || !factor_out || !dev_status || !ws) return TK_E_ARG;
  if (mode < 0 || mode >= p->order) return TK_E_ARG;
  const Geom g = make_geom(p);
  if (p->mask && !factor_masked_ok(g)) return TK_E_SHAPE;
  if (ws_bytes < tucker_workspace_bytes(p, nullptr, TK_CALL_FACTOR)) return TK_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws);
  FactorWS w;
  carve_factor(c, g, w, p->mask != nullptr);
  launch_fill_i32(1, 0, dev_status, st);
  if (p->mask) {
    // row-wise ridge over the observed entries (one pass over X and the mask)
    for (int n = 0; n < g.order; ++n)
      launch_cast_in(g.dims[n] * g.ranks[n], p->factors[n], p->dtype, w.A64 + g.qoff[n], st);
    launch_cast_in(g.d, core, p->dtype, w.G64, st);
    launch_factor_masked(g, mode, p->X, p->dtype, p->mask, w.A64, w.G64, p->lambda, factor_out,
                         dev_status, w.scratch, st);
    return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
  }
  launch_gram_modes(g, p->factors, p->dtype, w.C, st);
  for (int n = 0; n < g.order; ++n)
    launch_cast_in(g.dims[n] * g.ranks[n], p->factors[n], p->dtype, w.A64 + g.qoff[n], st);
  launch_cast_in(g.d, core, p->dtype, w.G64, st);
  // W = X x_{m != n} A(m)^T, longest mode first
  int64_t dims[kMaxOrder];
  for (int n = 0; n < g.order; ++n) dims[n] = g.dims[n];
  const void* cur = p->X;
  tk_dtype cur_dt = p->dtype;
  double* bufs[2] = {w.tA, w.tB};
  int which = 0;
  int seq[kMaxOrder];
  const int nseq = contraction_order(g, mode, seq);
  for (int k = 0; k < nseq; ++k) {
    const int m = seq[k];
    double* out = bufs[which];
    launch_ttm_any(cur, cur_dt, dims, g.order, m, w.A64 + g.qoff[m], g.ranks[m], true, out,
                   w.scratch, st);
    dims[m] = g.ranks[m];
    cur = out;
    cur_dt = TK_F64;
    which ^= 1;
  }
  const double* W;
  if (cur_dt != TK_F64 || cur == p->X) {
    launch_cast_in(g.numel, p->X, p->dtype, w.tA, st);
    W = w.tA;
  } else {
    W = static_cast<const double*>(cur);
  }
  int64_t P = 1, Q = 1;
  for (int m = 0; m < mode; ++m) P *= g.ranks[m];
  for (int m = mode + 1; m < g.order; ++m) Q *= g.ranks[m];
  const int64_t In = g.dims[mode];
  const int Rn = g.ranks[mode];
  // X_(n) K_n^T = W_(n) G_(n)^T
  launch_unfold_contract(W, w.G64, P, In, Rn, Q, w.rhs, st);
  // K_n K_n^T = G_(n) ((x)_{m != n} C_m) G_(n)^T
  {
    int64_t cd[kMaxOrder];
    for (int n = 0; n < g.order; ++n) cd[n] = g.ranks[n];
    const double* z = w.G64;
    double* zb[2] = {w.Z, w.Z2};
    int zi = 0;
    for (int m = 0; m < g.order; ++m) {
      if (m == mode) continue;
      launch_ttm(z, cd, g.order, m, w.C + g.roff[m], g.ranks[m], false, zb[zi], w.scratch, st);
      z = zb[zi];
      zi ^= 1;
    }
    launch_unfold_contract(w.G64, z, P, Rn, Rn, Q, w.KKt, st);
  }
  launch_factor_solve(w.KKt, w.rhs, In, Rn, p->lambda, factor_out, p->dtype, dev_status, st);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

tk_status tucker_loss(const tk_problem* p, const void* core, double* out, void* ws,
                      size_t ws_bytes, void* stream) {
  tk_status stt = check_problem(p, true);
  if (stt != TK_OK) return stt;
  if (!core || !out || !ws) return TK_E_ARG;
  if (ws_bytes < tucker_workspace_bytes(p, nullptr, TK_CALL_LOSS)) return TK_E_WORKSPACE;
  const Geom g = make_geom(p);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws);
  LossWS w;
  carve_loss(c, g, w);
  for (int n = 0; n < g.order; ++n)
    launch_cast_in(g.dims[n] * g.ranks[n], p->factors[n], p->dtype, w.A64 + g.qoff[n], st);
  launch_cast_in(g.d, core, p->dtype, w.G64, st);
  // H = G x_0 A(0) ... x_{N-2} A(N-2)
  int64_t dims[kMaxOrder];
  for (int n = 0; n < g.order; ++n) dims[n] = g.ranks[n];
  const double* cur = w.G64;
  double* bufs[2] = {w.tA, w.tB};
  int which = 0;
  for (int m = 0; m < g.order - 1; ++m) {
    launch_ttm(cur, dims, g.order, m, w.A64 + g.qoff[m], g.dims[m], false, bufs[which], w.scratch,
               st);
    dims[m] = g.dims[m];
    cur = bufs[which];
    which ^= 1;
  }
  launch_loss_stream(g, p->X, p->dtype, p->mask, cur, w.A64 + g.qoff[g.order - 1], w.psq, w.pcnt,
                     kLossParts, st);
  launch_sq_reduce(g.d, core, p->dtype, w.preg, 64, st);
  for (int n = 0; n < g.order; ++n)
    launch_sq_reduce(g.dims[n] * g.ranks[n], p->factors[n], p->dtype, w.preg + 64 * (n + 1), 64,
                     st);
  launch_loss_final(w.psq, w.pcnt, kLossParts, w.preg, 64 * (g.order + 1), p->lambda, out, st);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_E_HIP;
}

}  // extern "C"
