// solver.cpp -- host side of the library: argument validation, workspace,
// the per-chunk launch sequence of RAC-MBADMM, and the C ABI of racmb.h.
//
// One iteration (Eq.(3)) is four device phases with no host round trip:
//   assemble  k_gram + k_factor : every block matrix of the drawn partition and
//                                 its inverse, all blocks in parallel;
//   sweep     k_sweep2          : the sequential Gauss-Seidel pass (one
//                                 persistent launch of K cooperating groups);
//   z + dual  k_zdual           : z block, dual step, residual norms, history.
// The partitions of a whole chunk of T iterations are drawn by one set of
// sort launches up front (they depend only on the seed and the iteration
// index).  The block matrices of an iteration depend only on the data, the
// partition and beta, so they are built on a second stream while the previous
// iteration's sweep runs on the compute units it leaves idle; the inverses are
// double-buffered by iteration parity and events order the two streams.  After
// the chunk, k_kkt evaluates the KKT residual and k_control applies the
// stopping test and the penalty rule (beta changes only there, so the second
// stream waits for it at chunk boundaries); the host then reads the scalar
// block once to decide whether to continue.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "rac_internal.h"
#include "racmb.h"

using namespace rac;

namespace {

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return RAC_ERR_DEVICE;       \
  } while (0)

bool is_fin(double v) { return std::isfinite(v); }

size_t dtype_size(int32_t dt) {
  switch (dt) {
    case RAC_DT_F64: return 8;
    case RAC_DT_F32: return 4;
    case RAC_DT_BF16: return 2;
    default: return 0;
  }
}

bool is_dense(const rac_problem* P) { return P->Hd != nullptr; }
bool is_sparse(const rac_problem* P) { return P->colptr != nullptr; }
SparseF sparse_of(const rac_problem& P) { return SparseF{P.colptr, P.rowidx, P.F, P.F_dtype}; }

rac_status validate_problem(const rac_problem* P) {
  if (!P) return RAC_ERR_ARG;
  if (P->n < 1 || !P->c || P->n > (int64_t)INT32_MAX) return RAC_ERR_ARG;
  if (is_dense(P)) {
    // dense form: explicit Hessian, several equality rows, no factor F
    if (P->F || P->rows != 0 || P->a || P->ldH < P->n) return RAC_ERR_ARG;
    if (P->H_dtype != RAC_DT_F64 && P->H_dtype != RAC_DT_F32) return RAC_ERR_ARG;
    if (P->meq < 0 || P->meq > RAC_MAX_EQ || (P->meq > 0 && (!P->A || !P->beq))) return RAC_ERR_ARG;
    if (P->colptr || P->rowidx) return RAC_ERR_ARG;
  } else if (is_sparse(P)) {
    // sparse factor form: F holds the values of the compressed sparse columns
    if (P->rows < 1 || P->rows > (int64_t)INT32_MAX || !P->F || !P->rowidx) return RAC_ERR_ARG;
    if (P->F_dtype != RAC_DT_F64 && P->F_dtype != RAC_DT_F32) return RAC_ERR_ARG;
    if (P->meq != 0 || P->A || P->beq) return RAC_ERR_ARG;
  } else {
    if (P->rows < 1 || !P->F || P->ldF < P->rows || P->rowidx) return RAC_ERR_ARG;
    if (dtype_size(P->F_dtype) == 0) return RAC_ERR_ARG;
    if (P->meq != 0 || P->A || P->beq) return RAC_ERR_ARG;
  }
  if (P->prox < RAC_PROX_NONE || P->prox > RAC_PROX_BOX) return RAC_ERR_ARG;
  if (!is_fin(P->Ns) || !(P->Ns > 0.0) || !is_fin(P->b) || !is_fin(P->obj_const)) return RAC_ERR_ARG;
  if (P->prox == RAC_PROX_ELASTIC_NET &&
      (!is_fin(P->lambda) || P->lambda < 0.0 || !is_fin(P->alpha) || P->alpha < 0.0 || P->alpha > 1.0))
    return RAC_ERR_ARG;
  if (P->prox == RAC_PROX_BOX && (!is_fin(P->lo) || !is_fin(P->hi) || P->lo > P->hi)) return RAC_ERR_ARG;
  return RAC_OK;
}

int padded(int64_t s) { return s <= 16 ? 16 : (s <= 32 ? 32 : (s <= 64 ? 64 : 128)); }  // 16..128, power of two

struct Buffers {
  std::vector<void*> owned;
  template <typename T> rac_status alloc(T** p, size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, sizeof(T) * count) != hipSuccess) return RAC_ERR_NOMEM;
    owned.push_back(q);
    *p = (T*)q;
    return RAC_OK;
  }
  void release() {
    for (void* q : owned) (void)hipFree(q);
    owned.clear();
  }
};

#define ALLOC(buf, ptr, count)                    \
  do {                                            \
    rac_status r_ = (buf).alloc(&(ptr), (count)); \
    if (r_ != RAC_OK) return r_;                  \
  } while (0)

rac_status alloc_perm_work(Buffers& B, int64_t T, int64_t n, PermWork* w, int32_t** perm) {
  int64_t nb = 1;
  int lg = 0;
  while (nb < n) { nb <<= 1; ++lg; }
  w->nb = nb;
  w->log2nb = lg;
  ALLOC(B, w->keys, (size_t)(T * n));
  ALLOC(B, w->count, (size_t)(T * nb));
  ALLOC(B, w->offset, (size_t)(T * (nb + 1)));
  ALLOC(B, w->fill, (size_t)(T * nb));
  ALLOC(B, w->members, (size_t)(T * n));
  ALLOC(B, *perm, (size_t)(2 * T * n));
  HIPCHK(hipMemset(w->count, 0, sizeof(uint32_t) * T * nb));
  HIPCHK(hipMemset(w->fill, 0, sizeof(uint32_t) * T * nb));
  return RAC_OK;
}

// Register-tile shape of the sweep: B columns per wavefront covers the largest
// block; A rows per lane is the smallest shape that keeps the number of
// cooperating groups K = ceil(rows / 64A) at or below 128 (the all-to-all
// exchange of partials grows with K), else the largest compiled shape with
// K <= 256 (one group per compute unit).  Returns false when no register shape
// fits; the streaming sweep is used then.
bool choose_tile(int32_t dtype, int64_t rows, int64_t smax, int forced_K, int* A_out, int* B_out, int* K_out) {
  const int B = smax <= 32 ? 8 : (smax <= 64 ? 16 : 32);
  const int As[3] = {1, 2, 4};
  if (forced_K > 0) {
    const int64_t per = (rows + forced_K - 1) / forced_K;
    for (int A : As)
      if (per <= 64 * A && sweep_tile_supported(dtype, A, B)) {
        *A_out = A; *B_out = B; *K_out = forced_K;
        return true;
      }
    return false;
  }
  for (int lim : {128, 256}) {
    for (int A : As) {
      if (!sweep_tile_supported(dtype, A, B)) continue;
      const int64_t K = (rows + 64 * A - 1) / (64 * A);
      if (K <= lim) {
        *A_out = A; *B_out = B; *K_out = (int)K;
        return true;
      }
    }
  }
  return false;
}

int auto_sweep_groups(int64_t rows) {
  int64_t K = rows / 320;
  if (K < 1) K = 1;
  if (K > 64) K = 64;
  return (int)K;
}

int auto_row_chunks(int64_t p, int64_t rows) {
  int64_t R = (256 + p - 1) / p;
  int64_t rmax = rows / 256;
  if (rmax < 1) rmax = 1;
  if (R > rmax) R = rmax;
  if (R < 1) R = 1;
  return (int)R;
}

int matvec_parts(int64_t n) {
  int64_t q = (n + 255) / 256;
  return (int)(q < 1 ? 1 : (q > 64 ? 64 : q));
}

}  // namespace

// The problem's device arrays hold no NaN or infinity (one read of each on the null
// stream): F (or the sparse values, or the dense form's Hd, A and beq), c, h and a.
rac_status rac::check_problem_arrays(const rac_problem& P) {
  uint32_t* flag = nullptr;
  if (hipMalloc(&flag, sizeof(uint32_t)) != hipSuccess) return RAC_ERR_NOMEM;
  hipError_t e = hipMemset(flag, 0, sizeof(uint32_t));
  auto chk = [&](const void* p, int32_t dtype, int64_t rows, int64_t cols, int64_t ld) {
    if (e == hipSuccess && p) e = launch_nonfinite(p, dtype, rows, cols, ld, flag, nullptr);
  };
  if (P.Hd) {
    chk(P.Hd, P.H_dtype, P.n, P.n, P.ldH);
    if (P.meq > 0) {
      chk(P.A, RAC_DT_F64, P.n, P.meq, P.n);      // row-major meq x n: meq runs of n
      chk(P.beq, RAC_DT_F64, P.meq, 1, P.meq);
    }
  } else if (P.colptr) {
    int64_t nnz = 0;
    if (e == hipSuccess) e = hipMemcpy(&nnz, P.colptr + P.n, sizeof(int64_t), hipMemcpyDeviceToHost);
    chk(P.F, P.F_dtype, nnz, 1, nnz);
  } else {
    chk(P.F, P.F_dtype, P.rows, P.n, P.ldF);
  }
  chk(P.c, RAC_DT_F64, P.n, 1, P.n);
  chk(P.h, RAC_DT_F64, P.n, 1, P.n);
  chk(P.a, RAC_DT_F64, P.n, 1, P.n);
  uint32_t bad = 0;
  if (e == hipSuccess) e = hipMemcpy(&bad, flag, sizeof(uint32_t), hipMemcpyDeviceToHost);
  (void)hipFree(flag);
  if (e != hipSuccess) return RAC_ERR_DEVICE;
  return bad ? RAC_ERR_ARG : RAC_OK;
}


struct rac_solver_s {
  rac_problem P{};
  rac_opts O{};
  int64_t n = 0, rows = 0, p = 0, T = 1;
  int sp = 16, R = 1, K = 1;
  Buffers buf;
  int32_t* perm = nullptr;  // partitions of a chunk's iterations, two buffers of [T][n] (by chunk)
  int pbuf = 0;             // buffer of the current chunk
  PermWork pw{};
  double* partial = nullptr;
  double* Minv = nullptr;
  double *x = nullptr, *z = nullptr, *xi = nullptr, *zprev = nullptr, *u = nullptr;
  DevScalars* sc = nullptr;
  double* sweep_part = nullptr;
  uint64_t* flags = nullptr;
  uint64_t epoch = 0;
  double* red = nullptr;
  uint32_t* done = nullptr;
  double* kkt_out = nullptr;
  double* kkt_part = nullptr;   // [kKKTChunks][n] partial column products of the check
  double* obj_out = nullptr;
  double* hist = nullptr;
  int64_t hist_cap = 0, hist_count = 0;
  double* d_sched = nullptr;
  double* mv_part = nullptr;
  int mv_nparts = 1;
  double* uz = nullptr;     // F z for the objective
  int tileA = 0, tileB = 0; // register tile of the sweep (0: streaming sweep)
  uint8_t* Fp = nullptr;    // two packed copies of F in the sweep's register order (by iteration parity)
  size_t Fp_bytes = 0;      // bytes of one copy
  int64_t packRW = 0;       // rows per sweep group
  int max_spin = -1;        // sweep wait limit (RACMB_SWEEP_MAX_SPIN, for tests of the error path)
  bool overlap = false;     // assemble on a second stream during the previous sweep
  hipStream_t sB = nullptr;
  hipEvent_t ev_start = nullptr, ev_fac[2] = {nullptr, nullptr}, ev_sweep[2] = {nullptr, nullptr};
  hipEvent_t ev_check = nullptr;   // scalars of a chunk copied out: the next chunk's factor may run
  int64_t swept[2] = {-1, -1};     // iteration of the last sweep recorded in ev_sweep[parity] this run
  int64_t pre_k = -1;              // iteration whose partition, Gram and factor are already enqueued
  // RP-MBADMM (fixed contiguous blocks, random order): the block Grams and the packed copy
  // are formed once, the inverses whenever beta differs from the one they were formed with
  bool rp = false;
  int32_t* order = nullptr;        // solve orders of a chunk's iterations, [T][p]
  PermWork pw_order{};
  int32_t* iota = nullptr;         // the fixed partition: variable j at position j
  bool rp_gram = false;            // Grams (and packed copy) formed
  double fac_beta = NAN;           // beta of the current inverses (NaN: none)
  std::vector<double> sched_host;  // the given schedule (RP decides refactoring on the host)
  // dense form (explicit Hessian Hd, meq equality rows): the sweep reads H_beta = Hd + beta A'A
  // (or Hd itself without rows) and c_eff = c - A'(beta beq + mu); x is its own residual
  bool dense = false;
  bool sparse = false;             // F in compressed sparse columns: one-workgroup sweep, one stream
  int meq = 0;
  double* Hb = nullptr;            // H_beta (n x n FP64) when meq > 0
  double hb_beta = NAN;            // beta of H_beta (NaN: not formed)
  double* ceff = nullptr;          // c_eff (n) when meq > 0
  double* mu_vec = nullptr;        // multipliers (meq)
  double* t_vec = nullptr;         // A x after the last sweep (meq)
  double* eq_r2 = nullptr;         // |A x - beq|^2 of the last iteration
  double* eq_red = nullptr;        // per-row scratch of the multiplier step (RAC_MAX_EQ)
  uint32_t* eq_done = nullptr;
  DevScalars* hsc_pin = nullptr;   // pinned copy of the scalars read after each chunk
  DevScalars hsc{};
  // optional per-phase timing with HIP events on the run's stream
  uint32_t tmask = 0;                    // phases timed (bit q: phase q)
  int64_t tstride = 1;                   // per-iteration phases timed on iterations k % tstride == 0
  std::vector<hipEvent_t> ev;            // pool, two per timed launch
  std::vector<int> ev_phase;             // phase of each recorded pair in the current chunk
  double phase_ms[RAC_NUM_PHASES] = {0};
  int64_t phase_count[RAC_NUM_PHASES] = {0};
};

namespace {

DevScalars fresh_scalars(double beta) {
  DevScalars s{};
  s.t = 0.0;
  s.mu = 0.0;
  s.beta = beta;
  s.kkt = NAN;
  s.kkt_prev = -1.0;
  s.last_l10 = 0.0;
  s.rp_first = -1.0;
  s.rp = s.rd = s.rp_win = s.rd_win = 0.0;
  s.objective = NAN;
  s.k = 0;
  s.decisions = 0;
  s.fail_key = ~0ULL;
  s.status = 0;
  return s;
}

rac_status fx_into_u(rac_solver s, const double* x, double* u, hipStream_t st) {
  if (s->sparse) {
    HIPCHK(launch_sspmv(sparse_of(s->P), s->rows, s->n, x, u, st));
    return RAC_OK;
  }
  HIPCHK(launch_matvec_F_parts(s->P.F, s->P.F_dtype, s->P.ldF, s->rows, s->n, x, u, s->mv_part,
                               s->mv_nparts, st));
  return RAC_OK;
}

// Event pairs around timed launches of the phases selected in the timing mask:
// begin() records the start event of the next pair, end() its stop event and
// remembers the phase.
struct PhaseTimer {
  rac_solver s;
  hipStream_t st;
  int64_t k = -1;                        // iteration of the phase being enqueued (-1: once per chunk)
  bool on(int phase) const {
    return ((s->tmask >> phase) & 1u) != 0 && (k < 0 || s->tstride <= 1 || k % s->tstride == 0);
  }
  hipError_t begin(hipStream_t stream, int phase) { st = stream; return begin(phase); }
  hipError_t begin(int phase) {
    if (!on(phase)) return hipSuccess;
    const size_t i = 2 * s->ev_phase.size();
    while (s->ev.size() < i + 2) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      s->ev.push_back(e);
    }
    return hipEventRecord(s->ev[i], st);
  }
  hipError_t end(int phase) {
    if (!on(phase)) return hipSuccess;
    const size_t i = 2 * s->ev_phase.size();
    s->ev_phase.push_back(phase);
    return hipEventRecord(s->ev[i + 1], st);
  }
};

rac_status collect_timing(rac_solver s) {
  if (s->ev_phase.empty()) return RAC_OK;
  for (size_t q = 0; q < s->ev_phase.size(); ++q) {
    float ms = 0.f;
    HIPCHK(hipEventSynchronize(s->ev[2 * q + 1]));   // launches enqueued ahead may still run
    HIPCHK(hipEventElapsedTime(&ms, s->ev[2 * q], s->ev[2 * q + 1]));
    s->phase_ms[s->ev_phase[q]] += ms;
    s->phase_count[s->ev_phase[q]] += 1;
  }
  s->ev_phase.clear();
  return RAC_OK;
}

// Gram (with the packed copy) of iteration k on the assemble stream.  Its
// inverse and packed buffers (by parity of k) were last read by the sweep of
// iteration k - 2, which it waits for when that sweep belongs to this run.
rac_status enqueue_gram(rac_solver s, int64_t k, const int32_t* perm, hipStream_t sa, PhaseTimer& tm) {
  const rac_problem& P = s->P;
  const int par = (int)(k & 1);
  if (s->overlap && s->swept[par] >= 0) HIPCHK(hipStreamWaitEvent(sa, s->ev_sweep[par], 0));
  void* Fp = s->Fp ? (void*)(s->Fp + par * s->Fp_bytes) : nullptr;
  GramArgs g{P.F, P.F_dtype, P.ldF, s->rows, s->n, s->p, perm, s->O.precision, s->R, s->sp,
             s->partial, PackDst{Fp, s->packRW, s->K, s->tileA, s->tileB}};
  tm.k = k;
  HIPCHK(tm.begin(sa, RAC_PHASE_GRAM));
  HIPCHK(launch_gram(g, sa));
  HIPCHK(tm.end(RAC_PHASE_GRAM));
  return RAC_OK;
}

// Factor of iteration k after its Gram; with overlap the sweep's stream waits on ev_fac.
rac_status enqueue_factor(rac_solver s, int64_t k, const int32_t* perm, const double* beta_ptr, hipStream_t sa,
                          PhaseTimer& tm) {
  const rac_problem& P = s->P;
  const int par = (int)(k & 1);
  FactorArgs f{};
  f.partial = s->partial; f.R = s->R; f.sp = s->sp; f.n = s->n; f.p = s->p; f.perm = perm;
  f.Ns = P.Ns; f.h = P.h; f.a = P.a; f.beta_ptr = beta_ptr; f.beta_val = 0.0;
  f.Minv = s->Minv + par * (size_t)s->p * s->sp * s->sp;
  f.write_matrix = 0; f.sc = s->sc; f.iter_global = k;
  tm.k = k;
  HIPCHK(tm.begin(sa, RAC_PHASE_FACTOR));
  HIPCHK(launch_factor(f, sa));
  HIPCHK(tm.end(RAC_PHASE_FACTOR));
  if (s->overlap) HIPCHK(hipEventRecord(s->ev_fac[par], sa));
  return RAC_OK;
}

const double* beta_of(rac_solver s, int64_t run_offset) {
  return s->O.beta_mode == RAC_BETA_SCHEDULE ? s->d_sched + run_offset : &s->sc->beta;
}

// With overlap, the partitions of the next chunk (starting at iteration k1, Tn
// iterations) and the Gram of its first iteration go on the assemble stream
// right away, so they run during this chunk's last sweep; the factor, which
// needs the penalty decided at this chunk's check, waits for the check and the
// copy of the scalars.  None of this touches the iterate.
rac_status preissue_next_chunk(rac_solver s, int64_t k1, int64_t Tn, int64_t run_offset, hipStream_t st) {
  PhaseTimer tm{s, st};
  hipStream_t sa = s->sB;
  const int b = 1 - s->pbuf;
  int32_t* pb = s->perm + (size_t)b * s->T * s->n;
  // the buffer was last read by the previous chunk's sweeps, all before the sweep of k1 - 2
  if (s->swept[k1 & 1] >= 0) HIPCHK(hipStreamWaitEvent(sa, s->ev_sweep[k1 & 1], 0));
  tm.k = -1;
  HIPCHK(tm.begin(sa, RAC_PHASE_PARTITION));
  HIPCHK(launch_permutations(s->O.seed, s->O.instance, k1, Tn, s->n, s->pw, pb, sa));
  HIPCHK(tm.end(RAC_PHASE_PARTITION));
  rac_status e = enqueue_gram(s, k1, pb, sa, tm);
  if (e != RAC_OK) return e;
  HIPCHK(hipEventRecord(s->ev_check, st));
  HIPCHK(hipStreamWaitEvent(sa, s->ev_check, 0));
  e = enqueue_factor(s, k1, pb, beta_of(s, run_offset), sa, tm);
  if (e != RAC_OK) return e;
  s->pre_k = k1;
  return RAC_OK;
}

rac_status enqueue_check(rac_solver s, int64_t k0, int64_t Tc, int64_t run_offset, hipStream_t st, PhaseTimer& tm);

// RP-MBADMM chunk (one stream): the orders of the chunk's iterations, then per
// iteration the factor when beta has changed (the Grams once per solver), the
// sweep in the drawn order, and the z/dual step.  Within a chunk beta changes
// only under a given schedule; the controller changes it at the check, after
// which the host reads it with the scalars.
rac_status enqueue_rp_chunk(rac_solver s, int64_t Tc, int64_t run_offset, hipStream_t st) {
  const rac_problem& P = s->P;
  PhaseTimer tm{s, st};
  const int64_t k0 = s->hsc.k;
  const bool sched = s->O.beta_mode == RAC_BETA_SCHEDULE;
  tm.k = -1;
  HIPCHK(tm.begin(RAC_PHASE_PARTITION));
  HIPCHK(launch_permutations(s->O.seed, s->O.instance, k0, Tc, s->p, s->pw_order, s->order, st));
  HIPCHK(tm.end(RAC_PHASE_PARTITION));
  for (int64_t t = 0; t < Tc; ++t) {
    const int64_t k = k0 + t;
    const int32_t* ord = s->order + t * s->p;
    const double* beta_ptr = beta_of(s, run_offset + t);
    tm.k = k;
    if (!s->rp_gram) {
      GramArgs g{P.F, P.F_dtype, P.ldF, s->rows, s->n, s->p, s->iota, s->O.precision, s->R, s->sp,
                 s->partial, PackDst{s->Fp, s->packRW, s->K, s->tileA, s->tileB}};
      HIPCHK(tm.begin(st, RAC_PHASE_GRAM));
      HIPCHK(launch_gram(g, st));
      HIPCHK(tm.end(RAC_PHASE_GRAM));
      s->rp_gram = true;
      s->fac_beta = NAN;
    }
    const double bk = sched ? s->sched_host[run_offset + t] : s->hsc.beta;
    if (!(bk == s->fac_beta)) {
      FactorArgs f{};
      f.partial = s->partial; f.R = s->R; f.sp = s->sp; f.n = s->n; f.p = s->p; f.perm = s->iota;
      f.Ns = P.Ns; f.h = P.h; f.a = P.a; f.beta_ptr = beta_ptr; f.beta_val = 0.0; f.Minv = s->Minv;
      f.write_matrix = 0; f.sc = s->sc; f.iter_global = k; f.order = ord;
      HIPCHK(tm.begin(st, RAC_PHASE_FACTOR));
      HIPCHK(launch_factor(f, st));
      HIPCHK(tm.end(RAC_PHASE_FACTOR));
      s->fac_beta = bk;
    }
    SweepArgs w{P.F, P.F_dtype, P.ldF, s->rows, s->n, s->p, s->iota, s->Minv, s->sp, P.c, P.h, P.a,
                P.b, P.Ns, s->x, s->z, s->xi, s->u, s->sc, s->sweep_part, s->flags, s->epoch, s->K,
                beta_ptr, s->tileA, s->tileB, 1, s->Fp, s->max_spin, ord};
    HIPCHK(tm.begin(st, RAC_PHASE_SWEEP));
    HIPCHK(launch_sweep(w, st));
    HIPCHK(tm.end(RAC_PHASE_SWEEP));
    s->epoch += (uint64_t)s->p;
    UpdateArgs za{};
    za.n = s->n; za.prox = P.prox; za.lam = P.lambda; za.alpha = P.alpha; za.lo = P.lo; za.hi = P.hi;
    za.b = P.b; za.has_eq = P.a ? 1 : 0; za.x = s->x; za.z = s->z; za.xi = s->xi; za.zprev = s->zprev;
    za.sc = s->sc; za.red = s->red; za.done = s->done; za.hist = s->hist; za.hist_cap = s->hist_cap;
    za.hist_base = k0 - run_offset; za.T = s->T; za.beta_ptr = beta_ptr; za.publish_beta = sched ? 1 : 0;
    HIPCHK(tm.begin(st, RAC_PHASE_ZDUAL));
    HIPCHK(launch_zdual(za, st));
    HIPCHK(tm.end(RAC_PHASE_ZDUAL));
  }
  return enqueue_check(s, k0, Tc, run_offset, st, tm);
}

// The matrix the dense form's sweep and block matrices read: H_beta, or Hd without rows.
const void* dense_H(rac_solver s, int32_t* dtype, int64_t* ld) {
  if (s->Hb) { *dtype = RAC_DT_F64; *ld = s->n; return s->Hb; }
  *dtype = s->P.H_dtype;
  *ld = s->P.ldH;
  return s->P.Hd;
}

// Dense-form chunk (one stream): the partitions (RAC) or orders (RP) of the chunk;
// per iteration H_beta when beta changed, c_eff for the current multipliers, the
// block matrices gathered from H_beta and factored (RP: only when beta changed),
// the sweep with x as the group-resident residual, t = A x with the multiplier
// step, and the z/dual step; then the check.
rac_status enqueue_dense_chunk(rac_solver s, int64_t Tc, int64_t run_offset, hipStream_t st) {
  const rac_problem& P = s->P;
  PhaseTimer tm{s, st};
  const int64_t k0 = s->hsc.k;
  const bool sched = s->O.beta_mode == RAC_BETA_SCHEDULE;
  tm.k = -1;
  HIPCHK(tm.begin(RAC_PHASE_PARTITION));
  if (s->rp) HIPCHK(launch_permutations(s->O.seed, s->O.instance, k0, Tc, s->p, s->pw_order, s->order, st));
  else HIPCHK(launch_permutations(s->O.seed, s->O.instance, k0, Tc, s->n, s->pw, s->perm, st));
  HIPCHK(tm.end(RAC_PHASE_PARTITION));
  for (int64_t t = 0; t < Tc; ++t) {
    const int64_t k = k0 + t;
    const double* beta_ptr = beta_of(s, run_offset + t);
    const double bk = sched ? s->sched_host[run_offset + t] : s->hsc.beta;
    const int32_t* perm = s->rp ? s->iota : s->perm + t * s->n;
    const int32_t* ord = s->rp ? s->order + t * s->p : nullptr;
    tm.k = k;
    HIPCHK(tm.begin(st, RAC_PHASE_GRAM));
    if (s->Hb && !(bk == s->hb_beta)) {
      HIPCHK(launch_hbeta(P.Hd, P.H_dtype, P.ldH, s->n, s->meq, P.A, beta_ptr, s->Hb, st));
      s->hb_beta = bk;
      s->fac_beta = NAN;
    }
    if (s->meq > 0) HIPCHK(launch_ceff(s->n, s->meq, P.A, P.beq, s->mu_vec, beta_ptr, P.c, s->ceff, st));
    int32_t hdt = 0;
    int64_t hld = 0;
    const void* H = dense_H(s, &hdt, &hld);
    const bool refactor = !s->rp || !(bk == s->fac_beta);
    if (refactor) HIPCHK(launch_hgather(H, hdt, hld, s->n, s->p, perm, s->sp, s->partial, st));
    HIPCHK(tm.end(RAC_PHASE_GRAM));
    if (refactor) {
      FactorArgs f{};
      f.partial = s->partial; f.R = 1; f.sp = s->sp; f.n = s->n; f.p = s->p; f.perm = perm;
      f.Ns = 1.0; f.h = P.h; f.a = nullptr; f.beta_ptr = beta_ptr; f.beta_val = 0.0; f.Minv = s->Minv;
      f.write_matrix = 0; f.sc = s->sc; f.iter_global = k; f.order = ord;
      HIPCHK(tm.begin(st, RAC_PHASE_FACTOR));
      HIPCHK(launch_factor(f, st));
      HIPCHK(tm.end(RAC_PHASE_FACTOR));
      s->fac_beta = bk;
    }
    SweepArgs w{H, hdt, hld, s->n, s->n, s->p, perm, s->Minv, s->sp, s->meq > 0 ? s->ceff : P.c, P.h, nullptr,
                0.0, 1.0, s->x, s->z, s->xi, s->x, s->sc, s->sweep_part, s->flags, s->epoch, s->K,
                beta_ptr, s->tileA, s->tileB, 1, nullptr, s->max_spin, ord, 1};
    HIPCHK(tm.begin(st, RAC_PHASE_SWEEP));
    HIPCHK(launch_sweep(w, st));
    HIPCHK(tm.end(RAC_PHASE_SWEEP));
    s->epoch += (uint64_t)s->p;
    UpdateArgs za{};
    za.n = s->n; za.prox = P.prox; za.lam = P.lambda; za.alpha = P.alpha; za.lo = P.lo; za.hi = P.hi;
    za.b = 0.0; za.has_eq = 0; za.x = s->x; za.z = s->z; za.xi = s->xi; za.zprev = s->zprev;
    za.sc = s->sc; za.red = s->red; za.done = s->done; za.hist = s->hist; za.hist_cap = s->hist_cap;
    za.hist_base = k0 - run_offset; za.T = s->T; za.beta_ptr = beta_ptr; za.publish_beta = sched ? 1 : 0;
    za.extra_rp2 = s->meq > 0 ? s->eq_r2 : nullptr;
    HIPCHK(tm.begin(st, RAC_PHASE_ZDUAL));
    if (s->meq > 0)
      HIPCHK(launch_eq(s->n, s->meq, P.A, P.beq, s->x, beta_ptr, s->t_vec, s->mu_vec, s->eq_r2, s->eq_red,
                       s->eq_done, s->sc, st));
    HIPCHK(launch_zdual(za, st));
    HIPCHK(tm.end(RAC_PHASE_ZDUAL));
  }
  return enqueue_check(s, k0, Tc, run_offset, st, tm);
}

// Sparse-form chunk (one stream): partitions (RAC) or orders (RP); per iteration the
// block Grams from the sparse columns (RP: once) and their inverses (RP: when beta
// changed), the one-workgroup sweep, and the z/dual step; then the check.
rac_status enqueue_sparse_chunk(rac_solver s, int64_t Tc, int64_t run_offset, hipStream_t st) {
  const rac_problem& P = s->P;
  const SparseF SF = sparse_of(P);
  PhaseTimer tm{s, st};
  const int64_t k0 = s->hsc.k;
  const bool sched = s->O.beta_mode == RAC_BETA_SCHEDULE;
  tm.k = -1;
  HIPCHK(tm.begin(RAC_PHASE_PARTITION));
  if (s->rp) HIPCHK(launch_permutations(s->O.seed, s->O.instance, k0, Tc, s->p, s->pw_order, s->order, st));
  else HIPCHK(launch_permutations(s->O.seed, s->O.instance, k0, Tc, s->n, s->pw, s->perm, st));
  HIPCHK(tm.end(RAC_PHASE_PARTITION));
  for (int64_t t = 0; t < Tc; ++t) {
    const int64_t k = k0 + t;
    const double* beta_ptr = beta_of(s, run_offset + t);
    const double bk = sched ? s->sched_host[run_offset + t] : s->hsc.beta;
    const int32_t* perm = s->rp ? s->iota : s->perm + t * s->n;
    const int32_t* ord = s->rp ? s->order + t * s->p : nullptr;
    tm.k = k;
    if (!s->rp || !s->rp_gram) {
      HIPCHK(tm.begin(st, RAC_PHASE_GRAM));
      HIPCHK(launch_sgram(SF, s->n, s->p, perm, s->sp, s->partial, st));
      HIPCHK(tm.end(RAC_PHASE_GRAM));
      if (s->rp) { s->rp_gram = true; s->fac_beta = NAN; }
    }
    if (!s->rp || !(bk == s->fac_beta)) {
      FactorArgs f{};
      f.partial = s->partial; f.R = 1; f.sp = s->sp; f.n = s->n; f.p = s->p; f.perm = perm;
      f.Ns = P.Ns; f.h = P.h; f.a = P.a; f.beta_ptr = beta_ptr; f.beta_val = 0.0; f.Minv = s->Minv;
      f.write_matrix = 0; f.sc = s->sc; f.iter_global = k; f.order = ord;
      HIPCHK(tm.begin(st, RAC_PHASE_FACTOR));
      HIPCHK(launch_factor(f, st));
      HIPCHK(tm.end(RAC_PHASE_FACTOR));
      s->fac_beta = bk;
    }
    SweepArgs w{P.F, P.F_dtype, 0, s->rows, s->n, s->p, perm, s->Minv, s->sp, P.c, P.h, P.a, P.b, P.Ns, s->x,
                s->z, s->xi, s->u, s->sc, nullptr, nullptr, 0, 1, beta_ptr, 0, 0, 0, nullptr, s->max_spin, ord, 0};
    HIPCHK(tm.begin(st, RAC_PHASE_SWEEP));
    HIPCHK(launch_ssweep(SF, w, st));
    HIPCHK(tm.end(RAC_PHASE_SWEEP));
    UpdateArgs za{};
    za.n = s->n; za.prox = P.prox; za.lam = P.lambda; za.alpha = P.alpha; za.lo = P.lo; za.hi = P.hi;
    za.b = P.b; za.has_eq = P.a ? 1 : 0; za.x = s->x; za.z = s->z; za.xi = s->xi; za.zprev = s->zprev;
    za.sc = s->sc; za.red = s->red; za.done = s->done; za.hist = s->hist; za.hist_cap = s->hist_cap;
    za.hist_base = k0 - run_offset; za.T = s->T; za.beta_ptr = beta_ptr; za.publish_beta = sched ? 1 : 0;
    HIPCHK(tm.begin(st, RAC_PHASE_ZDUAL));
    HIPCHK(launch_zdual(za, st));
    HIPCHK(tm.end(RAC_PHASE_ZDUAL));
  }
  return enqueue_check(s, k0, Tc, run_offset, st, tm);
}

DenseKKTArgs dense_kkt_args(const rac_problem& P, const double* x, const double* z, const double* xi,
                            const double* t, const double* mu, double* part, double* red, uint32_t* done,
                            double* out) {
  DenseKKTArgs d{};
  d.Hd = P.Hd; d.dtype = P.H_dtype; d.ldH = P.ldH; d.n = P.n; d.h = P.h; d.c = P.c; d.meq = P.meq;
  d.A = P.A; d.beq = P.beq; d.t = t; d.mu = mu; d.prox = P.prox; d.lam = P.lambda; d.alpha = P.alpha;
  d.lo = P.lo; d.hi = P.hi; d.x = x; d.z = z; d.xi = xi; d.part = part; d.red = red; d.done = done; d.out = out;
  return d;
}

rac_status enqueue_iteration_chunk(rac_solver s, int64_t Tc, int64_t run_offset, hipStream_t st) {
  if (s->dense) return enqueue_dense_chunk(s, Tc, run_offset, st);
  if (s->sparse) return enqueue_sparse_chunk(s, Tc, run_offset, st);
  if (s->rp) return enqueue_rp_chunk(s, Tc, run_offset, st);
  const rac_problem& P = s->P;
  PhaseTimer tm{s, st};
  const int64_t k0 = s->hsc.k;
  const bool sched = s->O.beta_mode == RAC_BETA_SCHEDULE;
  hipStream_t sa = s->overlap ? s->sB : st;   // stream of the assemble phase
  const bool pre = s->overlap && s->pre_k == k0;   // partitions and first assemble already enqueued
  s->pre_k = -1;
  if (pre) {
    s->pbuf = 1 - s->pbuf;
  } else {
    s->pbuf = 0;
    tm.k = -1;
    HIPCHK(tm.begin(RAC_PHASE_PARTITION));
    HIPCHK(launch_permutations(s->O.seed, s->O.instance, k0, Tc, s->n, s->pw, s->perm, st));
    HIPCHK(tm.end(RAC_PHASE_PARTITION));
    if (s->overlap) {
      HIPCHK(hipEventRecord(s->ev_start, st));   // partitions drawn, previous chunk's penalty final
      HIPCHK(hipStreamWaitEvent(sa, s->ev_start, 0));
    }
  }
  const int32_t* pbase = s->perm + (size_t)s->pbuf * s->T * s->n;
  for (int64_t t = 0; t < Tc; ++t) {
    const int64_t k = k0 + t;
    const int32_t* perm = pbase + t * s->n;
    const int par = (int)(k & 1);
    double* Minv = s->Minv + par * (size_t)s->p * s->sp * s->sp;
    const double* beta_ptr = beta_of(s, run_offset + t);
    if (!(pre && t == 0)) {
      rac_status e = enqueue_gram(s, k, perm, sa, tm);
      if (e == RAC_OK) e = enqueue_factor(s, k, perm, beta_ptr, sa, tm);
      if (e != RAC_OK) return e;
    }
    if (s->overlap) HIPCHK(hipStreamWaitEvent(st, s->ev_fac[par], 0));
    const void* Fp = s->Fp ? (const void*)(s->Fp + par * s->Fp_bytes) : nullptr;
    SweepArgs w{P.F, P.F_dtype, P.ldF, s->rows, s->n, s->p, perm, Minv, s->sp, P.c, P.h, P.a,
                P.b, P.Ns, s->x, s->z, s->xi, s->u, s->sc, s->sweep_part, s->flags, s->epoch, s->K,
                beta_ptr, s->tileA, s->tileB, s->overlap ? 0 : 1, Fp, s->max_spin};
    tm.k = k;
    HIPCHK(tm.begin(st, RAC_PHASE_SWEEP));
    HIPCHK(launch_sweep(w, st));
    HIPCHK(tm.end(RAC_PHASE_SWEEP));
    if (s->overlap) {
      HIPCHK(hipEventRecord(s->ev_sweep[par], st));
      s->swept[par] = k;
    }
    s->epoch += (uint64_t)s->p;
    UpdateArgs za{};
    za.n = s->n; za.prox = P.prox; za.lam = P.lambda; za.alpha = P.alpha; za.lo = P.lo; za.hi = P.hi;
    za.b = P.b; za.has_eq = P.a ? 1 : 0; za.x = s->x; za.z = s->z; za.xi = s->xi; za.zprev = s->zprev;
    za.sc = s->sc; za.red = s->red; za.done = s->done; za.hist = s->hist; za.hist_cap = s->hist_cap;
    za.hist_base = k0 - run_offset; za.T = s->T; za.beta_ptr = beta_ptr; za.publish_beta = sched ? 1 : 0;
    tm.k = k;
    HIPCHK(tm.begin(st, RAC_PHASE_ZDUAL));
    HIPCHK(launch_zdual(za, st));
    HIPCHK(tm.end(RAC_PHASE_ZDUAL));
  }
  return enqueue_check(s, k0, Tc, run_offset, st, tm);
}

// KKT check after a chunk of Tc iterations starting at k0, then the stopping test
// and the penalty rule.
rac_status enqueue_check(rac_solver s, int64_t k0, int64_t Tc, int64_t run_offset, hipStream_t st, PhaseTimer& tm) {
  const rac_problem& P = s->P;
  if (s->dense) {
    tm.k = -1;
    HIPCHK(tm.begin(st, RAC_PHASE_CHECK));
    HIPCHK(launch_dkkt(dense_kkt_args(P, s->x, s->z, s->xi, s->t_vec, s->mu_vec, s->kkt_part, s->red, s->done,
                                      s->kkt_out), st));
    ControlArgs ca{};
    ca.sc = s->sc; ca.kkt_out = s->kkt_out; ca.beta_mode = s->O.beta_mode; ca.rb_mu = s->O.rb_mu;
    ca.rb_tau = s->O.rb_tau; ca.tol = s->O.tol; ca.mlp_w = s->O.mlp_weights; ca.mlp_ymax = s->O.mlp_ymax;
    ca.decide = ((k0 + Tc) % s->T == 0) ? 1 : 0; ca.hist = s->hist; ca.hist_cap = s->hist_cap;
    ca.hist_base = k0 - run_offset;
    HIPCHK(launch_control(ca, st));
    HIPCHK(tm.end(RAC_PHASE_CHECK));
    return RAC_OK;
  }
  KKTArgs ka{};
  ka.F = P.F; ka.dtype = P.F_dtype; ka.ldF = P.ldF; ka.rows = s->rows; ka.n = s->n; ka.Ns = P.Ns;
  ka.h = P.h; ka.c = P.c; ka.a = P.a; ka.b = P.b; ka.prox = P.prox; ka.lam = P.lambda;
  ka.alpha = P.alpha; ka.lo = P.lo; ka.hi = P.hi; ka.x = s->x; ka.z = s->z; ka.xi = s->xi;
  ka.u = s->u; ka.mu_ptr = &s->sc->mu; ka.mu_val = 0.0; ka.red = s->red; ka.done = s->done;
  ka.out = s->kkt_out; ka.part = s->kkt_part;
  tm.k = -1;
  HIPCHK(tm.begin(st, RAC_PHASE_CHECK));
  if (s->sparse) {
    HIPCHK(launch_sdots(sparse_of(P), s->n, s->u, 1.0, s->kkt_part, st));
    HIPCHK(launch_kkt_terms(ka, 1, st));
  } else {
    HIPCHK(launch_kkt(ka, st));
  }
  ControlArgs ca{};
  ca.sc = s->sc; ca.kkt_out = s->kkt_out; ca.beta_mode = s->O.beta_mode; ca.rb_mu = s->O.rb_mu;
  ca.rb_tau = s->O.rb_tau; ca.tol = s->O.tol; ca.mlp_w = s->O.mlp_weights; ca.mlp_ymax = s->O.mlp_ymax;
  ca.decide = ((k0 + Tc) % s->T == 0) ? 1 : 0; ca.hist = s->hist; ca.hist_cap = s->hist_cap;
  ca.hist_base = k0 - run_offset;
  HIPCHK(launch_control(ca, st));
  HIPCHK(tm.end(RAC_PHASE_CHECK));
  return RAC_OK;
}

}  // namespace

extern "C" {

const char* rac_status_str(rac_status s) {
  switch (s) {
    case RAC_OK: return "ok";
    case RAC_ERR_ARG: return "invalid argument";
    case RAC_ERR_NOT_PD: return "block matrix not positive definite (Assumption 2.1)";
    case RAC_ERR_DEVICE: return "HIP device error";
    case RAC_ERR_NOMEM: return "out of device memory";
    case RAC_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

rac_status rac_solver_create(const rac_problem* prob, const rac_opts* opts, rac_solver* out) {
  if (!out || !opts) return RAC_ERR_ARG;
  *out = nullptr;
  rac_status v = validate_problem(prob);
  if (v != RAC_OK) return v;
  v = check_problem_arrays(*prob);
  if (v != RAC_OK) return v;
  rac_opts O = *opts;
  const int64_t n = prob->n;
  if (O.num_blocks < 1 || O.num_blocks > n) return RAC_ERR_ARG;
  const int64_t smax = (n + O.num_blocks - 1) / O.num_blocks;
  if (smax > RAC_MAX_BLOCK) return RAC_ERR_ARG;
  if (!is_fin(O.beta0) || !(O.beta0 > 0.0)) return RAC_ERR_ARG;
  if (O.check_every < 1 || O.max_iter < 0 || !is_fin(O.tol) || O.tol < 0.0) return RAC_ERR_ARG;
  if (O.precision != RAC_PREC_FP64 && O.precision != RAC_PREC_MIXED) return RAC_ERR_ARG;
  if (O.beta_mode < RAC_BETA_FIXED || O.beta_mode > RAC_BETA_SCHEDULE) return RAC_ERR_ARG;
  if (O.rb_mu <= 0.0) O.rb_mu = 10.0;
  if (O.rb_tau <= 0.0) O.rb_tau = 2.0;
  if (!is_fin(O.rb_mu) || !is_fin(O.rb_tau) || O.rb_tau < 1.0) return RAC_ERR_ARG;
  if (!(O.mlp_ymax > 0.0)) O.mlp_ymax = std::log(10.0);
  if (O.beta_mode == RAC_BETA_MLP && !O.mlp_weights) return RAC_ERR_ARG;
  if (O.beta_mode == RAC_BETA_SCHEDULE) {
    if (!O.beta_schedule) return RAC_ERR_ARG;
    for (int64_t i = 0; i < O.max_iter; ++i)
      if (!is_fin(O.beta_schedule[i]) || !(O.beta_schedule[i] > 0.0)) return RAC_ERR_ARG;
  }
  if (O.sweep_groups < 0 || O.sweep_groups > 256 || O.row_chunks < 0) return RAC_ERR_ARG;
  if (O.variant != RAC_VARIANT_RAC && O.variant != RAC_VARIANT_RP) return RAC_ERR_ARG;

  rac_solver s = new (std::nothrow) rac_solver_s();
  if (!s) return RAC_ERR_NOMEM;
  s->P = *prob;
  s->O = O;
  s->n = n;
  s->rows = prob->rows;
  s->p = O.num_blocks;
  s->T = O.check_every;
  s->sp = padded(smax);
  s->rp = O.variant == RAC_VARIANT_RP;
  s->dense = is_dense(prob);
  s->sparse = is_sparse(prob);
  s->meq = s->dense ? prob->meq : 0;
  if (s->dense) s->rows = n;   // the sweep's rows are the Hessian's: x is its own residual
  // element type the sweep reads: F, or in the dense form H_beta (FP64) / Hd
  const int32_t sweep_dt = s->dense ? (s->meq > 0 ? (int32_t)RAC_DT_F64 : prob->H_dtype) : prob->F_dtype;
  {
    int A = 0, B = 0, K = 0;
    if (s->sparse) {
      s->tileA = s->tileB = 0;   // the sparse sweep is one workgroup
      s->K = 1;
    } else if (choose_tile(sweep_dt, s->rows, smax, O.sweep_groups, &A, &B, &K)) {
      s->tileA = A; s->tileB = B; s->K = K;
    } else if (s->dense) {
      delete s;
      return RAC_ERR_UNSUPPORTED;   // the dense form runs on the register-tile sweep only
    } else {
      s->tileA = s->tileB = 0;
      s->K = O.sweep_groups > 0 ? O.sweep_groups : auto_sweep_groups(prob->rows);
    }
  }
  if (s->K > s->rows) s->K = (int)s->rows;
  // overlap the assemble phase with the sweep when all sweep groups fit on the device at once
  const bool can_overlap = !s->rp && !s->dense && !s->sparse && s->tileA > 0 && s->K > 1 &&
                           s->K <= sweep_max_resident(prob->F_dtype, s->tileA, s->tileB) && O.overlap >= 0;
  s->R = (s->dense || s->sparse) ? 1 : (O.row_chunks > 0 ? O.row_chunks : auto_row_chunks(s->p, prob->rows));
  if (can_overlap && O.row_chunks == 0) {
    // leave the sweep's K compute units free of Gram workgroups: a sweep group needs
    // a whole compute unit, so the next iteration's Gram would otherwise delay it
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
      const int64_t cap = (cus - s->K) / s->p;
      if (cap < s->R) s->R = (int)(cap < 1 ? 1 : cap);
    }
  }
  if (s->R > s->rows) s->R = (int)s->rows;
  s->mv_nparts = matvec_parts(n);
  if (const char* e = std::getenv("RACMB_SWEEP_MAX_SPIN")) s->max_spin = std::atoi(e);

  auto fail = [&](rac_status r) {
    s->buf.release();
    if (s->hsc_pin) (void)hipHostFree(s->hsc_pin);
    if (s->ev_check) (void)hipEventDestroy(s->ev_check);
    if (s->ev_start) (void)hipEventDestroy(s->ev_start);
    for (int q = 0; q < 2; ++q) {
      if (s->ev_fac[q]) (void)hipEventDestroy(s->ev_fac[q]);
      if (s->ev_sweep[q]) (void)hipEventDestroy(s->ev_sweep[q]);
    }
    if (s->sB) (void)hipStreamDestroy(s->sB);
    delete s;
    return r;
  };
  rac_status r;
  if (hipHostMalloc((void**)&s->hsc_pin, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
    s->hsc_pin = nullptr;
    return fail(RAC_ERR_NOMEM);
  }
  if ((r = alloc_perm_work(s->buf, s->T, n, &s->pw, &s->perm)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->partial, (size_t)(s->p * s->R) * s->sp * s->sp)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->Minv, (size_t)(s->rp || s->dense || s->sparse ? 1 : 2) * s->p * s->sp * s->sp)) !=
      RAC_OK)
    return fail(r);
  if (s->dense) {
    if (s->meq > 0) {
      if ((r = s->buf.alloc(&s->Hb, (size_t)n * n)) != RAC_OK) return fail(r);
      if ((r = s->buf.alloc(&s->ceff, (size_t)n)) != RAC_OK) return fail(r);
    }
    if ((r = s->buf.alloc(&s->mu_vec, (size_t)RAC_MAX_EQ)) != RAC_OK) return fail(r);
    if ((r = s->buf.alloc(&s->t_vec, (size_t)RAC_MAX_EQ)) != RAC_OK) return fail(r);
    if ((r = s->buf.alloc(&s->eq_r2, 1)) != RAC_OK) return fail(r);
    if ((r = s->buf.alloc(&s->eq_red, (size_t)RAC_MAX_EQ)) != RAC_OK) return fail(r);
    if ((r = s->buf.alloc(&s->eq_done, 1)) != RAC_OK) return fail(r);
    if (hipMemset(s->mu_vec, 0, sizeof(double) * RAC_MAX_EQ) != hipSuccess ||
        hipMemset(s->t_vec, 0, sizeof(double) * RAC_MAX_EQ) != hipSuccess ||
        hipMemset(s->eq_r2, 0, sizeof(double)) != hipSuccess || hipMemset(s->eq_done, 0, sizeof(uint32_t)) != hipSuccess)
      return fail(RAC_ERR_DEVICE);
  }
  if (s->rp) {
    if ((r = alloc_perm_work(s->buf, s->T, s->p, &s->pw_order, &s->order)) != RAC_OK) return fail(r);
    if ((r = s->buf.alloc(&s->iota, (size_t)n)) != RAC_OK) return fail(r);
    std::vector<int32_t> id((size_t)n);
    for (int64_t j = 0; j < n; ++j) id[(size_t)j] = (int32_t)j;
    if (hipMemcpy(s->iota, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess)
      return fail(RAC_ERR_DEVICE);
  }
  if ((r = s->buf.alloc(&s->x, (size_t)n)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->z, (size_t)n)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->xi, (size_t)n)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->zprev, (size_t)n)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->u, (size_t)s->rows)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->sc, 1)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->sweep_part, (size_t)3 * s->K * kMaxBlock)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->flags, (size_t)s->K * kFlagStride)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->red, (size_t)kRedSlots)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->done, 4)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->kkt_out, 4)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->kkt_part, (size_t)kKKTChunks * n)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->obj_out, 1)) != RAC_OK) return fail(r);
  s->hist_cap = O.max_iter > 0 ? O.max_iter : 1;
  if ((r = s->buf.alloc(&s->hist, (size_t)s->hist_cap * 4)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->mv_part, (size_t)s->mv_nparts * s->rows)) != RAC_OK) return fail(r);
  if ((r = s->buf.alloc(&s->uz, (size_t)s->rows)) != RAC_OK) return fail(r);
  // packed copies of the blocks for the register-tile sweep (one per iteration parity)
  if (s->tileA > 0 && O.packed >= 0 && s->rows <= INT32_MAX && !s->dense && !s->sparse) {
    const size_t esz = prob->F_dtype == RAC_DT_F64 ? 8 : (prob->F_dtype == RAC_DT_F32 ? 4 : 2);
    s->Fp_bytes = (size_t)sweep_packed_elems(s->p, s->K, s->tileA, s->tileB) * esz;
    s->packRW = sweep_rows_per_group(s->rows, s->K, s->tileA);
    if (s->packRW <= 0) return fail(RAC_ERR_ARG);
    const size_t copies = s->rp ? 1 : 2;   // RP: one copy, written once
    if ((r = s->buf.alloc(&s->Fp, copies * s->Fp_bytes)) != RAC_OK) return fail(r);
    // positions that no entry of F maps to stay zero for the solver's lifetime
    if (hipMemset(s->Fp, 0, copies * s->Fp_bytes) != hipSuccess) return fail(RAC_ERR_DEVICE);
  }
  if (can_overlap) {
    if (hipStreamCreateWithFlags(&s->sB, hipStreamNonBlocking) != hipSuccess) return fail(RAC_ERR_DEVICE);
    bool ok = hipEventCreateWithFlags(&s->ev_start, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&s->ev_check, hipEventDisableTiming) == hipSuccess;
    for (int q = 0; q < 2 && ok; ++q)
      ok = hipEventCreateWithFlags(&s->ev_fac[q], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&s->ev_sweep[q], hipEventDisableTiming) == hipSuccess;
    if (!ok) return fail(RAC_ERR_DEVICE);
    s->overlap = true;
  }
  if (O.beta_mode == RAC_BETA_SCHEDULE) {
    if ((r = s->buf.alloc(&s->d_sched, (size_t)(O.max_iter > 0 ? O.max_iter : 1))) != RAC_OK) return fail(r);
    if (O.max_iter > 0 &&
        hipMemcpy(s->d_sched, O.beta_schedule, sizeof(double) * O.max_iter, hipMemcpyHostToDevice) != hipSuccess)
      return fail(RAC_ERR_DEVICE);
    if (s->rp || s->dense || s->sparse) s->sched_host.assign(O.beta_schedule, O.beta_schedule + O.max_iter);
    s->O.beta_schedule = nullptr;   // the caller's array is not kept
  }
  if (hipMemset(s->x, 0, sizeof(double) * n) != hipSuccess ||
      hipMemset(s->z, 0, sizeof(double) * n) != hipSuccess ||
      hipMemset(s->xi, 0, sizeof(double) * n) != hipSuccess ||
      hipMemset(s->zprev, 0, sizeof(double) * n) != hipSuccess ||
      hipMemset(s->u, 0, sizeof(double) * s->rows) != hipSuccess ||
      hipMemset(s->flags, 0, sizeof(uint64_t) * s->K * kFlagStride) != hipSuccess ||
      hipMemset(s->done, 0, sizeof(uint32_t) * 4) != hipSuccess)
    return fail(RAC_ERR_DEVICE);
  s->hsc = fresh_scalars(O.beta0);
  if (hipMemcpy(s->sc, &s->hsc, sizeof(DevScalars), hipMemcpyHostToDevice) != hipSuccess)
    return fail(RAC_ERR_DEVICE);
  if (hipDeviceSynchronize() != hipSuccess) return fail(RAC_ERR_DEVICE);
  *out = s;
  return RAC_OK;
}

rac_status rac_solver_destroy(rac_solver s) {
  if (!s) return RAC_ERR_ARG;
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  if (s->ev_start) (void)hipEventDestroy(s->ev_start);
  if (s->ev_check) (void)hipEventDestroy(s->ev_check);
  for (int q = 0; q < 2; ++q) {
    if (s->ev_fac[q]) (void)hipEventDestroy(s->ev_fac[q]);
    if (s->ev_sweep[q]) (void)hipEventDestroy(s->ev_sweep[q]);
  }
  if (s->sB) (void)hipStreamDestroy(s->sB);
  if (s->hsc_pin) (void)hipHostFree(s->hsc_pin);
  s->buf.release();
  delete s;
  return RAC_OK;
}

rac_status rac_solver_run(rac_solver s, void* stream, rac_result* res) {
  if (!s || !res) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  std::memset(res, 0, sizeof(*res));
  res->fail_iter = -1;
  res->fail_block = -1;
  s->hsc.status = 0;
  s->hsc.wait_abort = 0;
  s->hsc.fail_key = ~0ULL;
  HIPCHK(hipMemcpyAsync(&s->sc->status, &s->hsc.status, 2 * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(&s->sc->fail_key, &s->hsc.fail_key, sizeof(uint64_t), hipMemcpyHostToDevice, st));
  const int64_t budget = s->O.max_iter;
  const int64_t k_start = s->hsc.k;
  int64_t done_iters = 0;
  rac_status rc = RAC_OK;
  int32_t run_status = RAC_RUN_MAX_ITER;
  rac_status e = RAC_OK;
  s->pre_k = -1;
  s->swept[0] = s->swept[1] = -1;
  // the assemble stream starts after everything the caller enqueued before this run
  if (s->overlap) {
    HIPCHK(hipEventRecord(s->ev_start, st));
    HIPCHK(hipStreamWaitEvent(s->sB, s->ev_start, 0));
  }
  while (done_iters < budget) {
    const int64_t k = s->hsc.k;
    int64_t Tc = s->T - (k % s->T);
    if (Tc > budget - done_iters) Tc = budget - done_iters;
    e = enqueue_iteration_chunk(s, Tc, done_iters, st);
    if (e != RAC_OK) return e;
    HIPCHK(hipMemcpyAsync(s->hsc_pin, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    if (s->overlap && done_iters + Tc < budget) {
      const int64_t k1 = k + Tc;
      int64_t Tn = s->T - (k1 % s->T);
      if (Tn > budget - done_iters - Tc) Tn = budget - done_iters - Tc;
      if ((e = preissue_next_chunk(s, k1, Tn, done_iters + Tc, st)) != RAC_OK) return e;
    }
    HIPCHK(hipStreamSynchronize(st));
    s->hsc = *s->hsc_pin;
    if (s->hsc.wait_abort) {   // a sweep gave up waiting for its groups: the iterate is not usable
      if (s->overlap) (void)hipStreamSynchronize(s->sB);
      return RAC_ERR_DEVICE;
    }
    if ((e = collect_timing(s)) != RAC_OK) return e;
    done_iters += Tc;
    if (s->hsc.fail_key != ~0ULL) {
      res->fail_iter = (int64_t)(s->hsc.fail_key >> 32);
      res->fail_block = (int64_t)(s->hsc.fail_key & 0xffffffffULL);
      rc = RAC_ERR_NOT_PD;
      s->fac_beta = NAN;   // RP: the inverses of this beta are not usable
      break;
    }
    if (s->hsc.status == 1) { run_status = RAC_RUN_CONVERGED; break; }
    if (s->hsc.status == 2) { run_status = RAC_RUN_DIVERGED; break; }
  }
  s->hist_count = s->hsc.k - k_start;
  s->pre_k = -1;
  if (s->overlap) {   // work enqueued ahead on the assemble stream ends before anything after this run
    HIPCHK(hipEventRecord(s->ev_start, s->sB));
    HIPCHK(hipStreamWaitEvent(st, s->ev_start, 0));
  }
  // objective at z
  if (s->dense) {
    HIPCHK(launch_dobjective(dense_kkt_args(s->P, s->x, s->z, s->xi, s->t_vec, s->mu_vec, s->kkt_part, s->red,
                                            s->done, s->obj_out), s->z, s->P.obj_const, st));
  } else {
    e = fx_into_u(s, s->z, s->uz, st);
    if (e != RAC_OK) return e;
    HIPCHK(launch_objective_red(s->rows, s->n, s->P.Ns, s->P.h, s->P.c, s->P.prox, s->P.lambda,
                                s->P.alpha, s->P.obj_const, s->z, s->uz, s->red, s->done, s->obj_out, st));
  }
  double obj = NAN;
  HIPCHK(hipMemcpyAsync(&obj, s->obj_out, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  res->iters = s->hist_count;
  res->status = run_status;
  res->kkt = s->hsc.kkt;
  res->beta = s->hsc.beta;
  res->objective = obj;
  return rc;
}

rac_status rac_solver_set_state(rac_solver s, const double* x, const double* z, const double* xi,
                                double mu, double beta, int64_t iter, void* stream) {
  if (!s || !x || !z || !xi || !is_fin(mu) || !is_fin(beta) || !(beta > 0.0) || iter < 0)
    return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const size_t nb = sizeof(double) * s->n;
  HIPCHK(hipMemcpyAsync(s->x, x, nb, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(s->z, z, nb, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(s->xi, xi, nb, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(s->zprev, z, nb, hipMemcpyDeviceToDevice, st));
  if (!s->dense) {   // the dense form's residual is x itself
    rac_status e = fx_into_u(s, s->x, s->u, st);
    if (e != RAC_OK) return e;
  }
  s->hsc = fresh_scalars(beta);
  s->hsc.mu = mu;
  s->hsc.k = iter;
  HIPCHK(hipMemcpyAsync(s->sc, &s->hsc, sizeof(DevScalars), hipMemcpyHostToDevice, st));
  if (s->dense && s->meq > 0) {   // mu sets the first row's multiplier, the others start at zero
    double m[RAC_MAX_EQ] = {0.0};
    m[0] = mu;
    HIPCHK(hipMemcpyAsync(s->mu_vec, m, sizeof(double) * RAC_MAX_EQ, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (s->P.a) HIPCHK(launch_dot_red(s->P.a, s->x, s->n, s->red, s->done, &s->sc->t, st));
  HIPCHK(hipMemcpyAsync(&s->hsc, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

rac_status rac_solver_get_state(rac_solver s, double* x, double* z, double* xi, double* mu,
                                double* beta, int64_t* iter, void* stream) {
  if (!s) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const size_t nb = sizeof(double) * s->n;
  if (x) HIPCHK(hipMemcpyAsync(x, s->x, nb, hipMemcpyDeviceToDevice, st));
  if (z) HIPCHK(hipMemcpyAsync(z, s->z, nb, hipMemcpyDeviceToDevice, st));
  if (xi) HIPCHK(hipMemcpyAsync(xi, s->xi, nb, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(&s->hsc, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (mu) *mu = s->hsc.mu;
  if (beta) *beta = s->hsc.beta;
  if (iter) *iter = s->hsc.k;
  return RAC_OK;
}

rac_status rac_solver_set_timing(rac_solver s, int32_t enable) {
  return rac_solver_set_timing_mask(s, enable ? (1u << RAC_NUM_PHASES) - 1u : 0u);
}

rac_status rac_solver_set_timing_mask(rac_solver s, uint32_t mask) {
  if (!s || (mask >> RAC_NUM_PHASES) != 0) return RAC_ERR_ARG;
  s->tmask = mask;
  for (int q = 0; q < RAC_NUM_PHASES; ++q) { s->phase_ms[q] = 0.0; s->phase_count[q] = 0; }
  s->ev_phase.clear();
  return RAC_OK;
}

rac_status rac_solver_set_timing_stride(rac_solver s, int64_t stride) {
  if (!s || stride < 1) return RAC_ERR_ARG;
  s->tstride = stride;
  for (int q = 0; q < RAC_NUM_PHASES; ++q) { s->phase_ms[q] = 0.0; s->phase_count[q] = 0; }
  s->ev_phase.clear();
  return RAC_OK;
}

rac_status rac_solver_timing(rac_solver s, double* ms, int64_t* launches) {
  if (!s || !ms) return RAC_ERR_ARG;
  for (int q = 0; q < RAC_NUM_PHASES; ++q) {
    ms[q] = s->phase_ms[q];
    if (launches) launches[q] = s->phase_count[q];
  }
  return RAC_OK;
}

rac_status rac_solver_info(rac_solver s, int64_t* info) {
  if (!s || !info) return RAC_ERR_ARG;
  info[0] = s->p;
  info[1] = s->sp;
  info[2] = s->K;
  info[3] = s->R;
  info[4] = s->T;
  info[5] = s->tileA;
  info[6] = s->tileB;
  info[7] = s->overlap ? 1 : 0;
  return RAC_OK;
}

rac_status rac_solver_features(rac_solver s, float* out) {
  if (!s || !out) return RAC_ERR_ARG;
  DevScalars h;
  HIPCHK(hipMemcpy(&h, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
  for (int q = 0; q < RAC_MLP_IN; ++q) out[q] = h.feat[q];
  return RAC_OK;
}

rac_status rac_solver_scale_beta(rac_solver s, double mult, void* stream) {
  if (!s || !is_fin(mult) || !(mult > 0.0)) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_scale_beta(s->sc, mult, st));
  HIPCHK(hipMemcpyAsync(&s->hsc, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

rac_status rac_solver_history(rac_solver s, double* out, int64_t capacity, int64_t* count) {
  if (!s || !out || capacity < 0) return RAC_ERR_ARG;
  int64_t c = s->hist_count < s->hist_cap ? s->hist_count : s->hist_cap;
  if (c > capacity) c = capacity;
  if (c > 0) HIPCHK(hipMemcpy(out, s->hist, sizeof(double) * 4 * c, hipMemcpyDeviceToHost));
  if (count) *count = c;
  return RAC_OK;
}

namespace {
struct StateHeader {
  uint64_t magic;
  int64_t n, rows;
  uint64_t scalars_bytes;
  uint64_t epoch_unused;
};
constexpr uint64_t kStateMagic = 0x52414353544154ULL;  // "RACSTAT"
}  // namespace

size_t state_size(rac_solver s) {
  return sizeof(StateHeader) + sizeof(DevScalars) + sizeof(double) * (4 * s->n + s->rows) +
         (s->dense ? sizeof(double) * 2 * RAC_MAX_EQ : 0);
}

rac_status rac_state_export(rac_solver s, void* buf, size_t* bytes) {
  if (!s || !bytes) return RAC_ERR_ARG;
  const size_t need = state_size(s);
  if (!buf) {
    *bytes = need;
    return RAC_OK;
  }
  if (*bytes < need) return RAC_ERR_ARG;
  char* p = (char*)buf;
  StateHeader h{kStateMagic, s->n, s->rows, sizeof(DevScalars), 0};
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  HIPCHK(hipMemcpy(p, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
  p += sizeof(DevScalars);
  const size_t nb = sizeof(double) * s->n;
  HIPCHK(hipMemcpy(p, s->x, nb, hipMemcpyDeviceToHost)); p += nb;
  HIPCHK(hipMemcpy(p, s->z, nb, hipMemcpyDeviceToHost)); p += nb;
  HIPCHK(hipMemcpy(p, s->xi, nb, hipMemcpyDeviceToHost)); p += nb;
  HIPCHK(hipMemcpy(p, s->zprev, nb, hipMemcpyDeviceToHost)); p += nb;
  HIPCHK(hipMemcpy(p, s->u, sizeof(double) * s->rows, hipMemcpyDeviceToHost));
  p += sizeof(double) * s->rows;
  if (s->dense) {
    HIPCHK(hipMemcpy(p, s->mu_vec, sizeof(double) * RAC_MAX_EQ, hipMemcpyDeviceToHost));
    p += sizeof(double) * RAC_MAX_EQ;
    HIPCHK(hipMemcpy(p, s->t_vec, sizeof(double) * RAC_MAX_EQ, hipMemcpyDeviceToHost));
  }
  *bytes = need;
  return RAC_OK;
}

rac_status rac_state_import(rac_solver s, const void* buf, size_t bytes) {
  if (!s || !buf) return RAC_ERR_ARG;
  const size_t need = state_size(s);
  if (bytes < need) return RAC_ERR_ARG;
  const char* p = (const char*)buf;
  StateHeader h;
  std::memcpy(&h, p, sizeof(h));
  if (h.magic != kStateMagic || h.n != s->n || h.rows != s->rows || h.scalars_bytes != sizeof(DevScalars))
    return RAC_ERR_ARG;
  p += sizeof(h);
  std::memcpy(&s->hsc, p, sizeof(DevScalars));
  HIPCHK(hipMemcpy(s->sc, p, sizeof(DevScalars), hipMemcpyHostToDevice));
  p += sizeof(DevScalars);
  const size_t nb = sizeof(double) * s->n;
  HIPCHK(hipMemcpy(s->x, p, nb, hipMemcpyHostToDevice)); p += nb;
  HIPCHK(hipMemcpy(s->z, p, nb, hipMemcpyHostToDevice)); p += nb;
  HIPCHK(hipMemcpy(s->xi, p, nb, hipMemcpyHostToDevice)); p += nb;
  HIPCHK(hipMemcpy(s->zprev, p, nb, hipMemcpyHostToDevice)); p += nb;
  HIPCHK(hipMemcpy(s->u, p, sizeof(double) * s->rows, hipMemcpyHostToDevice));
  p += sizeof(double) * s->rows;
  if (s->dense) {
    HIPCHK(hipMemcpy(s->mu_vec, p, sizeof(double) * RAC_MAX_EQ, hipMemcpyHostToDevice));
    p += sizeof(double) * RAC_MAX_EQ;
    HIPCHK(hipMemcpy(s->t_vec, p, sizeof(double) * RAC_MAX_EQ, hipMemcpyHostToDevice));
  }
  return RAC_OK;
}

rac_status rac_permutation(uint64_t seed, uint64_t instance, int64_t iter, int64_t n, int32_t* perm,
                           void* stream) {
  if (n < 1 || n > (int64_t)INT32_MAX || !perm || iter < 0) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  Buffers B;
  PermWork w{};
  int32_t* tmp = nullptr;
  rac_status r = alloc_perm_work(B, 1, n, &w, &tmp);
  if (r != RAC_OK) { B.release(); return r; }
  hipError_t e = launch_permutations(seed, instance, iter, 1, n, w, tmp, st);
  if (e == hipSuccess) e = hipMemcpyAsync(perm, tmp, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  B.release();
  return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
}

rac_status rac_kkt_mu(const rac_problem* prob, const double* x, const double* z, const double* xi,
                      const double* mu, int64_t nmu, void* stream, double* out) {
  rac_status v = validate_problem(prob);
  if (v != RAC_OK) return v;
  const int64_t rows_eq = is_dense(prob) ? prob->meq : (prob->a ? 1 : 0);
  if (!x || !z || !xi || !out || nmu != rows_eq || (nmu > 0 && !mu)) return RAC_ERR_ARG;
  for (int64_t e = 0; e < nmu; ++e)
    if (!is_fin(mu[e])) return RAC_ERR_ARG;
  if (!is_dense(prob)) return rac_kkt(prob, x, z, xi, nmu ? mu[0] : 0.0, stream, out);
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = prob->n;
  Buffers B;
  double *t = nullptr, *mud = nullptr, *zero = nullptr, *r2 = nullptr, *ered = nullptr, *part = nullptr,
         *red = nullptr, *o = nullptr;
  uint32_t *done = nullptr, *edone = nullptr;
  rac_status r;
  if ((r = B.alloc(&t, RAC_MAX_EQ)) != RAC_OK || (r = B.alloc(&mud, RAC_MAX_EQ)) != RAC_OK ||
      (r = B.alloc(&zero, 1)) != RAC_OK || (r = B.alloc(&r2, 1)) != RAC_OK || (r = B.alloc(&ered, RAC_MAX_EQ)) != RAC_OK ||
      (r = B.alloc(&part, (size_t)kKKTChunks * n)) != RAC_OK || (r = B.alloc(&red, (size_t)kRedSlots)) != RAC_OK ||
      (r = B.alloc(&o, 4)) != RAC_OK || (r = B.alloc(&done, 1)) != RAC_OK || (r = B.alloc(&edone, 1)) != RAC_OK) {
    B.release();
    return r;
  }
  DevScalars* scr = nullptr;
  if ((r = B.alloc(&scr, 1)) != RAC_OK) { B.release(); return r; }
  const double z0 = 0.0;
  hipError_t e = hipMemsetAsync(done, 0, sizeof(uint32_t), st);
  if (e == hipSuccess) e = hipMemsetAsync(edone, 0, sizeof(uint32_t), st);
  if (e == hipSuccess) e = hipMemcpyAsync(zero, &z0, sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && nmu > 0) e = hipMemcpyAsync(mud, mu, sizeof(double) * nmu, hipMemcpyHostToDevice, st);
  // t = A x (a multiplier step with beta = 0 leaves mu as given)
  if (e == hipSuccess) e = launch_eq(n, prob->meq, prob->A, prob->beq, x, zero, t, mud, r2, ered, edone, scr, st);
  if (e == hipSuccess) e = launch_dkkt(dense_kkt_args(*prob, x, z, xi, t, mud, part, red, done, o), st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, o, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  B.release();
  return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
}

rac_status rac_kkt(const rac_problem* prob, const double* x, const double* z, const double* xi,
                   double mu, void* stream, double* out) {
  rac_status v = validate_problem(prob);
  if (v != RAC_OK) return v;
  if (!x || !z || !xi || !out || !is_fin(mu)) return RAC_ERR_ARG;
  if (is_dense(prob)) {
    if (prob->meq > 1) return RAC_ERR_ARG;   // several multipliers: rac_kkt_mu
    return rac_kkt_mu(prob, x, z, xi, &mu, prob->meq, stream, out);
  }
  hipStream_t st = (hipStream_t)stream;
  if (is_sparse(prob)) {
    Buffers B;
    double *u = nullptr, *part = nullptr, *red = nullptr, *o = nullptr;
    uint32_t* done = nullptr;
    rac_status r;
    if ((r = B.alloc(&u, (size_t)prob->rows)) != RAC_OK || (r = B.alloc(&part, (size_t)prob->n)) != RAC_OK ||
        (r = B.alloc(&red, (size_t)kRedSlots)) != RAC_OK || (r = B.alloc(&o, 4)) != RAC_OK ||
        (r = B.alloc(&done, 4)) != RAC_OK) {
      B.release();
      return r;
    }
    const SparseF SF = sparse_of(*prob);
    hipError_t e = hipMemsetAsync(done, 0, 4 * sizeof(uint32_t), st);
    if (e == hipSuccess) e = launch_sspmv(SF, prob->rows, prob->n, x, u, st);
    if (e == hipSuccess) e = launch_sdots(SF, prob->n, u, 1.0, part, st);
    if (e == hipSuccess) {
      KKTArgs ka{};
      ka.n = prob->n; ka.Ns = prob->Ns; ka.h = prob->h; ka.c = prob->c; ka.a = prob->a; ka.b = prob->b;
      ka.prox = prob->prox; ka.lam = prob->lambda; ka.alpha = prob->alpha; ka.lo = prob->lo; ka.hi = prob->hi;
      ka.x = x; ka.z = z; ka.xi = xi; ka.mu_ptr = nullptr; ka.mu_val = mu; ka.red = red; ka.done = done; ka.out = o;
      ka.part = part;
      e = launch_kkt_terms(ka, 1, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, o, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    B.release();
    return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
  }
  Buffers B;
  double *u = nullptr, *part = nullptr, *red = nullptr, *o = nullptr;
  uint32_t* done = nullptr;
  const int np = matvec_parts(prob->n);
  rac_status r;
  if ((r = B.alloc(&u, (size_t)prob->rows)) != RAC_OK || (r = B.alloc(&part, (size_t)np * prob->rows)) != RAC_OK ||
      (r = B.alloc(&red, (size_t)kRedSlots)) != RAC_OK || (r = B.alloc(&o, 4)) != RAC_OK ||
      (r = B.alloc(&done, 4)) != RAC_OK) {
    B.release();
    return r;
  }
  hipError_t e = hipMemsetAsync(done, 0, 4 * sizeof(uint32_t), st);
  if (e == hipSuccess)
    e = launch_matvec_F_parts(prob->F, prob->F_dtype, prob->ldF, prob->rows, prob->n, x, u, part, np, st);
  if (e == hipSuccess) {
    KKTArgs ka{};
    ka.F = prob->F; ka.dtype = prob->F_dtype; ka.ldF = prob->ldF; ka.rows = prob->rows; ka.n = prob->n;
    ka.Ns = prob->Ns; ka.h = prob->h; ka.c = prob->c; ka.a = prob->a; ka.b = prob->b;
    ka.prox = prob->prox; ka.lam = prob->lambda; ka.alpha = prob->alpha; ka.lo = prob->lo;
    ka.hi = prob->hi; ka.x = x; ka.z = z; ka.xi = xi; ka.u = u; ka.mu_ptr = nullptr; ka.mu_val = mu;
    ka.red = red; ka.done = done; ka.out = o;
    e = launch_kkt(ka, st);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, o, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  B.release();
  return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
}

rac_status rac_objective(const rac_problem* prob, const double* z, void* stream, double* out) {
  rac_status v = validate_problem(prob);
  if (v != RAC_OK) return v;
  if (!z || !out) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (is_dense(prob)) {
    Buffers B;
    double *part = nullptr, *red = nullptr, *o = nullptr;
    uint32_t* done = nullptr;
    rac_status r;
    if ((r = B.alloc(&part, (size_t)kKKTChunks * prob->n)) != RAC_OK || (r = B.alloc(&red, (size_t)kRedSlots)) != RAC_OK ||
        (r = B.alloc(&o, 1)) != RAC_OK || (r = B.alloc(&done, 1)) != RAC_OK) {
      B.release();
      return r;
    }
    hipError_t e = hipMemsetAsync(done, 0, sizeof(uint32_t), st);
    if (e == hipSuccess)
      e = launch_dobjective(dense_kkt_args(*prob, z, z, z, nullptr, nullptr, part, red, done, o), z, prob->obj_const,
                            st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, o, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    B.release();
    return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
  }
  Buffers B;
  double *u = nullptr, *part = nullptr, *red = nullptr, *o = nullptr;
  uint32_t* done = nullptr;
  const int np = matvec_parts(prob->n);
  rac_status r;
  if ((r = B.alloc(&u, (size_t)prob->rows)) != RAC_OK || (r = B.alloc(&part, (size_t)np * prob->rows)) != RAC_OK ||
      (r = B.alloc(&red, (size_t)kRedSlots)) != RAC_OK || (r = B.alloc(&o, 1)) != RAC_OK ||
      (r = B.alloc(&done, 4)) != RAC_OK) {
    B.release();
    return r;
  }
  hipError_t e = hipMemsetAsync(done, 0, 4 * sizeof(uint32_t), st);
  if (e == hipSuccess) {
    if (is_sparse(prob)) e = launch_sspmv(sparse_of(*prob), prob->rows, prob->n, z, u, st);
    else e = launch_matvec_F_parts(prob->F, prob->F_dtype, prob->ldF, prob->rows, prob->n, z, u, part, np, st);
  }
  if (e == hipSuccess)
    e = launch_objective_red(prob->rows, prob->n, prob->Ns, prob->h, prob->c, prob->prox, prob->lambda,
                             prob->alpha, prob->obj_const, z, u, red, done, o, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, o, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  B.release();
  return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
}

rac_status rac_regression_c_csc(const int64_t* colptr, const int32_t* rowidx, const void* values, int32_t dtype,
                                int64_t rows, int64_t n, double Ns, const double* y, double* c, void* stream) {
  if (!colptr || !rowidx || !values || !y || !c || rows < 1 || n < 1 || !is_fin(Ns) || !(Ns > 0.0) ||
      (dtype != RAC_DT_F64 && dtype != RAC_DT_F32))
    return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_sdots(SparseF{colptr, rowidx, values, dtype}, n, y, -1.0 / Ns, c, st));
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

rac_status rac_regression_c(const void* F, int32_t F_dtype, int64_t rows, int64_t n, int64_t ldF, double Ns,
                            const double* y, double* c, void* stream) {
  if (!F || !y || !c || rows < 1 || n < 1 || ldF < rows || dtype_size(F_dtype) == 0 || !is_fin(Ns) ||
      !(Ns > 0.0))
    return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_matvec_Ft(F, F_dtype, ldF, rows, n, y, -1.0 / Ns, c, st));
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

rac_status rac_block_matrices(const rac_problem* prob, int64_t p, uint64_t seed, uint64_t instance, int64_t iter,
                              double beta, int32_t precision, double* out, int64_t* sp_out, void* stream) {
  rac_status v = validate_problem(prob);
  if (v != RAC_OK) return v;
  if (p < 1 || p > prob->n || !out || iter < 0 || !is_fin(beta) || !(beta > 0.0)) return RAC_ERR_ARG;
  if (precision != RAC_PREC_FP64 && precision != RAC_PREC_MIXED) return RAC_ERR_ARG;
  const int64_t smax = (prob->n + p - 1) / p;
  if (smax > RAC_MAX_BLOCK) return RAC_ERR_ARG;
  if (is_dense(prob) && prob->meq > 1) return RAC_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int sp = padded(smax);
  const int R = auto_row_chunks(p, prob->rows);
  Buffers B;
  PermWork w{};
  int32_t* perm = nullptr;
  double* partial = nullptr;
  rac_status r = alloc_perm_work(B, 1, prob->n, &w, &perm);
  if (r == RAC_OK) r = B.alloc(&partial, (size_t)p * R * sp * sp);
  if (r != RAC_OK) { B.release(); return r; }
  const bool dense = is_dense(prob);
  hipError_t e = launch_permutations(seed, instance, iter, 1, prob->n, w, perm, st);
  if (e == hipSuccess) {
    if (dense) {
      e = launch_hgather(prob->Hd, prob->H_dtype, prob->ldH, prob->n, p, perm, sp, partial, st);
    } else if (is_sparse(prob)) {
      e = launch_sgram(sparse_of(*prob), prob->n, p, perm, sp, partial, st);
    } else {
      GramArgs g{prob->F, prob->F_dtype, prob->ldF, prob->rows, prob->n, p, perm, precision, R, sp, partial};
      e = launch_gram(g, st);
    }
  }
  if (e == hipSuccess) {
    FactorArgs f{};
    f.partial = partial; f.R = (dense || is_sparse(prob)) ? 1 : R; f.sp = sp; f.n = prob->n; f.p = p; f.perm = perm;
    f.Ns = dense ? 1.0 : prob->Ns;
    f.h = prob->h; f.a = dense ? (prob->meq == 1 ? prob->A : nullptr) : prob->a; f.beta_ptr = nullptr;
    f.beta_val = beta; f.Minv = out;
    f.write_matrix = 1; f.sc = nullptr; f.iter_global = iter;
    e = launch_factor(f, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  B.release();
  if (sp_out) *sp_out = sp;
  return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
}

rac_status rac_solver_get_multipliers(rac_solver s, double* mu, int64_t count) {
  if (!s || !mu) return RAC_ERR_ARG;
  const int64_t rows_eq = s->dense ? s->meq : (s->P.a ? 1 : 0);
  if (count != rows_eq) return RAC_ERR_ARG;
  if (count == 0) return RAC_OK;
  if (s->dense) {
    HIPCHK(hipMemcpy(mu, s->mu_vec, sizeof(double) * count, hipMemcpyDeviceToHost));
  } else {
    HIPCHK(hipMemcpy(&s->hsc, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
    mu[0] = s->hsc.mu;
  }
  return RAC_OK;
}

rac_status rac_solver_set_multipliers(rac_solver s, const double* mu, int64_t count) {
  if (!s || !mu) return RAC_ERR_ARG;
  const int64_t rows_eq = s->dense ? s->meq : (s->P.a ? 1 : 0);
  if (count != rows_eq) return RAC_ERR_ARG;
  for (int64_t e = 0; e < count; ++e)
    if (!is_fin(mu[e])) return RAC_ERR_ARG;
  if (count == 0) return RAC_OK;
  if (s->dense) HIPCHK(hipMemcpy(s->mu_vec, mu, sizeof(double) * count, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(&s->hsc, s->sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
  s->hsc.mu = mu[0];
  HIPCHK(hipMemcpy(&s->sc->mu, &mu[0], sizeof(double), hipMemcpyHostToDevice));
  return RAC_OK;
}

rac_status rac_svm_kernel_matrix(const void* X, int32_t X_dtype, int64_t n, int64_t r, const double* y, double gamma,
                                 double* Q, int64_t ldQ, void* stream) {
  if (!X || !y || !Q || n < 1 || r < 1 || ldQ < n || !is_fin(gamma) || !(gamma > 0.0)) return RAC_ERR_ARG;
  if (X_dtype != RAC_DT_F64 && X_dtype != RAC_DT_F32) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_gauss_q(X, X_dtype, n, r, y, gamma, Q, ldQ, st));
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

rac_status rac_svm_decision(const void* X, int32_t X_dtype, int64_t n, int64_t r, const double* y,
                            const double* alpha, double gamma, double bias, const void* V, int64_t m, double* f,
                            const double* labels, double* accuracy, void* stream) {
  if (!X || !y || !alpha || !V || !f || n < 1 || r < 1 || m < 1 || !is_fin(gamma) || !(gamma > 0.0) ||
      !is_fin(bias) || (accuracy && !labels))
    return RAC_ERR_ARG;
  if (X_dtype != RAC_DT_F64 && X_dtype != RAC_DT_F32) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_decision(X, X_dtype, n, r, alpha, y, gamma, V, m, bias, f, st));
  if (accuracy) {
    Buffers B;
    double *red = nullptr, *o = nullptr;
    uint32_t* done = nullptr;
    rac_status q;
    if ((q = B.alloc(&red, 256)) != RAC_OK || (q = B.alloc(&o, 1)) != RAC_OK || (q = B.alloc(&done, 1)) != RAC_OK) {
      B.release();
      return q;
    }
    hipError_t e = hipMemsetAsync(done, 0, sizeof(uint32_t), st);
    if (e == hipSuccess) e = launch_accuracy(f, labels, m, red, done, o, st);
    if (e == hipSuccess) e = hipMemcpyAsync(accuracy, o, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    B.release();
    return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
  }
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

rac_status rac_mlp_forward(const float* w, const float* feats, int64_t batch, float ymax, float* y, void* stream) {
  if (!w || !feats || !y || batch < 0 || !(ymax > 0.0f)) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_mlp_forward(w, feats, batch, ymax, y, st));
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

rac_status rac_mlp_loss_grad(const float* w, const float* feats, const float* target, int64_t batch, float ymax,
                             float* grad, double* loss, void* stream) {
  if (!w || !feats || !target || !grad || batch < 1 || !(ymax > 0.0f)) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  int nparts = (int)(batch < 256 ? batch : 256);
  Buffers B;
  float *part = nullptr, *lp = nullptr;
  rac_status r = B.alloc(&part, (size_t)nparts * RAC_MLP_NPARAM);
  if (r == RAC_OK) r = B.alloc(&lp, (size_t)nparts + 1);
  if (r != RAC_OK) { B.release(); return r; }
  hipError_t e = launch_mlp_loss_grad(w, feats, target, batch, ymax, grad, part, lp, nparts, st);
  float l = 0.f;
  if (e == hipSuccess) e = hipMemcpyAsync(&l, lp + nparts, sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  B.release();
  if (loss) *loss = (double)l;
  return e == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
}

rac_status rac_mlp_adam(float* w, const float* grad, float* m, float* v, int64_t t, float lr, float b1, float b2,
                        float eps, void* stream) {
  if (!w || !grad || !m || !v || t < 1) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_mlp_adam(w, grad, m, v, t, lr, b1, b2, eps, st));
  HIPCHK(hipStreamSynchronize(st));
  return RAC_OK;
}

}  // extern "C"
