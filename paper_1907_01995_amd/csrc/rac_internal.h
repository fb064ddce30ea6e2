// rac_internal.h -- shared declarations of the HIP kernels' host launchers and
// the device-side helpers used by every kernel file of the gfx950 library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "racmb.h"

namespace rac {

constexpr int kMaxBlock = RAC_MAX_BLOCK;
constexpr int kThreads = 256;           // four 64-wide wavefronts per workgroup
constexpr int kFlagStride = 16;         // uint64 words between sweep flags (128 B lines)

// Mutable scalar state kept on the device so the whole iteration runs without
// host round trips; the host reads it back once per chunk of T iterations.
struct DevScalars {
  double t;          // a'x, maintained by the sweep
  double mu;         // multiplier of the equality row
  double beta;       // current penalty
  double kkt;        // KKT residual at the last check
  double kkt_prev;   // KKT residual at the check before
  double last_l10;   // log10 of the last penalty multiplier
  double rp_first;   // primal residual of the first iteration (divergence test)
  double rp, rd;     // residuals of the last iteration
  double rp_win, rd_win;  // residuals at the first iteration of the current window
  double objective;
  int64_t k;         // iterations completed (global count)
  int64_t decisions; // controller decisions taken
  uint64_t fail_key; // (iteration << 32 | block) of the first non-PD block, or ~0
  int32_t status;    // 0 running, 1 converged, 2 diverged, 3 retired after a non-PD block
  int32_t wait_abort;  // set when a sweep's bounded wait for other groups ran out (device error)
  float feat[RAC_MLP_IN];   // controller features formed at the last check
};

// Element loads of the data matrix, converted exactly to FP64 / FP32.
__device__ __forceinline__ double ld_f64(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double ld_f64(const float* p, int64_t i) { return (double)p[i]; }
__device__ __forceinline__ double ld_f64(const uint16_t* p, int64_t i) {
  return (double)__uint_as_float(((uint32_t)p[i]) << 16);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// SplitMix64 (Steele, Lea & Flood 2014): state += 0x9e3779b97f4a7c15; output = mix(state).
__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;

__host__ __device__ __forceinline__ int64_t block_start(int64_t i, int64_t n, int64_t p) {
  return (i * n) / p;
}

// The batch stores each block inverse (symmetric, sp x sp) as its lower 16 x 16 tiles:
// tile (I, J), I >= J, row-major at (I (I + 1) / 2 + J) * 256.  Entry (i, j) is read
// from the tile that holds (max, min) of the tiles' indices (in a diagonal tile both).
__host__ __device__ __forceinline__ int64_t minv_off(int i, int j) {
  const int I = i >> 4, J = j >> 4;
  return I >= J ? (int64_t)((I * (I + 1) / 2 + J) * 256 + (i & 15) * 16 + (j & 15))
                : (int64_t)((J * (J + 1) / 2 + I) * 256 + (j & 15) * 16 + (i & 15));
}

// Partition key of variable j at iteration `iter` (a SplitMix64 chain).
__host__ __device__ __forceinline__ uint64_t perm_key(uint64_t seed, uint64_t inst, uint64_t iter,
                                                      uint64_t j) {
  uint64_t s1 = sm64_mix(seed + kGamma * (inst + 1));
  uint64_t s2 = sm64_mix(s1 + kGamma * (iter + 1));
  return sm64_mix(s2 + kGamma * (j + 1));
}

// ---------------------------------------------------------------------------
// Host launchers (one per kernel family).  All return hipError_t of the launch.

struct PermWork {          // scratch of the bucketed key sort (per iteration of a chunk)
  uint64_t* keys;          // [T][n]
  uint32_t* count;         // [T][nb]  (kept zero between uses)
  uint32_t* offset;        // [T][nb+1]
  uint32_t* fill;          // [T][nb]  (kept zero between uses)
  int32_t* members;        // [T][n]
  int64_t nb;              // buckets per iteration (power of two >= n)
  int log2nb;
};
hipError_t launch_permutations(uint64_t seed, uint64_t inst, int64_t iter0, int64_t T, int64_t n,
                               const PermWork& w, int32_t* perm /* [T][n] */, hipStream_t st);

// Destination of the packed copy that the Gram kernel writes for the register-tile
// sweep (Fp null: none): K groups of RW rows, tiles of 64A rows x 4B columns.
struct PackDst {
  void* Fp;
  int64_t RW;
  int K, A, B;
};
struct GramArgs {
  const void* F; int32_t dtype; int64_t ldF; int64_t rows; int64_t n; int64_t p;
  const int32_t* perm;     // this iteration's permutation
  int32_t precision;       // rac_precision
  int R;                   // row chunks
  int sp;                  // padded block size (multiple of 16, <= 128)
  double* partial;         // [p][R][sp*sp]
  PackDst pack;            // packed copy written alongside (optional)
};
hipError_t launch_gram(const GramArgs& a, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched engine: many instances (each with its own data) and lanes (each an
// independent solve on one instance's data, sharing its partitions and block
// Grams).  All arrays below are device resident.
struct BInst {             // one instance (data, sizes, partition)
  const void* F; int64_t ldF, rows, n, p;
  int64_t poff;            // offset of the instance's partitions in the chunk buffer (T * n entries)
  int64_t goff;            // first block Gram of the instance in the Gram buffer
  uint64_t key_instance;   // instance id mixed into the partition keys
  int32_t vec;             // 16-byte vector loads allowed
  int32_t pad;
};
struct BUnit {             // one lane: an independent solve on instance `inst`
  const void* F; int64_t ldF, rows, n, p; double Ns;
  const double* h; const double* c; const double* a; double b;
  int32_t prox; int32_t inst; double lam, alpha, lo, hi;
  int64_t xoff;            // offset of x, z, xi, zprev (n entries each)
  int64_t uoff;            // offset of u (rows entries)
  int64_t goff;            // first block Gram of its instance
  int64_t moff;            // first block inverse of this lane
  int64_t poff;            // partitions of its instance
};
struct BatchGramArgs {      // Grams of iterations t .. t + nt - 1 of a chunk, iteration t' into G + t' gslot
  int32_t dtype; int32_t precision; int sp; int ntasks; int t; int nt; int64_t gslot;
  const BInst* inst; const int2* tasks; const int32_t* perm; const int32_t* inst_active; double* G;
};
hipError_t launch_bgram(const BatchGramArgs& a, hipStream_t st);

struct BatchArgs {         // everything the per-lane kernels of one chunk need
  int32_t dtype; int sp; int T; int nunits; int ninst; int np2;
  uint64_t seed;
  const BInst* inst; const BUnit* units;
  int32_t* perm; const double* G; double* Minv;
  const int2* inv_tasks; int ninv;
  double* X; double* Z; double* XI; double* ZP; double* U;
  DevScalars* sc;
  double* kpart; int KC;   // KKT partials: [unit][KC][10]
  int32_t* inst_active; int32_t* nactive; int64_t* kdev;
  int32_t beta_mode; double rb_mu, rb_tau, tol; const float* mlp_w; double mlp_ymax;
  int unroll;              // sweep row unroll (autotuned: 1, 2 or 4)
  int64_t gslot, mslot;    // doubles between the Gram / inverse slots of consecutive iterations of
                           // a chunk (0: one slot, formed at each iteration)
};
struct BinvSlots {         // inverses of iterations t0 + blockIdx.y; tk0: the chunk iteration the
  int t0; int tk0;         // lanes' counters stand at when the launch runs (failure reports)
  int64_t gslot, mslot;
};
// Team sweep (tsweep.hip): lane groups of one instance advanced together.
struct TGroup {            // up to 16 lanes of one instance
  int32_t inst; int32_t nl;
  int32_t vec4;            // F columns allow aligned 4-element vector loads
  int32_t vec8;            // ... and aligned 16-byte loads of two-byte data
  int32_t span;            // vec4, and F's allocation holds n * ldF elements: loads clamped
                           // into a column's ldF rows stay inside it
  int32_t lane[16];        // lane ids of slots 0 .. nl-1
};
struct TeamArgs {
  const TGroup* groups;
  const int32_t* team_off; // groups of team k: team_list[team_off[k] .. team_off[k+1])
  const int32_t* team_list;
  const int32_t* team_w;   // workgroups of team k (16 or 32)
  const int64_t* team_part;// offset (doubles) of team k's partial area [2][16 slots][W_k][64 columns]
  const int32_t* blk_team; // team of workgroup b (-1: idle), and its member index
  const int32_t* blk_member;
  int nteams; int nblocks; // teams, workgroups launched
  int NT;                  // register tiles of 16 rows per wavefront (8, or 10 for BF16 data)
  double* part;            // gradient partials of all teams
  double* delta;           // [nteams][2][64 columns][16 slots] steps
  uint32_t* flags;         // [nteams][128]: [0, 64) partial epochs, [64, 128) step epochs
  uint32_t* abort_flag;    // raised when a wait gives up (the batch is then unusable)
};
// Instances with at most this many rows may run their lane groups solo (one workgroup,
// no exchange); larger ones run on teams.  A candidate stays solo only while its group's
// predicted sweep fits under the predicted sweep of the whole batch, and the groups go
// to teams once few lanes remain active.  RACMB_SOLO_ROWS overrides the bound at batch
// creation; RACMB_SOLO_FORCE=1 keeps every candidate solo at creation.  (Measured on 256
// elastic-net instances of 1000 to 20000 rows: 4000 and 6000 rows give the shortest
// sweep, 6.08 and 6.05 ms against 6.65 ms at 2500 and 7.54 ms with teams only.)
constexpr int64_t kSoloRows = 4000;
// Workgroups of the team sweep that can be resident at once (0 if NT unsupported).
int tsweep_max_resident(int32_t dtype, int NT);
hipError_t launch_tsweep(const BatchArgs& b, const TeamArgs& ta, int t, hipStream_t st);
// KKT terms of lane groups, one workgroup per (group, pair of 64-column chunks) task.
hipError_t launch_gkkt(const BatchArgs& b, const TGroup* groups, const int2* tasks, int ntasks, hipStream_t st);

hipError_t launch_bperm(const BatchArgs& b, hipStream_t st);
hipError_t launch_binv(const BatchArgs& b, int t0, int nt, int tk0, hipStream_t st);
hipError_t launch_bsweep(const BatchArgs& b, int t, hipStream_t st);
hipError_t launch_bzdual(const BatchArgs& b, hipStream_t st);
// KKT (unless grouped_kkt: already formed by launch_gkkt), control, activity
hipError_t launch_bcheck(const BatchArgs& b, int Tc, int decide, int grouped_kkt, hipStream_t st);

struct FactorArgs {
  const double* partial; int R; int sp; int64_t n; int64_t p; const int32_t* perm;
  double Ns; const double* h; const double* a; const double* beta_ptr; double beta_val;
  double* Minv;            // [p][sp*sp] inverse block matrices (or the block matrices
  int write_matrix;        //  themselves when write_matrix != 0)
  DevScalars* sc;          // failure reporting (may be null)
  int64_t iter_global;
  const int32_t* order;    // RP: solve order of iteration iter_global (a failure is reported at the
                           // failing block's position in it); null: blocks are positions already
};
hipError_t launch_factor(const FactorArgs& a, hipStream_t st);

struct SweepArgs {
  const void* F; int32_t dtype; int64_t ldF; int64_t rows; int64_t n; int64_t p;
  const int32_t* perm; const double* Minv; int sp;
  const double* c; const double* h; const double* a; double b; double Ns;
  double* x; const double* z; const double* xi; double* u;
  DevScalars* sc;
  double* partials;        // [3][K][kMaxBlock]
  uint64_t* flags;         // [K * kFlagStride], monotone epochs
  uint64_t epoch_base;
  int K;
  const double* beta_ptr;  // penalty of this iteration
  int tileA, tileB;        // register tile: rows per lane, columns per wavefront (0: streaming path)
  int cooperative;         // launch with the cooperative API (else a plain launch, K <= resident limit)
  const void* Fp;          // packed tiles of this iteration written by the Gram kernel, or null (gather from F)
  int max_spin;            // polls before a sweep group gives up waiting (negative: the default)
  const int32_t* order;    // RP: block solved at position i is order[i] (its inverse and packed tiles
                           // are stored at that index); null: position i is block i
  int dense;               // dense form: F is the symmetric n x n Hessian and u is x (register-tile sweep only)
};
// Rows per sweep group for K groups and A rows per lane (0 if 64A rows do not cover a group).
int64_t sweep_rows_per_group(int64_t rows, int K, int A);
// Elements of one packed copy of F for the register-tile sweep: p * K * 256 * A * B.
int64_t sweep_packed_elems(int64_t p, int K, int A, int B);

// Largest number of sweep workgroups that can be resident at once for a tile shape.
int sweep_max_resident(int32_t dtype, int A, int B);
// Register-tile shapes with a compiled sweep kernel (A rows per lane, B columns per wavefront).
bool sweep_tile_supported(int32_t dtype, int A, int B);
hipError_t launch_sweep(const SweepArgs& a, hipStream_t st);

// Dense form (dense.hip): H_beta = Hd + beta A'A, c_eff = c - A'(beta beq + mu), the
// block matrices gathered from H_beta, t = A x with the multiplier step, the KKT residual
// and the objective, and the Gaussian-kernel matrix and decision values of the SVM dual.
hipError_t launch_hbeta(const void* Hd, int32_t dtype, int64_t ldH, int64_t n, int meq, const double* A,
                        const double* beta_ptr, double* Hb, hipStream_t st);
hipError_t launch_ceff(int64_t n, int meq, const double* A, const double* beq, const double* mu,
                       const double* beta_ptr, const double* c, double* ceff, hipStream_t st);
hipError_t launch_hgather(const void* H, int32_t dtype, int64_t ldH, int64_t n, int64_t p, const int32_t* perm,
                          int sp, double* out, hipStream_t st);
hipError_t launch_eq(int64_t n, int meq, const double* A, const double* beq, const double* x, const double* beta_ptr,
                     double* t, double* mu, double* r2, double* red, uint32_t* done, DevScalars* sc, hipStream_t st);
struct DenseKKTArgs {
  const void* Hd; int32_t dtype; int64_t ldH; int64_t n;
  const double* h; const double* c; int meq; const double* A; const double* beq;
  const double* t;         // A x at the current x (meq)
  const double* mu;        // multipliers (meq)
  int32_t prox; double lam, alpha, lo, hi;
  const double* x; const double* z; const double* xi;
  double* part;            // [kKKTChunks][n] column products
  double* red; uint32_t* done;
  double* out;             // KKT: [4]; objective: [1]
};
hipError_t launch_dkkt(const DenseKKTArgs& k, hipStream_t st);
hipError_t launch_dobjective(const DenseKKTArgs& k, const double* z, double cst, hipStream_t st);
hipError_t launch_gauss_q(const void* X, int32_t dtype, int64_t n, int64_t r, const double* y, double gamma,
                          double* Q, int64_t ldQ, hipStream_t st);
hipError_t launch_decision(const void* X, int32_t dtype, int64_t n, int64_t r, const double* alpha,
                           const double* y, double gamma, const void* V, int64_t m, double bias, double* f,
                           hipStream_t st);
hipError_t launch_accuracy(const double* f, const double* labels, int64_t m, double* red, uint32_t* done,
                           double* out, hipStream_t st);
// Column products Hd_j'v over row chunks into part [nch][n] (nch returned through *nch).
hipError_t launch_hd_dots(const void* Hd, int32_t dtype, int64_t ldH, int64_t n, const double* v, double* part,
                          int* nch, hipStream_t st);

// Sparse factor form (sparse.hip): F as compressed sparse columns.
struct SparseF {
  const int64_t* colptr;   // n + 1 offsets
  const int32_t* rowidx;   // row of each stored entry, strictly increasing within a column
  const void* val;         // values, dtype RAC_DT_F64 or RAC_DT_F32
  int32_t dtype;
};
hipError_t launch_sgram(const SparseF& F, int64_t n, int64_t p, const int32_t* perm, int sp, double* out,
                        hipStream_t st);
hipError_t launch_ssweep(const SparseF& F, const SweepArgs& w, hipStream_t st);
// out[j] = scale * F_j'v
hipError_t launch_sdots(const SparseF& F, int64_t n, const double* v, double scale, double* out, hipStream_t st);
// u = F x (u zeroed first; device-scope atomic additions)
hipError_t launch_sspmv(const SparseF& F, int64_t rows, int64_t n, const double* x, double* u, hipStream_t st);

struct UpdateArgs {
  int64_t n; int32_t prox; double lam, alpha, lo, hi; double b; int has_eq;
  const double* x; double* z; double* xi; double* zprev;
  DevScalars* sc;
  double* red;             // reduction scratch (>= 2 per workgroup)
  uint32_t* done;          // completion counter (kept zero between uses)
  double* hist;            // [cap][4] or null
  int64_t hist_cap;
  int64_t hist_base;       // global iteration index of this run's first iteration
  int64_t T;               // check period (window start bookkeeping)
  const double* beta_ptr;  // penalty of this iteration
  int publish_beta;        // copy *beta_ptr into sc->beta (given schedules)
  const double* extra_rp2; // dense form: |A x - beq|^2 added to r_p^2 (formed with the multiplier step), or null
};
hipError_t launch_zdual(const UpdateArgs& a, hipStream_t st);

constexpr int kRedSlots = 10 * 256;   // doubles of reduction scratch needed by any kernel

struct KKTArgs {
  const void* F; int32_t dtype; int64_t ldF; int64_t rows; int64_t n; double Ns;
  const double* h; const double* c; const double* a; double b; int32_t prox;
  double lam, alpha, lo, hi;
  const double* x; const double* z; const double* xi;
  const double* u;         // F x (rows)
  const double* mu_ptr; double mu_val;   // mu from the device scalars, or a value
  double* red;             // kRedSlots doubles
  uint32_t* done;
  double* out;             // [4] KKT, feas, stat, dual
  double* part;            // [kKKTChunks][n] partial F_j'u over row chunks, or null (one pass per column)
};
constexpr int kKKTChunks = 4;   // row chunks of the two-pass KKT check
hipError_t launch_kkt(const KKTArgs& a, hipStream_t st);
// The per-column terms and reduction of the check from column products already in a.part
// (nch row chunks of n values each).
hipError_t launch_kkt_terms(const KKTArgs& a, int nch, hipStream_t st);

struct ControlArgs {
  DevScalars* sc; const double* kkt_out; int32_t beta_mode; double rb_mu, rb_tau, tol;
  const float* mlp_w; double mlp_ymax; int decide; double* hist; int64_t hist_cap;
  int64_t hist_base;
};
hipError_t launch_control(const ControlArgs& a, hipStream_t st);
// beta *= mult, recorded as a controller decision (log10 multiplier, decision count)
hipError_t launch_scale_beta(DevScalars* sc, double mult, hipStream_t st);

// u = F x through nparts column-chunk partials (part: nparts*rows doubles), fixed-order sum.
hipError_t launch_matvec_F_parts(const void* F, int32_t dtype, int64_t ldF, int64_t rows, int64_t n,
                                 const double* x, double* u, double* part, int nparts,
                                 hipStream_t st);
// *flag |= 1 if any of rows x cols elements (column-major, leading dimension ld) is NaN or
// infinite (BF16: exponent bits all set)
hipError_t launch_nonfinite(const void* p, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, uint32_t* flag,
                            hipStream_t st);
// RAC_ERR_ARG if a device array of a problem holds a NaN or an infinity (one read of it)
rac_status check_problem_arrays(const rac_problem& P);
// out = scale F'u
hipError_t launch_matvec_Ft(const void* F, int32_t dtype, int64_t ldF, int64_t rows, int64_t n,
                            const double* u, double scale, double* out, hipStream_t st);
hipError_t launch_dot_red(const double* a, const double* x, int64_t n, double* red, uint32_t* done,
                          double* out, hipStream_t st);
// objective from u = F z
hipError_t launch_objective_red(int64_t rows, int64_t n, double Ns, const double* h, const double* c,
                                int32_t prox, double lam, double alpha, double cst, const double* z,
                                const double* u, double* red, uint32_t* done, double* out,
                                hipStream_t st);

// Controller network
hipError_t launch_mlp_forward(const float* w, const float* feats, int64_t batch, float ymax,
                              float* y, hipStream_t st);
hipError_t launch_mlp_loss_grad(const float* w, const float* feats, const float* target,
                                int64_t batch, float ymax, float* grad, float* partial_grad,
                                float* loss_part, int nparts, hipStream_t st);
hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int64_t t, float lr,
                           float b1, float b2, float eps, hipStream_t st);

}  // namespace rac
