// batch.hip -- the batched engine: many instances of uneven size, each with
// several lanes (independent solves on the instance's data, e.g. the points of
// a lambda grid), advanced together one iteration at a time with one launch per
// phase for the whole batch.  Lanes of an instance share its partitions (the
// partition of Eq.(3) is drawn per instance) and its block Grams; each lane has
// its own penalty, block inverses, iterate, residual, duals and controller.
//
// Kernels (one launch each per iteration, all lanes at once):
//   k_bperm   one workgroup per (instance, iteration of the chunk): the
//             instance's keys sorted by a distribution sort in LDS (n <= 8192);
//   k_bgram   (assemble.hip) one workgroup per (instance, block), the Gram
//             stored whole (exactly symmetric) so that the inverse kernels
//             read its rows with coalesced loads;
//   k_binv    one wavefront per (lane, block): the block matrix in registers,
//             one column per lane, inverted by Gauss-Jordan with symmetric
//             pivots; the pivot row (equal to the pivot column) is gathered
//             with one LDS store per lane and read back as broadcasts -- no
//             workgroup barriers;
//   k_binv64  the same for blocks of 64, four pivots per step on the FP64
//             matrix cores.  The inverses are symmetric; only their lower 16 x 16
//             tiles are stored (minv_off);
//   k_tsweep  (tsweep.hip) the team sweep: the lanes of an instance in groups
//             of up to 16, one read of the data for the whole group;
//   k_bsweep  the per-lane fallback, one workgroup per lane: the Gauss-Seidel pass over the blocks,
//             gradient pass (rows over lanes, columns over wavefronts,
//             transposed butterfly) and residual update pass per block;
//   k_bzdual  one workgroup per lane: z block, dual step, norms;
//   k_bkkt / k_bcontrol / k_bactive: KKT residual per lane, the stopping test
//             and penalty rule (shared with the single-instance engine), and the
//             per-instance activity used to skip retired work.
// Retired lanes (converged or diverged) return immediately from every kernel.
#include "control.h"
#include "rac_internal.h"

namespace rac {
namespace {

__device__ __forceinline__ double bsum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  __syncthreads();
  return s;
}
__device__ __forceinline__ double bmax(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, sh[w]);
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Partitions: one workgroup per (instance, iteration of the chunk) sorts the
// instance's variables by (key, index) with a distribution sort in LDS.  Keys
// are uniform 64-bit values, so their top lg bits pick one of nb = 2^lg >= n
// buckets (about one key per bucket): the buckets are counted, scanned into
// output ranges, filled through per-bucket cursors (in arrival order), and each
// variable's position inside its bucket is its rank among the bucket's members
// under (key, index), with the members' keys recomputed from their indices.  The
// order is the exact lexicographic order, so it equals the single-instance
// permutation, whatever the atomics' arrival order.
__device__ __forceinline__ uint32_t key_bucket(uint64_t key, int lg) {
  return lg == 0 ? 0u : (uint32_t)(key >> (64 - lg));
}

__global__ void __launch_bounds__(1024) k_bperm(const BInst* __restrict__ inst, uint64_t seed,
                                                const int64_t* __restrict__ kdev, int32_t* __restrict__ perm,
                                                const int32_t* __restrict__ inst_active, int np2max) {
  const int i = blockIdx.x, t = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (!inst_active[i]) return;
  const BInst I = inst[i];
  const int n = (int)I.n;
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  const int nb = 1 << lg;                                   // nb <= np2max
  extern __shared__ unsigned char smem[];
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem);       // [np2max]: counts, then cursors
  uint32_t* off = cnt + np2max;                            // [np2max + 1]: bucket starts
  int32_t* slot = reinterpret_cast<int32_t*>(off + np2max + 1);   // [np2max]: members, by bucket
  __shared__ uint32_t wsum[16];
  const uint64_t iter = (uint64_t)(*kdev + t);
  for (int b = tid; b < nb; b += 1024) cnt[b] = 0u;
  __syncthreads();
  for (int j = tid; j < n; j += 1024) atomicAdd(&cnt[key_bucket(perm_key(seed, I.key_instance, iter, (uint64_t)j), lg)], 1u);
  __syncthreads();
  // exclusive scan of the counts: a contiguous segment per thread, the segments'
  // sums scanned within each wavefront and then over the wavefronts
  const int per = (nb + 1023) / 1024;
  const int lo = tid * per < nb ? tid * per : nb, hi = lo + per < nb ? lo + per : nb;
  uint32_t seg = 0u;
  for (int b = lo; b < hi; ++b) seg += cnt[b];
  uint32_t inc = seg;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t base = 0u;
  for (int w = 0; w < wave; ++w) base += wsum[w];
  uint32_t run = base + inc - seg;
  for (int b = lo; b < hi; ++b) {
    const uint32_t c = cnt[b];
    off[b] = run;
    cnt[b] = run;                                           // the bucket's cursor
    run += c;
  }
  if (tid == 0) off[nb] = (uint32_t)n;
  __syncthreads();
  for (int j = tid; j < n; j += 1024) {
    const uint32_t b = key_bucket(perm_key(seed, I.key_instance, iter, (uint64_t)j), lg);
    slot[atomicAdd(&cnt[b], 1u)] = j;
  }
  __syncthreads();
  int32_t* out = perm + I.poff + (int64_t)t * n;
  for (int j = tid; j < n; j += 1024) {
    const uint64_t key = perm_key(seed, I.key_instance, iter, (uint64_t)j);
    const uint32_t b = key_bucket(key, lg);
    const uint32_t s0 = off[b], s1 = off[b + 1];
    uint32_t rank = 0u;
    for (uint32_t s = s0; s < s1; ++s) {
      const int32_t m = slot[s];
      if (m == j) continue;
      const uint64_t km = perm_key(seed, I.key_instance, iter, (uint64_t)m);
      rank += (km < key || (km == key && m < j)) ? 1u : 0u;
    }
    out[s0 + rank] = j;
  }
}

// ---------------------------------------------------------------------------
// Block inverses: one wavefront per (lane, block).  Lane j holds column j of
// M = G/Ns + diag(h) + beta (I + a a') in registers and the wavefront applies
// the symmetric sweep operator to pivots 0..sb-1:
//   a_ij -= a_ik a_kj / d,  a_kj /= d,  a_ik /= d,  a_kk = -1/d   (d = a_kk),
// after which the block holds -M^{-1}.  d is the k-th Schur-complement pivot,
// i.e. the squared Cholesky pivot; a non-positive one is reported as a failure
// of Assumption 2.1 for the lane.  Because the running matrix stays symmetric,
// the pivot column a_ik equals the pivot row a_ki, which every lane holds in
// its own registers: one LDS store per lane gathers it for the whole wavefront.
// The registers are renumbered after every pivot (register r holds row
// (r + k) mod SP), so the pivot row is always register 0 and every register
// index is a compile-time constant.
template <int SP>
__global__ void __launch_bounds__(256) k_binv(const BUnit* __restrict__ units, const int2* __restrict__ tasks,
                                              int ntasks, const int32_t* __restrict__ perm, BinvSlots sl,
                                              const double* __restrict__ G, DevScalars* sc,
                                              double* __restrict__ Minv) {
  const int t = sl.t0 + (int)blockIdx.y;      // iteration of the chunk, and its Gram and inverse slots
  G += t * sl.gslot;
  Minv += t * sl.mslot;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double rowbuf[4][2 * SP];
  const int task = blockIdx.x * 4 + wave;
  if (task >= ntasks) return;   // wavefront-uniform; the kernel has no workgroup barrier
  const int2 tk = tasks[task];
  if (sc[tk.x].status != 0) return;
  const BUnit U = units[tk.x];
  const double beta = sc[tk.x].beta;
  const int blk = tk.y;
  const int64_t s0 = block_start(blk, U.n, U.p);
  const int sb = (int)(block_start(blk + 1, U.n, U.p) - s0);
  const int32_t* pm = perm + U.poff + (int64_t)t * U.n + s0;
  const int j = lane;
  const int colj = j < sb ? pm[j] : 0;
  const double hj = (U.h && j < sb) ? U.h[colj] : 0.0;
  const double aj = (U.a && j < sb) ? U.a[colj] : 0.0;
  const double* Gb = G + (U.goff + blk) * (int64_t)SP * SP;
  double* buf = rowbuf[wave];
  if (U.a && j < SP) buf[j] = aj;
  __builtin_amdgcn_wave_barrier();
  // column j of the Gram (stored whole and exactly symmetric, so row i of the column is
  // the lower entry), all SP loads of a lane in flight at once (addresses inside the
  // block's SP x SP matrix even for lanes past SP; entries outside the block unused)
  double col[SP];
  const int jl = j < SP ? j : SP - 1;
#pragma unroll
  for (int i = 0; i < SP; ++i) col[i] = Gb[i * SP + jl];
#pragma unroll
  for (int i = 0; i < SP; ++i) {
    double v;
    if (i < sb && j < sb) {
      v = col[i] / U.Ns;
      if (i == j) v += beta + hj;
      if (U.a) v += beta * buf[i] * aj;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    col[i] = v;
  }
  __builtin_amdgcn_wave_barrier();
  bool failed = false;
  for (int k = 0; k < sb; ++k) {
    const double r = col[0];                    // a_kj
    if (j < SP) { buf[j] = r; buf[j + SP] = r; }
    __builtin_amdgcn_wave_barrier();
    const double d = buf[k];                    // same value in every lane
    if (!(d > 0.0) || !isfinite(d)) {
      failed = true;
      if (lane == 0) {
        unsigned long long key = ((unsigned long long)(sc[tk.x].k + t - sl.tk0) << 32) | (unsigned)blk;
        atomicMin((unsigned long long*)&sc[tk.x].fail_key, key);
      }
      break;
    }
    const double invd = 1.0 / d;
    const bool piv = j == k;
    const double m = piv ? -invd : r * invd;
    // the pivot's own column is replaced (a select, exact); buf[k+q] = a_(k+q mod SP),k
#pragma unroll
    for (int q = 1; q < SP; ++q) col[q - 1] = fma(-buf[k + q], m, piv ? 0.0 : col[q]);
    col[SP - 1] = m;
    __builtin_amdgcn_wave_barrier();
  }
  double* out = Minv + (U.moff + blk) * (int64_t)SP * SP;
  if (j < SP) {   // lanes past the padded size hold no column; the lower tiles only
#pragma unroll
    for (int q = 0; q < SP; ++q) {
      int i = q + sb;                           // register q holds row (q + sb) mod SP
      if (i >= SP) i -= SP;
      if ((i >> 4) >= (j >> 4)) out[minv_off(i, j)] = (!failed && i < sb && j < sb) ? -col[q] : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Block inverses of 64 x 64 blocks on the FP64 matrix cores, one wavefront per
// (lane, block).  The block matrix lives in the wavefront's registers as 4 x 4
// tiles of 16 x 16 in the accumulator layout of v_mfma_f64_16x16x4f64: lane
// (q, c) = (lane / 16, lane % 16) holds rows 4r + q (r = 0..3) of column c of
// every tile.  The sweep takes the pivots four at a time: sweeping the set K of
// four consecutive indices at once equals sweeping them one after the other, and
// with P = A_KK, N = -P^{-1} (the 4 x 4 sweep of P), Y = A_K. (the rows of K) and
// Z = N Y it is
//   A_ij += sum_k Y_ki Z_kj   (i, j not in K; Y_ki = A_ik by symmetry),
//   A_iK  = -(Y' N)_i        (i not in K),   A_Kj = -Z_j,   A_KK = N,
// one rank-4 product per tile.  The rows of K are each lane's own registers in
// the operand layouts (as operand A for the row tiles, as operand B for Y_j, and
// Z_j likewise), Z is one more product with N in the first four rows of operand
// A, and the columns of K come out of the same products once their accumulator
// is cleared and their operand-B entries are -N.  The pivots of P's sweep are
// those of the scalar sweep, checked against Assumption 2.1 as in k_binv.
// Pivot blocks that hold no index below sb are identity and are not swept.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 1/d from the hardware reciprocal and two Newton steps (d > 0 and finite; other
// values only occur with a failed pivot, whose block is discarded).
__device__ __forceinline__ double recip_f64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// The symmetric sweep of the 4 x 4 block P held by lanes (k, 4 rK + l), k, l < 4, of
// the register y: read_p gathers its upper triangle (mirrored) into S, pivot_step(k)
// sweeps pivot k; after the four steps S = -P^{-1}.  Every lane computes the same
// values.  A non-positive or non-finite pivot sets failed.
__device__ __forceinline__ void read_p(double y, int rK, double (&S)[4][4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int l = k; l < 4; ++l) {
      S[k][l] = readlane_f64(y, 16 * k + 4 * rK + l);
      S[l][k] = S[k][l];
    }
}
__device__ __forceinline__ void pivot_step(int k, double (&S)[4][4], bool& failed) {
  const double d = S[k][k];
  failed = failed | !(d > 0.0) | !isfinite(d);
  const double invd = recip_f64(d);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i == k) continue;
    const double mi = S[i][k] * invd;
#pragma unroll
    for (int l = i; l < 4; ++l) {
      if (l == k) continue;
      S[i][l] = fma(-mi, S[k][l], S[i][l]);
      S[l][i] = S[i][l];
    }
  }
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    if (l == k) continue;
    S[k][l] *= invd;
    S[l][k] = S[k][l];
  }
  S[k][k] = -invd;
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_binv64(const BUnit* __restrict__ units, const int2* __restrict__ tasks,
                                                int ntasks, const int32_t* __restrict__ perm, BinvSlots sl,
                                                const double* __restrict__ G, DevScalars* sc,
                                                double* __restrict__ Minv) {
  const int t = sl.t0 + (int)blockIdx.y;      // iteration of the chunk, and its Gram and inverse slots
  G += t * sl.gslot;
  Minv += t * sl.mslot;
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  constexpr int SP = 64;
  const int lane = threadIdx.x & 63;
  constexpr int wave = 0;                      // one wavefront per workgroup: a finished task's
  const int q = lane >> 4, c = lane & 15;      // slot is reused at once
  __shared__ double abuf[1][SP], hbuf[1][SP], nbuf[1][16];
  const int task = blockIdx.x;
  if (task >= ntasks) return;   // wavefront-uniform; the kernel has no workgroup barrier
  const int2 tk = tasks[task];
  if (sc[tk.x].status != 0) return;
  const BUnit U = units[tk.x];
  const double beta = sc[tk.x].beta;
  const int blk = tk.y;
  const int64_t s0 = block_start(blk, U.n, U.p);
  const int sb = (int)(block_start(blk + 1, U.n, U.p) - s0);
  const int32_t* pm = perm + U.poff + (int64_t)t * U.n + s0;
  {
    const int col = lane < sb ? pm[lane] : 0;
    abuf[wave][lane] = (U.a && lane < sb) ? U.a[col] : 0.0;
    hbuf[wave][lane] = (U.h && lane < sb) ? U.h[col] : 0.0;
  }
  const double* Gb = G + (U.goff + blk) * (int64_t)SP * SP;
  const double invNs = 1.0 / U.Ns;
  f64x4 m[4][4];
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int J = 0; J < 4; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + 4 * r + q, j = 16 * J + c;
        m[I][J][r] = Gb[i * SP + j];   // the Gram is stored whole and exactly symmetric
      }
  __builtin_amdgcn_wave_barrier();
  // M = G/Ns + diag(h) + beta (I + a a'), identity outside the block; branch-free (a
  // and h read as zero where absent, and adding a zero term is exact)
  {
    double dcol[4];
#pragma unroll
    for (int J = 0; J < 4; ++J) dcol[J] = beta + hbuf[wave][16 * J + c];
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + 4 * r + q, j = 16 * J + c;
          double v = m[I][J][r] * invNs;
          if (I == J) v += (4 * r + q == c) ? dcol[J] : 0.0;
          m[I][J][r] = (i < sb && j < sb) ? v : ((i == j) ? 1.0 : 0.0);
        }
  }
  if (U.a) {
    // + beta a a' as a rank-1 product per tile: operand A holds beta a_i in its
    // first column, operand B holds a_j in its first row (zero outside the block)
    double ar[4], ac[4];
#pragma unroll
    for (int I = 0; I < 4; ++I) {
      const double ai = abuf[wave][16 * I + c];
      ar[I] = q == 0 ? beta * ai : 0.0;
      ac[I] = q == 0 ? ai : 0.0;
    }
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
      for (int J = 0; J < 4; ++J) m[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[I], ac[J], m[I][J], 0, 0, 0);
  }
  // Software pipeline: the 4 x 4 sweep of the next pivot block and the exchange of its
  // N run on the vector ALU and the LDS between the current block's products (fenced
  // so that the in-order issue alternates them), once the tile that holds the next P
  // has been updated.  After a failed pivot the arithmetic goes on and the output is
  // zero.
  bool failed = false;
  double S[4][4];
  const int c_lt4 = c < 4 ? c : 0;
  double aN, bn;                                // this block's N in the operand layouts
  auto exchange = [&](int rK) {                 // N = S to every lane (same values: no branch)
#pragma unroll
    for (int e = 0; e < 16; ++e) nbuf[wave][e] = S[e >> 2][e & 3];
    __builtin_amdgcn_wave_barrier();
    const int cc = c - 4 * rK;
    const double an = nbuf[wave][c_lt4 * 4 + q];
    bn = nbuf[wave][q * 4 + ((unsigned)cc < 4u ? cc : 0)];
    aN = c < 4 ? an : 0.0;                      // operand A: N in rows 0..3
    __builtin_amdgcn_wave_barrier();
  };
  read_p(m[0][0][0], 0, S);
#pragma unroll
  for (int k = 0; k < 4; ++k) pivot_step(k, S, failed);
  exchange(0);
#pragma unroll
  for (int K = 0; K < 16; ++K) {
    if (4 * K >= sb) continue;                  // uniform; no early exit, so the loop unrolls
    const int IK = K >> 2, rK = K & 3;
    double Y[4];
#pragma unroll
    for (int J = 0; J < 4; ++J) Y[J] = m[IK][J][rK];
    const int cc = c - 4 * rK;                  // the lane's column inside K (tile column IK)
    const bool inK = (unsigned)cc < 4u;
    const double keep = inK ? 0.0 : 1.0;        // clears the accumulator of the columns of K
    const double bK = bn;
    const f64x4 zero = {0.0, 0.0, 0.0, 0.0};
    const int I1 = ((K + 1) >> 2) & 3, r1 = (K + 1) & 3;
    double Z[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {               // in the order of the first products
      const int J = (I1 + o) & 3;
      Z[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(aN, Y[J], zero, 0, 0, 0)[0];
    }
    auto update = [&](int I, int J) {
      f64x4 acc = m[I][J];
      double b = Z[J];
      if (J == IK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] *= keep;
        b = inK ? -bK : b;
      }
      m[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[I], b, acc, 0, 0, 0);
    };
    // the tile that holds the next P first, then the rest of its tile row
#pragma unroll
    for (int J = 0; J < 4; ++J) update(I1, (I1 + J) & 3);
    // the other 12 tiles, two products per step of the next block's sweep
    if (K < 15) {
      __builtin_amdgcn_sched_barrier(0);
      read_p(m[I1][I1][r1], r1, S);
    }
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      if (K < 15) __builtin_amdgcn_sched_barrier(0);
      update((I1 + 1 + g / 2) & 3, (2 * g) & 3);
      update((I1 + 1 + g / 2) & 3, (2 * g + 1) & 3);
      if (K < 15 && g < 4) {
        __builtin_amdgcn_sched_barrier(0);
        pivot_step(g, S, failed);
      }
      if (K < 15 && g == 3) {
        __builtin_amdgcn_sched_barrier(0);
        exchange(r1);
      }
    }
    if (K < 15) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int J = 0; J < 4; ++J) m[IK][J][rK] = (J == IK && inK) ? bK : -Z[J];
  }
  if (failed && lane == 0) {
    unsigned long long key = ((unsigned long long)(sc[tk.x].k + t - sl.tk0) << 32) | (unsigned)blk;
    atomicMin((unsigned long long*)&sc[tk.x].fail_key, key);
  }
  double* out = Minv + (U.moff + blk) * (int64_t)SP * SP;   // the lower tiles only
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + 4 * r + q, j = 16 * J + c;
        out[(I * (I + 1) / 2 + J) * 256 + (4 * r + q) * 16 + c] = (!failed && i < sb && j < sb) ? -m[I][J][r] : 0.0;
      }
}

// ---------------------------------------------------------------------------
// One workgroup per lane: the whole Gauss-Seidel pass.  Per block:
//   gradient pass: lane l takes rows l, l+64, ...; wavefront w takes block
//   columns w, w+4, ... (16 of them); per-lane sums are reduced across lanes
//   by a transposed butterfly (15 + 2 exchanges for 16 columns);
//   step d = -M^{-1} g from the lane's stored block inverse (its lower tiles);
//   update pass: thread r takes rows r, r+256, ... and adds F_B d to u.
// The row loops keep UNR rows per lane in flight (autotuned).
template <int B>
__device__ __forceinline__ double tsum(double (&v)[B], int lane, int& c) {
  int half = B / 2, o = 32;
#pragma unroll
  for (; half >= 1; half >>= 1, o >>= 1) {
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int q = 0; q < half; ++q) {
      const double send = upper ? v[q] : v[q + half];
      const double keep = upper ? v[q + half] : v[q];
      v[q] = keep + __shfl_xor(send, o, 64);
    }
  }
  double r = v[0];
#pragma unroll
  for (; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
  int cc = 0, bit = 32;
#pragma unroll
  for (int t = B; t > 1; t >>= 1, bit >>= 1) cc = (cc << 1) | ((lane & bit) ? 1 : 0);
  c = cc;
  return r;
}

template <typename T, int SP, int UNR>
__global__ void __launch_bounds__(256) k_bsweep(const BUnit* __restrict__ units, const int32_t* __restrict__ perm,
                                                int t, const double* __restrict__ Minv, DevScalars* sc,
                                                double* __restrict__ X, const double* __restrict__ Z,
                                                const double* __restrict__ XI, double* __restrict__ Uall) {
  constexpr int CB = SP / 4;   // columns per wavefront
  const int u = blockIdx.x;
  if (sc[u].status != 0) return;
  const BUnit D = units[u];
  const T* F = (const T*)D.F;
  double* x = X + D.xoff;
  const double* z = Z + D.xoff;
  const double* xi = XI + D.xoff;
  double* uu = Uall + D.uoff;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int32_t cols[SP];
  __shared__ double gl[SP], dl[SP], pg[SP], gb[SP];
  __shared__ double psum[256];
  const double beta = sc[u].beta, mu = sc[u].mu;
  double tq = sc[u].t;
  const int32_t* pm = perm + D.poff + (int64_t)t * D.n;
  for (int64_t blk = 0; blk < D.p; ++blk) {
    const int64_t s0 = block_start(blk, D.n, D.p);
    const int sb = (int)(block_start(blk + 1, D.n, D.p) - s0);
    if (tid < sb) {
      const int col = pm[s0 + tid];
      cols[tid] = col;
      const double xc = x[col];
      double v = D.c[col] - xi[col] + beta * (xc - z[col]);
      if (D.h) v += D.h[col] * xc;
      if (D.a) v -= mu * D.a[col];
      gb[tid] = v;
    }
    __syncthreads();
    // gradient pass
    double acc[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[q] = 0.0;
    int64_t cbase[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const int j = wave + 4 * q;
      cbase[q] = j < sb ? (int64_t)cols[j] * D.ldF : -1;
    }
    for (int64_t r0 = lane; r0 < D.rows; r0 += 64 * UNR) {
#pragma unroll
      for (int e = 0; e < UNR; ++e) {
        const int64_t r = r0 + 64 * e;
        if (r < D.rows) {
          const double ur = uu[r];
#pragma unroll
          for (int q = 0; q < CB; ++q)
            if (cbase[q] >= 0) acc[q] += ld_f64(F, cbase[q] + r) * ur;
        }
      }
    }
    int cidx;
    const double tot = tsum<CB>(acc, lane, cidx);
    if ((lane & (64 / CB - 1)) == 0) {
      const int j = wave + 4 * cidx;
      if (j < sb) pg[j] = tot;
    }
    __syncthreads();
    if (tid < sb) {
      double v = pg[tid] / D.Ns + gb[tid];
      if (D.a) v += beta * D.a[cols[tid]] * (tq - D.b);
      gl[tid] = v;
    }
    __syncthreads();
    // step: four threads per column, combined in order
    {
      const double* Mi = Minv + (D.moff + blk) * (int64_t)SP * SP;
      const int j = tid % SP, part = tid / SP;
      constexpr int P = 256 / SP;
      double a2 = 0.0;
      if (j < sb)
        for (int k = part; k < sb; k += P) a2 += Mi[minv_off(k, j)] * gl[k];
      psum[part * SP + j] = a2;
    }
    __syncthreads();
    if (tid < SP) {
      double s = 0.0;
      for (int e = 0; e < 256 / SP; ++e) s += psum[e * SP + tid];
      dl[tid] = tid < sb ? -s : 0.0;
    }
    __syncthreads();
    if (D.a) {
      double dt = 0.0;
      for (int j = 0; j < sb; ++j) dt += D.a[cols[j]] * dl[j];
      tq += dt;
    }
    // update pass
    for (int64_t r = tid; r < D.rows; r += 256) {
      double a2 = 0.0;
      for (int j = 0; j < sb; ++j) a2 += ld_f64(F, (int64_t)cols[j] * D.ldF + r) * dl[j];
      uu[r] += a2;
    }
    if (tid < sb) x[cols[tid]] += dl[tid];
    __syncthreads();
  }
  if (tid == 0) sc[u].t = tq;
}

// ---------------------------------------------------------------------------
// z block, dual step and norms of one lane per workgroup.
__global__ void __launch_bounds__(256) k_bzdual(const BUnit* __restrict__ units, DevScalars* sc,
                                                const double* __restrict__ X, double* Z, double* XI, double* ZP,
                                                int64_t T) {
  __shared__ double sh[4];
  const int u = blockIdx.x;
  if (sc[u].status != 0) return;
  const BUnit D = units[u];
  const double* x = X + D.xoff;
  double* z = Z + D.xoff;
  double* xi = XI + D.xoff;
  double* zp = ZP + D.xoff;
  const double beta = sc[u].beta;
  double rp2 = 0.0, rd2 = 0.0;
  for (int64_t j = threadIdx.x; j < D.n; j += 256) {
    const double xj = x[j], xij = xi[j], zo = z[j];
    double zn;
    if (D.prox == RAC_PROX_ELASTIC_NET) {
      const double v = beta * xj - xij, th = D.lam * D.alpha;
      zn = (v > th ? v - th : (v < -th ? v + th : 0.0)) / (beta + D.lam * (1.0 - D.alpha));
    } else if (D.prox == RAC_PROX_BOX) {
      zn = fmin(fmax(xj - xij / beta, D.lo), D.hi);
    } else {
      zn = xj - xij / beta;
    }
    const double r = xj - zn, dz = zn - zo;
    xi[j] = xij - beta * r;
    z[j] = zn;
    zp[j] = zo;
    rp2 += r * r;
    rd2 += dz * dz;
  }
  rp2 = bsum(rp2, sh);
  rd2 = bsum(rd2, sh);
  if (threadIdx.x != 0) return;
  DevScalars& S = sc[u];
  if (D.a) {
    const double e = S.t - D.b;
    S.mu -= beta * e;
    rp2 += e * e;
  }
  const double rp = sqrt(rp2), rd = beta * sqrt(rd2);
  const int64_t k = S.k;
  S.rp = rp;
  S.rd = rd;
  if (k % T == 0) { S.rp_win = rp; S.rd_win = rd; }
  if (S.rp_first < 0.0) S.rp_first = rp;
  if (!isfinite(rp) || !isfinite(rd) || (S.rp_first > 0.0 && rp > 1e12 * S.rp_first)) S.status = 2;
  S.k = k + 1;
}

// ---------------------------------------------------------------------------
// KKT terms per (lane, chunk of 64 columns); chunks past a lane's n write zeros.
template <typename T>
__global__ void __launch_bounds__(256) k_bkkt(const BUnit* __restrict__ units, const DevScalars* sc,
                                              const double* __restrict__ X, const double* __restrict__ Z,
                                              const double* __restrict__ XI, const double* __restrict__ Uall,
                                              double* __restrict__ kpart, int KC) {
  __shared__ double sh[4];
  const int u = blockIdx.x, ch = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* outp = kpart + ((int64_t)u * KC + ch) * 10;
  if (sc[u].status != 0) return;
  const BUnit D = units[u];
  const T* F = (const T*)D.F;
  const double mu = sc[u].mu;
  double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t j0 = (int64_t)ch * 64;
  for (int64_t j = j0 + wave; j < j0 + 64 && j < D.n; j += 4) {
    const T* col = F + j * D.ldF;
    const double* uu = Uall + D.uoff;
    double acc = 0.0;
    for (int64_t r = lane; r < D.rows; r += 64) acc += ld_f64(col, r) * uu[r];
    acc = wave_sum(acc);
    if (lane == 0)
      kkt_column_terms(acc, D.Ns, D.h ? D.h[j] : 0.0, D.c[j], D.a ? D.a[j] : 0.0, X[D.xoff + j],
                       Z[D.xoff + j], XI[D.xoff + j], mu, D.prox, D.lam, D.alpha, D.lo, D.hi, m);
  }
  for (int q = 0; q < 9; ++q) {
    const double v = bmax(m[q], sh);
    if (threadIdx.x == 0) outp[q] = v;
  }
  const double v = bsum(m[9], sh);
  if (threadIdx.x == 0) outp[9] = v;
}

__global__ void __launch_bounds__(64) k_bcontrol(const BUnit* __restrict__ units, DevScalars* sc,
                                                 const double* __restrict__ kpart, int KC, int32_t beta_mode,
                                                 double rb_mu, double rb_tau, double tol,
                                                 const float* __restrict__ w, double ymax, int decide) {
  const int u = blockIdx.x;
  if (sc[u].status != 0) return;
  if (sc[u].fail_key != ~0ULL) {          // a block violated Assumption 2.1: retire the lane
    if (threadIdx.x == 0) sc[u].status = 3;
    return;
  }
  const BUnit D = units[u];
  const int nch = (int)((D.n + 63) / 64);
  double M[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = 0; c < nch; ++c) {
    const double* q = kpart + ((int64_t)u * KC + c) * 10;
    for (int e = 0; e < 9; ++e) M[e] = fmax(M[e], q[e]);
    M[9] += q[9];
  }
  double out[4];
  kkt_from_maxima(M, D.a != nullptr, D.b, sc[u].mu, out);
  control_block(&sc[u], out[0], beta_mode, rb_mu, rb_tau, tol, w, ymax, decide, nullptr, 0, 0);
}

// Active lanes, and for every instance whether any of its lanes is active; the
// batch's iteration counter advances by the chunk length.
__global__ void __launch_bounds__(256) k_bactive(const BUnit* __restrict__ units, int nunits, const DevScalars* sc,
                                                 int32_t* inst_active, int ninst, int32_t* nactive, int64_t* kdev,
                                                 int Tc) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  for (int i = threadIdx.x; i < ninst; i += 256) inst_active[i] = 0;
  __syncthreads();
  int mine = 0;
  for (int u = threadIdx.x; u < nunits; u += 256)
    if (sc[u].status == 0 && sc[u].fail_key == ~0ULL) {
      ++mine;
      atomicOr(&inst_active[units[u].inst], 1);
    }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) {
    *nactive = cnt;
    *kdev += Tc;
  }
}

template <typename T>
hipError_t bsweep_launch(const BatchArgs& b, int t, hipStream_t st) {
#define RAC_BS(SPV, UN)                                                                              \
  if (b.sp == SPV && b.unroll == UN) {                                                               \
    k_bsweep<T, SPV, UN><<<(unsigned)b.nunits, 256, 0, st>>>(b.units, b.perm, t, b.Minv, b.sc, b.X, b.Z, \
                                                            b.XI, b.U);                              \
    return hipGetLastError();                                                                        \
  }
  RAC_BS(16, 1) RAC_BS(16, 2) RAC_BS(16, 4)
  RAC_BS(32, 1) RAC_BS(32, 2) RAC_BS(32, 4)
  RAC_BS(64, 1) RAC_BS(64, 2) RAC_BS(64, 4)
#undef RAC_BS
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t bkkt_launch(const BatchArgs& b, hipStream_t st) {
  dim3 grid((unsigned)b.nunits, (unsigned)b.KC);
  k_bkkt<T><<<grid, 256, 0, st>>>(b.units, b.sc, b.X, b.Z, b.XI, b.U, b.kpart, b.KC);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bperm(const BatchArgs& b, hipStream_t st) {
  const size_t lds = (size_t)(3 * b.np2 + 1) * sizeof(uint32_t);   // counts, starts, members
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_bperm, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((3 * 8192 + 1) * sizeof(uint32_t)));
    if (e != hipSuccess) return e;
    attr = true;
  }
  dim3 grid((unsigned)b.ninst, (unsigned)b.T);
  k_bperm<<<grid, 1024, lds, st>>>(b.inst, b.seed, b.kdev, b.perm, b.inst_active, b.np2);
  return hipGetLastError();
}

hipError_t launch_binv(const BatchArgs& b, int t0, int nt, int tk0, hipStream_t st) {
  const dim3 grid((unsigned)((b.ninv + 3) / 4), (unsigned)nt);
  if (grid.x == 0 || nt <= 0) return hipSuccess;
  const BinvSlots sl{t0, tk0, b.gslot, b.mslot};
  switch (b.sp) {
    case 16: k_binv<16><<<grid, 256, 0, st>>>(b.units, b.inv_tasks, b.ninv, b.perm, sl, b.G, b.sc, b.Minv); break;
    case 32: k_binv<32><<<grid, 256, 0, st>>>(b.units, b.inv_tasks, b.ninv, b.perm, sl, b.G, b.sc, b.Minv); break;
    case 64: k_binv64<<<dim3((unsigned)b.ninv, (unsigned)nt), 64, 0, st>>>(b.units, b.inv_tasks, b.ninv, b.perm, sl, b.G, b.sc, b.Minv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bsweep(const BatchArgs& b, int t, hipStream_t st) {
  switch (b.dtype) {
    case RAC_DT_F64: return bsweep_launch<double>(b, t, st);
    case RAC_DT_F32: return bsweep_launch<float>(b, t, st);
    case RAC_DT_BF16: return bsweep_launch<uint16_t>(b, t, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bzdual(const BatchArgs& b, hipStream_t st) {
  k_bzdual<<<(unsigned)b.nunits, 256, 0, st>>>(b.units, b.sc, b.X, b.Z, b.XI, b.ZP, b.T);
  return hipGetLastError();
}

hipError_t launch_bcheck(const BatchArgs& b, int Tc, int decide, int grouped_kkt, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (!grouped_kkt) {
    switch (b.dtype) {
      case RAC_DT_F64: e = bkkt_launch<double>(b, st); break;
      case RAC_DT_F32: e = bkkt_launch<float>(b, st); break;
      case RAC_DT_BF16: e = bkkt_launch<uint16_t>(b, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  k_bcontrol<<<(unsigned)b.nunits, 64, 0, st>>>(b.units, b.sc, b.kpart, b.KC, b.beta_mode, b.rb_mu, b.rb_tau,
                                                 b.tol, b.mlp_w, b.mlp_ymax, decide);
  k_bactive<<<1, 256, 0, st>>>(b.units, b.nunits, b.sc, b.inst_active, b.ninst, b.nactive, b.kdev, Tc);
  return hipGetLastError();
}

}  // namespace rac
