// sparse.hip -- kernels of the sparse factor form: F (rows x n) stored as
// compressed sparse columns (colptr[n + 1], strictly increasing row indices per
// column, values), the data of the paper's sparse regressions (Sec.3.1, Tables
// 3-7, data sparsity 0.991-0.998).
//
// Block Grams: one workgroup per block; the block's columns are staged in LDS
// when they fit, and each entry (q, r) of the lower triangle is the merge of two
// sorted row lists (a sparse dot product), summed in row order.
//
// Sweep (Eq.(3), blocks in the drawn order): one persistent workgroup keeps the
// Gauss-Seidel order; per block, the products F_ij u_i of the block's stored
// entries are formed flat over all threads (u read from device memory at agent
// scope) and summed per column in entry order, the step d = -M_B^{-1} g_B
// follows from the inverse (four or two threads per column), and u += F_B d is
// applied with FP64 atomic additions (several columns of a block may share a
// row).  Everything of a block that does not depend on u (its
// columns, the inverse, the iterate-fixed terms) is loaded ahead of the chain
// that does.  The atomics make the order of same-row contributions within a block
// timing-dependent, so iterates agree with the oracle to rounding, not bitwise
// from run to run.
#include "rac_internal.h"
#include "control.h"

namespace rac {
namespace {

template <typename T> __device__ __forceinline__ double sv(const T* p, int64_t i) { return (double)p[i]; }

__device__ __forceinline__ double ld_u(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_u(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The sweep is one workgroup, the only reader and writer of u while it runs: its loads
// and additions need workgroup scope only (ordered by the workgroup barrier between a
// block's additions and the next block's loads), which keeps them in the XCD's L2.
__device__ __forceinline__ double ld_u_wg(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void add_u_wg(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

constexpr int kStage = 10240;  // block entries staged in LDS (row index + FP64 value: 120 KiB)

// Sparse dot of two sorted columns (two-pointer merge in row order).
__device__ __forceinline__ double merge_dot(const int32_t* ra, const double* va, int na, const int32_t* rb,
                                            const double* vb, int nb) {
  double s = 0.0;
  int i = 0, j = 0;
  while (i < na && j < nb) {
    const int32_t a = ra[i], b = rb[j];
    if (a == b) { s += va[i] * vb[j]; ++i; ++j; }
    else if (a < b) ++i;
    else ++j;
  }
  return s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_sgram(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                                               const T* __restrict__ val, int64_t n, int64_t p,
                                               const int32_t* __restrict__ perm, int sp, double* __restrict__ out) {
  __shared__ int32_t srow[kStage];
  __shared__ double sval[kStage];
  __shared__ int32_t off[kMaxBlock + 1];
  __shared__ int32_t cols[kMaxBlock];
  __shared__ int staged;
  const int64_t blk = blockIdx.x;
  const int64_t s0 = block_start(blk, n, p);
  const int sb = (int)(block_start(blk + 1, n, p) - s0);
  const int tid = threadIdx.x;
  if (tid < sb) cols[tid] = perm[s0 + tid];
  __syncthreads();
  if (tid == 0) {
    int64_t acc = 0;
    for (int j = 0; j < sb; ++j) {
      off[j] = (int32_t)(acc < kStage ? acc : kStage);
      acc += colptr[cols[j] + 1] - colptr[cols[j]];
    }
    off[sb] = (int32_t)(acc < kStage ? acc : kStage);
    staged = acc <= kStage;
  }
  __syncthreads();
  if (staged) {
    for (int j = 0; j < sb; ++j) {
      const int64_t c0 = colptr[cols[j]];
      const int len = off[j + 1] - off[j];
      for (int e = tid; e < len; e += 256) {
        srow[off[j] + e] = rowidx[c0 + e];
        sval[off[j] + e] = sv(val, c0 + e);
      }
    }
  }
  __syncthreads();
  double* o = out + blk * (int64_t)sp * sp;
  for (int e = tid; e < sp * sp; e += 256) {
    const int q = e / sp, r = e % sp;
    double v = 0.0;
    if (q < sb && r < sb && q >= r) {
      if (staged) {
        v = merge_dot(srow + off[q], sval + off[q], off[q + 1] - off[q], srow + off[r], sval + off[r],
                      off[r + 1] - off[r]);
      } else {   // columns read from device memory
        const int64_t a0 = colptr[cols[q]], a1 = colptr[cols[q] + 1], b0 = colptr[cols[r]], b1 = colptr[cols[r] + 1];
        int64_t i = a0, j = b0;
        while (i < a1 && j < b1) {
          const int32_t ra = rowidx[i], rb = rowidx[j];
          if (ra == rb) { v += sv(val, i) * sv(val, j); ++i; ++j; }
          else if (ra < rb) ++i;
          else ++j;
        }
      }
    }
    o[e] = v;
  }
}

struct SSweepArgs {
  const int64_t* colptr; const int32_t* rowidx; const void* val; int64_t n; int64_t p;
  const int32_t* perm; const int32_t* order; const double* Minv; int sp;
  const double* c; const double* h; const double* a; double b; double Ns;
  double* x; const double* z; const double* xi; double* u; DevScalars* sc; const double* beta_ptr;
  int fast;   // rows < 2^25: a block's entries can keep their column index beside the row
};

// Entries of a block are numbered flat (entry f of the block's columns in block order).
// Fast path (blocks of at most kFast entries): every thread holds entries f = tid,
// tid + 256, ... (at most kQ) in registers from the gradient to the update, with all
// their loads in flight at once -- row indices and values, then u at those rows -- and
// their column read from a map of the block's entries built with its column offsets.
// Each column's products are summed by four (or two) threads over consecutive ranges.  Larger blocks take the chunked path (chunks of kFlat entries, batches
// of kBatch loads per thread, the entries loaded again for the update).  The next
// block's columns and offsets are gathered while the current one finishes, and its
// inverse and iterate-fixed gradient terms are issued at the start of its own block,
// before its products.
constexpr int kFlat = 12288;   // entries per chunk: their products (FP64) in LDS
constexpr int kBatch = 8;      // chunked path: entries per thread whose loads are in flight together
constexpr int kQ = 40;         // fast path: entries per thread
constexpr int kFast = 256 * kQ;
constexpr uint32_t kRowMask = (1u << 25) - 1;

// Column of flat entry f: the last j with bo[j] <= f (bo ascending, bo[0] = 0).
__device__ __forceinline__ int column_of(const int32_t* bo, int sb, int f) {
  int lo = 0, hi = sb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bo[mid] <= f) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ void __launch_bounds__(256) k_ssweep(SSweepArgs s) {
  __shared__ double sh_g[kMaxBlock];
  __shared__ double sh_d[kMaxBlock];
  __shared__ double sh_a[kMaxBlock];        // a of the block's columns (equality row)
  __shared__ double sh_pg[4][kMaxBlock];    // parts of the solve's products
  __shared__ int32_t colsb[2][kMaxBlock];
  __shared__ int64_t cstb[2][kMaxBlock];    // first stored entry of each block column
  __shared__ int32_t boffb[2][kMaxBlock + 1];   // block-local entry offsets of the columns
  __shared__ int32_t scan[kMaxBlock];
  __shared__ uint8_t colof[kFast];          // fast path: the column of each entry of the block
  __shared__ double prod[kFlat];            // F_ij u_i of the (chunk's) entries
  const int tid = threadIdx.x, lane = tid & 63;
  const T* val = (const T*)s.val;
  const double beta = *s.beta_ptr;
  const double mu = s.sc->mu;
  double t = s.sc->t;
  // columns, first entries and entry offsets of block position i into buffer nb
  // (the column lengths are scanned by the first two wavefronts)
  auto gather_setup = [&](int64_t i, int nb, int32_t col) {
    const int64_t bi = s.order ? (int64_t)s.order[i] : i;
    const int sb = (int)(block_start(bi + 1, s.n, s.p) - block_start(bi, s.n, s.p));
    int32_t len = 0;
    if (tid < sb) {
      const int64_t c0 = s.colptr[col];
      colsb[nb][tid] = col;
      cstb[nb][tid] = c0;
      len = (int32_t)(s.colptr[col + 1] - c0);
    }
    if (tid < 128) {
      int32_t v = len;   // inclusive scan over the wavefront
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
      }
      scan[tid] = v;
    }
    __syncthreads();
    if (tid < sb) boffb[nb][tid + 1] = scan[tid] + (tid >= 64 ? scan[63] : 0);
    if (tid == 0) boffb[nb][0] = 0;
    const int E = scan[sb - 1] + (sb > 64 ? scan[63] : 0);
    if (E <= kFast && tid < sb) {            // each column marks its entries
      const int b0 = tid == 0 ? 0 : scan[tid - 1] + (tid - 1 >= 64 ? scan[63] : 0);
      for (int f = b0; f < b0 + len; ++f) colof[f] = (uint8_t)tid;
    }
  };
  auto first_col = [&](int64_t i) -> int32_t {   // column tid of block position i (tid < its size)
    const int64_t bi = s.order ? (int64_t)s.order[i] : i;
    const int64_t s0 = block_start(bi, s.n, s.p);
    const int sb = (int)(block_start(bi + 1, s.n, s.p) - s0);
    return tid < sb ? s.perm[s0 + tid] : 0;
  };
  gather_setup(0, 0, first_col(0));
  __syncthreads();
  for (int64_t i = 0; i < s.p; ++i) {
    const int cb = (int)(i & 1);
    const int32_t* cols = colsb[cb];
    const int64_t* cst = cstb[cb];
    const int32_t* boff = boffb[cb];
    const int64_t bi = s.order ? (int64_t)s.order[i] : i;
    const int sb = (int)(block_start(bi + 1, s.n, s.p) - block_start(bi, s.n, s.p));
    const int E = boff[sb];
    const int32_t ncol = i + 1 < s.p ? first_col(i + 1) : 0;   // the next block's columns, loaded early
    const double* Mi = s.Minv + bi * (int64_t)s.sp * s.sp;
    // iterate-fixed terms of column tid, issued before the products
    double tc = 0.0, txi = 0.0, tz = 0.0, tx = 0.0, th = 0.0, ta = 0.0;
    if (tid < sb) {
      const int col = cols[tid];
      tc = s.c[col]; txi = s.xi[col]; tz = s.z[col]; tx = s.x[col];
      if (s.h) th = s.h[col];
      if (s.a) ta = s.a[col];
    }
    // the block inverse: thread (jc, part) takes rows part*KP .. part*KP + KP - 1 of column jc
    // (4 parts of 16 rows for blocks of up to 64 columns, else 2 parts of 64 in batches of 16);
    // addresses clamped into the block's sp x sp matrix, rows past sb masked where used
    const int nparts = sb <= 64 ? 4 : 2;
    const int jc = nparts == 4 ? (tid & 63) : (tid & 127), part = nparts == 4 ? (tid >> 6) : (tid >> 7);
    const int KP = nparts == 4 ? 16 : 64;
    const int jcl = jc < s.sp ? jc : s.sp - 1;
    double mreg[16];
    auto minv_issue = [&](int k0) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int k = k0 + e;
        mreg[e] = Mi[(int64_t)(k < s.sp ? k : s.sp - 1) * s.sp + jcl];
      }
    };
    minv_issue(part * KP);
    if (s.fast && E <= kFast) {
      // ---- fast path: the block's entries stay in registers
      uint32_t rj[kQ];
      T v[kQ];
      uint32_t jq[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int f = tid + 256 * q;
        const int j = f < E ? colof[f] : 0;
        // past the block: entry 0 of the matrix, which exists (value unused)
        const int64_t e = f < E ? cst[j] + (f - boff[j]) : 0;
        jq[q] = (uint32_t)j;
        rj[q] = (uint32_t)s.rowidx[e];
        v[q] = val[e];
      }
#pragma unroll
      for (int q = 0; q < kQ; ++q) rj[q] |= jq[q] << 25;   // the column beside the row
      double uu[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) uu[q] = ld_u_wg(s.u + (rj[q] & kRowMask));
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int f = tid + 256 * q;
        if (f < E) prod[f] = (double)v[q] * uu[q];
      }
      __syncthreads();
      {
        // the column's products: thread (jc, part) sums its part of the column's entries in
        // entry order (the column split in nparts near-equal ranges), the parts added in order
        const int b0 = jc < sb ? boff[jc] : 0, len = jc < sb ? boff[jc + 1] - b0 : 0;
        const int lo = b0 + (len * part) / nparts, hi = b0 + (len * (part + 1)) / nparts;
        double acc = 0.0;
        for (int f = lo; f < hi; ++f) acc += prod[f];
        sh_pg[part][jc] = acc;
      }
      __syncthreads();
      if (tid < sb)
        sh_g[tid] = nparts == 4 ? ((sh_pg[0][tid] + sh_pg[1][tid]) + sh_pg[2][tid]) + sh_pg[3][tid]
                                : sh_pg[0][tid] + sh_pg[1][tid];
      __syncthreads();
      // the gradient, the step and x_B
      if (tid < sb) {
        double gg = sh_g[tid] / s.Ns + tc - txi + beta * (tx - tz);
        if (s.h) gg += th * tx;
        if (s.a) gg += -mu * ta + beta * ta * (t - s.b);
        sh_g[tid] = gg;
        sh_a[tid] = ta;
      }
      __syncthreads();
      {
        double a2 = 0.0;
        for (int k0 = part * KP; k0 < part * KP + KP; k0 += 16) {
          if (k0 != part * KP) minv_issue(k0);
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int k = k0 + e;
            a2 += (k < sb ? mreg[e] : 0.0) * (k < sb ? sh_g[k] : 0.0);
          }
        }
        if (jc < kMaxBlock) sh_pg[part][jc] = a2;
      }
      __syncthreads();
      if (tid < sb) {
        const double d = nparts == 4 ? -(((sh_pg[0][tid] + sh_pg[1][tid]) + sh_pg[2][tid]) + sh_pg[3][tid])
                                     : -(sh_pg[0][tid] + sh_pg[1][tid]);
        sh_d[tid] = d;
        s.x[cols[tid]] = tx + d;
      }
      __syncthreads();
      if (s.a) {
        double dt = 0.0;
        for (int j = 0; j < sb; ++j) dt += sh_a[j] * sh_d[j];
        t += dt;   // every thread forms the same sum in the same order
      }
      // residual update u += F_B d (atomic additions: columns may share rows)
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int f = tid + 256 * q;
        if (f < E) add_u_wg(s.u + (rj[q] & kRowMask), (double)v[q] * sh_d[rj[q] >> 25]);
      }
    } else {
      // ---- chunked path: gradient partials F_B'u chunk by chunk, column sums in entry order
      if (tid < sb) sh_g[tid] = 0.0;
      __syncthreads();
      for (int f0 = 0; f0 < E; f0 += kFlat) {
        const int fe = f0 + kFlat < E ? f0 + kFlat : E;
        for (int fb = f0 + tid; fb < fe; fb += 256 * kBatch) {
          int32_t row[kBatch];
          double vv[kBatch];
#pragma unroll
          for (int q = 0; q < kBatch; ++q) {
            const int f = fb + 256 * q;
            int64_t e = 0;
            if (f < fe) {
              const int j = column_of(boff, sb, f);
              e = cst[j] + (f - boff[j]);
            }
            row[q] = s.rowidx[e];
            vv[q] = sv(val, e);
          }
          double uu[kBatch];
#pragma unroll
          for (int q = 0; q < kBatch; ++q) uu[q] = ld_u_wg(s.u + row[q]);
#pragma unroll
          for (int q = 0; q < kBatch; ++q) {
            const int f = fb + 256 * q;
            if (f < fe) prod[f - f0] = vv[q] * uu[q];
          }
        }
        __syncthreads();
        if (tid < sb) {
          const int a = boff[tid] > f0 ? boff[tid] : f0, b = boff[tid + 1] < fe ? boff[tid + 1] : fe;
          double acc = sh_g[tid];
          for (int f = a; f < b; ++f) acc += prod[f - f0];
          sh_g[tid] = acc;
        }
        __syncthreads();
      }
      if (tid < sb) {
        double gg = sh_g[tid] / s.Ns + tc - txi + beta * (tx - tz);
        if (s.h) gg += th * tx;
        if (s.a) gg += -mu * ta + beta * ta * (t - s.b);
        sh_g[tid] = gg;
        sh_a[tid] = ta;
      }
      __syncthreads();
      {
        double a2 = 0.0;
        for (int k0 = part * KP; k0 < part * KP + KP; k0 += 16) {
          if (k0 != part * KP) minv_issue(k0);
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int k = k0 + e;
            a2 += (k < sb ? mreg[e] : 0.0) * (k < sb ? sh_g[k] : 0.0);
          }
        }
        if (jc < kMaxBlock) sh_pg[part][jc] = a2;
      }
      __syncthreads();
      if (tid < sb) {
        const double d = nparts == 4 ? -(((sh_pg[0][tid] + sh_pg[1][tid]) + sh_pg[2][tid]) + sh_pg[3][tid])
                                     : -(sh_pg[0][tid] + sh_pg[1][tid]);
        sh_d[tid] = d;
        s.x[cols[tid]] = tx + d;
      }
      __syncthreads();
      if (s.a) {
        double dt = 0.0;
        for (int j = 0; j < sb; ++j) dt += sh_a[j] * sh_d[j];
        t += dt;
      }
      for (int fb = tid; fb < E; fb += 256 * kBatch) {
        int32_t row[kBatch];
        double vv[kBatch];
        double dj[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          const int f = fb + 256 * q;
          int64_t e = 0;
          int j = 0;
          if (f < E) {
            j = column_of(boff, sb, f);
            e = cst[j] + (f - boff[j]);
          }
          row[q] = s.rowidx[e];
          vv[q] = sv(val, e);
          dj[q] = sh_d[j];
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q)
          if (fb + 256 * q < E) add_u_wg(s.u + row[q], vv[q] * dj[q]);
      }
    }
    // the next block's columns and offsets, while the additions complete
    if (i + 1 < s.p) gather_setup(i + 1, cb ^ 1, ncol);
    // the additions complete at device scope before the next block's loads of u
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  if (tid == 0) s.sc->t = t;
}

// The same sweep with u held in LDS for the whole launch (instances of at most
// kURows rows): a block's gathers of u and its additions into u are LDS operations
// instead of scattered device-memory requests, which one compute unit issues at
// about one address per cycle.  The column sums of the gradient products are LDS
// atomic additions (their order is timing-dependent, as the update's already is).
// Blocks of more than kFast entries run in chunks of kFast, the chunk's entries
// loaded again for the update.  (Measured alternatives, slower at 145 entries per
// column: a segmented scan over the wavefront before the additions, and one
// wavefront per column with fixed-order sums.)
constexpr int kURows = 17408;   // 136 KiB of FP64 u

template <typename T>
__global__ void __launch_bounds__(256) k_ssweep_lds(SSweepArgs s, int64_t rows) {
  __shared__ double uL[kURows];
  __shared__ uint8_t colof[kFast];
  __shared__ double sh_g[kMaxBlock];
  __shared__ double sh_d[kMaxBlock];
  __shared__ double sh_a[kMaxBlock];
  __shared__ double sh_pg[4][kMaxBlock];
  __shared__ int32_t colsb[2][kMaxBlock];
  __shared__ int64_t cstb[2][kMaxBlock];
  __shared__ int32_t boffb[2][kMaxBlock + 1];
  __shared__ int32_t scan[kMaxBlock];
  const int tid = threadIdx.x, lane = tid & 63;
  const T* val = (const T*)s.val;
  const double beta = *s.beta_ptr;
  const double mu = s.sc->mu;
  double t = s.sc->t;
  for (int64_t r = tid; r < rows; r += 256) uL[r] = s.u[r];
  auto gather_setup = [&](int64_t i, int nb, int32_t col) {
    const int64_t bi = s.order ? (int64_t)s.order[i] : i;
    const int sb = (int)(block_start(bi + 1, s.n, s.p) - block_start(bi, s.n, s.p));
    int32_t len = 0;
    if (tid < sb) {
      const int64_t c0 = s.colptr[col];
      colsb[nb][tid] = col;
      cstb[nb][tid] = c0;
      len = (int32_t)(s.colptr[col + 1] - c0);
    }
    if (tid < 128) {
      int32_t v = len;
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
      }
      scan[tid] = v;
    }
    __syncthreads();
    if (tid < sb) boffb[nb][tid + 1] = scan[tid] + (tid >= 64 ? scan[63] : 0);
    if (tid == 0) boffb[nb][0] = 0;
    const int E = scan[sb - 1] + (sb > 64 ? scan[63] : 0);
    if (E <= kFast && tid < sb) {
      const int b0 = tid == 0 ? 0 : scan[tid - 1] + (tid - 1 >= 64 ? scan[63] : 0);
      for (int f = b0; f < b0 + len; ++f) colof[f] = (uint8_t)tid;
    }
  };
  auto first_col = [&](int64_t i) -> int32_t {
    const int64_t bi = s.order ? (int64_t)s.order[i] : i;
    const int64_t s0 = block_start(bi, s.n, s.p);
    const int sb = (int)(block_start(bi + 1, s.n, s.p) - s0);
    return tid < sb ? s.perm[s0 + tid] : 0;
  };
  gather_setup(0, 0, first_col(0));
  __syncthreads();
  for (int64_t i = 0; i < s.p; ++i) {
    const int cb = (int)(i & 1);
    const int32_t* cols = colsb[cb];
    const int64_t* cst = cstb[cb];
    const int32_t* boff = boffb[cb];
    const int64_t bi = s.order ? (int64_t)s.order[i] : i;
    const int sb = (int)(block_start(bi + 1, s.n, s.p) - block_start(bi, s.n, s.p));
    const int E = boff[sb];
    const int32_t ncol = i + 1 < s.p ? first_col(i + 1) : 0;
    const double* Mi = s.Minv + bi * (int64_t)s.sp * s.sp;
    double tc = 0.0, txi = 0.0, tz = 0.0, tx = 0.0, th = 0.0, ta = 0.0;
    if (tid < sb) {
      const int col = cols[tid];
      tc = s.c[col]; txi = s.xi[col]; tz = s.z[col]; tx = s.x[col];
      if (s.h) th = s.h[col];
      if (s.a) ta = s.a[col];
      sh_g[tid] = 0.0;
    }
    const int nparts = sb <= 64 ? 4 : 2;
    const int jc = nparts == 4 ? (tid & 63) : (tid & 127), part = nparts == 4 ? (tid >> 6) : (tid >> 7);
    const int KP = nparts == 4 ? 16 : 64;
    const int jcl = jc < s.sp ? jc : s.sp - 1;
    double mreg[16];
    auto minv_issue = [&](int k0) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int k = k0 + e;
        mreg[e] = Mi[(int64_t)(k < s.sp ? k : s.sp - 1) * s.sp + jcl];
      }
    };
    minv_issue(part * KP);
    __syncthreads();   // sh_g zeroed
    // entries f0 + tid + 256 q of a chunk: row (and column beside it), value
    uint32_t rj[kQ];
    T v[kQ];
    auto load_chunk = [&](int f0) {
      const int fe = f0 + kFast < E ? f0 + kFast : E;
      const bool mapped = E <= kFast;
      uint32_t jq[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int f = f0 + tid + 256 * q;
        const int j = f < fe ? (mapped ? (int)colof[f] : column_of(boff, sb, f)) : 0;
        const int64_t e = f < fe ? cst[j] + (f - boff[j]) : 0;   // past the chunk: entry 0 (unused)
        jq[q] = (uint32_t)j;
        rj[q] = (uint32_t)s.rowidx[e];
        v[q] = val[e];
      }
#pragma unroll
      for (int q = 0; q < kQ; ++q) rj[q] |= jq[q] << 25;
      return fe;
    };
    for (int f0 = 0; f0 < E; f0 += kFast) {   // gradient products, summed per column in LDS
      const int fe = load_chunk(f0);
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int f = f0 + tid + 256 * q;
        if (f < fe) atomicAdd(&sh_g[rj[q] >> 25], (double)v[q] * uL[rj[q] & kRowMask]);
      }
    }
    __syncthreads();
    if (tid < sb) {
      double gg = sh_g[tid] / s.Ns + tc - txi + beta * (tx - tz);
      if (s.h) gg += th * tx;
      if (s.a) gg += -mu * ta + beta * ta * (t - s.b);
      sh_g[tid] = gg;
      sh_a[tid] = ta;
    }
    __syncthreads();
    {
      double a2 = 0.0;
      for (int k0 = part * KP; k0 < part * KP + KP; k0 += 16) {
        if (k0 != part * KP) minv_issue(k0);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int k = k0 + e;
          a2 += (k < sb ? mreg[e] : 0.0) * (k < sb ? sh_g[k] : 0.0);
        }
      }
      sh_pg[part][jc] = a2;
    }
    __syncthreads();
    if (tid < sb) {
      const double d = nparts == 4 ? -(((sh_pg[0][tid] + sh_pg[1][tid]) + sh_pg[2][tid]) + sh_pg[3][tid])
                                   : -(sh_pg[0][tid] + sh_pg[1][tid]);
      sh_d[tid] = d;
      s.x[cols[tid]] = tx + d;
    }
    __syncthreads();
    if (s.a) {
      double dt = 0.0;
      for (int j = 0; j < sb; ++j) dt += sh_a[j] * sh_d[j];
      t += dt;
    }
    // u += F_B d: the last (or only) chunk first, its entries still in registers, then the
    // earlier chunks loaded again
    const int flast = E > 0 ? ((E - 1) / kFast) * kFast : 0;
    for (int f0 = flast; f0 >= 0 && E > 0; f0 -= kFast) {
      const int fe = f0 == flast ? E : load_chunk(f0);
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int f = f0 + tid + 256 * q;
        if (f < fe) atomicAdd(&uL[rj[q] & kRowMask], (double)v[q] * sh_d[rj[q] >> 25]);
      }
    }
    if (i + 1 < s.p) gather_setup(i + 1, cb ^ 1, ncol);
    __syncthreads();
  }
  for (int64_t r = tid; r < rows; r += 256) s.u[r] = uL[r];
  if (tid == 0) s.sc->t = t;
}

// part[j] = F_j'v (one wavefront per column).
template <typename T>
__global__ void __launch_bounds__(256) k_sdots(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                                               const T* __restrict__ val, int64_t n, const double* __restrict__ v,
                                               double scale, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j = (int64_t)blockIdx.x * 4 + wave; j < n; j += (int64_t)gridDim.x * 4) {
    double acc = 0.0;
    for (int64_t e = colptr[j] + lane; e < colptr[j + 1]; e += 64) acc += sv(val, e) * v[rowidx[e]];
    acc = wave_sum(acc);
    if (lane == 0) out[j] = scale * acc;
  }
}

__global__ void __launch_bounds__(256) k_zero_f64(double* a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a[i] = 0.0;
}

// u = F x by scatter (device-scope atomic additions into a zeroed u).
template <typename T>
__global__ void __launch_bounds__(256) k_sspmv(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                                               const T* __restrict__ val, int64_t n, const double* __restrict__ x,
                                               double* u) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j = (int64_t)blockIdx.x * 4 + wave; j < n; j += (int64_t)gridDim.x * 4) {
    const double xj = x[j];
    if (xj == 0.0) continue;
    for (int64_t e = colptr[j] + lane; e < colptr[j + 1]; e += 64) add_u(u + rowidx[e], sv(val, e) * xj);
  }
}

unsigned grid_for(int64_t n, int per) {
  int64_t b = (n + per - 1) / per;
  if (b > 4096) b = 4096;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_sgram(const SparseF& F, int64_t n, int64_t p, const int32_t* perm, int sp, double* out,
                        hipStream_t st) {
  if (F.dtype == RAC_DT_F64)
    k_sgram<double><<<(unsigned)p, 256, 0, st>>>(F.colptr, F.rowidx, (const double*)F.val, n, p, perm, sp, out);
  else if (F.dtype == RAC_DT_F32)
    k_sgram<float><<<(unsigned)p, 256, 0, st>>>(F.colptr, F.rowidx, (const float*)F.val, n, p, perm, sp, out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_ssweep(const SparseF& F, const SweepArgs& w, hipStream_t st) {
  SSweepArgs s{F.colptr, F.rowidx, F.val, w.n, w.p, w.perm, w.order, w.Minv, w.sp, w.c, w.h, w.a, w.b, w.Ns,
               w.x, w.z, w.xi, w.u, w.sc, w.beta_ptr, w.rows < ((int64_t)1 << 25) ? 1 : 0};
  if (w.rows <= kURows) {   // u fits in LDS
    if (F.dtype == RAC_DT_F64) k_ssweep_lds<double><<<1, 256, 0, st>>>(s, w.rows);
    else if (F.dtype == RAC_DT_F32) k_ssweep_lds<float><<<1, 256, 0, st>>>(s, w.rows);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (F.dtype == RAC_DT_F64) k_ssweep<double><<<1, 256, 0, st>>>(s);
  else if (F.dtype == RAC_DT_F32) k_ssweep<float><<<1, 256, 0, st>>>(s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sdots(const SparseF& F, int64_t n, const double* v, double scale, double* out, hipStream_t st) {
  const unsigned g = grid_for(n, 4);
  if (F.dtype == RAC_DT_F64)
    k_sdots<double><<<g, 256, 0, st>>>(F.colptr, F.rowidx, (const double*)F.val, n, v, scale, out);
  else if (F.dtype == RAC_DT_F32)
    k_sdots<float><<<g, 256, 0, st>>>(F.colptr, F.rowidx, (const float*)F.val, n, v, scale, out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sspmv(const SparseF& F, int64_t rows, int64_t n, const double* x, double* u, hipStream_t st) {
  k_zero_f64<<<grid_for(rows, 256), 256, 0, st>>>(u, rows);
  const unsigned g = grid_for(n, 4);
  if (F.dtype == RAC_DT_F64)
    k_sspmv<double><<<g, 256, 0, st>>>(F.colptr, F.rowidx, (const double*)F.val, n, x, u);
  else if (F.dtype == RAC_DT_F32)
    k_sspmv<float><<<g, 256, 0, st>>>(F.colptr, F.rowidx, (const float*)F.val, n, x, u);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace rac
