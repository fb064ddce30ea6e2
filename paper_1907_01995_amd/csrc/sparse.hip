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
// follows from the inverse, and u += F_B d is applied with device-scope FP64
// atomic additions (several columns of a block may share a row).  The atomics make the order of same-row contributions within a block
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
};

// The block's stored entries are processed flat (entry f of the block's
// columns in block order, chunks of kFlat): every thread takes entries f = tid,
// tid + 256, ... in batches whose loads are all issued before any is used, so
// the dependent loads (row index, then u at that row) overlap across entries.
constexpr int kFlat = 12288;   // entries per chunk: their products (FP64) in LDS
constexpr int kBatch = 8;      // entries per thread whose loads are in flight together

template <typename T>
__global__ void __launch_bounds__(256) k_ssweep(SSweepArgs s) {
  __shared__ double sh_g[kMaxBlock];
  __shared__ double sh_d[kMaxBlock];
  __shared__ int32_t cols[kMaxBlock];
  __shared__ int64_t cst[kMaxBlock];        // first stored entry of each block column
  __shared__ int32_t boff[kMaxBlock + 1];   // block-local entry offsets of the columns
  __shared__ double prod[kFlat];            // F_ij u_i of the chunk's entries
  const int tid = threadIdx.x;
  const T* val = (const T*)s.val;
  const double beta = *s.beta_ptr;
  const double mu = s.sc->mu;
  double t = s.sc->t;
  for (int64_t i = 0; i < s.p; ++i) {
    const int64_t bi = s.order ? (int64_t)s.order[i] : i;
    const int64_t s0 = block_start(bi, s.n, s.p);
    const int sb = (int)(block_start(bi + 1, s.n, s.p) - s0);
    if (tid < sb) {
      const int col = s.perm[s0 + tid];
      cols[tid] = col;
      cst[tid] = s.colptr[col];
      boff[tid + 1] = (int32_t)(s.colptr[col + 1] - s.colptr[col]);
      sh_g[tid] = 0.0;
    }
    if (tid == 0) boff[0] = 0;
    __syncthreads();
    if (tid == 0)
      for (int j = 0; j < sb; ++j) boff[j + 1] += boff[j];
    __syncthreads();
    const int E = boff[sb];
    // gradient partials F_B'u, chunk by chunk; column sums in entry order
    for (int f0 = 0; f0 < E; f0 += kFlat) {
      const int fe = f0 + kFlat < E ? f0 + kFlat : E;
      for (int fb = f0 + tid; fb < fe; fb += 256 * kBatch) {
        int32_t row[kBatch];
        double v[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          const int f = fb + 256 * q;
          int64_t e = 0;   // past the chunk: entry 0 of the matrix, which exists (E >= 1), value unused
          if (f < fe) {    // the column of entry f: the last j with boff[j] <= f
            int lo = 0, hi = sb - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (boff[mid] <= f) lo = mid; else hi = mid - 1;
            }
            e = cst[lo] + (f - boff[lo]);
          }
          row[q] = s.rowidx[e];
          v[q] = sv(val, e);
        }
        double uu[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) uu[q] = ld_u(s.u + row[q]);
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          const int f = fb + 256 * q;
          if (f < fe) prod[f - f0] = v[q] * uu[q];
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
      const int col = cols[tid];
      const double xc = s.x[col];
      double v = sh_g[tid] / s.Ns + s.c[col] - s.xi[col] + beta * (xc - s.z[col]);
      if (s.h) v += s.h[col] * xc;
      if (s.a) v += -mu * s.a[col] + beta * s.a[col] * (t - s.b);
      sh_g[tid] = v;
    }
    __syncthreads();
    // step d = -M_B^{-1} g: thread j takes column j of the inverse in batches of 16 loads, summed in k order
    const double* Mi = s.Minv + bi * (int64_t)s.sp * s.sp;
    if (tid < sb) {
      double acc = 0.0;
      for (int k0 = 0; k0 < sb; k0 += 16) {
        double mv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) mv[q] = k0 + q < sb ? Mi[(int64_t)(k0 + q) * s.sp + tid] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (k0 + q < sb) acc += mv[q] * sh_g[k0 + q];
      }
      sh_d[tid] = -acc;
    }
    __syncthreads();
    if (s.a) {
      double dt = 0.0;
      for (int j = 0; j < sb; ++j) dt += s.a[cols[j]] * sh_d[j];
      t += dt;   // every thread forms the same sum in the same order
    }
    // residual update u += F_B d (device-scope atomics: columns may share rows), then x_B
    for (int fb = tid; fb < E; fb += 256 * kBatch) {
      int32_t row[kBatch];
      double v[kBatch];
      double dj[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int f = fb + 256 * q;
        int64_t e = 0;   // past the block: entry 0 of the matrix, value unused
        int j = 0;
        if (f < E) {
          int lo = 0, hi = sb - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (boff[mid] <= f) lo = mid; else hi = mid - 1;
          }
          j = lo;
          e = cst[j] + (f - boff[j]);
        }
        row[q] = s.rowidx[e];
        v[q] = sv(val, e);
        dj[q] = sh_d[j];
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q)
        if (fb + 256 * q < E) add_u(s.u + row[q], v[q] * dj[q]);
    }
    if (tid < sb) s.x[cols[tid]] += sh_d[tid];
    // the additions complete at device scope before the next block's loads of u
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
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
               w.x, w.z, w.xi, w.u, w.sc, w.beta_ptr};
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
