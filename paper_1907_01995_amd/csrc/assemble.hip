// assemble.hip -- phase 1 of an iteration: for every block B of the drawn
// partition, form M_B = F_B'F_B/Ns + diag(h_B) + beta (I + a_B a_B') and factor it.
//
// The block matrices depend only on the data, the partition and beta -- not on
// the iterate -- so all p of them are built in parallel before the sequential
// Gauss-Seidel sweep (the paper re-forms the sub-blocks every iteration and
// never forms the full F'F, Sec.3 and Sec.3.1).
//
// k_gram: grid (p blocks x R row chunks).  Each workgroup gathers its rows of
// the block's columns (columns are contiguous in the column-major data) into
// LDS as a column-major tile and accumulates the lower-triangular 16x16 tiles
// of F_B'F_B on the matrix cores:
//   FP64 precision  : v_mfma_f64_16x16x4f64   (data converted exactly to FP64)
//   mixed, FP32 data: v_mfma_f32_16x16x4f32   (FP32 accumulation)
//   mixed, BF16 data: v_mfma_f32_16x16x32_bf16 (FP32 accumulation)
// Partial Grams of the R chunks are written in FP64 and summed in a fixed order
// by k_factor, which then runs an FP64 Cholesky in LDS (Assumption 2.1: a
// non-positive pivot is reported with its iteration and block) and writes the
// explicit inverse M_B^{-1} = L^{-T} L^{-1}, so the sweep's block solve is a
// parallel matrix-vector product instead of two sequential triangular solves.
#include "rac_internal.h"

namespace rac {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

enum GramMode { G_F64 = 0, G_F32 = 1, G_BF16 = 2 };

template <int MODE> struct GramTraits;
template <> struct GramTraits<G_F64> {
  typedef double E; typedef f64x4 Acc; static constexpr int KT = 16; static constexpr int PAD = 1;
};
template <> struct GramTraits<G_F32> {
  typedef float E; typedef f32x4 Acc; static constexpr int KT = 32; static constexpr int PAD = 1;
};
template <> struct GramTraits<G_BF16> {
  typedef uint16_t E; typedef f32x4 Acc; static constexpr int KT = 64; static constexpr int PAD = 8;
};

template <typename E> __device__ __forceinline__ E to_lds(double v);
template <> __device__ __forceinline__ double to_lds<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_lds<float>(double v) { return (float)v; }

// Raw element -> LDS element.  BF16 data stays as its bit pattern; FP32 data stays FP32.
template <typename T, int MODE> struct Loader;
template <typename T> struct Loader<T, G_F64> {
  __device__ static double get(const T* F, int64_t i) { return ld_f64(F, i); }
};
template <> struct Loader<float, G_F32> {
  __device__ static float get(const float* F, int64_t i) { return F[i]; }
};
template <> struct Loader<uint16_t, G_BF16> {
  __device__ static uint16_t get(const uint16_t* F, int64_t i) { return F[i]; }
};

template <int MODE> struct Zero;
template <> struct Zero<G_F64> { __device__ static double v() { return 0.0; } };
template <> struct Zero<G_F32> { __device__ static float v() { return 0.f; } };
template <> struct Zero<G_BF16> { __device__ static uint16_t v() { return (uint16_t)0; } };

constexpr int kMaxPairsPerWave = 9;   // 36 lower tiles of a 128x128 block over 4 waves

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_gram(const T* __restrict__ F, int64_t ldF, int64_t rows,
                                              int64_t n, int64_t p, const int32_t* __restrict__ perm,
                                              int R, int sp, double* __restrict__ partial) {
  typedef GramTraits<MODE> Tr;
  typedef typename Tr::E E;
  typedef typename Tr::Acc Acc;
  constexpr int KT = Tr::KT;
  constexpr int LD = KT + Tr::PAD;              // LDS row stride of the column-major tile
  __shared__ E tile[kMaxBlock * LD];            // tile[m * LD + k] = F[r0 + k, col_m]
  __shared__ int64_t colbase[kMaxBlock];

  const int blk = blockIdx.x, chunk = blockIdx.y;
  const int64_t s0 = block_start(blk, n, p);
  const int sb = (int)(block_start(blk + 1, n, p) - s0);
  const int64_t rb = block_start(chunk, rows, R), re = block_start(chunk + 1, rows, R);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int NT = sp / 16;
  const int npairs = NT * (NT + 1) / 2;

  for (int m = tid; m < sp; m += 256) colbase[m] = m < sb ? (int64_t)perm[s0 + m] * ldF : -1;

  Acc acc[kMaxPairsPerWave];
  int pti[kMaxPairsPerWave], ptj[kMaxPairsPerWave];
#pragma unroll
  for (int q = 0; q < kMaxPairsPerWave; ++q) {
    acc[q] = Acc{0, 0, 0, 0};
    int pr = wave + 4 * q;               // pair index -> (ti >= tj), row-major over the lower triangle
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= pr) ++ti;
    pti[q] = ti;
    ptj[q] = pr - ti * (ti + 1) / 2;
  }
  __syncthreads();

  for (int64_t r0 = rb; r0 < re; r0 += KT) {
    const int kn = (int)((re - r0) < KT ? (re - r0) : KT);
    // gather: consecutive threads take consecutive rows of one column (contiguous in memory)
    for (int e = tid; e < sp * KT; e += 256) {
      const int m = e / KT, k = e - m * KT;
      const int64_t cb = colbase[m];
      E v = Zero<MODE>::v();
      if (cb >= 0 && k < kn) v = Loader<T, MODE>::get(F, cb + r0 + k);
      tile[m * LD + k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxPairsPerWave; ++q) {
      if (wave + 4 * q < npairs) {
        const int am = pti[q] * 16 + (lane & 15), bn = ptj[q] * 16 + (lane & 15);
        if constexpr (MODE == G_F64) {
#pragma unroll
          for (int kk = 0; kk < KT; kk += 4) {
            double av = tile[am * LD + kk + (lane >> 4)];
            double bv = tile[bn * LD + kk + (lane >> 4)];
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
          }
        } else if constexpr (MODE == G_F32) {
#pragma unroll
          for (int kk = 0; kk < KT; kk += 4) {
            float av = tile[am * LD + kk + (lane >> 4)];
            float bv = tile[bn * LD + kk + (lane >> 4)];
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[q], 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int kk = 0; kk < KT; kk += 32) {
            bf16x8 av, bv;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              av[e] = (short)tile[am * LD + kk + 8 * (lane >> 4) + e];
              bv[e] = (short)tile[bn * LD + kk + 8 * (lane >> 4) + e];
            }
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, av),
                                                             __builtin_bit_cast(bf16x8v, bv),
                                                             acc[q], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  // write the partial lower tiles in FP64
  double* out = partial + ((int64_t)blk * R + chunk) * (int64_t)sp * sp;
#pragma unroll
  for (int q = 0; q < kMaxPairsPerWave; ++q) {
    if (wave + 4 * q < npairs) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int row, col = ptj[q] * 16 + (lane & 15);
        if constexpr (MODE == G_F64) row = pti[q] * 16 + 4 * i + (lane >> 4);   // f64 output layout
        else row = pti[q] * 16 + 4 * (lane >> 4) + i;                           // f32 output layout
        out[(int64_t)row * sp + col] = (double)acc[q][i];
      }
    }
  }
}

// Sum the partial Grams, add the diagonal and penalty terms, Cholesky, inverse.
__global__ void __launch_bounds__(256) k_factor(const double* __restrict__ partial, int R, int sp,
                                                int64_t n, int64_t p, const int32_t* __restrict__ perm,
                                                double Ns, const double* __restrict__ h,
                                                const double* __restrict__ a, const double* beta_ptr,
                                                double beta_val, double* __restrict__ out,
                                                int write_matrix, DevScalars* sc, int64_t iter_global,
                                                int publish_beta) {
  extern __shared__ double smem[];
  const int LDM = sp + 1;
  double* M = smem;                  // M[i * LDM + j], lower triangle
  double* colj = smem + sp * LDM;    // one saved column
  __shared__ int32_t cols[kMaxBlock];
  __shared__ int failed;
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int64_t s0 = block_start(blk, n, p);
  const int sb = (int)(block_start(blk + 1, n, p) - s0);
  const double beta = beta_ptr ? *beta_ptr : beta_val;
  for (int m = tid; m < sp; m += 256) cols[m] = m < sb ? perm[s0 + m] : -1;
  if (tid == 0) failed = 0;
  if (publish_beta && sc && blk == 0 && tid == 0) sc->beta = beta;
  __syncthreads();

  const double* part = partial + (int64_t)blk * R * sp * sp;
  for (int e = tid; e < sp * sp; e += 256) {
    const int i = e / sp, j = e - i * sp;
    if (j > i) continue;
    double v;
    if (i < sb && j < sb) {
      double s = 0.0;
      for (int r = 0; r < R; ++r) s += part[(int64_t)r * sp * sp + e];
      v = s / Ns;
      if (i == j) v += beta + (h ? h[cols[i]] : 0.0);
      if (a) v += beta * a[cols[i]] * a[cols[j]];
    } else {
      v = (i == j) ? 1.0 : 0.0;   // padding: an identity block, decoupled from the real one
    }
    M[i * LDM + j] = v;
  }
  __syncthreads();

  double* dst = out + (int64_t)blk * sp * sp;
  if (write_matrix) {
    for (int e = tid; e < sp * sp; e += 256) {
      const int i = e / sp, j = e - i * sp;
      dst[e] = (j <= i && i < sb) ? M[i * LDM + j] : 0.0;
    }
    return;
  }

  // right-looking Cholesky, lower triangle in place
  for (int k = 0; k < sp; ++k) {
    const double d = M[k * LDM + k];
    if (!(d > 0.0) || !isfinite(d)) {          // same value seen by every thread
      if (tid == 0) {
        failed = 1;
        if (sc) {
          unsigned long long key = ((unsigned long long)iter_global << 32) | (unsigned)blk;
          atomicMin((unsigned long long*)&sc->fail_key, key);
        }
      }
      break;
    }
    const double piv = sqrt(d);
    __syncthreads();
    for (int i = k + 1 + tid; i < sp; i += 256) M[i * LDM + k] /= piv;
    if (tid == 0) M[k * LDM + k] = piv;
    __syncthreads();
    const int mm = sp - k - 1;
    for (int e = tid; e < mm * mm; e += 256) {
      const int ii = e / mm, jj = e - ii * mm;
      if (jj <= ii) {
        const int i = k + 1 + ii, j = k + 1 + jj;
        M[i * LDM + j] -= M[i * LDM + k] * M[j * LDM + k];
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (failed) {
    for (int e = tid; e < sp * sp; e += 256) dst[e] = 0.0;   // zero step for a failed block
    return;
  }

  // X = L^{-1} in place, columns from last to first:
  //   X_jj = 1/L_jj,  X_ij = -(sum_{k=j+1..i} X_ik L_kj) / L_jj  (i > j)
  for (int j = sp - 1; j >= 0; --j) {
    for (int i = j + tid; i < sp; i += 256) colj[i] = M[i * LDM + j];
    __syncthreads();
    for (int i = j + tid; i < sp; i += 256) {
      if (i == j) {
        M[j * LDM + j] = 1.0 / colj[j];
      } else {
        double s = 0.0;
        for (int k = j + 1; k <= i; ++k) s += M[i * LDM + k] * colj[k];
        M[i * LDM + j] = -s / colj[j];
      }
    }
    __syncthreads();
  }
  // M^{-1} = X'X:  (i, j) = sum_{k >= max(i,j)} X_ki X_kj  (symmetric, written in full)
  for (int e = tid; e < sp * sp; e += 256) {
    const int i = e / sp, j = e - i * sp;
    double v = 0.0;
    if (i < sb && j < sb) {
      const int k0 = i > j ? i : j;
      for (int k = k0; k < sb; ++k) v += M[k * LDM + i] * M[k * LDM + j];
    }
    dst[e] = v;
  }
}

template <typename T, int MODE>
hipError_t gram_launch(const GramArgs& g, hipStream_t st) {
  dim3 grid((unsigned)g.p, (unsigned)g.R);
  k_gram<T, MODE><<<grid, 256, 0, st>>>((const T*)g.F, g.ldF, g.rows, g.n, g.p, g.perm, g.R, g.sp,
                                        g.partial);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gram(const GramArgs& g, hipStream_t st) {
  const bool mixed = g.precision == RAC_PREC_MIXED;
  switch (g.dtype) {
    case RAC_DT_F64: return gram_launch<double, G_F64>(g, st);
    case RAC_DT_F32: return mixed ? gram_launch<float, G_F32>(g, st) : gram_launch<float, G_F64>(g, st);
    case RAC_DT_BF16:
      return mixed ? gram_launch<uint16_t, G_BF16>(g, st) : gram_launch<uint16_t, G_F64>(g, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_factor(const FactorArgs& f, hipStream_t st) {
  size_t lds = sizeof(double) * ((size_t)f.sp * (f.sp + 1) + f.sp);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_factor,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(double) * (kMaxBlock * (kMaxBlock + 1) + kMaxBlock)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  k_factor<<<(unsigned)f.p, 256, lds, st>>>(f.partial, f.R, f.sp, f.n, f.p, f.perm, f.Ns, f.h, f.a,
                                            f.beta_ptr, f.beta_val, f.Minv, f.write_matrix, f.sc,
                                            f.iter_global, f.publish_beta);
  return hipGetLastError();
}

}  // namespace rac
