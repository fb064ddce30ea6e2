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

// LDS element type and MFMA of each mode.
template <int MODE> struct GramTraits;
template <> struct GramTraits<G_F64> { typedef double E; typedef f64x4 Acc; static constexpr int PAD = 2; };
template <> struct GramTraits<G_F32> { typedef float E; typedef f32x4 Acc; static constexpr int PAD = 4; };
template <> struct GramTraits<G_BF16> { typedef uint16_t E; typedef f32x4 Acc; static constexpr int PAD = 8; };

// Raw data element (bits) -> LDS element: exact conversions only.
template <typename T, int MODE> __device__ __forceinline__ typename GramTraits<MODE>::E to_lds(T v);
template <> __device__ __forceinline__ double to_lds<double, G_F64>(double v) { return v; }
template <> __device__ __forceinline__ double to_lds<float, G_F64>(float v) { return (double)v; }
template <> __device__ __forceinline__ double to_lds<uint16_t, G_F64>(uint16_t v) {
  return (double)__uint_as_float(((uint32_t)v) << 16);
}
template <> __device__ __forceinline__ float to_lds<float, G_F32>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t to_lds<uint16_t, G_BF16>(uint16_t v) { return v; }

// Rows per LDS tile: about 64 KB of staged columns (at most 256 rows), so that
// each column segment fetched per tile is long (the block's columns are
// scattered over F, and short segments make the gather translation-bound).
template <int MODE, int NCOL>
constexpr int gram_kt() {
  constexpr int bytes = (int)sizeof(typename GramTraits<MODE>::E) * NCOL;
  constexpr int kt = 65536 / bytes;
  return kt >= 256 ? 256 : (kt >= 128 ? 128 : 64);
}

// One workgroup: block `blk`, rows [rb, re).  Data move as 16-byte vectors of
// VE = 16/sizeof(T) consecutive rows of one column; the next 64-row tile is
// loaded into registers while the matrix cores work on the current one.
// With a packed destination (pk.Fp non-null) the loaded values of the block's
// real entries are also written, unchanged, to the sweep's register-order copy:
// entry (row r, column m of block blk) goes to
//   ((((blk K + g) 4 + m % 4) B + m / 4) 64 A) + (r - g RW),   g = r / RW.
// Positions no real entry maps to (short blocks, rows past the end, group
// padding) are never written; the buffer is zeroed once when it is created.
template <typename T, int MODE, int SP>
__device__ __forceinline__ void gram_body(const T* __restrict__ F, int64_t ldF, int64_t rows, int64_t n,
                                          int64_t p, const int32_t* __restrict__ perm, int blk, int chunk,
                                          int R, int vec, double* __restrict__ out,
                                          PackDst pk = PackDst{}, bool mirror = false) {
  typedef GramTraits<MODE> Tr;
  typedef typename Tr::E E;
  typedef typename Tr::Acc Acc;
  constexpr int NCOL = SP;                      // staged columns
  constexpr int KT = gram_kt<MODE, NCOL>();     // rows per tile
  constexpr int VE = 16 / sizeof(T);            // elements per 16-byte vector
  constexpr int VPC = KT / VE;                  // vectors per column per tile
  constexpr int NVEC = NCOL * VPC;
  constexpr int NV = (NVEC + 255) / 256;        // vectors per thread per tile
  constexpr int LD = KT + Tr::PAD;              // LDS row stride of the column-major tile
  constexpr int NT = SP / 16, NPAIR = NT * (NT + 1) / 2;
  constexpr int MAXP = (NPAIR + 3) / 4;
  __shared__ __attribute__((aligned(16))) E tile[NCOL * LD];   // tile[m * LD + k] = F[r0 + k, col_m]
  __shared__ int64_t colbase[NCOL];

  const int64_t s0 = block_start(blk, n, p);
  const int sb = (int)(block_start(blk + 1, n, p) - s0);
  // row chunks are whole tiles except the last
  const int64_t ntiles = (rows + KT - 1) / KT;
  const int64_t rb = block_start(chunk, ntiles, R) * KT;
  const int64_t re_t = block_start(chunk + 1, ntiles, R) * KT;
  const int64_t re = re_t < rows ? re_t : rows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Padding columns (past a block's size) load the block's first column: every
  // consumer ignores the Gram entries of padding, and the packed copy skips them.
  for (int m = tid; m < NCOL; m += 256) colbase[m] = (int64_t)perm[s0 + (m < sb ? m : 0)] * ldF;

  // Every wavefront runs MAXP tile pairs; a wavefront with fewer real pairs runs
  // spare ones on pair 0 and never writes them, so the MFMA loop has no branches.
  Acc acc[MAXP];
  int pti[MAXP], ptj[MAXP];
#pragma unroll
  for (int q = 0; q < MAXP; ++q) {
    acc[q] = Acc{0, 0, 0, 0};
    int pr = wave + 4 * q < NPAIR ? wave + 4 * q : 0;
    int ti = 0;                          // pair index -> (ti >= tj), row-major over the lower triangle
    while ((ti + 1) * (ti + 2) / 2 <= pr) ++ti;
    pti[q] = ti;
    ptj[q] = pr - ti * (ti + 1) / 2;
  }
  __syncthreads();

  T stage[NV][VE];
  auto load = [&](int64_t r0) {
    if (vec && r0 + KT <= re) {   // a whole tile in range: plain vector loads
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int v = tid + 256 * q;
        if (v < NVEC) {
          const int m = v / VPC, seg = v % VPC;
          const uint4 raw = *reinterpret_cast<const uint4*>(F + colbase[m] + r0 + seg * VE);
          const T* e = reinterpret_cast<const T*>(&raw);
#pragma unroll
          for (int u = 0; u < VE; ++u) stage[q][u] = e[u];
        }
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      const int m = v / VPC, seg = v % VPC;
      const int64_t cb = (v < NVEC) ? colbase[m] : -1;
      const int64_t r = r0 + seg * VE;
      if (cb >= 0 && vec && r + VE <= re) {
        const uint4 raw = *reinterpret_cast<const uint4*>(F + cb + r);
        const T* e = reinterpret_cast<const T*>(&raw);
#pragma unroll
        for (int u = 0; u < VE; ++u) stage[q][u] = e[u];
      } else {
#pragma unroll
        for (int u = 0; u < VE; ++u) stage[q][u] = (cb >= 0 && r + u < re) ? F[cb + r + u] : (T)0;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      if (v < NVEC) {
        const int m = v / VPC, seg = v % VPC;
#pragma unroll
        for (int u = 0; u < VE; ++u) tile[m * LD + seg * VE + u] = to_lds<T, MODE>(stage[q][u]);
      }
    }
  };
  // The staged vectors of this tile (rows r0 ..) into the packed copy.  All of a
  // thread's vectors cover the same rows (VPC divides 256), so the group of those
  // rows is found once per tile; rows are below 2^31 (checked by the host).
  static_assert(256 % VPC == 0, "a thread's vectors share their rows");
  const bool pk_vec = pk.Fp && (pk.RW % VE) == 0;   // every vector lies inside one group, aligned
  auto pack = [&](int64_t r0) {
    T* Fp = (T*)pk.Fp;
    const int seg = tid % VPC;
    const int64_t r = r0 + seg * VE;
    if (r >= re) return;
    const uint32_t rw = (uint32_t)pk.RW;
    const uint32_t g = (uint32_t)r / rw;
    const int64_t rr = r - (int64_t)g * rw;
    const bool whole = pk_vec && r + VE <= re;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      const int m = v / VPC;
      if (v >= NVEC || m >= sb) continue;
      T* dst = Fp + (((((int64_t)blk * pk.K + g) * 4 + (m & 3)) * pk.B + (m >> 2)) * 64) * pk.A;
      if (whole) {
        uint4 raw;
        T* e = reinterpret_cast<T*>(&raw);
#pragma unroll
        for (int u = 0; u < VE; ++u) e[u] = stage[q][u];
        *reinterpret_cast<uint4*>(dst + rr) = raw;
      } else {
        for (int u = 0; u < VE && r + u < re; ++u) {
          const uint32_t gu = (uint32_t)(r + u) / rw;
          Fp[(((((int64_t)blk * pk.K + gu) * 4 + (m & 3)) * pk.B + (m >> 2)) * 64) * pk.A +
             (r + u - (int64_t)gu * rw)] = stage[q][u];
        }
      }
    }
  };

  if (rb < re) load(rb);
  for (int64_t r0 = rb; r0 < re; r0 += KT) {
    if (pk.Fp) pack(r0);
    store();
    __syncthreads();
    if (r0 + KT < re) load(r0 + KT);     // next tile in flight during the MFMAs
    // Each lane feeds the rows of one 16-byte LDS read to consecutive MFMAs (the
    // Gram sums over rows, so any assignment of rows to MFMA steps is valid as
    // long as both operands use the same one); the wave's tile pairs form
    // independent accumulation chains, interleaved.
    if constexpr (MODE == G_F64) {
#pragma unroll 2
      for (int kk = 0; kk < KT; kk += 8) {
#pragma unroll
        for (int q = 0; q < MAXP; ++q) {
          {
            const int am = pti[q] * 16 + (lane & 15), bn = ptj[q] * 16 + (lane & 15);
            const double2 a2 = *reinterpret_cast<const double2*>(&tile[am * LD + kk + 2 * (lane >> 4)]);
            const double2 b2 = *reinterpret_cast<const double2*>(&tile[bn * LD + kk + 2 * (lane >> 4)]);
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.x, b2.x, acc[q], 0, 0, 0);
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.y, b2.y, acc[q], 0, 0, 0);
          }
        }
      }
    } else if constexpr (MODE == G_F32) {
#pragma unroll 2
      for (int kk = 0; kk < KT; kk += 16) {
#pragma unroll
        for (int q = 0; q < MAXP; ++q) {
          {
            const int am = pti[q] * 16 + (lane & 15), bn = ptj[q] * 16 + (lane & 15);
            const float4 a4 = *reinterpret_cast<const float4*>(&tile[am * LD + kk + 4 * (lane >> 4)]);
            const float4 b4 = *reinterpret_cast<const float4*>(&tile[bn * LD + kk + 4 * (lane >> 4)]);
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, b4.x, acc[q], 0, 0, 0);
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, b4.y, acc[q], 0, 0, 0);
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, b4.z, acc[q], 0, 0, 0);
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, b4.w, acc[q], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll 2
      for (int kk = 0; kk < KT; kk += 32) {
#pragma unroll
        for (int q = 0; q < MAXP; ++q) {
          {
            const int am = pti[q] * 16 + (lane & 15), bn = ptj[q] * 16 + (lane & 15);
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&tile[am * LD + kk + 8 * (lane >> 4)]);
            const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&tile[bn * LD + kk + 8 * (lane >> 4)]);
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, av),
                                                             __builtin_bit_cast(bf16x8v, bv),
                                                             acc[q], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  // write the partial lower tiles in FP64.  With `mirror` (a whole Gram, R = 1) every
  // strictly lower entry is also written to its transposed place and the diagonal tiles'
  // upper halves are left to those writes: the stored matrix is exactly symmetric, its
  // lower triangle unchanged, and readers can take any row whole
#pragma unroll
  for (int q = 0; q < MAXP; ++q) {
    if (wave + 4 * q < NPAIR) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int row, col = ptj[q] * 16 + (lane & 15);
        if constexpr (MODE == G_F64) row = pti[q] * 16 + 4 * i + (lane >> 4);   // f64 output layout
        else row = pti[q] * 16 + 4 * (lane >> 4) + i;                           // f32 output layout
        const double v = (double)acc[q][i];
        if (!mirror || row >= col) out[(int64_t)row * SP + col] = v;
        if (mirror && row > col) out[(int64_t)col * SP + row] = v;
      }
    }
  }
}

template <typename T, int MODE, int SP>
__global__ void __launch_bounds__(256) k_gram(const T* __restrict__ F, int64_t ldF, int64_t rows,
                                              int64_t n, int64_t p, const int32_t* __restrict__ perm,
                                              int R, int vec, double* __restrict__ partial, PackDst pk) {
  const int blk = blockIdx.x, chunk = blockIdx.y;
  gram_body<T, MODE, SP>(F, ldF, rows, n, p, perm, blk, chunk, R, vec,
                         partial + ((int64_t)blk * R + chunk) * (int64_t)SP * SP, pk);
}

// Batched form: one workgroup per (instance, block) task of a batch; the Gram of
// each block is shared by all lanes of its instance.  Iteration t = t0 + blockIdx.y
// of the chunk selects the instance's partition for that iteration and the Gram
// slot G + t * gslot.
template <typename T, int MODE, int SP>
__global__ void __launch_bounds__(256) k_bgram(const BInst* __restrict__ inst, const int2* __restrict__ tasks,
                                               const int32_t* __restrict__ perm, int t0, int64_t gslot,
                                               const int32_t* __restrict__ inst_active,
                                               double* __restrict__ G) {
  const int t = t0 + (int)blockIdx.y;
  G += t * gslot;
  const int2 tk = tasks[blockIdx.x];
  if (!inst_active[tk.x]) return;
  const BInst I = inst[tk.x];
  gram_body<T, MODE, SP>((const T*)I.F, I.ldF, I.rows, I.n, I.p, perm + I.poff + (int64_t)t * I.n, tk.y,
                         0, 1, I.vec, G + (I.goff + tk.y) * (int64_t)SP * SP, PackDst{}, true);
}

// Position of block blk in the solve order of an RP iteration (the failure report
// names the position, as for a drawn partition); without an order, blk itself.
__device__ __forceinline__ int64_t order_position(const int32_t* order, int64_t p, int64_t blk) {
  if (!order) return blk;
  for (int64_t i = 0; i < p; ++i)
    if (order[i] == blk) return i;
  return blk;
}

// Sum the partial Grams, add the diagonal and penalty terms, then invert the
// block matrix by Gauss-Jordan elimination without pivoting.  For a symmetric
// positive definite matrix the k-th pivot is the k-th diagonal entry of the
// Schur complement, i.e. the square of the k-th Cholesky pivot, so Assumption
// 2.1 is checked exactly as a Cholesky factorisation would check it (a pivot
// that is not positive is reported with its iteration and block).
//
// The SP x SP matrix lives in registers: thread (ti, tj) of a 16 x 16 grid owns
// rows ti + 16a and columns tj + 16b (a, b < SP/16).  At pivot k only row k and
// column k travel through LDS (double-buffered by the parity of k, one barrier
// per step); every owned entry is then updated independently.
template <int SP>
__global__ void __launch_bounds__(256) k_factor(const double* __restrict__ partial, int R, int64_t n,
                                                int64_t p, const int32_t* __restrict__ perm, double Ns,
                                                const double* __restrict__ h, const double* __restrict__ a,
                                                const double* beta_ptr, double beta_val,
                                                double* __restrict__ out, int write_matrix, DevScalars* sc,
                                                int64_t iter_global, const int32_t* __restrict__ order) {
  constexpr int NA = SP / 16;
  __shared__ double rowk[2][SP];
  __shared__ double colk[2][SP];
  __shared__ int32_t cols[SP];
  const int blk = blockIdx.x, tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int64_t s0 = block_start(blk, n, p);
  const int sb = (int)(block_start(blk + 1, n, p) - s0);
  const double beta = beta_ptr ? *beta_ptr : beta_val;
  for (int m = tid; m < SP; m += 256) cols[m] = m < sb ? perm[s0 + m] : -1;
  __syncthreads();

  // gather: entry (i, j) is the lower-triangle partial (max, min); R partials summed in order
  const double* part = partial + (int64_t)blk * R * SP * SP;
  double Mr[NA][NA];
#pragma unroll
  for (int aa = 0; aa < NA; ++aa)
#pragma unroll
    for (int bb = 0; bb < NA; ++bb) Mr[aa][bb] = 0.0;
  for (int r = 0; r < R; ++r) {
    const double* pr = part + (int64_t)r * SP * SP;
    double v[NA][NA];
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
      for (int bb = 0; bb < NA; ++bb) {
        const int i = ti + 16 * aa, j = tj + 16 * bb;
        v[aa][bb] = (i < sb && j < sb) ? pr[i >= j ? i * SP + j : j * SP + i] : 0.0;
      }
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
      for (int bb = 0; bb < NA; ++bb) Mr[aa][bb] += v[aa][bb];
  }
#pragma unroll
  for (int aa = 0; aa < NA; ++aa)
#pragma unroll
    for (int bb = 0; bb < NA; ++bb) {
      const int i = ti + 16 * aa, j = tj + 16 * bb;
      double v;
      if (i < sb && j < sb) {
        v = Mr[aa][bb] / Ns;
        if (i == j) v += beta + (h ? h[cols[i]] : 0.0);
        if (a) v += beta * a[cols[i]] * a[cols[j]];
      } else {
        v = (i == j) ? 1.0 : 0.0;   // padding: an identity block, decoupled from the real one
      }
      Mr[aa][bb] = v;
    }

  double* dst = out + (int64_t)blk * SP * SP;
  if (write_matrix) {
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
      for (int bb = 0; bb < NA; ++bb) {
        const int i = ti + 16 * aa, j = tj + 16 * bb;
        dst[i * SP + j] = (j <= i && i < sb) ? Mr[aa][bb] : 0.0;
      }
    return;
  }

  bool failed = false;
  for (int k = 0; k < sb; ++k) {
    const int buf = k & 1;
    const int ka = k >> 4, kr = k & 15;
    // owners of row k and column k publish them
    if (ti == kr) {
#pragma unroll
      for (int aa = 0; aa < NA; ++aa)
        if (aa == ka)
#pragma unroll
          for (int bb = 0; bb < NA; ++bb) rowk[buf][tj + 16 * bb] = Mr[aa][bb];
    }
    if (tj == kr) {
#pragma unroll
      for (int bb = 0; bb < NA; ++bb)
        if (bb == ka)
#pragma unroll
          for (int aa = 0; aa < NA; ++aa) colk[buf][ti + 16 * aa] = Mr[aa][bb];
    }
    __syncthreads();
    const double piv = rowk[buf][k];           // the same value in every thread
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (tid == 0 && sc) {
        unsigned long long key = ((unsigned long long)iter_global << 32) | (unsigned)order_position(order, p, blk);
        atomicMin((unsigned long long*)&sc->fail_key, key);
      }
      failed = true;
      break;
    }
    const double ip = 1.0 / piv;
    double rk[NA], ck[NA];
#pragma unroll
    for (int bb = 0; bb < NA; ++bb) rk[bb] = rowk[buf][tj + 16 * bb] * ip;
#pragma unroll
    for (int aa = 0; aa < NA; ++aa) ck[aa] = colk[buf][ti + 16 * aa];
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
      for (int bb = 0; bb < NA; ++bb) {
        const bool ri = (ti + 16 * aa) == k, cj = (tj + 16 * bb) == k;
        double v;
        if (ri) v = cj ? ip : rk[bb];
        else if (cj) v = -ck[aa] * ip;
        else v = Mr[aa][bb] - ck[aa] * rk[bb];
        Mr[aa][bb] = v;
      }
  }
  if (failed) {
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
      for (int bb = 0; bb < NA; ++bb) dst[(ti + 16 * aa) * SP + tj + 16 * bb] = 0.0;   // zero step
    return;
  }
#pragma unroll
  for (int aa = 0; aa < NA; ++aa)
#pragma unroll
    for (int bb = 0; bb < NA; ++bb) {
      const int i = ti + 16 * aa, j = tj + 16 * bb;
      dst[i * SP + j] = (i < sb && j < sb) ? Mr[aa][bb] : 0.0;
    }
}

template <typename T, int MODE>
hipError_t gram_launch(const GramArgs& g, hipStream_t st) {
  dim3 grid((unsigned)g.p, (unsigned)g.R);
  const int vec = (g.ldF % (16 / (int)sizeof(T)) == 0) && ((uintptr_t)g.F % 16 == 0);
  const T* F = (const T*)g.F;
#define RAC_GRAM(SPV)                                                                          \
  if (g.sp == SPV) {                                                                           \
    k_gram<T, MODE, SPV><<<grid, 256, 0, st>>>(F, g.ldF, g.rows, g.n, g.p, g.perm, g.R, vec,   \
                                               g.partial, g.pack);                            \
    return hipGetLastError();                                                                 \
  }
  RAC_GRAM(16) RAC_GRAM(32) RAC_GRAM(64) RAC_GRAM(128)
#undef RAC_GRAM
  return hipErrorInvalidValue;
}

// One wavefront per block (SP <= 64), the lower-latency form of k_factor for
// the single-instance solver: lane j holds column j of M_B in registers and
// applies the symmetric sweep operator to pivots 0..sb-1,
//   a_ij -= a_ik a_kj / d,  a_kj /= d,  a_ik /= d,  a_kk = -1/d   (d = a_kk),
// after which the block holds -M_B^{-1}; d is the k-th Schur-complement pivot (the
// squared Cholesky pivot), so a non-positive one is the failure of Assumption 2.1
// reported with its iteration and block.  The running matrix stays symmetric, so
// the pivot column equals the pivot row, which every lane holds in register 0
// (registers are renumbered after every pivot; all indices are compile-time).
// No workgroup barrier: one LDS write and read per pivot within the wavefront.
template <int SP>
__global__ void __launch_bounds__(64) k_factor_wave(const double* __restrict__ partial, int R, int64_t n,
                                                    int64_t p, const int32_t* __restrict__ perm, double Ns,
                                                    const double* __restrict__ h, const double* __restrict__ a,
                                                    const double* beta_ptr, double beta_val,
                                                    double* __restrict__ out, DevScalars* sc,
                                                    int64_t iter_global, const int32_t* __restrict__ order) {
  static_assert(SP <= 64, "one lane per column");
  constexpr int HALF = SP > 32 ? SP / 2 : SP;
  __shared__ double buf[2 * SP];
  const int blk = blockIdx.x, j = threadIdx.x;
  const int64_t s0 = block_start(blk, n, p);
  const int sb = (int)(block_start(blk + 1, n, p) - s0);
  const double beta = beta_ptr ? *beta_ptr : beta_val;
  const int colj = j < sb ? perm[s0 + j] : 0;
  const double hj = (h && j < sb) ? h[colj] : 0.0;
  const double aj = (a && j < sb) ? a[colj] : 0.0;
  if (a && j < SP) buf[j] = aj;
  // column j of the summed Gram: the R row-chunk partials in order (lower triangle stored)
  double col[SP];
#pragma unroll
  for (int i = 0; i < SP; ++i) col[i] = 0.0;
  const double* part = partial + (int64_t)blk * R * SP * SP;
  for (int r = 0; r < R; ++r) {
    const double* pr = part + (int64_t)r * SP * SP;
#pragma unroll
    for (int h0 = 0; h0 < SP; h0 += HALF) {
      double v[HALF];
#pragma unroll
      for (int q = 0; q < HALF; ++q) {
        const int i = h0 + q;
        v[q] = (i < sb && j < sb) ? pr[i >= j ? i * SP + j : j * SP + i] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < HALF; ++q) col[h0 + q] += v[q];
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int i = 0; i < SP; ++i) {
    double v;
    if (i < sb && j < sb) {
      v = col[i] / Ns;
      if (i == j) v += beta + hj;
      if (a) v += beta * buf[i] * aj;
    } else {
      v = (i == j) ? 1.0 : 0.0;   // padding: an identity block, decoupled from the real one
    }
    col[i] = v;
  }
  __builtin_amdgcn_wave_barrier();
  bool failed = false;
  for (int k = 0; k < sb; ++k) {
    const double rk = col[0];                   // a_kj
    if (j < SP) { buf[j] = rk; buf[j + SP] = rk; }
    __builtin_amdgcn_wave_barrier();
    const double d = buf[k];                    // the same value in every lane
    if (!(d > 0.0) || !isfinite(d)) {
      failed = true;
      if (j == 0 && sc) {
        const unsigned long long key = ((unsigned long long)iter_global << 32) | (unsigned)order_position(order, p, blk);
        atomicMin((unsigned long long*)&sc->fail_key, key);
      }
      break;
    }
    const double invd = 1.0 / d;
    const bool pv = j == k;
    const double keep = pv ? 0.0 : 1.0;
    const double m = pv ? -invd : rk * invd;
#pragma unroll
    for (int q = 1; q < SP; ++q) col[q - 1] = fma(-buf[k + q], m, keep * col[q]);   // buf[k+q] = a_(k+q mod SP),k
    col[SP - 1] = m;
    __builtin_amdgcn_wave_barrier();
  }
  double* dst = out + (int64_t)blk * SP * SP;
  if (j < SP) {
#pragma unroll
    for (int q = 0; q < SP; ++q) {
      int i = q + sb;                           // register q holds row (q + sb) mod SP
      if (i >= SP) i -= SP;
      dst[i * SP + j] = (!failed && i < sb && j < sb) ? -col[q] : 0.0;
    }
  }
}

}  // namespace


template <typename T, int MODE>
hipError_t bgram_launch(const BatchGramArgs& g, hipStream_t st) {
  const T* dummy = nullptr;
  (void)dummy;
#define RAC_BGRAM(SPV)                                                                            \
  if (g.sp == SPV) {                                                                              \
    k_bgram<T, MODE, SPV><<<dim3((unsigned)g.ntasks, (unsigned)g.nt), 256, 0, st>>>(              \
        g.inst, g.tasks, g.perm, g.t, g.gslot, g.inst_active, g.G);                                \
    return hipGetLastError();                                                                    \
  }
  RAC_BGRAM(16) RAC_BGRAM(32) RAC_BGRAM(64)
#undef RAC_BGRAM
  return hipErrorInvalidValue;
}

hipError_t launch_bgram(const BatchGramArgs& g, hipStream_t st) {
  if (g.ntasks <= 0 || g.nt <= 0) return hipSuccess;
  const bool mixed = g.precision == RAC_PREC_MIXED;
  switch (g.dtype) {
    case RAC_DT_F64: return bgram_launch<double, G_F64>(g, st);
    case RAC_DT_F32: return mixed ? bgram_launch<float, G_F32>(g, st) : bgram_launch<float, G_F64>(g, st);
    case RAC_DT_BF16:
      return mixed ? bgram_launch<uint16_t, G_BF16>(g, st) : bgram_launch<uint16_t, G_F64>(g, st);
    default: return hipErrorInvalidValue;
  }
}

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
  if (!f.write_matrix && f.sp <= 64) {
#define RAC_FACTORW(SPV)                                                                                  \
    if (f.sp == SPV) {                                                                                   \
      k_factor_wave<SPV><<<(unsigned)f.p, 64, 0, st>>>(f.partial, f.R, f.n, f.p, f.perm, f.Ns, f.h, f.a,  \
                                                       f.beta_ptr, f.beta_val, f.Minv, f.sc,           \
                                                       f.iter_global, f.order);                        \
      return hipGetLastError();                                                                        \
    }
    RAC_FACTORW(16) RAC_FACTORW(32) RAC_FACTORW(64)
#undef RAC_FACTORW
  }
#define RAC_FACTOR(SPV)                                                                              \
  if (f.sp == SPV) {                                                                                 \
    k_factor<SPV><<<(unsigned)f.p, 256, 0, st>>>(f.partial, f.R, f.n, f.p, f.perm, f.Ns, f.h, f.a,     \
                                                  f.beta_ptr, f.beta_val, f.Minv, f.write_matrix, f.sc, \
                                                  f.iter_global, f.order);                              \
    return hipGetLastError();                                                                        \
  }
  RAC_FACTOR(16) RAC_FACTOR(32) RAC_FACTOR(64) RAC_FACTOR(128)
#undef RAC_FACTOR
  return hipErrorInvalidValue;
}

}  // namespace rac
