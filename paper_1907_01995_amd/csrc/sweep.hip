// sweep.hip -- phase 2 of an iteration: the cyclic Gauss-Seidel pass over the
// drawn blocks (Eq.(3), x_1 ... x_p in order), one persistent launch per sweep.
//
// For block B the exact minimiser of the augmented Lagrangian over x_B is
//   x_B <- x_B - M_B^{-1} g_B,
//   g_B = F_B'u/Ns + h_B.x_B + c_B - xi_B + beta(x_B - z_B) - mu a_B + beta a_B (t - b),
// where u = F x and t = a'x are maintained through the sweep (u += F_B d, t += a_B'd).
// Everything in g_B except F_B'u and the t term is fixed before the block is
// reached (x_B changes only when B itself is solved), so it is gathered while
// the previous block is still being exchanged.
//
// Work split: K cooperating workgroups each own a contiguous range of at most
// 64*A rows of F, and hence of u, which never leaves its owner (registers).
// Lane l of every wavefront holds rows A l .. A l + A - 1 of the range;
// wavefront w holds block columns w, w+4, ... (B of them).  Per block:
//   1. the block's tile of F (rows x columns) is already in registers: it was
//      read from the packed copy the Gram kernel wrote (or gathered from F)
//      while the previous block was finishing, so each element of F is read
//      from HBM once per sweep and serves both products below;
//   2. partial F_B'u over the group's rows (FP64 accumulation, transposed
//      lane exchanges), published with agent-scope relaxed atomic stores;
//   3. every group polls the K partials until none is the empty pattern (block
//      0: epoch flags first), then issues the next block's tile and gradient
//      inputs, which arrive during the solve and the update;
//   4. every group sums the K partials in the same fixed order, applies M_B^{-1}
//      (formed by the factor kernel) and so holds the identical step d;
//   5. its rows of u are updated from the register tile; group 0 writes x_B.
// Cross-group traffic uses only device-coherent (agent-scope) loads and stores
// and s_waitcnt -- no cache write-back or invalidation.  Partials rotate through
// three buffers; the protocol is described at the exchange below.
#include "rac_internal.h"
#include <type_traits>

namespace rac {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_sweep(const T* __restrict__ F, int64_t ldF, int64_t rows,
                                               int64_t n, int64_t p, const int32_t* __restrict__ perm,
                                               const double* __restrict__ Minv, int sp,
                                               const double* __restrict__ c, const double* __restrict__ h,
                                               const double* __restrict__ a, double b, double Ns,
                                               double* x, const double* __restrict__ z,
                                               const double* __restrict__ xi, double* u,
                                               DevScalars* sc, const double* beta_ptr,
                                               double* partials, uint64_t* flags, uint64_t epoch_base,
                                               int max_spin, const int32_t* __restrict__ order) {
  const int K = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = block_start(g, rows, K), r1 = block_start(g + 1, rows, K);
  __shared__ double gl[kMaxBlock];     // partial, then full gradient
  __shared__ double dl[kMaxBlock];     // step d = -M^{-1} g
  __shared__ int32_t cols[kMaxBlock];
  __shared__ double t_sh;
  __shared__ int abort_sh;
  if (tid == 0) abort_sh = 0;
  const double beta = *beta_ptr;
  const double mu = sc->mu;
  double t = sc->t;

  for (int64_t i = 0; i < p; ++i) {
    const int64_t bi = order ? (int64_t)order[i] : i;   // block solved at position i
    const int64_t s0 = block_start(bi, n, p);
    const int sb = (int)(block_start(bi + 1, n, p) - s0);
    for (int j = tid; j < sb; j += 256) cols[j] = perm[s0 + j];
    __syncthreads();

    // 1. partial F_B'u over this workgroup's rows; one wavefront per column
    double* buf = partials + (int64_t)(i & 1) * K * kMaxBlock;
    for (int j = wave; j < sb; j += 4) {
      const T* col = F + (int64_t)cols[j] * ldF;
      double acc = 0.0;
      for (int64_t r = r0 + lane; r < r1; r += 64) acc += ld_f64(col, r) * u[r];
      acc = wave_sum(acc);
      if (lane == 0) buf[(int64_t)g * kMaxBlock + j] = acc;
    }
    // 2. publish: make the partials visible device-wide, then raise this group's flag
    __threadfence();
    __syncthreads();
    const uint64_t epoch = epoch_base + (uint64_t)i + 1;
    if (K > 1) {
      if (tid == 0)
        __hip_atomic_store(&flags[(int64_t)g * kFlagStride], epoch, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      if (wave == 0) {   // bounded: gives up after max_spin polls of one flag
        bool gave_up = false;
        for (int q = lane; q < K && !gave_up; q += 64)
          for (int tries = 0; __hip_atomic_load(&flags[(int64_t)q * kFlagStride], __ATOMIC_ACQUIRE,
                                                __HIP_MEMORY_SCOPE_AGENT) < epoch; ++tries) {
            if (tries >= max_spin) { gave_up = true; break; }
            __builtin_amdgcn_s_sleep(1);
          }
        if (gave_up) abort_sh = 1;
      }
      __syncthreads();
      if (abort_sh) {   // a group never published: leave (every thread sees the same flag)
        if (tid == 0) __hip_atomic_store(&sc->wait_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
    }
    // 3. full gradient (fixed summation order over groups), then the step
    for (int j = tid; j < sb; j += 256) {
      double s = 0.0;
      for (int q = 0; q < K; ++q) s += buf[(int64_t)q * kMaxBlock + j];
      const int col = cols[j];
      double v = s / Ns + c[col] - xi[col] + beta * (x[col] - z[col]);
      if (h) v += h[col] * x[col];
      if (a) v += -mu * a[col] + beta * a[col] * (t - b);
      gl[j] = v;
    }
    __syncthreads();
    const double* Mi = Minv + bi * (int64_t)sp * sp;
    for (int j = tid; j < sb; j += 256) {
      double s = 0.0;
      for (int k = 0; k < sb; ++k) s += Mi[(int64_t)k * sp + j] * gl[k];
      dl[j] = -s;
    }
    __syncthreads();
    if (a) {
      if (tid == 0) {
        double dt = 0.0;
        for (int j = 0; j < sb; ++j) dt += a[cols[j]] * dl[j];
        t_sh = t + dt;
      }
      __syncthreads();
      t = t_sh;
    }
    // 4. own rows of u, and x_B
    for (int64_t r = r0 + tid; r < r1; r += 256) {
      double acc = u[r];
      for (int j = 0; j < sb; ++j) acc += ld_f64(F + (int64_t)cols[j] * ldF, r) * dl[j];
      u[r] = acc;
    }
    if (g == 0)
      for (int j = tid; j < sb; j += 256) x[cols[j]] += dl[j];
    __syncthreads();
  }
  if (g == 0 && tid == 0) sc->t = t;
}

// ---------------------------------------------------------------------------
// Register-tiled sweep (the default path).

template <typename T> struct RegT { typedef float type; };
template <> struct RegT<double> { typedef double type; };
__device__ __forceinline__ float ld_reg(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ld_reg(const uint16_t* p, int64_t i) {
  return __uint_as_float(((uint32_t)p[i]) << 16);
}
__device__ __forceinline__ double ld_reg(const double* p, int64_t i) { return p[i]; }

// Register tile of A rows x B columns of F in the storage type's register form:
// FP64 and FP32 one value per register, BF16 two per 32-bit register (rows 2r
// and 2r + 1 of a column in the low and high halves, as they lie in memory), so
// that two 32-column tiles leave room for the rest of the sweep.  at(aa, bb)
// converts exactly to FP64.
template <typename T, int A, int B>
struct Tile {
  typedef typename RegT<T>::type R;
  R v[A][B];
  __device__ __forceinline__ double at(int aa, int bb) const { return (double)v[aa][bb]; }
  __device__ __forceinline__ void zero(int bb) {
#pragma unroll
    for (int aa = 0; aa < A; ++aa) v[aa][bb] = (R)0;
  }
  // A consecutive, vector-aligned elements of a column
  __device__ __forceinline__ void load_vec(int bb, const T* p) {
    if constexpr (A > 1) {
      typedef T VT __attribute__((ext_vector_type(A)));
      const VT x = *reinterpret_cast<const VT*>(p);
#pragma unroll
      for (int aa = 0; aa < A; ++aa) v[aa][bb] = ld_reg(reinterpret_cast<const T*>(&x), aa);
    } else {
      v[0][bb] = ld_reg(p, 0);
    }
  }
  // the first nvalid of A consecutive elements, zeros after them
  __device__ __forceinline__ void load_elems(int bb, const T* p, int64_t nvalid) {
#pragma unroll
    for (int aa = 0; aa < A; ++aa) v[aa][bb] = aa < nvalid ? ld_reg(p, aa) : (R)0;
  }
};
template <int A, int B>
struct Tile<uint16_t, A, B> {
  static constexpr int W = (A + 1) / 2;
  uint32_t w[W][B];
  __device__ __forceinline__ double at(int aa, int bb) const {
    const uint32_t x = w[aa >> 1][bb];
    return (double)__uint_as_float((aa & 1) ? (x & 0xffff0000u) : (x << 16));
  }
  __device__ __forceinline__ void zero(int bb) {
#pragma unroll
    for (int q = 0; q < W; ++q) w[q][bb] = 0u;
  }
  __device__ __forceinline__ void load_vec(int bb, const uint16_t* p) {
    if constexpr (A == 1) {
      w[0][bb] = p[0];
    } else if constexpr (A == 2) {
      w[0][bb] = *reinterpret_cast<const uint32_t*>(p);
    } else {
      static_assert(A == 4, "BF16 tiles hold 1, 2 or 4 rows per lane");
      const uint2 x = *reinterpret_cast<const uint2*>(p);
      w[0][bb] = x.x;
      w[1][bb] = x.y;
    }
  }
  __device__ __forceinline__ void load_elems(int bb, const uint16_t* p, int64_t nvalid) {
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const uint32_t lo = 2 * q < nvalid ? (uint32_t)p[2 * q] : 0u;
      const uint32_t hi = (2 * q + 1 < A && 2 * q + 1 < nvalid) ? (uint32_t)p[2 * q + 1] : 0u;
      w[q][bb] = lo | (hi << 16);
    }
  }
};

__device__ __forceinline__ void st_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coherent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Sweep2Args {
  const void* F; int64_t ldF; int64_t rows; int64_t n; int64_t p;
  const int32_t* perm; const double* Minv; int sp;
  const double* c; const double* h; const double* xi; const double* z; const double* beta_ptr;
  const double* a; double b; double Ns;
  double* x; double* u; DevScalars* sc; double* partials; uint64_t* flags; uint64_t epoch_base;
  int64_t RW;              // rows per group (a multiple of A, at most 64A)
  int vec;                 // column starts allow A-element vector loads
  const void* Fp;          // packed tiles of this iteration's blocks, or null (gather from F)
  int max_spin;            // polls of one batch of partials before a group gives up
  const int32_t* order;    // RP: position i solves block order[i]; null: block i
  int dense;               // dense form: F is the symmetric Hessian (rows = variables) and u is x itself
};

// Lane l holds rows r0 + A l + a (a < A) of the group's range: A consecutive
// rows of a column form one vector load when the data are aligned.
template <typename T, int A, int B>
__device__ __forceinline__ void load_tile(const T* __restrict__ F, int64_t ldF, int64_t r0, int64_t r1,
                                          const int32_t* cols, int sb, int lane, int wave, int vec,
                                          Tile<T, A, B>& tile) {
  const int64_t rl = r0 + (int64_t)A * lane;
#pragma unroll
  for (int bb = 0; bb < B; ++bb) {
    const int j = wave + 4 * bb;
    if (j < sb) {
      const T* colp = F + (int64_t)cols[j] * ldF + rl;
      if (A > 1 && vec && rl + A <= r1) tile.load_vec(bb, colp);
      else tile.load_elems(bb, colp, r1 - rl);
    } else {
      tile.zero(bb);
    }
  }
}

// Packed tiles: the Gram kernel also copies each block's columns into the exact
// register order of the sweep, tile (block i, group g) = [4 wavefronts][B][64
// lanes][A] values of the storage type, zero outside the block and the rows.
// One group then reads one contiguous run per block instead of 4B scattered
// column segments (whose address translations dominate the fetch otherwise).
template <typename T, int A, int B>
__device__ __forceinline__ void load_packed(const T* __restrict__ Fp, int64_t i, int K, int g, int lane, int wave,
                                            Tile<T, A, B>& tile) {
  const T* base = Fp + ((((i * K + g) * 4 + wave) * B) * 64 + lane) * (int64_t)A;
#pragma unroll
  for (int bb = 0; bb < B; ++bb) tile.load_vec(bb, base + (int64_t)bb * 64 * A);
}

// An empty partial slot: a signalling-NaN bit pattern (arithmetic only produces
// quiet NaNs), compared bit for bit.
constexpr uint64_t kEmptyBits = 0x7FF4A5A55A5AA5A5ull;
constexpr double kEmpty = __builtin_bit_cast(double, kEmptyBits);
__device__ __forceinline__ bool is_empty(double v) { return __builtin_bit_cast(uint64_t, v) == kEmptyBits; }
constexpr int kMaxSpin = 1 << 20;   // default polls of one batch of partials before a group gives up

// Lane exchange x -> x of lane (l xor O).  Within the 16-lane rows (O <= 8) by
// DPP moves, which stay in the vector ALU: O = 8 is a row rotation by 8, O = 4 a
// half-row mirror (l xor 7) followed by the quad permutation l xor 3, O = 2 and
// O = 1 quad permutations.  Across rows (O = 16, 32) by the LDS permute unit.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int O>
__device__ __forceinline__ double lane_xor(double x) {
  if constexpr (O == 8) return dpp_move<0x128>(x);                      // row_ror:8
  else if constexpr (O == 4) return dpp_move<0x1B>(dpp_move<0x141>(x));  // row_half_mirror, quad_perm [3,2,1,0]
  else if constexpr (O == 2) return dpp_move<0x4E>(x);                  // quad_perm [2,3,0,1]
  else if constexpr (O == 1) return dpp_move<0xB1>(x);                  // quad_perm [1,0,3,2]
  else return __shfl_xor(x, O, 64);
}

// Per-column sums of B per-lane values (B = 8 or 16) over the 64 lanes: halving
// exchanges at lane distances 8, 4, 2 (, 1) inside each 16-lane row leave lane l
// with a row partial of column c = (l & 15) >> (4 - log2 B); full sums finish
// the row (B = 8: distance 1) and add the four rows (distances 16, 32).  Every
// lane ends with its column's total; the summation pattern is fixed.
template <int B>
__device__ __forceinline__ double row_transpose_sum(double (&v)[B], int lane, int& c) {
  static_assert(B == 8 || B == 16, "row-local transposition covers 8 or 16 columns");
  auto stage = [&](auto o_tag, int half) {
    constexpr int O = decltype(o_tag)::value;
    const bool upper = (lane & O) != 0;
#pragma unroll
    for (int q = 0; q < B / 2; ++q) {
      if (q < half) {
        const double send = upper ? v[q] : v[q + half];
        const double keep = upper ? v[q + half] : v[q];
        v[q] = keep + lane_xor<O>(send);
      }
    }
  };
  stage(std::integral_constant<int, 8>{}, B / 2);
  stage(std::integral_constant<int, 4>{}, B / 4);
  stage(std::integral_constant<int, 2>{}, B / 8);
  double r = v[0];
  if constexpr (B == 16) {
    stage(std::integral_constant<int, 1>{}, 1);
    r = v[0];
    c = lane & 15;
  } else {
    r += lane_xor<1>(r);
    c = (lane & 15) >> 1;
  }
  r += lane_xor<16>(r);
  r += lane_xor<32>(r);
  return r;
}

// Sum B per-lane values across the 64 lanes, transposed (B = 32): halving
// exchanges at lane distances 32, 16, 8, 4, 2 leave lane l with one column's
// partial over a lane subset, then a full reduction over the remaining lane
// bit.  Lane l ends with the total of column index c(l) (bits 5, 4, ... of l,
// most significant first); it is returned together with c.  The stages are
// unrolled at compile time so that v stays in registers, and the summation
// pattern is fixed.
template <int HALF, int O, int B>
__device__ __forceinline__ void transpose_stage(double (&v)[B], int lane) {
  const bool upper = (lane & O) != 0;
#pragma unroll
  for (int q = 0; q < HALF; ++q) {
    const double send = upper ? v[q] : v[q + HALF];
    const double keep = upper ? v[q + HALF] : v[q];
    v[q] = keep + lane_xor<O>(send);
  }
  if constexpr (HALF > 1) transpose_stage<HALF / 2, O / 2, B>(v, lane);
}
template <int B>
__device__ __forceinline__ double transpose_sum(double (&v)[B], int lane, int& c) {
  static_assert(B == 32, "the row-local transposition covers 8 or 16 columns");
  transpose_stage<B / 2, 32, B>(v, lane);
  double r = v[0];
  r += lane_xor<1>(r);
  c = lane >> 1;
  return r;
}

template <typename T, int A, int B>
__global__ void __launch_bounds__(256) k_sweep2(Sweep2Args s) {
  constexpr int NC = 4 * B, P = 256 / NC;         // columns per block (max), threads per column
  constexpr int KM = (NC + P - 1) / P;            // Minv entries per thread
  constexpr bool MREG = KM <= 16;                 // keep the next block's inverse in registers, else in LDS
  // partial loads per batch: 40 where a tile takes at most 32 registers (one batch then
  // covers 80 groups at two threads per column), else 32 (more spends registers the tile needs)
  constexpr int NLMAX = A * B * (int)sizeof(T) / 4 <= 32 ? 40 : 32;
  constexpr int NL = 128 / P > NLMAX ? NLMAX : 128 / P;
  const int K = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int jc = tid % NC, part = tid / NC;
  const int64_t r0 = (int64_t)g * s.RW;
  const int64_t r1 = r0 + s.RW < s.rows ? r0 + s.RW : s.rows;
  const T* F = (const T*)s.F;
  const T* Fp = (const T*)s.Fp;
  __shared__ __attribute__((aligned(16))) double sh_g[kMaxBlock];
  __shared__ double sh_d[kMaxBlock];
  __shared__ double sh_pg[256];
  __shared__ double sh_red[4 * 64 * A];
  __shared__ int32_t sh_cols[2][kMaxBlock];
  __shared__ int sh_abort;
  __shared__ double sh_a[2][kMaxBlock];          // equality-row entries of this block's and the next block's columns
  // blocks of more than 64 columns: the block's inverse (sp x sp, row stride sp), copied
  // into LDS while the group waits for the partials
  __shared__ __attribute__((aligned(16))) double sh_m[MREG ? 2 : NC * NC];
  const double beta = *s.beta_ptr;
  const double mu = s.sc->mu;
  double t = s.sc->t;
  // iterate-independent gradient terms of one column: c - xi + beta (x - z) + h x - mu a
  auto gbase = [&](int col) {
    const double xc = s.x[col];
    double v = s.c[col] - s.xi[col] + beta * (xc - s.z[col]);
    if (s.h) v += s.h[col] * xc;
    if (s.a) v -= mu * s.a[col];
    return v;
  };
  // block solved at position i (its inverse and packed tiles are stored at that index)
  auto bid = [&](int64_t i) -> int64_t { return s.order ? (int64_t)s.order[i] : i; };
  auto bsize = [&](int64_t i) {
    const int64_t b = bid(i);
    return (int)(block_start(b + 1, s.n, s.p) - block_start(b, s.n, s.p));
  };
  // tile of the block at position i: packed copy, else gathered through the block's column indices
  auto fetch = [&](int64_t i, Tile<T, A, B>& tile) {
    if (Fp) load_packed<T, A, B>(Fp, bid(i), K, g, lane, wave, tile);
    else load_tile<T, A, B>(F, s.ldF, r0, r1, sh_cols[i & 1], bsize(i), lane, wave, s.vec, tile);
  };
  double ureg[A];
#pragma unroll
  for (int aa = 0; aa < A; ++aa) {
    const int64_t r = r0 + (int64_t)A * lane + aa;
    ureg[aa] = r < r1 ? s.u[r] : 0.0;
  }
  Tile<T, A, B> ta, tb;
  double mreg[MREG ? KM : 1];
  auto load_minv = [&](int64_t i, int sbi) {
    if constexpr (MREG) {
      const double* Mi = s.Minv + bid(i) * (int64_t)s.sp * s.sp;
#pragma unroll
      for (int e = 0; e < KM; ++e) {   // rows part*KM .. of the inverse's column jc
        const int k = part * KM + e;
        mreg[e] = (jc < sbi && k < sbi) ? Mi[(int64_t)k * s.sp + jc] : 0.0;
      }
    }
  };
  // The whole stored inverse of the block at position i (sp * sp doubles, sp a power of
  // two from 16 to 128, so whole 1 KB runs) goes to LDS through the load-to-LDS path:
  // wavefront w copies runs w, w + 4, ..., lane l bytes [16 l, 16 l + 16) of each.  No
  // registers hold it, so nothing waits for it before the solve (the vector loads
  // issued after it, the partials' polls, return after it).
  auto minv_to_lds = [&](int64_t i) {
    if constexpr (!MREG) {
      const char* src = reinterpret_cast<const char*>(s.Minv + bid(i) * (int64_t)s.sp * s.sp) + 16 * lane;
      const int nrun = s.sp * s.sp / 128;
      for (int r = wave; r < nrun; r += 4)
        __builtin_amdgcn_global_load_lds(src + (int64_t)r * 1024,
                                         (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(sh_m) + r * 1024),
                                         16, 0, 0);
    }
  };
  double ga = 0.0, gbn = 0.0;
  {
    const int sb0 = bsize(0);
    const int64_t c0 = block_start(bid(0), s.n, s.p);
    if (tid < sb0) sh_cols[0][tid] = s.perm[c0 + tid];
    if (tid == 0) sh_abort = 0;
    __syncthreads();
    fetch(0, ta);
    load_minv(0, sb0);
    if (tid < sb0) {
      ga = gbase(sh_cols[0][tid]);
      if (s.a) sh_a[0][tid] = s.a[sh_cols[0][tid]];
    }
  }

  // Exchange of the per-group partials.  Block 0 uses epoch flags: partials
  // complete, then the group's flag, then loads after all flags are raised.
  // From block 1 on the partials themselves are polled: block i uses slot buffer i % 3, slots start as kEmpty (a signalling-NaN
  // pattern that no arithmetic produces), and a reader loads until none is empty.
  // A group empties its slot of block i - 1 once it has seen every group's
  // block-i partial (each group publishes block i only after reading block i - 1),
  // and waits for that store before publishing its next partials, so a reader
  // that has seen a group's block-i partial sees the emptied slot or the new
  // value, never the one from three blocks ago.  The same lane stores a slot's
  // values and empties it.  Block 0's flags order the first emptying of
  // buffers 1 and 2 before any reader.  Waits are bounded: a group that gives up
  // raises wait_abort and leaves, and so do the groups waiting on it.
  constexpr bool SENT = true;
  // the lane that stores a column's partial (and empties its slot), and that
  // column: after the transposed sums, lane l of a 16-lane row holds column l
  // (B = 16) or l / 2 (B = 8) of the row's totals, and lane l holds column
  // l / 2 (B = 32)
  const bool writer = B == 32 ? (lane & 1) == 0 : (B == 16 ? lane < 16 : (lane < 16 && (lane & 1) == 0));
  const int wcol = wave + 4 * (B == 32 ? (lane >> 1) : (B == 16 ? (lane & 15) : ((lane & 15) >> 1)));
  auto block = [&](int64_t i, Tile<T, A, B>& cur, Tile<T, A, B>& nxt, double& gcur, double& gnxt) -> bool {
    const int sb = bsize(i);
    const int32_t* cols = sh_cols[i & 1];
    const bool more = i + 1 < s.p;
    const int64_t s1 = more ? block_start(bid(i + 1), s.n, s.p) : 0;   // first column of the next block
    const int sb1 = more ? bsize(i + 1) : 0;
    if (tid < sb1) sh_cols[(i + 1) & 1][tid] = s.perm[s1 + tid];   // indices of the next block
    // partial F_B'u over this group's rows, transposed across lanes
    double* buf = s.partials + (int64_t)(SENT ? i % 3 : (i & 1)) * K * kMaxBlock;
    const bool poll_data = SENT && i > 0;
    {
      double v[B];
#pragma unroll
      for (int bb = 0; bb < B; ++bb) {
        double acc = 0.0;
#pragma unroll
        for (int aa = 0; aa < A; ++aa) acc += cur.at(aa, bb) * ureg[aa];
        v[bb] = acc;
      }
      int c;
      double tot;
      if constexpr (B <= 16) tot = row_transpose_sum<B>(v, lane, c);
      else tot = transpose_sum<B>(v, lane, c);
      {
        if (SENT && i == 0 && writer) {   // this group's slots of blocks 1 and 2 start empty
          st_coherent(&s.partials[((int64_t)1 * K + g) * kMaxBlock + wcol], kEmpty);
          st_coherent(&s.partials[((int64_t)2 * K + g) * kMaxBlock + wcol], kEmpty);
        }
        if (SENT && i > 0) __builtin_amdgcn_s_waitcnt(0);   // the emptying of this slot is visible first
        if (writer && wcol < sb) st_coherent(&buf[(int64_t)g * kMaxBlock + wcol], tot);
      }
    }
    if (!poll_data) {
      const uint64_t epoch = s.epoch_base + (uint64_t)i + 1;
      __builtin_amdgcn_s_waitcnt(0);   // partial stores complete at device scope; next indices landed
      __syncthreads();
      if (K > 1 && tid == 0)
        __hip_atomic_store(&s.flags[g], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (K > 1 && wave == 0) {
        // every lane checks its flags each round; the wavefront leaves when all are
        // raised, or gives up after max_spin rounds
        for (int tries = 0;; ++tries) {
          bool ok = true;
          for (int q = lane; q < K; q += 64)
            ok &= __hip_atomic_load(&s.flags[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
          if (__all(ok)) break;
          if (tries >= s.max_spin) {
            if (lane == 0) sh_abort = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    __syncthreads();
    // issued after the barrier: a barrier waits for the copy to land (the previous
    // block's solve has finished reading sh_m, barrier at its end)
    minv_to_lds(i);
    // This block's partials first; then the next block's tile and gradient
    // inputs, which stream in during the solve and the update (loads return in
    // order, so nothing below waits for them before the end of the block).
    double rx = 0.0, rc = 0.0, rxi = 0.0, rz = 0.0, rh = 0.0, ra = 0.0;
    {
      double acc = 0.0;
      for (int q = part; q < K; q += NL * P) {
        double v[NL];
        for (int tries = 0;; ++tries) {
          bool ok = true;
#pragma unroll
          for (int e = 0; e < NL; ++e) {
            v[e] = (q + e * P < K && jc < sb) ? ld_coherent(&buf[(int64_t)(q + e * P) * kMaxBlock + jc]) : 0.0;
            ok &= !(poll_data && is_empty(v[e]));
          }
          if (ok) break;
          if (tries >= s.max_spin) { sh_abort = 1; break; }
          __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int e = 0; e < NL; ++e) acc += v[e];
      }
      // the copy of the inverse was issued before the polls, which have all returned:
      // wait for it here, before the next block's loads are issued behind it
      if constexpr (!MREG) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
      fetch(more ? i + 1 : i, nxt);
      if (tid < sb1) {
        const int col = sh_cols[(i + 1) & 1][tid];
        rx = s.x[col]; rc = s.c[col]; rxi = s.xi[col]; rz = s.z[col];
        if (s.h) rh = s.h[col];
        if (s.a) ra = s.a[col];
      }
      sh_pg[part * NC + jc] = acc;
    }
    __syncthreads();
    // a group never published (its flag or its partials): leave, every thread
    // sees the same flag (the loads above stayed in bounds; their values are unused)
    if (sh_abort) {
      if (tid == 0) __hip_atomic_store(&s.sc->wait_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    if (poll_data) {
      // every group has published block i, so none still reads block i - 1: empty our slot of it
      if (writer) st_coherent(&s.partials[((int64_t)((i - 1) % 3) * K + g) * kMaxBlock + wcol], kEmpty);
    }
    if (tid < NC) {   // zero past the block, so the solve needs no masks
      double v = 0.0;
      if (tid < sb) {
        double tot = 0.0;
#pragma unroll
        for (int e = 0; e < P; ++e) tot += sh_pg[e * NC + tid];
        v = tot / s.Ns + gcur;
        if (s.a) v += beta * sh_a[i & 1][tid] * (t - s.b);
      }
      sh_g[tid] = v;
    }
    __syncthreads();
    // step d = -M^{-1} g, P threads per column, combined in order
    {
      double acc = 0.0;
      if constexpr (MREG) {
        // the part's KM consecutive entries of g as 16-byte broadcast reads
        const double* gk = sh_g + part * KM;
        static_assert(KM % 2 == 0, "pairs of g");
#pragma unroll
        for (int e = 0; e < KM; e += 2) {
          const double2 g2 = *reinterpret_cast<const double2*>(gk + e);
          acc += mreg[e] * g2.x;
          acc += mreg[e + 1] * g2.y;
        }
      } else {
        // the part's KM consecutive rows of column jc from the copy in LDS (consecutive
        // threads read consecutive columns); rows past the block are not read
        const int k0 = part * KM;
        const double* mk = sh_m + (int64_t)k0 * s.sp + jc;
        const double* gk = sh_g + k0;
#pragma unroll 8
        for (int e = 0; e < KM; e += 2) {
          const double2 g2 = *reinterpret_cast<const double2*>(gk + e);
          const double m0 = k0 + e < sb ? mk[(int64_t)e * s.sp] : 0.0;
          const double m1 = k0 + e + 1 < sb ? mk[(int64_t)(e + 1) * s.sp] : 0.0;
          acc += m0 * g2.x;
          acc += m1 * g2.y;
        }
      }
      sh_pg[part * NC + jc] = acc;
    }
    __syncthreads();
    if (tid < NC) {
      double tot = 0.0;
#pragma unroll
      for (int e = 0; e < P; ++e) tot += sh_pg[e * NC + tid];
      sh_d[tid] = tid < sb ? -tot : 0.0;
    }
    if (more) load_minv(i + 1, sb1);   // the next inverse arrives during the update below
    __syncthreads();
    if (s.a) {
      const double* ab = sh_a[i & 1];
      double dt = 0.0;
#pragma unroll 8
      for (int j = 0; j < sb; ++j) dt += ab[j] * sh_d[j];
      t += dt;   // every thread forms the same sum in the same order
    }
    if (s.dense) {
      // dense form: the registers hold x of the group's rows; the block's steps land on
      // the rows that are block columns (scattered through LDS, zero elsewhere)
      for (int e = tid; e < 64 * A; e += 256) sh_red[e] = 0.0;
      __syncthreads();
      if (tid < sb) {
        const int col = cols[tid];
        if (col >= r0 && col < r1) sh_red[col - r0] = sh_d[tid];
      }
      __syncthreads();
#pragma unroll
      for (int aa = 0; aa < A; ++aa) ureg[aa] += sh_red[A * lane + aa];
    } else {
      // rows of u from the register tile, summed over the four wavefronts in order
#pragma unroll
      for (int aa = 0; aa < A; ++aa) {
        double v = 0.0;
#pragma unroll
        for (int bb = 0; bb < B; ++bb) v += cur.at(aa, bb) * sh_d[wave + 4 * bb];
        sh_red[wave * 64 * A + 64 * aa + lane] = v;
      }
      __syncthreads();
#pragma unroll
      for (int aa = 0; aa < A; ++aa) {
        const int q = 64 * aa + lane;
        ureg[aa] += ((sh_red[q] + sh_red[64 * A + q]) + sh_red[2 * 64 * A + q]) + sh_red[3 * 64 * A + q];
      }
      if (g == 0 && tid < sb) s.x[cols[tid]] += sh_d[tid];
    }
    // the next block's iterate-independent gradient terms (its columns are untouched by this block)
    if (tid < sb1) {
      double v = rc - rxi + beta * (rx - rz);
      if (s.h) v += rh * rx;
      if (s.a) {
        v -= mu * ra;
        sh_a[(i + 1) & 1][tid] = ra;
      }
      gnxt = v;
    }
    __syncthreads();
    return true;
  };

  for (int64_t i = 0; i < s.p; i += 2) {
    if (!block(i, ta, tb, ga, gbn)) return;
    if (i + 1 < s.p && !block(i + 1, tb, ta, gbn, ga)) return;
  }
#pragma unroll
  for (int aa = 0; aa < A; ++aa) {
    const int64_t r = r0 + (int64_t)A * lane + aa;
    if (r < r1) s.u[r] = ureg[aa];
  }
  if (g == 0 && tid == 0) s.sc->t = t;
}

// A plain launch is used only when the caller has checked that all K groups can
// be resident together (every other kernel that may run beside the sweep
// finishes without waiting on it, so the late groups are always scheduled).
template <typename T, int A, int B>
hipError_t sweep2_launch(const Sweep2Args& a, int K, int coop, hipStream_t st) {
  if (K == 1 || !coop) {
    k_sweep2<T, A, B><<<(unsigned)K, 256, 0, st>>>(a);
    return hipGetLastError();
  }
  Sweep2Args c = a;
  void* args[] = {(void*)&c};
  return hipLaunchCooperativeKernel((const void*)k_sweep2<T, A, B>, dim3((unsigned)K), dim3(256), args, 0, st);
}

template <typename T, int A, int B>
int sweep2_resident() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_sweep2<T, A, B>, 256, 0) != hipSuccess)
    return 0;
  return cus * per;
}

template <typename T>
int sweep2_resident_dispatch(int A, int B) {
#define RAC_SR(AA, BB) if (A == AA && B == BB) return sweep2_resident<T, AA, BB>()
  RAC_SR(1, 8); RAC_SR(2, 8); RAC_SR(4, 8);
  RAC_SR(1, 16); RAC_SR(2, 16);
  RAC_SR(1, 32);
  if constexpr (sizeof(T) < 8) { RAC_SR(4, 16); RAC_SR(2, 32); }
#undef RAC_SR
  return 0;
}

template <typename T>
hipError_t sweep2_dispatch(const Sweep2Args& a, int K, int A, int B, int coop, hipStream_t st) {
#define RAC_SW(AA, BB) if (A == AA && B == BB) return sweep2_launch<T, AA, BB>(a, K, coop, st)
  RAC_SW(1, 8); RAC_SW(2, 8); RAC_SW(4, 8);
  RAC_SW(1, 16); RAC_SW(2, 16);
  RAC_SW(1, 32);
  if constexpr (sizeof(T) < 8) { RAC_SW(4, 16); RAC_SW(2, 32); }
#undef RAC_SW
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t sweep_launch(const SweepArgs& s, hipStream_t st) {
  const T* F = (const T*)s.F;
  const double* beta_ptr = s.beta_ptr;
  int max_spin = s.max_spin >= 0 ? s.max_spin : kMaxSpin;
  void* args[] = {(void*)&F, (void*)&s.ldF, (void*)&s.rows, (void*)&s.n, (void*)&s.p,
                  (void*)&s.perm, (void*)&s.Minv, (void*)&s.sp, (void*)&s.c, (void*)&s.h,
                  (void*)&s.a, (void*)&s.b, (void*)&s.Ns, (void*)&s.x, (void*)&s.z, (void*)&s.xi,
                  (void*)&s.u, (void*)&s.sc, (void*)&beta_ptr, (void*)&s.partials,
                  (void*)&s.flags, (void*)&s.epoch_base, (void*)&max_spin, (void*)&s.order};
  if (s.K == 1) {
    k_sweep<T><<<1, 256, 0, st>>>(F, s.ldF, s.rows, s.n, s.p, s.perm, s.Minv, s.sp, s.c, s.h, s.a,
                                  s.b, s.Ns, s.x, s.z, s.xi, s.u, s.sc, beta_ptr, s.partials,
                                  s.flags, s.epoch_base, max_spin, s.order);
    return hipGetLastError();
  }
  return hipLaunchCooperativeKernel((const void*)k_sweep<T>, dim3((unsigned)s.K), dim3(256), args, 0,
                                    st);
}

}  // namespace

int64_t sweep_rows_per_group(int64_t rows, int K, int A) {
  if (K < 1 || A < 1) return 0;
  int64_t rw = (rows + K - 1) / K;
  rw = (rw + A - 1) / A * A;
  return rw > 64 * A ? 0 : rw;
}

int64_t sweep_packed_elems(int64_t p, int K, int A, int B) { return p * K * 256 * (int64_t)A * B; }

hipError_t launch_sweep(const SweepArgs& s, hipStream_t st) {
  if (s.tileA > 0) {
    Sweep2Args a{s.F, s.ldF, s.rows, s.n, s.p, s.perm, s.Minv, s.sp, s.c, s.h, s.xi, s.z, s.beta_ptr,
                 s.a, s.b, s.Ns, s.x, s.u, s.sc, s.partials, s.flags, s.epoch_base, 0, 0, s.Fp,
                 s.max_spin >= 0 ? s.max_spin : kMaxSpin, s.order, s.dense};
    const int64_t rw = sweep_rows_per_group(s.rows, s.K, s.tileA);
    if (rw == 0) return hipErrorInvalidValue;
    a.RW = rw;
    const int esz = s.dtype == RAC_DT_F64 ? 8 : (s.dtype == RAC_DT_F32 ? 4 : 2);
    a.vec = (s.ldF % s.tileA == 0) && ((uintptr_t)s.F % (size_t)(esz * s.tileA) == 0);
    switch (s.dtype) {
      case RAC_DT_F64: return sweep2_dispatch<double>(a, s.K, s.tileA, s.tileB, s.cooperative, st);
      case RAC_DT_F32: return sweep2_dispatch<float>(a, s.K, s.tileA, s.tileB, s.cooperative, st);
      case RAC_DT_BF16: return sweep2_dispatch<uint16_t>(a, s.K, s.tileA, s.tileB, s.cooperative, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (s.dtype) {
    case RAC_DT_F64: return sweep_launch<double>(s, st);
    case RAC_DT_F32: return sweep_launch<float>(s, st);
    case RAC_DT_BF16: return sweep_launch<uint16_t>(s, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rac

namespace rac {
int sweep_max_resident(int32_t dtype, int A, int B) {
  switch (dtype) {
    case RAC_DT_F64: return sweep2_resident_dispatch<double>(A, B);
    case RAC_DT_F32: return sweep2_resident_dispatch<float>(A, B);
    case RAC_DT_BF16: return sweep2_resident_dispatch<uint16_t>(A, B);
    default: return 0;
  }
}

bool sweep_tile_supported(int32_t dtype, int A, int B) {
  const bool small = dtype != RAC_DT_F64;
  if (B == 8) return A == 1 || A == 2 || A == 4;
  if (B == 16) return A == 1 || A == 2 || (A == 4 && small);
  if (B == 32) return A == 1 || (A == 2 && small);
  return false;
}
}  // namespace rac
