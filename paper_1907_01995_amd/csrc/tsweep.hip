// tsweep.hip -- the batched Gauss-Seidel sweep of Eq.(3) with the lanes of an
// instance advanced together, so that one read of the instance's data serves
// every lane.
//
// Lanes of one instance share its partition, so for block B the products of a
// sweep are, for the group's (up to 16) lanes at once,
//     P = F_B' [u_1 .. u_16]          (gradient partial, block columns x lanes)
//     [u_1 .. u_16] += F_B [d_1 .. d_16]   (residual update)
// -- dense contractions over the rows of F, run on the matrix cores in FP64
// (v_mfma_f64_16x16x4f64: the u vectors and the steps are FP64, so the products
// are as exact as the single-lane FP64 path).
//
// Work split.  A team of W workgroups (W = 16 or 32, per team) processes a list of
// lane groups one after another; for each group, member w owns a contiguous
// slice of the instance's rows and holds u of those rows for all 16 lanes in
// registers for the whole sweep (four wavefronts, 16-row tiles dealt round-robin).  Per block:
//   1. every member computes its partial P over its rows (FP64 MFMA), reduces
//      it over its wavefronts in LDS and publishes it (agent-scope relaxed
//      stores, s_waitcnt, then an epoch flag);
//   2. lane slot L of the group is owned by member L (wavefront 0):
//      the owner waits for all partials, sums them in a fixed order, forms the
//      lane's gradient g_B, applies the lane's block inverse (staged in LDS by
//      all wavefronts at the block's start), updates x_B and t,
//      and publishes the step d (then a second epoch flag);
//   3. every member waits for all steps and updates its rows of u (FP64 MFMA,
//      u as the accumulator).
// Partials and steps are double-buffered by epoch parity.  The flags are
// monotone epochs that persist between launches: every member of a team
// advances its epochs by the same count per launch, so a member's own flag at
// launch start is the team's base.  The host's layout table gives each
// workgroup its team and member index; teams of 16 and 32 workgroups are placed
// within one XCD each (workgroup b runs on XCD b mod 8).
// All members of all teams are resident at once (the grid never exceeds the
// occupancy limit of the device), which every wait relies on.
#include "control.h"
#include "rac_internal.h"

namespace rac {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void st_c(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_c(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_flag(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The calling wavefront waits until flags[0..W) have all reached epoch e.  The
// wait is bounded: after kMaxPolls polls (seconds, against microseconds for a
// real exchange), or as soon as another workgroup has given up, it raises the
// abort flag and returns false; the kernel then leaves at its next barrier.
constexpr uint32_t kMaxPolls = 1u << 21;
__device__ __forceinline__ bool wait_team(const uint32_t* f, int W, uint32_t e, int lane, uint32_t* abort_flag) {
  for (uint32_t poll = 0;; ++poll) {
    const bool ok = lane >= W || (int32_t)(ld_flag(f + lane) - e) >= 0;
    if (__all(ok)) return true;
    if (poll >= kMaxPolls || ld_flag(abort_flag) != 0u) {
      if (lane == 0) st_flag(abort_flag, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

constexpr int NW = 4;          // wavefronts per workgroup (one per SIMD: 512 registers each)
constexpr int DS = 3;          // pipeline stages of the tile loads

// Raw storage of four consecutive elements of a column of F.
template <typename T> struct RawQ;
template <> struct RawQ<uint16_t> { uint2 v; };
template <> struct RawQ<float> { float4 v; };
template <> struct RawQ<double> { double2 a, b; };

__device__ __forceinline__ double to_f64(uint16_t v) { return (double)__uint_as_float(((uint32_t)v) << 16); }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(double v) { return v; }

// Rows o .. o+3 of a column (nvalid of them in range, the rest zero).  vec: the
// four elements are one aligned vector (o a multiple of 4, column base aligned).
template <typename T>
__device__ __forceinline__ RawQ<T> ld_quad(const T* F, int64_t o, int nvalid, bool vec) {
  RawQ<T> r;
  if (vec && nvalid == 4) {
    r = *reinterpret_cast<const RawQ<T>*>(F + o);
  } else {
    T e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = i < nvalid ? F[o + i] : (T)0;
    if constexpr (sizeof(T) == 2) {
      r.v.x = (uint32_t)e[0] | ((uint32_t)e[1] << 16);
      r.v.y = (uint32_t)e[2] | ((uint32_t)e[3] << 16);
    } else if constexpr (sizeof(T) == 4) {
      r.v = make_float4(e[0], e[1], e[2], e[3]);
    } else {
      r.a = make_double2(e[0], e[1]);
      r.b = make_double2(e[2], e[3]);
    }
  }
  return r;
}
// Element i of a quad, converted exactly to FP64.
template <typename T>
__device__ __forceinline__ double quad_at(const RawQ<T>& r, int i) {
  if constexpr (sizeof(T) == 2) {
    const uint32_t wv = i < 2 ? r.v.x : r.v.y;
    return (double)__uint_as_float((i & 1) ? (wv & 0xffff0000u) : (wv << 16));
  } else if constexpr (sizeof(T) == 4) {
    return (double)(i == 0 ? r.v.x : i == 1 ? r.v.y : i == 2 ? r.v.z : r.v.w);
  } else {
    return i == 0 ? r.a.x : i == 1 ? r.a.y : i == 2 ? r.b.x : r.b.y;
  }
}

// Solo groups (a team of one workgroup): the group's instance is small enough
// that one compute unit runs its products at the matrix cores' rate without a
// cross-unit exchange.  The workgroup streams all rows of the block's columns
// and of u (u of the 16 lanes stays in device memory, rows in 16-row tiles
// dealt to the wavefronts round-robin, loads issued several tiles ahead), reduces
// the gradient partials over its wavefronts in LDS, solves the 16 lanes'
// blocks itself, all at once (thread (column, part): a 16-row slice of every
// lane's product with its inverse, the inverses read from device memory a few
// lanes ahead), and applies the update product to u tile by tile.  Tile layouts are those of the team path below; the arithmetic of a
// group depends only on the group (a group is solo or not by its instance's
// row count alone), so every team layout gives the same results.

// Loads through the global address space (the pointers come from descriptor tables, so
// the compiler would otherwise issue flat loads, which also count against lgkmcnt).
template <typename V>
__device__ __forceinline__ V gld(const void* p) {
  return *(const __attribute__((address_space(1))) V*)p;
}
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ RawQ<T> gld_quad(const T* p) {
  RawQ<T> r;
  if constexpr (sizeof(T) == 2) {
    const u32x2_t v = gld<u32x2_t>(p);
    r.v.x = v.x;
    r.v.y = v.y;
  } else if constexpr (sizeof(T) == 4) {
    const f32x4_t v = gld<f32x4_t>(p);
    r.v = make_float4(v.x, v.y, v.z, v.w);
  } else {
    const f64x2_t a = gld<f64x2_t>(p), b = gld<f64x2_t>(p + 2);
    r.a = make_double2(a.x, a.y);
    r.b = make_double2(b.x, b.y);
  }
  return r;
}
// Zeroes the elements i >= nv (nv <= 0: all) of a quad loaded at a clamped address.
// Applied where the quad is consumed, so that its load can stay in flight until then.
template <typename T>
__device__ __forceinline__ RawQ<T> quad_keep(RawQ<T> r, int64_t nv) {
  if constexpr (sizeof(T) == 2) {
    r.v.x &= nv >= 2 ? 0xffffffffu : (nv == 1 ? 0x0000ffffu : 0u);
    r.v.y &= nv >= 4 ? 0xffffffffu : (nv == 3 ? 0x0000ffffu : 0u);
  } else if constexpr (sizeof(T) == 4) {
    r.v.x = nv > 0 ? r.v.x : 0.f;
    r.v.y = nv > 1 ? r.v.y : 0.f;
    r.v.z = nv > 2 ? r.v.z : 0.f;
    r.v.w = nv > 3 ? r.v.w : 0.f;
  } else {
    r.a.x = nv > 0 ? r.a.x : 0.0;
    r.a.y = nv > 1 ? r.a.y : 0.0;
    r.b.x = nv > 2 ? r.b.x : 0.0;
    r.b.y = nv > 3 ? r.b.y : 0.0;
  }
  return r;
}

template <typename T>
__device__ __forceinline__ void solo_group(const BatchArgs& B, const TGroup* G, int t, double (*red)[16][64],
                                           double* lds, int32_t* cols, double* TS, int32_t* SU) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, j = lane & 15;
  const int jc = tid & 63, part = tid >> 6;   // solve layout: column jc, rows 16 part .. 16 part + 15 of M^{-1}
  const int nl = G->nl;
  const BInst I = B.inst[G->inst];
  const T* F = (const T*)I.F;
  const int64_t n = I.n, p = I.p, rows = I.rows, ldF = I.ldF;
  const int ntile = (int)((rows + 15) >> 4);
  const int mine = ntile > wave ? (ntile - wave + NW - 1) / NW : 0;   // this wavefront's tiles
  const int uj = j < nl ? G->lane[j] : -1;
  const bool actj = uj >= 0 && B.sc[uj].status == 0;
  double* Uj = actj ? B.U + B.units[uj].uoff : nullptr;
  const double* Ubase = actj ? Uj : B.U;     // a valid address for the loads of idle slots
  const int64_t rpi = 4 * (j & 3) + (j >> 2);
  const int32_t* pm = B.perm + I.poff + (int64_t)t * n;
  // LDS (lds: 4096 doubles): [64 columns][16 slots] each of
  double* P = lds;                 // gradient partials, then gradients
  double* D = lds + 1024;          // steps
  double* GB = lds + 2048;         // iterate-fixed gradient terms
  // red: the products' partials per wavefront, then the solve's partial products;
  // TS: t = a'x of the 16 slots; SU: the lane of each slot, or -1 when the slot is idle
  __syncthreads();                 // the previous group is done with TS and SU
  if (tid < 16) {
    const int u = tid < nl ? G->lane[tid] : -1;
    const bool act = u >= 0 && B.sc[u].status == 0;
    SU[tid] = act ? u : -1;
    TS[tid] = act ? B.sc[u].t : 0.0;
  }
  __syncthreads();
  const int32_t* su = SU;
  // slots of inverse rows in flight ahead of their use (the first MD issued before the
  // gradient product, which they overlap), and the pipeline stages of the tile loads of the
  // two products (deeper pipelines measured no faster and spill registers)
  constexpr int MD = 4, SDG = 4, SDU = 4;
  for (int64_t blk = 0; blk < p; ++blk) {
    const int64_t s0 = block_start(blk, n, p);
    const int sb = (int)(block_start(blk + 1, n, p) - s0);
    __syncthreads();                       // the previous block is done with cols and the LDS arrays
    if (tid < 64) cols[tid] = tid < sb ? pm[s0 + tid] : pm[s0];
    __syncthreads();
    // the iterate-fixed gradient terms of every (column, slot) and the first MD inverses
    // are issued before the products, which they overlap
    double gbv[4], xcv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int L = 4 * part + e;   // thread: column jc, slots 4 part .. 4 part + 3
      gbv[e] = 0.0;
      xcv[e] = 0.0;
      if (su[L] >= 0 && jc < sb) {
        const BUnit* U = B.units + su[L];
        const int col = cols[jc];
        const double xc = B.X[U->xoff + col];
        double g = U->c[col] - B.XI[U->xoff + col] + B.sc[su[L]].beta * (xc - B.Z[U->xoff + col]);
        if (U->h) g += U->h[col] * xc;
        if (U->a) g -= B.sc[su[L]].mu * U->a[col];
        gbv[e] = g;
        xcv[e] = xc;
      }
    }
    double mreg[MD][16];
    // rows 16 part .. 16 part + 15 of column jc of slot L's inverse, from its stored lower
    // tiles (tile (part, jc / 16) or the transpose of tile (jc / 16, part)); addresses
    // clamped into the block, rows past sb masked where they are used
    auto minv_issue = [&](int L, double (&dst)[16]) {
      const int u = su[L];
      const double* Mo = B.Minv + (u >= 0 ? (B.units[u].moff + blk) * (int64_t)B.sp * B.sp : 0);
      const int jj = jc < B.sp ? jc : B.sp - 1;
      const int pp = 16 * part < B.sp ? part : (B.sp >> 4) - 1;
#pragma unroll
      for (int e = 0; e < 16; ++e) dst[e] = gld<double>(Mo + minv_off(16 * pp + e, jj));
    };
#pragma unroll
    for (int L = 0; L < MD; ++L) minv_issue(L, mreg[L]);
    // 1. P = F_B'[u_1 .. u_16] over all rows
    const T* fcg[4];             // columns 16 ct + j of the block (the first column past sb)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) fcg[ct] = F + (int64_t)cols[16 * ct + j] * ldF;
    f64x4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = (f64x4){0.0, 0.0, 0.0, 0.0};
    {
      RawQ<T> gq[SDG][4];
      double uv[SDG][4];
      // tile loads without branches: every address is clamped into the columns (rows past
      // the end and tiles past the wavefront's last read the column's last aligned quad, u
      // its last row), and the rows past the end are zeroed where the quad is consumed, so
      // that SDG - 1 tiles of loads stay in flight together
      auto gload = [&](int sidx, RawQ<T> (&dst)[4], double (&ud)[4]) {
        const int64_t r0 = 16 * (int64_t)(wave + NW * sidx) + 4 * q;
        const int64_t rc = r0 < ldF - 4 ? r0 : ldF - 4;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) dst[ct] = gld_quad<T>(fcg[ct] + rc);
#pragma unroll
        for (int i = 0; i < 4; ++i) ud[i] = gld<double>(Ubase + (r0 + i < rows ? r0 + i : rows - 1));
      };
#pragma unroll
      for (int sidx = 0; sidx < SDG - 1; ++sidx) gload(sidx, gq[sidx], uv[sidx]);
      for (int base = 0; base < mine; base += SDG) {
#pragma unroll
        for (int k = 0; k < SDG; ++k) {
          const int sidx = base + k;
          gload(sidx + SDG - 1, gq[(k + SDG - 1) % SDG], uv[(k + SDG - 1) % SDG]);
          // rows past the end (all rows of tiles past the wavefront's last) count zero; the
          // products of consecutive steps are independent
          const int64_t nv = rows - (16 * (int64_t)(wave + NW * sidx) + 4 * q);
          RawQ<T> fq[4];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) fq[ct] = quad_keep<T>(gq[k][ct], nv);
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
              acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(quad_at<T>(fq[ct], i), uv[k][i], acc[ct], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // acc[ct][r] of lane (q, j) = P[column 16 ct + 4 r + q][slot j]; summed over the wavefronts in order
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][4 * ct + r][lane] = acc[ct][r];
#pragma unroll
    for (int e = 0; e < 4; ++e) GB[jc * 16 + 4 * part + e] = gbv[e];
    __syncthreads();
    // 2. the gradients of the 16 slots: partials summed over the wavefronts in order, then
    //    scaled and completed with the iterate-fixed terms (the slot of a thread is tid mod 16)
    {
      const int sl = tid & 15, u = su[sl];
      double ns = 1.0, beta = 0.0, bb = 0.0;
      const double* av = nullptr;
      if (u >= 0) {
        const BUnit* U = B.units + u;
        ns = U->Ns;
        av = U->a;
        bb = U->b;
        beta = B.sc[u].beta;
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int e = tid + 256 * rr, el = e >> 6, ln = e & 63;
        const double v = ((red[0][el][ln] + red[1][el][ln]) + red[2][el][ln]) + red[3][el][ln];
        const int col = 16 * (el >> 2) + 4 * (el & 3) + (ln >> 4);
        double g = 0.0;
        if (u >= 0 && col < sb) {
          g = v / ns + GB[col * 16 + sl];
          if (av) g += beta * av[cols[col]] * (TS[sl] - bb);
        }
        P[col * 16 + sl] = g;
      }
    }
    __syncthreads();
    // 3. d = -M^{-1} g of the 16 slots at once: thread (jc, part) forms the 16-row slice
    //    part of every slot's product for column jc, the inverses MD slots ahead; the
    //    slices of a column are added in order
    double* PG = &red[0][0][0];   // [16 slots][4 parts][64 columns]
#pragma unroll
    for (int L = 0; L < 16; ++L) {
      double a2 = 0.0;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const double m = 16 * part + e < sb ? mreg[L % MD][e] : 0.0;
        a2 += m * P[(16 * part + e) * 16 + L];
      }
      PG[(L * 4 + part) * 64 + jc] = a2;
      if (L + MD < 16) minv_issue(L + MD, mreg[L % MD]);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int L = 4 * part + e, u = su[L];   // u is the same over the wavefront
      double d = 0.0;
      if (u >= 0 && jc < sb) {
        const double* pg = PG + L * 256 + jc;
        d = -(((pg[0] + pg[64]) + pg[128]) + pg[192]);
      }
      D[jc * 16 + L] = d;
      if (u >= 0) {
        const BUnit* U = B.units + u;
        if (jc < sb) B.X[U->xoff + cols[jc]] = xcv[e] + d;
        if (U->a) {
          const double dt = wave_sum(jc < sb ? U->a[cols[jc]] * d : 0.0);
          if (jc == 0) TS[L] += dt;
        }
      }
    }
    __syncthreads();
    // 4. [u_1 .. u_16] += F_B [d_1 .. d_16], tile by tile
    {
      double dreg[16];             // d of columns 4 m + q (zero past sb and for idle slots)
#pragma unroll
      for (int m = 0; m < 16; ++m) dreg[m] = actj ? D[(4 * m + q) * 16 + j] : 0.0;
      const T* fcu[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) fcu[m] = F + (int64_t)cols[4 * m + q] * ldF;
      T uq[SDU][16];
      double uv[SDU][4];
      // clamped loads again: a row past the end reads the column's last row and is not
      // stored; columns past the block read the block's first column, times d = 0
      auto uload = [&](int sidx, T (&dst)[16], double (&ud)[4]) {
        const int64_t rr = 16 * (int64_t)(wave + NW * sidx) + rpi;
        const int64_t rrc = rr < rows ? rr : rows - 1;
#pragma unroll
        for (int m = 0; m < 16; ++m) dst[m] = gld<T>(fcu[m] + rrc);
        const int64_t r0 = 16 * (int64_t)(wave + NW * sidx) + 4 * q;
#pragma unroll
        for (int i = 0; i < 4; ++i) ud[i] = gld<double>(Ubase + (r0 + i < rows ? r0 + i : rows - 1));
      };
#pragma unroll
      for (int sidx = 0; sidx < SDU - 1; ++sidx) uload(sidx, uq[sidx], uv[sidx]);
      for (int base = 0; base < mine; base += SDU) {
#pragma unroll
        for (int k = 0; k < SDU; ++k) {
          const int sidx = base + k;
          uload(sidx + SDU - 1, uq[(k + SDU - 1) % SDU], uv[(k + SDU - 1) % SDU]);
          {   // four independent accumulator chains (columns m mod 4), added in order
            f64x4 ac[4] = {{uv[k][0], uv[k][1], uv[k][2], uv[k][3]}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0},
                           {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
            for (int m = 0; m < 16; ++m)
              ac[m & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(to_f64(uq[k][m]), dreg[m], ac[m & 3], 0, 0, 0);
            const f64x4 a4 = (ac[0] + ac[1]) + (ac[2] + ac[3]);
            const int64_t r0 = 16 * (int64_t)(wave + NW * sidx) + 4 * q;
#pragma unroll
            for (int i = 0; i < 4; ++i)   // per-lane predicated stores (rows past the end, idle slots)
              if (actj && sidx < mine && r0 + i < rows) Uj[r0 + i] = a4[i];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }
  __syncthreads();
  if (tid < 16 && su[tid] >= 0 && B.units[su[tid]].a) B.sc[su[tid]].t = TS[tid];
}

// Register layout (wavefront v, lane = 16 q + j): tile = v + NW s covers rows
// rb + 16 tile .. +15; ur[s][i] holds u[rb + 16 tile + 4 q + i] of lane slot j.
// That is the B operand of the gradient product (k = q, n = j) and, with the
// update product's row order pi(m) = 4 (m mod 4) + m div 4, exactly its
// accumulator layout (row 4 r + q of the output is physical row 4 q + r).
// Both products stream the member's tiles with the next tile's loads issued
// DS-1 tiles ahead of the current tile's matrix-core work (fenced so that the
// compiler does not hoist further loads and run out of registers).
template <typename T, int NT>
__global__ void __launch_bounds__(NW * 64) k_tsweep(BatchArgs B, TeamArgs TA, int t) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, j = lane & 15;
  const int team = TA.blk_team[blockIdx.x];
  if (team < 0) return;                      // idle workgroup of the layout (no barrier reached)
  const int w = TA.blk_member[blockIdx.x];
  const int W = TA.team_w[team];
  uint32_t* fl_part = TA.flags + (int64_t)team * 128;
  uint32_t* fl_step = fl_part + 64;
  double* part = TA.part + TA.team_part[team];
  double* delta = TA.delta + (int64_t)team * 2 * 1024;
  uint32_t e = ld_flag(fl_part + w);
  // Two-byte data: the member's rows of the block's columns are staged in LDS
  // (column-major, stride SL elements: 32 bytes past a multiple of 128, so the
  // update product's four-column reads fall in distinct banks) with coalesced
  // 16-byte loads, all in flight at once; both products then read LDS.
  constexpr bool kSlice = sizeof(T) == 2;
  constexpr int SL = 64 * NT + 16;
  __shared__ __attribute__((aligned(16))) uint16_t slice[kSlice ? 64 * SL : 8];
  __shared__ double minv_lds[64 * 65];      // block inverse of the owned lane (row stride 65)
  __shared__ double red[NW][16][64];
  __shared__ double shg[NW][64];
  __shared__ int32_t colsb[2][64];           // column indices of this block and the next
  __shared__ int32_t give_up;
  __shared__ double solo_ts[16];
  __shared__ int32_t solo_su[16];
  if (tid == 0) give_up = 0;
  const int g0 = TA.team_off[team], g1 = TA.team_off[team + 1];
  if (W == 1) {   // a solo worker: its groups one after another, no exchange
    for (int gi = g0; gi < g1; ++gi) {
      const TGroup* G = TA.groups + TA.team_list[gi];
      bool any = false;
      for (int L = 0; L < G->nl; ++L) any |= B.sc[G->lane[L]].status == 0;
      if (any) solo_group<T>(B, G, t, red, minv_lds, colsb[0], solo_ts, solo_su);
    }
    return;
  }
  for (int gi = g0; gi < g1; ++gi) {
    const TGroup* G = TA.groups + TA.team_list[gi];
    const int nl = G->nl;
    bool any = false;
    for (int L = 0; L < nl; ++L) any |= B.sc[G->lane[L]].status == 0;
    if (!any) continue;                      // same decision in every member
    const BInst I = B.inst[G->inst];
    const T* F = (const T*)I.F;
    const int64_t n = I.n, p = I.p, rows = I.rows, ldF = I.ldF;
    const bool vec = G->vec4 != 0;
    const int64_t rb = w == 0 ? 0 : ((rows * w / W) & ~(int64_t)15);
    const int64_t re = w + 1 == W ? rows : ((rows * (w + 1) / W) & ~(int64_t)15);
    const int ntile = re > rb ? (int)((re - rb + 15) >> 4) : 0;
    const int uj = j < nl ? G->lane[j] : -1;
    const bool actj = uj >= 0 && B.sc[uj].status == 0;
    double* Uj = actj ? B.U + B.units[uj].uoff : nullptr;
    double ur[NT][4];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int tile = wave + NW * s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = rb + 16 * tile + 4 * q + i;
        ur[s][i] = (actj && tile < ntile && r < re) ? Uj[r] : 0.0;
      }
    }
    // member w owns lane slot L = w (W >= 16, so every slot has one owner); the
    // owner's wavefront 0 forms the slot's step, and `own` is the same in all of
    // the member's wavefronts (they stage the slot's block inverses)
    const int L = w;
    const int ou = L < nl ? G->lane[L] : -1;
    const bool own = ou >= 0 && B.sc[ou].status == 0;
    const BUnit* OU = own ? B.units + ou : nullptr;
    double obeta = 0.0, omu = 0.0, ot = 0.0, oNs = 1.0, ob = 0.0;
    if (own) {
      obeta = B.sc[ou].beta; omu = B.sc[ou].mu; ot = B.sc[ou].t; oNs = OU->Ns; ob = OU->b;
    }
    // the owned lane's descriptor and the group's layout flag, read once: read in the block
    // loop they would be loads whose waits also wait for the staging loads issued before
    const int64_t omoff = own ? OU->moff : 0, oxoff = own ? OU->xoff : 0;
    const double* oc = own ? OU->c : nullptr;
    const double* oh = own ? OU->h : nullptr;
    const double* oa = own ? OU->a : nullptr;
    const bool vec8 = G->vec8 != 0;
    const int32_t* pm = B.perm + I.poff + (int64_t)t * n;
    const int64_t rpi = 4 * (j & 3) + (j >> 2);       // row pi(j) of a tile in the update product
    // Block inverse of the owned lane (slot w), staged in LDS at the start of each block
    // together with the slice.  Thread tid takes entries (k, c) = (tid / 64 + 4 i,
    // tid % 64): those of the stored lower tiles are loaded (whole tile rows, coalesced)
    // and written to LDS at (k, c) and, below the diagonal tiles, at (c, k); the lanes of
    // upper tiles load their row of the diagonal tile instead (same lines) and store
    // nothing.  Row stride 65: the mirrored stores do not share banks.
    double pf[16];
    auto minv_load = [&](int64_t bk) {
      const int sbk = (int)(block_start(bk + 1, n, p) - block_start(bk, n, p));
      const double* Mo = own ? B.Minv + (omoff + bk) * (int64_t)B.sp * B.sp : nullptr;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int k = (tid >> 6) + 4 * i, c = tid & 63, I = i >> 2;
        const int cl = (c >> 4) <= I ? c : 16 * I + (c & 15);
        const int kk = k < B.sp ? k : B.sp - 1, cc = cl < B.sp ? cl : B.sp - 1;   // inside the block
        const double v = Mo ? Mo[minv_off(kk, cc)] : 0.0;
        pf[i] = (k < sbk && c < sbk) ? v : 0.0;
      }
    };
    auto minv_store = [&]() {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int k = (tid >> 6) + 4 * i, c = tid & 63, I = i >> 2, J = c >> 4;
        if (J <= I) minv_lds[k * 65 + c] = pf[i];
        if (J < I) minv_lds[c * 65 + k] = pf[i];
      }
    };
    // Two-byte data: the slice of a block is fetched into registers (chunk k of
    // column c = slice rows [8k, 8k + 8); rows past the member's range up to the
    // last tile are zero), all loads in flight at once, then stored to LDS.
    constexpr int PER = kSlice ? 2 * NT : 1;   // chunks per thread: a column has up to 8 NT chunks, 4 threads
    const int nr = (int)(re - rb), cpc = 2 * ntile;
    // Thread tid stages column c = tid / 4 of the slice: chunks sub + 4 i
    // (sub = tid % 4, i < PER; chunk k = slice rows [8k, 8k + 8)), so a thread
    // needs one base address and the loads of four neighbouring threads cover
    // 64 contiguous bytes.  Every load is in range: a column past the block's
    // width re-reads the block's first column and a chunk past the member's
    // rows re-reads its last chunk; both store zeros instead, so the slice is
    // zero outside the block's columns and the member's rows and the products
    // read it without masks.
    auto slice_load = [&](const int32_t* ccols, int sbk) {
      const int c = tid >> 2, sub = tid & 3;
      const bool cv = c < sbk;
      const int lastk = (nr - 1) >> 3;       // last chunk holding member rows (nr >= 1 when ntile >= 1)
      if (vec8) {
        // 16-byte aligned columns (ldF a multiple of 8): a chunk crossing the
        // member's last row reads at most 7 further elements of the same padded
        // column, zeroed in LDS below
        const uint16_t* base = (const uint16_t*)F + (int64_t)ccols[cv ? c : 0] * ldF + rb;
        uint4 sv[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          const int k = sub + 4 * i;
          sv[i] = *reinterpret_cast<const uint4*>(base + 8 * (k <= lastk ? k : lastk));
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {       // columns past the block's width are zeroed too
          const int k = sub + 4 * i;
          if (k < cpc)
            *reinterpret_cast<uint4*>(&slice[c * SL + 8 * k]) = (cv && k <= lastk) ? sv[i] : make_uint4(0u, 0u, 0u, 0u);
        }
        if (nr & 7) {
          __syncthreads();
          if (tid < sbk)
            for (int r = nr; r < ((nr + 7) & ~7); ++r) slice[tid * SL + r] = 0;
        }
      } else {                                // element loads (unaligned columns)
        const uint16_t* base = (const uint16_t*)F + (int64_t)ccols[cv ? c : 0] * ldF + rb;
        for (int i = 0; i < PER; ++i) {
          const int k = sub + 4 * i;
          if (k < cpc) {
            uint32_t h[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) h[e] = (cv && 8 * k + e < nr) ? (uint32_t)base[8 * k + e] : 0u;
            *reinterpret_cast<uint4*>(&slice[c * SL + 8 * k]) =
                make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
          }
        }
      }
    };
    {
      const int sb0 = (int)block_start(1, n, p);
      __syncthreads();                       // the previous group's last block is done with colsb
      if (tid < sb0) colsb[0][tid] = pm[tid];
    }
    for (int64_t blk = 0; blk < p; ++blk) {
      const int64_t s0 = block_start(blk, n, p);
      const int sb = (int)(block_start(blk + 1, n, p) - s0);
      const int32_t* cols = colsb[blk & 1];
      const int sbn = blk + 1 < p ? (int)(block_start(blk + 2, n, p) - block_start(blk + 1, n, p)) : 0;
      __syncthreads();                       // this block's cols and inverse are in LDS; the
      if (give_up) return;                   // previous block no longer reads the slice
      minv_load(blk);                        // in flight together with the slice
      if constexpr (kSlice) if (ntile > 0) slice_load(cols, sb);   // all of the slice's loads in flight at once
      minv_store();
      // the next block's indices: loaded after the staging loads, whose completion their
      // wait then shares
      if (tid < sbn) colsb[(blk + 1) & 1][tid] = pm[s0 + sb + tid];
      __syncthreads();
      ++e;
      const int par = (int)(e & 1u);
      // owner: iterate-fixed gradient terms of the lane
      double gb = 0.0, acol = 0.0, oxc = 0.0, odel = 0.0;
      if (own && lane < sb) {
        const int col = cols[lane];
        const double xc = B.X[oxoff + col];
        oxc = xc;
        gb = oc[col] - B.XI[oxoff + col] + obeta * (xc - B.Z[oxoff + col]);
        if (oh) gb += oh[col] * xc;
        if (oa) { acol = oa[col]; gb -= omu * acol; }
      }
      // 1. partial F_B' u over this member's rows, all lanes of the group
      {
        f64x4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = (f64x4){0.0, 0.0, 0.0, 0.0};
        if constexpr (kSlice) {
#pragma unroll
          for (int s = 0; s < NT; ++s) {
            const int tile = wave + NW * s;
            if (tile < ntile) {
#pragma unroll
              for (int ct = 0; ct < 4; ++ct) {
                const int c = 16 * ct + j;
                const uint2 r = *reinterpret_cast<const uint2*>(&slice[c * SL + 16 * tile + 4 * q]);
                const double f[4] = {(double)__uint_as_float(r.x << 16), (double)__uint_as_float(r.x & 0xffff0000u),
                                     (double)__uint_as_float(r.y << 16), (double)__uint_as_float(r.y & 0xffff0000u)};
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[i], ur[s][i], acc[ct], 0, 0, 0);
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        } else {
        RawQ<T> gq[DS][4];
        auto gload = [&](int s, RawQ<T> (&dst)[4]) {
          const int tile = wave + NW * s;
          const int64_t r0 = rb + 16 * tile + 4 * q;
          const int nv = tile >= ntile ? 0 : (re - r0 >= 4 ? 4 : (re > r0 ? (int)(re - r0) : 0));
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const int c = 16 * ct + j;
            const bool cv = c < sb && nv > 0;
            dst[ct] = ld_quad<T>(F, cv ? (int64_t)cols[c] * ldF + r0 : 0, cv ? nv : 0, vec);
          }
        };
#pragma unroll
        for (int s = 0; s < DS - 1 && s < NT; ++s) gload(s, gq[s]);
#pragma unroll
        for (int s = 0; s < NT; ++s) {
          if (s + DS - 1 < NT) gload(s + DS - 1, gq[(s + DS - 1) % DS]);
          if (wave + NW * s < ntile) {
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
              for (int i = 0; i < 4; ++i)
                acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(quad_at<T>(gq[s % DS][ct], i), ur[s][i],
                                                               acc[ct], 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        }
        // acc[ct][r] of lane (q, j) = P[column 16 ct + 4 r + q][slot j]
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[wave][4 * ct + r][lane] = acc[ct][r];
      }
      __syncthreads();
      {
        const int ln = tid & 63, qq = ln >> 4, jj = ln & 15;
        double* dst = part + (int64_t)par * 16 * W * 64;   // [slot][member][column]
#pragma unroll
        for (int rr = 0; rr < 16 / NW; ++rr) {
          const int el = (16 / NW) * (tid >> 6) + rr;          // = 4 ct + r
          double v = 0.0;
#pragma unroll
          for (int vv = 0; vv < NW; ++vv) v += red[vv][el][ln];
          const int col = 16 * (el >> 2) + 4 * (el & 3) + qq;
          st_c(dst + ((int64_t)jj * W + w) * 64 + col, v);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);         // partial stores complete at device scope
      __syncthreads();
      if (tid == 0) st_flag(fl_part + w, e);
      // 2. owners: full gradient (fixed member order), step, x_B, t
      if (own && wave == 0) {
        if (!wait_team(fl_part, W, e, lane, TA.abort_flag) && lane == 0) give_up = 1;
        double s = 0.0;
        if (lane < sb) {
          const double* pp = part + ((int64_t)par * 16 + L) * W * 64 + lane;   // member m at + 64 m
          double v[32];
#pragma unroll
          for (int m = 0; m < 32; ++m) v[m] = ld_c(pp + (int64_t)(m < W ? m : 0) * 64);
#pragma unroll
          for (int m = 0; m < 32; ++m) v[m] = m < W ? v[m] : 0.0;
#pragma unroll
          for (int m = 0; m < 32; ++m) s += v[m];
        }
        double g = s / oNs + gb;
        if (oa) g += obeta * acol * (ot - ob);
        shg[wave][lane] = lane < sb ? g : 0.0;
        __builtin_amdgcn_wave_barrier();
        const double* Ml = minv_lds;
        double dq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
        for (int k = 0; k < 64; ++k) dq[k & 3] += Ml[k * 65 + lane] * shg[wave][k];
        odel = lane < sb ? -((dq[0] + dq[1]) + (dq[2] + dq[3])) : 0.0;
        if (oa) ot += wave_sum(acol * odel);
        st_c(delta + ((int64_t)par * 64 + lane) * 16 + L, odel);   // [column][slot]
        __builtin_amdgcn_s_waitcnt(0);
      }
      __syncthreads();
      if (give_up) return;
      if (tid == 0) st_flag(fl_step + w, e);
      if (own && wave == 0 && lane < sb) B.X[oxoff + cols[lane]] = oxc + odel;   // only the owner writes x_B
      // 3. every member: steps of all lanes, then its rows of u
      if (!wait_team(fl_step, W, e, lane, TA.abort_flag) && lane == 0) give_up = 1;
      {
        double dreg[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) dreg[m] = ld_c(delta + ((int64_t)par * 64 + 4 * m + q) * 16 + j);
#pragma unroll
        for (int m = 0; m < 16; ++m) dreg[m] = actj ? dreg[m] : 0.0;   // slots without an active lane
        if constexpr (kSlice) {
          // two accumulator chains per tile (even and odd column groups), added at the end
#pragma unroll
          for (int s = 0; s < NT; ++s) {
            const int tile = wave + NW * s;
            if (tile < ntile) {
              f64x4 a0 = {ur[s][0], ur[s][1], ur[s][2], ur[s][3]};
              f64x4 a1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int m = 0; m < 16; m += 2) {
                const int c0 = 4 * m + q, c1 = c0 + 4;
                const uint32_t h0 = slice[c0 * SL + 16 * tile + rpi];
                const uint32_t h1 = slice[c1 * SL + 16 * tile + rpi];
                a0 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)__uint_as_float(h0 << 16), dreg[m], a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)__uint_as_float(h1 << 16), dreg[m + 1], a1, 0, 0, 0);
              }
              ur[s][0] = a0[0] + a1[0]; ur[s][1] = a0[1] + a1[1]; ur[s][2] = a0[2] + a1[2]; ur[s][3] = a0[3] + a1[3];
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        } else {
        T uq[DS][16];
        auto uload = [&](int s, T (&dst)[16]) {
          const int tile = wave + NW * s;
          const int64_t rr = rb + 16 * tile + rpi;
          const bool rv = tile < ntile && rr < re;
#pragma unroll
          for (int m = 0; m < 16; ++m) {
            const int c = 4 * m + q;
            dst[m] = (rv && c < sb) ? F[(int64_t)cols[c] * ldF + rr] : (T)0;
          }
        };
#pragma unroll
        for (int s = 0; s < DS - 1 && s < NT; ++s) uload(s, uq[s]);
#pragma unroll
        for (int s = 0; s < NT; ++s) {
          if (s + DS - 1 < NT) uload(s + DS - 1, uq[(s + DS - 1) % DS]);
          if (wave + NW * s < ntile) {
            f64x4 a4 = {ur[s][0], ur[s][1], ur[s][2], ur[s][3]};
#pragma unroll
            for (int m = 0; m < 16; ++m)
              a4 = __builtin_amdgcn_mfma_f64_16x16x4f64(to_f64(uq[s % DS][m]), dreg[m], a4, 0, 0, 0);
            ur[s][0] = a4[0]; ur[s][1] = a4[1]; ur[s][2] = a4[2]; ur[s][3] = a4[3];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        }
      }
    }
    // the group's u back to memory, and t of the owned lane
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int tile = wave + NW * s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = rb + 16 * tile + 4 * q + i;
        if (actj && tile < ntile && r < re) Uj[r] = ur[s][i];
      }
    }
    if (own && wave == 0 && lane == 0 && oa) B.sc[ou].t = ot;   // wavefront 0 carried t
  }
}

// ---------------------------------------------------------------------------
// KKT terms of a lane group: one workgroup per (group, pair of 64-column chunks).
// P = F_pair' [u_1 .. u_16] over all rows on the matrix cores (one read of the
// data for the whole group, and of u for two chunks; wavefront v takes tiles v,
// v+4, ...), then, chunk by chunk, the per-column terms of every active lane and
// their maxima / sums over the chunk, written where the per-lane control kernel
// reads them (kpart[lane][chunk][10]).
template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_gkkt(BatchArgs B, const TGroup* __restrict__ groups,
                                              const int2* __restrict__ tasks) {
  constexpr int NCT = 8;                     // 16-column tiles of the pair
  const int2 tk = tasks[blockIdx.x];
  if (tk.x < 0) return;                      // an empty task (keeps the others on their XCDs)
  const TGroup* G = groups + tk.x;
  const int pair = tk.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, j = lane & 15;
  const int nl = G->nl;
  bool any = false;
  for (int L = 0; L < nl; ++L) any |= B.sc[G->lane[L]].status == 0;
  if (!any) return;                          // uniform: the workgroup leaves together
  const BInst I = B.inst[G->inst];
  const T* F = (const T*)I.F;
  const int64_t rows = I.rows, ldF = I.ldF, c0 = 128 * (int64_t)pair;
  const int nc = I.n - c0 < 128 ? (int)(I.n - c0) : 128;   // columns of the pair
  const bool vec = G->vec4 != 0;
  const int uj = j < nl ? G->lane[j] : -1;
  const bool actj = uj >= 0 && B.sc[uj].status == 0;
  const double* Uj = B.U + (actj ? B.units[uj].uoff : 0);
  f64x4 acc[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) acc[ct] = (f64x4){0.0, 0.0, 0.0, 0.0};
  const int64_t ntile = (rows + 15) >> 4;
  if (G->span) {
    // branch-free tile loads, KD - 1 tiles in flight per wavefront: addresses clamped
    // into the columns (rows past the end and tiles past the wavefront's last read the
    // column's last aligned quad, u its last row; columns past the pair read its last
    // column, whose products are not used) and rows past the end zeroed where consumed
    constexpr int KD = 2;
    const int mine = ntile > wave ? (int)((ntile - wave + 3) / 4) : 0;
    const T* fcg[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) fcg[ct] = F + (c0 + (16 * ct + j < nc ? 16 * ct + j : nc - 1)) * ldF;
    const double* Ubase = actj ? Uj : B.U;
    RawQ<T> gq[KD][NCT];
    double uv[KD][4];
    auto gload = [&](int sidx, RawQ<T> (&dst)[NCT], double (&ud)[4]) {
      const int64_t r0 = 16 * (int64_t)(wave + 4 * sidx) + 4 * q;
      const int64_t rc = r0 < ldF - 4 ? r0 : ldF - 4;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) dst[ct] = gld_quad<T>(fcg[ct] + rc);
#pragma unroll
      for (int i = 0; i < 4; ++i) ud[i] = gld<double>(Ubase + (r0 + i < rows ? r0 + i : rows - 1));
    };
#pragma unroll
    for (int sidx = 0; sidx < KD - 1; ++sidx) gload(sidx, gq[sidx], uv[sidx]);
    for (int base = 0; base < mine; base += KD) {
#pragma unroll
      for (int k = 0; k < KD; ++k) {
        const int sidx = base + k;
        gload(sidx + KD - 1, gq[(k + KD - 1) % KD], uv[(k + KD - 1) % KD]);
        const int64_t nv = rows - (16 * (int64_t)(wave + 4 * sidx) + 4 * q);
        double ux[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ux[i] = actj && i < nv ? uv[k][i] : 0.0;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const RawQ<T> fq = quad_keep<T>(gq[k][ct], nv);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(quad_at<T>(fq, i), ux[i], acc[ct], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else
  for (int64_t tile = wave; tile < ntile; tile += 4) {
    const int64_t r0 = 16 * tile + 4 * q;
    const int nv = rows - r0 >= 4 ? 4 : (rows > r0 ? (int)(rows - r0) : 0);
    double uv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) uv[i] = Uj[actj && i < nv ? r0 + i : 0];
#pragma unroll
    for (int i = 0; i < 4; ++i) uv[i] = (actj && i < nv) ? uv[i] : 0.0;
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int c = 16 * ct + j;
      const bool cv = c < nc && nv > 0;
      const RawQ<T> f = ld_quad<T>(F, cv ? (c0 + c) * ldF + r0 : 0, cv ? nv : 0, vec);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(quad_at<T>(f, i), uv[i], acc[ct], 0, 0, 0);
    }
  }
  __shared__ double red[4][16][64];
  __shared__ double mred[16][16][10];
  // thread tid: slot tid & 15, columns 16 (tid >> 6) + 4 rr + ((tid & 63) >> 4), rr < 4
  const int slot = tid & 15, ln = tid & 63;
  const int us = slot < nl ? G->lane[slot] : -1;
  const bool acts = us >= 0 && B.sc[us].status == 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {              // the pair's chunks, one after the other
    const int chunk = 2 * pair + h, nch = nc - 64 * h;
    if (nch <= 0) break;                       // uniform
    if (h > 0) __syncthreads();                // the previous chunk's reads of red and mred are done
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][4 * ct + r][lane] = acc[4 * h + ct][r];
    __syncthreads();
    double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (acts) {
      const BUnit* D = B.units + us;
      const double mu = B.sc[us].mu;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int el = 4 * (tid >> 6) + rr;
        const int cl = 16 * (el >> 2) + 4 * (el & 3) + (ln >> 4);
        if (cl < nch) {
          const double v = red[0][el][ln] + red[1][el][ln] + red[2][el][ln] + red[3][el][ln];
          const int64_t col = c0 + 64 * h + cl;
          kkt_column_terms(v, D->Ns, D->h ? D->h[col] : 0.0, D->c[col], D->a ? D->a[col] : 0.0,
                           B.X[D->xoff + col], B.Z[D->xoff + col], B.XI[D->xoff + col], mu, D->prox, D->lam,
                           D->alpha, D->lo, D->hi, m);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 10; ++e) mred[slot][tid >> 4][e] = m[e];
    __syncthreads();
    if (tid < 16 && tid < nl) {
      const int u = G->lane[tid];
      if (B.sc[u].status == 0) {
        double* outp = B.kpart + ((int64_t)u * B.KC + chunk) * 10;
#pragma unroll
        for (int e = 0; e < 10; ++e) {
          double v = mred[tid][0][e];
          for (int k = 1; k < 16; ++k) v = e < 9 ? fmax(v, mred[tid][k][e]) : v + mred[tid][k][e];
          outp[e] = v;
        }
      }
    }
  }
}

template <typename T, int NT>
int tsweep_resident_t() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_tsweep<T, NT>, NW * 64, 0) != hipSuccess)
    return 0;
  return cus * per;
}

template <typename T>
int tsweep_resident_nt(int NT) {
  switch (NT) {
    case 8: return tsweep_resident_t<T, 8>();
    case 10:   // ten tiles (640 rows) fit LDS and the register file only with two-byte data
      if constexpr (sizeof(T) == 2) return tsweep_resident_t<T, 10>();
      return 0;
    default: return 0;
  }
}

template <typename T, int NT>
hipError_t tsweep_go(const BatchArgs& b, const TeamArgs& ta, int t, hipStream_t st) {
  k_tsweep<T, NT><<<(unsigned)ta.nblocks, NW * 64, 0, st>>>(b, ta, t);
  return hipGetLastError();
}

template <typename T>
hipError_t tsweep_launch(const BatchArgs& b, const TeamArgs& ta, int t, hipStream_t st) {
  switch (ta.NT) {
    case 8: return tsweep_go<T, 8>(b, ta, t, st);
    case 10:
      if constexpr (sizeof(T) == 2) return tsweep_go<T, 10>(b, ta, t, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_gkkt(const BatchArgs& b, const TGroup* groups, const int2* tasks, int ntasks, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  switch (b.dtype) {
    case RAC_DT_F64: k_gkkt<double><<<(unsigned)ntasks, 256, 0, st>>>(b, groups, tasks); break;
    case RAC_DT_F32: k_gkkt<float><<<(unsigned)ntasks, 256, 0, st>>>(b, groups, tasks); break;
    case RAC_DT_BF16: k_gkkt<uint16_t><<<(unsigned)ntasks, 256, 0, st>>>(b, groups, tasks); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int tsweep_max_resident(int32_t dtype, int NT) {
  switch (dtype) {
    case RAC_DT_F64: return tsweep_resident_nt<double>(NT);
    case RAC_DT_F32: return tsweep_resident_nt<float>(NT);
    case RAC_DT_BF16: return tsweep_resident_nt<uint16_t>(NT);
    default: return 0;
  }
}

hipError_t launch_tsweep(const BatchArgs& b, const TeamArgs& ta, int t, hipStream_t st) {
  switch (b.dtype) {
    case RAC_DT_F64: return tsweep_launch<double>(b, ta, t, st);
    case RAC_DT_F32: return tsweep_launch<float>(b, ta, t, st);
    case RAC_DT_BF16: return tsweep_launch<uint16_t>(b, ta, t, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rac
