// sweep.hip -- phase 2 of an iteration: the cyclic Gauss-Seidel pass over the
// drawn blocks (Eq.(3), x_1 ... x_p in order), one persistent launch per sweep.
//
// For block B the exact minimiser of the augmented Lagrangian over x_B is
//   x_B <- x_B - M_B^{-1} g_B,
//   g_B = F_B'u/Ns + h_B.x_B + c_B - xi_B + beta(x_B - z_B) - mu a_B + beta a_B (t - b),
// where u = F x and t = a'x are maintained through the sweep (u += F_B d, t += a_B'd).
//
// Work split: K cooperating workgroups each own a contiguous range of the rows
// of F, and hence of u, which never leaves its owner.  Per block:
//   1. every workgroup forms its partial F_B'u over its rows (FP64 accumulation,
//      wavefront-shuffle reductions) and publishes it;
//   2. one flag per workgroup (no contended counter) tells the others it is ready;
//   3. every workgroup sums the K partials in the same fixed order, adds the
//      remaining terms and applies M_B^{-1}, so all of them hold the identical
//      step d without a second exchange;
//   4. each updates its own rows of u; workgroup 0 writes x_B.
// Partials are double-buffered by block parity, so one exchange per block suffices.
#include "rac_internal.h"

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
                                               double* partials, uint64_t* flags, uint64_t epoch_base) {
  const int K = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = block_start(g, rows, K), r1 = block_start(g + 1, rows, K);
  __shared__ double gl[kMaxBlock];     // partial, then full gradient
  __shared__ double dl[kMaxBlock];     // step d = -M^{-1} g
  __shared__ int32_t cols[kMaxBlock];
  __shared__ double t_sh;
  const double beta = *beta_ptr;
  const double mu = sc->mu;
  double t = sc->t;

  for (int64_t i = 0; i < p; ++i) {
    const int64_t s0 = block_start(i, n, p);
    const int sb = (int)(block_start(i + 1, n, p) - s0);
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
      if (wave == 0) {
        for (int q = lane; q < K; q += 64)
          while (__hip_atomic_load(&flags[(int64_t)q * kFlagStride], __ATOMIC_ACQUIRE,
                                   __HIP_MEMORY_SCOPE_AGENT) < epoch)
            __builtin_amdgcn_s_sleep(1);
      }
      __syncthreads();
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
    const double* Mi = Minv + i * (int64_t)sp * sp;
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

template <typename T>
hipError_t sweep_launch(const SweepArgs& s, hipStream_t st) {
  const T* F = (const T*)s.F;
  const double* beta_ptr = &s.sc->beta;
  void* args[] = {(void*)&F, (void*)&s.ldF, (void*)&s.rows, (void*)&s.n, (void*)&s.p,
                  (void*)&s.perm, (void*)&s.Minv, (void*)&s.sp, (void*)&s.c, (void*)&s.h,
                  (void*)&s.a, (void*)&s.b, (void*)&s.Ns, (void*)&s.x, (void*)&s.z, (void*)&s.xi,
                  (void*)&s.u, (void*)&s.sc, (void*)&beta_ptr, (void*)&s.partials,
                  (void*)&s.flags, (void*)&s.epoch_base};
  if (s.K == 1) {
    k_sweep<T><<<1, 256, 0, st>>>(F, s.ldF, s.rows, s.n, s.p, s.perm, s.Minv, s.sp, s.c, s.h, s.a,
                                  s.b, s.Ns, s.x, s.z, s.xi, s.u, s.sc, beta_ptr, s.partials,
                                  s.flags, s.epoch_base);
    return hipGetLastError();
  }
  return hipLaunchCooperativeKernel((const void*)k_sweep<T>, dim3((unsigned)s.K), dim3(256), args, 0,
                                    st);
}

}  // namespace

hipError_t launch_sweep(const SweepArgs& s, hipStream_t st) {
  switch (s.dtype) {
    case RAC_DT_F64: return sweep_launch<double>(s, st);
    case RAC_DT_F32: return sweep_launch<float>(s, st);
    case RAC_DT_BF16: return sweep_launch<uint16_t>(s, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rac
