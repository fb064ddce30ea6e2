// update.hip -- the z block, the dual step, residual norms, the KKT residual,
// the penalty controller, and the small set-up products.
//
// z block (solved as one block after all x blocks, Sec.3.1):
//   elastic net: z = soft(beta x - xi, lambda alpha) / (beta + lambda (1 - alpha))
//   box:         z = clip(x - xi/beta, lo, hi)
//   none:        z = x - xi/beta
// dual step (Eq.(3)): xi <- xi - beta (x - z), mu <- mu - beta (a'x - b).
// Norms r_p = |(x - z, a'x - b)|_2, r_d = beta |z - z_prev|_2 in FP64 with a
// fixed-order two-level reduction (per-workgroup partials, summed in workgroup
// order by the last workgroup to finish), so results do not depend on timing.
#include "rac_internal.h"
#include "control.h"

namespace rac {
namespace {

constexpr int kRedBlocks = 256;

__device__ __forceinline__ double soft(double v, double t) {
  return v > t ? v - t : (v < -t ? v + t : 0.0);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  return s;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, sh[w]);
  return s;
}

// Returns true in exactly one workgroup: the last one to finish its partials.
__device__ __forceinline__ bool last_block(uint32_t* done) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t prev = atomicAdd(done, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last) __atomic_thread_fence(__ATOMIC_ACQUIRE);
  return is_last;
}

__global__ void __launch_bounds__(256) k_zdual(int64_t n, int32_t prox, double lam, double alpha,
                                               double lo, double hi, double b, int has_eq,
                                               const double* __restrict__ x, double* z, double* xi,
                                               double* zprev, DevScalars* sc, double* red,
                                               uint32_t* done, double* hist, int64_t hist_cap,
                                               int64_t hist_base, int64_t T, const double* beta_ptr,
                                               int publish_beta, const double* extra_rp2) {
  __shared__ double sh[4];
  const double beta = *beta_ptr;
  double rp2 = 0.0, rd2 = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const double xj = x[j], xij = xi[j], zo = z[j];
    double zn;
    if (prox == RAC_PROX_ELASTIC_NET) zn = soft(beta * xj - xij, lam * alpha) / (beta + lam * (1.0 - alpha));
    else if (prox == RAC_PROX_BOX) zn = fmin(fmax(xj - xij / beta, lo), hi);
    else zn = xj - xij / beta;
    const double r = xj - zn, dz = zn - zo;
    xi[j] = xij - beta * r;
    z[j] = zn;
    zprev[j] = zo;
    rp2 += r * r;
    rd2 += dz * dz;
  }
  rp2 = block_sum(rp2, sh);
  rd2 = block_sum(rd2, sh);
  if (threadIdx.x == 0) { red[2 * blockIdx.x] = rp2; red[2 * blockIdx.x + 1] = rd2; }
  if (!last_block(done)) return;
  if (threadIdx.x != 0) return;
  double P = 0.0, D = 0.0;
  for (unsigned q = 0; q < gridDim.x; ++q) { P += red[2 * q]; D += red[2 * q + 1]; }
  *done = 0u;
  if (has_eq) {
    const double e = sc->t - b;
    sc->mu -= beta * e;
    P += e * e;
  }
  if (extra_rp2) P += *extra_rp2;   // dense form: the equality rows, formed with their multiplier step
  const double rp = sqrt(P), rd = beta * sqrt(D);
  const int64_t k = sc->k;
  if (publish_beta) sc->beta = beta;
  sc->rp = rp;
  sc->rd = rd;
  if (k % T == 0) { sc->rp_win = rp; sc->rd_win = rd; }
  if (sc->rp_first < 0.0) sc->rp_first = rp;
  if (!isfinite(rp) || !isfinite(rd) || (sc->rp_first > 0.0 && rp > 1e12 * sc->rp_first))
    sc->status = 2;
  const int64_t hi_ = k - hist_base;
  if (hist && hi_ >= 0 && hi_ < hist_cap) {
    hist[4 * hi_ + 0] = rp;
    hist[4 * hi_ + 1] = rd;
    hist[4 * hi_ + 2] = beta;
    hist[4 * hi_ + 3] = __builtin_nan("");
  }
  sc->k = k + 1;
}

// ---------------------------------------------------------------------------
// KKT residual: one pass over F for grad f(x) = F'u/Ns + h.x + c (one wavefront
// per column, lanes over rows), per-column terms reduced to maxima; t = a'x is
// re-summed from x.  red holds 10 values per workgroup:
//   0 |Hx|, 1 |c|, 2 |xi|, 3 |x|, 4 |z|, 5 |x-z|, 6 |grad f - xi - mu a|,
//   7 dist(-xi, dP(z)), 8 |a|, 9 sum a.x
// Four consecutive entries of a column as doubles (16-byte loads for FP32 and
// FP64 storage, 8-byte for BF16); the caller guarantees the alignment.
__device__ __forceinline__ void ld4(const float* p, double (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const uint16_t* p, double (&o)[4]) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  o[0] = __uint_as_float(v.x << 16); o[1] = __uint_as_float(v.x & 0xffff0000u);
  o[2] = __uint_as_float(v.y << 16); o[3] = __uint_as_float(v.y & 0xffff0000u);
}
__device__ __forceinline__ void ld4(const double* p, double (&o)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p), b = *reinterpret_cast<const double2*>(p + 2);
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

// KKT check: each wavefront forms F_j'u for KC columns at once (u is read once
// per KC columns); lane l takes rows 4l.. of every 256-row step with vector
// loads when the columns are aligned (vec), the remaining rows one by one.
template <typename T>
__global__ void __launch_bounds__(256) k_kkt(const T* __restrict__ F, int64_t ldF, int64_t rows,
                                             int64_t n, double Ns, const double* __restrict__ h,
                                             const double* __restrict__ c, const double* __restrict__ a,
                                             double b, int32_t prox, double lam, double alpha, double lo,
                                             double hi, const double* __restrict__ x,
                                             const double* __restrict__ z, const double* __restrict__ xi,
                                             const double* __restrict__ u, const double* mu_ptr,
                                             double mu_val, double* red, uint32_t* done, double* out, int vec) {
  constexpr int KC = 2;
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double mu = mu_ptr ? *mu_ptr : mu_val;
  double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t rows4 = vec ? rows / 256 * 256 : 0;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * KC; j0 < n; j0 += nwaves * KC) {
    const T* col[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) col[k] = F + (j0 + k < n ? j0 + k : n - 1) * ldF;   // a valid column
    double acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = 0.0;
#pragma unroll 4
    for (int64_t r = 4 * lane; r < rows4; r += 256) {
      double uu[4];
      ld4(u + r, uu);
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        double f[4];
        ld4(col[k] + r, f);
        acc[k] += f[0] * uu[0];
        acc[k] += f[1] * uu[1];
        acc[k] += f[2] * uu[2];
        acc[k] += f[3] * uu[3];
      }
    }
    for (int64_t r = rows4 + lane; r < rows; r += 64) {
      const double ur = u[r];
#pragma unroll
      for (int k = 0; k < KC; ++k) acc[k] += ld_f64(col[k], r) * ur;
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int64_t j = j0 + k;
        if (j < n)
          kkt_column_terms(acc[k], Ns, h ? h[j] : 0.0, c[j], a ? a[j] : 0.0, x[j], z[j], xi[j], mu, prox, lam,
                           alpha, lo, hi, m);
      }
    }
  }
  for (int q = 0; q < 9; ++q) {
    double v = block_max(m[q], sh);
    if (threadIdx.x == 0) red[10 * blockIdx.x + q] = v;
  }
  {
    double v = block_sum(m[9], sh);
    if (threadIdx.x == 0) red[10 * blockIdx.x + 9] = v;
  }
  if (!last_block(done)) return;
  if (threadIdx.x != 0) return;
  double M[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (unsigned q = 0; q < gridDim.x; ++q) {
    for (int e = 0; e < 9; ++e) M[e] = fmax(M[e], red[10 * q + e]);
    M[9] += red[10 * q + 9];
  }
  *done = 0u;
  kkt_from_maxima(M, a != nullptr, b, mu, out);
}

// Two-pass form of the check for the solver: k_kkt_dots forms F_j'u over one of
// kKKTChunks row chunks (grid: column pairs x chunks, so that every compute unit
// streams its share of F), and k_kkt_terms sums the chunks of each column in
// order and reduces the per-column terms as k_kkt does.
template <typename T>
__global__ void __launch_bounds__(256) k_kkt_dots(const T* __restrict__ F, int64_t ldF, int64_t rows,
                                                  int64_t n, const double* __restrict__ u, double* part,
                                                  int vec) {
  constexpr int KC = 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunk = blockIdx.y, nch = gridDim.y;
  // row chunks are multiples of 256 rows except the last
  const int64_t steps = (rows + 255) / 256;
  const int64_t rb = block_start(chunk, steps, nch) * 256;
  const int64_t re_ = block_start(chunk + 1, steps, nch) * 256;
  const int64_t re = re_ < rows ? re_ : rows;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * KC; j0 < n; j0 += nwaves * KC) {
    const T* col[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) col[k] = F + (j0 + k < n ? j0 + k : n - 1) * ldF;
    double acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = 0.0;
    const int64_t rv = vec ? rb + (re - rb) / 256 * 256 : rb;   // vector loads up to rv
#pragma unroll 4
    for (int64_t r = rb + 4 * lane; r < rv; r += 256) {
      double uu[4];
      ld4(u + r, uu);
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        double f[4];
        ld4(col[k] + r, f);
        acc[k] += f[0] * uu[0];
        acc[k] += f[1] * uu[1];
        acc[k] += f[2] * uu[2];
        acc[k] += f[3] * uu[3];
      }
    }
    for (int64_t r = rv + lane; r < re; r += 64) {
      const double ur = u[r];
#pragma unroll
      for (int k = 0; k < KC; ++k) acc[k] += ld_f64(col[k], r) * ur;
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < KC; ++k)
        if (j0 + k < n) part[(int64_t)chunk * n + j0 + k] = acc[k];
    }
  }
}

__global__ void __launch_bounds__(256) k_kkt_terms(int64_t n, int nch, const double* __restrict__ part, double Ns,
                                                   const double* __restrict__ h, const double* __restrict__ c,
                                                   const double* __restrict__ a, double b, int32_t prox,
                                                   double lam, double alpha, double lo, double hi,
                                                   const double* __restrict__ x, const double* __restrict__ z,
                                                   const double* __restrict__ xi, const double* mu_ptr,
                                                   double mu_val, double* red, uint32_t* done, double* out) {
  __shared__ double sh[4];
  const double mu = mu_ptr ? *mu_ptr : mu_val;
  double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int q = 0; q < nch; ++q) acc += part[(int64_t)q * n + j];
    kkt_column_terms(acc, Ns, h ? h[j] : 0.0, c[j], a ? a[j] : 0.0, x[j], z[j], xi[j], mu, prox, lam, alpha,
                     lo, hi, m);
  }
  for (int q = 0; q < 9; ++q) {
    double v = block_max(m[q], sh);
    if (threadIdx.x == 0) red[10 * blockIdx.x + q] = v;
  }
  {
    double v = block_sum(m[9], sh);
    if (threadIdx.x == 0) red[10 * blockIdx.x + 9] = v;
  }
  if (!last_block(done)) return;
  if (threadIdx.x != 0) return;
  double M[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (unsigned q = 0; q < gridDim.x; ++q) {
    for (int e = 0; e < 9; ++e) M[e] = fmax(M[e], red[10 * q + e]);
    M[9] += red[10 * q + 9];
  }
  *done = 0u;
  kkt_from_maxima(M, a != nullptr, b, mu, out);
}

// ---------------------------------------------------------------------------
// Penalty controller (runs once per check, one workgroup of 64 threads); the
// logic is shared with the batched engine (control.h).
__global__ void __launch_bounds__(64) k_control(DevScalars* sc, const double* kkt_out,
                                                int32_t beta_mode, double rb_mu, double rb_tau,
                                                double tol, const float* __restrict__ w,
                                                double ymax, int decide, double* hist,
                                                int64_t hist_cap, int64_t hist_base) {
  control_block(sc, kkt_out[0], beta_mode, rb_mu, rb_tau, tol, w, ymax, decide, hist, hist_cap, hist_base);
}

// ---------------------------------------------------------------------------
// u = F x: partial sums over column chunks, then a fixed-order combination.
template <typename T>
__global__ void __launch_bounds__(256) k_matvec_F_part(const T* __restrict__ F, int64_t ldF,
                                                       int64_t rows, int64_t n, int64_t cpc,
                                                       const double* __restrict__ x, double* part) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * cpc;
  const int64_t j1 = j0 + cpc < n ? j0 + cpc : n;
  if (r >= rows) return;
  double acc = 0.0;
  for (int64_t j = j0; j < j1; ++j) acc += ld_f64(F + j * ldF, r) * x[j];
  part[(int64_t)blockIdx.y * rows + r] = acc;
}
__global__ void __launch_bounds__(256) k_sum_parts(int64_t rows, int nparts, const double* part,
                                                   double* u) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int q = 0; q < nparts; ++q) s += part[(int64_t)q * rows + r];
  u[r] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_matvec_Ft(const T* __restrict__ F, int64_t ldF, int64_t rows,
                                                   int64_t n, const double* __restrict__ u,
                                                   double scale, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j = (int64_t)blockIdx.x * 4 + wave; j < n; j += (int64_t)gridDim.x * 4) {
    const T* col = F + j * ldF;
    double acc = 0.0;
    for (int64_t r = lane; r < rows; r += 64) acc += ld_f64(col, r) * u[r];
    acc = wave_sum(acc);
    if (lane == 0) out[j] = scale * acc;
  }
}

__global__ void __launch_bounds__(256) k_dot(const double* __restrict__ a, const double* __restrict__ x,
                                             int64_t n, double* red, uint32_t* done, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    s += a[j] * x[j];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
  if (!last_block(done)) return;
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (unsigned q = 0; q < gridDim.x; ++q) t += red[q];
  *done = 0u;
  *out = t;
}

// objective = 1/2 (|u|^2/Ns + sum h z^2) + c'z + P(z) + const, with u = F z given.
__global__ void __launch_bounds__(256) k_objective(int64_t rows, int64_t n, double Ns,
                                                   const double* __restrict__ h,
                                                   const double* __restrict__ c, int32_t prox,
                                                   double lam, double alpha, double cst,
                                                   const double* __restrict__ z,
                                                   const double* __restrict__ u, double* red,
                                                   uint32_t* done, double* out) {
  __shared__ double sh[4];
  double q = 0.0, rest = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += stride) q += u[r] * u[r];
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += stride) {
    const double zj = z[j];
    double v = c[j] * zj;
    if (h) v += 0.5 * h[j] * zj * zj;
    if (prox == RAC_PROX_ELASTIC_NET) v += lam * (alpha * fabs(zj) + 0.5 * (1.0 - alpha) * zj * zj);
    rest += v;
  }
  q = block_sum(q, sh);
  rest = block_sum(rest, sh);
  if (threadIdx.x == 0) { red[2 * blockIdx.x] = q; red[2 * blockIdx.x + 1] = rest; }
  if (!last_block(done)) return;
  if (threadIdx.x != 0) return;
  double Q = 0.0, S = 0.0;
  for (unsigned e = 0; e < gridDim.x; ++e) { Q += red[2 * e]; S += red[2 * e + 1]; }
  *done = 0u;
  *out = 0.5 * Q / Ns + S + cst;
}

template <typename T>
hipError_t kkt_launch(const KKTArgs& k, hipStream_t st) {
  int64_t blocks = (k.n + 7) / 8;   // two columns per wavefront
  if (blocks > kRedBlocks) blocks = kRedBlocks;
  const size_t al = sizeof(T) == 8 ? 16 : 4 * sizeof(T);
  const int vec = (k.ldF % 4 == 0) && ((uintptr_t)k.F % al == 0) && ((uintptr_t)k.u % 16 == 0);
  if (k.part) {
    const int64_t steps = (k.rows + 255) / 256;
    const int nch = (int)(steps < kKKTChunks ? steps : kKKTChunks);
    int64_t cb = (k.n + 7) / 8;
    if (cb > 65535) cb = 65535;
    k_kkt_dots<T><<<dim3((unsigned)cb, (unsigned)nch), 256, 0, st>>>((const T*)k.F, k.ldF, k.rows, k.n, k.u,
                                                                      k.part, vec);
    int64_t tb = (k.n + 255) / 256;
    if (tb > kRedBlocks) tb = kRedBlocks;
    k_kkt_terms<<<(unsigned)tb, 256, 0, st>>>(k.n, nch, k.part, k.Ns, k.h, k.c, k.a, k.b, k.prox, k.lam,
                                              k.alpha, k.lo, k.hi, k.x, k.z, k.xi, k.mu_ptr, k.mu_val, k.red,
                                              k.done, k.out);
    return hipGetLastError();
  }
  k_kkt<T><<<(unsigned)blocks, 256, 0, st>>>((const T*)k.F, k.ldF, k.rows, k.n, k.Ns, k.h, k.c, k.a,
                                              k.b, k.prox, k.lam, k.alpha, k.lo, k.hi, k.x, k.z,
                                              k.xi, k.u, k.mu_ptr, k.mu_val, k.red, k.done, k.out, vec);
  return hipGetLastError();
}

template <typename T>
hipError_t matvec_F_launch(const void* F, int64_t ldF, int64_t rows, int64_t n, const double* x,
                           double* u, double* part, int nparts, int64_t cpc, hipStream_t st) {
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)nparts);
  k_matvec_F_part<T><<<grid, 256, 0, st>>>((const T*)F, ldF, rows, n, cpc, x, part);
  k_sum_parts<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(rows, nparts, part, u);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zdual(const UpdateArgs& z, hipStream_t st) {
  int64_t blocks = (z.n + 255) / 256;
  if (blocks > kRedBlocks) blocks = kRedBlocks;
  k_zdual<<<(unsigned)blocks, 256, 0, st>>>(z.n, z.prox, z.lam, z.alpha, z.lo, z.hi, z.b, z.has_eq,
                                            z.x, z.z, z.xi, z.zprev, z.sc, z.red, z.done, z.hist,
                                            z.hist_cap, z.hist_base, z.T, z.beta_ptr, z.publish_beta, z.extra_rp2);
  return hipGetLastError();
}

hipError_t launch_kkt_terms(const KKTArgs& k, int nch, hipStream_t st) {
  int64_t tb = (k.n + 255) / 256;
  if (tb > kRedBlocks) tb = kRedBlocks;
  k_kkt_terms<<<(unsigned)tb, 256, 0, st>>>(k.n, nch, k.part, k.Ns, k.h, k.c, k.a, k.b, k.prox, k.lam, k.alpha,
                                            k.lo, k.hi, k.x, k.z, k.xi, k.mu_ptr, k.mu_val, k.red, k.done, k.out);
  return hipGetLastError();
}

hipError_t launch_hd_dots(const void* Hd, int32_t dtype, int64_t ldH, int64_t n, const double* v, double* part,
                          int* nch_out, hipStream_t st) {
  const int64_t steps = (n + 255) / 256;
  const int nch = (int)(steps < kKKTChunks ? steps : kKKTChunks);
  int64_t cb = (n + 7) / 8;
  if (cb > 65535) cb = 65535;
  const dim3 grid((unsigned)cb, (unsigned)nch);
  if (nch_out) *nch_out = nch;
  if (dtype == RAC_DT_F64) {
    const int vec = (ldH % 4 == 0) && ((uintptr_t)Hd % 16 == 0) && ((uintptr_t)v % 16 == 0);
    k_kkt_dots<double><<<grid, 256, 0, st>>>((const double*)Hd, ldH, n, n, v, part, vec);
  } else if (dtype == RAC_DT_F32) {
    const int vec = (ldH % 4 == 0) && ((uintptr_t)Hd % 16 == 0) && ((uintptr_t)v % 16 == 0);
    k_kkt_dots<float><<<grid, 256, 0, st>>>((const float*)Hd, ldH, n, n, v, part, vec);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_kkt(const KKTArgs& k, hipStream_t st) {
  switch (k.dtype) {
    case RAC_DT_F64: return kkt_launch<double>(k, st);
    case RAC_DT_F32: return kkt_launch<float>(k, st);
    case RAC_DT_BF16: return kkt_launch<uint16_t>(k, st);
    default: return hipErrorInvalidValue;
  }
}

__global__ void k_scale_beta(DevScalars* sc, double mult) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->beta *= mult;
    sc->last_l10 = log10(mult);
    sc->decisions += 1;
  }
}

hipError_t launch_scale_beta(DevScalars* sc, double mult, hipStream_t st) {
  k_scale_beta<<<1, 64, 0, st>>>(sc, mult);
  return hipGetLastError();
}

hipError_t launch_control(const ControlArgs& c, hipStream_t st) {
  k_control<<<1, 64, 0, st>>>(c.sc, c.kkt_out, c.beta_mode, c.rb_mu, c.rb_tau, c.tol, c.mlp_w,
                              c.mlp_ymax, c.decide, c.hist, c.hist_cap, c.hist_base);
  return hipGetLastError();
}

// u = F x needs a scratch of nparts*rows doubles: the caller passes `u` of size
// rows and this routine allocates nothing, so the partials go through a
// temporary provided by the caller inside `u_part`.
hipError_t launch_matvec_F_parts(const void* F, int32_t dtype, int64_t ldF, int64_t rows, int64_t n,
                                 const double* x, double* u, double* part, int nparts,
                                 hipStream_t st) {
  const int64_t cpc = (n + nparts - 1) / nparts;
  switch (dtype) {
    case RAC_DT_F64: return matvec_F_launch<double>(F, ldF, rows, n, x, u, part, nparts, cpc, st);
    case RAC_DT_F32: return matvec_F_launch<float>(F, ldF, rows, n, x, u, part, nparts, cpc, st);
    case RAC_DT_BF16: return matvec_F_launch<uint16_t>(F, ldF, rows, n, x, u, part, nparts, cpc, st);
    default: return hipErrorInvalidValue;
  }
}

// Whether any of rows x cols elements (column-major, leading dimension ld, element type
// dtype) is NaN or infinite: a workgroup per column in turn, the flag raised once per
// wavefront that saw one.  BF16 values are tested on their exponent bits.
__global__ void __launch_bounds__(256) k_nonfinite(const void* __restrict__ p, int32_t dtype, int64_t rows,
                                                   int64_t cols, int64_t ld, uint32_t* flag) {
  bool bad = false;
  for (int64_t c = blockIdx.x; c < cols; c += gridDim.x) {
    const int64_t o = c * ld;
    for (int64_t r = threadIdx.x; r < rows; r += 256) {
      if (dtype == RAC_DT_F64) bad |= !isfinite(((const double*)p)[o + r]);
      else if (dtype == RAC_DT_F32) bad |= !isfinite(((const float*)p)[o + r]);
      else bad |= (((const uint16_t*)p)[o + r] & 0x7F80u) == 0x7F80u;
    }
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

hipError_t launch_nonfinite(const void* p, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, uint32_t* flag,
                            hipStream_t st) {
  if (rows < 1 || cols < 1) return hipSuccess;
  const int64_t blocks = cols < 65536 ? cols : 65536;
  k_nonfinite<<<(unsigned)blocks, 256, 0, st>>>(p, dtype, rows, cols, ld, flag);
  return hipGetLastError();
}

hipError_t launch_matvec_Ft(const void* F, int32_t dtype, int64_t ldF, int64_t rows, int64_t n,
                            const double* u, double scale, double* out, hipStream_t st) {
  int64_t blocks = (n + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  switch (dtype) {
    case RAC_DT_F64:
      k_matvec_Ft<double><<<(unsigned)blocks, 256, 0, st>>>((const double*)F, ldF, rows, n, u, scale, out);
      break;
    case RAC_DT_F32:
      k_matvec_Ft<float><<<(unsigned)blocks, 256, 0, st>>>((const float*)F, ldF, rows, n, u, scale, out);
      break;
    case RAC_DT_BF16:
      k_matvec_Ft<uint16_t><<<(unsigned)blocks, 256, 0, st>>>((const uint16_t*)F, ldF, rows, n, u, scale,
                                                               out);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dot_red(const double* a, const double* x, int64_t n, double* red, uint32_t* done,
                          double* out, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > kRedBlocks) blocks = kRedBlocks;
  k_dot<<<(unsigned)blocks, 256, 0, st>>>(a, x, n, red, done, out);
  return hipGetLastError();
}

hipError_t launch_objective_red(int64_t rows, int64_t n, double Ns, const double* h, const double* c,
                                int32_t prox, double lam, double alpha, double cst, const double* z,
                                const double* u, double* red, uint32_t* done, double* out,
                                hipStream_t st) {
  int64_t m = rows > n ? rows : n;
  int64_t blocks = (m + 255) / 256;
  if (blocks > kRedBlocks) blocks = kRedBlocks;
  k_objective<<<(unsigned)blocks, 256, 0, st>>>(rows, n, Ns, h, c, prox, lam, alpha, cst, z, u, red,
                                                done, out);
  return hipGetLastError();
}

}  // namespace rac
