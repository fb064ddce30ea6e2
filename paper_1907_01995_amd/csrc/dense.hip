// dense.hip -- kernels of the dense form: the general QP of Eq.(1) with an
// explicit symmetric Hessian Hd and several equality rows A x = beq (Eq.(4)),
// and the Gaussian-kernel matrix of the C-SVC dual (Sec.3.2, Eq.(9)).
//
// The equality rows enter the augmented Lagrangian (Eq.(2), one penalty beta)
// as beta/2 |A x - beq|^2 - mu'(A x - beq), whose gradient is
// beta A'A x - A'(beta beq + mu).  The sweep therefore works with
//   H_beta = Hd + beta A'A   and   c_eff = c - A'(beta beq + mu),
// formed here whenever beta (H_beta) or mu (c_eff) has changed: every block
// gradient g_B = (H_beta x)_B + h_B x_B + c_eff_B - xi_B + beta (x_B - z_B) and
// block matrix H_beta[B,B] + diag h_B + beta I are then those of Eq.(3).  After
// the sweep, t = A x is formed from x and mu <- mu - beta (t - beq).
#include "rac_internal.h"
#include "control.h"

namespace rac {
namespace {

template <typename T> __device__ __forceinline__ double ldd(const T* p, int64_t i) { return (double)p[i]; }

// H_beta = Hd + beta A'A (column-major n x n, FP64); a grid-stride loop over the
// entries, consecutive threads along a column.
template <typename T>
__global__ void __launch_bounds__(256) k_hbeta(const T* __restrict__ Hd, int64_t ldH, int64_t n, int meq,
                                               const double* __restrict__ A, const double* beta_ptr,
                                               double* __restrict__ Hb) {
  const double beta = *beta_ptr;
  const int64_t total = n * n;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
    const int64_t j = q / n, i = q - j * n;
    double aa = 0.0;
    for (int e = 0; e < meq; ++e) aa += A[(int64_t)e * n + i] * A[(int64_t)e * n + j];
    Hb[q] = ldd(Hd, j * ldH + i) + beta * aa;
  }
}

// c_eff = c - A'(beta beq + mu) for the iteration's beta and the current mu.
__global__ void __launch_bounds__(256) k_ceff(int64_t n, int meq, const double* __restrict__ A,
                                              const double* __restrict__ beq, const double* __restrict__ mu,
                                              const double* beta_ptr, const double* __restrict__ c,
                                              double* __restrict__ ceff) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const double beta = *beta_ptr;
  double v = c[j];
  for (int e = 0; e < meq; ++e) v -= A[(int64_t)e * n + j] * (beta * beq[e] + mu[e]);
  ceff[j] = v;
}

// Block matrices of the drawn partition: entry (q, r), q >= r, of block i is
// H[B_q, B_r] (the lower triangle, in the layout the factor kernel reads; one
// row chunk).  The factor adds diag h + beta I.
template <typename T>
__global__ void __launch_bounds__(256) k_hgather(const T* __restrict__ H, int64_t ldH, int64_t n, int64_t p,
                                                 const int32_t* __restrict__ perm, int sp, double* __restrict__ out) {
  const int64_t blk = blockIdx.x;
  const int64_t s0 = block_start(blk, n, p);
  const int sb = (int)(block_start(blk + 1, n, p) - s0);
  double* o = out + blk * (int64_t)sp * sp;
  for (int e = threadIdx.x; e < sp * sp; e += 256) {
    const int q = e / sp, r = e % sp;
    double v = 0.0;
    if (q < sb && r < sb && q >= r) v = ldd(H, (int64_t)perm[s0 + r] * ldH + perm[s0 + q]);
    o[e] = v;
  }
}

// t = A x, then mu <- mu - beta (t - beq) and the equality part of the primal
// residual, |t - beq|^2 (added to r_p by the z/dual step).  One workgroup per
// row, rows combined in order by the last workgroup; mu_0 is mirrored into the
// solver's scalars.
__global__ void __launch_bounds__(256) k_eq(int64_t n, int meq, const double* __restrict__ A,
                                            const double* __restrict__ beq, const double* __restrict__ x,
                                            const double* beta_ptr, double* t, double* mu, double* r2,
                                            double* red, uint32_t* done, DevScalars* sc) {
  __shared__ double sh[4];
  __shared__ int is_last;
  const int e = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) s += A[(int64_t)e * n + j] * x[j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double te = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    const double beta = *beta_ptr;
    const double r = te - beq[e];
    t[e] = te;
    mu[e] -= beta * r;
    red[e] = r * r;
    __threadfence();
    is_last = atomicAdd(done, 1u) == (unsigned)meq - 1;
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  double acc = 0.0;
  for (int q = 0; q < meq; ++q) acc += red[q];
  *r2 = acc;
  sc->mu = mu[0];
  sc->t = t[0];
  *done = 0u;
}

// KKT residual of the dense form from the column products dots (Hd_j'x summed
// over nch row chunks): the terms of the factor form with H x = dots + h.x and
// the multiplier term A'mu, plus the equality feasibility
// max_e |t_e - beq_e| / (1 + |beq|_inf + |A|_inf |x|_inf) with t = A x (current x).
// red: 10 values per workgroup (0 |Hx|, 1 |c|, 2 |xi|, 3 |x|, 4 |z|, 5 |x-z|,
// 6 |grad f - xi - A'mu|, 7 dist(-xi, dP(z)), 8 |A'mu|, 9 |A|).
__global__ void __launch_bounds__(256) k_dkkt_terms(int64_t n, int nch, const double* __restrict__ part,
                                                    const double* __restrict__ h, const double* __restrict__ c,
                                                    int meq, const double* __restrict__ A,
                                                    const double* __restrict__ beq, const double* __restrict__ t,
                                                    const double* __restrict__ mu, int32_t prox, double lam,
                                                    double alpha, double lo, double hi,
                                                    const double* __restrict__ x, const double* __restrict__ z,
                                                    const double* __restrict__ xi, double* red, uint32_t* done,
                                                    double* out) {
  __shared__ double sh[4];
  __shared__ int is_last;
  double mm[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int q = 0; q < nch; ++q) acc += part[(int64_t)q * n + j];
    double amu = 0.0, amax = 0.0;
    for (int e = 0; e < meq; ++e) {
      const double ae = A[(int64_t)e * n + j];
      amu += ae * mu[e];
      amax = fmax(amax, fabs(ae));
    }
    double cm[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    kkt_column_terms(acc, 1.0, h ? h[j] : 0.0, c[j], 1.0, x[j], z[j], xi[j], amu, prox, lam, alpha, lo, hi, cm);
    for (int q = 0; q < 8; ++q) mm[q] = fmax(mm[q], cm[q]);
    mm[8] = fmax(mm[8], fabs(amu));
    mm[9] = fmax(mm[9], amax);
  }
  for (int q = 0; q < 10; ++q) {
    double v = wave_max(mm[q]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) red[10 * blockIdx.x + q] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  }
  if (threadIdx.x == 0) {
    __threadfence();
    is_last = atomicAdd(done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  double M[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (unsigned q = 0; q < gridDim.x; ++q)
    for (int e = 0; e < 10; ++e) M[e] = fmax(M[e], red[10 * q + e]);
  *done = 0u;
  double feas = M[5] / (1.0 + fmax(M[3], M[4]));
  if (meq > 0) {
    double emax = 0.0, bmax = 0.0;
    for (int e = 0; e < meq; ++e) {
      emax = fmax(emax, fabs(t[e] - beq[e]));
      bmax = fmax(bmax, fabs(beq[e]));
    }
    feas = fmax(feas, emax / (1.0 + bmax + M[9] * M[3]));
  }
  double scale = fmax(fmax(M[0], M[1]), M[2]);
  if (meq > 0) scale = fmax(scale, M[8]);
  if (scale < 1e-300) scale = 1e-300;
  out[1] = feas;
  out[2] = M[6] / scale;
  out[3] = M[7] / scale;
  out[0] = fmax(out[1], fmax(out[2], out[3]));
}

// Objective of the dense form at z from dots = Hd z (summed over row chunks):
// 1/2 z'(Hd z) + 1/2 sum h z^2 + c'z + P(z) + const; fixed-order reduction.
__global__ void __launch_bounds__(256) k_dobjective(int64_t n, int nch, const double* __restrict__ part,
                                                    const double* __restrict__ h, const double* __restrict__ c,
                                                    int32_t prox, double lam, double alpha, double cst,
                                                    const double* __restrict__ z, double* red, uint32_t* done,
                                                    double* out) {
  __shared__ double sh[4];
  __shared__ int is_last;
  double s = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    double hz = 0.0;
    for (int q = 0; q < nch; ++q) hz += part[(int64_t)q * n + j];
    const double zj = z[j];
    double v = 0.5 * zj * hz + c[j] * zj;
    if (h) v += 0.5 * h[j] * zj * zj;
    if (prox == RAC_PROX_ELASTIC_NET) v += lam * (alpha * fabs(zj) + 0.5 * (1.0 - alpha) * zj * zj);
    s += v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    red[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __threadfence();
    is_last = atomicAdd(done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  double acc = 0.0;
  for (unsigned q = 0; q < gridDim.x; ++q) acc += red[q];
  *done = 0u;
  *out = acc + cst;
}

// ---------------------------------------------------------------------------
// Gaussian kernel (Sec.3.2): K(u, v) = exp(-gamma |u - v|^2).  Q_ij = y_i y_j
// K(x_i, x_j) for the training points (n x n, column-major), and decision
// values f(v) = sum_j alpha_j y_j K(x_j, v) + bias for query points.  Squared
// distances are summed over the features from the differences (FP64), so Q is
// exactly symmetric.  Tiles of 64 x 64 points: both point sets' feature chunks
// are staged in LDS.
constexpr int kKT = 64;      // points per tile side
constexpr int kKF = 32;      // features per LDS chunk

template <typename T>
__device__ __forceinline__ void kernel_tile(const T* __restrict__ X, int64_t n, int64_t r, const T* __restrict__ V,
                                            int64_t m, int64_t i0, int64_t j0, double (&acc)[16],
                                            double (*xs)[kKF + 1], double (*vs)[kKF + 1]) {
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;   // 4 x 4 outputs per thread
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  for (int64_t f0 = 0; f0 < r; f0 += kKF) {
    for (int e = tid; e < kKT * kKF; e += 256) {
      const int pnt = e / kKF, f = e % kKF;
      const int64_t gi = i0 + pnt, gj = j0 + pnt, gf = f0 + f;
      xs[pnt][f] = (gi < n && gf < r) ? (double)X[gi * r + gf] : 0.0;
      vs[pnt][f] = (gj < m && gf < r) ? (double)V[gj * r + gf] : 0.0;
    }
    __syncthreads();
    for (int f = 0; f < kKF; ++f) {
      double a[4], b[4];
      for (int q = 0; q < 4; ++q) { a[q] = xs[ti + 16 * q][f]; b[q] = vs[tj + 16 * q][f]; }
      for (int q = 0; q < 4; ++q)
        for (int w = 0; w < 4; ++w) {
          const double d = a[q] - b[w];
          acc[4 * q + w] += d * d;
        }
    }
    __syncthreads();
  }
}

// Q (ldQ >= n) from X (n x r, row-major: point i's features contiguous) and labels y.
template <typename T>
__global__ void __launch_bounds__(256) k_gauss_q(const T* __restrict__ X, int64_t n, int64_t r,
                                                 const double* __restrict__ y, double gamma, double* __restrict__ Q,
                                                 int64_t ldQ) {
  __shared__ double xs[kKT][kKF + 1], vs[kKT][kKF + 1];
  const int64_t i0 = (int64_t)blockIdx.x * kKT, j0 = (int64_t)blockIdx.y * kKT;
  double acc[16];
  kernel_tile<T>(X, n, r, X, n, i0, j0, acc, xs, vs);
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  for (int q = 0; q < 4; ++q)
    for (int w = 0; w < 4; ++w) {
      const int64_t i = i0 + ti + 16 * q, j = j0 + tj + 16 * w;
      if (i < n && j < n) Q[j * ldQ + i] = y[i] * y[j] * exp(-gamma * acc[4 * q + w]);
    }
}

// f(v_k) = sum_j alpha_j y_j K(x_j, v_k) + bias: one workgroup per
// 64 query points, the training points in tiles; per-thread partial sums over
// the tile's training points, then a fixed-order sum over the 16 thread rows.
template <typename T>
__global__ void __launch_bounds__(256) k_decision(const T* __restrict__ X, int64_t n, int64_t r,
                                                  const double* __restrict__ alpha, const double* __restrict__ y,
                                                  double gamma,
                                                  const T* __restrict__ V, int64_t m, double bias,
                                                  double* __restrict__ f) {
  __shared__ double xs[kKT][kKF + 1], vs[kKT][kKF + 1];
  __shared__ double part[16][kKT];
  const int64_t j0 = (int64_t)blockIdx.x * kKT;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = 0; i0 < n; i0 += kKT) {
    double acc[16];
    kernel_tile<T>(X, n, r, V, m, i0, j0, acc, xs, vs);
    for (int w = 0; w < 4; ++w)
      for (int q = 0; q < 4; ++q) {
        const int64_t i = i0 + ti + 16 * q;
        if (i < n) sum[w] += (alpha[i] * y[i]) * exp(-gamma * acc[4 * q + w]);
      }
  }
  for (int w = 0; w < 4; ++w) part[ti][tj + 16 * w] = sum[w];
  __syncthreads();
  if (threadIdx.x < kKT) {
    const int64_t j = j0 + threadIdx.x;
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += part[q][threadIdx.x];
    if (j < m) f[j] = s + bias;
  }
}

// Fraction of query points whose label has the sign of the decision value (f = 0
// counts as +1); fixed-order reduction.
__global__ void __launch_bounds__(256) k_accuracy(const double* __restrict__ f, const double* __restrict__ labels,
                                                  int64_t m, double* red, uint32_t* done, double* out) {
  __shared__ double sh[4];
  __shared__ int is_last;
  double s = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)gridDim.x * 256)
    s += ((f[j] >= 0.0 ? 1.0 : -1.0) == labels[j]) ? 1.0 : 0.0;
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    red[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __threadfence();
    is_last = atomicAdd(done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  double acc = 0.0;
  for (unsigned q = 0; q < gridDim.x; ++q) acc += red[q];
  *done = 0u;
  *out = acc / (double)m;
}

}  // namespace

hipError_t launch_hbeta(const void* Hd, int32_t dtype, int64_t ldH, int64_t n, int meq, const double* A,
                        const double* beta_ptr, double* Hb, hipStream_t st) {
  int64_t blocks = (n * n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  const unsigned grid = (unsigned)blocks;
  if (dtype == RAC_DT_F64) k_hbeta<double><<<grid, 256, 0, st>>>((const double*)Hd, ldH, n, meq, A, beta_ptr, Hb);
  else if (dtype == RAC_DT_F32) k_hbeta<float><<<grid, 256, 0, st>>>((const float*)Hd, ldH, n, meq, A, beta_ptr, Hb);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_ceff(int64_t n, int meq, const double* A, const double* beq, const double* mu,
                       const double* beta_ptr, const double* c, double* ceff, hipStream_t st) {
  k_ceff<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, meq, A, beq, mu, beta_ptr, c, ceff);
  return hipGetLastError();
}

hipError_t launch_hgather(const void* H, int32_t dtype, int64_t ldH, int64_t n, int64_t p, const int32_t* perm,
                          int sp, double* out, hipStream_t st) {
  if (dtype == RAC_DT_F64) k_hgather<double><<<(unsigned)p, 256, 0, st>>>((const double*)H, ldH, n, p, perm, sp, out);
  else if (dtype == RAC_DT_F32) k_hgather<float><<<(unsigned)p, 256, 0, st>>>((const float*)H, ldH, n, p, perm, sp, out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_eq(int64_t n, int meq, const double* A, const double* beq, const double* x, const double* beta_ptr,
                     double* t, double* mu, double* r2, double* red, uint32_t* done, DevScalars* sc, hipStream_t st) {
  if (meq <= 0) return hipSuccess;
  k_eq<<<(unsigned)meq, 256, 0, st>>>(n, meq, A, beq, x, beta_ptr, t, mu, r2, red, done, sc);
  return hipGetLastError();
}

hipError_t launch_dkkt(const DenseKKTArgs& k, hipStream_t st) {
  int nch = 1;
  const hipError_t e = launch_hd_dots(k.Hd, k.dtype, k.ldH, k.n, k.x, k.part, &nch, st);
  if (e != hipSuccess) return e;
  int64_t tb = (k.n + 255) / 256;
  if (tb > 256) tb = 256;
  k_dkkt_terms<<<(unsigned)tb, 256, 0, st>>>(k.n, nch, k.part, k.h, k.c, k.meq, k.A, k.beq, k.t, k.mu, k.prox,
                                             k.lam, k.alpha, k.lo, k.hi, k.x, k.z, k.xi, k.red, k.done, k.out);
  return hipGetLastError();
}

hipError_t launch_dobjective(const DenseKKTArgs& k, const double* z, double cst, hipStream_t st) {
  int nch = 1;
  const hipError_t e = launch_hd_dots(k.Hd, k.dtype, k.ldH, k.n, z, k.part, &nch, st);
  if (e != hipSuccess) return e;
  int64_t tb = (k.n + 255) / 256;
  if (tb > 256) tb = 256;
  k_dobjective<<<(unsigned)tb, 256, 0, st>>>(k.n, nch, k.part, k.h, k.c, k.prox, k.lam, k.alpha, cst, z, k.red,
                                             k.done, k.out);
  return hipGetLastError();
}

hipError_t launch_gauss_q(const void* X, int32_t dtype, int64_t n, int64_t r, const double* y, double gamma,
                          double* Q, int64_t ldQ, hipStream_t st) {
  dim3 grid((unsigned)((n + kKT - 1) / kKT), (unsigned)((n + kKT - 1) / kKT));
  if (dtype == RAC_DT_F64) k_gauss_q<double><<<grid, 256, 0, st>>>((const double*)X, n, r, y, gamma, Q, ldQ);
  else if (dtype == RAC_DT_F32) k_gauss_q<float><<<grid, 256, 0, st>>>((const float*)X, n, r, y, gamma, Q, ldQ);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_decision(const void* X, int32_t dtype, int64_t n, int64_t r, const double* alpha,
                           const double* y, double gamma, const void* V, int64_t m, double bias, double* f,
                           hipStream_t st) {
  const unsigned grid = (unsigned)((m + kKT - 1) / kKT);
  if (dtype == RAC_DT_F64)
    k_decision<double><<<grid, 256, 0, st>>>((const double*)X, n, r, alpha, y, gamma, (const double*)V, m, bias, f);
  else if (dtype == RAC_DT_F32)
    k_decision<float><<<grid, 256, 0, st>>>((const float*)X, n, r, alpha, y, gamma, (const float*)V, m, bias, f);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_accuracy(const double* f, const double* labels, int64_t m, double* red, uint32_t* done,
                           double* out, hipStream_t st) {
  int64_t blocks = (m + 255) / 256;
  if (blocks > 256) blocks = 256;
  k_accuracy<<<(unsigned)blocks, 256, 0, st>>>(f, labels, m, red, done, out);
  return hipGetLastError();
}

}  // namespace rac
