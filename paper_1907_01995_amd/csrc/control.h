// control.h -- device logic shared by the single-instance and batched check
// kernels: per-column KKT terms, the KKT residual from their maxima, and the
// penalty controller (residual balancing or the 8-64-64-1 network).
#pragma once

#include "rac_internal.h"

namespace rac {

// Per-column terms of the KKT residual at (x, z, xi, mu), given Hx_j without h
// (acc = F_j'u) -- see rac_kkt in racmb.h.  m[0..9] accumulate
//   0 |Hx|, 1 |c|, 2 |xi|, 3 |x|, 4 |z|, 5 |x-z|, 6 |grad f - xi - mu a|,
//   7 dist(-xi, dP(z)), 8 |a|, 9 sum a.x
__device__ __forceinline__ void kkt_column_terms(double acc, double Ns, double hj, double cj, double aj,
                                                 double xj, double zj, double xij, double mu, int32_t prox,
                                                 double lam, double alpha, double lo, double hi,
                                                 double* m) {
  const double hx = acc / Ns + hj * xj;
  const double g = hx + cj - xij - mu * aj;
  double d;
  if (prox == RAC_PROX_NONE) {
    d = fabs(xij);
  } else if (prox == RAC_PROX_ELASTIC_NET) {
    const double la = lam * alpha, l2 = lam * (1.0 - alpha);
    if (zj > 0) d = fabs(-xij - (la + l2 * zj));
    else if (zj < 0) d = fabs(-xij - (-la + l2 * zj));
    else d = fabs(xij) > la ? fabs(xij) - la : 0.0;
  } else {
    const double w = -xij;
    const bool at_lo = zj <= lo, at_hi = zj >= hi;
    if (at_lo && at_hi) d = 0.0;
    else if (at_lo) d = w > 0 ? w : 0.0;
    else if (at_hi) d = w < 0 ? -w : 0.0;
    else d = fabs(w);
  }
  m[0] = fmax(m[0], fabs(hx));
  m[1] = fmax(m[1], fabs(cj));
  m[2] = fmax(m[2], fabs(xij));
  m[3] = fmax(m[3], fabs(xj));
  m[4] = fmax(m[4], fabs(zj));
  m[5] = fmax(m[5], fabs(xj - zj));
  m[6] = fmax(m[6], fabs(g));
  m[7] = fmax(m[7], d);
  m[8] = fmax(m[8], fabs(aj));
  m[9] += aj * xj;
}

// out = {KKT, feasibility, stationarity, dual feasibility} from the maxima above.
__device__ __forceinline__ void kkt_from_maxima(const double* M, bool has_a, double b, double mu, double* out) {
  double feas = M[5] / (1.0 + fmax(M[3], M[4]));
  if (has_a) feas = fmax(feas, fabs(M[9] - b) / (1.0 + fabs(b) + M[8] * M[3]));
  double scale = fmax(fmax(M[0], M[1]), M[2]);
  if (has_a) scale = fmax(scale, fabs(mu) * M[8]);
  if (scale < 1e-300) scale = 1e-300;
  const double stat = M[6] / scale, dual = M[7] / scale;
  out[1] = feas;
  out[2] = stat;
  out[3] = dual;
  out[0] = fmax(feas, fmax(stat, dual));
}

__device__ __forceinline__ double lg10c(double v) { return log10(v > 1e-300 ? v : 1e-300); }
__device__ __forceinline__ double clip4(double v) { return v < -4.0 ? -4.0 : (v > 4.0 ? 4.0 : v); }

// Stopping test and penalty rule at a check, executed by one 64-thread group:
//   residual balancing: beta *= tau if r_p > mu_rb r_d; beta /= tau if r_d > mu_rb r_p
//   network: features -> 8-64-64-1 tanh perceptron -> beta *= exp(ymax tanh(o));
//   a non-finite network output falls back to residual balancing.
// The features of every check are stored in sc->feat.
__device__ __forceinline__ void control_block(DevScalars* sc, double kkt, int32_t beta_mode, double rb_mu,
                                              double rb_tau, double tol, const float* __restrict__ w,
                                              double ymax, int decide, double* hist, int64_t hist_cap,
                                              int64_t hist_base) {
  __shared__ float f[RAC_MLP_IN];
  __shared__ float h1[RAC_MLP_HIDDEN];
  __shared__ float h2[RAC_MLP_HIDDEN];
  __shared__ double mult_sh;
  const int tid = threadIdx.x;
  const double rp = sc->rp, rd = sc->rd;
  const int status0 = sc->status;
  const bool conv = status0 == 0 && kkt <= tol;
  __syncthreads();   // every thread has read the scalars before thread 0 updates them
  if (tid == 0) {
    sc->kkt = kkt;
    const int64_t hi_ = sc->k - 1 - hist_base;
    if (hist && hi_ >= 0 && hi_ < hist_cap) hist[4 * hi_ + 3] = kkt;
    if (conv) sc->status = 1;
  }
  const bool act = decide && status0 == 0 && !conv &&
                   (beta_mode == RAC_BETA_RESBAL || beta_mode == RAC_BETA_MLP);
  if (tid == 0) {
    const double rpo = sc->rp_win, rdo = sc->rd_win, kp = sc->kkt_prev;
    f[0] = (float)clip4(0.5 * (lg10c(rp) - lg10c(rd)));
    f[1] = (float)clip4(0.5 * (lg10c(rpo) - lg10c(rdo)));
    f[2] = (float)clip4(lg10c(rp) - lg10c(rpo));
    f[3] = (float)clip4(lg10c(rd) - lg10c(rdo));
    f[4] = (float)clip4(kp > 0.0 ? lg10c(kkt) - lg10c(kp) : 0.0);
    f[5] = (float)clip4(sc->last_l10);
    f[6] = (float)clip4((lg10c(kkt) + 6.0) / 3.0);
    f[7] = (float)clip4((double)sc->decisions / 10.0);
    for (int q = 0; q < RAC_MLP_IN; ++q) sc->feat[q] = f[q];
  }
  __syncthreads();
  if (act) {
    double rb = 1.0;
    if (rp > rb_mu * rd) rb = rb_tau;
    else if (rd > rb_mu * rp) rb = 1.0 / rb_tau;
    if (beta_mode == RAC_BETA_RESBAL) {
      if (tid == 0) mult_sh = rb;
    } else {
      const float* W1 = w;
      const float* B1 = W1 + RAC_MLP_HIDDEN * RAC_MLP_IN;
      const float* W2 = B1 + RAC_MLP_HIDDEN;
      const float* B2 = W2 + RAC_MLP_HIDDEN * RAC_MLP_HIDDEN;
      const float* W3 = B2 + RAC_MLP_HIDDEN;
      const float* B3 = W3 + RAC_MLP_HIDDEN;
      float s = B1[tid];
      for (int k = 0; k < RAC_MLP_IN; ++k) s += W1[tid * RAC_MLP_IN + k] * f[k];
      h1[tid] = tanhf(s);
      __syncthreads();
      s = B2[tid];
      for (int k = 0; k < RAC_MLP_HIDDEN; ++k) s += W2[tid * RAC_MLP_HIDDEN + k] * h1[k];
      h2[tid] = tanhf(s);
      __syncthreads();
      float o = W3[tid] * h2[tid];
      for (int off = 32; off >= 1; off >>= 1) o += __shfl_xor(o, off, 64);
      if (tid == 0) {
        const double y = ymax * tanh((double)(o + B3[0]));
        mult_sh = isfinite(y) ? exp(y) : rb;
      }
    }
    __syncthreads();
    if (tid == 0) {
      sc->beta *= mult_sh;
      sc->last_l10 = log10(mult_sh);
      sc->decisions += 1;
    }
  }
  if (tid == 0) sc->kkt_prev = kkt;
}

}  // namespace rac
