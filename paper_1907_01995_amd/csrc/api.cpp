// api.cpp -- one-call entry points of racmb.h built on the handle API
// (rac_solve, rac_solve_batch) and the host form of the partition draw
// (rac_permutation_host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "rac_internal.h"
#include "racmb.h"

extern "C" {

rac_status rac_solve(const rac_problem* prob, const rac_opts* opts, void* stream, double* x, double* z,
                     double* xi, double* mu, rac_result* res) {
  if (!res) return RAC_ERR_ARG;
  rac_solver s = nullptr;
  rac_status r = rac_solver_create(prob, opts, &s);
  if (r != RAC_OK) return r;
  const rac_status rr = rac_solver_run(s, stream, res);
  if (rr == RAC_OK || rr == RAC_ERR_NOT_PD) {
    double m = 0.0, beta = 0.0;
    int64_t it = 0;
    r = rac_solver_get_state(s, x, z, xi, &m, &beta, &it, stream);
    if (r == RAC_OK && mu) *mu = m;
  }
  rac_solver_destroy(s);
  return rr != RAC_OK ? rr : r;
}

rac_status rac_solve_batch(int32_t ninst, const rac_problem* inst, int32_t nlanes, const rac_lane* lanes,
                           const rac_batch_opts* opts, void* stream, double* x, double* z, double* xi,
                           rac_result* res) {
  if (!res || !lanes || !inst || nlanes < 1 || ninst < 1) return RAC_ERR_ARG;
  for (int32_t u = 0; u < nlanes; ++u)
    if (lanes[u].problem < 0 || lanes[u].problem >= ninst) return RAC_ERR_ARG;
  rac_batch b = nullptr;
  rac_status r = rac_batch_create(ninst, inst, nlanes, lanes, opts, &b);
  if (r != RAC_OK) return r;
  int64_t iters = 0;
  int32_t active = 0;
  r = rac_batch_run(b, stream, &iters, &active);
  if (r == RAC_OK) {
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) r = RAC_ERR_DEVICE;
  }
  int64_t off = 0;
  rac_status lane_status = RAC_OK;
  for (int32_t u = 0; u < nlanes && r == RAC_OK; ++u) {
    const rac_status q = rac_batch_lane(b, u, res + u, x ? x + off : nullptr, z ? z + off : nullptr,
                                        xi ? xi + off : nullptr);
    if (q == RAC_ERR_NOT_PD) lane_status = RAC_ERR_NOT_PD;
    else if (q != RAC_OK) r = q;
    off += inst[lanes[u].problem].n;
  }
  rac_batch_destroy(b);
  return r != RAC_OK ? r : lane_status;
}

rac_status rac_permutation_host(uint64_t seed, uint64_t instance, int64_t iter, int64_t n, int32_t* perm) {
  if (n < 1 || n > (int64_t)INT32_MAX || !perm || iter < 0) return RAC_ERR_ARG;
  std::vector<uint64_t> key((size_t)n);
  for (int64_t j = 0; j < n; ++j) key[(size_t)j] = rac::perm_key(seed, instance, (uint64_t)iter, (uint64_t)j);
  for (int64_t j = 0; j < n; ++j) perm[j] = (int32_t)j;
  // ascending (key, index): the same total order as the device's bucket sort
  std::sort(perm, perm + n, [&](int32_t a, int32_t b) {
    return key[(size_t)a] < key[(size_t)b] || (key[(size_t)a] == key[(size_t)b] && a < b);
  });
  return RAC_OK;
}

}  // extern "C"
