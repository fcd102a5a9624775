/*
 * A plain C consumer of the library: solves the 2-D 5-point Dirichlet
 * Poisson problem on an m x m grid (symmetrically scaled to unit diagonal,
 * i.e. A/4) with Algorithm 5 through the C ABI alone, then recomputes the
 * relative residual ||b - A x|| / ||b|| on the host.  b = A x* with
 * x*_k = sin(k + 1), x0 = 0.  Device memory comes from the HIP runtime.
 *
 * Usage: poisson2d [m] [basis: c(hebyshev) | n(ewton)] [s_max]
 * Exit status 0 when the solve converged to tol = 1e-10 and the host
 * residual agrees, 1 otherwise.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "assg.h"

#define HIP_CHECK(call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));          \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

#define ASSG_CHECK(h, call)                                                      \
  do {                                                                           \
    assg_status_t s_ = (call);                                                   \
    if (s_ != ASSG_OK) {                                                         \
      fprintf(stderr, "%s: %s (%s)\n", #call, assg_status_string(s_),            \
              (h) ? assg_last_error(h) : "");                                    \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

int main(int argc, char** argv) {
  const int m = argc > 1 ? atoi(argv[1]) : 64;
  const int newton = argc > 2 && argv[2][0] == 'n';
  const int smax = argc > 3 ? atoi(argv[3]) : 10;
  if (m < 1 || m > 4096 || smax < 1 || smax > ASSG_MAX_S) {
    fprintf(stderr, "bad arguments\n");
    return 1;
  }
  const int64_t n = (int64_t)m * m;

  /* CSR of A/4: diagonal 1, neighbours -1/4, columns ascending per row */
  int32_t* rp = malloc((size_t)(n + 1) * sizeof(int32_t));
  int32_t* ci = malloc((size_t)5 * n * sizeof(int32_t));
  double* va = malloc((size_t)5 * n * sizeof(double));
  double* xs = malloc((size_t)n * sizeof(double));
  double* b = malloc((size_t)n * sizeof(double));
  double* x = malloc((size_t)n * sizeof(double));
  if (!rp || !ci || !va || !xs || !b || !x) return 1;
  int64_t nnz = 0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const int64_t r = (int64_t)i * m + j;
      rp[r] = (int32_t)nnz;
      if (i > 0) { ci[nnz] = (int32_t)(r - m); va[nnz++] = -0.25; }
      if (j > 0) { ci[nnz] = (int32_t)(r - 1); va[nnz++] = -0.25; }
      ci[nnz] = (int32_t)r; va[nnz++] = 1.0;
      if (j < m - 1) { ci[nnz] = (int32_t)(r + 1); va[nnz++] = -0.25; }
      if (i < m - 1) { ci[nnz] = (int32_t)(r + m); va[nnz++] = -0.25; }
    }
  rp[n] = (int32_t)nnz;
  for (int64_t k = 0; k < n; ++k) xs[k] = sin((double)(k + 1));
  for (int64_t r = 0; r < n; ++r) {
    double s = 0.0;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) s += va[e] * xs[ci[e]];
    b[r] = s;
  }

  int32_t *drp, *dci;
  double *dva, *db, *dx;
  HIP_CHECK(hipMalloc((void**)&drp, (size_t)(n + 1) * sizeof(int32_t)));
  HIP_CHECK(hipMalloc((void**)&dci, (size_t)nnz * sizeof(int32_t)));
  HIP_CHECK(hipMalloc((void**)&dva, (size_t)nnz * sizeof(double)));
  HIP_CHECK(hipMalloc((void**)&db, (size_t)n * sizeof(double)));
  HIP_CHECK(hipMalloc((void**)&dx, (size_t)n * sizeof(double)));
  HIP_CHECK(hipMemcpy(drp, rp, (size_t)(n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_CHECK(hipMemcpy(dci, ci, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_CHECK(hipMemcpy(dva, va, (size_t)nnz * sizeof(double), hipMemcpyHostToDevice));
  HIP_CHECK(hipMemcpy(db, b, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
  HIP_CHECK(hipMemset(dx, 0, (size_t)n * sizeof(double)));

  assg_handle_t h = NULL;
  ASSG_CHECK(h, assg_create(&h, NULL));
  const assg_csr_t A = {n, nnz, drp, dci, dva};
  ASSG_CHECK(h, assg_analyze(h, &A));
  assg_opts_t o;
  ASSG_CHECK(h, assg_default_opts(&o));
  o.s_max = smax;
  o.s_init = smax;
  o.growth = smax;
  o.tol = 1e-10;
  o.basis = newton ? ASSG_BASIS_NEWTON : ASSG_BASIS_CHEBYSHEV;
  assg_info_t info;
  ASSG_CHECK(h, assg_solve(h, &A, db, dx, &o, NULL, 0, &info));
  HIP_CHECK(hipMemcpy(x, dx, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));

  double rr = 0.0, bb = 0.0, ee = 0.0, xx = 0.0;
  for (int64_t r = 0; r < n; ++r) {
    double s = 0.0;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) s += va[e] * x[ci[e]];
    rr += (b[r] - s) * (b[r] - s);
    bb += b[r] * b[r];
    ee += (x[r] - xs[r]) * (x[r] - xs[r]);
    xx += xs[r] * xs[r];
  }
  const double relres = sqrt(rr / bb);
  printf("poisson2d m=%d n=%lld nnz=%lld basis=%s s_max=%d: outcome=%s outer=%lld iters=%lld "
         "relres(host)=%.3e relres(lib)=%.3e err=%.3e\n",
         m, (long long)n, (long long)nnz, newton ? "newton" : "chebyshev", smax,
         info.outcome == ASSG_CONVERGED ? "CONVERGED" : "not converged",
         (long long)info.outer_iters, (long long)info.total_iters, relres, info.relres_true,
         sqrt(ee / xx));

  ASSG_CHECK(h, assg_destroy(h));
  hipFree(drp); hipFree(dci); hipFree(dva); hipFree(db); hipFree(dx);
  free(rp); free(ci); free(va); free(xs); free(b); free(x);
  const int ok = info.outcome == ASSG_CONVERGED && relres <= 1e-10 &&
                 fabs(relres - info.relres_true) <= 1e-3 * relres + 1e-300;
  return ok ? 0 : 1;
}
