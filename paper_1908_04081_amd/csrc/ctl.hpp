// Device control block of one solve and helpers shared by host and device.
//
// All decisions of Algorithm 5 (s-bar, s~, s_k, alpha/beta, the Ritz
// estimates, c, the basis parameters, convergence) live in this block in
// device memory; kernels read what they need from it, so an outer loop is
// enqueued without any host round trip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "assg.h"

namespace assg {

constexpr int MAXS = ASSG_MAX_S;
constexpr int MAXC = ASSG_MAX_COLS;   // 2*MAXS+1 basis columns
constexpr double UNIT_ROUNDOFF = 0x1p-53;   // eps of Section 5 (~2^-53)

// Status values share the public outcome codes; RUNNING while iterating.
constexpr int ST_RUNNING = ASSG_RUNNING;

struct alignas(256) Ctl {
  // ---------------------------------------------------------------- state
  int32_t status;        // committed outcome; kernels do nothing unless RUNNING
  int32_t pending;       // outcome decided inside the loop, committed at its end
  int32_t k;             // outer loops completed
  int32_t sbar;          // basis levels of the current loop
  int32_t sbar_next;     // s-bar of the next loop (committed at loop end)
  int32_t stilde, sk;    // s~ and s_k of the current loop
  int32_t candidate;     // updated residual reached tol in this loop
  int32_t skip_recover;  // breakdown/divergence: leave x, r, p untouched
  int32_t fail_streak;   // failed true-residual confirmations
  int32_t flags;
  int32_t mode;          // 0: s-step, 1: HSCG
  int32_t variant;       // assg_variant_t
  int64_t m;             // inner iterations done

  // -------------------------------------------------------------- options
  int32_t sigma, growth, basis, record_trace;
  int64_t trace_cap, max_outer, max_iters;
  const int32_t* forced_sk;   // test hook: s_k of every loop given (device), else null
  int64_t forced_len;
  double tol;
  double c_const;        // c of the old adaptive method

  // -------------------------------------------------------------- scalars
  double nb;             // ||b||
  double c, psi;         // (4.6), (4.5)
  double lmin, lmax;     // Algorithm 4 / 3 estimates
  double alpha_prev, beta_prev;
  double mx_omega, mx_h, mx_zeta;                 // Algorithm 3 state
  double mn_omega, mn_a, mn_d, mn_g, mn_h;        // Algorithm 4 state
  double best_true, relres_true, relres_upd, phi, thr, rho_m;
  double h_rho, h_alpha, h_beta;                  // HSCG scalars

  // ---------------------------------------------------- basis parameters
  double theta[MAXS], gamma[MAXS], mu[MAXS];
  double leja[MAXS];     // Leja points of [-1, 1], order of (2.7)

  // ------------------------------------------- results of the current loop
  double cx[MAXC], cr[MAXC], cp[MAXC];            // x', r', p' (interleaved)
  double alphas[MAXS], betas[MAXS], kappa[MAXS];

  // ------------------------------------------------------------- the Gram
  double G[MAXC * MAXC];                          // row-major, interleaved order

};

// Basis parameters of (2.3) for s levels (Section 2 monomial, (2.7) Newton,
// (2.8) Chebyshev read as the Chebyshev recurrence of [lmin, lmax]).
__host__ __device__ inline void basis_params(int kind, double lmin, double lmax, int s,
                                             const double* leja, double* th, double* ga,
                                             double* mu) {
  const double c = 0.5 * (lmin + lmax);
  const double h = 0.5 * (lmax - lmin);
  const double d = lmax - lmin;
  for (int l = 0; l < s; ++l) {
    if (kind == ASSG_BASIS_NEWTON) {
      th[l] = (l == 0) ? lmax : (l == 1 ? lmin : c + h * leja[l]);
      ga[l] = 1.0;
      if (l + 1 < s) mu[l] = 0.0;
    } else if (kind == ASSG_BASIS_CHEBYSHEV) {
      th[l] = c;
      ga[l] = (l == 0) ? 0.5 * d : 0.25 * d;
      if (l + 1 < s) mu[l] = 0.25 * d;
    } else {
      th[l] = 0.0;
      ga[l] = 1.0;
      if (l + 1 < s) mu[l] = 0.0;
    }
  }
}

}  // namespace assg
