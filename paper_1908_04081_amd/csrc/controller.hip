// Controller of one outer loop of Algorithm 5, one workgroup, FP64.
//
// Wave w (w < s-bar) estimates kappa(Y_{k,w+1}) ~ sqrt(kappa(G_{w+1})) from
// the leading (2w+3)x(2w+3) block of G (Section 3): Householder
// tridiagonalization in LDS, then Sturm-count multisection for the smallest
// and largest eigenvalue.  Wave 0 then selects s~ by (3.2), runs the inner
// loop with alpha and beta through G and the change of basis B (2.5), phi,
// psi (4.5), the Ritz estimates of Algorithms 3 and 4, c (4.6), the break
// rule (4.7) and the stopping candidate, and finally sets the recovery
// coordinates, m, s-bar of the next loop and the next basis parameters
// ((2.7)/(2.8), once m > 1).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "launch.hpp"

namespace assg {

__host__ __device__ constexpr int scratch_offset(int l) {
  int o = 0;
  for (int j = 1; j < l; ++j) o += (2 * j + 1) * (2 * j + 1);
  return o;
}
constexpr int SCRATCH = scratch_offset(MAXS + 1);

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x.
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x,
                                           double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// sqrt(lambda_max / lambda_min) of the symmetric n x n matrix T (row-major,
// LDS, destroyed); +inf when lambda_min <= 0.  One wave; scratch vectors
// v, w, d, e2 hold MAXC doubles each.
__device__ double kappa_wave(double* T, int n, int lane, double* v, double* w, double* d,
                             double* e2) {
  // Householder reduction to tridiagonal form
  for (int k = 0; k + 2 < n; ++k) {
    const int m0 = k + 1;
    const bool in = (lane >= m0) && (lane < n);
    const double xi = in ? T[lane * n + k] : 0.0;
    const double x0 = T[m0 * n + k];
    const double ss = wave_sum((lane > m0 && lane < n) ? xi * xi : 0.0);
    if (lane == 0) d[k] = T[k * n + k];
    if (ss == 0.0) {
      if (lane == 0) e2[k] = x0 * x0;
      wave_lds_sync();
      continue;
    }
    const double nrm = sqrt(x0 * x0 + ss);
    const double alpha = (x0 > 0.0) ? -nrm : nrm;
    const double vi = in ? (lane == m0 ? x0 - alpha : xi) : 0.0;
    const double vtv = (x0 - alpha) * (x0 - alpha) + ss;
    const double beta = 2.0 / vtv;
    if (lane < MAXC) v[lane] = vi;
    wave_lds_sync();
    double pi = 0.0;
    if (in)
      for (int j = m0; j < n; ++j) pi = fma(T[lane * n + j], v[j], pi);
    pi *= beta;
    const double K = 0.5 * beta * wave_sum(pi * vi);
    const double wi = pi - K * vi;
    if (lane < MAXC) w[lane] = wi;
    wave_lds_sync();
    if (in)
      for (int j = m0; j < n; ++j) T[lane * n + j] -= vi * w[j] + wi * v[j];
    if (lane == 0) e2[k] = alpha * alpha;
    wave_lds_sync();
  }
  if (lane == 0) {
    d[n - 2] = T[(n - 2) * n + (n - 2)];
    const double el = T[(n - 1) * n + (n - 2)];
    e2[n - 2] = el * el;
    d[n - 1] = T[(n - 1) * n + (n - 1)];
  }
  wave_lds_sync();

  // Gershgorin interval and pivot guard
  double glo = INFINITY, ghi = -INFINITY, emax = 0.0;
  if (lane < n) {
    const double el = (lane > 0) ? sqrt(e2[lane - 1]) : 0.0;
    const double er = (lane < n - 1) ? sqrt(e2[lane]) : 0.0;
    glo = d[lane] - el - er;
    ghi = d[lane] + el + er;
    emax = (lane < n - 1) ? e2[lane] : 0.0;
  }
  glo = wave_min(glo);
  ghi = wave_max(ghi);
  emax = wave_max(emax);
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
  const double pad = 4.0 * UNIT_ROUNDOFF * fmax(fabs(glo), fabs(ghi)) + pivmin;
  glo -= pad;
  ghi += pad;

  // multisection: lanes 0..31 bracket lambda_min, lanes 32..63 lambda_max
  double loA = glo, hiA = ghi, loB = glo, hiB = ghi;
  const int j = lane & 31;
  const bool first = lane < 32;
  for (int it = 0; it < 16; ++it) {
    const double L = first ? loA : loB;
    const double H = first ? hiA : hiB;
    const double x = L + (H - L) * (double)(j + 1) / 33.0;
    const int target = first ? 1 : n;
    const bool ok = sturm_count(d, e2, n, x, pivmin) >= target;
    const uint64_t mask = __ballot(ok);
    const uint32_t ma = (uint32_t)(mask & 0xffffffffu), mb = (uint32_t)(mask >> 32);
    if (ma == 0u) {
      loA = loA + (hiA - loA) * 32.0 / 33.0;
    } else {
      const int j0 = __builtin_ctz(ma);
      const double nh = loA + (hiA - loA) * (double)(j0 + 1) / 33.0;
      const double nl = (j0 > 0) ? loA + (hiA - loA) * (double)j0 / 33.0 : loA;
      loA = nl;
      hiA = nh;
    }
    if (mb == 0u) {
      loB = loB + (hiB - loB) * 32.0 / 33.0;
    } else {
      const int j0 = __builtin_ctz(mb);
      const double nh = loB + (hiB - loB) * (double)(j0 + 1) / 33.0;
      const double nl = (j0 > 0) ? loB + (hiB - loB) * (double)j0 / 33.0 : loB;
      loB = nl;
      hiB = nh;
    }
    if (hiA - loA <= 2.0 * UNIT_ROUNDOFF * fmax(fabs(loA), fabs(hiA)) &&
        hiB - loB <= 2.0 * UNIT_ROUNDOFF * fmax(fabs(loB), fabs(hiB)))
      break;
  }
  const double lmin = 0.5 * (loA + hiA);
  const double lmax = 0.5 * (loB + hiB);
  if (!(lmin > 0.0) || !isfinite(lmin) || !isfinite(lmax)) return INFINITY;
  return sqrt(lmax / lmin);
}

// (B v)_i for the change of basis (2.5) of s~ levels, interleaved order:
// P_j = 2j, R_j = 2j+1; block column j holds theta_j (diagonal), gamma_j
// (next level), mu_{j-1} (previous level); the last P and last R columns are 0.
__device__ __forceinline__ double apply_B(const double* v, int st, int lane, const double* th,
                                          const double* ga, const double* mu) {
  const int n = 2 * st + 1;
  if (lane >= n) return 0.0;
  const int j = lane >> 1;
  const int lastcol = (lane & 1) ? st - 2 : st - 1;
  double r = 0.0;
  if (j >= 1 && j - 1 <= lastcol) r = fma(ga[j - 1], v[lane - 2], r);
  if (j <= lastcol) r = fma(th[j], v[lane], r);
  if (j + 1 <= lastcol) r = fma(mu[j], v[lane + 2], r);
  return r;
}

// (G v)_lane over the leading n entries.
__device__ __forceinline__ double gmv(const double* G, const double* v, int n, int lane) {
  double s = 0.0;
  if (lane < n)
    for (int c = 0; c < n; ++c) s = fma(G[lane * MAXC + c], v[c], s);
  return s;
}

__global__ __launch_bounds__(1024) void k_controller(Ctl* __restrict__ ctl,
                                                     assg_trace_t* __restrict__ trace) {
  if (ctl->status != ST_RUNNING) return;
  __shared__ double sG[MAXC * MAXC];
  __shared__ double sScr[SCRATCH];
  __shared__ double sVec[MAXS][4][MAXC];
  __shared__ double sKappa[MAXS + 2];
  __shared__ double sTh[MAXS], sGa[MAXS], sMu[MAXS];
  __shared__ double vp[MAXC], vr[MAXC], vx[MAXC], vt[MAXC];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int sbar = ctl->sbar;
  const int nc = 2 * sbar + 1;
  for (int i = tid; i < nc * nc; i += blockDim.x) {
    const int a = i / nc, b = i % nc;
    sG[a * MAXC + b] = ctl->G[a * MAXC + b];
  }
  if (tid < MAXS) {
    sTh[tid] = ctl->theta[tid];
    sGa[tid] = ctl->gamma[tid];
    sMu[tid] = ctl->mu[tid];
  }
  if (tid < MAXS + 2) sKappa[tid] = INFINITY;
  __syncthreads();

  // ---- kappa(Y_{k,l}) for l = 1..sbar, one wave each
  if (wave < sbar) {
    const int l = wave + 1, n = 2 * l + 1;
    double* T = sScr + scratch_offset(l);
    for (int i = lane; i < n * n; i += 64) T[i] = sG[(i / n) * MAXC + (i % n)];
    wave_lds_sync();
    const double kap = kappa_wave(T, n, lane, sVec[wave][0], sVec[wave][1], sVec[wave][2],
                                  sVec[wave][3]);
    if (lane == 0) sKappa[l] = kap;
  }
  __syncthreads();
  if (wave != 0) return;

  // ---- s~ by (3.2) with the current c and relative ||r_m||
  const double u = UNIT_ROUNDOFF;
  const double nb = ctl->nb, tol = ctl->tol;
  double c = ctl->c;
  const double rGr0 = fmax(sG[1 * MAXC + 1], 0.0);
  const double rho_m = sqrt(rGr0) / nb;
  const double thr = (rho_m > 0.0) ? tol / (c * u * rho_m) : INFINITY;
  int st = 1;
  for (int l = 1; l <= sbar; ++l) {
    if (sKappa[l] <= thr)
      st = l;
    else
      break;
  }
  const int n = 2 * st + 1;

  // ---- inner loop (interleaved coordinates; lane i owns coordinate i)
  if (lane < MAXC) {
    vp[lane] = (lane == 0) ? 1.0 : 0.0;
    vr[lane] = (lane == 1) ? 1.0 : 0.0;
    vx[lane] = 0.0;
  }
  wave_lds_sync();
  double rGr = rGr0;
  double phi = sqrt(rGr) / nb;
  double psi = ctl->psi;
  double lmin = ctl->lmin, lmax = ctl->lmax;
  double alpha_prev = ctl->alpha_prev, beta_prev = ctl->beta_prev;
  double mx_omega = ctl->mx_omega, mx_h = ctl->mx_h, mx_zeta = ctl->mx_zeta;
  double mn_omega = ctl->mn_omega, mn_a = ctl->mn_a, mn_d = ctl->mn_d, mn_g = ctl->mn_g,
         mn_h = ctl->mn_h;
  const int64_t m = ctl->m;
  int sk = 0, candidate = 0, outcome = ST_RUNNING;
  for (int j = 0; j < st; ++j) {
    sk = j + 1;
    const double bp = apply_B(vp, st, lane, sTh, sGa, sMu);
    if (lane < MAXC) vt[lane] = bp;
    wave_lds_sync();
    const double gb = gmv(sG, vt, n, lane);
    const double den = wave_sum(lane < n ? vp[lane] * gb : 0.0);
    if (!isfinite(den)) { outcome = ASSG_DIVERGED; break; }
    if (den <= 0.0 || rGr <= 0.0) { outcome = ASSG_BREAKDOWN; break; }
    const double alpha = rGr / den;
    const double q = (lane < n) ? alpha * vp[lane] : 0.0;
    wave_lds_sync();
    if (lane < MAXC) {
      vx[lane] += q;
      vt[lane] = q;
    }
    wave_lds_sync();
    const double bq = apply_B(vt, st, lane, sTh, sGa, sMu);
    const double rnew = (lane < n) ? vr[lane] - bq : 0.0;
    wave_lds_sync();
    if (lane < MAXC) vr[lane] = rnew;
    wave_lds_sync();
    const double gr = gmv(sG, vr, n, lane);
    const double rGr_new = fmax(wave_sum(lane < n ? rnew * gr : 0.0), 0.0);
    const double beta = rGr_new / rGr;
    const double pnew = (lane < n) ? rnew + beta * vp[lane] : 0.0;
    wave_lds_sync();
    if (lane < MAXC) vp[lane] = pnew;
    wave_lds_sync();
    rGr = rGr_new;
    const double rho = sqrt(rGr) / nb;
    phi = fmax(phi, rho);
    psi = psi / (psi + beta);                               // (4.5)
    const int64_t i = m + j;                                // global iteration index
    const double zeta = 1.0 / sqrt(alpha);                  // (4.1)
    if (i == 0) {
      mx_omega = zeta * zeta; mx_h = 1.0; mx_zeta = zeta;   // Algorithm 3 start
      mn_omega = 1.0 / (zeta * zeta); mn_a = mn_omega;      // Algorithm 4 start
      mn_d = 0.0; mn_g = 0.0; mn_h = 1.0;
    } else {
      const double eta = sqrt(beta_prev / alpha_prev);
      {  // Algorithm 3 step (a uses zeta_{l+1})
        const double dd = mx_zeta * mx_zeta * eta * eta * mx_h;
        const double a = eta * eta + zeta * zeta;
        const double chi = sqrt((mx_omega - a) * (mx_omega - a) + 4.0 * dd);
        const double h = (chi == 0.0) ? 0.0 : 0.5 * (1.0 - (mx_omega - a) / chi);
        mx_omega = mx_omega + chi * h;
        mx_h = h;
        mx_zeta = zeta;
      }
      {  // Algorithm 4 step
        const double dd = -(eta / zeta) * (mn_g * mn_d + mn_h * mn_a);
        const double a = (eta * eta * mn_a + 1.0) / (zeta * zeta);
        const double chi = sqrt((mn_omega - a) * (mn_omega - a) + 4.0 * dd * dd);
        const double h = (chi == 0.0) ? 0.0 : sqrt(fmax(0.0, 0.5 * (1.0 - (mn_omega - a) / chi)));
        mn_omega = mn_omega + chi * h * h;
        mn_g = sqrt(fmax(0.0, 1.0 - h * h));
        mn_h = fabs(h) * (dd < 0.0 ? -1.0 : 1.0);
        mn_d = dd;
        mn_a = a;
      }
      lmax = mx_omega;
      lmin = 1.0 / mn_omega;
      c = fmax(1.0, lmax * sqrt(psi / lmin));               // (4.6)
    }
    alpha_prev = alpha;
    beta_prev = beta;
    if (lane == 0 && j < MAXS) {
      ctl->alphas[j] = alpha;
      ctl->betas[j] = beta;
    }
    if (!isfinite(alpha) || !isfinite(beta)) { outcome = ASSG_DIVERGED; break; }
    if (rho <= tol) { candidate = 1; break; }
    if (j < st - 1 && sKappa[j + 2] >= tol / (c * u * phi)) break;   // (4.7), gamma_{j+1}
  }

  // ---- results
  if (lane < MAXC) {
    const bool keep = lane < n;
    ctl->cx[lane] = keep ? vx[lane] : 0.0;
    ctl->cr[lane] = keep ? vr[lane] : 0.0;
    ctl->cp[lane] = keep ? vp[lane] : 0.0;
  }
  if (lane < MAXS) ctl->kappa[lane] = (lane < sbar) ? sKappa[lane + 1] : 0.0;
  if (lane == 0) {
    const int64_t k = ctl->k;
    ctl->stilde = st;
    ctl->thr = thr;
    ctl->rho_m = rho_m;
    ctl->phi = phi;
    ctl->relres_upd = sqrt(rGr) / nb;
    if (ctl->record_trace && k < ctl->trace_cap) {
      assg_trace_t& tr = trace[k];
      tr.k = (int32_t)k;
      tr.sbar = sbar;
      tr.stilde = st;
      tr.sk = sk;
      tr.m = m;
      tr.candidate = candidate;
      tr.flags = (outcome == ASSG_BREAKDOWN ? 1 : 0) | (outcome == ASSG_DIVERGED ? 2 : 0);
      tr.c_in = ctl->c;
      tr.thr = thr;
      tr.rho_m = rho_m;
      tr.phi = phi;
      tr.c = c;
      tr.lmin = lmin;
      tr.lmax = lmax;
      tr.psi = psi;
      tr.relres_updated = sqrt(rGr) / nb;
      tr.relres_true = -1.0;
      for (int l = 0; l < MAXS; ++l) tr.kappa[l] = (l < sbar) ? sKappa[l + 1] : 0.0;
    }
    if (outcome != ST_RUNNING) {
      ctl->pending = outcome;
      ctl->skip_recover = 1;
      ctl->sk = sk;
      ctl->candidate = 0;
    } else {
      const int64_t m_new = m + sk;
      ctl->sk = sk;
      ctl->candidate = candidate;
      ctl->m = m_new;
      ctl->c = c;
      ctl->psi = psi;
      ctl->lmin = lmin;
      ctl->lmax = lmax;
      ctl->alpha_prev = alpha_prev;
      ctl->beta_prev = beta_prev;
      ctl->mx_omega = mx_omega; ctl->mx_h = mx_h; ctl->mx_zeta = mx_zeta;
      ctl->mn_omega = mn_omega; ctl->mn_a = mn_a; ctl->mn_d = mn_d;
      ctl->mn_g = mn_g; ctl->mn_h = mn_h;
      const int sn = sk + ctl->growth;
      ctl->sbar_next = sn < ctl->sigma ? sn : ctl->sigma;
      // dynamic basis update once two iterations are done (Algorithm 5)
      if (m_new > 1 && isfinite(lmin) && isfinite(lmax) && lmax - lmin > 0.0)
        basis_params(ctl->basis, lmin, lmax, ctl->sigma, ctl->leja, ctl->theta, ctl->gamma,
                     ctl->mu);
      if (!candidate && (m_new >= ctl->max_iters || k + 1 >= ctl->max_outer))
        ctl->pending = ASSG_MAX_ITER;
    }
  }
}

void launch_controller(hipStream_t s, Ctl* ctl, assg_trace_t* trace, int sigma) {
  const int waves = sigma < 1 ? 1 : sigma;
  hipLaunchKernelGGL(k_controller, dim3(1), dim3(64 * waves), 0, s, ctl, trace);
}

}  // namespace assg
