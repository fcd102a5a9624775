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

__host__ __device__ constexpr int scratch_offset(int l) {   // rows of the blocks before block l
  int o = 0;
  for (int j = 1; j < l; ++j) o += 2 * j + 1;
  return o;
}
constexpr int SCRATCH_ROWS = scratch_offset(MAXS + 1);   // 288 rows of MAXC doubles

// sqrt(lambda_max / lambda_min) of the symmetric n x n matrix T (LDS, row
// stride MAXC, columns n..MAXC-1 zero, destroyed); +inf when lambda_min <= 0.
// One wave: Householder reduction to tridiagonal form (lane i owns row i;
// vectors are held one entry per lane and broadcast with readlane), then
// Sturm-count multisection for the two extreme eigenvalues (lanes 0..31
// bracket lambda_min, lanes 32..63 lambda_max, 33 sub-intervals per round)
// down to a width of 2u times the Gershgorin scale, the accuracy any
// backward-stable eigensolver attains.
template <int N>
__device__ double kappa_wave(double* T, int lane, double* dsh, double* esh) {
  constexpr int n = N;
  const int rowoff = (lane < n ? lane : 0) * MAXC;
  for (int k = 0; k + 2 < n; ++k) {
    const int m0 = k + 1;
    const bool in = (lane >= m0) && (lane < n);
    const double xi = in ? T[rowoff + k] : 0.0;
    const double x0 = readlane_d(xi, m0);
    const double ss = wave_sum_dpp((lane > m0 && lane < n) ? xi * xi : 0.0);
    if (lane == 0) dsh[k] = T[k * MAXC + k];
    if (ss == 0.0) {
      if (lane == 0) esh[k] = x0 * x0;
      continue;
    }
    const double nrm = sqrt(x0 * x0 + ss);
    const double alpha = (x0 > 0.0) ? -nrm : nrm;
    const double vi = in ? (lane == m0 ? x0 - alpha : xi) : 0.0;
    const double beta = 2.0 / ((x0 - alpha) * (x0 - alpha) + ss);
    double pa[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < N; ++j) pa[j & 3] = fma(T[rowoff + j], readlane_d(vi, j), pa[j & 3]);
    double pi = (pa[0] + pa[1]) + (pa[2] + pa[3]);
    pi = in ? pi * beta : 0.0;
    const double K = 0.5 * beta * wave_sum_dpp(pi * vi);
    const double wi = pi - K * vi;
    if (in) {
#pragma unroll
      for (int j = 0; j < N; ++j)
        T[rowoff + j] -= vi * readlane_d(wi, j) + wi * readlane_d(vi, j);
    }
    if (lane == 0) esh[k] = alpha * alpha;
    wave_lds_sync();
  }
  if (lane == 0) {
    dsh[n - 2] = T[(n - 2) * MAXC + (n - 2)];
    const double el = T[(n - 1) * MAXC + (n - 2)];
    esh[n - 2] = el * el;
    dsh[n - 1] = T[(n - 1) * MAXC + (n - 1)];
  }
  wave_lds_sync();

  double glo = INFINITY, ghi = -INFINITY, emax = 0.0;
  if (lane < n) {
    const double el = (lane > 0) ? sqrt(esh[lane - 1]) : 0.0;
    const double er = (lane < n - 1) ? sqrt(esh[lane]) : 0.0;
    glo = dsh[lane] - el - er;
    ghi = dsh[lane] + el + er;
    emax = (lane < n - 1) ? esh[lane] : 0.0;
  }
  glo = wave_min_dpp(glo);
  ghi = wave_max_dpp(ghi);
  emax = wave_max_dpp(emax);
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
  const double scale = fmax(fabs(glo), fabs(ghi));
  const double pad = 4.0 * UNIT_ROUNDOFF * scale + pivmin;
  glo -= pad;
  ghi += pad;
  const double width = 2.0 * UNIT_ROUNDOFF * scale + pivmin;

  // the tridiagonal in registers, entry i in lane i, broadcast by readlane
  const double dl = (lane < n) ? dsh[lane] : 0.0;
  const double el2 = (lane < n - 1) ? esh[lane] : 0.0;
  double loA = glo, hiA = ghi, loB = glo, hiB = ghi;
  const int j = lane & 31;
  const bool first = lane < 32;
  for (int it = 0; it < 16; ++it) {
    const double L = first ? loA : loB;
    const double H = first ? hiA : hiB;
    const double x = L + (H - L) * (double)(j + 1) * (1.0 / 33.0);
    const int target = first ? 1 : n;
    double q = readlane_d(dl, 0) - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
#pragma unroll
    for (int i = 1; i < N; ++i) {
      double rq = __builtin_amdgcn_rcp(q);            // ~26-bit seed
      rq = fma(rq, fma(-q, rq, 1.0), rq);               // one Newton step: ~full precision
      q = (readlane_d(dl, i) - x) - readlane_d(el2, i - 1) * rq;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    const uint64_t mask = __ballot(cnt >= target);
    const uint32_t ma = (uint32_t)(mask & 0xffffffffu), mb = (uint32_t)(mask >> 32);
    if (ma == 0u) {
      loA = loA + (hiA - loA) * (32.0 / 33.0);
    } else {
      const int j0 = __builtin_ctz(ma);
      const double nh = loA + (hiA - loA) * (double)(j0 + 1) * (1.0 / 33.0);
      const double nl = (j0 > 0) ? loA + (hiA - loA) * (double)j0 * (1.0 / 33.0) : loA;
      loA = nl;
      hiA = nh;
    }
    if (mb == 0u) {
      loB = loB + (hiB - loB) * (32.0 / 33.0);
    } else {
      const int j0 = __builtin_ctz(mb);
      const double nh = loB + (hiB - loB) * (double)(j0 + 1) * (1.0 / 33.0);
      const double nl = (j0 > 0) ? loB + (hiB - loB) * (double)j0 * (1.0 / 33.0) : loB;
      loB = nl;
      hiB = nh;
    }
    if (hiA - loA <= width && hiB - loB <= width) break;
  }
  const double lmin = 0.5 * (loA + hiA);
  const double lmax = 0.5 * (loB + hiB);
  if (!(lmin > 0.0) || !isfinite(lmin) || !isfinite(lmax)) return INFINITY;
  return sqrt(lmax / lmin);
}

// (B v)_i for the change of basis (2.5) of s~ levels, interleaved order:
// P_j = 2j, R_j = 2j+1; block column j holds theta_j (diagonal), gamma_j
// (next level), mu_{j-1} (previous level); the last P and last R columns
// are 0.  Lane i holds v_i; neighbours two lanes away come by shuffles.
__device__ __forceinline__ double apply_B(double v, int st, int lane, const double* th,
                                          const double* ga, const double* mu) {
  const double vm2 = __shfl_up(v, 2, 64);
  const double vp2 = __shfl_down(v, 2, 64);
  const int n = 2 * st + 1;
  if (lane >= n) return 0.0;
  const int j = lane >> 1;
  const int lastcol = (lane & 1) ? st - 2 : st - 1;
  double r = 0.0;
  if (j >= 1 && j - 1 <= lastcol) r = fma(ga[j - 1], vm2, r);
  if (j <= lastcol) r = fma(th[j], v, r);
  if (j + 1 <= lastcol) r = fma(mu[j], vp2, r);
  return r;
}

// (G v)_lane with lane i holding row i of G in registers and v_i.
__device__ __forceinline__ double gmv(const double* grow, double v) {
  double s = 0.0;   // column order, one chain (as a row of a plain matrix-vector product)
#pragma unroll
  for (int c = 0; c < MAXC; ++c) s = fma(grow[c], readlane_d(v, c), s);
  return s;
}

constexpr int CTL_WAVES = 12;  // wave 0: the inner loop; the others: kappa of the leading blocks

// Scalars of the inner loop after each step (one record per step).
enum StepScalar {
  SS_RGR, SS_PHI, SS_PSI, SS_LMIN, SS_LMAX, SS_C, SS_ALPHA, SS_BETA, SS_RHO,
  SS_MXO, SS_MXH, SS_MXZ, SS_MNO, SS_MNA, SS_MND, SS_MNG, SS_MNH, SS_N
};
// How the speculative inner loop ended at its last recorded step.
enum StepEvent { EV_NONE = 0, EV_BREAKDOWN, EV_DIVERGED_DEN, EV_DIVERGED, EV_CANDIDATE };

// Inner step j of Algorithm 5 works in span Y_{k,j+2} only: its coordinate
// vectors have support on the leading 2j+1 (p') and 2j+3 (r') coordinates,
// so it never reaches the last P and R columns of Y_{k,s~} (whose images B
// drops) for j < s~, and its result does not depend on s~.  Wave 0 runs the
// steps on the whole basis (s-bar levels) while the other waves estimate
// kappa; once s~ is known, the break (4.7) and the stopping test pick s_k
// among the recorded steps.
__global__ __launch_bounds__(64 * CTL_WAVES) void k_controller(Ctl* __restrict__ ctls,
                                                     assg_trace_t* __restrict__ trace) {
  Ctl* __restrict__ ctl = ctls + blockIdx.x;   // one workgroup per system
  if (ctl->status != ST_RUNNING) return;
  __shared__ double sG[MAXC * MAXC];
  __shared__ double sScr[SCRATCH_ROWS * MAXC];
  __shared__ double sDE[MAXS][2][MAXC];
  __shared__ double sKappa[MAXS + 2];
  __shared__ double sTh[MAXS], sGa[MAXS], sMu[MAXS];
  __shared__ double sVec[MAXS][3][MAXC];      // x', r', p' after each step
  __shared__ double sStep[MAXS][SS_N];        // scalars after each step
  __shared__ int sEvent[2];                   // steps recorded, event of the last one

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nwaves = blockDim.x >> 6;
  const int sbar = ctl->sbar;
  const int nc = 2 * sbar + 1;
  ASSG_DCHECK(sbar >= 1 && sbar <= MAXS && sbar <= ctl->sigma && nwaves >= 2, 31);
  for (int i = tid; i < MAXC * MAXC; i += blockDim.x) {
    const int a = i / MAXC, b = i % MAXC;
    sG[i] = (a < nc && b < nc) ? ctl->G[a * MAXC + b] : 0.0;
  }
  if (tid < MAXS) {
    sTh[tid] = ctl->theta[tid];
    sGa[tid] = ctl->gamma[tid];
    sMu[tid] = ctl->mu[tid];
  }
  if (tid < MAXS + 2) sKappa[tid] = INFINITY;
  __syncthreads();

  const double u = UNIT_ROUNDOFF;
  const double nb = ctl->nb, tol = ctl->tol;
  const double c_in = ctl->c;
  const int variant = ctl->variant;
  const bool forced = ctl->forced_sk && (int64_t)ctl->k < ctl->forced_len;
  const int64_t m = ctl->m;
  const double rGr0 = fmax(sG[1 * MAXC + 1], 0.0);

  if (wave == 0) {
    // ---- the inner loop on the whole basis (interleaved coordinates; lane i
    // owns coordinate i and row i of G); products are masked to the step's
    // support, so rows of G past it never enter a sum
    double grow[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) grow[c] = (lane < nc && c < nc) ? sG[lane * MAXC + c] : 0.0;
    double vp = (lane == 0) ? 1.0 : 0.0;
    double vr = (lane == 1) ? 1.0 : 0.0;
    double vx = 0.0;
    double rGr = rGr0;
    double phi = sqrt(rGr) / nb;
    double c = c_in;
    double psi = ctl->psi;
    double lmin = ctl->lmin, lmax = ctl->lmax;
    double alpha_prev = ctl->alpha_prev, beta_prev = ctl->beta_prev;
    double mx_omega = ctl->mx_omega, mx_h = ctl->mx_h, mx_zeta = ctl->mx_zeta;
    double mn_omega = ctl->mn_omega, mn_a = ctl->mn_a, mn_d = ctl->mn_d, mn_g = ctl->mn_g,
           mn_h = ctl->mn_h;
    int steps = 0, event = EV_NONE;
    for (int j = 0; j < sbar; ++j) {
      const int sup = 2 * j + 3;                              // support of B p' and r'_{j+1}
      const double bp = apply_B(vp, sbar, lane, sTh, sGa, sMu);
      const double den = wave_sum_dpp(lane < sup ? vp * gmv(grow, bp) : 0.0);
      if (!isfinite(den)) { steps = j + 1; event = EV_DIVERGED_DEN; break; }
      if (den <= 0.0 || rGr <= 0.0) { steps = j + 1; event = EV_BREAKDOWN; break; }
      const double alpha = rGr / den;
      const double q = (lane < nc) ? alpha * vp : 0.0;
      vx += q;
      const double rnew = (lane < nc) ? vr - apply_B(q, sbar, lane, sTh, sGa, sMu) : 0.0;
      vr = rnew;
      const double rGr_new =
          fmax(wave_sum_dpp(lane < sup ? rnew * gmv(grow, rnew) : 0.0), 0.0);
      const double beta = rGr_new / rGr;
      vp = (lane < nc) ? rnew + beta * vp : 0.0;
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
          const double h =
              (chi == 0.0) ? 0.0 : sqrt(fmax(0.0, 0.5 * (1.0 - (mn_omega - a) / chi)));
          mn_omega = mn_omega + chi * h * h;
          mn_g = sqrt(fmax(0.0, 1.0 - h * h));
          mn_h = fabs(h) * (dd < 0.0 ? -1.0 : 1.0);
          mn_d = dd;
          mn_a = a;
        }
        lmax = mx_omega;
        lmin = 1.0 / mn_omega;
        if (variant == ASSG_IMPROVED)
          c = fmax(1.0, lmax * sqrt(psi / lmin));             // (4.6)
        else if (variant == ASSG_IMPROVED_C_RATIO)
          c = lmax / lmin;                                    // Section 5.1
      }
      alpha_prev = alpha;
      beta_prev = beta;
      if (lane < MAXC) {
        sVec[j][0][lane] = vx;
        sVec[j][1][lane] = vr;
        sVec[j][2][lane] = vp;
      }
      if (lane == 0) {
        double* r = sStep[j];
        r[SS_RGR] = rGr; r[SS_PHI] = phi; r[SS_PSI] = psi; r[SS_LMIN] = lmin;
        r[SS_LMAX] = lmax; r[SS_C] = c; r[SS_ALPHA] = alpha; r[SS_BETA] = beta; r[SS_RHO] = rho;
        r[SS_MXO] = mx_omega; r[SS_MXH] = mx_h; r[SS_MXZ] = mx_zeta;
        r[SS_MNO] = mn_omega; r[SS_MNA] = mn_a; r[SS_MND] = mn_d; r[SS_MNG] = mn_g;
        r[SS_MNH] = mn_h;
      }
      steps = j + 1;
      if (!isfinite(alpha) || !isfinite(beta)) { event = EV_DIVERGED; break; }
      if (!forced && rho <= tol) { event = EV_CANDIDATE; break; }
    }
    if (lane == 0) {
      sEvent[0] = steps;
      sEvent[1] = event;
    }
  } else {
    // ---- kappa(Y_{k,l}) for l = 1..sbar: the blocks, largest first, dealt
    // to waves 1.. in snake order (one block per wave up to s-bar = 11)
    const int kw = nwaves - 1;
    for (int idx = 0; idx < sbar; ++idx) {
      const int round = idx / kw, pos = idx % kw;
      const int owner = 1 + ((round & 1) ? kw - 1 - pos : pos);
      if (owner != wave) continue;
      const int l = sbar - idx;
      const int n = 2 * l + 1;
      double* T = sScr + scratch_offset(l) * MAXC;
      for (int i = lane; i < n * MAXC; i += 64) {
        const int a = i / MAXC, b = i % MAXC;
        T[i] = (b < n) ? sG[a * MAXC + b] : 0.0;
      }
      wave_lds_sync();
      double kap = INFINITY;
      double* dsh = sDE[l - 1][0];
      double* esh = sDE[l - 1][1];
      switch (l) {
        case 1: kap = kappa_wave<3>(T, lane, dsh, esh); break;
        case 2: kap = kappa_wave<5>(T, lane, dsh, esh); break;
        case 3: kap = kappa_wave<7>(T, lane, dsh, esh); break;
        case 4: kap = kappa_wave<9>(T, lane, dsh, esh); break;
        case 5: kap = kappa_wave<11>(T, lane, dsh, esh); break;
        case 6: kap = kappa_wave<13>(T, lane, dsh, esh); break;
        case 7: kap = kappa_wave<15>(T, lane, dsh, esh); break;
        case 8: kap = kappa_wave<17>(T, lane, dsh, esh); break;
        case 9: kap = kappa_wave<19>(T, lane, dsh, esh); break;
        case 10: kap = kappa_wave<21>(T, lane, dsh, esh); break;
        case 11: kap = kappa_wave<23>(T, lane, dsh, esh); break;
        case 12: kap = kappa_wave<25>(T, lane, dsh, esh); break;
        case 13: kap = kappa_wave<27>(T, lane, dsh, esh); break;
        case 14: kap = kappa_wave<29>(T, lane, dsh, esh); break;
        case 15: kap = kappa_wave<31>(T, lane, dsh, esh); break;
        default: kap = kappa_wave<33>(T, lane, dsh, esh); break;
      }
      if (lane == 0) sKappa[l] = kap;
    }
  }
  __syncthreads();
  if (wave != 0) return;

  // ---- s~ by (3.2) with the current c and relative ||r_m||
  const double rho_m = sqrt(rGr0) / nb;
  const double thr = (rho_m > 0.0) ? tol / (c_in * u * rho_m) : INFINITY;
  int st = 1;
  for (int l = 1; l <= sbar; ++l) {
    if (sKappa[l] <= thr)
      st = l;
    else
      break;
  }
  if (variant == ASSG_FIXED_SSTEP) st = sbar;   // fixed s-step CG: the whole basis
  // a given schedule replaces (3.2), the break and the in-loop stopping test
  // in its loops; the loops after it decide for themselves
  const bool last_forced = forced && (int64_t)ctl->k + 1 == ctl->forced_len;
  if (forced) {
    const int32_t f = ctl->forced_sk[ctl->k];
    st = f < 1 ? 1 : (f > sbar ? sbar : f);
  }
  const int n = 2 * st + 1;

  // ---- s_k: the first of breakdown/divergence, the stopping candidate, the
  // break (4.7) after the step, or s~ steps; `last` is the record whose
  // state the loop ends with (-1: the state on entry)
  const int steps = sEvent[0], event = sEvent[1];
  int sk = 0, candidate = 0, outcome = ST_RUNNING, last = -1;
  for (int j = 0; j < st; ++j) {
    sk = j + 1;
    if (j == steps - 1 && (event == EV_BREAKDOWN || event == EV_DIVERGED_DEN)) {
      outcome = (event == EV_BREAKDOWN) ? ASSG_BREAKDOWN : ASSG_DIVERGED;
      break;
    }
    last = j;
    if (j == steps - 1 && event == EV_DIVERGED) { outcome = ASSG_DIVERGED; break; }
    if (j == steps - 1 && event == EV_CANDIDATE) { candidate = 1; break; }
    if (forced) continue;
    const double cj = sStep[j][SS_C];
    if (variant <= ASSG_IMPROVED_C_ONE) {
      if (j < st - 1 && sKappa[j + 2] >= tol / (cj * u * sStep[j][SS_PHI])) break;   // (4.7)
    } else if (variant == ASSG_OLD_ADAPTIVE) {
      // Algorithm 2: gamma = kappa(Y_{k,s~}) against the current residual
      if (j < st - 1 && sKappa[st] >= tol / (cj * u * sStep[j][SS_RHO])) break;
    }
  }
  ASSG_DCHECK(st >= 1 && st <= sbar && sk <= st && last < steps && last < sk, 32);
  // the last loop of a given schedule ends with the true-residual check
  if (last_forced && outcome == ST_RUNNING) candidate = 1;

  // the state the loop ends with
  double rGr = rGr0, phi = sqrt(rGr0) / nb, c = c_in, psi = ctl->psi;
  double lmin = ctl->lmin, lmax = ctl->lmax;
  double alpha_prev = ctl->alpha_prev, beta_prev = ctl->beta_prev;
  double mx_omega = ctl->mx_omega, mx_h = ctl->mx_h, mx_zeta = ctl->mx_zeta;
  double mn_omega = ctl->mn_omega, mn_a = ctl->mn_a, mn_d = ctl->mn_d, mn_g = ctl->mn_g,
         mn_h = ctl->mn_h;
  double vx = 0.0, vr = (lane == 1) ? 1.0 : 0.0, vp = (lane == 0) ? 1.0 : 0.0;
  if (last >= 0) {
    const double* r = sStep[last];
    rGr = r[SS_RGR]; phi = r[SS_PHI]; psi = r[SS_PSI]; lmin = r[SS_LMIN]; lmax = r[SS_LMAX];
    c = r[SS_C]; alpha_prev = r[SS_ALPHA]; beta_prev = r[SS_BETA];
    mx_omega = r[SS_MXO]; mx_h = r[SS_MXH]; mx_zeta = r[SS_MXZ];
    mn_omega = r[SS_MNO]; mn_a = r[SS_MNA]; mn_d = r[SS_MND]; mn_g = r[SS_MNG]; mn_h = r[SS_MNH];
    if (lane < MAXC) {
      vx = sVec[last][0][lane];
      vr = sVec[last][1][lane];
      vp = sVec[last][2][lane];
    }
  }
  {
    // the recorded steps (a breakdown is found before its step's update)
    const int rec = (event == EV_BREAKDOWN || event == EV_DIVERGED_DEN) ? steps - 1 : steps;
    if (lane < MAXS && lane < rec) {
      ctl->alphas[lane] = sStep[lane][SS_ALPHA];
      ctl->betas[lane] = sStep[lane][SS_BETA];
    }
  }

  // ---- results
  if (lane < MAXC) {
    const bool keep = lane < n;
    ctl->cx[lane] = keep ? vx : 0.0;
    ctl->cr[lane] = keep ? vr : 0.0;
    ctl->cp[lane] = keep ? vp : 0.0;
  }
  if (lane < MAXS) ctl->kappa[lane] = (lane < sbar) ? sKappa[lane + 1] : 0.0;
  if (lane == 0) {
    const int64_t k = ctl->k;
    ctl->stilde = st;
    ctl->thr = thr;
    ctl->rho_m = rho_m;
    ctl->phi = phi;
    ctl->relres_upd = sqrt(rGr) / nb;
    if (trace && ctl->record_trace && k < ctl->trace_cap) {
      assg_trace_t& tr = trace[k];
      tr.k = (int32_t)k;
      tr.sbar = sbar;
      tr.stilde = st;
      tr.sk = sk;
      tr.m = m;
      tr.candidate = candidate;
      tr.flags = (outcome == ASSG_BREAKDOWN ? 1 : 0) | (outcome == ASSG_DIVERGED ? 2 : 0);
      tr.c_in = c_in;
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

void launch_controller(hipStream_t s, Ctl* ctl, assg_trace_t* trace, int sigma, int nsys) {
  // one wave for the inner loop and up to CTL_WAVES - 1 for the kappa blocks
  const int waves = sigma < 1 ? 2 : (sigma + 1 < CTL_WAVES ? sigma + 1 : CTL_WAVES);
  hipLaunchKernelGGL(k_controller, dim3(nsys), dim3(64 * waves), 0, s, ctl,
                     nsys == 1 ? trace : nullptr);
}

// The first failed check of a debug build since the last call (0: none, or
// a release build), cleared.
int debug_code_take_controller(hipStream_t s) {
#ifdef ASSG_DEBUG
  int v = 0;
  if (hipMemcpyFromSymbolAsync(&v, HIP_SYMBOL(g_debug_code), sizeof(int), 0,
                               hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -1;
  if (v != 0) {
    const int z = 0;
    if (hipMemcpyToSymbolAsync(HIP_SYMBOL(g_debug_code), &z, sizeof(int), 0,
                               hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return -1;
  }
  return v;
#else
  (void)s;
  return 0;
#endif
}

}  // namespace assg
