// C ABI of the library (include/assg.h) for single systems and HSCG:
// argument checks, workspace, the host side of the outer loop (enqueue only;
// every decision is made on the device), timing and result copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "handle.hpp"

using namespace assg;
using namespace assg::host;

namespace assg {
namespace host {

// Leja points of [-1, 1] in the order of (2.7): t0 = 1, t1 = -1, then each
// point maximizes prod |t - t_m|.  In every gap between consecutive points
// the logarithmic derivative sum 1/(t - t_m) decreases from +inf to -inf;
// its zero (bisection to the last bit) is the gap's maximizer.  The largest
// product wins; products equal to a relative 1e-9 count as ties, broken
// towards the smaller t.
void leja_table(double* t, int count) {
  t[0] = 1.0;
  if (count > 1) t[1] = -1.0;
  for (int l = 2; l < count; ++l) {
    std::vector<double> s(t, t + l);
    std::sort(s.begin(), s.end());
    std::vector<double> cand, val;
    for (int g = 0; g + 1 < l; ++g) {
      double lo = s[g], hi = s[g + 1];
      for (int it = 0; it < 2000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double f = 0.0;
        for (int q = 0; q < l; ++q) f += 1.0 / (mid - s[q]);
        if (f > 0.0) lo = mid; else hi = mid;
      }
      const double tc = 0.5 * (lo + hi);
      double v = 0.0;
      for (int q = 0; q < l; ++q) v += std::log(std::fabs(tc - s[q]));
      cand.push_back(tc);
      val.push_back(v);
    }
    double vmax = -INFINITY;
    for (double v : val) vmax = std::max(vmax, v);
    double best = INFINITY;
    for (size_t q = 0; q < cand.size(); ++q)
      if (val[q] >= vmax - 1e-9) best = std::min(best, cand[q]);
    t[l] = best;
  }
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }


WsLayout ws_layout(int64_t n, int32_t s_max) {
  WsLayout w;
  w.ld = (int64_t)align_up((size_t)n, 32);
  const size_t vec = (size_t)w.ld * sizeof(double);
  const size_t basis = std::max((size_t)s_max * 2 * vec + vec, 4 * vec);
  w.pairs_off = 0;
  w.plast_off = (size_t)s_max * 2 * vec;
  w.grampart_off = align_up(basis, 256);
  const size_t np = (size_t)(2 * s_max + 1) * (2 * s_max + 2) / 2;
  w.total = w.grampart_off + align_up(np * 4096 * sizeof(double), 256);
  return w;
}

assg_status_t fail(assg_handle_t h, assg_status_t st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}


bool csr_ok(const assg_csr_t* A) {
  return A && A->n >= 1 && A->n < (int64_t(1) << 31) && A->nnz >= 1 &&
         A->nnz < (int64_t(1) << 31) && A->row_ptr && A->col_idx && A->val;
}

assg_status_t check_columns(assg_handle_t h, const int32_t* ci, int64_t nnz, int64_t n) {
  HIP_OR_FAIL(h, hipMemsetAsync(h->d_flag, 0, sizeof(int32_t), h->stream));
  launch_check_cols(h->stream, ci, nnz, (int32_t)n, h->d_flag);
  HIP_OR_FAIL(h, hipGetLastError());
  HIP_OR_FAIL(h, hipMemcpyAsync(h->h_status, h->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost,
                                h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (h->h_status[0] != 0) return fail(h, ASSG_ERR_INVALID_ARG, "column index outside [0, n)");
  return ASSG_OK;
}

assg_status_t check_analyzed(assg_handle_t h, const assg_csr_t* A) {
  if (!csr_ok(A)) return fail(h, ASSG_ERR_INVALID_ARG, "invalid CSR descriptor");
  if (A->n != h->an_n || A->nnz != h->an_nnz || A->row_ptr != h->an_rp ||
      A->col_idx != h->an_ci)
    return fail(h, ASSG_ERR_NOT_ANALYZED, "matrix not analyzed (call assg_analyze)");
  return ASSG_OK;
}

assg_status_t get_workspace(assg_handle_t h, int64_t n, int32_t s_max, void* ws, size_t bytes,
                            char** base, WsLayout* lay) {
  *lay = ws_layout(n, s_max);
  if (ws) {
    if (bytes < lay->total) return fail(h, ASSG_ERR_INVALID_ARG, "workspace too small");
    *base = static_cast<char*>(ws);
    return ASSG_OK;
  }
  if (h->ws_bytes < lay->total) {
    if (h->ws) {
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      HIP_OR_FAIL(h, hipFree(h->ws));
      h->ws = nullptr;
      h->ws_bytes = 0;
    }
    if (hipMalloc(&h->ws, lay->total) != hipSuccess) {
      h->ws = nullptr;
      return fail(h, ASSG_ERR_ALLOC, "workspace allocation failed");
    }
    h->ws_bytes = lay->total;
  }
  *base = static_cast<char*>(h->ws);
  return ASSG_OK;
}

void init_ctl(assg_handle_t h, Ctl* c, int mode) {
  std::memset(c, 0, sizeof(Ctl));
  c->status = ST_RUNNING;
  c->pending = ST_RUNNING;
  c->mode = mode;
  c->psi = 1.0;
  c->c = 1.0 / std::sqrt(UNIT_ROUNDOFF);   // c_1 = eps^{-1/2}
  c->lmin = NAN;
  c->lmax = NAN;
  c->alpha_prev = NAN;
  c->beta_prev = NAN;
  c->best_true = INFINITY;
  c->relres_true = -1.0;
  for (int l = 0; l < MAXS; ++l) {
    c->theta[l] = 0.0;
    c->gamma[l] = 1.0;
    c->mu[l] = 0.0;
    c->leja[l] = h->leja[l];
  }
}

// b = 0: the solution is x = 0 (nothing to iterate).  Reads ||b|| computed
// by the setup kernel; returns true (with *st set) when the solve is done.
bool zero_rhs(assg_handle_t h, double* x, int64_t n, assg_info_t* info, assg_status_t* st) {
  double* nbh = reinterpret_cast<double*>(h->h_status + 8);
  *st = ASSG_OK;
  if (hipMemcpyAsync(nbh, &h->d_ctl->nb, sizeof(double), hipMemcpyDeviceToHost, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    *st = fail(h, ASSG_ERR_HIP, "reading ||b|| failed");
    return true;
  }
  if (*nbh != 0.0) return false;
  if (hipMemsetAsync(x, 0, (size_t)n * sizeof(double), h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    *st = fail(h, ASSG_ERR_HIP, "clearing x failed");
    return true;
  }
  info->outcome = ASSG_CONVERGED;
  info->relres_true = 0.0;
  info->relres_updated = 0.0;
  return true;
}

assg_status_t debug_verdict(assg_handle_t h) {
  const int a = debug_code_take_kernels(h->stream);
  const int b = debug_code_take_controller(h->stream);
  if (a == 0 && b == 0) return ASSG_OK;
  return fail(h, ASSG_ERR_HIP, "kernel debug check failed (row kernels: code " +
                                   std::to_string(a) + ", controller: code " +
                                   std::to_string(b) + ")");
}

void log_solve(const char* what, int64_t n, int sigma, const assg_info_t* info) {
  static const bool on = [] {
    const char* v = std::getenv("ASSG_LOG");
    return v && v[0] == '1';
  }();
  if (!on) return;
  static const char* names[] = {"CONVERGED", "STAGNATED", "DIVERGED", "BREAKDOWN", "MAX_ITER",
                                "RUNNING"};
  const int o = info->outcome;
  std::fprintf(stderr,
               "assg: %s n=%lld s_max=%d outcome=%s outer=%lld iters=%lld relres_true=%.3e "
               "relres_updated=%.3e device_ms=%.3f\n",
               what, (long long)n, sigma, (o >= 0 && o <= 5) ? names[o] : "?",
               (long long)info->outer_iters, (long long)info->total_iters, info->relres_true,
               info->relres_updated, info->solve_ms);
}

// Outer loops completed: a loop that ended in breakdown or divergence is
// committed on the device (its trace record is kept) but not counted.
int64_t completed_loops(const Ctl* c) {
  const bool broke = c->status == ASSG_BREAKDOWN || c->status == ASSG_DIVERGED;
  return (broke && c->k > 0) ? c->k - 1 : c->k;
}

// The method of opts in a fresh control block: the monomial-basis methods
// keep theta = 0, gamma = 1, mu = 0 throughout; the starting c is 1 for
// Algorithm 5 with c = 1 and c_const for the old adaptive method.
void apply_variant(Ctl* c, const assg_opts_t* o) {
  c->variant = o->variant;
  c->c_const = o->c_const;
  if (o->variant == ASSG_OLD_ADAPTIVE || o->variant == ASSG_FIXED_SSTEP)
    c->basis = ASSG_BASIS_MONOMIAL;
  if (o->variant == ASSG_IMPROVED_C_ONE) c->c = 1.0;
  if (o->variant == ASSG_OLD_ADAPTIVE) c->c = o->c_const;
}

// The kernels' view of the analyzed single matrix (a batch of one).
CsrView view(assg_handle_t h, const assg_csr_t* A) {
  CsrView v{};
  v.n = A->n;
  v.nnz = A->nnz;
  v.rp = A->row_ptr;
  v.ci = A->col_idx;
  v.va = A->val;
  v.blk = h->d_blk;
  v.blke = h->d_blke;
  v.nblk = h->nblk;
  v.bsys = nullptr;
  v.cblk = h->d_chunks;
  v.csys = nullptr;
  v.sys_chunk = h->d_chunks + h->nchunk + 1;
  v.nchunk = h->nchunk;
  v.nsys = 1;
  if (h->fmt == ASSG_FORMAT_DIA) v.dia = h->dia.view;
  return v;
}

void refresh_dia(assg_handle_t h, const assg_csr_t* A) {
  if (h->fmt == ASSG_FORMAT_DIA)
    launch_dia_fill(h->stream, A->row_ptr, A->col_idx, A->val, h->dia.rec[0], h->dia.val);
}

// The offsets of the sampled rows (dia_sample_rows) are the candidates
// (dia_offsets); a kernel then checks that every row's entries lie on them,
// in order.
assg_status_t dia_detect(assg_handle_t h, const assg_csr_t* A, const int32_t* rp, bool check_fill,
                         DiaSys* R, bool* fits, std::string* why) {
  *fits = false;
  const int64_t n = A->n;
  std::vector<int64_t> rows, offs;
  dia_sample_rows(n, rows);
  std::vector<int32_t> cols;
  int64_t max_row = 0;
  for (const int64_t i : rows) {
    const int32_t e0 = rp[i], e1 = rp[i + 1];
    max_row = std::max<int64_t>(max_row, e1 - e0);
    if (e1 - e0 > DIA_MAX) break;
    cols.resize(e1 - e0);
    if (e1 > e0) {
      HIP_OR_FAIL(h, hipMemcpyAsync(cols.data(), A->col_idx + e0, (e1 - e0) * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, h->stream));
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    }
    for (int32_t c : cols) offs.push_back((int64_t)c - i);
  }
  if (const char* no = dia_offsets(offs, max_row, n, A->nnz, check_fill)) {
    *why = no;
    return ASSG_OK;
  }
  *R = DiaSys{};
  R->n = (int32_t)n;
  R->nd = (int32_t)offs.size();
  for (int d = 0; d < R->nd; ++d) R->off[d] = (int32_t)offs[d];
  HIP_OR_FAIL(h, hipMemsetAsync(h->d_flag, 0, sizeof(int32_t), h->stream));
  launch_dia_probe(h->stream, A->row_ptr, A->col_idx, *R, h->d_flag);
  HIP_OR_FAIL(h, hipGetLastError());
  HIP_OR_FAIL(h, hipMemcpyAsync(h->h_status, h->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost,
                                h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (h->h_status[0] != 0) {
    *why = "an entry lies off the diagonals of the sampled rows";
    return ASSG_OK;
  }
  *fits = true;
  return ASSG_OK;
}

void dia_release(DiaStore* S) {
  for (void* p : {(void*)S->val, (void*)S->sys, (void*)S->tab})
    if (p) (void)hipFree(p);
  *S = DiaStore{};
}

assg_status_t dia_build(assg_handle_t h, std::vector<DiaSys>& R, int chunk_target, DiaStore* S) {
  dia_release(S);
  const int nsys = (int)R.size();
  std::vector<int32_t> blk, bsys, sys_blk{0};
  int64_t nval = 0;
  int32_t ndmax = 0;
  for (int i = 0; i < nsys; ++i) {
    R[i].val0 = nval;
    nval += (int64_t)R[i].nd * R[i].n;
    ndmax = std::max(ndmax, R[i].nd);
    for (int64_t r = 0; r < R[i].n; r += SB_ROWS) {
      blk.push_back((int32_t)(R[i].row0 + r));
      bsys.push_back(i);
    }
    sys_blk.push_back((int32_t)blk.size());
  }
  blk.push_back((int32_t)(R[nsys - 1].row0 + R[nsys - 1].n));
  std::vector<int32_t> cblk, csys, sys_chunk;
  make_chunks(sys_blk, chunk_target, cblk, csys, sys_chunk);
  std::vector<int32_t> tab(blk);
  tab.insert(tab.end(), bsys.begin(), bsys.end());
  tab.insert(tab.end(), cblk.begin(), cblk.end());
  tab.insert(tab.end(), csys.begin(), csys.end());
  tab.insert(tab.end(), sys_chunk.begin(), sys_chunk.end());
  if (hipMalloc(&S->val, (size_t)nval * sizeof(double)) != hipSuccess) {
    S->val = nullptr;
    (void)hipGetLastError();
    return ASSG_ERR_ALLOC;
  }
  HIP_OR_FAIL(h, hipMalloc(&S->sys, (size_t)nsys * sizeof(DiaSys)));
  HIP_OR_FAIL(h, hipMalloc(&S->tab, tab.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMemcpyAsync(S->sys, R.data(), (size_t)nsys * sizeof(DiaSys),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(S->tab, tab.data(), tab.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));   // the host tables go out of scope
  DiaView& D = S->view;
  D = DiaView{};
  D.nd = ndmax;
  D.sys = S->sys;
  D.val = S->val;
  D.nblk = (int32_t)bsys.size();
  D.blk = S->tab;
  D.bsys = nsys > 1 ? S->tab + blk.size() : nullptr;
  D.nchunk = (int32_t)cblk.size() - 1;
  D.cblk = S->tab + blk.size() + bsys.size();
  D.csys = nsys > 1 ? D.cblk + cblk.size() : nullptr;
  D.sys_chunk = D.cblk + cblk.size() + csys.size();
  S->rec = R;
  return ASSG_OK;
}

// Diagonal storage of a single system at analysis: sets h->fmt to
// ASSG_FORMAT_DIA when A fits it; a matrix that does not fit is an error
// only when the storage was forced.
static assg_status_t analyze_dia(assg_handle_t h, const assg_csr_t* A,
                                 const std::vector<int32_t>& rp) {
  const bool forced = h->fmt_req == ASSG_FORMAT_DIA;
  std::vector<DiaSys> R(1);
  bool fits = false;
  std::string why;
  assg_status_t st = dia_detect(h, A, rp.data(), !forced, &R[0], &fits, &why);
  if (st != ASSG_OK) return st;
  if (!fits) return forced ? fail(h, ASSG_ERR_UNSUPPORTED, "diagonal storage: " + why) : ASSG_OK;
  st = dia_build(h, R, h->gram_blocks[10], &h->dia);
  if (st == ASSG_ERR_ALLOC) {   // AUTO falls back to CSR
    dia_release(&h->dia);
    return forced ? fail(h, ASSG_ERR_ALLOC, "diagonal storage allocation failed") : ASSG_OK;
  }
  if (st != ASSG_OK) return st;
  h->fmt = ASSG_FORMAT_DIA;
  return ASSG_OK;
}





hipEvent_t pool_event(assg_handle_t h, size_t i) {
  while (h->evpool.size() <= i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->evpool.push_back(e);
  }
  return h->evpool[i];
}

assg_status_t validate_opts(assg_handle_t h, const assg_opts_t* o) {
  if (!o) return fail(h, ASSG_ERR_INVALID_ARG, "null options");
  if (o->s_max < 1 || o->s_max > ASSG_MAX_S)
    return fail(h, ASSG_ERR_INVALID_ARG, "s_max must be in 1..ASSG_MAX_S");
  if (o->s_init < 0 || o->s_init > o->s_max)
    return fail(h, ASSG_ERR_INVALID_ARG, "s_init must be in 1..s_max (0: s_max)");
  if (o->growth < 0) return fail(h, ASSG_ERR_INVALID_ARG, "growth must be >= 1 (0: s_max)");
  if (o->basis != ASSG_BASIS_MONOMIAL && o->basis != ASSG_BASIS_NEWTON &&
      o->basis != ASSG_BASIS_CHEBYSHEV)
    return fail(h, ASSG_ERR_INVALID_ARG, "unknown basis");
  if (!(o->tol > 0.0 && o->tol < 1.0)) return fail(h, ASSG_ERR_INVALID_ARG, "tol must be in (0,1)");
  if (o->max_outer < 0 || o->max_iters < 0)
    return fail(h, ASSG_ERR_INVALID_ARG, "iteration caps must be >= 0");
  if (o->variant < ASSG_IMPROVED || o->variant > ASSG_FIXED_SSTEP)
    return fail(h, ASSG_ERR_INVALID_ARG, "unknown variant");
  if (o->variant == ASSG_OLD_ADAPTIVE && !(o->c_const > 0.0 && std::isfinite(o->c_const)))
    return fail(h, ASSG_ERR_INVALID_ARG, "c_const must be positive and finite");
  return ASSG_OK;
}

}  // namespace host
}  // namespace assg

extern "C" {

assg_status_t assg_default_opts(assg_opts_t* o) {
  if (!o) return ASSG_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->s_max = 10;
  o->s_init = 0;   // s-bar_0 = sigma
  o->growth = 0;   // f = sigma
  o->basis = ASSG_BASIS_CHEBYSHEV;
  o->tol = 1e-10;
  o->max_outer = 0;
  o->max_iters = 0;
  o->record_trace = 0;
  o->time_kernels = 0;
  o->variant = ASSG_IMPROVED;
  o->c_const = 1.0;
  return ASSG_OK;
}

const char* assg_status_string(assg_status_t s) {
  switch (s) {
    case ASSG_OK: return "ok";
    case ASSG_ERR_INVALID_ARG: return "invalid argument";
    case ASSG_ERR_HIP: return "HIP error";
    case ASSG_ERR_ALLOC: return "allocation failed";
    case ASSG_ERR_UNSUPPORTED: return "unsupported (device or storage)";
    case ASSG_ERR_NOT_ANALYZED: return "matrix not analyzed";
  }
  return "unknown status";
}

const char* assg_last_error(assg_handle_t h) { return h ? h->err.c_str() : ""; }

int32_t assg_struct_sizes(int64_t* sizes, int32_t cap) {
  const int64_t s[] = {(int64_t)sizeof(assg_opts_t),        (int64_t)sizeof(assg_info_t),
                       (int64_t)sizeof(assg_trace_t),       (int64_t)sizeof(assg_block_state_t),
                       (int64_t)sizeof(assg_block_result_t), (int64_t)sizeof(assg_csr_t),
                       (int64_t)sizeof(assg_tune_class_t)};
  int32_t k = 0;
  for (; k < cap && k < 7; ++k) sizes[k] = s[k];
  return k;
}

assg_status_t assg_basis_params(int32_t kind, double lmin, double lmax, int32_t s, double* theta,
                                double* gamma, double* mu) {
  if (s < 1 || s > ASSG_MAX_S || !theta || !gamma || (s > 1 && !mu)) return ASSG_ERR_INVALID_ARG;
  if (kind != ASSG_BASIS_MONOMIAL && kind != ASSG_BASIS_NEWTON && kind != ASSG_BASIS_CHEBYSHEV)
    return ASSG_ERR_INVALID_ARG;
  if (kind != ASSG_BASIS_MONOMIAL && !(lmin < lmax && std::isfinite(lmin) && std::isfinite(lmax)))
    return ASSG_ERR_INVALID_ARG;
  double t[MAXS];
  leja_table(t, MAXS);
  double th[MAXS], ga[MAXS], m[MAXS];
  basis_params(kind, lmin, lmax, s, t, th, ga, m);
  for (int l = 0; l < s; ++l) {
    theta[l] = th[l];
    gamma[l] = ga[l];
    if (l + 1 < s) mu[l] = m[l];
  }
  return ASSG_OK;
}

assg_status_t assg_workspace_size(int64_t n, int32_t s_max, size_t* bytes) {
  if (n < 1 || s_max < 1 || s_max > ASSG_MAX_S || !bytes) return ASSG_ERR_INVALID_ARG;
  *bytes = ws_layout(n, s_max).total;
  return ASSG_OK;
}

// Scratch of assg_solve_noalloc (basis and Gram partials of solves whose
// callers cannot allocate).  Each GPU the library runs on holds its own copy
// from the library's load until the process ends; in host code the name is
// only a stand-in, so kernels get the address that hipGetSymbolAddress
// returns for the current device, taken once per device in assg_create.
static __device__ __align__(256) char scratch[ASSG_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[ASSG_MAX_DEVICES];

static assg_status_t scratch_setup(assg_handle_t h) {
  if (h->device < 0 || h->device >= ASSG_MAX_DEVICES)
    return fail(h, ASSG_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[h->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(h, ASSG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
    g_scratch_ptr[h->device] = p;
  }
  h->scratch = g_scratch_ptr[h->device];
  return ASSG_OK;
}

assg_status_t assg_create(assg_handle_t* out, void* stream) {
  if (!out) return ASSG_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return ASSG_ERR_UNSUPPORTED;
  assg_handle_t h = new assg_handle_s();
  HIP_OR_FAIL(h, hipGetDevice(&h->device));
  hipDeviceProp_t prop;
  HIP_OR_FAIL(h, hipGetDeviceProperties(&prop, h->device));
  h->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  h->user_stream = static_cast<hipStream_t>(stream);
  HIP_OR_FAIL(h, hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
  HIP_OR_FAIL(h, hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
  HIP_OR_FAIL(h, hipEventCreate(&h->ev_start));
  HIP_OR_FAIL(h, hipEventCreate(&h->ev_stop));
  HIP_OR_FAIL(h, hipMalloc(&h->d_ctl, sizeof(Ctl)));
  HIP_OR_FAIL(h, hipHostMalloc(&h->h_ctl, sizeof(Ctl), hipHostMallocDefault));
  HIP_OR_FAIL(h, hipHostMalloc(&h->h_status, 128, hipHostMallocDefault));
  HIP_OR_FAIL(h, hipMalloc(&h->d_flag, sizeof(int32_t)));
  leja_table(h->leja, MAXS);
  for (int s = 1; s <= MAXS; ++s) h->gram_blocks[s] = last_gram_blocks(s, h->cus);
  {
    const assg_status_t st = scratch_setup(h);
    if (st != ASSG_OK) {
      assg_destroy(h);
      return st;
    }
  }
  *out = h;
  return ASSG_OK;
}

assg_status_t assg_destroy(assg_handle_t h) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
  if (h->ws) (void)hipFree(h->ws);
  if (h->d_trace) (void)hipFree(h->d_trace);
  if (h->d_blk) (void)hipFree(h->d_blk);
  if (h->d_blke) (void)hipFree(h->d_blke);
  if (h->d_chunks) (void)hipFree(h->d_chunks);
  if (h->d_part) (void)hipFree(h->d_part);
  dia_release(&h->dia);
  drop_graph(h->g_sstep);
  drop_graph(h->g_hscg);
  if (h->d_forced) (void)hipFree(h->d_forced);
  batch_release(h);
  if (h->d_ctl) (void)hipFree(h->d_ctl);
  if (h->d_flag) (void)hipFree(h->d_flag);
  if (h->h_ctl) (void)hipHostFree(h->h_ctl);
  if (h->h_status) (void)hipHostFree(h->h_status);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->ev_start) (void)hipEventDestroy(h->ev_start);
  if (h->ev_stop) (void)hipEventDestroy(h->ev_stop);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return ASSG_OK;
}

assg_status_t assg_set_stream(assg_handle_t h, void* stream) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  h->user_stream = static_cast<hipStream_t>(stream);
  return ASSG_OK;
}

assg_status_t assg_analyze(assg_handle_t h, const assg_csr_t* A) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  h->an_n = -1;   // no solve runs on an earlier analysis once a new one is asked for
  // the cached graphs were captured with the old partition tables and sizes
  if (h->stream) HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  drop_graph(h->g_sstep);
  drop_graph(h->g_hscg);
  h->fmt = ASSG_FORMAT_CSR;
  dia_release(&h->dia);
  if (!csr_ok(A)) return fail(h, ASSG_ERR_INVALID_ARG, "invalid CSR descriptor");
  std::vector<int32_t> rp((size_t)A->n + 1);
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  HIP_OR_FAIL(h, hipMemcpyAsync(rp.data(), A->row_ptr, rp.size() * sizeof(int32_t),
                                hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (rp[0] != 0 || (int64_t)rp[A->n] != A->nnz)
    return fail(h, ASSG_ERR_INVALID_ARG, "row_ptr[0] must be 0 and row_ptr[n] must be nnz");
  for (int64_t i = 0; i < A->n; ++i)
    if (rp[i + 1] < rp[i]) return fail(h, ASSG_ERR_INVALID_ARG, "row_ptr must be nondecreasing");
  {
    const assg_status_t st = check_columns(h, A->col_idx, A->nnz, A->n);
    if (st != ASSG_OK) return st;
  }
  std::vector<int32_t> blk, blke;
  make_blocks(rp.data(), A->n, blk);
  blke.resize(blk.size());
  for (size_t i = 0; i < blk.size(); ++i) blke[i] = rp[blk[i]];
  if (h->d_blk) HIP_OR_FAIL(h, hipFree(h->d_blk));
  if (h->d_blke) HIP_OR_FAIL(h, hipFree(h->d_blke));
  h->d_blk = h->d_blke = nullptr;
  h->an_n = -1;
  HIP_OR_FAIL(h, hipMalloc(&h->d_blk, blk.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMalloc(&h->d_blke, blke.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_blk, blk.data(), blk.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_blke, blke.data(), blke.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  h->nblk = (int32_t)(blk.size() - 1);
  {
    std::vector<int32_t> cblk, csys, sys_chunk, sys_blk{0, h->nblk};
    make_chunks(sys_blk, h->gram_blocks[10], cblk, csys, sys_chunk);
    if (h->d_chunks) HIP_OR_FAIL(h, hipFree(h->d_chunks));
    h->d_chunks = nullptr;
    std::vector<int32_t> tab(cblk);
    tab.insert(tab.end(), sys_chunk.begin(), sys_chunk.end());
    HIP_OR_FAIL(h, hipMalloc(&h->d_chunks, tab.size() * sizeof(int32_t)));
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_chunks, tab.data(), tab.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, h->stream));
    h->nchunk = (int32_t)cblk.size() - 1;
  }
  if (h->d_part) HIP_OR_FAIL(h, hipFree(h->d_part));
  h->d_part = nullptr;
  HIP_OR_FAIL(h, hipMalloc(&h->d_part, reduce_doubles(h->nblk) * sizeof(double)));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));   // host tables above go out of scope
  if (h->fmt_req != ASSG_FORMAT_CSR) {
    const assg_status_t st = analyze_dia(h, A, rp);
    if (st != ASSG_OK) return st;
  }
  h->an_n = A->n;
  h->an_nnz = A->nnz;
  h->an_rp = A->row_ptr;
  h->an_ci = A->col_idx;
  h->err.clear();
  return ASSG_OK;
}

assg_status_t assg_set_format(assg_handle_t h, int32_t format) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (format != ASSG_FORMAT_AUTO && format != ASSG_FORMAT_CSR && format != ASSG_FORMAT_DIA)
    return fail(h, ASSG_ERR_INVALID_ARG, "format must be AUTO, CSR or DIA");
  h->fmt_req = format;
  return ASSG_OK;
}

assg_status_t assg_get_format(assg_handle_t h, int32_t* format) {
  if (!h || !format) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  if (h->an_n < 0) return fail(h, ASSG_ERR_NOT_ANALYZED, "no analysis");
  *format = h->fmt;
  return ASSG_OK;
}

assg_status_t assg_spmv(assg_handle_t h, const assg_csr_t* A, const double* x, double* y) {
  if (!h || !x || !y) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  assg_status_t st = check_analyzed(h, A);
  if (st != ASSG_OK) return st;
  if (overlap(x, y, A->n)) return fail(h, ASSG_ERR_INVALID_ARG, "x and y overlap");
  const CsrView Av = view(h, A);
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  launch_spmv(h->stream, Av, x, y);
  HIP_OR_FAIL(h, hipGetLastError());
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  return debug_verdict(h);
}

assg_status_t assg_csr_outer_on_pattern(assg_handle_t h, const assg_csr_t* A, const double* u,
                                        const double* v, double alpha, double* out) {
  if (!h || !u || !v || !out) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  assg_status_t st = check_analyzed(h, A);
  if (st != ASSG_OK) return st;
  const CsrView Av = view(h, A);
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  launch_outer_pattern(h->stream, Av, u, v, alpha, out);
  HIP_OR_FAIL(h, hipGetLastError());
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  return debug_verdict(h);
}


// assg_solve, and with ``forced`` (host, nsk entries) its schedule-replay
// form assg_solve_forced_schedule.
static assg_status_t solve_impl(assg_handle_t h, const assg_csr_t* A, const double* b, double* x,
                                const assg_opts_t* opts, const int32_t* forced, int64_t nsk,
                                void* workspace, size_t workspace_bytes, assg_info_t* info,
                                bool noalloc = false) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!b || !x || !info) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  assg_status_t st = validate_opts(h, opts);
  if (st != ASSG_OK) return st;
  if (noalloc) {
    // nothing below may allocate: no trace buffer, no timing events, no graph
    if (opts->record_trace || opts->time_kernels)
      return fail(h, ASSG_ERR_INVALID_ARG,
                  "assg_solve_noalloc: record_trace and time_kernels must be 0");
    st = check_analyzed(h, A);
    if (st != ASSG_OK) return st;
    const size_t need = ws_layout(A->n, opts->s_max).total;
    if (need > ASSG_NOALLOC_SCRATCH_BYTES)
      return fail(h, ASSG_ERR_INVALID_ARG,
                  "assg_solve_noalloc: n = " + std::to_string(A->n) + " at s_max = " +
                      std::to_string(opts->s_max) + " needs " + std::to_string(need) +
                      " bytes of scratch; the limit is " +
                      std::to_string((size_t)ASSG_NOALLOC_SCRATCH_BYTES));
    workspace = h->scratch;
    workspace_bytes = ASSG_NOALLOC_SCRATCH_BYTES;
  }
  st = check_analyzed(h, A);
  if (st != ASSG_OK) return st;
  if (overlap(b, x, A->n)) return fail(h, ASSG_ERR_INVALID_ARG, "b and x overlap");
  const int sigma = opts->s_max;
  if (forced) {
    // every s_k must fit the s-bar its predecessor implies
    const int growth = opts->growth > 0 ? opts->growth : sigma;
    int sbar = opts->s_init > 0 ? opts->s_init : sigma;
    if (nsk < 1 || nsk > (1 << 20)) return fail(h, ASSG_ERR_INVALID_ARG, "schedule length out of range");
    for (int64_t k = 0; k < nsk; ++k) {
      if (forced[k] < 1 || forced[k] > sbar)
        return fail(h, ASSG_ERR_INVALID_ARG, "schedule entry " + std::to_string(k) +
                                                 " outside 1..s-bar of its loop");
      sbar = std::min(forced[k] + growth, sigma);
    }
    if (h->forced_cap < nsk) {
      if (h->d_forced) HIP_OR_FAIL(h, hipFree(h->d_forced));
      h->d_forced = nullptr;
      h->forced_cap = 0;
      if (hipMalloc(&h->d_forced, nsk * sizeof(int32_t)) != hipSuccess)
        return fail(h, ASSG_ERR_ALLOC, "schedule allocation failed");
      h->forced_cap = nsk;
    }
  }
  std::memset(info, 0, sizeof(*info));
  const int64_t n = A->n;
  char* base = nullptr;
  WsLayout lay;
  st = get_workspace(h, n, sigma, workspace, workspace_bytes, &base, &lay);
  if (st != ASSG_OK) return st;
  double2* pairs = reinterpret_cast<double2*>(base + lay.pairs_off);
  double* plast = reinterpret_cast<double*>(base + lay.plast_off);
  double* grampart = reinterpret_cast<double*>(base + lay.grampart_off);
  const int64_t max_iters = opts->max_iters > 0 ? opts->max_iters : 10 * n;
  const int64_t max_outer = opts->max_outer > 0 ? opts->max_outer : max_iters;
  if (opts->record_trace) {
    const int64_t cap = std::min<int64_t>(max_outer, 1 << 20);
    if (h->trace_cap < cap) {
      if (h->d_trace) HIP_OR_FAIL(h, hipFree(h->d_trace));
      h->d_trace = nullptr;
      h->trace_cap = 0;
      if (hipMalloc(&h->d_trace, cap * sizeof(assg_trace_t)) != hipSuccess)
        return fail(h, ASSG_ERR_ALLOC, "trace allocation failed");
      h->trace_cap = cap;
    }
  }
  const CsrView Av = view(h, A);

  Ctl* c = h->h_ctl;
  init_ctl(h, c, 0);
  c->sbar = opts->s_init > 0 ? opts->s_init : opts->s_max;
  c->sbar_next = c->sbar;
  c->sigma = sigma;
  c->growth = opts->growth > 0 ? opts->growth : opts->s_max;
  c->basis = opts->basis;
  c->record_trace = opts->record_trace ? 1 : 0;
  c->trace_cap = opts->record_trace ? h->trace_cap : 0;
  c->max_outer = max_outer;
  c->max_iters = max_iters;
  c->tol = opts->tol;
  c->forced_sk = forced ? h->d_forced : nullptr;
  c->forced_len = forced ? nsk : 0;
  apply_variant(c, opts);

  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  if (forced)
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_forced, forced, nsk * sizeof(int32_t),
                                  hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_ctl, c, sizeof(Ctl), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipEventRecord(h->ev_start, h->stream));
  refresh_dia(h, A);
  launch_setup(h->stream, h->d_ctl, Av, b, x, pairs, h->d_part);
  HIP_OR_FAIL(h, hipGetLastError());
  if (zero_rhs(h, x, n, info, &st)) return st;

  // per-kernel timing: events bracket each matrix-powers launch of a loop
  const bool timing = opts->time_kernels != 0;
  const bool eager = timing || noalloc;   // kernels launched one by one, no graph
  struct Timed { int64_t loop; int kind; size_t ev; };   // kind 0: sweep1, 1: sweep>=2, 2: last+gram
  std::vector<Timed> timed;
  size_t evn = 0;
  double t_sweep = 0, t_sweep1 = 0, t_last = 0;
  int64_t n_sweep = 0, n_sweep1 = 0, n_last = 0;

  int32_t status = ST_RUNNING;
  if (!eager) {
    // outer loops replayed from a captured graph of LOOPS_PER_GRAPH loops
    constexpr int LOOPS_PER_GRAPH = 4;
    const std::vector<const void*> key{A->row_ptr, A->col_idx, A->val, b, x, base, h->d_trace,
                                       h->d_blk, h->d_blke, h->d_chunks, h->d_part,
                                       reinterpret_cast<const void*>((intptr_t)sigma),
                                       reinterpret_cast<const void*>((intptr_t)n),
                                       reinterpret_cast<const void*>((intptr_t)A->nnz),
                                       reinterpret_cast<const void*>((intptr_t)h->nblk),
                                       reinterpret_cast<const void*>((intptr_t)h->nchunk),
                                       h->dia.val, h->dia.tab};
    st = cached_graph(h, h->g_sstep, key, [&]() {
      for (int r = 0; r < LOOPS_PER_GRAPH; ++r) {
        for (int l = 1; l < sigma; ++l) launch_sweep(h->stream, h->d_ctl, l, Av, pairs, lay.ld);
        launch_last_gram(h->stream, h->d_ctl, sigma, Av, pairs, plast, lay.ld, grampart);
        launch_gram_reduce(h->stream, h->d_ctl, sigma, Av, grampart);
        launch_controller(h->stream, h->d_ctl, h->d_trace, sigma, 1);
        launch_recover(h->stream, h->d_ctl, Av, pairs, plast, lay.ld, x);
        launch_check(h->stream, h->d_ctl, h->d_trace, Av, b, x, h->d_part, 0);
      }
    });
    if (st != ASSG_OK) return st;
    while (true) {
      HIP_OR_FAIL(h, hipGraphLaunch(h->g_sstep.exec, h->stream));
      HIP_OR_FAIL(h, hipMemcpyAsync(h->h_status, h->d_ctl, sizeof(int32_t),
                                    hipMemcpyDeviceToHost, h->stream));
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      status = h->h_status[0];
      if (status != ST_RUNNING) break;
    }
  }
  // with kernel timing: eager launches, events around each matrix-powers launch
  int64_t enqueued = 0;
  int batch = 1;
  while (eager) {
    timed.clear();
    evn = 0;
    for (int bi = 0; bi < batch; ++bi, ++enqueued) {
      for (int l = 1; l < sigma; ++l) {
        if (timing) {
          timed.push_back({enqueued, l == 1 ? 0 : 1, evn});
          HIP_OR_FAIL(h, hipEventRecord(pool_event(h, evn++), h->stream));
        }
        launch_sweep(h->stream, h->d_ctl, l, Av, pairs, lay.ld);
        if (timing) HIP_OR_FAIL(h, hipEventRecord(pool_event(h, evn++), h->stream));
      }
      if (timing) {
        timed.push_back({enqueued, 2, evn});
        HIP_OR_FAIL(h, hipEventRecord(pool_event(h, evn++), h->stream));
      }
      launch_last_gram(h->stream, h->d_ctl, sigma, Av, pairs, plast, lay.ld, grampart);
      if (timing) HIP_OR_FAIL(h, hipEventRecord(pool_event(h, evn++), h->stream));
      launch_gram_reduce(h->stream, h->d_ctl, sigma, Av, grampart);
      launch_controller(h->stream, h->d_ctl, h->d_trace, sigma, 1);
      launch_recover(h->stream, h->d_ctl, Av, pairs, plast, lay.ld, x);
      launch_check(h->stream, h->d_ctl, h->d_trace, Av, b, x, h->d_part, 0);
    }
    HIP_OR_FAIL(h, hipGetLastError());
    HIP_OR_FAIL(h, hipMemcpyAsync(h->h_status, h->d_ctl, 2 * sizeof(int32_t) + sizeof(int32_t),
                                  hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    status = h->h_status[0];
    const int64_t kdone = h->h_status[2];   // ctl->k: loops committed so far
    if (timing) {
      for (const Timed& tm : timed) {
        // loops enqueued after the final one exit at once and are not counted;
        // with f < sigma a sweep past the loop's s-bar also exits at once
        if (tm.loop >= kdone) continue;
        float ms = 0.f;
        HIP_OR_FAIL(h, hipEventElapsedTime(&ms, h->evpool[tm.ev], h->evpool[tm.ev + 1]));
        if (tm.kind == 0) { t_sweep1 += ms; ++n_sweep1; }
        else if (tm.kind == 1) { t_sweep += ms; ++n_sweep; }
        else { t_last += ms; ++n_last; }
      }
    }
    if (status != ST_RUNNING) break;
    if (batch < 8) batch *= 2;
  }
  HIP_OR_FAIL(h, hipEventRecord(h->ev_stop, h->stream));
  if (status != ASSG_CONVERGED) {
    launch_check(h->stream, h->d_ctl, h->d_trace, Av, b, x, h->d_part, 1);
    HIP_OR_FAIL(h, hipGetLastError());
  }
  HIP_OR_FAIL(h, hipMemcpyAsync(c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIP_OR_FAIL(h, hipEventElapsedTime(&ms, h->ev_start, h->ev_stop));
  info->outcome = c->status;
  info->outer_iters = completed_loops(c);
  info->total_iters = c->m;
  info->relres_updated = c->relres_upd;
  info->relres_true = c->relres_true;
  info->lambda_min_est = c->lmin;
  info->lambda_max_est = c->lmax;
  info->c_last = c->c;
  info->solve_ms = ms;
  info->sweep_ms = t_sweep;
  info->sweep_launches = n_sweep;
  info->sweep1_ms = t_sweep1;
  info->sweep1_launches = n_sweep1;
  info->last_gram_ms = t_last;
  info->last_gram_launches = n_last;
  info->other_ms = timing ? std::max(0.0, (double)ms - t_sweep - t_sweep1 - t_last) : 0.0;
  log_solve(noalloc ? "solve_noalloc" : (forced ? "solve_forced_schedule" : "solve"), n, sigma,
            info);
  st = debug_verdict(h);
  if (st != ASSG_OK) return st;
  h->trace_count = opts->record_trace ? std::min<int64_t>(c->k, h->trace_cap) : 0;
  return ASSG_OK;
}

assg_status_t assg_solve(assg_handle_t h, const assg_csr_t* A, const double* b, double* x,
                         const assg_opts_t* opts, void* workspace, size_t workspace_bytes,
                         assg_info_t* info) {
  return solve_impl(h, A, b, x, opts, nullptr, 0, workspace, workspace_bytes, info);
}

assg_status_t assg_solve_noalloc(assg_handle_t h, const assg_csr_t* A, const double* b, double* x,
                                 const assg_opts_t* opts, assg_info_t* info) {
  return solve_impl(h, A, b, x, opts, nullptr, 0, nullptr, 0, info, true);
}

assg_status_t assg_solve_forced_schedule(assg_handle_t h, const assg_csr_t* A, const double* b,
                                         double* x, const assg_opts_t* opts, const int32_t* sk,
                                         int64_t nsk, void* workspace, size_t workspace_bytes,
                                         assg_info_t* info) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!sk) return fail(h, ASSG_ERR_INVALID_ARG, "null schedule");
  return solve_impl(h, A, b, x, opts, sk, nsk, workspace, workspace_bytes, info);
}

assg_status_t assg_get_trace(assg_handle_t h, assg_trace_t* host_buf, int64_t cap,
                             int64_t* count) {
  if (!h || !count || (cap > 0 && !host_buf)) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  *count = h->trace_count;
  const int64_t nc = std::min(cap, h->trace_count);
  if (nc > 0) {
    HIP_OR_FAIL(h, hipMemcpyAsync(host_buf, h->d_trace, nc * sizeof(assg_trace_t),
                                  hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  }
  return ASSG_OK;
}

assg_status_t assg_hscg_solve(assg_handle_t h, const assg_csr_t* A, const double* b, double* x,
                              double tol, int64_t max_iters, void* workspace,
                              size_t workspace_bytes, assg_info_t* info) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!b || !x || !info) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  if (!(tol > 0.0 && tol < 1.0) || max_iters < 0)
    return fail(h, ASSG_ERR_INVALID_ARG, "tol must be in (0,1), max_iters >= 0");
  assg_status_t st = check_analyzed(h, A);
  if (st != ASSG_OK) return st;
  if (overlap(b, x, A->n)) return fail(h, ASSG_ERR_INVALID_ARG, "b and x overlap");
  std::memset(info, 0, sizeof(*info));
  const int64_t n = A->n;
  char* base = nullptr;
  WsLayout lay;
  st = get_workspace(h, n, 1, workspace, workspace_bytes, &base, &lay);
  if (st != ASSG_OK) return st;
  double* r = reinterpret_cast<double*>(base);
  double* p = r + lay.ld;
  double* w = r + 2 * lay.ld;
  const CsrView Av = view(h, A);
  Ctl* c = h->h_ctl;
  init_ctl(h, c, 1);
  c->tol = tol;
  c->max_iters = max_iters > 0 ? max_iters : 10 * n;
  c->max_outer = c->max_iters + 1;
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_ctl, c, sizeof(Ctl), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipEventRecord(h->ev_start, h->stream));
  refresh_dia(h, A);
  launch_h_init(h->stream, h->d_ctl, Av, b, x, r, p, h->d_part);
  HIP_OR_FAIL(h, hipGetLastError());
  if (zero_rhs(h, x, n, info, &st)) return st;
  // iterations replayed from a captured graph of ITERS_PER_GRAPH iterations
  constexpr int ITERS_PER_GRAPH = 16;
  const std::vector<const void*> key{A->row_ptr, A->col_idx, A->val, b, x, base, h->d_blk,
                                     h->d_blke, h->d_chunks, h->d_part,
                                     reinterpret_cast<const void*>((intptr_t)n),
                                     reinterpret_cast<const void*>((intptr_t)A->nnz),
                                     reinterpret_cast<const void*>((intptr_t)h->nblk),
                                     reinterpret_cast<const void*>((intptr_t)h->nchunk),
                                     h->dia.val, h->dia.tab};
  st = cached_graph(h, h->g_hscg, key, [&]() {
    for (int it = 0; it < ITERS_PER_GRAPH; ++it) {
      launch_h_spmv(h->stream, h->d_ctl, Av, p, w, h->d_part);
      launch_h_update(h->stream, h->d_ctl, Av, x, r, p, w, h->d_part);
      launch_h_dir(h->stream, h->d_ctl, Av, r, p);
      launch_check(h->stream, h->d_ctl, nullptr, Av, b, x, h->d_part, 0);
    }
  });
  if (st != ASSG_OK) return st;
  int32_t status = ST_RUNNING;
  while (true) {
    HIP_OR_FAIL(h, hipGraphLaunch(h->g_hscg.exec, h->stream));
    HIP_OR_FAIL(h, hipMemcpyAsync(h->h_status, h->d_ctl, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    status = h->h_status[0];
    if (status != ST_RUNNING) break;
  }
  HIP_OR_FAIL(h, hipEventRecord(h->ev_stop, h->stream));
  if (status != ASSG_CONVERGED) {
    launch_check(h->stream, h->d_ctl, nullptr, Av, b, x, h->d_part, 1);
    HIP_OR_FAIL(h, hipGetLastError());
  }
  HIP_OR_FAIL(h, hipMemcpyAsync(c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIP_OR_FAIL(h, hipEventElapsedTime(&ms, h->ev_start, h->ev_stop));
  info->outcome = c->status;
  info->outer_iters = c->m;
  info->total_iters = c->m;
  info->relres_updated = c->relres_upd;
  info->relres_true = c->relres_true;
  info->lambda_min_est = NAN;
  info->lambda_max_est = NAN;
  info->c_last = NAN;
  info->solve_ms = ms;
  log_solve("hscg", n, 1, info);
  return debug_verdict(h);
}

assg_status_t assg_basis_gram(assg_handle_t h, const assg_csr_t* A, const double* p,
                              const double* r, int32_t s, const double* theta,
                              const double* gamma, const double* mu, double* Y_out,
                              double* G_out) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!p || !r || !theta || !gamma || (s > 1 && !mu) || !G_out)
    return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  if (s < 1 || s > ASSG_MAX_S) return fail(h, ASSG_ERR_INVALID_ARG, "s must be in 1..ASSG_MAX_S");
  assg_status_t st = check_analyzed(h, A);
  if (st != ASSG_OK) return st;
  const int64_t n = A->n;
  char* base = nullptr;
  WsLayout lay;
  st = get_workspace(h, n, s, nullptr, 0, &base, &lay);
  if (st != ASSG_OK) return st;
  double2* pairs = reinterpret_cast<double2*>(base + lay.pairs_off);
  double* plast = reinterpret_cast<double*>(base + lay.plast_off);
  double* grampart = reinterpret_cast<double*>(base + lay.grampart_off);
  const CsrView Av = view(h, A);
  Ctl* c = h->h_ctl;
  init_ctl(h, c, 0);
  c->sbar = s;
  c->sigma = s;
  for (int l = 0; l < s; ++l) {
    c->theta[l] = theta[l];
    c->gamma[l] = gamma[l];
    c->mu[l] = (l + 1 < s) ? mu[l] : 0.0;
  }
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_ctl, c, sizeof(Ctl), hipMemcpyHostToDevice, h->stream));
  refresh_dia(h, A);
  launch_pair_init(h->stream, n, p, r, pairs);
  for (int l = 1; l < s; ++l) launch_sweep(h->stream, h->d_ctl, l, Av, pairs, lay.ld);
  launch_last_gram(h->stream, h->d_ctl, s, Av, pairs, plast, lay.ld, grampart);
  launch_gram_reduce(h->stream, h->d_ctl, s, Av, grampart);
  if (Y_out) launch_export_Y(h->stream, n, s, pairs, plast, lay.ld, Y_out);
  HIP_OR_FAIL(h, hipGetLastError());
  HIP_OR_FAIL(h, hipMemcpyAsync(c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  const int nc = 2 * s + 1;
  for (int a = 0; a < nc; ++a)
    for (int bb = 0; bb < nc; ++bb) G_out[a * nc + bb] = c->G[a * MAXC + bb];
  return debug_verdict(h);
}

assg_status_t assg_block_controller(assg_handle_t h, const double* G, int32_t sbar, double nb,
                                    double tol, int32_t basis, int32_t s_max,
                                    assg_block_state_t* state, assg_block_result_t* res) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!G || !state || !res) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  if (s_max < 1 || s_max > ASSG_MAX_S || sbar < 1 || sbar > s_max)
    return fail(h, ASSG_ERR_INVALID_ARG, "need 1 <= sbar <= s_max <= ASSG_MAX_S");
  if (!(nb > 0.0) || !(tol > 0.0 && tol < 1.0))
    return fail(h, ASSG_ERR_INVALID_ARG, "need nb > 0 and tol in (0,1)");
  if (basis != ASSG_BASIS_MONOMIAL && basis != ASSG_BASIS_NEWTON && basis != ASSG_BASIS_CHEBYSHEV)
    return fail(h, ASSG_ERR_INVALID_ARG, "unknown basis");
  Ctl* c = h->h_ctl;
  init_ctl(h, c, 0);
  const int nc = 2 * sbar + 1;
  for (int a = 0; a < nc; ++a)
    for (int bb = 0; bb < nc; ++bb) c->G[a * MAXC + bb] = G[a * nc + bb];
  c->sbar = sbar;
  c->sigma = s_max;
  c->growth = s_max;
  c->basis = basis;
  c->tol = tol;
  c->nb = nb;
  c->max_iters = INT64_MAX / 2;
  c->max_outer = INT64_MAX / 2;
  c->m = state->m;
  c->c = state->c;
  c->psi = state->psi;
  c->alpha_prev = state->alpha_prev;
  c->beta_prev = state->beta_prev;
  c->mx_omega = state->mt_max_omega;
  c->mx_h = state->mt_max_h;
  c->mx_zeta = state->mt_max_zeta;
  c->mn_omega = state->mt_min_omega;
  c->mn_a = state->mt_min_a;
  c->mn_d = state->mt_min_d;
  c->mn_g = state->mt_min_g;
  c->mn_h = state->mt_min_h;
  c->lmin = state->lmin;
  c->lmax = state->lmax;
  for (int l = 0; l < MAXS; ++l) {
    c->theta[l] = state->theta[l];
    c->gamma[l] = state->gamma[l];
    c->mu[l] = state->mu[l];
  }
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_ctl, c, sizeof(Ctl), hipMemcpyHostToDevice, h->stream));
  launch_controller(h->stream, h->d_ctl, nullptr, s_max, 1);
  HIP_OR_FAIL(h, hipGetLastError());
  HIP_OR_FAIL(h, hipMemcpyAsync(c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  std::memset(res, 0, sizeof(*res));
  res->stilde = c->stilde;
  res->sk = c->sk;
  res->candidate = c->candidate;
  res->flags = (c->pending == ASSG_BREAKDOWN ? 1 : 0) | (c->pending == ASSG_DIVERGED ? 2 : 0);
  res->thr = c->thr;
  res->rho_m = c->rho_m;
  res->phi = c->phi;
  res->relres_updated = c->relres_upd;
  for (int l = 0; l < MAXS; ++l) {
    res->kappa[l] = c->kappa[l];
    res->alpha[l] = c->alphas[l];
    res->beta[l] = c->betas[l];
  }
  for (int i = 0; i < MAXC; ++i) {
    res->coef_x[i] = c->cx[i];
    res->coef_r[i] = c->cr[i];
    res->coef_p[i] = c->cp[i];
  }
  state->m = c->m;
  state->c = c->c;
  state->psi = c->psi;
  state->alpha_prev = c->alpha_prev;
  state->beta_prev = c->beta_prev;
  state->mt_max_omega = c->mx_omega;
  state->mt_max_h = c->mx_h;
  state->mt_max_zeta = c->mx_zeta;
  state->mt_min_omega = c->mn_omega;
  state->mt_min_a = c->mn_a;
  state->mt_min_d = c->mn_d;
  state->mt_min_g = c->mn_g;
  state->mt_min_h = c->mn_h;
  state->lmin = c->lmin;
  state->lmax = c->lmax;
  for (int l = 0; l < MAXS; ++l) {
    state->theta[l] = c->theta[l];
    state->gamma[l] = c->gamma[l];
    state->mu[l] = c->mu[l];
  }
  return debug_verdict(h);
}

}  // extern "C"
