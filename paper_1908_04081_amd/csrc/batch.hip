// C ABI of the batched solve (include/assg.h): a batch of independent
// systems is analyzed into one block-diagonal matrix with per-system control
// blocks, and its outer loops are replayed from a captured graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "handle.hpp"

using namespace assg;
using namespace assg::host;

namespace {

// The kernels' view of the analyzed batch.
CsrView batch_view(assg_handle_t h) {
  const auto& B = h->bat;
  CsrView v{};
  v.n = B.ntot;
  v.nnz = B.nnztot;
  v.rp = B.rpc;
  v.ci = B.cic;
  v.va = B.vac;
  v.blk = B.blk;
  v.blke = B.blke;
  v.nblk = B.nblk;
  v.bsys = B.bsys;
  v.cblk = B.chunks;
  v.csys = B.chunks + B.nchunk + 1;
  v.sys_chunk = B.chunks + 2 * B.nchunk + 1;
  v.nchunk = B.nchunk;
  v.nsys = B.nsys;
  if (B.fmt == ASSG_FORMAT_DIA) v.dia = B.dia.view;
  return v;
}

// Row blocks of every system, system i cut with the shape shape[i] = (rows,
// cap): global row starts, nonzero starts and the system of each block;
// sys_blk[i] = first block of system i.
void batch_blocks(const std::vector<std::vector<int32_t>>& rps, const std::vector<int64_t>& row0,
                  const std::vector<int64_t>& nz0, const std::vector<std::pair<int, int>>& shape,
                  std::vector<int32_t>& blk, std::vector<int32_t>& blke,
                  std::vector<int32_t>& bsys, std::vector<int32_t>& sys_blk) {
  blk.clear();
  blke.clear();
  bsys.clear();
  sys_blk.assign(1, 0);
  std::vector<int32_t> b;
  for (size_t i = 0; i < rps.size(); ++i) {
    const int64_t n = (int64_t)rps[i].size() - 1;
    make_blocks(rps[i].data(), n, b, shape[i].first, shape[i].second);
    for (size_t k = 0; k + 1 < b.size(); ++k) {
      blk.push_back((int32_t)(row0[i] + b[k]));
      blke.push_back((int32_t)(nz0[i] + rps[i][b[k]]));
      bsys.push_back((int32_t)i);
    }
    sys_blk.push_back((int32_t)blk.size());
  }
  const int64_t ntot = row0.back(), nnztot = nz0.back();
  blk.push_back((int32_t)ntot);
  blke.push_back((int32_t)nnztot);
}

// Size class of a system by its rows (see assg_batch_tuning).
int size_class(int64_t n) {
  return n < 4096 ? 0 : n < 65536 ? 1 : n < 1048576 ? 2 : 3;
}

// The tuner's choices for this process: (class, average nonzeros per row)
// -> (rows, cap).
std::mutex g_tune_mu;
std::map<std::pair<int, int>, std::pair<int, int>> g_tune_cache;

}  // namespace

namespace assg {
namespace host {

void batch_release(assg_handle_t h) {
  auto& B = h->bat;
  if (B.graph) (void)hipGraphExecDestroy(B.graph);
  for (void* p : {(void*)B.rpc, (void*)B.cic, (void*)B.vac, (void*)B.blk, (void*)B.blke,
                  (void*)B.bsys, (void*)B.chunks, (void*)B.part, (void*)B.dctl, (void*)B.b,
                  (void*)B.x, B.ws})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)B.hctl, (void*)B.hstat, (void*)B.hnb})
    if (p) (void)hipHostFree(p);
  dia_release(&B.dia);
  B = assg_handle_s::Batch();
}

}  // namespace host
}  // namespace assg

extern "C" {

// ---------------------------------------------------------------- batches
static constexpr int BATCH_LOOPS_PER_GRAPH = 4;
static const int TUNE_SHAPES[ASSG_TUNE_SHAPES][2] = {{256, 2048}, {256, 1024}, {128, 2048},
                                                     {128, 1024}, {64, 1024},  {64, 512}};

assg_status_t assg_batch_analyze(assg_handle_t h, int32_t nsys, const assg_csr_t* A) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!A || nsys < 1 || nsys > ASSG_MAX_BATCH)
    return fail(h, ASSG_ERR_INVALID_ARG, "nsys must be in 1..ASSG_MAX_BATCH");
  for (int i = 0; i < nsys; ++i)
    if (!csr_ok(&A[i])) return fail(h, ASSG_ERR_INVALID_ARG, "invalid CSR descriptor in batch");
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  batch_release(h);
  auto& B = h->bat;
  std::vector<std::vector<int32_t>> rps(nsys);
  std::vector<int64_t> row0(nsys + 1, 0), nz0(nsys + 1, 0);
  for (int i = 0; i < nsys; ++i) {
    rps[i].resize((size_t)A[i].n + 1);
    HIP_OR_FAIL(h, hipMemcpyAsync(rps[i].data(), A[i].row_ptr, rps[i].size() * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, h->stream));
    row0[i + 1] = row0[i] + A[i].n;
    nz0[i + 1] = nz0[i] + A[i].nnz;
  }
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (row0[nsys] >= (int64_t(1) << 31) || nz0[nsys] >= (int64_t(1) << 31))
    return fail(h, ASSG_ERR_INVALID_ARG, "batch too large (rows and nonzeros must be < 2^31)");
  for (int i = 0; i < nsys; ++i) {
    const auto& rp = rps[i];
    if (rp[0] != 0 || (int64_t)rp[A[i].n] != A[i].nnz)
      return fail(h, ASSG_ERR_INVALID_ARG, "row_ptr[0] must be 0 and row_ptr[n] must be nnz");
    for (int64_t r = 0; r < A[i].n; ++r)
      if (rp[r + 1] < rp[r]) return fail(h, ASSG_ERR_INVALID_ARG, "row_ptr must be nondecreasing");
    const assg_status_t st = check_columns(h, A[i].col_idx, A[i].nnz, A[i].n);
    if (st != ASSG_OK) return st;
  }
  B.nsys = nsys;
  B.ntot = row0[nsys];
  B.nnztot = nz0[nsys];
  for (int i = 0; i < nsys; ++i) {
    B.n.push_back(A[i].n);
    B.nnz.push_back(A[i].nnz);
    B.rp.push_back(A[i].row_ptr);
  }
  B.row0.assign(row0.begin(), row0.begin() + nsys);
  B.nz0.assign(nz0.begin(), nz0.begin() + nsys);
  // concatenated pattern and values
  std::vector<int32_t> rpc((size_t)B.ntot + 1);
  for (int i = 0; i < nsys; ++i)
    for (int64_t r = 0; r < A[i].n; ++r) rpc[row0[i] + r] = (int32_t)(nz0[i] + rps[i][r]);
  rpc[B.ntot] = (int32_t)B.nnztot;
  HIP_OR_FAIL(h, hipMalloc(&B.rpc, rpc.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMalloc(&B.cic, (size_t)B.nnztot * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMalloc(&B.vac, (size_t)B.nnztot * sizeof(double)));
  HIP_OR_FAIL(h, hipMalloc(&B.b, (size_t)B.ntot * sizeof(double)));
  HIP_OR_FAIL(h, hipMalloc(&B.x, (size_t)B.ntot * sizeof(double)));
  HIP_OR_FAIL(h, hipMemcpyAsync(B.rpc, rpc.data(), rpc.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  for (int i = 0; i < nsys; ++i) {
    launch_offset_copy(h->stream, A[i].col_idx, B.cic + nz0[i], A[i].nnz, (int32_t)row0[i]);
    HIP_OR_FAIL(h, hipMemcpyAsync(B.vac + nz0[i], A[i].val, (size_t)A[i].nnz * sizeof(double),
                                  hipMemcpyDeviceToDevice, h->stream));
  }
  HIP_OR_FAIL(h, hipGetLastError());
  HIP_OR_FAIL(h, hipMemsetAsync(B.x, 0, (size_t)B.ntot * sizeof(double), h->stream));

  // row-block shape per size class, the largest class first: time one
  // product of the whole batch for each candidate shape of the class (the
  // other classes keep their current shapes), unless the process cache has
  // a choice for the class
  std::vector<int32_t> blk, blke, bsys, sys_blk;
  std::vector<std::pair<int, int>> shape(nsys, {SB_ROWS, SB_CAP});
  for (int cl = ASSG_TUNE_CLASSES - 1; cl >= 0; --cl) {
    assg_tune_class_t& T = B.tune[cl];
    T = assg_tune_class_t{};
    std::vector<int> sel;
    int64_t cn = 0, cnz = 0;
    for (int i = 0; i < nsys; ++i)
      if (size_class(A[i].n) == cl) {
        sel.push_back(i);
        cn += A[i].n;
        cnz += A[i].nnz;
      }
    T.systems = (int32_t)sel.size();
    if (sel.empty()) continue;
    const std::pair<int, int> key{cl, (int)((cnz + cn / 2) / cn)};
    std::pair<int, int> pick{SB_ROWS, SB_CAP};
    bool cached = false;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      const auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        pick = it->second;
        cached = true;
      }
    }
    if (!cached) {
      double best = INFINITY;
      for (int c = 0; c < ASSG_TUNE_SHAPES; ++c) {
        std::vector<std::pair<int, int>> sh(shape);
        for (const int i : sel) sh[i] = {TUNE_SHAPES[c][0], TUNE_SHAPES[c][1]};
        batch_blocks(rps, row0, nz0, sh, blk, blke, bsys, sys_blk);
        int32_t *dblk = nullptr, *dblke = nullptr;
        HIP_OR_FAIL(h, hipMalloc(&dblk, blk.size() * sizeof(int32_t)));
        HIP_OR_FAIL(h, hipMalloc(&dblke, blke.size() * sizeof(int32_t)));
        HIP_OR_FAIL(h, hipMemcpyAsync(dblk, blk.data(), blk.size() * sizeof(int32_t),
                                      hipMemcpyHostToDevice, h->stream));
        HIP_OR_FAIL(h, hipMemcpyAsync(dblke, blke.data(), blke.size() * sizeof(int32_t),
                                      hipMemcpyHostToDevice, h->stream));
        CsrView v{};
        v.n = B.ntot;
        v.nnz = B.nnztot;
        v.rp = B.rpc;
        v.ci = B.cic;
        v.va = B.vac;
        v.blk = dblk;
        v.blke = dblke;
        v.nblk = (int32_t)blk.size() - 1;
        launch_spmv(h->stream, v, B.x, B.b);   // warm-up
        hipEvent_t e0 = pool_event(h, 0), e1 = pool_event(h, 1);
        if (!e0 || !e1) return fail(h, ASSG_ERR_HIP, "event creation failed");
        HIP_OR_FAIL(h, hipEventRecord(e0, h->stream));
        for (int r = 0; r < 5; ++r) launch_spmv(h->stream, v, B.x, B.b);
        HIP_OR_FAIL(h, hipEventRecord(e1, h->stream));
        HIP_OR_FAIL(h, hipGetLastError());
        HIP_OR_FAIL(h, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_OR_FAIL(h, hipEventElapsedTime(&ms, e0, e1));
        T.candidate_us[c] = 1e3 * ms / 5.0;
        if (T.candidate_us[c] < best) {
          best = T.candidate_us[c];
          pick = {TUNE_SHAPES[c][0], TUNE_SHAPES[c][1]};
        }
        HIP_OR_FAIL(h, hipFree(dblk));
        HIP_OR_FAIL(h, hipFree(dblke));
      }
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tune_cache[key] = pick;
    }
    T.rows = pick.first;
    T.nnz_cap = pick.second;
    T.cached = cached ? 1 : 0;
    for (const int i : sel) shape[i] = pick;
  }
  batch_blocks(rps, row0, nz0, shape, blk, blke, bsys, sys_blk);
  std::vector<int32_t> cblk, csys, sys_chunk;
  make_chunks(sys_blk, h->gram_blocks[10], cblk, csys, sys_chunk);
  if (cblk.size() - 1 > 4096)
    return fail(h, ASSG_ERR_INVALID_ARG, "too many systems for the reduction chunks");
  B.nblk = (int32_t)blk.size() - 1;
  B.nchunk = (int32_t)cblk.size() - 1;
  std::vector<int32_t> tab(cblk);
  tab.insert(tab.end(), csys.begin(), csys.end());
  tab.insert(tab.end(), sys_chunk.begin(), sys_chunk.end());
  HIP_OR_FAIL(h, hipMalloc(&B.blk, blk.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMalloc(&B.blke, blke.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMalloc(&B.bsys, bsys.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMalloc(&B.chunks, tab.size() * sizeof(int32_t)));
  HIP_OR_FAIL(h, hipMemcpyAsync(B.blk, blk.data(), blk.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(B.blke, blke.data(), blke.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(B.bsys, bsys.data(), bsys.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(B.chunks, tab.data(), tab.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMalloc(&B.part, reduce_doubles(B.nblk) * sizeof(double)));
  HIP_OR_FAIL(h, hipMalloc(&B.dctl, (size_t)nsys * sizeof(Ctl)));
  // the diagonal storage when every system fits it (assg_set_format; a
  // batch is read in one storage)
  B.fmt = ASSG_FORMAT_CSR;
  if (h->fmt_req != ASSG_FORMAT_CSR) {
    const bool forced = h->fmt_req == ASSG_FORMAT_DIA;
    std::vector<DiaSys> R(nsys);
    bool all = true;
    std::string why;
    for (int i = 0; i < nsys && all; ++i) {
      const assg_status_t st = dia_detect(h, &A[i], rps[i].data(), !forced, &R[i], &all, &why);
      if (st != ASSG_OK) return st;
      R[i].row0 = row0[i];
      if (!all) why = "system " + std::to_string(i) + ": " + why;
    }
    if (!all && forced) {
      batch_release(h);
      return fail(h, ASSG_ERR_UNSUPPORTED, "diagonal storage: " + why);
    }
    if (all) {
      const assg_status_t st = dia_build(h, R, h->gram_blocks[10], &B.dia);
      if (st == ASSG_ERR_ALLOC && forced) {
        batch_release(h);
        return fail(h, ASSG_ERR_ALLOC, "diagonal storage allocation failed");
      }
      if (st == ASSG_OK && B.dia.view.nchunk > 4096) {
        dia_release(&B.dia);
        if (forced) {
          batch_release(h);
          return fail(h, ASSG_ERR_INVALID_ARG, "too many systems for the reduction chunks");
        }
      } else if (st == ASSG_OK) {
        B.fmt = ASSG_FORMAT_DIA;
      } else if (st != ASSG_ERR_ALLOC) {
        return st;
      }
    }
  }
  HIP_OR_FAIL(h, hipHostMalloc(&B.hctl, (size_t)nsys * sizeof(Ctl), hipHostMallocDefault));
  HIP_OR_FAIL(h, hipHostMalloc(&B.hstat, (size_t)nsys * sizeof(int32_t), hipHostMallocDefault));
  HIP_OR_FAIL(h, hipHostMalloc(&B.hnb, (size_t)nsys * sizeof(double), hipHostMallocDefault));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));   // host tables above go out of scope
  h->err.clear();
  return ASSG_OK;
}

assg_status_t assg_batch_format(assg_handle_t h, int32_t* format) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!format) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  if (h->bat.nsys < 1) return fail(h, ASSG_ERR_NOT_ANALYZED, "no batch analyzed");
  *format = h->bat.fmt;
  return ASSG_OK;
}

assg_status_t assg_batch_tuning(assg_handle_t h, assg_tune_class_t* classes) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  if (!classes) return fail(h, ASSG_ERR_INVALID_ARG, "null argument");
  if (h->bat.nsys < 1) return fail(h, ASSG_ERR_NOT_ANALYZED, "no batch analyzed");
  for (int c = 0; c < ASSG_TUNE_CLASSES; ++c) classes[c] = h->bat.tune[c];
  return ASSG_OK;
}

// One outer loop of every system (the kernels of assg_solve's loop).
static void enqueue_batch_loop(assg_handle_t h, const CsrView& v, int sigma, double2* pairs,
                               double* plast, double* grampart, int64_t ld) {
  auto& B = h->bat;
  for (int l = 1; l < sigma; ++l) launch_sweep(h->stream, B.dctl, l, v, pairs, ld);
  launch_last_gram(h->stream, B.dctl, sigma, v, pairs, plast, ld, grampart);
  launch_gram_reduce(h->stream, B.dctl, sigma, v, grampart);
  launch_controller(h->stream, B.dctl, nullptr, sigma, B.nsys);
  launch_recover(h->stream, B.dctl, v, pairs, plast, ld, B.x);
  launch_check(h->stream, B.dctl, nullptr, v, B.b, B.x, B.part, 0);
}

assg_status_t assg_batch_solve(assg_handle_t h, int32_t nsys, const assg_csr_t* A,
                               const double* const* b, double* const* x, const assg_opts_t* opts,
                               assg_info_t* info) {
  if (!h) return ASSG_ERR_INVALID_ARG;
  auto& B = h->bat;
  if (B.nsys < 1) return fail(h, ASSG_ERR_NOT_ANALYZED, "no batch analyzed");
  if (!A || !b || !x || !info || nsys != B.nsys)
    return fail(h, ASSG_ERR_INVALID_ARG, "batch arguments do not match the analyzed batch");
  assg_status_t st = validate_opts(h, opts);
  if (st != ASSG_OK) return st;
  if (opts->record_trace) return fail(h, ASSG_ERR_INVALID_ARG, "no traces for batch solves");
  for (int i = 0; i < nsys; ++i) {
    if (A[i].n != B.n[i] || A[i].nnz != B.nnz[i] || A[i].row_ptr != B.rp[i] || !A[i].val)
      return fail(h, ASSG_ERR_NOT_ANALYZED, "system differs from assg_batch_analyze");
    if (!b[i] || !x[i]) return fail(h, ASSG_ERR_INVALID_ARG, "null right-hand side or iterate");
  }
  const int sigma = opts->s_max;
  const WsLayout lay = ws_layout(B.ntot, sigma);
  if (B.ws_bytes < lay.total) {
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    if (B.ws) HIP_OR_FAIL(h, hipFree(B.ws));
    B.ws = nullptr;
    B.ws_bytes = 0;
    if (B.graph) HIP_OR_FAIL(h, hipGraphExecDestroy(B.graph));
    B.graph = nullptr;
    if (hipMalloc(&B.ws, lay.total) != hipSuccess) {
      B.ws = nullptr;
      return fail(h, ASSG_ERR_ALLOC, "batch workspace allocation failed");
    }
    B.ws_bytes = lay.total;
  }
  char* base = static_cast<char*>(B.ws);
  double2* pairs = reinterpret_cast<double2*>(base + lay.pairs_off);
  double* plast = reinterpret_cast<double*>(base + lay.plast_off);
  double* grampart = reinterpret_cast<double*>(base + lay.grampart_off);
  const CsrView v = batch_view(h);

  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, h->user_stream));
  HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->ev_in, 0));
  for (int i = 0; i < nsys; ++i) {
    if (B.fmt == ASSG_FORMAT_DIA)
      launch_dia_fill(h->stream, A[i].row_ptr, A[i].col_idx, A[i].val, B.dia.rec[i],
                      B.dia.val + B.dia.rec[i].val0);
    HIP_OR_FAIL(h, hipMemcpyAsync(B.vac + B.nz0[i], A[i].val, (size_t)B.nnz[i] * sizeof(double),
                                  hipMemcpyDeviceToDevice, h->stream));
    HIP_OR_FAIL(h, hipMemcpyAsync(B.b + B.row0[i], b[i], (size_t)B.n[i] * sizeof(double),
                                  hipMemcpyDeviceToDevice, h->stream));
    HIP_OR_FAIL(h, hipMemcpyAsync(B.x + B.row0[i], x[i], (size_t)B.n[i] * sizeof(double),
                                  hipMemcpyDeviceToDevice, h->stream));
  }
  for (int i = 0; i < nsys; ++i) {
    Ctl* c = B.hctl + i;
    init_ctl(h, c, 0);
    const int64_t max_iters = opts->max_iters > 0 ? opts->max_iters : 10 * B.n[i];
    c->sbar = opts->s_init > 0 ? opts->s_init : opts->s_max;
    c->sbar_next = c->sbar;
    c->sigma = sigma;
    c->growth = opts->growth > 0 ? opts->growth : opts->s_max;
    c->basis = opts->basis;
    c->record_trace = 0;
    c->max_outer = opts->max_outer > 0 ? opts->max_outer : max_iters;
    c->max_iters = max_iters;
    c->tol = opts->tol;
    apply_variant(c, opts);
  }
  HIP_OR_FAIL(h, hipMemcpyAsync(B.dctl, B.hctl, (size_t)nsys * sizeof(Ctl),
                                hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipEventRecord(h->ev_start, h->stream));
  launch_setup(h->stream, B.dctl, v, B.b, B.x, pairs, B.part);
  HIP_OR_FAIL(h, hipGetLastError());
  // b_i = 0: x_i = 0, converged (nothing to iterate)
  HIP_OR_FAIL(h, hipMemcpy2DAsync(B.hnb, sizeof(double), &B.dctl->nb, sizeof(Ctl), sizeof(double),
                                  nsys, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < nsys; ++i)
    if (B.hnb[i] == 0.0) {
      B.hstat[i] = ASSG_CONVERGED;
      HIP_OR_FAIL(h, hipMemcpyAsync(&B.dctl[i].status, &B.hstat[i], sizeof(int32_t),
                                    hipMemcpyHostToDevice, h->stream));
      HIP_OR_FAIL(h, hipMemsetAsync(B.x + B.row0[i], 0, (size_t)B.n[i] * sizeof(double),
                                    h->stream));
    }

  // the outer loops: a captured graph of BATCH_LOOPS_PER_GRAPH loops, replayed
  if (!B.graph || B.graph_sigma != sigma) {
    if (B.graph) HIP_OR_FAIL(h, hipGraphExecDestroy(B.graph));
    B.graph = nullptr;
    hipGraph_t g = nullptr;
    HIP_OR_FAIL(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
    for (int r = 0; r < BATCH_LOOPS_PER_GRAPH; ++r)
      enqueue_batch_loop(h, v, sigma, pairs, plast, grampart, lay.ld);
    const hipError_t ce = hipStreamEndCapture(h->stream, &g);
    if (ce != hipSuccess) return fail(h, ASSG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
    const hipError_t ie = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      B.graph = nullptr;
      return fail(h, ASSG_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(ie));
    }
    B.graph_sigma = sigma;
  }
  while (true) {
    HIP_OR_FAIL(h, hipGraphLaunch(B.graph, h->stream));
    HIP_OR_FAIL(h, hipMemcpy2DAsync(B.hstat, sizeof(int32_t), &B.dctl->status, sizeof(Ctl),
                                    sizeof(int32_t), nsys, hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    bool running = false;
    for (int i = 0; i < nsys && !running; ++i) running = B.hstat[i] == ST_RUNNING;
    if (!running) break;
  }
  HIP_OR_FAIL(h, hipEventRecord(h->ev_stop, h->stream));
  launch_check(h->stream, B.dctl, nullptr, v, B.b, B.x, B.part, 1);   // true residual of each
  HIP_OR_FAIL(h, hipGetLastError());
  for (int i = 0; i < nsys; ++i)
    HIP_OR_FAIL(h, hipMemcpyAsync(x[i], B.x + B.row0[i], (size_t)B.n[i] * sizeof(double),
                                  hipMemcpyDeviceToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(B.hctl, B.dctl, (size_t)nsys * sizeof(Ctl), hipMemcpyDeviceToHost,
                                h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIP_OR_FAIL(h, hipEventElapsedTime(&ms, h->ev_start, h->ev_stop));
  for (int i = 0; i < nsys; ++i) {
    const Ctl* c = B.hctl + i;
    assg_info_t& o = info[i];
    std::memset(&o, 0, sizeof(o));
    o.outcome = c->status;
    o.outer_iters = completed_loops(c);
    o.total_iters = c->m;
    o.relres_updated = c->relres_upd;
    o.relres_true = c->relres_true;
    o.lambda_min_est = c->lmin;
    o.lambda_max_est = c->lmax;
    o.c_last = c->c;
    o.solve_ms = ms;
    log_solve("batch system", B.n[i], opts->s_max, &o);
  }
  return debug_verdict(h);
}

}  // extern "C"
