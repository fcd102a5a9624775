// The library handle and the host helpers shared by the C ABI files
// (api.hip: single systems and HSCG; batch.hip: batches).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "assg.h"
#include "ctl.hpp"
#include "launch.hpp"

// Diagonal storage of an analysis (single system or batch): the kernels'
// view, the systems' records (host copy, for the refills) and the device
// buffers.
struct DiaStore {
  assg::DiaView view{};                // view.nd = 0: not in use
  std::vector<assg::DiaSys> rec;
  double* val = nullptr;
  assg::DiaSys* sys = nullptr;
  int32_t* tab = nullptr;              // blk, bsys, cblk, csys, sys_chunk
};

// The state behind an assg_handle_t.
struct assg_handle_s {
  int device = 0;
  int cus = 256;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_start = nullptr, ev_stop = nullptr;
  assg::Ctl* d_ctl = nullptr;
  assg::Ctl* h_ctl = nullptr;          // pinned mirror
  int32_t* h_status = nullptr;   // pinned
  int32_t* d_flag = nullptr;     // device flag of the analysis checks
  assg_trace_t* d_trace = nullptr;
  int64_t trace_cap = 0;
  int64_t trace_count = 0;
  void* scratch = nullptr;       // this device's no-alloc scratch (device address)
  int32_t* d_forced = nullptr;   // schedule of assg_solve_forced_schedule
  int64_t forced_cap = 0;
  void* ws = nullptr;            // owned workspace
  size_t ws_bytes = 0;
  // analysis
  int64_t an_n = -1, an_nnz = -1;
  const int32_t* an_rp = nullptr;
  const int32_t* an_ci = nullptr;
  int32_t* d_blk = nullptr;      // row-block partition (row starts, nonzero starts)
  int32_t* d_blke = nullptr;
  int32_t nblk = 0;
  int32_t* d_chunks = nullptr;   // chunk starts (nchunk + 1) then system chunk starts (2)
  int32_t nchunk = 0;
  double* d_part = nullptr;      // per-workgroup partial sums (sized at analyze)
  // storage of A's values for the matrix-powers kernels (assg_set_format)
  int32_t fmt_req = ASSG_FORMAT_AUTO;
  int32_t fmt = ASSG_FORMAT_CSR;          // chosen by the last analysis
  DiaStore dia;                           // in use when fmt is ASSG_FORMAT_DIA
  int gram_blocks[assg::MAXS + 1] = {0};   // resident last-sweep workgroups per sigma (chunk count)
  // captured graphs of the single solve's outer loops and of HSCG iterations,
  // valid while the pointers and sizes they were captured with are unchanged
  struct GraphCache {
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> key;
  } g_sstep, g_hscg;
  // batch analysis (assg_batch_analyze) and its solve state
  struct Batch {
    int32_t nsys = 0;
    std::vector<int64_t> n, nnz, row0, nz0;   // sizes and offsets in the concatenation
    std::vector<const int32_t*> rp;            // the caller's row pointers (identity check)
    int64_t ntot = 0, nnztot = 0;
    int32_t *rpc = nullptr, *cic = nullptr;    // concatenated pattern
    double* vac = nullptr;                     // concatenated values (copied per solve)
    int32_t *blk = nullptr, *blke = nullptr, *bsys = nullptr, *chunks = nullptr;
    int32_t nblk = 0, nchunk = 0;
    double* part = nullptr;
    assg::Ctl* dctl = nullptr;
    assg::Ctl* hctl = nullptr;                       // pinned, nsys
    int32_t* hstat = nullptr;                  // pinned, nsys
    double* hnb = nullptr;                     // pinned, nsys
    double *b = nullptr, *x = nullptr;         // concatenated right-hand sides / iterates
    void* ws = nullptr;
    size_t ws_bytes = 0;
    assg_tune_class_t tune[ASSG_TUNE_CLASSES] = {};        // the tuner's choice per size class
    hipGraphExec_t graph = nullptr;            // captured outer loops
    int graph_sigma = 0;
    int32_t fmt = ASSG_FORMAT_CSR;             // storage the batch analysis chose
    DiaStore dia;
    std::vector<const int32_t*> ci;            // the caller's column indices (refills)
  } bat;
  double leja[assg::MAXS];
  std::string err;
  std::vector<hipEvent_t> evpool;
};

namespace assg {
namespace host {

#define HIP_OR_FAIL(h, call)                                                         \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail((h), ASSG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Workspace: the basis (s_max pair vectors + P_s; for HSCG r, two p
// buffers and w in the same region) and the Gram partials.
struct WsLayout {
  int64_t ld;
  size_t pairs_off, plast_off, grampart_off, total;
};

WsLayout ws_layout(int64_t n, int32_t s_max);
assg_status_t fail(assg_handle_t h, assg_status_t st, const std::string& msg);
bool csr_ok(const assg_csr_t* A);
// True when the n-element vectors at a and b share any element.
inline bool overlap(const double* a, const double* b, int64_t n) {
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  const uintptr_t len = static_cast<uintptr_t>(n) * sizeof(double);
  return pa < pb + len && pb < pa + len;
}
// Column indices of A inside [0, n), checked on the device (analysis time).
assg_status_t check_columns(assg_handle_t h, const int32_t* ci, int64_t nnz, int64_t n);
assg_status_t validate_opts(assg_handle_t h, const assg_opts_t* o);
// Rewrites the single analysis's diagonal storage from A's CSR values when
// it chose that storage (enqueued on the handle's stream; nothing otherwise).
void refresh_dia(assg_handle_t h, const assg_csr_t* A);
// Diagonal storage of one system: the offsets of 64 sampled rows (rp: its
// row pointers on the host), checked on every row on the device.  *fits is
// false (why set) when an entry lies off at most DIA_MAX diagonals, or, with
// check_fill, when the diagonals hold more than 15% more positions than A
// has entries; R gets n, nd and the offsets.
assg_status_t dia_detect(assg_handle_t h, const assg_csr_t* A, const int32_t* rp, bool check_fill,
                         DiaSys* R, bool* fits, std::string* why);
// Allocates the storage of the systems in R (their val0 set here; row0 and
// row counts as given) with blocks of at most SB_ROWS rows per system and
// reduction chunks over them; an allocation failure leaves S empty and
// returns ASSG_ERR_ALLOC.
assg_status_t dia_build(assg_handle_t h, std::vector<DiaSys>& R, int chunk_target, DiaStore* S);
void dia_release(DiaStore* S);
void init_ctl(assg_handle_t h, Ctl* c, int mode);
void apply_variant(Ctl* c, const assg_opts_t* o);
int64_t completed_loops(const Ctl* c);
// Debug builds: ASSG_ERR_HIP when a kernel check failed since the last call
// (release builds: always ASSG_OK, no device access).
assg_status_t debug_verdict(assg_handle_t h);
// Host-side logging of finished solves to stderr when ASSG_LOG=1.
void log_solve(const char* what, int64_t n, int sigma, const assg_info_t* info);
hipEvent_t pool_event(assg_handle_t h, size_t i);
void batch_release(assg_handle_t h);

// The graph of ``enqueue``'s launches on the handle's stream for ``key``:
// captured and instantiated when the key differs from the cached one.
// Forgets a cached graph (its kernels hold the partition tables and sizes of
// the analysis they were captured under).
inline void drop_graph(assg_handle_s::GraphCache& gc) {
  if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
  gc.exec = nullptr;
  gc.key.clear();
}

template <class F>
assg_status_t cached_graph(assg_handle_t h, assg_handle_s::GraphCache& gc,
                           const std::vector<const void*>& key, F enqueue) {
  if (gc.exec && gc.key == key) return ASSG_OK;
  if (gc.exec) HIP_OR_FAIL(h, hipGraphExecDestroy(gc.exec));
  gc.exec = nullptr;
  gc.key.clear();
  hipGraph_t g = nullptr;
  HIP_OR_FAIL(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
  enqueue();
  const hipError_t ce = hipStreamEndCapture(h->stream, &g);
  if (ce != hipSuccess)
    return fail(h, ASSG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  const hipError_t ie = hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    gc.exec = nullptr;
    return fail(h, ASSG_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(ie));
  }
  gc.key = key;
  return ASSG_OK;
}

}  // namespace host
}  // namespace assg
