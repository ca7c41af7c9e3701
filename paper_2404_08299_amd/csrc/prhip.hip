// Host side of libprhip.so: the C ABI of include/prhip.h.
//
// Method: S. Sahu, "Efficient GPU Implementation of Static and Incrementally
// Expanding DF-P PageRank for Dynamic Graphs" (arXiv 2404.08299), Alg. 1-5.
//
// Control flow per call: argument checks (no HIP call before they pass),
// workspace (grow-only, per device, reused), partition by degree (Alg. 4),
// initialisation, then the iteration loop. Each iteration enqueues the fused
// rank kernel, the L-infinity final reduction (which records the outcome in a
// device control block), for DF-P the apply/expand kernel, and an 8-byte-ish
// copy of the control block into pinned host memory. The host keeps up to
// `iters_per_sync` iterations in flight and waits only on the oldest one's
// copy, so the device does not idle on the host between iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "batched.h"
#include "apply.h"
#include "kernels.h"
#include "ppr.h"
#include "prhip.h"

using namespace prhip;

namespace {

thread_local hipStream_t t_stream = nullptr;
thread_local std::string t_err;
thread_local pr_stats t_stats;
thread_local int t_profiling = 0;

std::mutex g_mu;

pr_tuning default_tuning() {
  pr_tuning t;
  std::memset(&t, 0, sizeof(t));
  t.lane_max_degree = 128;
  t.wave_max_degree = 4096;
  t.expand_lane_max_degree = 32;
  t.iters_per_sync = 2;
  t.hub_chunk_edges = 4096;
  t.grid_blocks = 0;
  t.relabel = -1;
  t.xcd_split_degree = 129;
  t.expand_pull_per_mille = 20;
  t.frontier_list = 1;
  t.chain_numbering = -1;
  t.ppr_chunk_edges = 256;
  return t;
}
pr_tuning g_tuning = default_tuning();

constexpr int kRing = 8;  // pinned control-block snapshots

struct Workspace {
  size_t cap_n = 0, cap_chunks = 0, cap_partials = 0, cap_m = 0;
  int num_cus = 0;
  double *R1 = nullptr, *X0 = nullptr, *X1 = nullptr, *T = nullptr;
  uint8_t *flags = nullptr;  // dV | dN | cv, n bytes each
  uint32_t *fbits = nullptr;  // frontier bitmap, (n + 31) / 32 words
  int *hi_in = nullptr, *hi_out = nullptr;
  int *hub_start_in = nullptr, *hub_start_out = nullptr;  // [n + 1]
  int *chunk_hub_in = nullptr, *chunk_hub_out = nullptr;  // [cap_chunks]
  double *hub_part = nullptr;                             // [cap_chunks]
  double *w_out = nullptr;     // [m] edge weights in out-CSR order (adjoint)
  size_t cap_w_out = 0;
  int *alist = nullptr;        // [3][n] affected lists of DF/DF-P/DT (by iteration parity),
                               // then the frontier's wavefront-class vertices
  int *newid = nullptr;        // [n] gather-side numbering
  int *src_p = nullptr;        // [m] in-CSR sources in that numbering
  // DF/DF-P/DT chains (tuning chain_numbering): the numbering of such calls,
  // kept across them, and the in-CSR the last one mapped (row offsets,
  // sources, their numbers), two of each so that a call maps from one pair
  // while writing the other. nc_cur < 0: nothing kept.
  int *nc_newid = nullptr;
  int *nc_off[2] = {}, *nc_raw[2] = {}, *nc_map[2] = {};
  size_t nc_cap_n = 0, nc_cap_m = 0;
  int nc_cur = -1, nc_n = 0, nc_m[2] = {};
  long long nc_miss = 0, nc_built_m = 0;  // entries missed since the numbering was built
  int *tile_counts = nullptr;  // [kGroups][ntiles]
  int *counts = nullptr;       // [kNumCounts]
  int *group_totals = nullptr; // [kGroups]
  // die-split class: source range starts, scan totals, list offsets (small),
  // per-row chunk counts [kXcds + 1][nb] and the work items
  int *xrs = nullptr, *xtot = nullptr, *xoff = nullptr;
  int *xrt = nullptr;  // target ranges of the die-split expand (DF-P)
  int *xmat = nullptr;
  int4 *xitems = nullptr;
  size_t cap_xmat = 0, cap_xitems = 0;
  double *partials = nullptr;  // [cap_partials]
  // personalised PageRank: 4 [n][K] buffers (R, R', X, X'), chunk partials,
  // per-workgroup per-vector maxima, per-vector state
  double *ppr_buf = nullptr, *ppr_part = nullptr, *ppr_pmax = nullptr, *ppr_vdelta = nullptr;
  int *ppr_vdone = nullptr, *ppr_viters = nullptr;
  uint8_t *ppr_split = nullptr;
  size_t cap_ppr_buf = 0, cap_ppr_part = 0, cap_ppr_pmax = 0, cap_ppr_k = 0, cap_ppr_n = 0;
  // batched Static: union CSR, graph ids, per-graph state
  int *u_in_off = nullptr, *u_in_src = nullptr, *u_out_off = nullptr, *u_gid = nullptr;
  size_t cap_u_n = 0, cap_u_m = 0;
  int *b_vbase = nullptr, *b_ebase = nullptr, *b_gdone = nullptr, *b_giters = nullptr;
  double *b_c0 = nullptr, *b_gdelta = nullptr, *b_gpart = nullptr;
  BatchDesc *b_desc = nullptr;
  double **b_outs = nullptr;
  const double **b_tele = nullptr;  // [G] per-graph teleport vectors (null: uniform)
  hipGraphExec_t b_exec = nullptr;  // instantiated iteration graph, updated per call
  long long b_exec_key[4] = {};     // its launch shapes: graphs, grid, item dealing, kernel
  int *b_xrs = nullptr;  // [G][kXcds + 1] die-split ranges per graph
  size_t cap_b_g = 0, cap_b_part = 0;
  hipStream_t cap_stream = nullptr;
  hipEvent_t cap_ev[2] = {};
  Ctrl *ctrl = nullptr;
  Ctrl *host_ctrl = nullptr;  // pinned ring
  int *host_counts = nullptr;  // pinned
  int *host_xoff = nullptr;    // pinned copy of the die-split list offsets
  hipEvent_t sync_ev[kRing] = {};
  std::vector<hipEvent_t> prof_ev;
  hipEvent_t call_ev[2] = {};
  bool events_ready = false;
};
std::map<int, Workspace> g_ws;

int fail(int code, const std::string &msg) {
  t_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(PR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define LAUNCH_TRY()                                                                   \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess)                                                              \
      return fail(PR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_));   \
  } while (0)

void free_arrays(Workspace &w) {
  (void)hipFree(w.R1); (void)hipFree(w.X0); (void)hipFree(w.X1); (void)hipFree(w.T);
  (void)hipFree(w.flags); (void)hipFree(w.fbits); (void)hipFree(w.hi_in); (void)hipFree(w.hi_out);
  w.fbits = nullptr;
  (void)hipFree(w.hub_start_in); (void)hipFree(w.hub_start_out);
  (void)hipFree(w.chunk_hub_in); (void)hipFree(w.chunk_hub_out); (void)hipFree(w.hub_part);
  (void)hipFree(w.tile_counts); (void)hipFree(w.partials);
  (void)hipFree(w.newid); (void)hipFree(w.src_p); (void)hipFree(w.alist);
  w.newid = w.src_p = w.alist = nullptr;
  w.R1 = w.X0 = w.X1 = w.T = nullptr;
  w.flags = nullptr;
  w.hi_in = w.hi_out = w.hub_start_in = w.hub_start_out = nullptr;
  w.chunk_hub_in = w.chunk_hub_out = nullptr;
  w.hub_part = nullptr;
  w.tile_counts = nullptr;
  w.partials = nullptr;
  w.cap_n = w.cap_chunks = w.cap_partials = w.cap_m = 0;
}

void free_ppr(Workspace &w) {
  (void)hipFree(w.ppr_buf); (void)hipFree(w.ppr_part); (void)hipFree(w.ppr_pmax);
  (void)hipFree(w.ppr_vdelta); (void)hipFree(w.ppr_vdone); (void)hipFree(w.ppr_viters);
  (void)hipFree(w.ppr_split);
  w.ppr_buf = w.ppr_part = w.ppr_pmax = w.ppr_vdelta = nullptr;
  w.ppr_vdone = w.ppr_viters = nullptr;
  w.ppr_split = nullptr;
  w.cap_ppr_buf = w.cap_ppr_part = w.cap_ppr_pmax = w.cap_ppr_k = w.cap_ppr_n = 0;
}

void free_batch(Workspace &w) {
  (void)hipFree(w.u_in_off); (void)hipFree(w.u_in_src); (void)hipFree(w.u_out_off);
  (void)hipFree(w.u_gid); (void)hipFree(w.b_vbase); (void)hipFree(w.b_ebase);
  (void)hipFree(w.b_gdone); (void)hipFree(w.b_giters); (void)hipFree(w.b_c0);
  (void)hipFree(w.b_gdelta); (void)hipFree(w.b_gpart); (void)hipFree(w.b_desc);
  (void)hipFree(w.b_outs); (void)hipFree(w.b_xrs); (void)hipFree(w.b_tele);
  w.b_xrs = nullptr;
  w.b_tele = nullptr;
  if (w.b_exec) (void)hipGraphExecDestroy(w.b_exec);
  w.b_exec = nullptr;
  w.u_in_off = w.u_in_src = w.u_out_off = w.u_gid = nullptr;
  w.b_vbase = w.b_ebase = w.b_gdone = w.b_giters = nullptr;
  w.b_c0 = w.b_gdelta = w.b_gpart = nullptr;
  w.b_desc = nullptr;
  w.b_outs = nullptr;
  w.cap_u_n = w.cap_u_m = w.cap_b_g = w.cap_b_part = 0;
}

void free_chain(Workspace &w) {
  (void)hipFree(w.nc_newid);
  w.nc_newid = nullptr;
  for (int i = 0; i < 2; ++i) {
    (void)hipFree(w.nc_off[i]); (void)hipFree(w.nc_raw[i]); (void)hipFree(w.nc_map[i]);
    w.nc_off[i] = w.nc_raw[i] = w.nc_map[i] = nullptr;
  }
  w.nc_cap_n = w.nc_cap_m = 0;
  w.nc_cur = -1;
}

void free_xsplit(Workspace &w) {
  (void)hipFree(w.xmat); (void)hipFree(w.xitems);
  w.xmat = nullptr;
  w.xitems = nullptr;
  w.cap_xmat = w.cap_xitems = 0;
}

void free_ws(Workspace &w) {
  free_arrays(w);
  free_chain(w);
  free_xsplit(w);
  (void)hipFree(w.xrs);
  free_ppr(w);
  free_batch(w);
  if (w.cap_stream) (void)hipStreamDestroy(w.cap_stream);
  for (auto &e : w.cap_ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(w.w_out);
  w.w_out = nullptr;
  w.cap_w_out = 0;
  (void)hipFree(w.counts); (void)hipFree(w.group_totals); (void)hipFree(w.ctrl);
  if (w.host_ctrl) (void)hipHostFree(w.host_ctrl);
  if (w.host_counts) (void)hipHostFree(w.host_counts);
  if (w.host_xoff) (void)hipHostFree(w.host_xoff);
  if (w.events_ready) {
    for (auto &e : w.sync_ev) (void)hipEventDestroy(e);
    for (auto &e : w.call_ev) (void)hipEventDestroy(e);
  }
  for (auto &e : w.prof_ev) (void)hipEventDestroy(e);
  w = Workspace();
}

size_t ntiles_for(size_t n) { return (n + kPartTile - 1) / kPartTile; }
size_t flag_stride(size_t n) { return (n + 255) / 256 * 256; }

// Workgroups of a fixed-size launch: the tuning value, else as many as can
// be resident at once (occupancy of `kernel` times the compute units).
template <class K>
int grid_blocks(const Workspace &w, const pr_tuning &tn, K kernel) {
  if (tn.grid_blocks > 0) return tn.grid_blocks;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  return per_cu * std::max(1, w.num_cus);
}

// Die-split class under the current tuning: lower in-degree bound (0 = off),
// a bound on its row count (+1) and on its work items.
int xsplit_min_degree(const pr_tuning &tn) {
  if (tn.xcd_split_degree <= 0) return 0;
  return std::max(tn.xcd_split_degree, tn.lane_max_degree + 1);
}
size_t xsplit_rows_bound(size_t n, size_t m, int T) {
  return T ? std::min(n, m / (size_t)T) + 1 : 0;
}
size_t xsplit_items_bound(size_t n, size_t m, int CH, int T) {
  const size_t nb = xsplit_rows_bound(n, m, T);
  return nb ? kXcds * nb + m / (size_t)std::max(CH, 1) + kXcds : 0;
}

int xsplit_ws(Workspace &w, size_t nb, size_t items) {
  const size_t need_mat = (kXcds + 1) * nb;
  if (need_mat > w.cap_xmat || items > w.cap_xitems) {
    // 1/8 headroom, as for the workspace's edge-sized arrays
    const size_t a = std::max(need_mat + need_mat / 8, w.cap_xmat);
    const size_t b = std::max(items + items / 8, w.cap_xitems);
    free_xsplit(w);
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&w.xmat, a * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.xitems, b * sizeof(int4))) != hipSuccess) {
      (void)hipGetLastError();
      free_xsplit(w);
      return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP,
                  std::string("die-split workspace allocation: ") + hipGetErrorString(e));
    }
    w.cap_xmat = a;
    w.cap_xitems = b;
  }
  return PR_OK;
}

// Workspace for n vertices, m edges and chunk size CH (grow-only, per device).
int get_ws(size_t n, size_t m, int CH, int B, Workspace **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace &w = g_ws[dev];
  if (!w.events_ready) {
    for (auto &e : w.sync_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &e : w.call_ev) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipMalloc(&w.ctrl, sizeof(Ctrl)));
    HIP_TRY(hipMalloc(&w.counts, kNumCounts * sizeof(int)));
    HIP_TRY(hipMalloc(&w.group_totals, kGroups * sizeof(int)));
    HIP_TRY(hipMalloc(&w.xrs, 4 * 16 * sizeof(int)));
    w.xtot = w.xrs + 16;
    w.xoff = w.xrs + 32;
    w.xrt = w.xrs + 48;
    HIP_TRY(hipHostMalloc(&w.host_ctrl, kRing * sizeof(Ctrl), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&w.host_counts, kNumCounts * sizeof(int), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&w.host_xoff, 16 * sizeof(int), hipHostMallocDefault));
    HIP_TRY(hipDeviceGetAttribute(&w.num_cus, hipDeviceAttributeMultiprocessorCount, dev));
    w.events_ready = true;
  }
  if (B <= 0) B = 32 * std::max(1, w.num_cus);  // bound on any occupancy-derived grid
  // chunks of the split class: sum over its vertices of ceil(deg / CH)
  // <= m / CH + (number of split vertices) <= m / CH + n; die-split rows have
  // up to kXcds segments each
  const size_t need_chunks =
      std::max(m / (size_t)CH + n + 1, xsplit_items_bound(n, m, CH, xsplit_min_degree(g_tuning)));
  const size_t need_partials = (size_t)B + kHubFinalizeBlocks + 16;
  if (n > w.cap_n || m > w.cap_m || need_chunks > w.cap_chunks ||
      need_partials > w.cap_partials) {
    // the edge-sized arrays grow with 1/8 headroom: along a chain of updates
    // m drifts up by a batch at a time, and a reallocation per call would
    // cost more than the call
    const size_t nn = std::max(n, w.cap_n);
    const size_t mm = std::max(m + m / 8, w.cap_m);
    const size_t nc = std::max(need_chunks + need_chunks / 8, w.cap_chunks);
    const size_t np = std::max(need_partials, w.cap_partials);
    free_arrays(w);
    const size_t nt = ntiles_for(nn);
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&w.R1, nn * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.X0, nn * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.X1, nn * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.T, nn * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.flags, 3 * flag_stride(nn))) != hipSuccess ||
        (e = hipMalloc(&w.fbits, ((nn + 31) / 32 + 16) * sizeof(uint32_t))) != hipSuccess ||
        (e = hipMalloc(&w.hi_in, nn * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.hi_out, nn * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.hub_start_in, (nn + 1) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.hub_start_out, (nn + 1) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.chunk_hub_in, nc * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.chunk_hub_out, nc * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.hub_part, nc * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.tile_counts, (size_t)kGroups * nt * sizeof(int) + 64)) != hipSuccess ||
        (e = hipMalloc(&w.newid, nn * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.alist, 3 * nn * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.src_p, mm * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.partials, np * sizeof(double))) != hipSuccess) {
      (void)hipGetLastError();
      free_arrays(w);
      return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP,
                  std::string("workspace allocation: ") + hipGetErrorString(e));
    }
    w.cap_n = nn;
    w.cap_m = mm;
    w.cap_chunks = nc;
    w.cap_partials = np;
  }
  *out = &w;
  return PR_OK;
}

hipEvent_t prof_event(Workspace &w, size_t i) {
  while (w.prof_ev.size() <= i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    w.prof_ev.push_back(e);
  }
  return w.prof_ev[i];
}

// A caller's array must be device (or managed) memory of the current
// device: host memory handed to a kernel would fault the GPU, so it is
// refused here. NULL passes (whether an array is required is checked by the
// caller). Pageable host memory reads as unregistered, pinned host memory as
// host memory; both are refused.
int check_dev_ptr(const void *p, const char *name) {
  if (!p) return PR_OK;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(PR_EINVAL, std::string(name) + " is not device memory");
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(PR_EINVAL, std::string(name) + " is not device memory");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (a.type == hipMemoryTypeDevice && a.device != dev)
    return fail(PR_EINVAL, std::string(name) + " is memory of another device");
  return PR_OK;
}

int check_csr(const pr_csr *g, bool need_out_targets) {
  if (!g) return fail(PR_EINVAL, "csr is NULL");
  if (g->n <= 0) return fail(PR_EINVAL, "n must be > 0");
  if (g->m < g->n) return fail(PR_EINVAL, "m must be >= n (one self-loop per vertex)");
  if (!g->in_offsets || !g->in_sources || !g->out_offsets)
    return fail(PR_EINVAL, "in_offsets, in_sources and out_offsets are required");
  if (need_out_targets && !g->out_targets) return fail(PR_EINVAL, "out_targets is required");
  return PR_OK;
}

// The graph's arrays, and then up to four more, on the current device. Entry
// points call this after their scalar and structural checks, so those report
// first.
int on_device(const pr_csr *g, std::initializer_list<std::pair<const void *, const char *>> more) {
  int rc;
  if (g && ((rc = check_dev_ptr(g->in_offsets, "in_offsets")) ||
            (rc = check_dev_ptr(g->in_sources, "in_sources")) ||
            (rc = check_dev_ptr(g->out_offsets, "out_offsets")) ||
            (rc = check_dev_ptr(g->out_targets, "out_targets"))))
    return rc;
  for (const auto &pm : more)
    if ((rc = check_dev_ptr(pm.first, pm.second))) return rc;
  return PR_OK;
}

int edges_on_device(const pr_edges *e, const char *src_name, const char *dst_name) {
  if (!e || e->count <= 0) return PR_OK;
  int rc;
  if ((rc = check_dev_ptr(e->src, src_name)) || (rc = check_dev_ptr(e->dst, dst_name))) return rc;
  return PR_OK;
}

int check_params(double alpha, double tol, int max_iter) {
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(PR_EINVAL, "alpha must be in (0, 1)");
  if (!(tol >= 0.0)) return fail(PR_EINVAL, "tol must be >= 0");
  if (max_iter <= 0) return fail(PR_EINVAL, "max_iter must be > 0");
  return PR_OK;
}

// Alg. 4 on an offsets array: class lists into `hi`, class sizes into
// counts[slot], counts[slot + 1]; then the chunk plan of the split class.
// Work lists of the die-split class (null items: the class is off).
struct XPlan {
  const int4 *items = nullptr;
  const int *off = nullptr;
};

// Source ranges of the die split (w.xrs), balanced by the gather-side
// degrees goff.
int xcd_ranges(Workspace &w, const int *goff, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_xcd_ranges, dim3(1), dim3(64), 0, s, goff, (const int *)nullptr, n,
                     w.xrs);
  LAUNCH_TRY();
  return PR_OK;
}

// Degree classes of the rows `off` (Alg. 4 with three classes) and the plan of
// the top class. With `xidx` (the rows' original, ascending indices; needs
// the ranges in w.xrs) the top class is the die-split class of rows with
// degree >= Tx (Tx = 0: max(xsplit_min_degree, t1 + 1)); otherwise rows above
// t2, cut into chunks.
// Exclusive scan of `nrows` rows of `rows` (row r at rows + r * stride), each
// min(stride, *dlen) long (dlen a device count, or null), in place; totals[r]
// gets row r's sum. Rows longer than a few thousand entries are scanned by
// tiles over the whole chip, with `scratch` (cap ints, not `rows`) holding the
// tile sums; shorter rows by one workgroup each.
void scan_rows(int *rows, int nrows, int stride, int *totals, const int *dlen, int *scratch,
               size_t cap, hipStream_t s) {
  const int ntmax = (stride + kScanTile - 1) / kScanTile;
  if (stride <= 8 * kFinalBlock || (size_t)nrows * ntmax > cap || scratch == rows) {
    hipLaunchKernelGGL(k_scan_rows, dim3(nrows), dim3(kFinalBlock), 0, s, rows, stride, totals,
                       dlen);
    return;
  }
  hipLaunchKernelGGL(k_rows_tile_sums, dim3(ntmax, nrows), dim3(kBlock), 0, s,
                     (const int *)rows, stride, dlen, scratch, ntmax);
  hipLaunchKernelGGL(k_scan_rows, dim3(nrows), dim3(kFinalBlock), 0, s, scratch, ntmax, totals,
                     (const int *)nullptr);
  hipLaunchKernelGGL(k_rows_tile_apply, dim3(ntmax, nrows), dim3(kBlock), 0, s, rows, stride,
                     dlen, (const int *)scratch, ntmax);
}

int partition(Workspace &w, const int *off, int n, int m, int t1, int t2, int CH, int *hi,
              int slot, int chunk_slot, int *hub_start, int *chunk_hub, hipStream_t s,
              const int *xidx = nullptr, XPlan *xp = nullptr, const int *xrs = nullptr,
              const int *gid = nullptr, int Tx = 0) {
  if (!xrs) xrs = w.xrs;
  const int T = !xidx ? 0 : Tx > 0 ? Tx : std::max(xsplit_min_degree(g_tuning), t1 + 1);
  if (T) t2 = T - 1;
  const int nt = (int)ntiles_for(n);
  hipLaunchKernelGGL(k_part_count, dim3(nt), dim3(kBlock), 0, s, off, n, t1, t2, w.tile_counts,
                     nt);
  hipLaunchKernelGGL(k_scan_rows, dim3(2), dim3(kFinalBlock), 0, s, w.tile_counts, nt,
                     w.counts + slot, (const int *)nullptr);
  hipLaunchKernelGGL(k_part_scatter, dim3(nt), dim3(kBlock), 0, s, off, n, t1, t2,
                     w.tile_counts, nt, (const int *)(w.counts + slot), hi);
  if (!T) {
    hipLaunchKernelGGL(k_hub_plan, dim3(1), dim3(kFinalBlock), 0, s, off, (const int *)hi,
                       w.counts, slot, chunk_slot, CH, hub_start, chunk_hub);
    LAUNCH_TRY();
    if (xp) *xp = XPlan{};
    return PR_OK;
  }
  const size_t nb = xsplit_rows_bound((size_t)n, (size_t)m, T);
  int rc = xsplit_ws(w, nb, xsplit_items_bound((size_t)n, (size_t)m, CH, T));
  if (rc) return rc;
  const int gb = (int)std::min<size_t>((nb + kBlock - 1) / kBlock, 16 * std::max(1, w.num_cus));
  hipLaunchKernelGGL(k_xsplit_count, dim3(gb), dim3(kBlock), 0, s, off, xidx, (const int *)hi,
                     (const int *)w.counts, slot, xrs, gid, CH, (int)nb, w.xmat);
  scan_rows(w.xmat, kXcds + 1, (int)nb, w.xtot, (const int *)(w.counts + slot + 1), w.tile_counts,
            kGroups * ntiles_for(w.cap_n), s);
  hipLaunchKernelGGL(k_xsplit_fill, dim3(gb), dim3(kBlock), 0, s, off, xidx, (const int *)hi,
                     w.counts, slot, chunk_slot, xrs, gid, CH, (int)nb,
                     (const int *)w.xmat, (const int *)w.xtot, w.xoff, hub_start, w.xitems);
  LAUNCH_TRY();
  if (xp) *xp = XPlan{w.xitems, w.xoff};
  return PR_OK;
}

// The die-split list offsets of plan xp on the host (one wait on the stream),
// for item_lg below. No plan: nothing to read.
int read_plan(Workspace &w, const XPlan &xp, hipStream_t s) {
  if (!xp.items) return PR_OK;
  HIP_TRY(hipMemcpyAsync(w.host_xoff, xp.off, (kXcds + 1) * sizeof(int), hipMemcpyDeviceToHost,
                         s));
  HIP_TRY(hipStreamSynchronize(s));
  return PR_OK;
}

// How a grid of B workgroups deals out each die's items (see item_of): in
// runs of 16 when every one of the die's wavefronts gets kItemSpread runs of
// the shortest list, one by one otherwise. Returns LG (4 or 0).
int item_lg(const Workspace &w, const XPlan &xp, int B) {
  if (!xp.items) return 4;
  long long shortest = -1;
  for (int x = 0; x < kXcds; ++x) {
    const long long len = (long long)w.host_xoff[x + 1] - w.host_xoff[x];
    if (shortest < 0 || len < shortest) shortest = len;
  }
  const long long Wd = (long long)std::max(1, B / kXcds) * kWavesPerBlock;
  return shortest >= Wd * 16 * kItemSpread ? 4 : 0;
}

// Gather-side numbering (degree-based grouping by the degrees of
// `group_off`) and the row indices `idx` mapped into it. Returns the
// numbering to use (nullptr = identity) and the index array the pull kernels
// gather through.
struct Locality {
  const int *pos;
  const int *src;
};

bool relabel_on(const pr_tuning &tn, int n) {
  return tn.relabel > 0 || (tn.relabel < 0 && n >= (1 << 20));
}

// newid = the degree-based grouping of group_off (inside the ranges rs, if
// given).
int build_numbering(Workspace &w, int n, const int *group_off, const int *rs, int *newid,
                    hipStream_t s) {
  const int nt = (int)ntiles_for(n);
  hipLaunchKernelGGL(k_group_count, dim3(nt), dim3(kBlock), 0, s, group_off, n, w.tile_counts,
                     nt);
  hipLaunchKernelGGL(k_scan_rows, dim3(kGroups), dim3(kFinalBlock), 0, s, w.tile_counts, nt,
                     w.group_totals, (const int *)nullptr);
  hipLaunchKernelGGL(k_group_scatter, dim3(nt), dim3(kBlock), 0, s, group_off, n,
                     (const int *)w.tile_counts, (const int *)w.group_totals, nt, rs, newid);
  LAUNCH_TRY();
  return PR_OK;
}

// dst = newid applied to the entries of the in-CSR (row_off, idx): rows with
// at least T entries item by item along the die-split plan xp (if it has
// items), the others by k_map_short. From a kept mapping (MODE 2), whose
// hits read no newid and so gain nothing from the die split, k_map_short
// streams every row below kKeptItemLen entries too, and only the longer
// rows are left to the items.
constexpr int kKeptItemLen = 4096;

// MODE 2 needs dlist (n ints of scratch) for the rows of kKeptRowLen .. Ts - 1
// entries, which k_map_rows_kept maps after k_map_short.
template <int MODE>
int map_rows(Workspace &w, const XPlan &xp, const int *row_off, const int *idx, int n, int T,
             const int *newid, int *dst, const MapCache &c, hipStream_t s,
             int *dlist = nullptr) {
  const int Ts = MODE == 2 ? std::max(T, kKeptItemLen) : T;
  int *dcount = w.counts + kMapRows;
  if (MODE == 2) HIP_TRY(hipMemsetAsync(dcount, 0, sizeof(int), s));
  if (xp.items) {
    const int gs = kXcds * 4 * std::max(1, w.num_cus);
    auto map_fn = item_lg(w, xp, gs) ? k_map_split<4, MODE> : k_map_split<0, MODE>;
    hipLaunchKernelGGL(map_fn, dim3(gs), dim3(kBlock), 0, s, (const int4 *)xp.items,
                       (const int *)xp.off, row_off, idx, newid, dst, c, Ts);
  }
  // a few groups of 64 rows per wavefront, so that their offsets are
  // fetched ahead
  const int gr = (int)std::min<long long>(((long long)n + kBlock - 1) / kBlock,
                                          64LL * std::max(1, w.num_cus));
  hipLaunchKernelGGL(k_map_short<MODE>, dim3(gr), dim3(kBlock), 0, s, row_off, idx, n, Ts,
                     newid, dst, c, dlist, dcount);
  if (MODE == 2)
    hipLaunchKernelGGL(k_map_rows_kept, dim3(16 * std::max(1, w.num_cus)), dim3(kBlock), 0, s,
                       row_off, idx, newid, dst, c, (const int *)dlist, (const int *)dcount);
  LAUNCH_TRY();
  return PR_OK;
}

// With a die-split plan `xp` over the rows of row_off (those with at least T
// entries, ranges rs), the split rows are mapped on the die that owns each
// segment and the shorter rows by k_map_short; otherwise one edge-parallel
// pass maps every entry.
int locality(Workspace &w, int n, int m, const int *group_off, const int *idx,
             const pr_tuning &tn, bool allowed, hipStream_t s, Locality *out,
             const int *rs = nullptr, const XPlan *xp = nullptr, const int *row_off = nullptr,
             int T = 0) {
  if (!allowed || !relabel_on(tn, n)) {
    *out = Locality{nullptr, idx};
    return PR_OK;
  }
  int rc = build_numbering(w, n, group_off, rs, w.newid, s);
  if (rc) return rc;
  t_stats.numbering = 1;
  if (xp && xp->items && rs && row_off && T > 0) {
    if ((rc = map_rows<0>(w, *xp, row_off, idx, n, T, w.newid, w.src_p, MapCache{}, s)))
      return rc;
  } else {
    const int mb = std::min((m + kBlock - 1) / kBlock, 8 * std::max(1, w.num_cus) * 4);
    hipLaunchKernelGGL(k_map_sources, dim3(mb), dim3(kBlock), 0, s, idx, m, (const int *)w.newid,
                       w.src_p);
    LAUNCH_TRY();
  }
  *out = Locality{w.newid, w.src_p};
  return PR_OK;
}

// Storage of the numbering kept along DF/DF-P/DT chains (grow-only; the edge
// arrays get 1/16 headroom, as a chain's edge count drifts). Growing drops
// what was kept.
int chain_ws(Workspace &w, size_t n, size_t m) {
  if (n <= w.nc_cap_n && m <= w.nc_cap_m) return PR_OK;
  const size_t nn = std::max(n, w.nc_cap_n), mm = std::max(m + m / 16 + 1024, w.nc_cap_m);
  free_chain(w);
  hipError_t e = hipMalloc(&w.nc_newid, nn * sizeof(int));
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    if ((e = hipMalloc(&w.nc_off[i], (nn + 1) * sizeof(int))) != hipSuccess) break;
    if ((e = hipMalloc(&w.nc_raw[i], mm * sizeof(int))) != hipSuccess) break;
    e = hipMalloc(&w.nc_map[i], mm * sizeof(int));
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    free_chain(w);
    return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP,
                std::string("chain numbering allocation: ") + hipGetErrorString(e));
  }
  w.nc_cap_n = nn;
  w.nc_cap_m = mm;
  return PR_OK;
}

// Kept numbering is rebuilt once the entries that its kept mappings did not
// find, added over the calls since it was built, pass 1/kChainRebuild of the
// edges it was built on (a measure of how far the graph has moved from it).
constexpr long long kChainRebuild = 8;

// Gather-side numbering of a DF/DF-P/DT call with the die split (arguments
// as for locality). With chain_numbering on, the numbering is kept across
// such calls on graphs of n vertices, and each call maps its in-CSR from the
// mapping the previous one left (MapCache: a streamed copy wherever the rows
// match, the numbering itself elsewhere) and leaves its own. The rank sums
// do not depend on the numbering (rows keep their order, and the die
// segments follow this call's ranges rs), so the ranks are the same bits
// whether the numbering is kept or built anew.
int locality_chain(Workspace &w, int n, int m, const int *group_off, const int *idx,
                   const pr_tuning &tn, hipStream_t s, Locality *out, const int *rs,
                   const XPlan &xp, const int *row_off, int T, int *dlist) {
  if (tn.chain_numbering == 0 && w.nc_cap_n) {
    HIP_TRY(hipStreamSynchronize(s));
    free_chain(w);  // turned off: what was kept is released
  }
  // automatic: kept from 2^23 vertices on. Below, each die's eighth of the
  // numbering (4n / 8 bytes) fits its 4 MB L2, so the fresh map's lookups hit
  // L2 and its 8 bytes per entry beat the kept map's 20.
  const bool on = tn.chain_numbering > 0 || (tn.chain_numbering < 0 && n >= (1 << 23));
  if (!on || !relabel_on(tn, n) || !rs || T <= 0)
    return locality(w, n, m, group_off, idx, tn, true, s, out, rs, &xp, row_off, T);
  int rc = chain_ws(w, (size_t)n, (size_t)m);
  if (rc == PR_ENOMEM) {  // no room to keep it: built inside the call, as with 0
    t_err.clear();
    return locality(w, n, m, group_off, idx, tn, true, s, out, rs, &xp, row_off, T);
  }
  if (rc) return rc;
  const int cur = w.nc_cur;
  const bool keep = cur >= 0 && w.nc_n == n && w.nc_miss * kChainRebuild <= w.nc_built_m;
  const int nx = cur >= 0 ? 1 - cur : 0;
  w.nc_cur = -1;  // until this call's mapping is enqueued
  MapCache c{};
  c.raw_out = w.nc_raw[nx];
  c.off_out = w.nc_off[nx];
  if (keep) {
    c.old_off = w.nc_off[cur];
    c.old_raw = w.nc_raw[cur];
    c.old_map = w.nc_map[cur];
    c.old_m = w.nc_m[cur];
    c.miss = w.counts + kMapMiss;
    HIP_TRY(hipMemsetAsync(c.miss, 0, sizeof(int), s));
    rc = map_rows<2>(w, xp, row_off, idx, n, T, w.nc_newid, w.nc_map[nx], c, s, dlist);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(w.host_counts + kMapMiss, c.miss, sizeof(int),
                           hipMemcpyDeviceToHost, s));
  } else {
    if ((rc = build_numbering(w, n, group_off, rs, w.nc_newid, s))) return rc;
    rc = map_rows<1>(w, xp, row_off, idx, n, T, w.nc_newid, w.nc_map[nx], c, s);
    if (rc) return rc;
    w.host_counts[kMapMiss] = 0;
    w.nc_miss = 0;
    w.nc_built_m = m;
  }
  w.nc_cur = nx;
  w.nc_n = n;
  w.nc_m[nx] = m;
  t_stats.numbering = keep ? 2 : 1;
  *out = Locality{w.nc_newid, w.nc_map[nx]};
  return PR_OK;
}

struct CallTimer {
  Workspace &w;
  hipStream_t s;
  bool on;
  CallTimer(Workspace &w_, hipStream_t s_) : w(w_), s(s_), on(t_profiling != 0) {
    if (on) (void)hipEventRecord(w.call_ev[0], s);
  }
  void stop() {
    if (on) (void)hipEventRecord(w.call_ev[1], s);
  }
  double ms() {
    float f = 0.f;
    if (on && hipEventElapsedTime(&f, w.call_ev[0], w.call_ev[1]) == hipSuccess) return f;
    return 0.0;
  }
};

// The iteration loop shared by Static and DF/DF-P. `launch(it)` enqueues the
// work of iteration `it` between the profiling events.
template <class F>
int iterate(Workspace &w, hipStream_t s, int max_iter, F &&launch, int *iters_out,
            int *launched_out) {
  const int K = std::max(1, std::min(g_tuning.iters_per_sync, kRing - 1));
  int it = 0;
  bool done = false;
  while (it < max_iter && !done) {
    if (t_profiling) {
      hipEvent_t a = prof_event(w, 2 * (size_t)it), b = prof_event(w, 2 * (size_t)it + 1);
      if (!a || !b) return fail(PR_EHIP, "hipEventCreate failed");
      HIP_TRY(hipEventRecord(a, s));
      int rc = launch(it, true, b);
      if (rc) return rc;
    } else {
      int rc = launch(it, false, nullptr);
      if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(&w.host_ctrl[it % kRing], w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipEventRecord(w.sync_ev[it % kRing], s));
    ++it;
    const int j = it - K;
    if (j >= 0) {
      HIP_TRY(hipEventSynchronize(w.sync_ev[j % kRing]));
      if (w.host_ctrl[j % kRing].done) done = true;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  const Ctrl &last = w.host_ctrl[(it - 1) % kRing];
  *iters_out = last.done ? last.iters : std::min(it, max_iter);
  *launched_out = it;
  t_stats.converged = last.done;
  t_stats.final_delta = last.delta;
  t_stats.iterations = *iters_out;
  return PR_OK;
}

void collect_profile(Workspace &w, int iters) {
  if (!t_profiling) return;
  double tot = 0.0;
  for (int i = 0; i < iters; ++i) {
    float f = 0.f;
    if (hipEventElapsedTime(&f, w.prof_ev[2 * i], w.prof_ev[2 * i + 1]) == hipSuccess) tot += f;
  }
  t_stats.rank_kernel_ms = tot;
  t_stats.rank_kernel_launches = iters;
}

void reset_stats() {
  std::memset(&t_stats, 0, sizeof(t_stats));
  t_stats.affected_initial = -1;
  t_stats.affected_max = -1;
  t_stats.edges_processed = -1;
  t_err.clear();
}

// One full-pull iteration problem:
//   x_new[v] = tele ? tscale * tele[v] + alpha * S(v) : (1 - alpha)/n + alpha * S(v)
//   S(v) = sum over row v of (w ? w[e] * x[idx[e]] : x[idx[e]] / |out(idx[e])|)
// Static (Alg. 1, Eq. 1), Naive-dynamic (init = R^{t-1}), the weighted
// forward and the adjoint iteration are instances.
struct PullProblem {
  int n, m;
  const int *row_off, *row_idx;  // CSR pulled over (rows = updated vertices)
  const int *deg_off;            // offsets giving |out(u)| (unweighted only)
  const int *group_off;          // degrees that group the gather side
  const double *w;               // per-edge weights aligned with row_idx, or null
  const double *tele;            // teleport term or null
  double tscale;
  const double *init;            // start vector or null (then r0)
  double r0;
  bool relabel;                  // gather-side renumbering allowed
};

int run_pull(const PullProblem &P, double alpha, double tol, int max_iter, double *ranks_out) {
  hipStream_t s = t_stream;
  const int n = P.n;
  const pr_tuning tn = g_tuning;
  Workspace *wp = nullptr;
  int rc = get_ws((size_t)n, (size_t)P.m, tn.hub_chunk_edges, tn.grid_blocks, &wp);
  if (rc) return rc;
  Workspace &w = *wp;
  const bool weighted = P.w != nullptr;
  const int B = weighted ? grid_blocks(w, tn, k_rank_static<true, 4>)
                         : grid_blocks(w, tn, k_rank_static<false, 4>);
  const int np = B + kHubFinalizeBlocks;
  CallTimer timer(w, s);
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, w.ctrl);
  const bool xs = xsplit_min_degree(tn) > 0;
  if (xs && (rc = xcd_ranges(w, P.group_off, n, s))) return rc;
  XPlan xp;
  rc = partition(w, P.row_off, n, P.m, tn.lane_max_degree, tn.wave_max_degree,
                 tn.hub_chunk_edges, w.hi_in, kInWave, kInChunks, w.hub_start_in,
                 w.chunk_hub_in, s, xs ? P.row_idx : nullptr, &xp);
  if (rc) return rc;
  if ((rc = read_plan(w, xp, s))) return rc;
  const int lg = item_lg(w, xp, B);
  auto rank_w = lg ? k_rank_static<true, 4> : k_rank_static<true, 0>;
  auto rank_u = lg ? k_rank_static<false, 4> : k_rank_static<false, 0>;
  Locality loc;
  if ((rc = locality(w, n, P.m, P.group_off, P.row_idx, tn, P.relabel, s, &loc,
                     xs ? w.xrs : nullptr, &xp, P.row_off,
                     std::max(xsplit_min_degree(tn), tn.lane_max_degree + 1))))
    return rc;
  // R[0] is the caller's output vector; with `init` (which may alias it) the
  // start vector is copied into it.
  double *R[2] = {ranks_out, w.R1};
  double *X[2] = {w.X0, w.X1};
  int *tq = w.counts + kTileQueue;
  hipLaunchKernelGGL(k_static_init, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                     P.deg_off, loc.pos, P.init, P.r0, (int)weighted, R[0], X[0], tq);
  LAUNCH_TRY();
  const double C0 = (1.0 - alpha) / (double)n;
  const int t1 = tn.lane_max_degree, CH = tn.hub_chunk_edges;
  auto launch = [&](int it, bool prof, hipEvent_t after) -> int {
    const int a = it & 1, b = a ^ 1;
    if (weighted)
      hipLaunchKernelGGL(rank_w, dim3(B), dim3(kBlock), 0, s, P.row_off, loc.src,
                         P.w, P.deg_off, loc.pos, (const double *)X[a], (const double *)R[a],
                         R[b], X[b], (const int *)w.hi_in, (const int *)w.counts,
                         (const int *)w.hub_start_in, (const int *)w.chunk_hub_in, w.hub_part, CH,
                         n, t1, xp.items, xp.off, C0, alpha, P.tele, P.tscale, w.partials, tq,
                         (const Ctrl *)w.ctrl);
    else
      hipLaunchKernelGGL(rank_u, dim3(B), dim3(kBlock), 0, s, P.row_off, loc.src,
                         (const double *)nullptr, P.deg_off, loc.pos, (const double *)X[a],
                         (const double *)R[a], R[b], X[b], (const int *)w.hi_in,
                         (const int *)w.counts, (const int *)w.hub_start_in,
                         (const int *)w.chunk_hub_in, w.hub_part, CH, n, t1, xp.items, xp.off,
                         C0, alpha, P.tele, P.tscale, w.partials, tq, (const Ctrl *)w.ctrl);
    if (prof) HIP_TRY(hipEventRecord(after, s));
    hipLaunchKernelGGL(k_hub_finalize_static, dim3(kHubFinalizeBlocks), dim3(kBlock), 0, s,
                       (const int *)w.hi_in, (const int *)w.counts, (const int *)w.hub_start_in,
                       (const double *)w.hub_part, P.deg_off, loc.pos, (const double *)R[a], R[b],
                       X[b], C0, alpha, P.tele, P.tscale, (int)weighted, w.partials + B, tq,
                       (const Ctrl *)w.ctrl);
    hipLaunchKernelGGL(k_linf_final, dim3(1), dim3(kFinalBlock), 0, s,
                       (const double *)w.partials, np, w.ctrl, tol, it);
    LAUNCH_TRY();
    return PR_OK;
  };
  int iters = 0, launched = 0;
  rc = iterate(w, s, max_iter, launch, &iters, &launched);
  if (rc) return rc;
  double *result = R[iters & 1];
  if (result != ranks_out)
    HIP_TRY(hipMemcpyAsync(ranks_out, result, (size_t)n * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  timer.stop();
  HIP_TRY(hipStreamSynchronize(s));
  t_stats.total_ms = timer.ms();
  collect_profile(w, iters);
  return t_stats.converged ? PR_OK : PR_NOT_CONVERGED;
}

// Static iteration (Alg. 1), from 1/n or from `init` (Naive-dynamic).
int run_static(const pr_csr *g, double alpha, double tol, int max_iter, const double *init,
               double *ranks_out) {
  PullProblem P{};
  P.n = g->n;
  P.m = g->m;
  P.row_off = g->in_offsets;
  P.row_idx = g->in_sources;
  P.deg_off = g->out_offsets;
  P.group_off = g->out_offsets;
  P.init = init;
  P.r0 = 1.0 / (double)g->n;
  P.relabel = true;
  return run_pull(P, alpha, tol, max_iter, ranks_out);
}

int run_dynamic_frontier(const pr_csr *g, const pr_edges *del, const pr_edges *ins,
                         const double *prev, double alpha, double tol, double tau_f,
                         double tau_p, int max_iter, int mode, double *ranks_out) {
  hipStream_t s = t_stream;
  const bool prune = mode == PR_MODE_DFP, dt = mode == PR_MODE_DT;
  const int n = g->n;
  const pr_tuning tn = g_tuning;
  Workspace *wp = nullptr;
  int rc = get_ws((size_t)n, (size_t)g->m, tn.hub_chunk_edges, tn.grid_blocks, &wp);
  if (rc) return rc;
  Workspace &w = *wp;
  const int B = prune ? grid_blocks(w, tn, k_rank_dfp<true, 4, true>)
                      : grid_blocks(w, tn, k_rank_dfp<false, 4, true>);
  // affected lists (one per iteration parity) and their sizes
  const bool use_list = tn.frontier_list != 0;
  int *alist[2] = {w.alist, w.alist + (size_t)n};
  // per parity: {list size, tile queue of the rank update}
  int *acnt[2] = {w.counts + kAffList, w.counts + kAffList + 2};
  // the frontier's wavefront-class vertices and their count per parity
  int *cand = w.alist + 2 * (size_t)n, *ccnt = w.counts + kCands;
  const int np = B + kHubFinalizeBlocks;
  CallTimer timer(w, s);
  const size_t fs = flag_stride((size_t)n);  // each flag array 256-byte aligned
  uint8_t *dV = w.flags, *dN = w.flags + fs, *cv = w.flags + 2 * fs;
  double *R = ranks_out;
  const int t1 = tn.lane_max_degree, t_exp = tn.expand_lane_max_degree, CH = tn.hub_chunk_edges;
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, w.ctrl);
  if (use_list) HIP_TRY(hipMemsetAsync(ccnt, 0, 2 * sizeof(int), s));
  const bool xs = xsplit_min_degree(tn) > 0;
  if (xs && (rc = xcd_ranges(w, g->out_offsets, n, s))) return rc;
  if (xs) {
    // marks land in proportion to in-degree: target ranges balanced by it
    hipLaunchKernelGGL(k_xcd_ranges, dim3(1), dim3(64), 0, s, g->in_offsets,
                       (const int *)nullptr, n, w.xrt);
    LAUNCH_TRY();
  }
  XPlan xp;
  rc = partition(w, g->in_offsets, n, g->m, t1, tn.wave_max_degree, CH, w.hi_in, kInWave,
                 kInChunks, w.hub_start_in, w.chunk_hub_in, s, xs ? g->in_sources : nullptr,
                 &xp);
  if (rc) return rc;
  if ((rc = read_plan(w, xp, s))) return rc;
  const int lg = item_lg(w, xp, B);
  auto rank_p = lg ? (use_list ? k_rank_dfp<true, 4, true> : k_rank_dfp<true, 4, false>)
                   : (use_list ? k_rank_dfp<true, 0, true> : k_rank_dfp<true, 0, false>);
  auto rank_d = lg ? (use_list ? k_rank_dfp<false, 4, true> : k_rank_dfp<false, 4, false>)
                   : (use_list ? k_rank_dfp<false, 0, true> : k_rank_dfp<false, 0, false>);
  Locality loc;
  // the frontier list's storage serves the mapping as scratch (n ints)
  if ((rc = locality_chain(w, n, g->m, g->out_offsets, g->in_sources, tn, s, &loc,
                           xs ? w.xrs : nullptr, xp, g->in_offsets,
                           std::max(xsplit_min_degree(tn), t1 + 1), cand)))
    return rc;
  double *X = w.X0;
  hipLaunchKernelGGL(k_dfp_init, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                     g->out_offsets, loc.pos, prev, R, X, dV, dN, cv, acnt[0]);
  LAUNCH_TRY();
  rc = partition(w, g->out_offsets, n, g->m, t_exp, tn.wave_max_degree, CH, w.hi_out, kOutWave,
                 kOutChunks, w.hub_start_out, w.chunk_hub_out, s);
  if (rc) return rc;
  const int nd = del ? del->count : 0, ni = ins ? ins->count : 0;
  if (nd + ni > 0) {
    hipLaunchKernelGGL(k_mark_initial, dim3((nd + ni + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       del ? del->src : nullptr, del ? del->dst : nullptr, nd,
                       ins ? ins->src : nullptr, ni, n, dV, dN, g->out_offsets, t_exp,
                       tn.wave_max_degree, use_list ? cand : nullptr, ccnt + 1, w.ctrl);
    LAUNCH_TRY();
  }
  // frontier size above which expandAffected pulls (-1: always push)
  const long long pull_thresh =
      tn.expand_pull_per_mille > 0 ? (long long)n * tn.expand_pull_per_mille / 1000 : -1;
  const int fgrid = std::max(1, std::min((n / 32 + kBlock) / kBlock, 4 * std::max(1, w.num_cus)));
  // compaction of the affected set after the marking of iteration it, for
  // iteration it + 1 (list by parity of it + 1)
  const int cgrid_list =
      std::max(1, std::min((n + kCompactRun - 1) / kCompactRun, 2 * std::max(1, w.num_cus)));
  auto compact = [&](int it) {
    const int q = (it + 1) & 1;
    hipLaunchKernelGGL(k_compact_affected, dim3(cgrid_list), dim3(kBlock), 0, s,
                       (const uint8_t *)dV, dN, n, alist[q], acnt[q], acnt[q] + 1,
                       (const Ctrl *)w.ctrl);
  };
  auto apply_expand = [&](int it, bool mark) {
    // the initial expansion (it = -1) marks from the batch sources, which
    // are in no list: it sweeps ID tiles
    const bool lst = use_list && it >= 0;
    if (mark && pull_thresh >= 0) {
      // with a short list, the frontier is counted over it, and the bitmap
      // is only built when the marking pulls
      if (lst)
        hipLaunchKernelGGL(k_frontier_count, dim3(cgrid_list), dim3(kBlock), 0, s,
                           (const int *)alist[it & 1], (const int *)acnt[it & 1],
                           (const uint8_t *)dN, n, w.ctrl, it);
      hipLaunchKernelGGL(k_frontier, dim3(fgrid), dim3(kBlock), 0, s, (const uint8_t *)dN, n,
                         w.fbits, w.ctrl, it, lst ? pull_thresh : -1LL,
                         lst ? (const int *)acnt[it & 1] : nullptr);
      hipLaunchKernelGGL(k_pull_mark, dim3(B), dim3(kBlock), 0, s, g->in_offsets,
                         g->in_sources, (const int *)w.hi_in, (const int *)w.counts,
                         (const int *)w.hub_start_in, (const int *)w.chunk_hub_in, CH, xp.items,
                         xp.off, (const uint32_t *)w.fbits, dV, n, t1, pull_thresh,
                         (uint8_t *)nullptr, (int *)nullptr, (const Ctrl *)w.ctrl, it);
    }
    // with the list, the frontier's wavefront-class vertices are listed
    // first (for the initial expansion by k_mark_initial, in parity 1), so
    // the marking does not check the whole class
    const bool cands = use_list && mark;
    if (lst && mark)
      hipLaunchKernelGGL(k_expand_cands, dim3(cgrid_list), dim3(kBlock), 0, s,
                         (const int *)alist[it & 1], (const int *)acnt[it & 1],
                         (const uint8_t *)dN, g->out_offsets, t_exp, tn.wave_max_degree,
                         pull_thresh, cand, ccnt + (it & 1), ccnt + ((it + 1) & 1),
                         (const Ctrl *)w.ctrl, it);
    hipLaunchKernelGGL(k_apply_expand, dim3(B), dim3(kBlock), 0, s, g->out_offsets,
                       g->out_targets, loc.pos, R, X, (const double *)w.T, dV,
                       (const uint8_t *)dN, cv,
                       (const int *)w.hi_out, (const int *)w.counts,
                       (const int *)w.hub_start_out, (const int *)w.chunk_hub_out, CH, n, t_exp,
                       xs ? (const int *)w.xrt : nullptr, pull_thresh, mark ? 1 : 0,
                       lst ? (const int *)alist[it & 1] : nullptr,
                       lst ? (const int *)acnt[it & 1] : nullptr,
                       cands ? (const int *)cand : nullptr,
                       cands ? (const int *)ccnt + (it & 1) : nullptr, (const Ctrl *)w.ctrl, it);
    if (use_list) compact(it);
  };
  // initial expandAffected (Alg. 2, after initialAffected)
  apply_expand(-1, true);
  LAUNCH_TRY();
  if (dt) {
    // Dynamic Traversal (Alg. 7): close the affected set under out-edges,
    // one level per pass (the vertices with an in-neighbour in the previous
    // level's marks), until a pass marks nothing
    HIP_TRY(hipMemcpyAsync(dN, dV, (size_t)n, hipMemcpyDeviceToDevice, s));
    int *changed = w.counts + kDtChanged;
    for (int level = 0;; ++level) {
      hipLaunchKernelGGL(k_frontier, dim3(fgrid), dim3(kBlock), 0, s, (const uint8_t *)dN, n,
                         w.fbits, w.ctrl, level, -1LL, (const int *)nullptr);
      HIP_TRY(hipMemsetAsync(cv, 0, (size_t)n, s));
      HIP_TRY(hipMemsetAsync(changed, 0, sizeof(int), s));
      hipLaunchKernelGGL(k_pull_mark, dim3(B), dim3(kBlock), 0, s, g->in_offsets,
                         g->in_sources, (const int *)w.hi_in, (const int *)w.counts,
                         (const int *)w.hub_start_in, (const int *)w.chunk_hub_in, CH, xp.items,
                         xp.off, (const uint32_t *)w.fbits, dV, n, t1, -1LL, cv, changed,
                         (const Ctrl *)w.ctrl, level);
      LAUNCH_TRY();
      HIP_TRY(hipMemcpyAsync(w.host_counts, changed, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (!w.host_counts[0]) break;
      HIP_TRY(hipMemcpyAsync(dN, cv, (size_t)n, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipMemsetAsync(cv, 0, (size_t)n, s));
    HIP_TRY(hipMemsetAsync(dN, 0, (size_t)n, s));
    if (use_list) {  // the list of the closed set
      HIP_TRY(hipMemsetAsync(acnt[0], 0, sizeof(int), s));
      compact(-1);
    }
  }
  // profiling: the affected set each iteration is about to update (counted
  // after the marking that produced it, outside the rank-kernel timing)
  const int cgrid = std::min(1024, (n + kBlock - 1) / kBlock);
  auto count_affected = [&]() {
    hipLaunchKernelGGL(k_count_affected, dim3(cgrid), dim3(kBlock), 0, s, (const uint8_t *)dV,
                       g->in_offsets, n, w.ctrl);
    hipLaunchKernelGGL(k_affected_fold, dim3(1), dim3(64), 0, s, w.ctrl);
  };
  const bool counters = t_profiling >= 2;
  if (counters) {
    hipLaunchKernelGGL(k_count_flags, dim3(cgrid), dim3(kBlock), 0, s, (const uint8_t *)dV, n,
                       w.ctrl, 0);
    count_affected();
    LAUNCH_TRY();
  }
  const double C0 = (1.0 - alpha) / (double)n;
  auto launch = [&](int it, bool prof, hipEvent_t after) -> int {
    if (prune) {
      hipLaunchKernelGGL(rank_p, dim3(B), dim3(kBlock), 0, s, g->in_offsets,
                         loc.src, g->out_offsets, (const double *)X, (const double *)R, w.T, dV,
                         dN, cv,
                         (const int *)w.hi_in, (const int *)w.counts,
                         (const int *)w.hub_start_in, (const int *)w.chunk_hub_in, w.hub_part, CH,
                         n, t1, xp.items, xp.off, C0, alpha, tau_f, tau_p, w.partials,
                         (const int *)alist[it & 1], acnt[it & 1], acnt[(it + 1) & 1],
                         (const Ctrl *)w.ctrl);
      if (prof) HIP_TRY(hipEventRecord(after, s));
      hipLaunchKernelGGL(k_hub_finalize_dfp<true>, dim3(kHubFinalizeBlocks), dim3(kBlock), 0, s,
                         (const int *)w.hi_in, (const int *)w.counts, (const int *)w.hub_start_in,
                         (const double *)w.hub_part, g->out_offsets, (const double *)R, w.T, dV,
                         dN, cv, C0, alpha, tau_f, tau_p, w.partials + B, (const Ctrl *)w.ctrl);
    } else {
      hipLaunchKernelGGL(rank_d, dim3(B), dim3(kBlock), 0, s, g->in_offsets,
                         loc.src, g->out_offsets, (const double *)X, (const double *)R, w.T, dV,
                         dN, cv,
                         (const int *)w.hi_in, (const int *)w.counts,
                         (const int *)w.hub_start_in, (const int *)w.chunk_hub_in, w.hub_part, CH,
                         n, t1, xp.items, xp.off, C0, alpha, tau_f, tau_p, w.partials,
                         (const int *)alist[it & 1], acnt[it & 1], acnt[(it + 1) & 1],
                         (const Ctrl *)w.ctrl);
      if (prof) HIP_TRY(hipEventRecord(after, s));
      hipLaunchKernelGGL(k_hub_finalize_dfp<false>, dim3(kHubFinalizeBlocks), dim3(kBlock), 0, s,
                         (const int *)w.hi_in, (const int *)w.counts, (const int *)w.hub_start_in,
                         (const double *)w.hub_part, g->out_offsets, (const double *)R, w.T, dV,
                         dN, cv, C0, alpha, tau_f, tau_p, w.partials + B, (const Ctrl *)w.ctrl);
    }
    hipLaunchKernelGGL(k_linf_final, dim3(1), dim3(kFinalBlock), 0, s,
                       (const double *)w.partials, np, w.ctrl, tol, it);
    apply_expand(it, !dt);  // DT: the affected set stays fixed
    if (counters) count_affected();
    LAUNCH_TRY();
    return PR_OK;
  };
  int iters = 0, launched = 0;
  rc = iterate(w, s, max_iter, launch, &iters, &launched);
  if (rc) return rc;
  timer.stop();
  HIP_TRY(hipStreamSynchronize(s));
  if (w.nc_cur >= 0 && loc.pos == w.nc_newid) w.nc_miss += w.host_counts[kMapMiss];
  const Ctrl &last = w.host_ctrl[(launched - 1) % kRing];
  if (last.err) return fail(PR_EBATCH, "batch vertex ID outside [0, n)");
  if (counters) {
    t_stats.affected_initial = last.aux[0];
    t_stats.affected_max = last.aux[5];
    t_stats.edges_processed = last.aux[6];
  }
  t_stats.total_ms = timer.ms();
  collect_profile(w, iters);
  return t_stats.converged ? PR_OK : PR_NOT_CONVERGED;
}

// In-edges per wavefront before a PPR row is split (tuning ppr_chunk_edges):
// rows up to C are summed whole, longer ones in chunks of C, and with the die
// split on every row longer than C is a die-split row.
int ppr_chunk(const pr_tuning &tn) { return tn.ppr_chunk_edges > 0 ? tn.ppr_chunk_edges : 256; }

int ppr_ws(Workspace &w, size_t n, size_t m, size_t K, size_t B, int C) {
  const size_t nbuf = 4 * n * K;
  const size_t npart = std::max(m / C + n + 1, xsplit_items_bound(n, m, C, C + 1)) * K;
  // partial maxima of the rank and finalize workgroups, then the chunk maxima
  const size_t npmax = (B + kHubFinalizeBlocks + 16 + kPprColBlocks) * K;
  if (nbuf > w.cap_ppr_buf || npart > w.cap_ppr_part || npmax > w.cap_ppr_pmax ||
      K > w.cap_ppr_k || n > w.cap_ppr_n) {
    const size_t a = std::max(nbuf, w.cap_ppr_buf), b = std::max(npart, w.cap_ppr_part);
    const size_t c = std::max(npmax, w.cap_ppr_pmax), kk = std::max(K, w.cap_ppr_k);
    const size_t nn = std::max(n, w.cap_ppr_n);
    free_ppr(w);
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&w.ppr_buf, a * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.ppr_part, b * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.ppr_pmax, c * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.ppr_vdelta, kk * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.ppr_vdone, kk * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.ppr_viters, kk * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.ppr_split, 2 * nn)) != hipSuccess) {  // split flags, teleport flags
      (void)hipGetLastError();
      free_ppr(w);
      return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP,
                  std::string("PPR workspace allocation: ") + hipGetErrorString(e));
    }
    w.cap_ppr_buf = a;
    w.cap_ppr_part = b;
    w.cap_ppr_pmax = c;
    w.cap_ppr_k = kk;
    w.cap_ppr_n = nn;
  }
  return PR_OK;
}

int run_ppr(const pr_csr *g, const double *teleport, int K, double alpha, double tol,
            int max_iter, double *ranks_out, int32_t *iters_out) {
  hipStream_t s = t_stream;
  const int n = g->n;
  const pr_tuning tn = g_tuning;
  Workspace *wp = nullptr;
  const int C = ppr_chunk(tn);
  int rc = get_ws((size_t)n, (size_t)g->m, C, tn.grid_blocks, &wp);
  if (rc) return rc;
  Workspace &w = *wp;
  const int B = grid_blocks(w, tn, k_ppr_rank);
  const int F = kHubFinalizeBlocks;
  if ((rc = ppr_ws(w, (size_t)n, (size_t)g->m, (size_t)K, (size_t)B, C))) return rc;
  CallTimer timer(w, s);
  const size_t nk = (size_t)n * K;
  double *Rb[2] = {w.ppr_buf, w.ppr_buf + nk};
  double *Xb[2] = {w.ppr_buf + 2 * nk, w.ppr_buf + 3 * nk};
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, w.ctrl);
  // rows longer than C form the split class (class 1 of Alg. 4 empty), cut
  // by source range as well when the die split is on: its threshold is C + 1
  // here, whatever the tuning's, so that every split row is in the plan
  const bool xs = xsplit_min_degree(tn) > 0;
  if (xs && (rc = xcd_ranges(w, g->out_offsets, n, s))) return rc;
  XPlan xp;
  rc = partition(w, g->in_offsets, n, g->m, C, C, C, w.hi_in, kInWave, kInChunks,
                 w.hub_start_in, w.chunk_hub_in, s, xs ? g->in_sources : nullptr, &xp, nullptr,
                 nullptr, C + 1);
  if (rc) return rc;
  Locality loc;
  if ((rc = locality(w, n, g->m, g->out_offsets, g->in_sources, tn, true, s, &loc,
                     xs ? w.xrs : nullptr)))
    return rc;
  const int ib = (int)std::min<size_t>((nk + kBlock - 1) / kBlock, (size_t)B * 4);
  int *rq = w.counts + kTileQueue;  // the rank kernel's 8 per-die row queues
  hipLaunchKernelGGL(k_ppr_init, dim3(ib), dim3(kBlock), 0, s, n, K, g->out_offsets, loc.pos,
                     Rb[0], Xb[0], w.ppr_vdone, w.ppr_viters, rq);
  hipLaunchKernelGGL(k_split_flags, dim3(std::min(B, (n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, g->in_offsets, n, C, w.ppr_split);
  uint8_t *tnz = w.ppr_split + w.cap_ppr_n;
  hipLaunchKernelGGL(k_tele_flags, dim3(std::min((n + kWavesPerBlock - 1) / kWavesPerBlock, 65536)),
                     dim3(kBlock), 0, s, teleport, n, K, tnz);
  LAUNCH_TRY();
  const size_t shm = (size_t)kWavesPerBlock * K * sizeof(double);
  auto launch = [&](int it, bool prof, hipEvent_t after) -> int {
    const int a = it & 1, b = a ^ 1;
    hipLaunchKernelGGL(k_ppr_rank, dim3(B), dim3(kBlock), shm, s, g->in_offsets, loc.src,
                       g->out_offsets, loc.pos, (const int *)w.hi_in, (const int *)w.counts,
                       (const int *)w.hub_start_in, (const int *)w.chunk_hub_in,
                       (const uint8_t *)w.ppr_split, C, n, K, (const double *)Xb[a],
                       (const double *)Rb[a], Rb[b], Xb[b], teleport, (const uint8_t *)tnz,
                       w.ppr_part, (const int *)w.ppr_vdone, alpha, w.ppr_pmax, xp.items, xp.off,
                       rq, (const Ctrl *)w.ctrl);
    if (prof) HIP_TRY(hipEventRecord(after, s));
    hipLaunchKernelGGL(k_ppr_finalize, dim3(F), dim3(kBlock), shm, s, g->out_offsets, loc.pos,
                       (const int *)w.hi_in, (const int *)w.counts, (const int *)w.hub_start_in,
                       K, (const double *)w.ppr_part, (const double *)Rb[a], Rb[b], Xb[b],
                       teleport, (const uint8_t *)tnz, (const int *)w.ppr_vdone, alpha,
                       w.ppr_pmax + (size_t)B * K, rq, (const Ctrl *)w.ctrl);
    double *cmax = w.ppr_pmax + (size_t)(B + F + 16) * K;
    hipLaunchKernelGGL(k_ppr_colmax, dim3(kPprColBlocks), dim3(kBlock), 0, s,
                       (const double *)w.ppr_pmax, B + F, K, cmax, (const Ctrl *)w.ctrl);
    hipLaunchKernelGGL(k_ppr_linf, dim3(1), dim3(kBlock), 0, s, (const double *)cmax,
                       kPprColBlocks, K, w.ppr_vdone, w.ppr_viters, w.ppr_vdelta, w.ctrl, tol,
                       it);
    LAUNCH_TRY();
    return PR_OK;
  };
  int iters = 0, launched = 0;
  rc = iterate(w, s, max_iter, launch, &iters, &launched);
  if (rc) return rc;
  hipLaunchKernelGGL(k_ppr_gather_out, dim3(ib), dim3(kBlock), 0, s, n, K,
                     (const double *)Rb[0], (const double *)Rb[1], (const int *)w.ppr_viters,
                     ranks_out);
  LAUNCH_TRY();
  if (iters_out)
    HIP_TRY(hipMemcpyAsync(iters_out, w.ppr_viters, (size_t)K * sizeof(int),
                           hipMemcpyDeviceToHost, s));
  timer.stop();
  HIP_TRY(hipStreamSynchronize(s));
  t_stats.total_ms = timer.ms();
  collect_profile(w, iters);
  return t_stats.converged ? PR_OK : PR_NOT_CONVERGED;
}

// Weighted forward: r = alpha * A r + (1 - alpha) s with A[v][u] = w(u -> v).
int run_weighted(const pr_csr *g, const double *in_w, const double *tele, double alpha,
                 double tol, int max_iter, double *ranks_out) {
  PullProblem P{};
  P.n = g->n;
  P.m = g->m;
  P.row_off = g->in_offsets;
  P.row_idx = g->in_sources;
  P.deg_off = g->out_offsets;
  P.group_off = g->out_offsets;
  P.w = in_w;
  P.tele = tele;
  P.tscale = 1.0 - alpha;
  P.r0 = 1.0 / (double)g->n;
  P.relabel = true;
  return run_pull(P, alpha, tol, max_iter, ranks_out);
}

// Adjoint of the weighted forward: lambda = g + alpha * A^T lambda, pulled
// over the out-CSR with the weights transposed into out-CSR order, from
// lambda = 0; then the edge and teleport gradients.
int run_adjoint(const pr_csr *g, const double *in_w, const double *r, const double *grad_r,
                double alpha, double tol, int max_iter, double *grad_w, double *grad_s,
                double *lambda_out, double *lambda_tmp_owner) {
  hipStream_t s = t_stream;
  const int n = g->n, m = g->m;
  Workspace *wp = nullptr;
  const pr_tuning tn = g_tuning;
  int rc = get_ws((size_t)n, (size_t)m, tn.hub_chunk_edges, tn.grid_blocks, &wp);
  if (rc) return rc;
  Workspace &w = *wp;
  if ((size_t)m > w.cap_w_out) {
    (void)hipFree(w.w_out);
    w.w_out = nullptr;
    w.cap_w_out = 0;
    hipError_t e = hipMalloc(&w.w_out, (size_t)m * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP,
                  std::string("adjoint workspace: ") + hipGetErrorString(e));
    }
    w.cap_w_out = (size_t)m;
  }
  const int gb = std::min((m + kBlock - 1) / kBlock, 8 * std::max(1, w.num_cus) * 4);
  hipLaunchKernelGGL(k_fill, dim3(gb), dim3(kBlock), 0, s, w.w_out, (size_t)m, 0.0);
  hipLaunchKernelGGL(k_transpose_weights, dim3(gb), dim3(kBlock), 0, s, g->in_offsets,
                     g->in_sources, in_w, g->out_offsets, g->out_targets, n, m, w.w_out);
  LAUNCH_TRY();
  PullProblem P{};
  P.n = n;
  P.m = m;
  P.row_off = g->out_offsets;
  P.row_idx = g->out_targets;
  P.deg_off = g->out_offsets;
  P.group_off = g->in_offsets;
  P.w = w.w_out;
  P.tele = grad_r;
  P.tscale = 1.0;
  P.r0 = 0.0;
  P.relabel = true;
  double *lam = lambda_out ? lambda_out : lambda_tmp_owner;
  rc = run_pull(P, alpha, tol, max_iter, lam);
  if (rc < 0) return rc;
  const pr_stats keep = t_stats;
  hipLaunchKernelGGL(k_adjoint_grads, dim3(gb), dim3(kBlock), 0, s, g->in_offsets, g->in_sources,
                     n, m, r, (const double *)lam, alpha, grad_w, grad_s);
  LAUNCH_TRY();
  HIP_TRY(hipStreamSynchronize(s));
  t_stats = keep;
  return rc;
}

constexpr int kMaxBatchGraphs = 4096;  // per-graph maxima live in LDS (8 bytes each)

int batch_ws(Workspace &w, size_t N, size_t M, size_t G, size_t part_rows) {
  const size_t npart = part_rows * G;
  if (N > w.cap_u_n || M > w.cap_u_m || G > w.cap_b_g || npart > w.cap_b_part) {
    const size_t nn = std::max(N, w.cap_u_n), mm = std::max(M, w.cap_u_m);
    const size_t gg = std::max(G, w.cap_b_g), pp = std::max(npart, w.cap_b_part);
    free_batch(w);
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&w.u_in_off, (nn + 1) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.u_out_off, (nn + 1) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.u_in_src, mm * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.u_gid, nn * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.b_vbase, (gg + 1) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.b_ebase, (gg + 1) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.b_gdone, gg * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.b_giters, gg * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&w.b_c0, gg * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.b_gdelta, gg * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.b_gpart, pp * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.b_desc, gg * sizeof(BatchDesc))) != hipSuccess ||
        (e = hipMalloc(&w.b_outs, gg * sizeof(double *))) != hipSuccess ||
        (e = hipMalloc(&w.b_tele, gg * sizeof(double *))) != hipSuccess ||
        (e = hipMalloc(&w.b_xrs, gg * (kXcds + 1) * sizeof(int))) != hipSuccess) {
      (void)hipGetLastError();
      free_batch(w);
      return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP,
                  std::string("batch workspace allocation: ") + hipGetErrorString(e));
    }
    w.cap_u_n = nn;
    w.cap_u_m = mm;
    w.cap_b_g = gg;
    w.cap_b_part = pp;
  }
  if (!w.cap_stream) {
    HIP_TRY(hipStreamCreateWithFlags(&w.cap_stream, hipStreamNonBlocking));
    for (auto &e : w.cap_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  return PR_OK;
}

// Iterations captured in the hipGraph of a batched call (even: the buffers
// swap back at its end). Iterations enqueued after every graph converged exit
// at once on the device, so a replay wastes at most a few microseconds each.
constexpr int kReplayIters = 4;

// Static PageRank (Alg. 1) on G graphs at once: union CSR, one partition and
// renumbering, per-graph teleport (uniform or a personalised vector) and
// convergence; the iterations run as replays of one captured hipGraph of
// kReplayIters iterations, whose instantiation is kept and updated in place
// by the next call.
int run_batched(const pr_csr *graphs, int G, const double *const *tele, double alpha, double tol,
                int max_iter, double *const *outs, int32_t *iters_out) {
  hipStream_t s = t_stream;
  const pr_tuning tn = g_tuning;
  std::vector<int> vbase(G + 1), ebase(G + 1);
  std::vector<BatchDesc> desc(G);
  std::vector<double> c0(G);
  long long N = 0, M = 0;
  for (int g = 0; g < G; ++g) {
    vbase[g] = (int)N;
    ebase[g] = (int)M;
    desc[g] = BatchDesc{graphs[g].in_offsets, graphs[g].in_sources, graphs[g].out_offsets,
                        (int)N, (int)M, graphs[g].n, graphs[g].m};
    c0[g] = (1.0 - alpha) / (double)graphs[g].n;
    N += graphs[g].n;
    M += graphs[g].m;
    if (N > INT_MAX - 1 || M > INT_MAX - 1)
      return fail(PR_EINVAL, "batch too large for int32 vertex/edge indices");
  }
  vbase[G] = (int)N;
  ebase[G] = (int)M;
  const int n = (int)N, m = (int)M;
  Workspace *wp = nullptr;
  int rc = get_ws((size_t)n, (size_t)m, tn.hub_chunk_edges, tn.grid_blocks, &wp);
  if (rc) return rc;
  Workspace &w = *wp;
  const int B = grid_blocks(w, tn, k_rank_batched<4>);
  const int F = kHubFinalizeBlocks;
  if ((rc = batch_ws(w, (size_t)n, (size_t)m, (size_t)G, (size_t)(B + F)))) return rc;
  CallTimer timer(w, s);
  HIP_TRY(hipMemcpyAsync(w.b_desc, desc.data(), G * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(w.b_vbase, vbase.data(), (G + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(w.b_ebase, ebase.data(), (G + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(w.b_c0, c0.data(), G * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(w.b_outs, outs, G * sizeof(double *), hipMemcpyHostToDevice, s));
  bool any_tele = false;
  for (int g = 0; tele && g < G; ++g) any_tele = any_tele || tele[g] != nullptr;
  if (any_tele)
    HIP_TRY(hipMemcpyAsync(w.b_tele, tele, G * sizeof(double *), hipMemcpyHostToDevice, s));
  const double *const *dtele = any_tele ? (const double *const *)w.b_tele : nullptr;
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, w.ctrl);
  const int ub = std::min((std::max(n, m) + kBlock - 1) / kBlock, 32 * std::max(1, w.num_cus));
  hipLaunchKernelGGL(k_union_build, dim3(ub), dim3(kBlock), 0, s, (const BatchDesc *)w.b_desc,
                     (const int *)w.b_vbase, (const int *)w.b_ebase, G, n, m, w.u_in_off,
                     w.u_in_src, w.u_out_off, w.u_gid);
  LAUNCH_TRY();
  // die-split ranges per graph (each graph is cut as when run alone, so the
  // summation order and the result match pr_static on it bit for bit)
  const bool xs = xsplit_min_degree(tn) > 0;
  if (xs) {
    hipLaunchKernelGGL(k_xcd_ranges, dim3(G), dim3(64), 0, s, (const int *)w.u_out_off,
                       (const int *)w.b_vbase, n, w.b_xrs);
    LAUNCH_TRY();
  }
  XPlan xp;
  rc = partition(w, w.u_in_off, n, m, tn.lane_max_degree, tn.wave_max_degree,
                 tn.hub_chunk_edges, w.hi_in, kInWave, kInChunks, w.hub_start_in,
                 w.chunk_hub_in, s, xs ? w.u_in_src : nullptr, &xp, w.b_xrs,
                 (const int *)w.u_gid);
  if (rc) return rc;
  Locality loc;
  if ((rc = locality(w, n, m, w.u_out_off, w.u_in_src, tn, true, s, &loc))) return rc;
  if ((rc = read_plan(w, xp, s))) return rc;
  const int lg = item_lg(w, xp, B);
  auto rank_fn = lg ? k_rank_batched<4> : k_rank_batched<0>;
  double *R[2] = {w.T, w.R1};
  double *X[2] = {w.X0, w.X1};
  hipLaunchKernelGGL(k_batched_init, dim3(ub), dim3(kBlock), 0, s, n, G, (const int *)w.u_gid,
                     (const int *)w.b_vbase, (const int *)w.u_out_off, loc.pos, R[0], X[0],
                     w.b_gdone, w.b_giters, w.counts + kTileQueue);
  LAUNCH_TRY();
  // kReplayIters iterations captured on the library stream, after the work above
  hipStream_t cs = w.cap_stream;
  HIP_TRY(hipEventRecord(w.cap_ev[0], s));
  HIP_TRY(hipStreamWaitEvent(cs, w.cap_ev[0], 0));
  const size_t shm = (size_t)G * sizeof(unsigned long long);
  const int t1 = tn.lane_max_degree, CH = tn.hub_chunk_edges;
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  for (int it = 0; it < kReplayIters; ++it) {
    const int a = it & 1, b = a ^ 1;
    hipLaunchKernelGGL(rank_fn, dim3(B), dim3(kBlock), shm, cs, (const int *)w.u_in_off,
                       loc.src, (const int *)w.u_out_off, loc.pos, (const double *)X[a],
                       (const double *)R[a], R[b], X[b], (const int *)w.hi_in,
                       (const int *)w.counts, (const int *)w.hub_start_in,
                       (const int *)w.chunk_hub_in, w.hub_part, CH, n, t1, xp.items, xp.off,
                       (const int *)w.u_gid, (const double *)w.b_c0, dtele,
                       (const int *)w.b_vbase, (const int *)w.b_gdone, G, alpha, w.b_gpart,
                       w.counts + kTileQueue, (const Ctrl *)w.ctrl);
    hipLaunchKernelGGL(k_hub_finalize_batched, dim3(F), dim3(kBlock), shm, cs,
                       (const int *)w.hi_in, (const int *)w.counts, (const int *)w.hub_start_in,
                       (const double *)w.hub_part, (const int *)w.u_out_off, loc.pos,
                       (const double *)R[a], R[b], X[b], (const int *)w.u_gid,
                       (const double *)w.b_c0, dtele, (const int *)w.b_vbase,
                       (const int *)w.b_gdone, G, alpha, w.b_gpart + (size_t)B * G,
                       w.counts + kTileQueue, (const Ctrl *)w.ctrl);
    hipLaunchKernelGGL(k_batched_final, dim3(G), dim3(kBlock), 0, cs, (const double *)w.b_gpart,
                       B + F, G, w.b_gdone, w.b_giters, w.b_gdelta, (const Ctrl *)w.ctrl, tol);
    hipLaunchKernelGGL(k_batched_done, dim3(1), dim3(kBlock), 0, cs, (const int *)w.b_gdone, G,
                       w.ctrl, max_iter);
  }
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(cs, &graph);
  if (ce != hipSuccess) return fail(PR_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
  // the previous call's instantiation takes this call's kernel arguments in
  // place when every launch has the same shape (grids, LDS size and kernels
  // depend only on the key); otherwise it is rebuilt
  const long long key[4] = {G, B, lg, tn.lane_max_degree};
  if (w.b_exec && !std::equal(key, key + 4, w.b_exec_key)) {
    (void)hipGraphExecDestroy(w.b_exec);
    w.b_exec = nullptr;
  }
  if (w.b_exec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(w.b_exec, graph, &bad, &res) != hipSuccess ||
        res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(w.b_exec);
      w.b_exec = nullptr;
    }
  }
  if (!w.b_exec) {
    ce = hipGraphInstantiate(&w.b_exec, graph, nullptr, nullptr, 0);
    if (ce != hipSuccess) {
      (void)hipGraphDestroy(graph);
      w.b_exec = nullptr;
      return fail(PR_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ce));
    }
    std::copy(key, key + 4, w.b_exec_key);
  }
  (void)hipGraphDestroy(graph);
  hipGraphExec_t exec = w.b_exec;
  const int K = std::max(1, std::min(g_tuning.iters_per_sync, kRing - 1));
  const int replays = (max_iter + kReplayIters - 1) / kReplayIters;
  int r = 0;
  bool done = false;
  int err = PR_OK;
  while (r < replays && !done) {
    hipError_t e1 = hipGraphLaunch(exec, cs);
    hipError_t e2 = hipMemcpyAsync(&w.host_ctrl[r % kRing], w.ctrl, sizeof(Ctrl),
                                   hipMemcpyDeviceToHost, cs);
    hipError_t e3 = hipEventRecord(w.sync_ev[r % kRing], cs);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      err = fail(PR_EHIP, "graph replay failed");
      break;
    }
    ++r;
    const int j = r - K;
    if (j >= 0) {
      if (hipEventSynchronize(w.sync_ev[j % kRing]) != hipSuccess) {
        err = fail(PR_EHIP, "hipEventSynchronize failed");
        break;
      }
      if (w.host_ctrl[j % kRing].done) done = true;
    }
  }
  (void)hipStreamSynchronize(cs);
  if (err) return err;
  HIP_TRY(hipEventRecord(w.cap_ev[1], cs));
  HIP_TRY(hipStreamWaitEvent(s, w.cap_ev[1], 0));
  const Ctrl &last = w.host_ctrl[(r - 1) % kRing];
  hipLaunchKernelGGL(k_batched_out, dim3(ub), dim3(kBlock), 0, s, n, (const int *)w.u_gid,
                     (const int *)w.b_vbase, (const int *)w.b_giters, (const double *)R[0],
                     (const double *)R[1], (double *const *)w.b_outs);
  LAUNCH_TRY();
  std::vector<int> gi(G), gd(G);
  HIP_TRY(hipMemcpyAsync(gi.data(), w.b_giters, G * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(gd.data(), w.b_gdone, G * sizeof(int), hipMemcpyDeviceToHost, s));
  timer.stop();
  HIP_TRY(hipStreamSynchronize(s));
  bool all = true;
  for (int g = 0; g < G; ++g) {
    all = all && gd[g];
    if (iters_out) iters_out[g] = gi[g];
  }
  t_stats.iterations = last.iters;
  t_stats.converged = all;
  t_stats.total_ms = timer.ms();
  return all ? PR_OK : PR_NOT_CONVERGED;
}

// ------------------------------------------------------------ allocation-free Static
// pr_static_noalloc takes its scratch from a device-resident array of fixed
// size instead of the grow-only workspace, so it calls no allocator. Each
// device holds its own copy of the array (from the time the library's code
// is loaded on it until the process ends); its address on a device is looked
// up once, with that device current, and kept. In host code the name
// `scratch` is only a stand-in: kernels get the looked-up address.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxN = 1 << 20;
constexpr int kNoAllocMaxDevices = 64;
constexpr int kNoAllocMaxGrid = 16384;
constexpr int kNoAllocSyncEvery = 4;  // iterations enqueued per convergence read
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
unsigned char *g_scratch_ptr[kNoAllocMaxDevices] = {};
int g_scratch_cus[kNoAllocMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Scratch layout of one call: byte offsets of each array, and the total.
struct NoAllocLayout {
  size_t ctrl, counts, partials, R1, X0, X1, hi, hub_start, chunk_hub, hub_part, tiles, total;
};
NoAllocLayout noalloc_layout(size_t n, size_t m, int CH, int B) {
  NoAllocLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += align256(bytes); return at; };
  const size_t chunks = m / (size_t)std::max(CH, 1) + n + 1;
  L.ctrl = take(sizeof(Ctrl));
  L.counts = take(kNumCounts * sizeof(int));
  L.partials = take(((size_t)B + kHubFinalizeBlocks + 16) * sizeof(double));
  L.R1 = take(n * sizeof(double));
  L.X0 = take(n * sizeof(double));
  L.X1 = take(n * sizeof(double));
  L.hi = take(n * sizeof(int));
  L.hub_start = take((n + 1) * sizeof(int));
  L.chunk_hub = take(chunks * sizeof(int));
  L.hub_part = take(chunks * sizeof(double));
  L.tiles = take(2 * ntiles_for(n) * sizeof(int) + 64);
  L.total = o;
  return L;
}

// Static PageRank as run_pull does it for pr_static, with the relabel and the
// die split off (lane class staged in LDS, wavefront class, split class cut
// into chunks), every array in the scratch array, and the convergence flag
// read by a copy into host stack memory every kNoAllocSyncEvery iterations.
int run_static_noalloc(const pr_csr *g, double alpha, double tol, int max_iter,
                       double *ranks_out) {
  hipStream_t s = t_stream;
  const pr_tuning tn = g_tuning;
  const int n = g->n, m = g->m, CH = tn.hub_chunk_edges;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(PR_EINVAL, "pr_static_noalloc: device index beyond the supported 64");
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    g_scratch_cus[dev] = std::max(1, cus);
    g_scratch_ptr[dev] = (unsigned char *)p;
  }
  unsigned char *base = g_scratch_ptr[dev];
  int B = tn.grid_blocks;
  if (B <= 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rank_static<false, 4>, kBlock,
                                                     0) != hipSuccess ||
        per_cu <= 0)
      per_cu = 4;
    B = per_cu * g_scratch_cus[dev];
  }
  B = std::min(B, kNoAllocMaxGrid);
  const NoAllocLayout L = noalloc_layout((size_t)n, (size_t)m, CH, B);
  if (L.total > kNoAllocBytes)
    return fail(PR_EINVAL, "pr_static_noalloc: the graph needs " + std::to_string(L.total) +
                               " bytes of scratch, more than the fixed " +
                               std::to_string(kNoAllocBytes) + " (fewer edges or vertices, or a "
                               "larger hub_chunk_edges)");
  Ctrl *ctrl = (Ctrl *)(base + L.ctrl);
  int *counts = (int *)(base + L.counts);
  double *partials = (double *)(base + L.partials);
  int *hi = (int *)(base + L.hi), *hub_start = (int *)(base + L.hub_start);
  int *chunk_hub = (int *)(base + L.chunk_hub), *tiles = (int *)(base + L.tiles);
  double *hub_part = (double *)(base + L.hub_part);
  double *R[2] = {ranks_out, (double *)(base + L.R1)};
  double *X[2] = {(double *)(base + L.X0), (double *)(base + L.X1)};
  const int t1 = tn.lane_max_degree, t2 = tn.wave_max_degree;
  const int nt = (int)ntiles_for((size_t)n);
  // Alg. 4: in-degree classes and the chunk plan of the split class
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, ctrl);
  hipLaunchKernelGGL(k_part_count, dim3(nt), dim3(kBlock), 0, s, g->in_offsets, n, t1, t2, tiles,
                     nt);
  hipLaunchKernelGGL(k_scan_rows, dim3(2), dim3(kFinalBlock), 0, s, tiles, nt, counts + kInWave,
                     (const int *)nullptr);
  hipLaunchKernelGGL(k_part_scatter, dim3(nt), dim3(kBlock), 0, s, g->in_offsets, n, t1, t2,
                     (const int *)tiles, nt, (const int *)(counts + kInWave), hi);
  hipLaunchKernelGGL(k_hub_plan, dim3(1), dim3(kFinalBlock), 0, s, g->in_offsets,
                     (const int *)hi, counts, (int)kInWave, (int)kInChunks, CH, hub_start,
                     chunk_hub);
  hipLaunchKernelGGL(k_static_init, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                     g->out_offsets, (const int *)nullptr, (const double *)nullptr,
                     1.0 / (double)n, 0, R[0], X[0], counts + kTileQueue);
  LAUNCH_TRY();
  const double C0 = (1.0 - alpha) / (double)n;
  const int np = B + kHubFinalizeBlocks;
  auto rank = k_rank_static<false, 4>;
  Ctrl host{};
  int it = 0;
  bool done = false;
  while (it < max_iter && !done) {
    const int upto = std::min(max_iter, it + kNoAllocSyncEvery);
    for (; it < upto; ++it) {
      const int a = it & 1, b = a ^ 1;
      hipLaunchKernelGGL(rank, dim3(B), dim3(kBlock), 0, s, g->in_offsets,
                         g->in_sources, (const double *)nullptr, g->out_offsets,
                         (const int *)nullptr, (const double *)X[a], (const double *)R[a], R[b],
                         X[b], (const int *)hi, (const int *)counts, (const int *)hub_start,
                         (const int *)chunk_hub, hub_part, CH, n, t1, (const int4 *)nullptr,
                         (const int *)nullptr, C0, alpha, (const double *)nullptr, 0.0, partials,
                         counts + kTileQueue, (const Ctrl *)ctrl);
      hipLaunchKernelGGL(k_hub_finalize_static, dim3(kHubFinalizeBlocks), dim3(kBlock), 0, s,
                         (const int *)hi, (const int *)counts, (const int *)hub_start,
                         (const double *)hub_part, g->out_offsets, (const int *)nullptr,
                         (const double *)R[a], R[b], X[b], C0, alpha, (const double *)nullptr,
                         0.0, 0, partials + B, counts + kTileQueue, (const Ctrl *)ctrl);
      hipLaunchKernelGGL(k_linf_final, dim3(1), dim3(kFinalBlock), 0, s,
                         (const double *)partials, np, ctrl, tol, it);
      LAUNCH_TRY();
    }
    HIP_TRY(hipMemcpyAsync(&host, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    done = host.done != 0;
  }
  const int iters = host.done ? host.iters : std::min(it, max_iter);
  double *result = R[iters & 1];
  if (result != ranks_out) {
    HIP_TRY(hipMemcpyAsync(ranks_out, result, (size_t)n * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  t_stats.iterations = iters;
  t_stats.converged = host.done;
  t_stats.final_delta = host.delta;
  return host.done ? PR_OK : PR_NOT_CONVERGED;
}

int check_edges(const pr_edges *e, const char *name) {
  if (!e) return PR_OK;
  if (e->count < 0) return fail(PR_EINVAL, std::string(name) + ".count < 0");
  if (e->count > 0 && !e->src) return fail(PR_EINVAL, std::string(name) + ".src is NULL");
  return PR_OK;
}

}  // namespace

extern "C" {

int pr_static(const pr_csr *csr, double alpha, double tol, int max_iter, double *ranks_out) {
  reset_stats();
  int rc = check_csr(csr, false);
  if (rc) return rc;
  if ((rc = check_params(alpha, tol, max_iter))) return rc;
  if (!ranks_out) return fail(PR_EINVAL, "ranks_out is NULL");
  if ((rc = on_device(csr, {{ranks_out, "ranks_out"}}))) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  return run_static(csr, alpha, tol, max_iter, nullptr, ranks_out);
}

int pr_static_noalloc(const pr_csr *csr, double alpha, double tol, int max_iter,
                      double *ranks_out) {
  reset_stats();
  int rc = check_csr(csr, false);
  if (rc) return rc;
  if ((rc = check_params(alpha, tol, max_iter))) return rc;
  if (!ranks_out) return fail(PR_EINVAL, "ranks_out is NULL");
  if (csr->n > kNoAllocMaxN)
    return fail(PR_EINVAL, "pr_static_noalloc: n must be <= " + std::to_string(kNoAllocMaxN));
  if ((rc = on_device(csr, {{ranks_out, "ranks_out"}}))) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  return run_static_noalloc(csr, alpha, tol, max_iter, ranks_out);
}

int pr_dfp_ex(const pr_csr *csr_old, const pr_csr *csr_new, const pr_edges *deletions,
              const pr_edges *insertions, const double *ranks_prev, double alpha, double tol,
              double frontier_tol, double prune_tol, int max_iter, int mode, double *ranks_out) {
  reset_stats();
  (void)csr_old;
  int rc = check_csr(csr_new, mode != PR_MODE_ND);
  if (rc) return rc;
  if ((rc = check_params(alpha, tol, max_iter))) return rc;
  if (!ranks_prev || !ranks_out) return fail(PR_EINVAL, "ranks_prev and ranks_out are required");
  if (mode != PR_MODE_DFP && mode != PR_MODE_DF && mode != PR_MODE_ND && mode != PR_MODE_DT)
    return fail(PR_EINVAL, "unknown mode");
  if (std::isnan(frontier_tol) || std::isnan(prune_tol))
    return fail(PR_EINVAL, "tolerances must not be NaN");
  if ((rc = check_edges(deletions, "deletions"))) return rc;
  if ((rc = check_edges(insertions, "insertions"))) return rc;
  if (deletions && deletions->count > 0 && !deletions->dst)
    return fail(PR_EINVAL, "deletions.dst is NULL");
  if ((rc = on_device(csr_new, {{ranks_prev, "ranks_prev"}, {ranks_out, "ranks_out"}})) ||
      (rc = edges_on_device(deletions, "deletions.src", "deletions.dst")) ||
      (rc = edges_on_device(insertions, "insertions.src", "insertions.dst")))
    return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  if (mode == PR_MODE_ND) return run_static(csr_new, alpha, tol, max_iter, ranks_prev, ranks_out);
  return run_dynamic_frontier(csr_new, deletions, insertions, ranks_prev, alpha, tol,
                              frontier_tol, prune_tol, max_iter, mode, ranks_out);
}

int pr_dfp(const pr_csr *csr_old, const pr_csr *csr_new, const pr_edges *deletions,
           const pr_edges *insertions, const double *ranks_prev, double alpha, double tol,
           double frontier_tol, double prune_tol, double *ranks_out) {
  return pr_dfp_ex(csr_old, csr_new, deletions, insertions, ranks_prev, alpha, tol, frontier_tol,
                   prune_tol, PR_MAX_ITERATIONS, PR_MODE_DFP, ranks_out);
}

int pr_ppr(const pr_csr *csr, const double *teleport, int k, double alpha, double tol,
           int max_iter, double *ranks_out, int32_t *iters_out) {
  reset_stats();
  int rc = check_csr(csr, false);
  if (rc) return rc;
  if ((rc = check_params(alpha, tol, max_iter))) return rc;
  if (k <= 0) return fail(PR_EINVAL, "k must be > 0");
  if (!teleport || !ranks_out) return fail(PR_EINVAL, "teleport and ranks_out are required");
  if ((size_t)csr->n * (size_t)k > ((size_t)1 << 40))
    return fail(PR_EINVAL, "n * k too large");
  if ((rc = on_device(csr, {{teleport, "teleport"}, {ranks_out, "ranks_out"}}))) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  return run_ppr(csr, teleport, k, alpha, tol, max_iter, ranks_out, iters_out);
}

int pr_static_batched(const pr_csr *graphs, int num_graphs, const double *const *teleport,
                      double alpha, double tol, int max_iter, double *const *ranks_out,
                      int32_t *iters_out) {
  reset_stats();
  if (!graphs || !ranks_out) return fail(PR_EINVAL, "graphs and ranks_out are required");
  if (num_graphs <= 0 || num_graphs > kMaxBatchGraphs)
    return fail(PR_EINVAL, "num_graphs must be in [1, 4096]");
  int rc;
  for (int g = 0; g < num_graphs; ++g) {
    if ((rc = check_csr(&graphs[g], false))) return rc;
    if (!ranks_out[g]) return fail(PR_EINVAL, "ranks_out[g] is NULL");
  }
  if ((rc = check_params(alpha, tol, max_iter))) return rc;
  for (int g = 0; g < num_graphs; ++g)
    if ((rc = on_device(&graphs[g], {{ranks_out[g], "ranks_out[g]"},
                                     {teleport ? teleport[g] : nullptr, "teleport[g]"}})))
      return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  return run_batched(graphs, num_graphs, teleport, alpha, tol, max_iter, ranks_out, iters_out);
}

int pr_weighted(const pr_csr *csr, const double *in_weights, const double *teleport,
                double alpha, double tol, int max_iter, double *ranks_out) {
  reset_stats();
  int rc = check_csr(csr, false);
  if (rc) return rc;
  if ((rc = check_params(alpha, tol, max_iter))) return rc;
  if (!in_weights || !ranks_out) return fail(PR_EINVAL, "in_weights and ranks_out are required");
  if ((rc = on_device(csr, {{in_weights, "in_weights"}, {teleport, "teleport"},
                            {ranks_out, "ranks_out"}})))
    return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  return run_weighted(csr, in_weights, teleport, alpha, tol, max_iter, ranks_out);
}

int pr_adjoint(const pr_csr *csr, const double *in_weights, const double *ranks,
               const double *grad_ranks, double alpha, double tol, int max_iter,
               double *grad_weights, double *grad_teleport, double *lambda_out) {
  reset_stats();
  int rc = check_csr(csr, true);
  if (rc) return rc;
  if ((rc = check_params(alpha, tol, max_iter))) return rc;
  if (!in_weights || !ranks || !grad_ranks)
    return fail(PR_EINVAL, "in_weights, ranks and grad_ranks are required");
  if (!grad_weights && !grad_teleport && !lambda_out)
    return fail(PR_EINVAL, "no output requested");
  if ((rc = on_device(csr, {{in_weights, "in_weights"}, {ranks, "ranks"},
                            {grad_ranks, "grad_ranks"}})) ||
      (rc = on_device(nullptr, {{grad_weights, "grad_weights"}, {grad_teleport, "grad_teleport"},
                                {lambda_out, "lambda_out"}})))
    return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  double *tmp = nullptr;
  if (!lambda_out) {
    hipError_t e = hipMallocAsync((void **)&tmp, (size_t)csr->n * sizeof(double), t_stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(PR_ENOMEM, "lambda buffer");
    }
  }
  rc = run_adjoint(csr, in_weights, ranks, grad_ranks, alpha, tol, max_iter, grad_weights,
                   grad_teleport, lambda_out, tmp);
  if (tmp) {
    (void)hipFreeAsync(tmp, t_stream);
    (void)hipStreamSynchronize(t_stream);
  }
  return rc;
}

int pr_apply_batch(const pr_csr *old, const pr_edges *deletions, const pr_edges *insertions,
                   const pr_csr_out *out) {
  reset_stats();
  int rc = check_csr(old, false);
  if (rc) return rc;
  if (!out || !out->in_offsets || !out->in_sources)
    return fail(PR_EINVAL, "out and its in view are required");
  const bool outview = out->out_offsets != nullptr;
  if (outview && (!out->out_targets || !old->out_targets))
    return fail(PR_EINVAL, "the out view needs old->out_targets and out->out_targets");
  if ((rc = check_edges(deletions, "deletions"))) return rc;
  if ((rc = check_edges(insertions, "insertions"))) return rc;
  const int nd = deletions ? deletions->count : 0, ni = insertions ? insertions->count : 0;
  if ((nd > 0 && !deletions->dst) || (ni > 0 && !insertions->dst))
    return fail(PR_EINVAL, "deletions.dst and insertions.dst are required");
  if (out->n != old->n || (long long)out->m != (long long)old->m - nd + ni)
    return fail(PR_EINVAL, "out->n must equal old->n and out->m = old->m - deletions + insertions");
  if ((rc = on_device(old, {{out->in_offsets, "out->in_offsets"},
                            {out->in_sources, "out->in_sources"},
                            {out->out_offsets, "out->out_offsets"},
                            {out->out_targets, "out->out_targets"}})) ||
      (rc = edges_on_device(deletions, "deletions.src", "deletions.dst")) ||
      (rc = edges_on_device(insertions, "insertions.src", "insertions.dst")))
    return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  const int32_t *ds = nd ? deletions->src : nullptr, *dd = nd ? deletions->dst : nullptr;
  const int32_t *is = ni ? insertions->src : nullptr, *id = ni ? insertions->dst : nullptr;
  int err = 0;
  const char *what = nullptr;
  // in view: rows are targets, entries sources
  int e = prhip_apply_view(old->n, old->in_offsets, old->in_sources, old->m, out->m, dd, ds, nd, id, is, ni,
                           out->in_offsets, out->in_sources, t_stream, &err, &what);
  if (e) return fail(PR_EHIP, std::string("pr_apply_batch: ") + (what ? what : "") + ": " +
                                  hipGetErrorString((hipError_t)e));
  if (!err && outview) {
    e = prhip_apply_view(old->n, old->out_offsets, old->out_targets, old->m, out->m, ds, dd, nd, is, id, ni,
                         out->out_offsets, out->out_targets, t_stream, &err, &what);
    if (e) return fail(PR_EHIP, std::string("pr_apply_batch: ") + (what ? what : "") + ": " +
                                    hipGetErrorString((hipError_t)e));
  }
  if (err) {
    std::string msg = "batch is not a normalised update of this graph:";
    if (err & 1) msg += " vertex ID out of range;";
    if (err & 2) msg += " repeated pair;";
    if (err & 4) msg += " deletion absent;";
    if (err & 8) msg += " insertion already present;";
    if (err & (16 | 32)) msg += " edge count inconsistent;";
    return fail(PR_EBATCH, msg);
  }
  return PR_OK;
}

int pr_validate_csr(const pr_csr *g) {
  reset_stats();
  int rc = check_csr(g, false);
  if (rc) return rc;
  if ((rc = on_device(g, {}))) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  hipStream_t s = t_stream;
  Workspace *wp = nullptr;
  if ((rc = get_ws(1, 1, 4096, 0, &wp))) return rc;
  Workspace &w = *wp;
  int *err = w.counts;  // reuse a device int
  const int n = g->n, nb = (n + kBlock - 1) / kBlock;
  HIP_TRY(hipMemsetAsync(err, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_validate_offsets, dim3(nb), dim3(kBlock), 0, s, g->in_offsets, n, g->m,
                     err, 1);
  hipLaunchKernelGGL(k_validate_offsets, dim3(nb), dim3(kBlock), 0, s, g->out_offsets, n, g->m,
                     err, 16);
  LAUNCH_TRY();
  HIP_TRY(hipMemcpyAsync(w.host_counts, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int e = w.host_counts[0];
  if (e & 1) return fail(PR_EGRAPH, "in_offsets: not 0 .. m non-decreasing");
  if (e & 16) return fail(PR_EGRAPH, "out_offsets: not 0 .. m non-decreasing");
  hipLaunchKernelGGL(k_validate_rows, dim3(nb), dim3(kBlock), 0, s, g->in_offsets, g->in_sources,
                     n, err, 0);
  if (g->out_targets)
    hipLaunchKernelGGL(k_validate_rows, dim3(nb), dim3(kBlock), 0, s, g->out_offsets,
                       g->out_targets, n, err, 4);
  LAUNCH_TRY();
  HIP_TRY(hipMemcpyAsync(w.host_counts, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  e = w.host_counts[0];
  if (e & 2) return fail(PR_EGRAPH, "in_sources: vertex ID outside [0, n)");
  if (e & 4) return fail(PR_EGRAPH, "in_sources: a row is not strictly ascending");
  if (e & 8) return fail(PR_EGRAPH, "in view: a vertex lacks its self-loop");
  if (e & 32) return fail(PR_EGRAPH, "out_targets: vertex ID outside [0, n)");
  if (e & 64) return fail(PR_EGRAPH, "out_targets: a row is not strictly ascending");
  if (e & 128) return fail(PR_EGRAPH, "out view: a vertex lacks its self-loop");
  return PR_OK;
}

int pr_set_tuning(const pr_tuning *t) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!t) {
    g_tuning = default_tuning();
    return PR_OK;
  }
  if (t->lane_max_degree < 0 || t->wave_max_degree < t->lane_max_degree ||
      t->expand_lane_max_degree < 0 || t->expand_lane_max_degree > t->wave_max_degree ||
      t->iters_per_sync < 1 || t->iters_per_sync >= kRing || t->hub_chunk_edges < 0 ||
      t->grid_blocks < 0 || t->grid_blocks > (1 << 20) || t->relabel < -1 || t->relabel > 1 ||
      t->xcd_split_degree < 0 || t->xcd_split_degree == 1 || t->expand_pull_per_mille < 0 ||
      t->expand_pull_per_mille > 1000 || t->frontier_list < 0 || t->frontier_list > 1 ||
      t->chain_numbering < -1 || t->chain_numbering > 1 || t->ppr_chunk_edges < 0 ||
      (t->ppr_chunk_edges > 0 && t->ppr_chunk_edges < 16) || t->ppr_chunk_edges > (1 << 20))
    return fail(PR_EINVAL, "tuning field out of range");
  g_tuning = *t;
  if (g_tuning.hub_chunk_edges == 0) g_tuning.hub_chunk_edges = 4096;
  if (g_tuning.ppr_chunk_edges == 0) g_tuning.ppr_chunk_edges = 256;
  return PR_OK;
}

int pr_get_tuning(pr_tuning *t) {
  if (!t) return fail(PR_EINVAL, "NULL");
  std::lock_guard<std::mutex> lock(g_mu);
  *t = g_tuning;
  return PR_OK;
}

int pr_last_stats(pr_stats *out) {
  if (!out) return fail(PR_EINVAL, "NULL");
  *out = t_stats;
  return PR_OK;
}

int pr_set_profiling(int level) {
  if (level < 0 || level > 2) return fail(PR_EINVAL, "profiling level must be 0, 1 or 2");
  t_profiling = level;
  return PR_OK;
}

void pr_set_stream(void *hip_stream) { t_stream = (hipStream_t)hip_stream; }

const char *pr_last_error(void) { return t_err.c_str(); }

void pr_release(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : g_ws) {
    (void)hipSetDevice(kv.first);
    free_ws(kv.second);
  }
  g_ws.clear();
  (void)hipSetDevice(cur);
}

}  // extern "C"
