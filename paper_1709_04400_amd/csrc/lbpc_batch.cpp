// lbpc_batch.cpp -- runtime of the batched form (include/lbpc.h, "batches"):
// workspace plan for many lattices, the per-lattice parameter table (one
// entry per lattice and buffer parity), the tile work list, hipGraph capture
// of one ping-pong period, and the tile-shape autotuner.
#include <algorithm>
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "lbpc_host.h"

using namespace lbpc_host;

namespace {

thread_local std::string g_berr = "";

struct WorkItem {  // mirrors the device-side work item
  int c, bx, by, slot;
};

// candidate tile shapes of the autotuner
constexpr int CAND_BW[3] = {64, 128, 256};
constexpr int CAND_H[6] = {16, 20, 24, 32, 48, 64};
constexpr int MIN_ROWS = 4;

struct CaseLayout {
  size_t dist[2][2];
  size_t rest[2];   // FP16 deviation form: FP32 rest populations per buffer
  size_t phi;
  size_t tune_phi;  // phi(t) written here while the autotuner times steps
};

struct BatchLayout {
  // partial: one diagnostic record (8 FP64) per work item; ranges: the
  // records of each lattice; diag_out: 8 FP64 results per lattice
  size_t table, work, scratch, partial, ranges, diag_out;
  size_t stage;          // nodes per field of the staging scratch
  size_t work_capacity;  // items
  std::vector<CaseLayout> cases;
  size_t total;
};

size_t max_items(const lbpc_config* cfgs, int n, int min_rows) {
  size_t items = 0;
  const int W = 64 - 2 * lbpc::HALO;
  for (int c = 0; c < n; ++c)
    items += (size_t)((cfgs[c].nx + W - 1) / W) *
             (size_t)((cfgs[c].ny + min_rows - 1) / min_rows);
  return items;
}

BatchLayout plan_batch(const lbpc_config* cfgs, int n) {
  BatchLayout L;
  size_t off = 0;
  L.table = off;
  off += align_up(2 * (size_t)n * sizeof(StepParams));
  L.work_capacity = max_items(cfgs, n, MIN_ROWS);
  L.work = off;
  off += align_up(L.work_capacity * sizeof(WorkItem));
  const size_t cap = stage_cap();
  L.stage = 0;
  for (int c = 0; c < n; ++c)
    L.stage = std::max(L.stage, stage_nodes(cfgs[c].nx, cfgs[c].ny, cap));
  L.scratch = off;
  off += align_up(5 * L.stage * sizeof(double));
  L.partial = off;
  off += align_up(L.work_capacity * 8 * sizeof(double));
  L.ranges = off;
  off += align_up(2 * (size_t)n * sizeof(int));
  L.diag_out = off;
  off += align_up((size_t)n * 8 * sizeof(double));
  L.cases.resize(n);
  for (int c = 0; c < n; ++c) {
    const size_t N = (size_t)cfgs[c].nx * cfgs[c].ny;
    for (int b = 0; b < 2; ++b) {
      for (int k = 0; k < 2; ++k) {
        L.cases[c].dist[b][k] = off;
        off += align_up(dist_bytes(cfgs[c], k));
      }
      if (dist_bytes(cfgs[c], 1) == 0)
        L.cases[c].dist[b][1] = L.cases[c].dist[b][0];
    }
    for (int b = 0; b < 2; ++b) {
      L.cases[c].rest[b] = off;
      off += align_up(rest_bytes(cfgs[c]));
    }
    const size_t h =
        align_up(hist_arrays(cfgs[c]) * N * compute_bytes(cfgs[c].precision));
    L.cases[c].phi = off;
    off += h;
    L.cases[c].tune_phi = off;
    off += h;
  }
  L.total = off;
  return L;
}

const char* check_batch(const lbpc_config* cfgs, int n) {
  if (!cfgs || n < 1) return "need at least one configuration";
  for (int c = 0; c < n; ++c) {
    const char* bad = check_config(&cfgs[c]);
    if (bad) return bad;
    if (cfgs[c].precision != cfgs[0].precision)
      return "all lattices of a batch share one precision";
    if (cfgs[c].flags != 0) return "flags are test hooks of the oracle only";
  }
  return nullptr;
}

}  // namespace

struct lbpc_batch {
  std::vector<lbpc_config> cfgs;
  int n;
  int prec;
  hipStream_t stream;
  char* ws;
  BatchLayout L;
  std::vector<StepParams> base;        // per-lattice constants
  std::vector<StepParams> table_host;  // [2n] as uploaded
  std::vector<WorkItem> work_host;
  std::vector<int> initialised;
  std::vector<double> rho_ave;
  int cur, fresh, phi_valid;
  int64_t step;
  int bw, rows, nwork, grid;
  int table_fresh, table_phi_valid;  // flags the uploaded table carries
  int tuning;  // timing launches: state read in place, phi(t) to scratch
  hipGraphExec_t graph[2];
  int use_graph;
  // per-lattice invalid-state flags written by the step kernel
  // (host-mapped pinned memory, readable without waiting), and the pinned
  // block the per-lattice diagnostic results are copied to
  int* bad_host;
  int* bad_dev;
  double* res_host;
  hipEvent_t diag_ev;
  std::string err;
};

namespace {

lbpc_status bfail(lbpc_batch* b, lbpc_status st, const std::string& msg) {
  if (b)
    b->err = msg;
  else
    g_berr = msg;
  return st;
}

#define BHIP(b, expr, what)                                                 \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return bfail(b, LBPC_ERR_HIP, std::string(what) + ": " +              \
                                        hipGetErrorString(e_));             \
  } while (0)

void* at(lbpc_batch* b, size_t off) { return b->ws + off; }

const char* const BAD_STATE =
    "a step met an invalid node state (non-finite T, rho outside (0, 1/b) "
    "or psi^2 < 0) in this lattice";

bool flagged(const lbpc_batch* b, int c) {
  return b->bad_host && static_cast<volatile int*>(b->bad_host)[c] != 0;
}

// per-lattice flags, allocated by the first initialisation (the first call
// that touches the device)
lbpc_status ensure_flags(lbpc_batch* b) {
  if (b->bad_host) return LBPC_OK;
  if (hipHostMalloc(reinterpret_cast<void**>(&b->res_host),
                    (size_t)b->n * 8 * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    b->res_host = nullptr;
    return bfail(b, LBPC_ERR_OOM, "pinned host buffer allocation failed");
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&b->bad_host),
                    (size_t)b->n * sizeof(int), hipHostMallocMapped) !=
      hipSuccess) {
    b->bad_host = nullptr;
    return bfail(b, LBPC_ERR_OOM, "pinned host flag allocation failed");
  }
  for (int c = 0; c < b->n; ++c) b->bad_host[c] = 0;
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&b->bad_dev),
                              b->bad_host, 0) != hipSuccess) {
    (void)hipHostFree(b->bad_host);
    b->bad_host = nullptr;
    return bfail(b, LBPC_ERR_HIP, "device address of the flags");
  }
  return LBPC_OK;
}

// parameters of lattice c when buffer `par` holds its state
StepParams case_params(lbpc_batch* b, int c, int par) {
  StepParams p = b->base[c];
  const CaseLayout& cl = b->L.cases[c];
  p.fin = at(b, cl.dist[par][0]);
  p.gin = at(b, cl.dist[par][1]);
  p.fout = at(b, cl.dist[1 - par][0]);
  p.gout = at(b, cl.dist[1 - par][1]);
  p.phi = at(b, cl.phi);
  p.phi_out = b->tuning ? at(b, cl.tune_phi) : p.phi;
  const bool rest = rest_bytes(b->cfgs[c]) > 0;
  p.rin = rest ? at(b, cl.rest[par]) : nullptr;
  p.rout = rest ? at(b, cl.rest[1 - par]) : nullptr;
  p.fresh = b->fresh;
  p.phi_valid = b->phi_valid;
  p.rho_ave = b->rho_ave[c];
  p.bad = b->bad_dev + c;
  p.bw = b->bw;
  strip_shape(p.nx, b->bw, true, p.nbx, p.W);
  p.H = b->rows;
  p.He = b->rows;  // batches run uniform row runs
  p.nby = (p.ny + p.H - 1) / p.H;
  p.xcd_order = 0;
  return p;
}

lbpc_status upload_table(lbpc_batch* b) {
  b->table_host.resize(2 * (size_t)b->n);
  for (int c = 0; c < b->n; ++c)
    for (int par = 0; par < 2; ++par)
      b->table_host[2 * c + par] = case_params(b, c, par);
  BHIP(b,
       hipMemcpyAsync(at(b, b->L.table), b->table_host.data(),
                      b->table_host.size() * sizeof(StepParams),
                      hipMemcpyHostToDevice, b->stream),
       "parameter table upload");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronise");
  b->table_fresh = b->fresh;
  b->table_phi_valid = b->phi_valid;
  return LBPC_OK;
}

void drop_graphs(lbpc_batch* b) {
  for (int k = 0; k < 2; ++k)
    if (b->graph[k]) {
      (void)hipGraphExecDestroy(b->graph[k]);
      b->graph[k] = nullptr;
    }
}

// work list for the current tile shape: tiles of the largest lattices first
lbpc_status build_work(lbpc_batch* b) {
  std::vector<int> order(b->n);
  for (int c = 0; c < b->n; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (long long)b->cfgs[x].nx * b->cfgs[x].ny >
           (long long)b->cfgs[y].nx * b->cfgs[y].ny;
  });
  // each tile's diagnostic record is its index here, so the records of a
  // lattice are contiguous: [ranges[2c], ranges[2c + 1])
  std::vector<WorkItem> tiles;
  std::vector<int> ranges(2 * (size_t)b->n);
  for (int c : order) {
    int nbx, W;
    strip_shape(b->cfgs[c].nx, b->bw, true, nbx, W);
    const int nby = (b->cfgs[c].ny + b->rows - 1) / b->rows;
    ranges[2 * c] = (int)tiles.size();
    for (int by = 0; by < nby; ++by)
      for (int bx = 0; bx < nbx; ++bx)
        tiles.push_back({c, bx, by, (int)tiles.size()});
    ranges[2 * c + 1] = (int)tiles.size();
  }
  if (tiles.size() > b->L.work_capacity)
    return bfail(b, LBPC_ERR_OOM, "work list exceeds its reserved space");
  BHIP(b,
       hipMemcpyAsync(at(b, b->L.ranges), ranges.data(),
                      ranges.size() * sizeof(int), hipMemcpyHostToDevice,
                      b->stream),
       "diagnostic ranges upload");
  b->work_host = xcd_order(tiles);
  b->nwork = (int)b->work_host.size();
  BHIP(b,
       hipMemcpyAsync(at(b, b->L.work), b->work_host.data(),
                      b->work_host.size() * sizeof(WorkItem),
                      hipMemcpyHostToDevice, b->stream),
       "work list upload");
  b->grid = tile_grid(b->nwork, b->prec, b->bw);
  drop_graphs(b);
  return upload_table(b);
}

lbpc_status launch(lbpc_batch* b, int parity) {
  BHIP(b,
       lbpc::launch_step_batch(
           static_cast<const StepParams*>(at(b, b->L.table)),
           at(b, b->L.work), b->nwork, parity, b->grid, b->prec, b->bw,
           b->stream),
       "batched step kernel");
  return LBPC_OK;
}

lbpc_status check_ready(lbpc_batch* b) {
  for (int c = 0; c < b->n; ++c)
    if (!b->initialised[c])
      return bfail(b, LBPC_ERR_STATE, "step before every lattice is set");
  for (int c = 0; c < b->n; ++c)
    if (flagged(b, c))
      return bfail(b, LBPC_ERR_NUMERIC,
                   std::string(BAD_STATE) + " (lattice " + std::to_string(c) +
                       ")");
  return LBPC_OK;
}

// A diagnostic launch over every lattice on the current state (with stores:
// a real step, booked by the caller; nostore: nothing is written), the
// per-lattice final reductions, the copy of the results into the pinned
// block and an event after it.
lbpc_status enqueue_diag(lbpc_batch* b, bool nostore) {
  if (b->table_fresh != b->fresh || b->table_phi_valid != b->phi_valid) {
    lbpc_status st = upload_table(b);
    if (st != LBPC_OK) return st;
  }
  if (!b->diag_ev)
    BHIP(b, hipEventCreateWithFlags(&b->diag_ev, hipEventDisableTiming),
         "event");
  double* part = static_cast<double*>(at(b, b->L.partial));
  BHIP(b,
       lbpc::launch_step_batch(
           static_cast<const StepParams*>(at(b, b->L.table)),
           at(b, b->L.work), b->nwork, b->cur, b->grid, b->prec, b->bw,
           b->stream, true, part, nostore ? 1 : 0),
       "diagnostic step kernel");
  double* dout = static_cast<double*>(at(b, b->L.diag_out));
  BHIP(b,
       lbpc::launch_diag_reduce(part,
                                static_cast<const int*>(at(b, b->L.ranges)),
                                0, 0, b->n, dout, b->stream),
       "diagnostic reduction");
  BHIP(b,
       hipMemcpyAsync(b->res_host, dout, (size_t)b->n * 8 * sizeof(double),
                      hipMemcpyDeviceToHost, b->stream),
       "copy of the diagnostics");
  BHIP(b, hipEventRecord(b->diag_ev, b->stream), "event");
  return LBPC_OK;
}

lbpc_status run_batch_steps(lbpc_batch* b, int64_t n);

}  // namespace

extern "C" {

lbpc_status lbpc_batch_workspace_bytes(const lbpc_config* cfgs, int32_t n,
                                       size_t* bytes) {
  const char* bad = check_batch(cfgs, n);
  if (bad) return bfail(nullptr, LBPC_ERR_ARG, bad);
  if (!bytes) return bfail(nullptr, LBPC_ERR_ARG, "bytes is NULL");
  *bytes = plan_batch(cfgs, n).total;
  return LBPC_OK;
}

lbpc_status lbpc_batch_create(const lbpc_config* cfgs, int32_t n,
                              void* dev_workspace, size_t workspace_bytes,
                              void* hip_stream, lbpc_batch** out) {
  if (!out) return bfail(nullptr, LBPC_ERR_ARG, "out is NULL");
  *out = nullptr;
  const char* bad = check_batch(cfgs, n);
  if (bad) return bfail(nullptr, LBPC_ERR_ARG, bad);
  BatchLayout L = plan_batch(cfgs, n);
  if (!dev_workspace || workspace_bytes < L.total)
    return bfail(nullptr, LBPC_ERR_OOM, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN != 0)
    return bfail(nullptr, LBPC_ERR_ARG, "workspace must be 256-byte aligned");
  lbpc_batch* b = new (std::nothrow) lbpc_batch();
  if (!b) return bfail(nullptr, LBPC_ERR_OOM, "host allocation failed");
  b->cfgs.assign(cfgs, cfgs + n);
  b->n = n;
  b->prec = cfgs[0].precision;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->ws = static_cast<char*>(dev_workspace);
  b->L = L;
  b->bad_host = nullptr;
  b->bad_dev = nullptr;
  b->res_host = nullptr;
  b->diag_ev = nullptr;
  b->base.resize(n);
  for (int c = 0; c < n; ++c) derive_params(cfgs[c], b->base[c]);
  b->initialised.assign(n, 0);
  b->rho_ave.assign(n, 0.0);
  b->cur = 0;
  b->fresh = 1;
  b->phi_valid = 0;
  b->step = 0;
  b->bw = env_int("LBPC_TILE_BW", 256);
  if (!valid_block_width(b->bw)) b->bw = 256;
  b->rows = std::max(MIN_ROWS, env_int("LBPC_TILE_H", 32));
  b->graph[0] = b->graph[1] = nullptr;
  // graph replay (on request: eager launches measured faster here) needs a
  // capturable (non-NULL) stream
  b->use_graph = b->stream != nullptr && env_int("LBPC_BATCH_GRAPH", 0) != 0;
  lbpc_status st = build_work(b);
  if (st != LBPC_OK) {
    g_berr = b->err;
    delete b;
    return st;
  }
  *out = b;
  return LBPC_OK;
}

lbpc_status lbpc_batch_init_fields(lbpc_batch* b, int32_t c,
                                   const double* rho, const double* ux,
                                   const double* uy, const double* T) {
  if (!b) return bfail(nullptr, LBPC_ERR_ARG, "batch is NULL");
  if (c < 0 || c >= b->n) return bfail(b, LBPC_ERR_ARG, "lattice index");
  if (!rho || !ux || !uy || !T)
    return bfail(b, LBPC_ERR_ARG, "field pointer is NULL");
  if (b->step != 0)
    return bfail(b, LBPC_ERR_STATE, "initial fields after the first step");
  const char* bad = check_fields(b->cfgs[c], rho, ux, uy, T, &b->rho_ave[c]);
  if (bad) return bfail(b, LBPC_ERR_ARG, bad);
  {
    lbpc_status st = ensure_flags(b);
    if (st != LBPC_OK) return st;
  }
  double* scr = static_cast<double*>(at(b, b->L.scratch));
  const double* src[4] = {rho, ux, uy, T};
  StepParams p = case_params(b, c, b->cur);
  {
    const char* what = "";
    BHIP(b, stage_init(p, b->prec, scr, b->L.stage, src, b->stream, &what), what);
  }
  b->bad_host[c] = 0;
  b->initialised[c] = 1;
  b->fresh = 1;
  b->phi_valid = 0;
  return upload_table(b);
}

lbpc_status lbpc_batch_set_tiles(lbpc_batch* b, int32_t block_width,
                                 int32_t rows) {
  if (!b) return bfail(nullptr, LBPC_ERR_ARG, "batch is NULL");
  if (!valid_block_width(block_width))
    return bfail(b, LBPC_ERR_ARG, "block width must be 64, 128, 256 or 512");
  if (rows < MIN_ROWS) return bfail(b, LBPC_ERR_ARG, "rows must be >= 4");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronise");
  b->bw = block_width;
  b->rows = rows;
  return build_work(b);
}

lbpc_status lbpc_batch_autotune(lbpc_batch* b, int32_t steps,
                                int32_t* block_width, int32_t* rows,
                                double* ms_per_step) {
  if (!b) return bfail(nullptr, LBPC_ERR_ARG, "batch is NULL");
  if (steps < 1) return bfail(b, LBPC_ERR_ARG, "steps < 1");
  for (int c = 0; c < b->n; ++c)
    if (!b->initialised[c])
      return bfail(b, LBPC_ERR_STATE, "autotune before every lattice is set");
  // timing launches read the current buffer and write the other one (whose
  // contents the next real step overwrites) and send phi(t) to scratch, so
  // the state and the phi history are left as they are
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0), "event");
  BHIP(b, hipEventCreate(&e1), "event");
  float best = 1e30f;
  int best_bw = b->bw, best_rows = b->rows;
  // candidates: the shape in place, then the fixed set
  std::vector<std::array<int, 2>> cand{{b->bw, b->rows}};
  for (int bw : CAND_BW)
    for (int h : CAND_H) cand.push_back({bw, h});
  b->tuning = 1;
  lbpc_status st = LBPC_OK;
  for (size_t k = 0; k < cand.size(); ++k) {
    bool seen = false;
    for (size_t j = 0; j < k; ++j) seen = seen || cand[j] == cand[k];
    if (seen) continue;
    b->bw = cand[k][0];
    b->rows = cand[k][1];
    st = build_work(b);
    if (st == LBPC_OK) st = launch(b, b->cur);  // warm-up
    if (st != LBPC_OK) break;
    hipError_t e = hipEventRecord(e0, b->stream);
    for (int s = 0; s < steps && st == LBPC_OK; ++s) st = launch(b, b->cur);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess && st == LBPC_OK)
      st = bfail(b, LBPC_ERR_HIP, std::string("autotune timing: ") +
                                      hipGetErrorString(e));
    if (st != LBPC_OK) break;
    if (ms < best) {
      best = ms;
      best_bw = cand[k][0];
      best_rows = cand[k][1];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tuning = 0;
  b->bw = best_bw;
  b->rows = best_rows;
  lbpc_status st2 = build_work(b);
  if (st != LBPC_OK) return st;
  if (st2 != LBPC_OK) return st2;
  if (block_width) *block_width = best_bw;
  if (rows) *rows = best_rows;
  if (ms_per_step) *ms_per_step = best / steps;
  return LBPC_OK;
}

lbpc_status lbpc_batch_step(lbpc_batch* b, int64_t n) {
  if (!b) return bfail(nullptr, LBPC_ERR_ARG, "batch is NULL");
  if (n < 0) return bfail(b, LBPC_ERR_ARG, "n < 0");
  lbpc_status st0 = check_ready(b);
  if (st0 != LBPC_OK) return st0;
  return run_batch_steps(b, n);
}

lbpc_status lbpc_batch_step_diag(lbpc_batch* b, int64_t n, lbpc_diag* out) {
  if (!b) return bfail(nullptr, LBPC_ERR_ARG, "batch is NULL");
  if (n < 1 || !out) return bfail(b, LBPC_ERR_ARG, "n < 1 or out is NULL");
  lbpc_status st = check_ready(b);
  if (st != LBPC_OK) return st;
  st = enqueue_diag(b, false);
  if (st != LBPC_OK) return st;
  const int64_t t0 = b->step;
  b->cur = 1 - b->cur;
  b->fresh = 0;
  b->phi_valid = 1;
  b->step += 1;
  st = run_batch_steps(b, n - 1);
  BHIP(b, hipEventSynchronize(b->diag_ev), "synchronise");
  bool bad = false;
  for (int c = 0; c < b->n; ++c) {
    fill_diag(&out[c], b->res_host + 8 * (size_t)c, b->cfgs[c].cv, t0,
              flagged(b, c));
    bad = bad || out[c].nonfinite;
  }
  if (st != LBPC_OK) return st;
  if (bad) return bfail(b, LBPC_ERR_NUMERIC, BAD_STATE);
  return LBPC_OK;
}

}  // extern "C"

namespace {

lbpc_status run_batch_steps(lbpc_batch* b, int64_t n) {
  while (n > 0) {
    const bool steady = !b->fresh && b->phi_valid;
    if (steady && (b->table_fresh || !b->table_phi_valid)) {
      lbpc_status st = upload_table(b);
      if (st != LBPC_OK) return st;
    }
    if (steady && b->use_graph && n >= 2) {
      hipGraphExec_t& g = b->graph[b->cur];
      if (!g) {
        hipGraph_t graph = nullptr;
        BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal),
             "graph capture");
        lbpc_status st = launch(b, b->cur);
        lbpc_status st2 = st == LBPC_OK ? launch(b, 1 - b->cur) : st;
        hipError_t e = hipStreamEndCapture(b->stream, &graph);
        if (e == hipSuccess && st2 == LBPC_OK)
          e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
        // the captured graph is not needed once instantiated, nor on failure
        if (graph) (void)hipGraphDestroy(graph);
        if (st2 != LBPC_OK) return st2;
        if (e != hipSuccess) g = nullptr;
        BHIP(b, e, "graph capture");
      }
      const int64_t pairs = n / 2;
      for (int64_t k = 0; k < pairs; ++k)
        BHIP(b, hipGraphLaunch(g, b->stream), "graph launch");
      b->step += 2 * pairs;
      n -= 2 * pairs;
      continue;
    }
    if (!steady && (b->table_fresh != b->fresh ||
                    b->table_phi_valid != b->phi_valid)) {
      lbpc_status st = upload_table(b);
      if (st != LBPC_OK) return st;
    }
    lbpc_status st = launch(b, b->cur);
    if (st != LBPC_OK) return st;
    b->cur = 1 - b->cur;
    b->fresh = 0;
    b->phi_valid = 1;
    b->step += 1;
    n -= 1;
  }
  return LBPC_OK;
}

}  // namespace

extern "C" {

lbpc_status lbpc_batch_get_rho_u_T(lbpc_batch* b, int32_t c, double* rho,
                                   double* ux, double* uy, double* T) {
  if (!b) return bfail(nullptr, LBPC_ERR_ARG, "batch is NULL");
  if (c < 0 || c >= b->n) return bfail(b, LBPC_ERR_ARG, "lattice index");
  if (!b->initialised[c]) return bfail(b, LBPC_ERR_STATE, "not initialised");
  const size_t N = (size_t)b->cfgs[c].nx * b->cfgs[c].ny;
  double* scr = static_cast<double*>(at(b, b->L.scratch));
  StepParams p = case_params(b, c, b->cur);
  double* dst[4] = {rho, ux, uy, T};
  {
    const char* what = "";
    BHIP(b, stage_fields(p, b->prec, scr, b->L.stage, dst, b->stream, &what), what);
  }
  if (flagged(b, c)) return bfail(b, LBPC_ERR_NUMERIC, BAD_STATE);
  for (int k = 0; k < 4; ++k)
    if (dst[k])
      for (size_t i = 0; i < N; ++i)
        if (!std::isfinite(dst[k][i]))
          return bfail(b, LBPC_ERR_NUMERIC, "non-finite field value");
  return LBPC_OK;
}

lbpc_status lbpc_batch_get_diag(lbpc_batch* b, int32_t c, lbpc_diag* out) {
  if (!b) return bfail(nullptr, LBPC_ERR_ARG, "batch is NULL");
  if (c < 0 || c >= b->n || !out) return bfail(b, LBPC_ERR_ARG, "argument");
  for (int k = 0; k < b->n; ++k)
    if (!b->initialised[k])
      return bfail(b, LBPC_ERR_STATE, "not every lattice is initialised");
  lbpc_status st = enqueue_diag(b, true);
  if (st != LBPC_OK) return st;
  BHIP(b, hipEventSynchronize(b->diag_ev), "synchronise");
  fill_diag(out, b->res_host + 8 * (size_t)c, b->cfgs[c].cv, b->step,
            flagged(b, c));
  if (out->nonfinite) return bfail(b, LBPC_ERR_NUMERIC, BAD_STATE);
  return LBPC_OK;
}

lbpc_status lbpc_batch_nodes(const lbpc_batch* b, int64_t* nodes) {
  if (!b || !nodes) return bfail(nullptr, LBPC_ERR_ARG, "NULL argument");
  int64_t s = 0;
  for (const auto& c : b->cfgs) s += (int64_t)c.nx * c.ny;
  *nodes = s;
  return LBPC_OK;
}

void lbpc_batch_destroy(lbpc_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  if (b->diag_ev) (void)hipEventDestroy(b->diag_ev);
  if (b->bad_host) (void)hipHostFree(b->bad_host);
  if (b->res_host) (void)hipHostFree(b->res_host);
  delete b;
}

const char* lbpc_batch_last_error(const lbpc_batch* b) {
  return b ? b->err.c_str() : g_berr.c_str();
}

}  // extern "C"
