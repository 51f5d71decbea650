// lbpc_api.cpp -- host runtime behind include/lbpc.h: configuration checks,
// derived constants, the workspace plan, state bookkeeping (ping-pong
// buffer, fresh / phi_prev flags) and the launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <mutex>
#include <string>
#include <vector>

#include "lbpc_host.h"

using namespace lbpc_host;

namespace {
thread_local std::string g_err = "";
}  // namespace

struct lbpc_handle {
  lbpc_config cfg;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  Layout L;
  StepParams base;
  int cur;        // buffer holding the state
  int fresh;      // state buffer holds pre-collision f(t)
  int phi_valid;  // phi history holds phi(t-1)
  int initialised;
  int64_t step;
  double rho_ave;
  // non-periodic lattices run the persistent tile kernel, which reads its
  // parameters from a device table (one entry per buffer parity)
  int tiled;
  int force_gen;  // LBPC_FORCE_GEN: boundary-capable kernel on periodic sides
  int cus;        // compute units of the device (default tile heights)
  int table_fresh, table_phi_valid, table_valid, table_tuning;
  int nwork, grid;
  StepParams table_host[2];
  // invalid-state flag written by the step kernel: host-mapped pinned
  // memory, so lbpc_step can read it without waiting; the diagnostic
  // results are copied into the same pinned block (res_host)
  int* bad_host;
  int* bad_dev;
  double* res_host;
  hipEvent_t diag_ev;  // recorded after a diagnostic's copy to res_host
  // steady-state steps are replayed from a captured graph of one ping-pong
  // period (two launches), one per starting buffer
  hipGraphExec_t graph[2];
  int use_graph;
  // two steps per launch (4-byte storage forms, periodic lattices): its own
  // tile shape, and the phi history in one of two arrays (phi_sel), since
  // that kernel reads phi(t-1) of nodes other blocks write phi(t+1) of
  int two_step;
  StepParams ts;
  int phi_sel;
  std::string err;
};

namespace {

lbpc_status fail(lbpc_handle* h, lbpc_status st, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_err = msg;
  return st;
}

const char* const BAD_STATE =
    "a step met an invalid node state (non-finite T, rho outside (0, 1/b) "
    "or psi^2 < 0); load a saved state to continue";

// flag of the invalid-state check (only meaningful once the launches that
// may set it have completed)
bool flagged(const lbpc_handle* h) {
  return h->bad_host && *static_cast<volatile int*>(h->bad_host) != 0;
}

// the flag is allocated by the first call that touches the device (an
// initialisation or a state load), and cleared there
lbpc_status reset_flag(lbpc_handle* h) {
  if (!h->bad_host) {
    // 64 bytes for the flag, then the 8 diagnostic results
    if (hipHostMalloc(reinterpret_cast<void**>(&h->bad_host),
                      64 + 8 * sizeof(double), hipHostMallocMapped) !=
        hipSuccess) {
      h->bad_host = nullptr;
      return fail(h, LBPC_ERR_OOM, "pinned host flag allocation failed");
    }
    h->res_host = reinterpret_cast<double*>(
        reinterpret_cast<char*>(h->bad_host) + 64);
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&h->bad_dev),
                                h->bad_host, 0) != hipSuccess) {
      (void)hipHostFree(h->bad_host);
      h->bad_host = nullptr;
      return fail(h, LBPC_ERR_HIP, "device address of the flag");
    }
    h->base.bad = h->bad_dev;
    h->table_valid = 0;
  }
  *h->bad_host = 0;
  return LBPC_OK;
}

lbpc_status hip_fail(lbpc_handle* h, hipError_t e, const char* what) {
  return fail(h, LBPC_ERR_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, expr, what)                 \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_fail(h, e_, what); \
  } while (0)

void* at(lbpc_handle* h, size_t off) { return h->ws + off; }
double* ws_part(lbpc_handle* h) {
  return static_cast<double*>(at(h, h->L.partial));
}
double* ws_dout(lbpc_handle* h) {
  return static_cast<double*>(at(h, h->L.diag_out));
}

// Scratch of lbpc_get_diag_noalloc, for callers that cannot allocate:
// NOALLOC_RECORDS tile records of 8 FP64 values, then the 8 results (4 MiB
// in all), held by every GPU the library runs on until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address on the current GPU comes from hipGetSymbolAddress, taken
// once per device (at the first initialisation on it) and kept below.
constexpr int NOALLOC_RECORDS = 65536;
__device__ __align__(256) double scratch[((size_t)NOALLOC_RECORDS + 1) * 8];
constexpr int MAX_DEVICES = 64;
double* g_scratch_ptr[MAX_DEVICES];
std::mutex g_scratch_mu;

// device address of this GPU's scratch (looked up on the current device)
lbpc_status scratch_for_device(lbpc_handle* h, double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(h, e, "current device");
  if (dev < 0 || dev >= MAX_DEVICES)
    return fail(h, LBPC_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return hip_fail(h, e != hipSuccess ? e : hipErrorInvalidSymbol,
                      "address of the diagnostic scratch");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return LBPC_OK;
}

// the two phi history arrays: the state's (phi_sel) and the other one,
// scratch for launches that must not touch the history
void* phi_buf(lbpc_handle* h, int sel) {
  return at(h, sel ? h->L.tune_phi : h->L.phi);
}

// step parameters for the current state (input = buffer cur)
StepParams params_now(lbpc_handle* h) {
  StepParams p = h->base;
  p.fin = at(h, h->L.dist[h->cur][0]);
  p.gin = at(h, h->L.dist[h->cur][1]);
  p.fout = at(h, h->L.dist[1 - h->cur][0]);
  p.gout = at(h, h->L.dist[1 - h->cur][1]);
  p.phi = phi_buf(h, h->phi_sel);
  p.phi_out = p.phi;
  const bool rest = rest_bytes(h->cfg) > 0;
  p.rin = rest ? at(h, h->L.rest[h->cur]) : nullptr;
  p.rout = rest ? at(h, h->L.rest[1 - h->cur]) : nullptr;
  p.fresh = h->fresh;
  p.phi_valid = h->phi_valid;
  p.rho_ave = h->rho_ave;
  return p;
}

void drop_graphs(lbpc_handle* h) {
  for (int k = 0; k < 2; ++k)
    if (h->graph[k]) {
      (void)hipGraphExecDestroy(h->graph[k]);
      h->graph[k] = nullptr;
    }
}

// tile shape of the step launches (rows_edge: runs of the x-edge strips on
// the non-periodic path); the tile list of that path is rebuilt (and
// re-uploaded) at the next launch
void set_tiles_impl(lbpc_handle* h, int bw, int rows, int rows_edge) {
  drop_graphs(h);
  StepParams& p = h->base;
  p.bw = bw;
  strip_shape(h->cfg.nx, bw, balanced_strips(h->cfg.precision, bw), p.nbx, p.W);
  p.H = rows;
  // the step kernels take a separate edge-strip height in FP64 and the FP16
  // forms only
  p.He = h->cfg.precision == LBPC_FP32 ||
                 h->cfg.precision == LBPC_FP32_SHIFTED
             ? rows
             : rows_edge;
  p.nby = (h->cfg.ny + p.H - 1) / p.H;
  if (h->tiled) {
    h->nwork = (int)tile_list(p).size();
    h->grid = tile_grid(h->nwork, h->cfg.precision, bw);
    h->table_valid = 0;
  }
}

// uploads the non-periodic path needs before its launches (tile list,
// parameter table for the current state flags); none when they are current
lbpc_status prepare_step(lbpc_handle* h, bool tuning) {
  if (!h->tiled) return LBPC_OK;
  if (!h->table_valid) {
    std::vector<std::array<int, 4>> work = xcd_order(tile_list(h->base));
    if (work.size() > h->L.work_capacity)
      return fail(h, LBPC_ERR_ARG, "tile list exceeds the workspace's capacity");
    HIP_TRY(h,
            hipMemcpyAsync(at(h, h->L.work), work.data(),
                           work.size() * sizeof(work[0]),
                           hipMemcpyHostToDevice, h->stream),
            "tile list upload");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    h->table_valid = 1;
    h->table_fresh = -1;
  }
  const int want_tune = tuning ? 1 : 0;
  if (h->table_fresh != h->fresh || h->table_phi_valid != h->phi_valid ||
      h->table_tuning != want_tune) {
    const int keep = h->cur;
    for (int par = 0; par < 2; ++par) {
      h->cur = par;
      h->table_host[par] = params_now(h);
      if (tuning) h->table_host[par].phi_out = phi_buf(h, 1 - h->phi_sel);
    }
    h->cur = keep;
    HIP_TRY(h,
            hipMemcpyAsync(at(h, h->L.table), h->table_host,
                           sizeof(h->table_host), hipMemcpyHostToDevice,
                           h->stream),
            "parameter table upload");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    h->table_fresh = h->fresh;
    h->table_phi_valid = h->phi_valid;
    h->table_tuning = want_tune;
  }
  return LBPC_OK;
}

// the launch alone (capturable: no uploads, no waits)
lbpc_status launch_now(lbpc_handle* h, bool tuning) {
  StepParams p = params_now(h);
  if (tuning) p.phi_out = phi_buf(h, 1 - h->phi_sel);
  if (!h->tiled)
    return lbpc::launch_step(p, h->cfg.precision, h->stream) == hipSuccess
               ? LBPC_OK
               : fail(h, LBPC_ERR_HIP, "step kernel launch");
  HIP_TRY(h,
          lbpc::launch_step_batch(
              static_cast<const StepParams*>(at(h, h->L.table)),
              at(h, h->L.work), h->nwork, h->cur, h->grid, h->cfg.precision,
              p.bw, h->stream,
              !(p.perx && p.pery) || h->force_gen),
          "step kernel");
  return LBPC_OK;
}

// one launch of the step on the current state (buffer cur -> 1 - cur); the
// caller flips the state afterwards, except for the autotuner, whose timing
// launches send phi(t) to scratch and leave the state as it is
lbpc_status enqueue_step(lbpc_handle* h, bool tuning) {
  lbpc_status st = prepare_step(h, tuning);
  return st == LBPC_OK ? launch_now(h, tuning) : st;
}

// A diagnostic launch of the step kernel on the current state (with stores:
// a real step, which the caller then books; nostore: nothing is written),
// the final reduction of its tile records, the copy of the 8 results into
// the pinned block and an event after it.
// Tile records of the current shape (one per tile of the launch).
int tile_count(const lbpc_handle* h) {
  return h->tiled ? h->nwork : h->base.nbx * h->base.nby;
}

// part: the tile records (tile_count of them), dout: the 8 results; both in
// the workspace, or in the static scratch of the no-allocation variant.
lbpc_status enqueue_diag(lbpc_handle* h, bool nostore, double* part,
                         double* dout) {
  lbpc_status st = prepare_step(h, false);
  if (st != LBPC_OK) return st;
  if (!h->diag_ev)
    HIP_TRY(h, hipEventCreateWithFlags(&h->diag_ev, hipEventDisableTiming),
            "event");
  StepParams p = params_now(h);
  int ntiles;
  if (!h->tiled) {
    ntiles = p.nbx * p.nby;
    HIP_TRY(h, lbpc::launch_step(p, h->cfg.precision, h->stream, part,
                                 nostore ? 1 : 0),
            "diagnostic step kernel");
  } else {
    ntiles = h->nwork;
    HIP_TRY(h,
            lbpc::launch_step_batch(
                static_cast<const StepParams*>(at(h, h->L.table)),
                at(h, h->L.work), h->nwork, h->cur, h->grid,
                h->cfg.precision, p.bw, h->stream,
                !(p.perx && p.pery) || h->force_gen, part, nostore ? 1 : 0),
            "diagnostic step kernel");
  }
  HIP_TRY(h,
          lbpc::launch_diag_reduce(part, nullptr, 0, ntiles, 1, dout,
                                   h->stream),
          "diagnostic reduction");
  HIP_TRY(h,
          hipMemcpyAsync(h->res_host, dout, 8 * sizeof(double),
                         hipMemcpyDeviceToHost, h->stream),
          "copy of the diagnostics");
  HIP_TRY(h, hipEventRecord(h->diag_ev, h->stream), "event");
  return LBPC_OK;
}

lbpc_status run_steps(lbpc_handle* h, int64_t n);

}  // namespace

extern "C" {

lbpc_status lbpc_workspace_bytes(const lbpc_config* cfg, size_t* bytes) {
  const char* bad = check_config(cfg);
  if (bad) return fail(nullptr, LBPC_ERR_ARG, bad);
  if (!bytes) return fail(nullptr, LBPC_ERR_ARG, "bytes is NULL");
  *bytes = plan(*cfg).total;
  return LBPC_OK;
}

lbpc_status lbpc_create(const lbpc_config* cfg, void* dev_workspace,
                        size_t workspace_bytes, void* hip_stream,
                        lbpc_handle** out) {
  if (!out) return fail(nullptr, LBPC_ERR_ARG, "out is NULL");
  *out = nullptr;
  const char* bad = check_config(cfg);
  if (bad) return fail(nullptr, LBPC_ERR_ARG, bad);
  if (cfg->flags != 0)
    return fail(nullptr, LBPC_ERR_UNSUPPORTED,
                "flags are test hooks of the CPU oracle only");
  Layout L = plan(*cfg);
  if (!dev_workspace || workspace_bytes < L.total)
    return fail(nullptr, LBPC_ERR_OOM, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN != 0)
    return fail(nullptr, LBPC_ERR_ARG, "workspace must be 256-byte aligned");
  lbpc_handle* h = new (std::nothrow) lbpc_handle();
  if (!h) return fail(nullptr, LBPC_ERR_OOM, "host allocation failed");
  h->cfg = *cfg;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(dev_workspace);
  h->ws_bytes = workspace_bytes;
  h->L = L;
  StepParams& p = h->base;
  derive_params(*cfg, p);
  {
    // default tile shape; LBPC_TILE_BW and LBPC_TILE_H override it, and
    // lbpc_autotune / lbpc_set_tiles change it
    h->tiled = !(p.perx && p.pery) || env_int("LBPC_FORCE_TILED", 0);
    h->force_gen = env_int("LBPC_FORCE_GEN", 0) != 0;
    int bw, rows, rows_edge, dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                  dev);
    if (cus < 1) cus = 256;
    h->cus = cus;
    default_tiles(*cfg, h->tiled != 0, cus, bw, rows, rows_edge);
    p.xcd_order = env_int("LBPC_XCD_ORDER", 1);
    // graph replay (on request: eager launches measured faster here) needs
    // a capturable (non-NULL) stream
    h->use_graph = h->stream != nullptr && env_int("LBPC_GRAPH", 0) != 0;
    set_tiles_impl(h, bw, rows, rows_edge);
    h->two_step = two_step_tiles(*cfg, h->tiled != 0, h->use_graph != 0,
                                 cus, h->ts);
    if (h->two_step) {
      StepParams& q = h->ts;
      const StepParams keep = q;
      q = h->base;  // constants of the lattice, then the two-step tiling
      q.bw = keep.bw;
      q.W = keep.W;
      q.H = keep.H;
      q.He = keep.H;
      q.nbx = keep.nbx;
      q.nby = keep.nby;
    }
  }
  *out = h;
  return LBPC_OK;
}

lbpc_status lbpc_init_fields(lbpc_handle* h, const double* rho,
                             const double* ux, const double* uy,
                             const double* T) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (!rho || !ux || !uy || !T)
    return fail(h, LBPC_ERR_ARG, "field pointer is NULL");
  const lbpc_config& c = h->cfg;
  const char* bad = check_fields(c, rho, ux, uy, T, &h->rho_ave);
  if (bad) return fail(h, LBPC_ERR_ARG, bad);
  double* scr = static_cast<double*>(at(h, h->L.scratch));
  const double* src[4] = {rho, ux, uy, T};
  h->cur = 0;
  h->phi_sel = 0;
  StepParams p = params_now(h);
  drop_graphs(h);
  {
    const char* what = "";
    hipError_t e = stage_init(p, c.precision, scr, h->L.stage, src, h->stream, &what);
    if (e != hipSuccess) return hip_fail(h, e, what);
  }
  {
    lbpc_status st = reset_flag(h);
    if (st != LBPC_OK) return st;
    double* sp = nullptr;  // set-up of lbpc_get_diag_noalloc on this device
    st = scratch_for_device(h, &sp);
    if (st != LBPC_OK) return st;
  }
  h->fresh = 1;
  h->phi_valid = 0;
  h->step = 0;
  h->initialised = 1;
  h->table_fresh = -1;
  return LBPC_OK;
}

lbpc_status lbpc_step(lbpc_handle* h, int64_t n) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (n < 0) return fail(h, LBPC_ERR_ARG, "n < 0");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "step before init");
  // steps already completed may have flagged an invalid state
  if (flagged(h)) return fail(h, LBPC_ERR_NUMERIC, BAD_STATE);
  return run_steps(h, n);
}

lbpc_status lbpc_step_diag(lbpc_handle* h, int64_t n, lbpc_diag* out) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (n < 1 || !out) return fail(h, LBPC_ERR_ARG, "n < 1 or out is NULL");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "step before init");
  if (flagged(h)) return fail(h, LBPC_ERR_NUMERIC, BAD_STATE);
  lbpc_status st = enqueue_diag(h, false, ws_part(h), ws_dout(h));
  if (st != LBPC_OK) return st;
  const int64_t t0 = h->step;
  h->cur = 1 - h->cur;
  h->fresh = 0;
  h->phi_valid = 1;
  h->step += 1;
  st = run_steps(h, n - 1);
  HIP_TRY(h, hipEventSynchronize(h->diag_ev), "synchronise");
  fill_diag(out, h->res_host, h->cfg.cv, t0, flagged(h));
  if (st != LBPC_OK) return st;
  if (out->nonfinite) return fail(h, LBPC_ERR_NUMERIC, BAD_STATE);
  return LBPC_OK;
}

}  // extern "C"

namespace {

lbpc_status run_steps(lbpc_handle* h, int64_t n) {
  while (n >= 2 && h->two_step) {
    // two steps in one launch: state buffer cur -> 1 - cur, phi history
    // from one array to the other
    StepParams p = params_now(h);
    StepParams q = h->ts;
    q.fin = p.fin;
    q.gin = p.gin;
    q.fout = p.fout;
    q.gout = p.gout;
    q.phi = p.phi;
    q.phi_out = phi_buf(h, 1 - h->phi_sel);
    q.fresh = p.fresh;
    q.phi_valid = p.phi_valid;
    q.rho_ave = p.rho_ave;
    q.bad = p.bad;
    HIP_TRY(h, lbpc::launch_two_steps(q, h->cfg.precision, h->stream),
            "two-step kernel");
    h->cur = 1 - h->cur;
    h->phi_sel = 1 - h->phi_sel;
    h->fresh = 0;
    h->phi_valid = 1;
    h->step += 2;
    n -= 2;
  }
  while (n > 0) {
    // steady state (state flags fixed): pairs of steps replay the graph of
    // one ping-pong period that starts from the current buffer
    if (h->use_graph && !h->fresh && h->phi_valid && n >= 2) {
      lbpc_status st = prepare_step(h, false);
      if (st != LBPC_OK) return st;
      hipGraphExec_t& g = h->graph[h->cur];
      if (!g) {
        hipGraph_t graph = nullptr;
        HIP_TRY(h,
                hipStreamBeginCapture(h->stream,
                                      hipStreamCaptureModeThreadLocal),
                "graph capture");
        const int keep = h->cur;
        st = launch_now(h, false);
        h->cur = 1 - keep;
        lbpc_status st2 = st == LBPC_OK ? launch_now(h, false) : st;
        h->cur = keep;
        hipError_t e = hipStreamEndCapture(h->stream, &graph);
        if (e == hipSuccess && st2 == LBPC_OK)
          e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
        // the captured graph is not needed once instantiated, nor on failure
        if (graph) (void)hipGraphDestroy(graph);
        if (st2 != LBPC_OK) return st2;
        if (e != hipSuccess) g = nullptr;
        HIP_TRY(h, e, "graph capture");
      }
      const int64_t pairs = n / 2;
      for (int64_t k = 0; k < pairs; ++k)
        HIP_TRY(h, hipGraphLaunch(g, h->stream), "graph launch");
      h->step += 2 * pairs;
      n -= 2 * pairs;
      continue;
    }
    lbpc_status st = enqueue_step(h, false);
    if (st != LBPC_OK) return st;
    h->cur = 1 - h->cur;
    h->fresh = 0;
    h->phi_valid = 1;
    h->step += 1;
    n -= 1;
  }
  return LBPC_OK;
}

}  // namespace

extern "C" {

lbpc_status lbpc_set_tiles(lbpc_handle* h, int32_t block_width,
                           int32_t rows) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (!valid_block_width(block_width))
    return fail(h, LBPC_ERR_ARG, "block width must be 64, 128, 256 or 512");
  if (rows < 4) return fail(h, LBPC_ERR_ARG, "rows must be >= 4");
  set_tiles_impl(h, block_width, rows, rows);
  return LBPC_OK;
}

lbpc_status lbpc_steps_per_launch(const lbpc_handle* h, int32_t* steps) {
  if (!h || !steps) return fail(nullptr, LBPC_ERR_ARG, "NULL argument");
  *steps = h->two_step ? 2 : 1;
  return LBPC_OK;
}

lbpc_status lbpc_get_tiles(const lbpc_handle* h, int32_t* block_width,
                           int32_t* rows, int32_t* rows_edge) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (block_width) *block_width = h->base.bw;
  if (rows) *rows = h->base.H;
  if (rows_edge) *rows_edge = h->base.He;
  return LBPC_OK;
}

lbpc_status lbpc_autotune(lbpc_handle* h, int32_t steps, int32_t* block_width,
                          int32_t* rows, double* ms_per_step) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (steps < 1) return fail(h, LBPC_ERR_ARG, "steps < 1");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "autotune before init");
  static const int CBW[4] = {64, 128, 256, 512};
  static const int CH[7] = {4, 8, 16, 24, 32, 48, 64};
  // candidates (block width, rows, rows of the x-edge strips): the shape in
  // place, then per block width its default heights and the fixed heights
  std::vector<std::array<int, 3>> cand{{h->base.bw, h->base.H, h->base.He}};
  for (int bw : CBW) {
    int r, re;
    default_rows(h->cfg, h->tiled != 0, h->cus, bw, r, re);
    cand.push_back({bw, r, re});
    for (int r2 : CH)
      if (r2 <= h->cfg.ny) cand.push_back({bw, r2, r2});
  }
  hipEvent_t e0, e1;
  HIP_TRY(h, hipEventCreate(&e0), "event");
  HIP_TRY(h, hipEventCreate(&e1), "event");
  float best = 1e30f;
  std::array<int, 3> pick = cand[0];
  lbpc_status st = LBPC_OK;
  for (size_t k = 0; k < cand.size(); ++k) {
    bool seen = false;
    for (size_t j = 0; j < k; ++j) seen = seen || cand[j] == cand[k];
    if (seen) continue;
    set_tiles_impl(h, cand[k][0], cand[k][1], cand[k][2]);
    st = enqueue_step(h, true);  // warm-up (and uploads)
    if (st != LBPC_OK) break;
    hipError_t e = hipEventRecord(e0, h->stream);
    for (int s = 0; s < steps && st == LBPC_OK; ++s)
      st = enqueue_step(h, true);
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess && st == LBPC_OK) st = hip_fail(h, e, "timing");
    if (st != LBPC_OK) break;
    if (ms < best) {
      best = ms;
      pick = cand[k];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_tiles_impl(h, pick[0], pick[1], pick[2]);
  if (st != LBPC_OK) return st;
  if (block_width) *block_width = pick[0];
  if (rows) *rows = pick[1];
  if (ms_per_step) *ms_per_step = best / steps;
  return LBPC_OK;
}

lbpc_status lbpc_memory_probe(lbpc_handle* h, int32_t launches,
                              double* ms_per_launch) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (launches < 1 || !ms_per_launch)
    return fail(h, LBPC_ERR_ARG, "launches < 1 or output is NULL");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "probe before init");
  if (h->tiled)
    return fail(h, LBPC_ERR_UNSUPPORTED, "memory probe: periodic lattices only");
  // reads the current buffer and the phi history; writes the other buffer
  // (which the next step overwrites) and phi to scratch
  StepParams p = params_now(h);
  // the probe kernel is built for the default block widths only
  if (p.bw != 256 && p.bw != 512)
    return fail(h, LBPC_ERR_UNSUPPORTED,
                "memory probe: 256- or 512-thread tiles only");
  p.phi_out = phi_buf(h, 1 - h->phi_sel);
  hipEvent_t e0, e1;
  HIP_TRY(h, hipEventCreate(&e0), "event");
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(h, e, "event");
  }
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = lbpc::launch_step_probe(p, h->cfg.precision, h->stream);
  if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
  for (int k = 0; k < launches && e == hipSuccess; ++k)
    e = lbpc::launch_step_probe(p, h->cfg.precision, h->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(h, e, "memory probe");
  *ms_per_launch = ms / launches;
  return LBPC_OK;
}

lbpc_status lbpc_get_rho_u_T(lbpc_handle* h, double* rho, double* ux,
                             double* uy, double* T) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "get before init");
  const size_t N = (size_t)h->cfg.nx * h->cfg.ny;
  double* scr = static_cast<double*>(at(h, h->L.scratch));
  StepParams p = params_now(h);
  double* dst[4] = {rho, ux, uy, T};
  {
    const char* what = "";
    hipError_t e = stage_fields(p, h->cfg.precision, scr, h->L.stage, dst,
                                  h->stream, &what);
    if (e != hipSuccess) return hip_fail(h, e, what);
  }
  if (flagged(h)) return fail(h, LBPC_ERR_NUMERIC, BAD_STATE);
  for (int k = 0; k < 4; ++k)
    if (dst[k])
      for (size_t i = 0; i < N; ++i)
        if (!std::isfinite(dst[k][i]))
          return fail(h, LBPC_ERR_NUMERIC, "non-finite field value");
  return LBPC_OK;
}

lbpc_status lbpc_get_diag(lbpc_handle* h, lbpc_diag* out) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (!out) return fail(h, LBPC_ERR_ARG, "out is NULL");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "diag before init");
  lbpc_status st = enqueue_diag(h, true, ws_part(h), ws_dout(h));
  if (st != LBPC_OK) return st;
  HIP_TRY(h, hipEventSynchronize(h->diag_ev), "synchronise");
  fill_diag(out, h->res_host, h->cfg.cv, h->step, flagged(h));
  if (out->nonfinite) return fail(h, LBPC_ERR_NUMERIC, BAD_STATE);
  return LBPC_OK;
}

lbpc_status lbpc_get_diag_noalloc(lbpc_handle* h, lbpc_diag* out) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (!out) return fail(h, LBPC_ERR_ARG, "out is NULL");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "diag before init");
  if (tile_count(h) > NOALLOC_RECORDS)
    return fail(h, LBPC_ERR_UNSUPPORTED,
                "more tiles than the static diagnostic scratch holds "
                "(65536): use lbpc_get_diag or taller tiles");
  double* base = nullptr;
  lbpc_status st = scratch_for_device(h, &base);
  if (st != LBPC_OK) return st;
  st = enqueue_diag(h, true, base, base + (size_t)NOALLOC_RECORDS * 8);
  if (st != LBPC_OK) return st;
  HIP_TRY(h, hipEventSynchronize(h->diag_ev), "synchronise");
  fill_diag(out, h->res_host, h->cfg.cv, h->step, flagged(h));
  if (out->nonfinite) return fail(h, LBPC_ERR_NUMERIC, BAD_STATE);
  return LBPC_OK;
}

lbpc_status lbpc_state_bytes(const lbpc_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(nullptr, LBPC_ERR_ARG, "NULL argument");
  const size_t N = (size_t)h->cfg.nx * h->cfg.ny;
  *bytes = (18 + hist_arrays(h->cfg)) * N * sizeof(double) +
           3 * sizeof(int64_t);
  return LBPC_OK;
}

lbpc_status lbpc_save_state(lbpc_handle* h, void* host, size_t bytes) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  if (!h->initialised) return fail(h, LBPC_ERR_STATE, "save before init");
  size_t need;
  lbpc_state_bytes(h, &need);
  if (!host || bytes < need) return fail(h, LBPC_ERR_ARG, "buffer too small");
  HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
  if (flagged(h)) return fail(h, LBPC_ERR_NUMERIC, BAD_STATE);
  const size_t N = (size_t)h->cfg.nx * h->cfg.ny;
  double* scr = static_cast<double*>(at(h, h->L.scratch));
  double* dst = static_cast<double*>(host);
  StepParams p = params_now(h);
  const int nh = hist_arrays(h->cfg);
  for (int which = 0; which < 18 + nh; ++which) {
    StepParams q = p;
    if (which >= 18)
      q.phi = static_cast<char*>(p.phi) +
              (which - 18) * N * compute_bytes(h->cfg.precision);
    const char* what = "";
    hipError_t e = stage_state(q, h->cfg.precision, which < 18 ? which : -1,
                               true, scr, h->L.stage, dst + which * N,
                               h->stream, &what);
    if (e != hipSuccess) return hip_fail(h, e, what);
  }
  int64_t meta[3];
  meta[0] = h->phi_valid;
  std::memcpy(&meta[1], &h->rho_ave, sizeof(double));
  meta[2] = h->step;
  std::memcpy(dst + (18 + nh) * N, meta, sizeof(meta));
  return LBPC_OK;
}

lbpc_status lbpc_load_state(lbpc_handle* h, const void* host, size_t bytes) {
  if (!h) return fail(nullptr, LBPC_ERR_ARG, "handle is NULL");
  size_t need;
  lbpc_state_bytes(h, &need);
  if (!host || bytes < need) return fail(h, LBPC_ERR_ARG, "buffer too small");
  const size_t N = (size_t)h->cfg.nx * h->cfg.ny;
  double* scr = static_cast<double*>(at(h, h->L.scratch));
  const double* src = static_cast<const double*>(host);
  drop_graphs(h);
  h->cur = 0;
  h->phi_sel = 0;
  StepParams p = params_now(h);
  const int nh = hist_arrays(h->cfg);
  for (int which = 0; which < 18 + nh; ++which) {
    StepParams q = p;
    if (which >= 18)
      q.phi = static_cast<char*>(p.phi) +
              (which - 18) * N * compute_bytes(h->cfg.precision);
    const char* what = "";
    hipError_t e = stage_state(q, h->cfg.precision, which < 18 ? which : -1,
                               false, scr, h->L.stage,
                               const_cast<double*>(src + which * N),
                               h->stream, &what);
    if (e != hipSuccess) return hip_fail(h, e, what);
  }
  int64_t meta[3];
  std::memcpy(meta, src + (18 + nh) * N, sizeof(meta));
  h->phi_valid = meta[0] != 0;
  std::memcpy(&h->rho_ave, &meta[1], sizeof(double));
  h->step = meta[2];
  {
    lbpc_status st = reset_flag(h);
    if (st != LBPC_OK) return st;
  }
  h->fresh = 1;
  h->initialised = 1;
  h->table_fresh = -1;
  return LBPC_OK;
}

void lbpc_destroy(lbpc_handle* h) {
  if (!h) return;
  if (h->initialised) (void)hipStreamSynchronize(h->stream);
  drop_graphs(h);
  if (h->diag_ev) (void)hipEventDestroy(h->diag_ev);
  if (h->bad_host) (void)hipHostFree(h->bad_host);
  delete h;
}

const char* lbpc_last_error(const lbpc_handle* h) {
  return h ? h->err.c_str() : g_err.c_str();
}

}  // extern "C"
