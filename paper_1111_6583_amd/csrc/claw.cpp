// claw.cpp -- host side of libclaw: the C ABI declared in include/claw.h.
//
// Validates configurations, carves the caller's workspace, launches the
// gfx950 kernels, runs the step controller (host or device resident),
// captures HIP graphs, manages batches and the tiling autotuner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/claw.h"
#include "claw_internal.h"

namespace claw {
hipError_t launch_classic2d(int riemann, int prec, int lim, int trans, int nblocks, hipStream_t st,
                            const GridDesc* d_grids, const int* d_bstart, int ngrids, int mode,
                            double dt, int src);
hipError_t launch_classic1d(int riemann, int fp32, int nblocks, hipStream_t st,
                            const GridDesc* d_grids, int mode, double dt, int src);
hipError_t launch_classic1d_run(int riemann, int fp32, int m, int nx, hipStream_t st,
                                const GridDesc* d_grids);
size_t classic1d_run_smem(int m, int nx, int fp32);
hipError_t launch_sharp_stage(int ndim, int riemann, int prec, int weno_r, int kind, int nblocks,
                              hipStream_t st, const GridDesc* d_grids, int mode, double dt,
                              const StageArgs& sa);
hipError_t launch_sweep(int dir, int riemann, int fp32, int lim, hipStream_t st,
                        const GridDesc* d_grid, int mode, double dt, int src, const SweepArgs& sa);
hipError_t launch_load_state(int fp32, void* q, void* c, const double* in, size_t n,
                             hipStream_t st);
hipError_t launch_store_state(int fp32, double* out, const void* q, const void* c, size_t n,
                              hipStream_t st);
hipError_t launch_convert(int fp32, void* dst, const double* src, size_t n, hipStream_t st);
hipError_t launch_cell_speed(int ndim, int riemann, int fp32, const GridDesc* g, int src, size_t n,
                             unsigned long long* out, hipStream_t st);
int totals_blocks();
hipError_t launch_totals(int fp32, const void* q, const void* c, int m, size_t n, double cell,
                         double* part, double* out, hipStream_t st);
hipError_t launch_static_setup(const GridDesc& g, GridDesc* d_grid, Ctrl* d_ctrl,
                               SpeedSlot* d_slots, hipStream_t st);
hipError_t launch_static_courant(const Ctrl* d_ctrl, double dt, double* out, hipStream_t st);
}  // namespace claw

using namespace claw;

#define HIPCHK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return CLAW_E_DEVICE; \
  } while (0)

namespace {

constexpr size_t kAlign = 256;
constexpr int kMarchLanesClassic = kLanes - 4;   // useful columns per classic strip
// useful columns per SharpClaw strip: r halo lanes a side for WENO order 2r-1
int march_lanes_sharp(int weno_r) { return kLanes - 2 * weno_r; }
constexpr size_t kRun1dSmemMax = 64 * 1024;      // LDS budget of the 1D whole-run kernel

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int num_eqn_of(const claw_config& c) {
  switch (c.riemann) {
    case CLAW_RP_ADVECTION: return 1;
    case CLAW_RP_SW_ROE: return c.ndim == 1 ? 2 : 3;
    case CLAW_RP_EULER_HLLE: return c.ndim == 1 ? 3 : 4;
    case CLAW_RP_ELASTIC_VC: return 5;
    case CLAW_RP_EULER_ROE: return (c.ndim == 1 ? 3 : 4) + (c.tracer ? 1 : 0);
    case CLAW_RP_PSYSTEM: return c.ndim == 1 ? 2 : 3;
  }
  return 0;
}
// Kernel variant of the Riemann solver (the tracer is a separate instance).
int kernel_riemann(const claw_config& c) {
  if (c.riemann == CLAW_RP_PSYSTEM) return 7;
  return c.riemann == CLAW_RP_EULER_ROE && c.tracer ? 6 : c.riemann;
}
int num_aux_of(const claw_config& c) {
  return c.riemann == CLAW_RP_ELASTIC_VC ? 3 : (c.riemann == CLAW_RP_PSYSTEM ? 2 : 0);
}

bool valid_bc(int b) { return b >= CLAW_BC_EXTRAP && b <= CLAW_BC_DIRICHLET; }

int validate(const claw_config* c) {
  if (!c) return CLAW_E_INVAL;
  if (c->ndim != 1 && c->ndim != 2) return CLAW_E_INVAL;
  if (c->num_cells[0] < 4 || (c->ndim == 2 && c->num_cells[1] < 4)) return CLAW_E_INVAL;
  if ((double)c->num_cells[0] * (c->ndim == 2 ? c->num_cells[1] : 1) > 2.0e9) return CLAW_E_INVAL;
  for (int d = 0; d < c->ndim; ++d) {
    if (!(c->upper[d] > c->lower[d])) return CLAW_E_INVAL;
    if (!valid_bc(c->bc_lower[d]) || !valid_bc(c->bc_upper[d])) return CLAW_E_INVAL;
    if ((c->bc_lower[d] == CLAW_BC_PERIODIC) != (c->bc_upper[d] == CLAW_BC_PERIODIC))
      return CLAW_E_INVAL;
  }
  if (c->precision != CLAW_FP64 && c->precision != CLAW_FP32_KAHAN && c->precision != CLAW_FP32)
    return CLAW_E_INVAL;
  if (c->precision == CLAW_FP32) {
    // plain FP32 kernels exist for the two workloads its comparison is made on
    const bool sw = c->scheme == CLAW_CLASSIC && c->riemann == CLAW_RP_SW_ROE && c->ndim == 2 &&
                    c->dimensional_split == CLAW_SPLIT_NONE;
    const bool eu = c->scheme == CLAW_SHARPCLAW && c->riemann == CLAW_RP_EULER_HLLE &&
                    c->ndim == 2 && (c->weno_order == 0 || c->weno_order == 5);
    if (!sw && !eu) return CLAW_E_INVAL;
  }
  if (c->tracer != 0 && (c->tracer != 1 || c->riemann != CLAW_RP_EULER_ROE)) return CLAW_E_INVAL;
  if (c->source != CLAW_SOURCE_NONE &&
      (c->source != CLAW_SOURCE_AXISYMMETRIC || c->riemann != CLAW_RP_EULER_ROE || c->ndim != 2 ||
       !(c->lower[1] >= 0.0)))
    return CLAW_E_INVAL;
  if (c->scheme == CLAW_CLASSIC) {
    if (c->riemann == CLAW_RP_EULER_HLLE) return CLAW_E_INVAL;
    if (c->riemann == CLAW_RP_ELASTIC_VC && c->ndim != 2) return CLAW_E_INVAL;
    if (c->riemann < 1 || c->riemann > 5) return CLAW_E_INVAL;
    if (c->limiter < CLAW_LIM_NONE || c->limiter > CLAW_LIM_MC) return CLAW_E_INVAL;
    if (c->transverse < 0 || c->transverse > 2) return CLAW_E_INVAL;
    if (c->dimensional_split < CLAW_SPLIT_NONE || c->dimensional_split > CLAW_SPLIT_STRANG)
      return CLAW_E_INVAL;
    if (c->dimensional_split != CLAW_SPLIT_NONE && c->ndim != 2) return CLAW_E_INVAL;
  } else if (c->scheme == CLAW_SHARPCLAW) {
    if (c->riemann != CLAW_RP_ADVECTION && c->riemann != CLAW_RP_EULER_HLLE &&
        c->riemann != CLAW_RP_PSYSTEM)
      return CLAW_E_INVAL;
    if (c->time_integrator != 0 && c->time_integrator != CLAW_SSP33 &&
        c->time_integrator != CLAW_SSP104)
      return CLAW_E_INVAL;
    if (c->weno_order != 0 && (c->weno_order < 5 || c->weno_order > 17 || c->weno_order % 2 == 0))
      return CLAW_E_INVAL;
    // the r = (order + 1) / 2 ghost layers map to interior cells (wrap or mirror once)
    const int r = c->weno_order == 0 ? 3 : (c->weno_order + 1) / 2;
    if (c->num_cells[0] < r || (c->ndim == 2 && c->num_cells[1] < r)) return CLAW_E_INVAL;
    if (c->dimensional_split != CLAW_SPLIT_NONE) return CLAW_E_INVAL;
  } else {
    return CLAW_E_INVAL;
  }
  if (!(c->cfl_max > 0.0) || !(c->cfl_desired > 0.0)) return CLAW_E_INVAL;
  return CLAW_OK;
}

// Process-wide tiling cache: (4 scheme + split mode, riemann, precision, WENO order, nx, ny)
// -> (row segments, seg_rows_x).
std::mutex g_tune_mu;
struct Tiling {
  int segs, seg_rows_x, order;
};
std::map<std::tuple<int, int, int, int, int, int>, Tiling> g_tune;

int weno_r_of(const claw_config& c) { return c.weno_order >= 7 ? (c.weno_order + 1) / 2 : 3; }
bool ssp104(const claw_config& c) { return c.time_integrator == CLAW_SSP104; }
bool split(const claw_config& c) {
  return c.scheme == CLAW_CLASSIC && c.dimensional_split != CLAW_SPLIT_NONE;
}
bool strang(const claw_config& c) { return split(c) && c.dimensional_split == CLAW_SPLIT_STRANG; }

int default_segs(int ny) { return (ny + 15) / 16; }
// x sweeps of a split step: rows are independent, so short row segments buy
// more wavefronts at no extra work
int default_seg_rows_x(int ny) { return std::min(ny, 4); }

}  // namespace

struct claw_solver {
  claw_config cfg;
  int device = 0;
  int m = 0, na = 0, fp32 = 0;   // fp32: float32 storage (both FP32 precisions)
  int pk = 0;                    // kernel precision: 0 FP64, 1 FP32 + Kahan, 2 plain FP32
  int kr = 0;                    // kernel variant of the Riemann solver
  void* split_c[2] = {nullptr, nullptr};   // compensations of the split step's intermediates
  int seg_rows_x = 0;            // rows per workgroup of the split step's x sweeps
  size_t ncell = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // device pointers carved from the workspace
  GridDesc* d_grid = nullptr;
  Ctrl* d_ctrl = nullptr;
  double* d_part = nullptr;
  double* d_tot = nullptr;
  unsigned long long* d_speed = nullptr;
  GridDesc hg{};                 // host copy of the grid descriptor
  Ctrl* h_ctrl = nullptr;        // pinned staging
  bool state_set = false, aux_set = false;
  int src = 0;                   // buffer holding Q^n (classic)
  claw_stats clock{};
  // graphs
  hipGraphExec_t graph = nullptr;
  int graph_k = 0;
};

// Launch groups of a batch that may be in flight at once (claw_batch_launch
// without claw_batch_wait).
constexpr int kBatchInFlight = 2;

struct claw_batch {
  int max_grids = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  GridDesc* d_grids = nullptr;
  int* d_bstart = nullptr;
  Ctrl* d_ctrls = nullptr;        // gathered copies of member controllers (one set per group)
  std::vector<claw_t> members;
  std::vector<int> bstart;
  bool dirty = true;
  int riemann = 0, fp32 = 0, limiter = 0, transverse = 0;   // fp32: the members' kernel precision
  hipGraphExec_t graph = nullptr;
  int graph_k = 0;
  // groups in flight: their member lists, pinned controller copies, events
  Ctrl* h_ctrls[kBatchInFlight] = {nullptr, nullptr};
  std::vector<claw_t> snap[kBatchInFlight];
  hipEvent_t ev[kBatchInFlight] = {nullptr, nullptr};
  long long launched = 0, waited = 0;   // groups launched / completed (waited for)
  // the view: member controllers as of the last completed group
  const Ctrl* view = nullptr;
  const std::vector<claw_t>* view_members = nullptr;
  // pinned upload buffers of the grid tables, one per group slot (a slot's
  // buffer is rewritten only after the group that used it has completed)
  GridDesc* h_grids[kBatchInFlight] = {nullptr, nullptr};
  int* h_bstart[kBatchInFlight] = {nullptr, nullptr};
  // graphs replaced while groups that launch them may still be in flight,
  // with the number of groups launched when they were replaced
  std::vector<std::pair<hipGraphExec_t, long long>> retired;
};

namespace {

// Byte offsets of every array of a handle's workspace (slot -> offset, -1 if
// absent).  caller_state: the layout of claw_step_static's scratch, where an
// FP64 state and aux stay in the caller's buffers and the totals and a-priori
// speed are not needed.
size_t layout(const claw_config& c, size_t off[16], bool caller_state = false) {
  const int m = num_eqn_of(c), na = num_aux_of(c);
  const size_t N = (size_t)c.num_cells[0] * (c.ndim == 2 ? c.num_cells[1] : 1);
  const size_t rb = c.precision == CLAW_FP64 ? 8 : 4;
  const bool fp32 = c.precision != CLAW_FP64;
  const bool kahan = c.precision == CLAW_FP32_KAHAN;
  const bool classic = c.scheme == CLAW_CLASSIC;
  size_t p = 0;
  auto take = [&](int slot, size_t bytes) {
    off[slot] = p;
    p += align_up(bytes);
  };
  for (int s = 0; s < 16; ++s) off[s] = (size_t)-1;
  const bool own_state = !(caller_state && !fp32);          // FP64 static step: caller's buffers
  take(0, sizeof(GridDesc));
  take(1, sizeof(Ctrl));
  if (!caller_state) {
    take(2, (size_t)m * totals_blocks() * sizeof(double)); // totals partials
    take(3, 8 * sizeof(double));                           // totals out
    take(4, sizeof(unsigned long long));                   // a-priori speed
  }
  take(15, kSpeedSlots * sizeof(SpeedSlot));               // launch-end Courant reduction
  if (own_state) {
    take(5, m * N * rb);                                   // q[0]
    if (classic) take(6, m * N * rb);                      // q[1]
  }
  if (kahan) {
    take(7, m * N * rb);                                   // c[0]
    if (classic) take(8, m * N * rb);                      // c[1]
  }
  if (!classic) {
    take(9, m * N * rb);                                   // s1
    take(10, m * N * rb);                                  // s2
    if (ssp104(c)) take(12, m * N * rb);                   // s3
  } else if (split(c)) {
    take(9, m * N * rb);                                   // state after the first sweep
    if (kahan) take(13, m * N * rb);                       //   and its compensation
    if (strang(c)) {
      take(10, m * N * rb);                                // state after the second sweep
      if (kahan) take(14, m * N * rb);
    }
  }
  if (na && own_state) take(11, na * N * rb);              // aux
  return p;
}

std::tuple<int, int, int, int, int, int> tune_key(claw_t h) {
  return std::make_tuple(h->cfg.scheme * 4 + h->cfg.dimensional_split, h->kr, h->cfg.precision,
                         h->cfg.weno_order, h->cfg.num_cells[0],
                         h->cfg.ndim == 2 ? h->cfg.num_cells[1] : 1);
}

Tiling tiling_for(claw_t h) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(h));
  const int ny = h->cfg.ndim == 2 ? h->cfg.num_cells[1] : 1;
  return it != g_tune.end() ? it->second : Tiling{default_segs(ny), default_seg_rows_x(ny), 0};
}

int segs_from_rows(int ny, int seg_rows) {
  seg_rows = std::max(1, std::min(seg_rows, ny));
  return (ny + seg_rows - 1) / seg_rows;
}

// Tile the 2D kernels into column strips x `segs` row segments (rows split
// as evenly as possible).
void set_tiling(claw_t h, int segs) {
  GridDesc& g = h->hg;
  const int lanes =
      h->cfg.scheme == CLAW_CLASSIC ? kMarchLanesClassic : march_lanes_sharp(weno_r_of(h->cfg));
  g.strips = (g.nx + lanes - 1) / lanes;
  if (h->cfg.ndim == 2) {
    g.segs = std::max(1, std::min(segs, g.ny));
    g.seg_rows = (g.ny + g.segs - 1) / g.segs;
  } else {
    g.seg_rows = 1;
    g.segs = 1;
  }
  g.nblocks = g.strips * g.segs;
}

int upload_grid(claw_t h) {
  HIPCHK(hipMemcpyAsync(h->d_grid, &h->hg, sizeof(GridDesc), hipMemcpyHostToDevice, h->stream));
  return CLAW_OK;
}

int sync(claw_t h) {
  HIPCHK(hipStreamSynchronize(h->stream));
  return CLAW_OK;
}

int read_ctrl(claw_t h) {
  HIPCHK(hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return CLAW_OK;
}

// The stage sequence of one SharpClaw attempt (see k_sharp.hip):
//   SSPRK(3,3): Q -> S1 = y;  S1 -> S2 = 3/4 Q + 1/4 y;  S2 -> Q = 1/3 Q + 2/3 y.
//   SSPRK(10,4): stages 1-4, 6-9 y = S + dt/6 L(S) alternating S1/S2;
//                stage 5 S3 = Q/25 + 9/25 y, S1 = 3/5 Q + 2/5 y (= 15 S3 - 5 y);
//                stage 10 Q = S3 + 3/5 y.
int sharp_plan(claw_t h, StageArgs* st, int* kind) {
  const GridDesc& g = h->hg;
  void* Q = g.q[0];
  for (int s = 0; s < 10; ++s) std::memset(&st[s], 0, sizeof(StageArgs));
  auto plain = [&](int s, void* in, void* out, double gamma) {
    st[s].in = in;
    st[s].out1 = out;
    st[s].gamma = gamma;
    st[s].b1 = 1.0;
    kind[s] = kStagePlain;
  };
  if (ssp104(h->cfg)) {
    void* S1 = g.s1;
    void* S2 = g.s2;
    void* S3 = g.s3;
    const double g6 = 1.0 / 6.0;
    plain(0, Q, S1, g6);
    plain(1, S1, S2, g6);
    plain(2, S2, S1, g6);
    plain(3, S1, S2, g6);
    st[4].in = S2;
    st[4].out1 = S3;
    st[4].out2 = S1;
    st[4].p1 = Q;
    st[4].gamma = g6;
    st[4].a1 = 1.0 / 25.0;
    st[4].b1 = 9.0 / 25.0;
    st[4].a2 = 3.0 / 5.0;
    st[4].b2 = 2.0 / 5.0;
    kind[4] = kStageCombine;
    plain(5, S1, S2, g6);
    plain(6, S2, S1, g6);
    plain(7, S1, S2, g6);
    plain(8, S2, S1, g6);
    st[9].in = S1;
    st[9].out1 = Q;
    st[9].p1 = S3;
    st[9].gamma = g6;
    st[9].a1 = 1.0;
    st[9].b1 = 3.0 / 5.0;
    st[9].w = (1.0 - 3.0 / 5.0) / 1.0;
    kind[9] = kStageFinal;
    st[0].first = 1;
    return 10;
  }
  plain(0, Q, g.s1, 1.0);
  st[0].first = 1;
  st[1].in = g.s1;
  st[1].out1 = g.s2;
  st[1].p1 = Q;
  st[1].gamma = 1.0;
  st[1].a1 = 0.75;
  st[1].b1 = 0.25;
  kind[1] = kStageCombine;
  st[2].in = g.s2;
  st[2].out1 = Q;
  st[2].p1 = Q;
  st[2].p1_is_q = 1;
  st[2].gamma = 1.0;
  st[2].a1 = 1.0 / 3.0;
  st[2].b1 = 2.0 / 3.0;
  st[2].w = 1.0;
  kind[2] = kStageFinal;
  return 3;
}

// Launch SharpClaw stages [from, to) of one attempt.
int launch_sharp_stages(claw_t h, int from, int to, int mode, double dt) {
  StageArgs st[10];
  int kind[10];
  const int n = sharp_plan(h, st, kind);
  for (int s = from; s < std::min(to, n); ++s)
    HIPCHK(launch_sharp_stage(h->cfg.ndim, h->kr, h->pk, h->hg.weno_r, kind[s],
                              h->hg.nblocks, h->stream, h->d_grid, mode, dt, st[s]));
  return CLAW_OK;
}

// The sweeps of one dimensionally split step (see k_split.hip):
//   Godunov: x over dt  Q^n -> W1;  y over dt  W1 -> Q^{n+1}
//   Strang:  x over dt/2  Q^n -> W1;  y over dt  W1 -> W2;  x over dt/2  W2 -> Q^{n+1}
// Q^n is never overwritten, so a rejected step leaves it intact.
int launch_split(claw_t h, int mode, double dt) {
  const GridDesc& g = h->hg;
  const int segs_y = g.segs;
  const int segs_x = segs_from_rows(g.ny, h->seg_rows_x > 0 ? h->seg_rows_x : g.seg_rows);
  int index = 0;
  auto sweep = [&](int dir, const void* in, const void* cin, void* out, void* cout, double frac,
                   int fin) -> int {
    SweepArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.in = in;
    sa.cin = cin;
    sa.out = out;
    sa.cout = cout;
    sa.frac = frac;
    sa.index = index++;
    sa.final_sweep = fin;
    sa.strips = dir == 0 ? (g.nx + kMarchLanesClassic - 1) / kMarchLanesClassic
                         : (g.nx + kLanes - 1) / kLanes;
    sa.segs = dir == 0 ? segs_x : segs_y;
    sa.nblocks = sa.strips * sa.segs;
    HIPCHK(launch_sweep(dir, h->kr, h->fp32, g.limiter, h->stream, h->d_grid, mode, dt, h->src,
                        sa));
    return CLAW_OK;
  };
  void* w1 = g.s1;
  void* c1 = h->split_c[0];
  int rc;
  if (strang(h->cfg)) {
    void* w2 = g.s2;
    void* c2 = h->split_c[1];
    if ((rc = sweep(0, nullptr, nullptr, w1, c1, 0.5, 0))) return rc;
    if ((rc = sweep(1, w1, c1, w2, c2, 1.0, 0))) return rc;
    return sweep(0, w2, c2, nullptr, nullptr, 0.5, 1);
  }
  if ((rc = sweep(0, nullptr, nullptr, w1, c1, 1.0, 0))) return rc;
  return sweep(1, w1, c1, nullptr, nullptr, 1.0, 1);
}

// One attempt's kernels in host-dt mode (classic: one kernel; SharpClaw: the
// first stage only when `stage1_only`).
int launch_attempt_host(claw_t h, double dt, bool stage1_only) {
  const GridDesc& g = h->hg;
  if (split(h->cfg)) return launch_split(h, kHostDt, dt);
  if (h->cfg.scheme == CLAW_CLASSIC) {
    if (h->cfg.ndim == 2)
      HIPCHK(launch_classic2d(h->kr, h->pk, g.limiter, g.transverse, g.nblocks, h->stream, h->d_grid, nullptr, 1,
                              kHostDt, dt, h->src));
    else
      HIPCHK(launch_classic1d(h->kr, h->fp32, g.nblocks, h->stream, h->d_grid, kHostDt, dt,
                              h->src));
  } else {
    return launch_sharp_stages(h, 0, stage1_only ? 1 : 10, kHostDt, dt);
  }
  return CLAW_OK;
}

int sharp_finish_host(claw_t h, double dt) { return launch_sharp_stages(h, 1, 10, kHostDt, dt); }

// One attempt in device-controller mode (what a graph node sequence holds).
int launch_attempt_device(claw_t h) {
  const GridDesc& g = h->hg;
  if (split(h->cfg)) return launch_split(h, kDeviceCtrl, 0.0);
  if (h->cfg.scheme == CLAW_CLASSIC) {
    if (h->cfg.ndim == 2)
      HIPCHK(launch_classic2d(h->kr, h->pk, g.limiter, g.transverse, g.nblocks, h->stream, h->d_grid, nullptr, 1,
                              kDeviceCtrl, 0.0, 0));
    else
      HIPCHK(launch_classic1d(h->kr, h->fp32, g.nblocks, h->stream, h->d_grid, kDeviceCtrl,
                              0.0, 0));
  } else {
    return launch_sharp_stages(h, 0, 10, kDeviceCtrl, 0.0);
  }
  return CLAW_OK;
}

// A-priori first dt: cfl_desired / max cell speed.
int apriori_dt(claw_t h, double* dt) {
  HIPCHK(hipMemsetAsync(h->d_speed, 0, sizeof(unsigned long long), h->stream));
  HIPCHK(launch_cell_speed(h->cfg.ndim, h->kr, h->fp32, h->d_grid, h->src, h->ncell,
                           h->d_speed, h->stream));
  unsigned long long bits = 0;
  HIPCHK(hipMemcpyAsync(&bits, h->d_speed, sizeof(bits), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double s;
  std::memcpy(&s, &bits, sizeof(s));
  const double dtmax = h->cfg.dt_max > 0.0 ? h->cfg.dt_max : std::numeric_limits<double>::infinity();
  *dt = s > 0.0 ? std::min(dtmax, h->cfg.cfl_desired / s) : dtmax;
  if (!std::isfinite(*dt)) return CLAW_E_NONPHYSICAL;
  return CLAW_OK;
}

int first_dt(claw_t h, double* dt) {
  if (h->clock.dt_next > 0.0) {
    *dt = h->clock.dt_next;
    return CLAW_OK;
  }
  if (h->cfg.dt_initial > 0.0) {
    *dt = h->cfg.dt_initial;
    return CLAW_OK;
  }
  return apriori_dt(h, dt);
}

void clock_out(claw_t h, claw_stats* st) {
  if (st) *st = h->clock;
}

void* buf(claw_t h, const size_t off[16], int slot, char* base) {
  return off[slot] == (size_t)-1 ? nullptr : base + off[slot];
}

// Fill a controller record for a device-resident advance to t_end.
void prepare_ctrl(claw_t h, Ctrl& c, double t_end, double dt, long long max_attempts) {
  std::memset(&c, 0, sizeof(c));
  c.src = h->src;
  c.t = h->clock.t;
  c.t_end = t_end;
  c.dt = dt;
  c.cfl_desired = h->cfg.cfl_desired;
  c.cfl_max = h->cfg.cfl_max;
  c.dt_max = h->cfg.dt_max > 0.0 ? h->cfg.dt_max : std::numeric_limits<double>::infinity();
  c.max_attempts = max_attempts > 0 ? max_attempts : 0;
  c.active = c.t < t_end ? 1 : 0;
  c.clipped = c.t + dt >= t_end;
  c.dt_try = c.clipped ? t_end - c.t : dt;
  c.max_courant = h->clock.max_courant;
}

void absorb_ctrl(claw_t h, const Ctrl& c) {
  h->src = c.src;
  h->clock.t = c.t;
  h->clock.dt_next = c.dt;
  h->clock.accepted += c.accepted;
  h->clock.rejected += c.rejected;
  h->clock.max_courant = c.max_courant;
}

// Defaults of optional configuration fields filled in.
claw_config normalised(const claw_config& c) {
  claw_config n = c;
  if (n.weno_eps <= 0.0) n.weno_eps = 1e-6;
  if (n.time_integrator == 0) n.time_integrator = CLAW_SSP33;
  if (n.weno_order == 0) n.weno_order = 5;
  return n;
}

// Everything of a handle that follows from its configuration and its
// workspace: counts, the host copy of the grid descriptor, device pointers
// carved from `base` at the offsets `off`, and the tiling.
void fill_handle(claw_t h, const size_t off[16], char* base) {
  const claw_config* cfg = &h->cfg;
  h->m = num_eqn_of(*cfg);
  h->na = num_aux_of(*cfg);
  h->kr = kernel_riemann(*cfg);
  h->fp32 = cfg->precision != CLAW_FP64;
  h->pk = cfg->precision == CLAW_FP64 ? 0 : (cfg->precision == CLAW_FP32_KAHAN ? 1 : 2);
  h->ncell = (size_t)cfg->num_cells[0] * (cfg->ndim == 2 ? cfg->num_cells[1] : 1);
  h->d_grid = (GridDesc*)buf(h, off, 0, base);
  h->d_ctrl = (Ctrl*)buf(h, off, 1, base);
  h->d_part = (double*)buf(h, off, 2, base);
  h->d_tot = (double*)buf(h, off, 3, base);
  h->d_speed = (unsigned long long*)buf(h, off, 4, base);
  GridDesc& g = h->hg;
  std::memset(&g, 0, sizeof(g));
  g.nx = cfg->num_cells[0];
  g.ny = cfg->ndim == 2 ? cfg->num_cells[1] : 1;
  g.bc[0] = cfg->bc_lower[0];
  g.bc[1] = cfg->bc_upper[0];
  g.bc[2] = cfg->ndim == 2 ? cfg->bc_lower[1] : CLAW_BC_EXTRAP;
  g.bc[3] = cfg->ndim == 2 ? cfg->bc_upper[1] : CLAW_BC_EXTRAP;
  g.limiter = cfg->limiter;
  g.transverse = cfg->ndim == 2 ? cfg->transverse : 0;
  g.efix = cfg->entropy_fix;
  g.scheme = cfg->scheme;
  g.dx = (cfg->upper[0] - cfg->lower[0]) / g.nx;
  g.dy = cfg->ndim == 2 ? (cfg->upper[1] - cfg->lower[1]) / g.ny : 1.0;
  g.ylo = cfg->ndim == 2 ? cfg->lower[1] : 0.0;
  g.source = cfg->source;
  g.weno_eps = h->cfg.weno_eps;
  g.cfl_max = cfg->cfl_max;
  std::memcpy(g.bcstate, cfg->bc_state, sizeof(g.bcstate));
  std::memcpy(g.pd, cfg->problem_data, sizeof(g.pd));
  g.q[0] = buf(h, off, 5, base);
  g.q[1] = buf(h, off, 6, base);
  g.c[0] = buf(h, off, 7, base);
  g.c[1] = buf(h, off, 8, base);
  g.s1 = buf(h, off, 9, base);
  g.s2 = buf(h, off, 10, base);
  g.s3 = buf(h, off, 12, base);
  g.weno_r = weno_r_of(h->cfg);
  g.aux = buf(h, off, 11, base);
  g.ctrl = h->d_ctrl;
  g.slots = (SpeedSlot*)buf(h, off, 15, base);
  h->split_c[0] = buf(h, off, 13, base);
  h->split_c[1] = buf(h, off, 14, base);
  {
    const Tiling t = tiling_for(h);
    set_tiling(h, t.segs);
    h->seg_rows_x = t.seg_rows_x;
    h->hg.order = h->cfg.ndim == 2 ? t.order : 0;
  }
}

}  // namespace

extern "C" {

const char* claw_strerror(int s) {
  switch (s) {
    case CLAW_OK: return "ok";
    case CLAW_E_INVAL: return "invalid argument or unsupported configuration";
    case CLAW_E_NOMEM: return "workspace smaller than claw_workspace_bytes()";
    case CLAW_E_DEVICE: return "HIP runtime call failed";
    case CLAW_E_REJECTED: return "step rejected: Courant number above cfl_max";
    case CLAW_E_NONPHYSICAL: return "non-finite Courant number (NaN or Inf in the state)";
    case CLAW_E_BUDGET: return "no free batch slot";
    case CLAW_E_STATE: return "call order: state not set or handle in use";
    case CLAW_E_MAXSTEPS: return "max_steps attempts did not reach t_end";
    case CLAW_E_TOOBIG:
      return "grid needs more than the CLAW_STATIC_SCRATCH_BYTES of claw_step_static";
  }
  return "unknown status";
}

int claw_num_eqn(const claw_config* cfg) { return validate(cfg) ? 0 : num_eqn_of(*cfg); }
int claw_num_aux(const claw_config* cfg) { return validate(cfg) ? 0 : num_aux_of(*cfg); }

size_t claw_workspace_bytes(const claw_config* cfg) {
  if (validate(cfg) != CLAW_OK) return 0;
  size_t off[16];
  return layout(*cfg, off);
}

int claw_create(const claw_config* cfg, void* d_ws, size_t ws_bytes, void* hip_stream,
                claw_t* out) {
  if (!out) return CLAW_E_INVAL;
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0) return CLAW_E_INVAL;
  size_t off[16];
  const size_t need = layout(*cfg, off);
  if (ws_bytes < need) return CLAW_E_NOMEM;
  claw_t h = new (std::nothrow) claw_solver();
  if (!h) return CLAW_E_NOMEM;
  h->cfg = normalised(*cfg);
  if (hipGetDevice(&h->device) != hipSuccess) { delete h; return CLAW_E_DEVICE; }
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&h->stream) != hipSuccess) { delete h; return CLAW_E_DEVICE; }
    h->own_stream = true;
  }
  if (hipHostMalloc((void**)&h->h_ctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) {
    if (h->own_stream) hipStreamDestroy(h->stream);
    delete h;
    return CLAW_E_DEVICE;
  }
  fill_handle(h, off, (char*)d_ws);
  Ctrl c0;
  std::memset(&c0, 0, sizeof(c0));
  rc = CLAW_OK;
  if (hipMemcpyAsync(h->d_ctrl, &c0, sizeof(Ctrl), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemsetAsync(h->hg.slots, 0, kSpeedSlots * sizeof(SpeedSlot), h->stream) != hipSuccess ||
      upload_grid(h) != CLAW_OK || hipStreamSynchronize(h->stream) != hipSuccess)
    rc = CLAW_E_DEVICE;
  if (rc) {
    claw_destroy(h);
    return rc;
  }
  *out = h;
  return CLAW_OK;
}

int claw_destroy(claw_t h) {
  if (!h) return CLAW_E_INVAL;
  hipSetDevice(h->device);
  if (h->stream) hipStreamSynchronize(h->stream);
  if (h->graph) hipGraphExecDestroy(h->graph);
  if (h->h_ctrl) hipHostFree(h->h_ctrl);
  if (h->own_stream) hipStreamDestroy(h->stream);
  delete h;
  return CLAW_OK;
}

int claw_set_state(claw_t h, const double* q, int on_device) {
  if (!h || !q) return CLAW_E_INVAL;
  HIPCHK(hipSetDevice(h->device));
  const size_t n = (size_t)h->m * h->ncell;
  void* dq = h->hg.q[h->src];
  void* dc = h->hg.c[h->src];
  if (on_device) {
    HIPCHK(hipStreamSynchronize(0));
    if (!h->fp32)
      HIPCHK(hipMemcpyAsync(dq, q, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    else
      HIPCHK(launch_load_state(1, dq, dc, q, n, h->stream));
  } else if (!h->fp32) {
    HIPCHK(hipMemcpyAsync(dq, q, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  } else {
    std::vector<float> tmp(n);
    for (size_t t = 0; t < n; ++t) tmp[t] = (float)q[t];
    HIPCHK(hipMemcpyAsync(dq, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, h->stream));
    if (dc) HIPCHK(hipMemsetAsync(dc, 0, n * sizeof(float), h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  h->state_set = true;
  return CLAW_OK;
}

int claw_set_aux(claw_t h, const double* aux, int on_device) {
  if (!h || !aux) return CLAW_E_INVAL;
  if (h->na == 0) return CLAW_OK;
  HIPCHK(hipSetDevice(h->device));
  const size_t n = (size_t)h->na * h->ncell;
  void* da = (void*)h->hg.aux;
  if (on_device) {
    HIPCHK(hipStreamSynchronize(0));
    if (!h->fp32)
      HIPCHK(hipMemcpyAsync(da, aux, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    else
      HIPCHK(launch_convert(1, da, aux, n, h->stream));
  } else if (!h->fp32) {
    HIPCHK(hipMemcpyAsync(da, aux, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  } else {
    std::vector<float> tmp(n);
    for (size_t t = 0; t < n; ++t) tmp[t] = (float)aux[t];
    HIPCHK(hipMemcpyAsync(da, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  h->aux_set = true;
  return CLAW_OK;
}

int claw_get_state(claw_t h, double* out, int on_device) {
  if (!h || !out) return CLAW_E_INVAL;
  if (!h->state_set) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(h->device));
  const size_t n = (size_t)h->m * h->ncell;
  const void* dq = h->hg.q[h->src];
  const void* dc = h->hg.c[h->src];
  if (on_device) {
    if (!h->fp32)
      HIPCHK(hipMemcpyAsync(out, dq, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    else
      HIPCHK(launch_store_state(1, out, dq, dc, n, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  } else if (!h->fp32) {
    HIPCHK(hipMemcpyAsync(out, dq, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  } else {
    std::vector<float> tq(n), tc(n, 0.0f);
    HIPCHK(hipMemcpyAsync(tq.data(), dq, n * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    if (dc) HIPCHK(hipMemcpyAsync(tc.data(), dc, n * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (size_t t = 0; t < n; ++t) out[t] = (double)tq[t] - (double)tc[t];
  }
  return CLAW_OK;
}

int claw_step(claw_t h, double dt, double* courant_out) {
  if (!h || !(dt > 0.0)) return CLAW_E_INVAL;
  if (!h->state_set || (h->na && !h->aux_set)) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(h->device));
  int rc = launch_attempt_host(h, dt, false);
  if (rc) return rc;
  if ((rc = read_ctrl(h))) return rc;
  const double C = dt * h->h_ctrl->last_speed;
  if (h->cfg.scheme == CLAW_CLASSIC) h->src ^= 1;
  h->clock.t += dt;
  h->clock.accepted += 1;
  if (courant_out) *courant_out = C;
  if (!std::isfinite(C)) return CLAW_E_NONPHYSICAL;
  h->clock.max_courant = std::max(h->clock.max_courant, C);
  return CLAW_OK;
}

int claw_advance(claw_t h, double t_end, long long max_steps, claw_stats* st) {
  if (!h) return CLAW_E_INVAL;
  if (!h->state_set || (h->na && !h->aux_set)) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(h->device));
  double dt;
  int rc = first_dt(h, &dt);
  if (rc) return rc;
  const double dt_max =
      h->cfg.dt_max > 0.0 ? h->cfg.dt_max : std::numeric_limits<double>::infinity();
  long long attempts = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, h->stream));
  while (h->clock.t < t_end) {
    if (max_steps > 0 && attempts >= max_steps) { rc = CLAW_E_MAXSTEPS; break; }
    const bool clipped = h->clock.t + dt >= t_end;
    const double dt_try = clipped ? t_end - h->clock.t : dt;
    if ((rc = launch_attempt_host(h, dt_try, true))) break;
    if ((rc = read_ctrl(h))) break;
    const double C = dt_try * h->h_ctrl->last_speed;
    ++attempts;
    if (!std::isfinite(C)) { rc = CLAW_E_NONPHYSICAL; break; }
    if (C <= h->cfg.cfl_max) {
      if (h->cfg.scheme == CLAW_CLASSIC) h->src ^= 1;
      else if ((rc = sharp_finish_host(h, dt_try))) break;
      h->clock.t = clipped ? t_end : h->clock.t + dt_try;
      h->clock.accepted += 1;
      h->clock.max_courant = std::max(h->clock.max_courant, C);
    } else {
      h->clock.rejected += 1;
    }
    dt = C > 0.0 ? std::min(dt_max, dt_try * h->cfg.cfl_desired / C) : dt_max;
  }
  h->clock.dt_next = dt;
  if (hipEventRecord(e1, h->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) h->clock.gpu_ms = ms;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == CLAW_OK && (rc = sync(h))) return rc;
  clock_out(h, st);
  return rc;
}

int claw_advance_graph(claw_t h, double t_end, int k, long long max_steps, claw_stats* st) {
  if (!h || k < 1) return CLAW_E_INVAL;
  if (!h->state_set || (h->na && !h->aux_set)) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(h->device));
  if (!(h->clock.t < t_end)) { clock_out(h, st); return CLAW_OK; }
  double dt;
  int rc = first_dt(h, &dt);
  if (rc) return rc;
  Ctrl c;
  prepare_ctrl(h, c, t_end, dt, max_steps);
  *h->h_ctrl = c;
  HIPCHK(hipMemcpyAsync(h->d_ctrl, h->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, h->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, h->stream));
  const bool run1d = h->cfg.ndim == 1 && h->cfg.scheme == CLAW_CLASSIC &&
                     classic1d_run_smem(h->m, h->hg.nx, h->fp32) <= kRun1dSmemMax;
  if (run1d) {
    HIPCHK(launch_classic1d_run(h->kr, h->fp32, h->m, h->hg.nx, h->stream, h->d_grid));
    if ((rc = read_ctrl(h))) return rc;
  } else {
    if (!h->graph || h->graph_k != k) {
      if (h->graph) { hipGraphExecDestroy(h->graph); h->graph = nullptr; }
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      for (int s = 0; s < k; ++s) {
        if (launch_attempt_device(h) != CLAW_OK) {
          hipStreamEndCapture(h->stream, &g);
          if (g) hipGraphDestroy(g);
          return CLAW_E_DEVICE;
        }
      }
      HIPCHK(hipStreamEndCapture(h->stream, &g));
      const hipError_t e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      HIPCHK(e);
      h->graph_k = k;
    }
    for (;;) {
      // estimate the attempts still needed and launch that many graphs
      const Ctrl& hc = *h->h_ctrl;
      double est = hc.dt_try > 0.0 ? (hc.t_end - hc.t) / hc.dt_try + 1.0 : 1.0;
      if (hc.max_attempts > 0) est = std::min(est, (double)(hc.max_attempts - hc.attempts));
      long long launches = (long long)std::ceil(est / k);
      launches = std::max(1LL, std::min(launches, 4096LL));
      for (long long l = 0; l < launches; ++l) HIPCHK(hipGraphLaunch(h->graph, h->stream));
      if ((rc = read_ctrl(h))) return rc;
      if (!h->h_ctrl->active) break;
    }
  }
  {
    float ms = 0.f;
    if (hipEventRecord(e1, h->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
        hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      h->clock.gpu_ms = ms;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  const Ctrl& r = *h->h_ctrl;
  absorb_ctrl(h, r);
  clock_out(h, st);
  if (r.status) return r.status;
  if (r.t < t_end) return CLAW_E_MAXSTEPS;
  return CLAW_OK;
}

int claw_totals(claw_t h, double* totals) {
  if (!h || !totals) return CLAW_E_INVAL;
  if (!h->state_set) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(h->device));
  const double cell = h->hg.dx * h->hg.dy;
  HIPCHK(launch_totals(h->fp32, h->hg.q[h->src], h->hg.c[h->src], h->m, h->ncell, cell, h->d_part,
                       h->d_tot, h->stream));
  HIPCHK(hipMemcpyAsync(totals, h->d_tot, h->m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return CLAW_OK;
}

int claw_get_clock(claw_t h, claw_stats* st) {
  if (!h || !st) return CLAW_E_INVAL;
  *st = h->clock;
  return CLAW_OK;
}

int claw_set_clock(claw_t h, const claw_stats* st) {
  if (!h || !st) return CLAW_E_INVAL;
  h->clock = *st;
  return CLAW_OK;
}

int claw_set_tuning(claw_t h, const claw_tuning* tn) {
  if (!h || !tn || (tn->seg_rows < 1 && tn->segs < 1) || tn->order < 0 || tn->order > 3)
    return CLAW_E_INVAL;
  HIPCHK(hipSetDevice(h->device));
  set_tiling(h, tn->segs > 0 ? tn->segs : segs_from_rows(h->hg.ny, tn->seg_rows));
  h->seg_rows_x = tn->seg_rows_x > 0 ? tn->seg_rows_x : 0;
  h->hg.order = h->cfg.ndim == 2 ? tn->order : 0;
  int rc = upload_grid(h);
  if (rc) return rc;
  if (h->graph) { hipGraphExecDestroy(h->graph); h->graph = nullptr; }
  return sync(h);
}

int claw_get_tuning(claw_t h, claw_tuning* tn) {
  if (!h || !tn) return CLAW_E_INVAL;
  std::memset(tn, 0, sizeof(*tn));
  tn->seg_rows = h->hg.seg_rows;
  tn->seg_rows_x = h->seg_rows_x > 0 ? h->seg_rows_x : h->hg.seg_rows;
  tn->segs = h->hg.segs;
  tn->order = h->hg.order;
  return CLAW_OK;
}

int claw_autotune(claw_t h, int reps, claw_tuning* out) {
  if (!h) return CLAW_E_INVAL;
  if (!h->state_set || (h->na && !h->aux_set)) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(h->device));
  if (reps < 1) reps = 3;
  const int ny = h->hg.ny;
  // candidate segment counts: those of 4..128 rows per segment, and those
  // that bring the workgroup count just under a whole number of waves per
  // SIMD (a launch whose last round leaves some SIMDs with one wave less
  // takes as long as if they all had it)
  std::vector<int> cands;
  if (h->cfg.ndim == 2) {
    for (int c : {4, 5, 6, 7, 8, 9, 10, 11, 12, 14, 16, 20, 24, 28, 32, 40, 48, 64, 96, 128})
      if (c <= ny) cands.push_back(segs_from_rows(ny, c));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) !=
        hipSuccess)
      cus = 0;
    const int simds = 4 * cus;
    const int strips = h->hg.strips;
    for (int w = 1; w <= 8 && simds > 0; ++w) {
      const int s = w * simds / strips;
      if (s >= 1 && s <= ny && (ny + s - 1) / s >= 4) cands.push_back(s);
    }
    if (cands.empty()) cands.push_back(1);
    std::sort(cands.begin(), cands.end());
    cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
  } else {
    cands.push_back(1);
  }
  double dt;
  int rc = first_dt(h, &dt);
  if (rc) return rc;
  dt *= 0.5;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // warm-up, then timed repetitions; host-dt launches write the other
  // buffer (classic), the split step's intermediates or the stage buffers
  // (SharpClaw stages 1-2) and leave the state untouched
  auto run = [&]() -> int {
    if (h->cfg.scheme == CLAW_CLASSIC) return launch_attempt_host(h, dt, true);
    return launch_sharp_stages(h, 0, 2, kHostDt, dt);
  };
  // time every candidate of one tiling parameter (`apply` installs it) and
  // leave the fastest installed
  auto tune = [&](const std::vector<int>& cs, auto apply) -> int {
    int best = cs[0];
    float best_ms = std::numeric_limits<float>::infinity();
    for (int c : cs) {
      apply(c);
      if ((rc = upload_grid(h))) return best;
      if ((rc = run())) return best;
      if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = CLAW_E_DEVICE; return best; }
      for (int r = 0; r < reps && !rc; ++r) rc = run();
      if (rc) return best;
      float ms = 0.f;
      if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = CLAW_E_DEVICE;
        return best;
      }
      if (ms < best_ms) { best_ms = ms; best = c; }
    }
    apply(best);
    return best;
  };
  h->hg.order = 0;
  const int best = tune(cands, [&](int c) { set_tiling(h, c); });
  int best_x = 0, best_order = 0;
  if (!rc && split(h->cfg)) {
    std::vector<int> cx;
    for (int c : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32})
      if (c <= ny) cx.push_back(c);
    best_x = tune(cx, [&](int c) { h->seg_rows_x = c; });
  }
  if (!rc && h->cfg.ndim == 2)
    best_order = tune(std::vector<int>{0, 1, 2, 3}, [&](int o) { h->hg.order = o; });
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(h)] = Tiling{best, best_x, best_order};
  }
  if ((rc = upload_grid(h))) return rc;
  if (h->graph) { hipGraphExecDestroy(h->graph); h->graph = nullptr; }
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->seg_rows = h->hg.seg_rows;
    out->seg_rows_x = best_x > 0 ? best_x : h->hg.seg_rows;
    out->segs = h->hg.segs;
    out->order = h->hg.order;
  }
  return sync(h);
}

int claw_time_kernel(claw_t h, double dt, int reps, double* avg_ms) {
  if (!h || !avg_ms || reps < 1 || !(dt > 0.0)) return CLAW_E_INVAL;
  if (!h->state_set || (h->na && !h->aux_set)) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(h->device));
  auto one = [&]() -> int {
    if (h->cfg.scheme == CLAW_CLASSIC) return launch_attempt_host(h, dt, true);
    return launch_sharp_stages(h, 0, 2, kHostDt, dt);
  };
  int rc = one();
  if (rc) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, h->stream));
  for (int r = 0; r < reps && !rc; ++r) rc = one();
  HIPCHK(hipEventRecord(e1, h->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  *avg_ms = (double)ms / reps / (h->cfg.scheme == CLAW_CLASSIC ? 1 : 2);
  return CLAW_OK;
}

// ---------------------------------------------------------------------------
// Batches.
// ---------------------------------------------------------------------------
size_t claw_batch_workspace_bytes(int max_grids) {
  if (max_grids < 1) return 0;
  return align_up((size_t)max_grids * sizeof(GridDesc)) +
         align_up((size_t)(max_grids + 1) * sizeof(int)) +
         kBatchInFlight * align_up((size_t)max_grids * sizeof(Ctrl));
}

}  // extern "C"

namespace {
Ctrl* batch_dctrls(claw_batch_t b, int slot) {
  return (Ctrl*)((char*)b->d_ctrls + slot * align_up((size_t)b->max_grids * sizeof(Ctrl)));
}

// Enqueue the copy of every member's controller into one contiguous device
// array and from there into the pinned host array of group slot `slot`
// (one readback), then the group's completion event.  No synchronisation.
int batch_gather_async(claw_batch_t b, int slot) {
  Ctrl* d = batch_dctrls(b, slot);
  for (size_t k = 0; k < b->members.size(); ++k)
    HIPCHK(hipMemcpyAsync(d + k, b->members[k]->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToDevice,
                          b->stream));
  if (!b->members.empty())
    HIPCHK(hipMemcpyAsync(b->h_ctrls[slot], d, b->members.size() * sizeof(Ctrl),
                          hipMemcpyDeviceToHost, b->stream));
  b->snap[slot] = b->members;
  HIPCHK(hipEventRecord(b->ev[slot], b->stream));
  return CLAW_OK;
}

// The member's controller as of the view (nullptr if it is not in it).
const Ctrl* view_of(claw_batch_t b, claw_t h) {
  if (!b->view || !b->view_members) return nullptr;
  const std::vector<claw_t>& v = *b->view_members;
  for (size_t k = 0; k < v.size(); ++k)
    if (v[k] == h) return b->view + k;
  return nullptr;
}

// Upload the member tables for the group about to be launched (slot `slot`),
// stream-ordered after the groups already in flight, which keep reading the
// previous tables until they end.
int batch_rebuild(claw_batch_t b, int slot) {
  const size_t ng = b->members.size();
  GridDesc* gd = b->h_grids[slot];
  int* bs = b->h_bstart[slot];
  b->bstart.assign(ng + 1, 0);
  for (size_t k = 0; k < ng; ++k) {
    gd[k] = b->members[k]->hg;
    b->bstart[k + 1] = b->bstart[k] + gd[k].nblocks;
  }
  for (size_t k = 0; k <= ng; ++k) bs[k] = b->bstart[k];
  if (ng) {
    HIPCHK(hipMemcpyAsync(b->d_grids, gd, ng * sizeof(GridDesc), hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipMemcpyAsync(b->d_bstart, bs, (ng + 1) * sizeof(int), hipMemcpyHostToDevice,
                          b->stream));
  }
  if (b->graph) {
    b->retired.emplace_back(b->graph, b->launched);
    b->graph = nullptr;
  }
  b->dirty = false;
  return CLAW_OK;
}

// Destroy the replaced graphs whose last launches have completed.
void batch_reap(claw_batch_t b) {
  auto it = b->retired.begin();
  while (it != b->retired.end()) {
    if (it->second <= b->waited) {
      hipGraphExecDestroy(it->first);
      it = b->retired.erase(it);
    } else {
      ++it;
    }
  }
}
}  // namespace

extern "C" {

int claw_batch_create(int max_grids, void* d_ws, size_t ws_bytes, void* hip_stream,
                      claw_batch_t* out) {
  if (!out || max_grids < 1 || !d_ws || ((uintptr_t)d_ws % kAlign) != 0) return CLAW_E_INVAL;
  if (ws_bytes < claw_batch_workspace_bytes(max_grids)) return CLAW_E_NOMEM;
  claw_batch_t b = new (std::nothrow) claw_batch();
  if (!b) return CLAW_E_NOMEM;
  b->max_grids = max_grids;
  hipGetDevice(&b->device);
  char* base = (char*)d_ws;
  b->d_grids = (GridDesc*)base;
  b->d_bstart = (int*)(base + align_up((size_t)max_grids * sizeof(GridDesc)));
  b->d_ctrls = (Ctrl*)(base + align_up((size_t)max_grids * sizeof(GridDesc)) +
                       align_up((size_t)(max_grids + 1) * sizeof(int)));
  if (hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else if (hipStreamCreate(&b->stream) == hipSuccess) {
    b->own_stream = true;
  } else {
    delete b;
    return CLAW_E_DEVICE;
  }
  for (int k = 0; k < kBatchInFlight; ++k) {
    if (hipHostMalloc((void**)&b->h_ctrls[k], (size_t)max_grids * sizeof(Ctrl),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_grids[k], (size_t)max_grids * sizeof(GridDesc),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_bstart[k], (size_t)(max_grids + 1) * sizeof(int),
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming) != hipSuccess) {
      claw_batch_destroy(b);
      return CLAW_E_DEVICE;
    }
  }
  *out = b;
  return CLAW_OK;
}

int claw_batch_destroy(claw_batch_t b) {
  if (!b) return CLAW_E_INVAL;
  hipSetDevice(b->device);
  if (b->stream) hipStreamSynchronize(b->stream);
  if (b->graph) hipGraphExecDestroy(b->graph);
  for (auto& r : b->retired) hipGraphExecDestroy(r.first);
  for (int k = 0; k < kBatchInFlight; ++k) {
    if (b->h_ctrls[k]) hipHostFree(b->h_ctrls[k]);
    if (b->h_grids[k]) hipHostFree(b->h_grids[k]);
    if (b->h_bstart[k]) hipHostFree(b->h_bstart[k]);
    if (b->ev[k]) hipEventDestroy(b->ev[k]);
  }
  if (b->own_stream) hipStreamDestroy(b->stream);
  delete b;
  return CLAW_OK;
}

int claw_batch_add(claw_batch_t b, claw_t h, double t_end) {
  if (!b || !h) return CLAW_E_INVAL;
  if ((int)b->members.size() >= b->max_grids) return CLAW_E_BUDGET;
  if (h->cfg.scheme != CLAW_CLASSIC || h->cfg.ndim != 2 || split(h->cfg)) return CLAW_E_INVAL;
  if (h->device != b->device) return CLAW_E_INVAL;
  if (!h->state_set || (h->na && !h->aux_set)) return CLAW_E_STATE;
  for (claw_t o : b->members)
    if (o == h) return CLAW_E_INVAL;
  if (!b->members.empty() &&
      (b->riemann != h->kr || b->fp32 != h->pk || b->limiter != h->hg.limiter ||
       b->transverse != h->hg.transverse))
    return CLAW_E_INVAL;
  HIPCHK(hipSetDevice(b->device));
  double dt;
  int rc = first_dt(h, &dt);
  if (rc) return rc;
  Ctrl c;
  prepare_ctrl(h, c, t_end, dt, 0);
  *h->h_ctrl = c;
  HIPCHK(hipMemcpyAsync(h->d_ctrl, h->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  b->riemann = h->kr;
  b->fp32 = h->pk;
  b->limiter = h->hg.limiter;
  b->transverse = h->hg.transverse;
  b->members.push_back(h);
  b->dirty = true;
  return CLAW_OK;
}

int claw_batch_remove(claw_batch_t b, claw_t h) {
  if (!b || !h) return CLAW_E_INVAL;
  auto it = std::find(b->members.begin(), b->members.end(), h);
  if (it == b->members.end()) return CLAW_E_INVAL;
  HIPCHK(hipSetDevice(b->device));
  const Ctrl* v = view_of(b, h);
  if (v && !v->active) {
    // stopped as of the view: later groups skip it (a stopped controller
    // never restarts), so the view holds its final controller (no wait)
    absorb_ctrl(h, *v);
  } else {
    if (b->launched > b->waited) HIPCHK(hipStreamSynchronize(b->stream));
    int rc = read_ctrl(h);
    if (rc) return rc;
    absorb_ctrl(h, *h->h_ctrl);
  }
  b->members.erase(it);
  b->dirty = true;
  return CLAW_OK;
}

int claw_batch_member_clock(claw_batch_t b, claw_t h, claw_stats* st) {
  if (!b || !h || !st) return CLAW_E_INVAL;
  auto it = std::find(b->members.begin(), b->members.end(), h);
  if (it == b->members.end()) return CLAW_E_INVAL;
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipStreamSynchronize(b->stream));
  int rc = read_ctrl(h);
  if (rc) return rc;
  const Ctrl& c = *h->h_ctrl;
  *st = h->clock;
  st->t = c.t;
  st->dt_next = c.dt;
  st->accepted += c.accepted;
  st->rejected += c.rejected;
  st->max_courant = c.max_courant;
  return c.status ? c.status : CLAW_OK;
}

int claw_batch_finished(claw_batch_t b, claw_t* out, int cap, int* n_out) {
  if (!b || !n_out || (cap > 0 && !out)) return CLAW_E_INVAL;
  int n = 0;
  if (b->view && b->view_members) {
    const std::vector<claw_t>& v = *b->view_members;
    for (size_t k = 0; k < v.size(); ++k) {
      if (b->view[k].active) continue;
      if (std::find(b->members.begin(), b->members.end(), v[k]) == b->members.end()) continue;
      if (n < cap) out[n] = v[k];
      ++n;
    }
  }
  *n_out = std::min(n, cap);
  return CLAW_OK;
}

int claw_batch_launch(claw_batch_t b, int attempts) {
  if (!b || attempts < 0) return CLAW_E_INVAL;
  if (b->launched - b->waited >= kBatchInFlight) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(b->device));
  int rc;
  const int slot = (int)(b->launched % kBatchInFlight);
  if (b->dirty && (rc = batch_rebuild(b, slot))) return rc;
  const int ng = (int)b->members.size();
  if (ng > 0) {
    const int total = b->bstart[ng];
    constexpr int kGraph = 16;
    if (attempts >= kGraph && !b->graph) {
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      for (int s = 0; s < kGraph; ++s)
        launch_classic2d(b->riemann, b->fp32, b->limiter, b->transverse, total, b->stream,
                         b->d_grids, b->d_bstart, ng, kDeviceCtrl, 0.0, 0);
      HIPCHK(hipStreamEndCapture(b->stream, &g));
      const hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      HIPCHK(e);
      b->graph_k = kGraph;
    }
    int done = 0;
    while (b->graph && attempts - done >= b->graph_k) {
      HIPCHK(hipGraphLaunch(b->graph, b->stream));
      done += b->graph_k;
    }
    for (; done < attempts; ++done)
      HIPCHK(launch_classic2d(b->riemann, b->fp32, b->limiter, b->transverse, total, b->stream,
                              b->d_grids, b->d_bstart, ng, kDeviceCtrl, 0.0, 0));
  }
  if ((rc = batch_gather_async(b, slot))) return rc;
  b->launched += 1;
  return CLAW_OK;
}

int claw_batch_wait(claw_batch_t b, int* n_active) {
  if (!b) return CLAW_E_INVAL;
  if (b->launched == b->waited) return CLAW_E_STATE;
  HIPCHK(hipSetDevice(b->device));
  const int slot = (int)(b->waited % kBatchInFlight);
  HIPCHK(hipEventSynchronize(b->ev[slot]));
  b->waited += 1;
  batch_reap(b);
  b->view = b->h_ctrls[slot];
  b->view_members = &b->snap[slot];
  int act = 0, status = 0;
  for (size_t k = 0; k < b->snap[slot].size(); ++k) {
    act += b->view[k].active ? 1 : 0;
    if (b->view[k].status) status = b->view[k].status;
  }
  if (n_active) *n_active = act;
  return status ? status : CLAW_OK;
}

int claw_batch_advance(claw_batch_t b, int attempts, int* n_active) {
  if (!b || attempts < 0) return CLAW_E_INVAL;
  int rc = CLAW_OK;
  while (b->launched > b->waited && rc == CLAW_OK) rc = claw_batch_wait(b, nullptr);
  if (rc) return rc;
  if ((rc = claw_batch_launch(b, attempts))) return rc;
  return claw_batch_wait(b, n_active);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// claw_step_static: one step without a caller workspace.
// ---------------------------------------------------------------------------
namespace {

// Device memory of claw_step_static: grid descriptor, controller record,
// Courant-reduction slots and, as the configuration needs them, the
// working-precision state, stage and sweep buffers and aux.  Each device
// holds its own copy from the library's first use on it until the process
// ends.  In host code the symbol is a stand-in, not a device address: only
// the address hipGetSymbolAddress returns on a device is used.
static __device__ __align__(256) unsigned char scratch[CLAW_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// The current device's scratch address, looked up once per device (with
// that device current).
int scratch_base(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return CLAW_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CLAW_E_DEVICE;
    g_scratch[dev] = (char*)p;
  }
  *out = g_scratch[dev];
  return CLAW_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

size_t claw_static_bytes(const claw_config* cfg) {
  if (validate(cfg) != CLAW_OK) return 0;
  size_t off[16];
  return layout(normalised(*cfg), off, true);
}

int claw_step_static(const claw_config* cfg, const double* d_q_in, const double* d_aux,
                     double* d_q_out, double dt, double* d_courant, void* hip_stream) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!d_q_in || !d_q_out || !d_courant || !(dt > 0.0)) return CLAW_E_INVAL;
  const claw_config c = normalised(*cfg);
  const int m = num_eqn_of(c), na = num_aux_of(c);
  if (na && !d_aux) return CLAW_E_INVAL;
  const size_t N = (size_t)c.num_cells[0] * (c.ndim == 2 ? c.num_cells[1] : 1);
  const size_t n = (size_t)m * N;
  if (overlap(d_q_in, n * sizeof(double), d_q_out, n * sizeof(double)) ||
      overlap(d_courant, sizeof(double), d_q_out, n * sizeof(double)) ||
      overlap(d_courant, sizeof(double), d_q_in, n * sizeof(double)))
    return CLAW_E_INVAL;
  size_t off[16];
  if (layout(c, off, true) > CLAW_STATIC_SCRATCH_BYTES) return CLAW_E_TOOBIG;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  char* base = nullptr;
  if ((rc = scratch_base(dev, &base))) return rc;
  // a handle on the stack over the scratch: nothing is allocated
  claw_solver h{};
  h.cfg = c;
  h.device = dev;
  h.stream = (hipStream_t)hip_stream;
  fill_handle(&h, off, base);
  GridDesc& g = h.hg;
  const bool classic = c.scheme == CLAW_CLASSIC;
  const hipStream_t st = h.stream;
  if (!h.fp32) {
    g.aux = d_aux;
    if (classic) {
      // the step reads Q^n from q[0] and writes Q^{n+1} to q[1]
      g.q[0] = const_cast<double*>(d_q_in);
      g.q[1] = d_q_out;
    } else {
      // the Runge-Kutta stages update Q in place: start from a copy
      HIPCHK(hipMemcpyAsync(d_q_out, d_q_in, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      g.q[0] = d_q_out;
      g.q[1] = nullptr;
    }
  }
  HIPCHK(launch_static_setup(g, h.d_grid, h.d_ctrl, g.slots, st));
  if (h.fp32) {
    HIPCHK(launch_load_state(1, g.q[0], g.c[0], d_q_in, n, st));
    if (na) HIPCHK(launch_convert(1, (void*)g.aux, d_aux, (size_t)na * N, st));
  }
  if ((rc = launch_attempt_host(&h, dt, false))) return rc;
  HIPCHK(launch_static_courant(h.d_ctrl, dt, d_courant, st));
  if (h.fp32) {
    const int dst = classic ? 1 : 0;
    HIPCHK(launch_store_state(1, d_q_out, g.q[dst], g.c[dst], n, st));
  }
  return CLAW_OK;
}

}  // extern "C"
