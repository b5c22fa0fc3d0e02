// ctu_runtime.cpp -- host runtime behind the C ABI of include/ctu.h: configuration checks,
// workspace carving, stream-ordered launch sequences, host<->device transfers, error words,
// and the batch scheduler.  Device memory is always the caller's.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctu.h"
#include "ctu_kernels.hpp"

using ctu::DevScalars;
using ctu::GridParams;

namespace {

// Message of the last failing call on this thread, in fixed storage (setting it allocates
// nothing).
thread_local char g_err[512];

ctu_status fail(ctu_status s, const char* msg) {
  std::snprintf(g_err, sizeof(g_err), "%s", msg);
  return s;
}

ctu_status fail(ctu_status s, const std::string& msg) { return fail(s, msg.c_str()); }

ctu_status hip_fail(hipError_t e, const char* where) {
  std::snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
  return CTU_EDEVICE;
}

#define HIP_TRY(expr, where)                  \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// Workspace header: device scalars, totals partials, and the one-grid launch plan.
constexpr size_t kScalarsOffset = 0;
constexpr size_t kPartialOffset = 4096;
constexpr int kTotalsBlocks = 1024;
constexpr size_t kTotalsOutOffset = kPartialOffset + sizeof(double) * 5 * kTotalsBlocks;
constexpr size_t kDescOffset = 49152;
constexpr size_t kStartOffset = 53248;
constexpr size_t kHeaderBytes = 65536;
static_assert(kTotalsOutOffset + 5 * sizeof(double) <= kDescOffset, "header overlap");
static_assert(kDescOffset + sizeof(ctu::GridDesc) <= kStartOffset, "descriptor too large");
static_assert(kStartOffset + sizeof(int) * ctu::P_NUM * 2 <= kHeaderBytes, "header overflow");

size_t elem_bytes(int prec) { return prec == CTU_FP32 ? 4 : 8; }

GridParams make_params(const ctu_config& c);

// One double per block of the fused update, for the block-partial CFL reduction.
size_t partial_bytes(const ctu_config& c) {
  const long long blocks = ctu::update_blocks(make_params(c)) + 64;
  return (size_t)((blocks * 8 + 255) / 256 * 256);
}

// Ghost layers: the PPMC stencil reaches two cells and the CTU transverse correction one
// more; PPMP's flattening reaches three.
// The H correction reads second-stage states one cell beyond the real box: one more.
int ghost_layers(const ctu_config& c) {
  return (c.recon == CTU_RECON_PPMP ? 4 : 3) + (c.h_correction ? 1 : 0);
}

long long alloc_cells(const ctu_config& c) {
  const int g = ghost_layers(c);
  return (long long)(c.nx + 2 * g) * (c.ny + 2 * g) * (c.nz + 2 * g);
}

// Workspace fields: first-stage and CTU flux differences (3 x 5 each); PPMP adds its
// flattening and steepening coefficients per axis (3 x 2), the H correction its face eta
// per axis (3).
int coef_fields(const ctu_config& c) { return c.recon == CTU_RECON_PPMP ? 6 : 0; }
int fields_per_grid(const ctu_config& c) { return 30 + coef_fields(c) + (c.h_correction ? 3 : 0); }

long long field_stride(const ctu_config& c) {
  long long n = alloc_cells(c);
  return (n + 63) / 64 * 64;
}

ctu_status validate(const ctu_config* c) {
  if (!c) return fail(CTU_EINVAL, "null config");
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(CTU_EINVAL, "cell counts must be >= 1");
  if (!(c->dx > 0 && c->dy > 0 && c->dz > 0)) return fail(CTU_EINVAL, "cell widths must be > 0");
  if (!(c->gamma > 1.0)) return fail(CTU_EINVAL, "gamma must be > 1");
  if (!(c->cfl > 0.0 && c->cfl < 0.5)) return fail(CTU_EINVAL, "cfl must lie in (0, 0.5)");
  if (!(c->newton_tol > 0.0)) return fail(CTU_EINVAL, "newton_tol must be > 0");
  if (c->newton_max_iter < 1) return fail(CTU_EINVAL, "newton_max_iter must be >= 1");
  if (!(c->p_floor > 0.0)) return fail(CTU_EINVAL, "p_floor must be > 0");
  if (c->prec != CTU_FP64 && c->prec != CTU_FP32) return fail(CTU_EINVAL, "unknown precision");
  if (c->riemann != CTU_RIEMANN_EXACT && c->riemann != CTU_RIEMANN_ROE)
    return fail(CTU_EINVAL, "unknown Riemann solver");
  if (c->recon != CTU_RECON_PPMC && c->recon != CTU_RECON_PPMP)
    return fail(CTU_EINVAL, "unknown reconstruction");
  if (c->h_correction != 0 && c->h_correction != 1)
    return fail(CTU_EINVAL, "h_correction must be 0 or 1");
  if (c->h_correction && c->riemann != CTU_RIEMANN_ROE)
    return fail(CTU_EINVAL, "the H correction needs the Roe solver");
  for (int a = 0; a < 2; ++a)
    if (c->march_seg[a] < 0 || c->march_seg[a] > 4096)
      return fail(CTU_EINVAL, "march_seg must lie in [0, 4096]");
  if (c->x_rows < 0 || c->x_rows > 8) return fail(CTU_EINVAL, "x_rows must lie in [0, 8]");
  if (c->x_chunks < 0 || c->x_chunks > 16) return fail(CTU_EINVAL, "x_chunks must lie in [0, 16]");
  if (c->schedule < CTU_SCHEDULE_AUTO || c->schedule > CTU_SCHEDULE_FUSED_Z)
    return fail(CTU_EINVAL, "unknown schedule");
  for (int a = 0; a < 3; ++a) {
    int lo = c->bc[2 * a], hi = c->bc[2 * a + 1];
    for (int b : {lo, hi})
      if (b != CTU_BC_PERIODIC && b != CTU_BC_OUTFLOW && b != CTU_BC_REFLECT)
        return fail(CTU_EINVAL, "unknown boundary type");
    if ((lo == CTU_BC_PERIODIC) != (hi == CTU_BC_PERIODIC))
      return fail(CTU_EINVAL, "periodic boundaries must pair");
    const int n = a == 0 ? c->nx : a == 1 ? c->ny : c->nz;
    if ((lo == CTU_BC_REFLECT || hi == CTU_BC_REFLECT) && n < ghost_layers(*c))
      return fail(CTU_EINVAL, "a reflecting boundary needs as many cells on its axis as there "
                              "are ghost layers");
  }
  const long long ncell = (long long)c->nx * c->ny * c->nz;
  if (ncell > (1LL << 31)) return fail(CTU_EINVAL, "grid too large");
  return CTU_OK;
}

GridParams make_params(const ctu_config& c) {
  GridParams P;
  P.n[0] = c.nx;
  P.n[1] = c.ny;
  P.n[2] = c.nz;
  P.ng = ghost_layers(c);
  for (int a = 0; a < 3; ++a) P.N[a] = P.n[a] + 2 * P.ng;
  P.stride = field_stride(c);
  P.dx[0] = c.dx;
  P.dx[1] = c.dy;
  P.dx[2] = c.dz;
  P.gamma = c.gamma;
  P.newton_tol = c.newton_tol;
  P.newton_max_iter = c.newton_max_iter;
  P.p_floor = c.p_floor;
  P.cfl = c.cfl;
  const double g = c.gamma;
  P.gm1 = g - 1.0;
  P.z_exp = (g - 1.0) / (2.0 * g);
  P.inv_gamma = 1.0 / g;
  P.two_over_gm1 = 2.0 / (g - 1.0);
  P.two_over_gp1 = 2.0 / (g + 1.0);
  P.gm1_over_gp1 = (g - 1.0) / (g + 1.0);
  P.shock_a = (g + 1.0) / (2.0 * g);
  P.shock_b = (g - 1.0) / (2.0 * g);
  double e = 2.0 / (g - 1.0);
  double r = std::nearbyint(e);
  P.fan_int_exp = (std::fabs(e - r) < 1e-12 && r >= 1.0 && r <= 16.0) ? (int)r : 0;
  double m = 2.0 * g / (g - 1.0);
  double mr = std::nearbyint(m);
  P.root_m = (std::fabs(m - mr) < 1e-12 && mr >= 2.0 && mr <= 16.0) ? (int)mr : 0;
  P.inv_root_m = (g - 1.0) / (2.0 * g);
  P.inv_gm1 = 1.0 / (g - 1.0);
  P.riemann = c.riemann;
  P.recon = c.recon;
  P.ext = c.h_correction ? 1 : 0;
  // march segments: round(n/target) equal segments of the n cells of the axis
  P.seg[0] = 0;
  for (int a = 1; a < 3; ++a) {
    const int cells = P.n[a];
    const int target = c.march_seg[a - 1] > 0 ? c.march_seg[a - 1] : ctu::kSegDefault;
    int nseg = (int)std::lround((double)cells / target);
    nseg = nseg < 1 ? 1 : (nseg > cells ? cells : nseg);
    P.seg[a] = (cells + nseg - 1) / nseg;
  }
  P.xrows = c.x_rows > 0 ? (c.x_rows < c.ny ? c.x_rows : c.ny) : ctu::choose_xrows(c.nx, c.ny);
  P.xchunks = c.x_chunks > 0 ? c.x_chunks : ctu::kXChunks;
  return P;
}

// Block table of a launch over the grids Ps: for every pass, grid g owns the blocks
// [start[p*(n+1)+g], start[p*(n+1)+g+1]), its count padded to a multiple of 8 so that every
// grid's range starts on the first XCD of the round-robin dispatch.  False if a pass would
// exceed the launch limit.
bool build_starts(const std::vector<GridParams>& Ps, std::vector<int>& start) {
  const int n = (int)Ps.size();
  start.assign((size_t)ctu::P_NUM * (n + 1), 0);
  for (int p = 0; p < ctu::P_NUM; ++p) {
    long long off = 0;
    for (int g = 0; g < n; ++g) {
      start[(size_t)p * (n + 1) + g] = (int)off;
      off += (ctu::pass_blocks(Ps[g], p) + 7) / 8 * 8;
      // a dispatch holds at most 2^32 - 1 work-items along x
      if (off * ctu::kBlock > 0xffffffffLL) return false;
    }
    start[(size_t)p * (n + 1) + n] = (int)off;
  }
  return true;
}

// build_starts for one grid, into a caller array of 2 * P_NUM ints (allocates nothing).
bool build_starts_one(const GridParams& P, int* start) {
  for (int p = 0; p < ctu::P_NUM; ++p) {
    const long long nb = (ctu::pass_blocks(P, p) + 7) / 8 * 8;
    if (nb * ctu::kBlock > 0xffffffffLL) return false;
    start[2 * p] = 0;
    start[2 * p + 1] = (int)nb;
  }
  return true;
}

}  // namespace

struct ctu_grid {
  ctu_config cfg;
  GridParams P;
  hipStream_t stream;
  char* d_state;
  char* d_work;
  size_t work_bytes;
  bool dt_valid;  // device dt_next_bits holds the CFL bound of the current state
  bool in_batch = false;
  ctu::Profiler* prof = nullptr;  // per-kernel timing when enabled
  ctu::GridDesc desc;             // host copy of the descriptor at d_work + kDescOffset
  std::vector<int> h_start;       // host copy of the one-grid block table
  // the side stream and events of the overlapped sweep schedule (null when serial)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, xdone = nullptr, join = nullptr, ydone = nullptr;
  int schedule = CTU_SCHEDULE_IN_ORDER;  // the schedule steps use
  ~ctu_grid() {
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    for (hipEvent_t ev : {fork, xdone, join, ydone})
      if (ev) (void)hipEventDestroy(ev);
  }
  DevScalars* scalars() const { return reinterpret_cast<DevScalars*>(d_work + kScalarsOffset); }
  double* partial() const { return reinterpret_cast<double*>(d_work + kPartialOffset); }
  double* totals_out() const { return reinterpret_cast<double*>(d_work + kTotalsOutOffset); }
  char* fields() const { return d_work + kHeaderBytes; }
  double* partials() const {
    return reinterpret_cast<double*>(d_work + kHeaderBytes + (size_t)fields_per_grid(cfg) * fbytes());
  }
  size_t fbytes() const { return (size_t)P.stride * elem_bytes(cfg.prec); }
  ctu::GridDesc* d_desc() const { return reinterpret_cast<ctu::GridDesc*>(d_work + kDescOffset); }
  int* d_start() const { return reinterpret_cast<int*>(d_work + kStartOffset); }
  ctu::PlanView plan() const {
    return ctu::PlanView{d_desc(), d_start(), 1, h_start.data(), cfg.prec == CTU_FP32 ? 1 : 0,
                         ctu::gas_class(P), P.recon, side, fork, xdone, join, ydone,
                         schedule == CTU_SCHEDULE_FUSED_Z};
  }
};

namespace {

ctu_status step_impl(ctu_grid* g, bool device_dt) {
  hipError_t e = ctu::launch_step(g->plan(), device_dt, g->stream, g->prof);
  if (e != hipSuccess) return hip_fail(e, "step launch");
  g->dt_valid = true;
  return CTU_OK;
}

ctu_status ensure_dt(ctu_grid* g) {
  if (g->dt_valid) return CTU_OK;
  hipError_t e = ctu::launch_dt(g->plan(), g->stream);
  if (e != hipSuccess) return hip_fail(e, "dt launch");
  g->dt_valid = true;
  return CTU_OK;
}

ctu_status not_in_batch(const ctu_grid* g) {
  if (g->in_batch) return fail(CTU_EINVAL, "grid is submitted to a batch until its ticket ends");
  return CTU_OK;
}

ctu_status reset_scalars(ctu_grid* g) {
  DevScalars s;
  std::memset(&s, 0, sizeof(s));
  s.dt_next_bits = 0x7ff0000000000000ull;
  HIP_TRY(hipMemcpyAsync(g->scalars(), &s, sizeof(s), hipMemcpyHostToDevice, g->stream), "reset");
  HIP_TRY(hipStreamSynchronize(g->stream), "reset sync");
  g->dt_valid = false;
  return CTU_OK;
}

ctu_status read_scalars(ctu_grid* g, DevScalars* s) {
  HIP_TRY(hipMemcpyAsync(s, g->scalars(), sizeof(*s), hipMemcpyDeviceToHost, g->stream), "read scalars");
  HIP_TRY(hipStreamSynchronize(g->stream), "sync");
  return CTU_OK;
}

}  // namespace

extern "C" {

const char* ctu_last_error(void) { return g_err; }

ctu_status ctu_config_default(ctu_config* c) {
  if (!c) return fail(CTU_EINVAL, "null config");
  std::memset(c, 0, sizeof(*c));
  c->nx = c->ny = c->nz = 1;
  c->dx = c->dy = c->dz = 1.0;
  c->gamma = 5.0 / 3.0;
  for (int i = 0; i < 6; ++i) c->bc[i] = CTU_BC_PERIODIC;
  c->prec = CTU_FP64;
  c->cfl = 0.3;
  c->newton_tol = 1e-6;
  c->newton_max_iter = 50;
  c->p_floor = 1e-20;
  return CTU_OK;
}

ctu_status ctu_workspace_bytes(const ctu_config* cfg, size_t* state_bytes, size_t* work_bytes) {
  ctu_status s = validate(cfg);
  if (s != CTU_OK) return s;
  const size_t eb = elem_bytes(cfg->prec);
  const long long stride = field_stride(*cfg);
  if (state_bytes) *state_bytes = (size_t)5 * stride * eb;
  if (work_bytes)
    *work_bytes = kHeaderBytes + (size_t)fields_per_grid(*cfg) * stride * eb + partial_bytes(*cfg);
  return CTU_OK;
}

ctu_status ctu_grid_create(const ctu_config* cfg, void* d_state, void* d_work, size_t work_bytes,
                           void* hip_stream, ctu_grid** out) {
  if (!out) return fail(CTU_EINVAL, "null output handle");
  *out = nullptr;
  ctu_status s = validate(cfg);
  if (s != CTU_OK) return s;
  if (!d_state || !d_work) return fail(CTU_EINVAL, "null device buffer");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0 || reinterpret_cast<uintptr_t>(d_state) % 256 != 0)
    return fail(CTU_EINVAL, "device buffers must be 256-byte aligned");
  size_t need_state = 0, need_work = 0;
  ctu_workspace_bytes(cfg, &need_state, &need_work);
  if (work_bytes < need_work)
    return fail(CTU_ENOMEM, "workspace too small: need " + std::to_string(need_work) + " bytes");
  ctu_grid* g = new ctu_grid();
  g->cfg = *cfg;
  g->P = make_params(*cfg);
  g->stream = reinterpret_cast<hipStream_t>(hip_stream);
  g->d_state = reinterpret_cast<char*>(d_state);
  g->d_work = reinterpret_cast<char*>(d_work);
  g->work_bytes = work_bytes;
  g->dt_valid = false;
  g->desc.P = g->P;
  g->desc.u = g->d_state;
  g->desc.flux = g->fields();
  g->desc.s = g->scalars();
  g->desc.part = g->partials();
  g->desc.coef = cfg->recon == CTU_RECON_PPMP ? g->fields() + 30 * g->fbytes() : nullptr;
  g->desc.eta = cfg->h_correction ? g->fields() + (30 + coef_fields(*cfg)) * g->fbytes() : nullptr;
  for (int i = 0; i < 6; ++i) g->desc.bc[i] = cfg->bc[i];
  g->desc.flags = 0;
  if (!build_starts({g->P}, g->h_start)) {
    delete g;
    return fail(CTU_EINVAL, "grid too large for one launch per pass");
  }
  hipError_t e = hipSuccess;
  // the schedule (fused z has no H correction variant: its eta pass along z needs the second-
  // stage states of the ring columns, so such grids take the overlapped schedule)
  const bool hcorr = ctu::gas_class(g->P) == ctu::kRoeH;
  const long long cells = (long long)cfg->nx * cfg->ny * cfg->nz;
  switch (cfg->schedule) {
    case CTU_SCHEDULE_IN_ORDER: g->schedule = CTU_SCHEDULE_IN_ORDER; break;
    case CTU_SCHEDULE_OVERLAP: g->schedule = CTU_SCHEDULE_OVERLAP; break;
    case CTU_SCHEDULE_FUSED_Z:
      g->schedule = hcorr ? CTU_SCHEDULE_OVERLAP : CTU_SCHEDULE_FUSED_Z;
      break;
    default:
      if (hcorr)
        g->schedule = g->fbytes() <= CTU_OVERLAP_MAX_FIELD_BYTES ? CTU_SCHEDULE_OVERLAP
                                                                  : CTU_SCHEDULE_IN_ORDER;
      else
        g->schedule = cells <= CTU_OVERLAP_MAX_CELLS ? CTU_SCHEDULE_OVERLAP : CTU_SCHEDULE_FUSED_Z;
  }
  if (g->schedule != CTU_SCHEDULE_IN_ORDER) {
    // default priority, like every stream of the library
    e = hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking);
    // the events only order the grid's two streams on one GPU: a device-scope release is
    // enough (measured: 4% per step at 64^3 against the default system-scope fence)
    for (hipEvent_t* ev : {&g->fork, &g->xdone, &g->join, &g->ydone})
      if (e == hipSuccess)
        e = hipEventCreateWithFlags(ev, hipEventDisableTiming | hipEventDisableSystemFence);
    if (e != hipSuccess) {
      delete g;
      return hip_fail(e, "side stream");
    }
  }
  e = hipMemcpyAsync(g->d_desc(), &g->desc, sizeof(g->desc), hipMemcpyHostToDevice,
                                g->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->d_start(), g->h_start.data(), sizeof(int) * g->h_start.size(),
                       hipMemcpyHostToDevice, g->stream);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "descriptor upload");
  }
  s = reset_scalars(g);  // synchronizes, so the host copies above are no longer read
  if (s != CTU_OK) {
    delete g;
    return s;
  }
  *out = g;
  return CTU_OK;
}

ctu_status ctu_grid_destroy(ctu_grid* g) {
  if (!g) return fail(CTU_EINVAL, "null grid");
  if (ctu_status st = not_in_batch(g)) return st;
  (void)hipStreamSynchronize(g->stream);
  delete g->prof;
  delete g;
  return CTU_OK;
}

ctu_status ctu_profile_enable(ctu_grid* g, int32_t enable) {
  if (!g) return fail(CTU_EINVAL, "null grid");
  if (enable & ~(CTU_PROFILE_TIMING | CTU_PROFILE_NEWTON)) return fail(CTU_EINVAL, "unknown mode");
  if ((enable & CTU_PROFILE_NEWTON) && g->P.riemann != CTU_RIEMANN_EXACT)
    return fail(CTU_EINVAL, "the Newton histogram needs the exact solver");
  if (enable) {
    if (!g->prof) g->prof = new ctu::Profiler();
    HIP_TRY(hipStreamSynchronize(g->stream), "profile sync");
    g->prof->reset();
    g->prof->timing = (enable & CTU_PROFILE_TIMING) != 0;
    g->prof->hist = (enable & CTU_PROFILE_NEWTON) != 0;
    if (g->prof->hist) {
      HIP_TRY(hipMemsetAsync(reinterpret_cast<char*>(g->scalars()) +
                                 offsetof(DevScalars, newton_hist),
                             0, sizeof(DevScalars::newton_hist), g->stream),
              "histogram clear");
      HIP_TRY(hipStreamSynchronize(g->stream), "profile sync");
    }
  } else if (g->prof) {
    HIP_TRY(hipStreamSynchronize(g->stream), "profile sync");
    delete g->prof;
    g->prof = nullptr;
  }
  return CTU_OK;
}

ctu_status ctu_profile_read(ctu_grid* g, int32_t max_classes, double* ms, int64_t* launches,
                            int32_t* count) {
  if (!g || !count) return fail(CTU_EINVAL, "null argument");
  *count = ctu::K_NUM_CLASSES;
  if (!g->prof) return fail(CTU_EINVAL, "profiling not enabled");
  HIP_TRY(g->prof->collect(), "profile collect");
  for (int k = 0; k < ctu::K_NUM_CLASSES && k < max_classes; ++k) {
    if (ms) ms[k] = g->prof->ms[k];
    if (launches) launches[k] = g->prof->launches[k];
  }
  return CTU_OK;
}

const char* ctu_profile_name(int32_t k) { return ctu::kernel_class_name(k); }

size_t ctu_stream_probe_blocks(size_t n) { return ctu::stream_probe_blocks(n); }

ctu_status ctu_stream_probe(int32_t kind, const double* a, const double* b, double* c, size_t n,
                            void* hip_stream) {
  if (kind < CTU_STREAM_READ || kind > CTU_STREAM_COMBINE5)
    return fail(CTU_EINVAL, "unknown stream kind");
  if (!a || !c || (kind == CTU_STREAM_ADD && !b) || n == 0)
    return fail(CTU_EINVAL, "null array or empty stream");
  HIP_TRY(ctu::launch_stream_probe(kind, a, b, c, n, (hipStream_t)hip_stream), "stream probe");
  return CTU_OK;
}

ctu_status ctu_newton_histogram(ctu_grid* g, uint64_t hist[8]) {
  if (!g || !hist) return fail(CTU_EINVAL, "null argument");
  if (!g->prof || !g->prof->hist) return fail(CTU_EINVAL, "Newton histogram not enabled");
  DevScalars s;
  ctu_status st = read_scalars(g, &s);
  if (st != CTU_OK) return st;
  for (int k = 0; k < 8; ++k) hist[k] = s.newton_hist[k];
  return CTU_OK;
}

ctu_status ctu_grid_info_get(ctu_grid* g, ctu_grid_info* info) {
  if (!g || !info) return fail(CTU_EINVAL, "null argument");
  DevScalars s;
  ctu_status st = read_scalars(g, &s);
  if (st != CTU_OK) return st;
  info->alloc_cells = alloc_cells(g->cfg);
  info->field_stride = g->P.stride;
  info->elem_bytes = (int32_t)elem_bytes(g->cfg.prec);
  info->t = s.t;
  info->steps = s.steps;
  info->ghost = g->P.ng;
  info->schedule = g->schedule;
  return CTU_OK;
}

ctu_status ctu_set_state(ctu_grid* g, const void* const h_fields[5]) {
  if (!g || !h_fields) return fail(CTU_EINVAL, "null argument");
  if (ctu_status st_ = not_in_batch(g)) return st_;
  for (int f = 0; f < 5; ++f)
    if (!h_fields[f]) return fail(CTU_EINVAL, "null host field");
  const size_t ncell = (size_t)g->cfg.nx * g->cfg.ny * g->cfg.nz;
  const size_t eb = elem_bytes(g->cfg.prec);
  char* staging = g->fields();
  for (int f = 0; f < 5; ++f)
    HIP_TRY(hipMemcpyAsync(staging + f * ncell * eb, h_fields[f], ncell * eb, hipMemcpyHostToDevice,
                           g->stream),
            "set_state copy");
  hipError_t e = g->cfg.prec == CTU_FP64
                     ? ctu::launch_scatter<double>(reinterpret_cast<double*>(staging),
                                                   reinterpret_cast<double*>(g->d_state), g->P, g->stream)
                     : ctu::launch_scatter<float>(reinterpret_cast<float*>(staging),
                                                  reinterpret_cast<float*>(g->d_state), g->P, g->stream);
  if (e != hipSuccess) return hip_fail(e, "scatter");
  return reset_scalars(g);
}

ctu_status ctu_set_primitive(ctu_grid* g, const double* const h_fields[5]) {
  if (!g || !h_fields) return fail(CTU_EINVAL, "null argument");
  if (ctu_status st_ = not_in_batch(g)) return st_;
  for (int f = 0; f < 5; ++f)
    if (!h_fields[f]) return fail(CTU_EINVAL, "null host field");
  const size_t ncell = (size_t)g->cfg.nx * g->cfg.ny * g->cfg.nz;
  double* staging = reinterpret_cast<double*>(g->fields());
  for (int f = 0; f < 5; ++f)
    HIP_TRY(hipMemcpyAsync(staging + f * ncell, h_fields[f], ncell * sizeof(double),
                           hipMemcpyHostToDevice, g->stream),
            "set_primitive copy");
  hipError_t e = g->cfg.prec == CTU_FP64
                     ? ctu::launch_prim_to_cons<double>(staging, reinterpret_cast<double*>(g->d_state),
                                                        g->P, g->stream)
                     : ctu::launch_prim_to_cons<float>(staging, reinterpret_cast<float*>(g->d_state),
                                                       g->P, g->stream);
  if (e != hipSuccess) return hip_fail(e, "prim_to_cons");
  return reset_scalars(g);
}

ctu_status ctu_get_state(ctu_grid* g, void* const h_fields[5]) {
  if (!g || !h_fields) return fail(CTU_EINVAL, "null argument");
  if (ctu_status st_ = not_in_batch(g)) return st_;
  for (int f = 0; f < 5; ++f)
    if (!h_fields[f]) return fail(CTU_EINVAL, "null host field");
  const size_t ncell = (size_t)g->cfg.nx * g->cfg.ny * g->cfg.nz;
  const size_t eb = elem_bytes(g->cfg.prec);
  char* staging = g->fields();
  hipError_t e = g->cfg.prec == CTU_FP64
                     ? ctu::launch_gather<double>(reinterpret_cast<double*>(g->d_state),
                                                  reinterpret_cast<double*>(staging), g->P, g->stream)
                     : ctu::launch_gather<float>(reinterpret_cast<float*>(g->d_state),
                                                 reinterpret_cast<float*>(staging), g->P, g->stream);
  if (e != hipSuccess) return hip_fail(e, "gather");
  for (int f = 0; f < 5; ++f)
    HIP_TRY(hipMemcpyAsync(h_fields[f], staging + f * ncell * eb, ncell * eb, hipMemcpyDeviceToHost,
                           g->stream),
            "get_state copy");
  // the staging area is the flux scratch: the device CFL bound stays valid
  DevScalars s;
  ctu_status st = read_scalars(g, &s);
  if (st != CTU_OK) return st;
  if (s.flags & (CTU_FLAG_NONFINITE | CTU_FLAG_DENSITY))
    return fail(CTU_ENONPHYS, "non-physical state flagged on the device");
  return CTU_OK;
}

ctu_status ctu_compute_dt(ctu_grid* g, double* dt) {
  if (!g || !dt) return fail(CTU_EINVAL, "null argument");
  if (ctu_status st_ = not_in_batch(g)) return st_;
  ctu_status st = ensure_dt(g);
  if (st != CTU_OK) return st;
  DevScalars s;
  st = read_scalars(g, &s);
  if (st != CTU_OK) return st;
  double bound;
  std::memcpy(&bound, &s.dt_next_bits, sizeof(bound));
  *dt = g->cfg.cfl * bound;
  if (!(std::isfinite(*dt) && *dt > 0.0)) return fail(CTU_ENONPHYS, "no finite CFL time step");
  return CTU_OK;
}

ctu_status ctu_step(ctu_grid* g, double dt) {
  if (!g) return fail(CTU_EINVAL, "null grid");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CTU_EINVAL, "dt must be finite and > 0");
  if (ctu_status st = not_in_batch(g)) return st;
  HIP_TRY(ctu::launch_set_dt(g->scalars(), dt, g->stream), "set_dt");
  return step_impl(g, false);
}

ctu_status ctu_advance(ctu_grid* g, int32_t nsteps, double t_end) {
  if (!g) return fail(CTU_EINVAL, "null grid");
  if (nsteps < 0) return fail(CTU_EINVAL, "nsteps must be >= 0");
  if (std::isnan(t_end)) return fail(CTU_EINVAL, "t_end is NaN");
  if (ctu_status st = not_in_batch(g)) return st;
  if (nsteps == 0) return CTU_OK;
  ctu_status st = ensure_dt(g);
  if (st != CTU_OK) return st;
  HIP_TRY(ctu::launch_set_end(g->scalars(), t_end, nsteps, g->stream), "set_end");
  for (int32_t n = 0; n < nsteps; ++n) {
    st = step_impl(g, true);
    if (st != CTU_OK) return st;
  }
  return CTU_OK;
}

ctu_status ctu_totals(ctu_grid* g, double out[5]) {
  if (!g || !out) return fail(CTU_EINVAL, "null argument");
  if (ctu_status st_ = not_in_batch(g)) return st_;
  hipError_t e = g->cfg.prec == CTU_FP64
                     ? ctu::launch_totals<double>(reinterpret_cast<double*>(g->d_state), g->P,
                                                  g->partial(), kTotalsBlocks, g->totals_out(), g->stream)
                     : ctu::launch_totals<float>(reinterpret_cast<float*>(g->d_state), g->P,
                                                 g->partial(), kTotalsBlocks, g->totals_out(), g->stream);
  if (e != hipSuccess) return hip_fail(e, "totals");
  HIP_TRY(hipMemcpyAsync(out, g->totals_out(), 5 * sizeof(double), hipMemcpyDeviceToHost, g->stream),
          "totals copy");
  HIP_TRY(hipStreamSynchronize(g->stream), "totals sync");
  return CTU_OK;
}

ctu_status ctu_check(ctu_grid* g, uint32_t* flags, uint64_t counters[4]) {
  if (!g) return fail(CTU_EINVAL, "null grid");
  if (ctu_status st_ = not_in_batch(g)) return st_;
  DevScalars s;
  ctu_status st = read_scalars(g, &s);
  if (st != CTU_OK) return st;
  if (flags) *flags = s.flags;
  if (counters)
    for (int i = 0; i < 4; ++i) counters[i] = s.counters[i];
  // clear flags and counters on the device
  DevScalars z = s;
  z.flags = 0;
  for (int i = 0; i < 4; ++i) z.counters[i] = 0;
  HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(g->scalars()) + offsetof(DevScalars, flags),
                         reinterpret_cast<char*>(&z) + offsetof(DevScalars, flags),
                         offsetof(DevScalars, steps) - offsetof(DevScalars, flags),
                         hipMemcpyHostToDevice, g->stream),
          "check clear");
  HIP_TRY(hipStreamSynchronize(g->stream), "check sync");
  if (s.flags & (CTU_FLAG_NONFINITE | CTU_FLAG_DENSITY))
    return fail(CTU_ENONPHYS, "non-physical state flagged on the device");
  if (s.flags & CTU_FLAG_NEWTON_CAP) return fail(CTU_ENOCONV, "Newton iteration cap reached");
  return CTU_OK;
}

ctu_status ctu_debug_keep_fluxes(ctu_grid* g, int32_t keep) {
  if (!g) return fail(CTU_EINVAL, "null grid");
  if (ctu_status st = not_in_batch(g)) return st;
  const int flags = keep ? (g->desc.flags | ctu::GRID_KEEP_X_FLUXES)
                         : (g->desc.flags & ~ctu::GRID_KEEP_X_FLUXES);
  if (flags == g->desc.flags) return CTU_OK;
  g->desc.flags = flags;
  HIP_TRY(hipMemcpyAsync(g->d_desc(), &g->desc, sizeof(g->desc), hipMemcpyHostToDevice,
                         g->stream),
          "descriptor upload");
  HIP_TRY(hipStreamSynchronize(g->stream), "descriptor sync");
  return CTU_OK;
}

ctu_status ctu_debug_fluxes(ctu_grid* g, int32_t which, int32_t dir, double* const h_fields[5]) {
  if (!g || !h_fields || which < 0 || which > 1 || dir < 0 || dir > 2)
    return fail(CTU_EINVAL, "bad argument");
  if (which == 1 && dir == 0 && !(g->desc.flags & ctu::GRID_KEEP_X_FLUXES))
    return fail(CTU_EINVAL, "x CTU differences are stored only after ctu_debug_keep_fluxes(g, 1)");
  const size_t n = (size_t)alloc_cells(g->cfg);
  const size_t eb = elem_bytes(g->cfg.prec);
  const size_t base = (which == 0 ? 0 : 15) + 5 * dir;
  std::vector<char> tmp(n * eb);
  for (int f = 0; f < 5; ++f) {
    HIP_TRY(hipMemcpyAsync(tmp.data(), g->fields() + (base + f) * g->fbytes(), n * eb,
                           hipMemcpyDeviceToHost, g->stream),
            "debug copy");
    HIP_TRY(hipStreamSynchronize(g->stream), "debug sync");
    if (eb == 8) {
      std::memcpy(h_fields[f], tmp.data(), n * 8);
    } else {
      const float* src = reinterpret_cast<const float*>(tmp.data());
      for (size_t i = 0; i < n; ++i) h_fields[f][i] = src[i];
    }
  }
  return CTU_OK;
}

// ---- the step without device allocation ------------------------------------------------------

}  // extern "C"

// Workspace of ctu_step_noalloc: one fixed array per GPU in the library's own device memory,
// allocated with the code object and held until the process ends.  Host code uses only the
// address hipGetSymbolAddress returns for the current device (kept in g_scratch_ptr), never
// the array's name, which on the host is a stand-in and not a device address.
static __device__ __align__(256) char scratch[CTU_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per device.
ctu_status scratch_for_current_device(char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(CTU_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return fail(CTU_EDEVICE, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_ptr[dev] = reinterpret_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CTU_OK;
}

// Header of one step in the scratch array, passed by value as a kernel argument.
struct NoAllocHeader {
  ctu::GridDesc desc;
  int start[2 * ctu::P_NUM];
  double dt;
};

// Writes the grid descriptor, the block table and fresh scalars (time step dt, no CFL
// bound, cleared error word and counters) into the scratch header.
__global__ void k_noalloc_header(NoAllocHeader h, char* base) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  DevScalars z;
  std::memset(&z, 0, sizeof(z));
  z.dt = h.dt;
  z.dt_next_bits = 0x7ff0000000000000ull;
  *reinterpret_cast<DevScalars*>(base + kScalarsOffset) = z;
  *reinterpret_cast<ctu::GridDesc*>(base + kDescOffset) = h.desc;
  int* st = reinterpret_cast<int*>(base + kStartOffset);
  for (int i = 0; i < 2 * ctu::P_NUM; ++i) st[i] = h.start[i];
}

}  // namespace

extern "C" {

ctu_status ctu_step_noalloc(const ctu_config* cfg, void* d_state, double dt, void* hip_stream) {
  ctu_status s = validate(cfg);
  if (s != CTU_OK) return s;
  if (!d_state) return fail(CTU_EINVAL, "null device buffer");
  if (reinterpret_cast<uintptr_t>(d_state) % 256 != 0)
    return fail(CTU_EINVAL, "the state buffer must be 256-byte aligned");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CTU_EINVAL, "dt must be finite and > 0");
  size_t need_state = 0, need_work = 0;
  ctu_workspace_bytes(cfg, &need_state, &need_work);
  if (need_work > CTU_NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    std::snprintf(msg, sizeof(msg),
                  "grid needs %zu bytes of workspace; the fixed scratch holds %zu",
                  need_work, (size_t)CTU_NOALLOC_SCRATCH_BYTES);
    return fail(CTU_EINVAL, msg);
  }
  char* base = nullptr;
  s = scratch_for_current_device(&base);
  if (s != CTU_OK) return s;
  NoAllocHeader h;
  std::memset(&h, 0, sizeof(h));
  h.desc.P = make_params(*cfg);
  const size_t fb = (size_t)h.desc.P.stride * elem_bytes(cfg->prec);
  char* fields = base + kHeaderBytes;
  h.desc.u = d_state;
  h.desc.flux = fields;
  h.desc.s = reinterpret_cast<DevScalars*>(base + kScalarsOffset);
  h.desc.part = reinterpret_cast<double*>(fields + (size_t)fields_per_grid(*cfg) * fb);
  h.desc.coef = cfg->recon == CTU_RECON_PPMP ? fields + 30 * fb : nullptr;
  h.desc.eta = cfg->h_correction ? fields + (30 + coef_fields(*cfg)) * fb : nullptr;
  for (int i = 0; i < 6; ++i) h.desc.bc[i] = cfg->bc[i];
  h.desc.flags = 0;
  if (!build_starts_one(h.desc.P, h.start))
    return fail(CTU_EINVAL, "grid too large for one launch per pass");
  h.dt = dt;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_noalloc_header, dim3(1), dim3(64), 0, stream, h, base);
  HIP_TRY(hipGetLastError(), "scratch header");
  const ctu::PlanView v{reinterpret_cast<ctu::GridDesc*>(base + kDescOffset),
                        reinterpret_cast<int*>(base + kStartOffset), 1, h.start,
                        cfg->prec == CTU_FP32 ? 1 : 0, ctu::gas_class(h.desc.P), h.desc.P.recon};
  HIP_TRY(ctu::launch_step(v, false, stream, nullptr), "step launch");
  return CTU_OK;
}

// ---- batches ---------------------------------------------------------------------------------

}  // extern "C"

struct ctu_batch {
  struct Slot {
    bool used = false;
    uint64_t ticket = 0;
    ctu_grid* grid = nullptr;
    double t_end = 0.0;
    int32_t state = CTU_TICKET_UNKNOWN;
  };
  // Grids of one precision and gas class launched together: descriptors and block table
  // on the device, host copies of both (the block counts are needed at launch).
  struct Group {
    int prec = 0;
    int gclass = 0;
    int recon = 0;
    std::vector<ctu::GridDesc> descs;
    std::vector<int> start;
    ctu::GridDesc* d_desc = nullptr;
    int* d_start = nullptr;
    ctu::PlanView view(const ctu_batch* b) const {
      return ctu::PlanView{d_desc, d_start, (int)descs.size(), start.data(), prec, gclass, recon,
                           b->side, b->fork, b->xdone, b->join, b->ydone};
    }
  };
  // {FP64, FP32} x {PPMC, PPMP} x solver class {0, 3, 5, Roe, RoeH}
  static constexpr int kGroups = 20;
  std::vector<Slot> slots;
  int32_t flags = 0;
  hipStream_t caller = nullptr;  // the caller's stream: batch work is ordered after its work
  hipStream_t stream = nullptr;  // the batch's own stream (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // side stream and events of the overlapped sweep schedule, shared by the groups in turn
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, xdone = nullptr, join = nullptr, ydone = nullptr;
  Group groups[kGroups];
  DevScalars** d_sptr = nullptr;  // scalars of the used slots, gathered for poll
  DevScalars* d_sout = nullptr;
  std::vector<DevScalars*> h_sptr;
  std::vector<DevScalars> h_sout;
  std::vector<int> sout_slot;  // slot of each gathered entry
  bool fresh = false;          // h_sout reflects all work enqueued so far
  bool dirty = true;           // the groups do not match the running slots
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t next_ticket = 1;
};

namespace {

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Batch workspace: per precision a descriptor array and a block table, then the scalar
// pointer table and the gathered scalars.
size_t batch_group_bytes(int32_t max_slots) {
  return round256(sizeof(ctu::GridDesc) * (size_t)max_slots) +
         round256(sizeof(int) * (size_t)ctu::P_NUM * (max_slots + 1));
}

size_t batch_bytes(int32_t max_slots) {
  return ctu_batch::kGroups * batch_group_bytes(max_slots) +
         round256(sizeof(DevScalars*) * (size_t)max_slots) +
         round256(sizeof(DevScalars) * (size_t)max_slots);
}

// Batch group of a grid; within each precision the groups follow kClass and kRecon below.
int group_of(const ctu_grid* g) {
  const int c = ctu::gas_class(g->P);
  const int k = c == 3 ? 1 : c == 5 ? 2 : c == ctu::kRoe ? 3 : c == ctu::kRoeH ? 4 : 0;
  return (g->cfg.prec == CTU_FP32 ? 10 : 0) + 5 * g->P.recon + k;
}

void drop_graph(ctu_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Rebuild both precision groups from the running slots and upload them.
ctu_status rebuild(ctu_batch* b) {
  // earlier uploads read the host vectors until the stream reaches them
  HIP_TRY(hipStreamSynchronize(b->stream), "batch sync");
  drop_graph(b);
  for (int p = 0; p < ctu_batch::kGroups; ++p) {
    ctu_batch::Group& G = b->groups[p];
    G.descs.clear();
    std::vector<GridParams> Ps;
    for (const auto& sl : b->slots) {
      if (!sl.used || sl.state != CTU_TICKET_RUNNING) continue;
      if (group_of(sl.grid) != p) continue;
      G.descs.push_back(sl.grid->desc);
      Ps.push_back(sl.grid->P);
    }
    if (!build_starts(Ps, G.start)) return fail(CTU_EINVAL, "batch too large for one launch per pass");
    if (G.descs.empty()) continue;
    HIP_TRY(hipMemcpyAsync(G.d_desc, G.descs.data(), sizeof(ctu::GridDesc) * G.descs.size(),
                           hipMemcpyHostToDevice, b->stream),
            "batch descriptor upload");
    HIP_TRY(hipMemcpyAsync(G.d_start, G.start.data(), sizeof(int) * G.start.size(),
                           hipMemcpyHostToDevice, b->stream),
            "batch table upload");
  }
  b->dirty = false;
  return CTU_OK;
}

ctu_status enqueue_batch_step(ctu_batch* b) {
  for (int p = 0; p < ctu_batch::kGroups; ++p) {
    if (b->groups[p].descs.empty()) continue;
    hipError_t e = ctu::launch_step(b->groups[p].view(b), true, b->stream, nullptr);
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
  }
  return CTU_OK;
}

// One read-back of the scalars of every used slot (syncs the batch stream).
ctu_status refresh(ctu_batch* b) {
  if (b->fresh) return CTU_OK;
  HIP_TRY(hipStreamSynchronize(b->stream), "batch sync");  // host tables are free to change
  b->h_sptr.clear();
  b->sout_slot.clear();
  for (size_t i = 0; i < b->slots.size(); ++i) {
    if (!b->slots[i].used) continue;
    b->h_sptr.push_back(b->slots[i].grid->scalars());
    b->sout_slot.push_back((int)i);
  }
  const int n = (int)b->h_sptr.size();
  b->h_sout.resize(b->slots.size());
  if (n > 0) {
    std::vector<DevScalars> tmp(n);
    HIP_TRY(hipMemcpyAsync(b->d_sptr, b->h_sptr.data(), sizeof(DevScalars*) * n,
                           hipMemcpyHostToDevice, b->stream),
            "batch pointer upload");
    HIP_TRY(ctu::launch_gather_scalars(b->d_sptr, n, b->d_sout, b->stream), "batch gather");
    HIP_TRY(hipMemcpyAsync(tmp.data(), b->d_sout, sizeof(DevScalars) * n, hipMemcpyDeviceToHost,
                           b->stream),
            "batch scalars copy");
    HIP_TRY(hipStreamSynchronize(b->stream), "batch sync");
    for (int k = 0; k < n; ++k) b->h_sout[b->sout_slot[k]] = tmp[k];
  }
  b->fresh = true;
  return CTU_OK;
}

}  // namespace

extern "C" {

ctu_status ctu_batch_workspace_bytes(int32_t max_slots, size_t* work_bytes) {
  if (!work_bytes || max_slots < 1 || max_slots > (1 << 16))
    return fail(CTU_EINVAL, "max_slots must lie in [1, 65536]");
  *work_bytes = batch_bytes(max_slots);
  return CTU_OK;
}

ctu_status ctu_batch_create(int32_t max_slots, void* d_work, size_t work_bytes, void* hip_stream,
                            int32_t flags, ctu_batch** out) {
  if (!out) return fail(CTU_EINVAL, "null output handle");
  *out = nullptr;
  size_t need = 0;
  if (ctu_status st = ctu_batch_workspace_bytes(max_slots, &need)) return st;
  if (!d_work) return fail(CTU_EINVAL, "null device buffer");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return fail(CTU_EINVAL, "device buffer must be 256-byte aligned");
  if (flags & ~CTU_BATCH_GRAPH) return fail(CTU_EINVAL, "unknown batch flag");
  if (work_bytes < need)
    return fail(CTU_ENOMEM, "batch workspace too small: need " + std::to_string(need) + " bytes");
  ctu_batch* b = new ctu_batch();
  b->slots.resize(max_slots);
  b->flags = flags;
  b->caller = reinterpret_cast<hipStream_t>(hip_stream);
  char* w = reinterpret_cast<char*>(d_work);
  static const int kClass[5] = {0, 3, 5, ctu::kRoe, ctu::kRoeH};
  for (int p = 0; p < ctu_batch::kGroups; ++p) {
    b->groups[p].prec = p / 10;
    b->groups[p].recon = (p % 10) / 5;
    b->groups[p].gclass = kClass[p % 5];
    b->groups[p].d_desc = reinterpret_cast<ctu::GridDesc*>(w);
    b->groups[p].d_start =
        reinterpret_cast<int*>(w + round256(sizeof(ctu::GridDesc) * (size_t)max_slots));
    w += batch_group_bytes(max_slots);
  }
  b->d_sptr = reinterpret_cast<DevScalars**>(w);
  w += round256(sizeof(DevScalars*) * (size_t)max_slots);
  b->d_sout = reinterpret_cast<DevScalars*>(w);
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
  for (hipEvent_t* ev : {&b->ev_in, &b->ev_out})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  // the schedule's events only order the batch's two streams on one GPU
  for (hipEvent_t* ev : {&b->fork, &b->xdone, &b->join, &b->ydone})
    if (e == hipSuccess)
      e = hipEventCreateWithFlags(ev, hipEventDisableTiming | hipEventDisableSystemFence);
  if (e != hipSuccess) {
    ctu_batch_destroy(b);
    return hip_fail(e, "batch stream");
  }
  *out = b;
  return CTU_OK;
}

ctu_status ctu_batch_submit(ctu_batch* b, ctu_grid* g, int32_t nsteps, double t_end,
                            uint64_t* ticket) {
  if (!b || !g || !ticket || nsteps < 0 || std::isnan(t_end)) return fail(CTU_EINVAL, "bad argument");
  if (ctu_status st = not_in_batch(g)) return st;
  ctu_batch::Slot* slot = nullptr;
  for (auto& s : b->slots)
    if (!s.used) {
      slot = &s;
      break;
    }
  if (!slot) return fail(CTU_EAGAIN, "no free batch slot");
  // on the grid's stream: CFL bound of the current state, end time and step budget; the
  // batch stream then waits for that work
  if (ctu_status st = ensure_dt(g)) return st;
  HIP_TRY(ctu::launch_set_end(g->scalars(), t_end, nsteps, g->stream), "set_end");
  HIP_TRY(hipEventRecord(b->ev_in, g->stream), "submit record");
  HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_in, 0), "submit wait");
  slot->used = true;
  slot->ticket = b->next_ticket++;
  slot->grid = g;
  slot->t_end = t_end;
  slot->state = CTU_TICKET_RUNNING;
  g->in_batch = true;
  b->dirty = true;
  b->fresh = false;
  *ticket = slot->ticket;
  return CTU_OK;
}

ctu_status ctu_batch_run(ctu_batch* b, int32_t steps) {
  if (!b || steps < 0) return fail(CTU_EINVAL, "bad argument");
  if (steps == 0) return CTU_OK;
  if (b->dirty) {
    if (ctu_status st = rebuild(b)) return st;
  }
  bool any = false;
  for (const auto& G : b->groups) any = any || !G.descs.empty();
  if (!any) return CTU_OK;
  HIP_TRY(hipEventRecord(b->ev_in, b->caller), "batch record");
  HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_in, 0), "batch wait");
  if (b->flags & CTU_BATCH_GRAPH) {
    if (!b->exec) {
      HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "capture begin");
      ctu_status st = enqueue_batch_step(b);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(b->stream, &graph);
      if (st != CTU_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (e != hipSuccess) return hip_fail(e, "capture end");
      b->graph = graph;
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
    }
    for (int32_t k = 0; k < steps; ++k) HIP_TRY(hipGraphLaunch(b->exec, b->stream), "graph launch");
  } else {
    for (int32_t k = 0; k < steps; ++k)
      if (ctu_status st = enqueue_batch_step(b)) return st;
  }
  HIP_TRY(hipEventRecord(b->ev_out, b->stream), "batch record");
  HIP_TRY(hipStreamWaitEvent(b->caller, b->ev_out, 0), "batch wait");
  b->fresh = false;
  return CTU_OK;
}

ctu_status ctu_batch_poll(ctu_batch* b, uint64_t ticket, int32_t* state, double* t_now) {
  if (!b || !state) return fail(CTU_EINVAL, "bad argument");
  *state = CTU_TICKET_UNKNOWN;
  for (size_t i = 0; i < b->slots.size(); ++i) {
    ctu_batch::Slot& s = b->slots[i];
    if (!s.used || s.ticket != ticket) continue;
    if (ctu_status st = refresh(b)) return st;
    const DevScalars& sc = b->h_sout[i];
    if (t_now) *t_now = sc.t;
    if (s.state == CTU_TICKET_RUNNING) {
      if (sc.flags & (CTU_FLAG_NONFINITE | CTU_FLAG_DENSITY))
        s.state = CTU_TICKET_FAILED;
      else if (sc.steps_left <= 0 || sc.t >= s.t_end)
        s.state = CTU_TICKET_DONE;
    }
    *state = s.state;
    if (s.state == CTU_TICKET_DONE || s.state == CTU_TICKET_FAILED) {
      // the batch stream is idle (refresh synchronized it): the grid is the caller's again
      s.grid->in_batch = false;
      s = ctu_batch::Slot();
      b->dirty = true;
    }
    return CTU_OK;
  }
  return CTU_OK;
}

ctu_status ctu_batch_destroy(ctu_batch* b) {
  if (!b) return fail(CTU_EINVAL, "null batch");
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->side) (void)hipStreamSynchronize(b->side);
  for (auto& s : b->slots)
    if (s.used && s.grid) s.grid->in_batch = false;
  drop_graph(b);
  for (hipEvent_t ev : {b->ev_in, b->ev_out, b->fork, b->xdone, b->join, b->ydone})
    if (ev) (void)hipEventDestroy(ev);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return CTU_OK;
}

}  // extern "C"
