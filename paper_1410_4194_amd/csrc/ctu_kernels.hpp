// ctu_kernels.hpp -- launch interface between the host runtime and the CTU kernels.
//
// Every pass of a step is one launch over a table of grids: grid g owns the blocks
// [start[g], start[g+1]) of the launch, and each block finds its grid by binary search.
// A single grid is a one-entry table, so solo, batched and served grids share one code path
// (and one launch sequence, which can be captured in a HIP graph).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "ctu_device.hpp"

namespace ctu {

// Passes of one step, in launch order, plus the stand-alone CFL reduction.
enum Pass {
  P_BC, P_COEF_X, P_COEF_Y, P_COEF_Z, P_S1_X, P_S1_Y, P_S1_Z, P_ETA_X,
  P_ETA_Z, P_S2_Y, P_S2_Z, P_S2_X, P_DT, P_NUM
};

constexpr int kBlock = 256;  // threads per block of every pass
// Consecutive chunks of XW positions per wavefront of the first-stage x sweep (default; a
// grid may set its own): the wavefront's set-up (grid lookup, parameters, task arithmetic)
// is paid once for all of them.
constexpr int kXChunks = 4;
constexpr int kSegDefault = 32;  // target cells per thread segment in the marching sweeps
constexpr int XW = 58;       // x-cells per wavefront in the first-stage x sweep
constexpr int XU = 58;       // x-cells per chunk of the second-stage x sweep with the update

// The second-stage x sweep carries the update and the CFL bound: one wavefront per group of
// P.xrows x-rows of real cells, kBlock/64 groups per block, one CFL partial per block.
__host__ __device__ inline long long update_blocks(const GridParams& P) {
  const long long groups = (long long)((P.n[1] + P.xrows - 1) / P.xrows) * P.n[2];
  return (groups + kBlock / 64 - 1) / (kBlock / 64);
}

// Rows per wavefront of the fused x update: the count of whole rows (1..8) that wastes the
// fewest lanes over the chunks of XU positions that march over them.  Longer marches hide
// latency worse (measured: two rows per wavefront at 256^3 are 14% slower than one, for 11%
// fewer idle lanes), so more than one row is taken only when it cuts idle lanes by 20%.
inline int choose_xrows(int nx, int ny) {
  const int N0 = nx + 6;
  auto eff = [&](int R) {
    const long long last = (long long)(R - 1) * N0 + nx + 2;  // last real-cell position
    const long long chunks = (last - 3) / XU + 1;
    const long long groups = (ny + R - 1) / R;
    // lanes used over lanes issued, rows of the last partial group included
    return (double)ny * nx / ((double)groups * chunks * 64.0);
  };
  int best = 1;
  double best_eff = eff(1);
  for (int R = 2; R <= 8 && R <= ny; ++R) {
    if (eff(R) > best_eff * 1.0001) {
      best_eff = eff(R);
      best = R;
    }
  }
  return best_eff >= 1.2 * eff(1) ? best : 1;
}

// Everything a kernel needs about one grid, resident in device memory.
struct GridDesc {
  GridParams P;
  void* u;          // state, 5 fields of P.stride elements (T)
  void* flux;       // 30 fields: F*_x, F*_y, F*_z, then F^{n+1/2}_x, _y, _z (5 fields each)
  DevScalars* s;    // dt, time, CFL bound, error word
  double* part;     // CFL partials, one per update block
  void* coef;       // PPMP only: flattening and steepening coefficients, 2 fields per axis (T)
  void* eta;        // H correction only: eta of the faces, 1 field per axis (T), face c-1/2
                    // at cell c
  int bc[6];
  int flags;        // GRID_KEEP_X_FLUXES: also store F^{n+1/2}_x (debug read-back only)
};

enum { GRID_KEEP_X_FLUXES = 1 };

struct LaunchTab {
  const GridDesc* grids;
  const int* start;  // ngrids + 1 block offsets of this pass (each a multiple of 8)
  int ngrids;
};

// Blocks a pass needs for one grid (before padding to a multiple of 8).
long long pass_blocks(const GridParams& P, int pass);

// Per-kernel timing with HIP events recorded on the launch stream, accumulated per class.
enum KernelClass {
  K_BC, K_PPMP_COEF, K_SWEEP1_X, K_SWEEP1_Y, K_SWEEP1_Z, K_HCORR_ETA,
  K_SWEEP2_Y, K_SWEEP2_Z, K_SWEEP2_X_UPDATE, K_DT_FINAL, K_NUM_CLASSES
};
const char* kernel_class_name(int k);

struct Profiler {
  struct Pair {
    int cls;
    hipEvent_t start, stop;
  };
  std::vector<Pair> pending;
  std::vector<hipEvent_t> pool;
  double ms[K_NUM_CLASSES] = {};
  long long launches[K_NUM_CLASSES] = {};
  bool timing = true;  // bracket kernels with events
  bool hist = false;   // launch the sweeps that count Newton iterations per solve
  hipEvent_t take();
  void begin(int cls, hipStream_t s);
  void end(hipStream_t s);
  hipError_t collect();  // synchronizes on the recorded events
  void reset();
  ~Profiler();
};

// A set of grids of one precision launched together: device descriptors and block tables
// (start[pass * (ngrids + 1) + g]), with host copies of the launch sizes.
struct PlanView {
  const GridDesc* d_grids;
  const int* d_start;
  int ngrids;
  const int* h_start;  // same layout as d_start
  int prec;            // 0 = double, 1 = float
  int gclass;          // solver class: exact with gas class 3 (gamma 5/3), 5 (gamma 7/5) or
                       // 0 (other), kRoe, or kRoeH
  int recon;           // 0 PPMC, 1 PPMP
  // Optional second stream (default priority) and four events for the overlapped schedule
  // of the sweeps (enqueue_sweeps); null side: every pass in order on the launch stream.
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, xdone = nullptr, join = nullptr, ydone = nullptr;
  bool fused_z = false;  // with the side stream: both z stages in one march (k_sweep_z_both)
};

// Solver class of a grid: kRoe for the Roe solver; for the exact solver its gas class, K
// when 2/(gamma-1) = K and 2 gamma/(gamma-1) = K + 2 for K in {3, 5}, else 0.
inline int gas_class(const GridParams& P) {
  if (P.riemann == 1) return P.ext ? kRoeH : kRoe;
  return ((P.fan_int_exp == 3 || P.fan_int_exp == 5) && P.root_m == P.fan_int_exp + 2)
             ? P.fan_int_exp
             : 0;
}

// Whether a step of the plan takes the overlapped schedule of enqueue_sweeps: a side stream
// and its events are there and kernels are not being timed one by one.
inline bool overlapped(const PlanView& v, const Profiler* prof) {
  return v.side && v.fork && v.xdone && v.join && v.ydone && !(prof && prof->timing);
}

// The fused-z variant of that schedule (never with the H correction).
inline bool fused_z(const PlanView& v, const Profiler* prof) {
  return v.fused_z && v.gclass != kRoeH && overlapped(v, prof);
}

// PPMP coefficients along axis D for every grid of the plan (ctu_kernels.hip).
template <typename T, int D>
void launch_ppmp_coef(const PlanView& v, hipStream_t stream);

// The three sweeps of stage 1 or 2 for every grid of a plan; one specialization per
// (T, K, R) is compiled in its own translation unit (ctu_sweeps.hip).
template <typename T, int K, int R>
hipError_t launch_sweeps(const PlanView& v, int stage, hipStream_t stream, Profiler* prof);
#define CTU_DECLARE_SWEEPS(T, K, R) \
  template <>                       \
  hipError_t launch_sweeps<T, K, R>(const PlanView&, int, hipStream_t, Profiler*);
CTU_DECLARE_SWEEPS(double, 0, 0)
CTU_DECLARE_SWEEPS(double, 3, 0)
CTU_DECLARE_SWEEPS(double, 5, 0)
CTU_DECLARE_SWEEPS(double, kRoe, 0)
CTU_DECLARE_SWEEPS(double, 0, 1)
CTU_DECLARE_SWEEPS(double, 3, 1)
CTU_DECLARE_SWEEPS(double, 5, 1)
CTU_DECLARE_SWEEPS(double, kRoe, 1)
CTU_DECLARE_SWEEPS(double, kRoeH, 0)
CTU_DECLARE_SWEEPS(double, kRoeH, 1)
CTU_DECLARE_SWEEPS(float, 0, 0)
CTU_DECLARE_SWEEPS(float, 3, 0)
CTU_DECLARE_SWEEPS(float, 5, 0)
CTU_DECLARE_SWEEPS(float, kRoe, 0)
CTU_DECLARE_SWEEPS(float, 0, 1)
CTU_DECLARE_SWEEPS(float, 3, 1)
CTU_DECLARE_SWEEPS(float, 5, 1)
CTU_DECLARE_SWEEPS(float, kRoe, 1)
CTU_DECLARE_SWEEPS(float, kRoeH, 0)
CTU_DECLARE_SWEEPS(float, kRoeH, 1)
#undef CTU_DECLARE_SWEEPS

// Brackets one launch with profiler events when timing is on.
#define CTU_TIMED(cls, launch)                                \
  do {                                                        \
    if (prof && prof->timing) prof->begin(cls, stream);       \
    launch;                                                   \
    if (prof && prof->timing) prof->end(stream);              \
  } while (0)

// One step for every grid of the plan.  device_dt: take dt from each grid's CFL bound and
// end time (taken by the first ghost-fill pass); otherwise each grid's dt was set beforehand.
hipError_t launch_step(const PlanView& v, bool device_dt, hipStream_t stream, Profiler* prof);
// CFL bound of the current state of every grid of the plan (into dt_next_bits).
hipError_t launch_dt(const PlanView& v, hipStream_t stream);

hipError_t launch_set_dt(DevScalars* s, double dt, hipStream_t stream);
hipError_t launch_set_end(DevScalars* s, double t_end, long long steps_left, hipStream_t stream);
// out[i] = *src[i] for i < n (src and out in device memory).
hipError_t launch_gather_scalars(DevScalars* const* src, int n, DevScalars* out,
                                 hipStream_t stream);

// Plain streaming kernels (ctu_stream.hip): kinds as in ctu_stream_probe of ctu.h.
enum { STREAM_READ = 0, STREAM_COPY = 1, STREAM_ADD = 2, STREAM_COMBINE5 = 3 };
size_t stream_probe_blocks(size_t n);
hipError_t launch_stream_probe(int kind, const double* a, const double* b, double* c, size_t n,
                               hipStream_t stream);

template <typename T>
hipError_t launch_totals(const T* u, const GridParams& P, double* part, int nblocks, double* out,
                         hipStream_t stream);
template <typename T>
hipError_t launch_scatter(const T* packed, T* u, const GridParams& P, hipStream_t stream);
template <typename T>
hipError_t launch_gather(const T* u, T* packed, const GridParams& P, hipStream_t stream);
template <typename T>
hipError_t launch_prim_to_cons(const double* packed, T* u, const GridParams& P,
                               hipStream_t stream);

}  // namespace ctu
