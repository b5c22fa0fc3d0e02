// ctu_kernels.hpp -- launch interface between the host runtime and the CTU kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "ctu_device.hpp"

namespace ctu {

// Device buffers of one grid.  fstar[d] (first-stage fluxes) and fhalf[d] (CTU fluxes):
// 5 fields each with the grid's field stride, face c+1/2 at the index of cell c;
// fstar[0..2] and fhalf[0..2] are equally spaced (kernels address them from [0]).
// part: one double per update block for the CFL reduction.
template <typename T>
struct StepBuffers {
  T* u;
  T* fstar[3];
  T* fhalf[3];
  DevScalars* scalars;
  double* part;
};

// Optional per-kernel timing: HIP events recorded on the launch stream around every kernel
// of a step, accumulated per kernel class.
enum KernelClass {
  K_BC_X, K_BC_Y, K_BC_Z, K_SWEEP1_X, K_SWEEP1_Y, K_SWEEP1_Z, K_SWEEP2_X, K_SWEEP2_Y,
  K_SWEEP2_Z, K_UPDATE, K_DT_FINAL, K_NUM_CLASSES
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
  hipEvent_t take();
  void begin(int cls, hipStream_t s);
  void end(hipStream_t s);
  hipError_t collect();  // synchronizes on the recorded events
  void reset();
  ~Profiler();
};

template <typename T>
hipError_t launch_step(const StepBuffers<T>& b, const GridParams& P, const int bc[6],
                       hipStream_t stream, Profiler* prof);
template <typename T>
hipError_t launch_dt(T* u, const GridParams& P, DevScalars* s, double* part, hipStream_t stream);
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
hipError_t launch_set_dt(DevScalars* s, double dt, hipStream_t stream);
hipError_t launch_begin_step(DevScalars* s, double cfl, double t_end, hipStream_t stream);
hipError_t launch_end_step(DevScalars* s, hipStream_t stream);

}  // namespace ctu
